// Continuous-batching server: requests of different L, T and sweep counts
// share the GPU.  Their packed lattices and sweep counters stay resident in
// one device arena; every quantum advances all resident lattices together
// (tiled lattices in shared half-sweep launches, small ones one workgroup
// each), and requests join and leave between quanta.  Admission is by
// memory footprint (first-fit in the arena) and free slots, in arrival order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "ising_host.hpp"
#include "ising_launch.hpp"
#include "ising_sched.hpp"

using namespace ising;

struct ising_server {
    Scheduler sched;
    hipStream_t stream = nullptr;
    int device = 0;
    uint8_t* arena = nullptr;
    LatticeDesc* d_desc = nullptr;
    LatticeState* d_state = nullptr;
    LatticeDesc* h_desc = nullptr;  // pinned staging
    WaveItem* h_waves = nullptr;    // pinned staging
    WaveItem* d_waves = nullptr;
    int64_t waves_cap = 0;
    int32_t* h_ids = nullptr;       // pinned staging of resident ids
    int32_t* d_ids = nullptr;
    int32_t* h_fin = nullptr;       // pinned staging of finished ids
    int32_t* d_fin = nullptr;
    // quantum prepared by prepare_quantum()
    int32_t q_sweeps = 0, q_res = 0;
    int64_t q_waves = 0;
    size_t q_lds = 0;
    bool staged = false;  // pinned staging buffers may still be read by an enqueued copy
    size_t lds_limit = 0;
    int32_t resident_max_L = 256;
    bool inflight = false;
    std::vector<ising_result> done;
    std::vector<LatticeState> h_state;

    ising_server(size_t budget, int32_t slots, int32_t quantum) : sched(budget, slots, quantum) {}
};

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void release(ising_server* s) {
    if (!s) return;
    if (s->arena) (void)hipFree(s->arena);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_state) (void)hipFree(s->d_state);
    if (s->d_waves) (void)hipFree(s->d_waves);
    if (s->d_ids) (void)hipFree(s->d_ids);
    if (s->d_fin) (void)hipFree(s->d_fin);
    if (s->h_desc) (void)hipHostFree(s->h_desc);
    if (s->h_waves) (void)hipHostFree(s->h_waves);
    if (s->h_ids) (void)hipHostFree(s->h_ids);
    if (s->h_fin) (void)hipHostFree(s->h_fin);
    delete s;
}

int grow_waves(ising_server* s, int64_t need) {
    if (need <= s->waves_cap) return ISING_OK;
    int64_t cap = std::max<int64_t>(need, 2 * s->waves_cap);
    if (s->d_waves) (void)hipFree(s->d_waves);
    if (s->h_waves) (void)hipHostFree(s->h_waves);
    s->d_waves = nullptr;
    s->h_waves = nullptr;
    s->waves_cap = 0;
    ISING_HIP(hipMalloc(&s->d_waves, sizeof(WaveItem) * cap));
    ISING_HIP(hipHostMalloc(&s->h_waves, sizeof(WaveItem) * cap, hipHostMallocDefault));
    s->waves_cap = cap;
    return ISING_OK;
}

// Read back E, M of finished requests and free their slots.
int retire_finished(ising_server* s) {
    const std::vector<int32_t> fin = s->sched.finished();
    if (fin.empty()) return ISING_OK;
    for (size_t i = 0; i < fin.size(); ++i) s->h_fin[i] = fin[i];
    const int32_t nf = (int32_t)fin.size();
    ISING_HIP(hipMemcpyAsync(s->d_fin, s->h_fin, sizeof(int32_t) * nf, hipMemcpyHostToDevice, s->stream));
    ISING_HIP(launch_observe_multi(s->d_desc, s->d_state, s->d_fin, nf, s->stream));
    const int32_t slots = (int32_t)s->sched.slots().size();
    ISING_HIP(hipMemcpyAsync(s->h_state.data(), s->d_state, sizeof(LatticeState) * slots, hipMemcpyDeviceToHost,
                             s->stream));
    ISING_HIP(hipStreamSynchronize(s->stream));
    s->staged = false;
    const double t = now_s();
    for (int32_t i : fin) {
        const Slot& sl = s->sched.slots()[i];
        ising_result r;
        r.req_id = sl.req.id;
        r.L = sl.req.L;
        r.status = ISING_OK;
        r.T = sl.req.T;
        r.sweeps = sl.req.sweeps;
        r.E = s->h_state[i].last_E;
        r.M = s->h_state[i].last_M;
        r.t_submit_s = sl.req.t_submit;
        r.t_admit_s = sl.t_admit;
        r.t_done_s = t;
        s->done.push_back(r);
        s->sched.retire(i);
    }
    return ISING_OK;
}

int admit_queued(ising_server* s) {
    const std::vector<int32_t> adm = s->sched.admit(now_s());
    for (int32_t i : adm) {
        const Slot& sl = s->sched.slots()[i];
        const Geometry g = make_geometry(sl.req.L);
        ISING_HIP(launch_init(reinterpret_cast<uint64_t*>(s->arena + sl.off), g, sl.req.seed, sl.req.init, s->stream));
        ISING_HIP(hipMemsetAsync(s->d_state + i, 0, sizeof(LatticeState), s->stream));
    }
    return ISING_OK;
}

// Plan the next quantum and upload the slot table: descriptors of every
// active slot (finished ones included, with no sweeps), the wave table of
// tiled lattices and the ids of resident ones.
int prepare_quantum(ising_server* s) {
    if (s->staged) {  // the previous upload must finish before its staging is rewritten
        ISING_HIP(hipStreamSynchronize(s->stream));
        s->staged = false;
    }
    Scheduler& sc = s->sched;
    sc.plan_quantum();
    const int32_t slots = (int32_t)sc.slots().size();
    const int wpt = 4;
    int64_t n_waves = 0;
    for (int32_t i = 0; i < slots; ++i) {
        const Slot& sl = sc.slots()[i];
        if (!sl.active || sl.planned <= 0) continue;
        const Geometry g = make_geometry(sl.req.L);
        const bool res = g.L <= s->resident_max_L && (size_t)g.N * g.L * 8 <= s->lds_limit;
        if (!res) n_waves += (units_per_colour(g, wpt) + 63) / 64;
    }
    int rc = grow_waves(s, std::max<int64_t>(n_waves, 1));
    if (rc != ISING_OK) return rc;
    int32_t n_res = 0, K = 0;
    size_t lds = 0;
    n_waves = 0;
    for (int32_t i = 0; i < slots; ++i) {
        const Slot& sl = sc.slots()[i];
        LatticeDesc& d = s->h_desc[i];
        d = LatticeDesc{};
        if (!sl.active) continue;
        const Geometry g = make_geometry(sl.req.L);
        d.W = reinterpret_cast<uint64_t*>(s->arena + sl.off);
        d.L = g.L;
        d.N = g.N;
        d.istar = g.istar;
        d.sh_star = g.sh_star;
        d.k0 = (uint32_t)sl.req.seed;
        d.k1 = (uint32_t)(sl.req.seed >> 32);
        thresholds_of(sl.req.T, &d.t4, &d.t8);
        d.segs = segments_per_row(g.L, wpt);
        d.sweep_limit = (int32_t)sl.planned;
        if (sl.planned <= 0) continue;
        K = std::max<int32_t>(K, (int32_t)sl.planned);
        const bool res = g.L <= s->resident_max_L && (size_t)g.N * g.L * 8 <= s->lds_limit;
        if (res) {
            d.resident = 1;
            s->h_ids[n_res++] = i;
            lds = std::max(lds, (size_t)g.N * g.L * 8);
        } else {
            d.units = units_per_colour(g, wpt);
            d.part_begin = (int32_t)n_waves;
            for (int64_t u0 = 0; u0 < d.units; u0 += 64) s->h_waves[n_waves++] = {i, (int32_t)u0};
            d.part_count = (int32_t)(n_waves - d.part_begin);
        }
    }
    ISING_HIP(hipMemcpyAsync(s->d_desc, s->h_desc, sizeof(LatticeDesc) * slots, hipMemcpyHostToDevice, s->stream));
    if (n_waves)
        ISING_HIP(hipMemcpyAsync(s->d_waves, s->h_waves, sizeof(WaveItem) * n_waves, hipMemcpyHostToDevice, s->stream));
    if (n_res) ISING_HIP(hipMemcpyAsync(s->d_ids, s->h_ids, sizeof(int32_t) * n_res, hipMemcpyHostToDevice, s->stream));
    s->staged = true;
    s->q_sweeps = K;
    s->q_res = n_res;
    s->q_waves = n_waves;
    s->q_lds = lds;
    return ISING_OK;
}

// Enqueue the prepared quantum.
int launch_quantum(ising_server* s) {
    const int32_t K = s->q_sweeps;
    if (K == 0) return ISING_OK;
    const int wpt = 4, block = 256, rblock = 256;
    const int32_t slots = (int32_t)s->sched.slots().size();
    if (s->q_res) {
        ISING_HIP(set_resident_lds(wpt, s->q_lds));
        ISING_HIP(launch_resident(wpt, rblock, s->d_desc, s->d_state, s->d_ids, s->q_res, K, 0, s->q_lds, s->stream));
    }
    for (int32_t k = 0; k < K && s->q_waves; ++k) {
        ISING_HIP(launch_halfsweep_multi(wpt, block, s->d_desc, s->d_state, s->d_waves, s->q_waves, 0, (uint32_t)k,
                                         nullptr, s->stream));
        ISING_HIP(launch_halfsweep_multi(wpt, block, s->d_desc, s->d_state, s->d_waves, s->q_waves, 1, (uint32_t)k,
                                         nullptr, s->stream));
    }
    ISING_HIP(launch_advance(s->d_desc, s->d_state, slots, (uint32_t)K, s->stream));
    s->inflight = true;
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_server_create(size_t hbm_budget, int32_t max_slots, int32_t quantum_sweeps, void* stream,
                        ising_server** out) {
    if (!out) return fail(ISING_EINVAL, "ising_server_create: null output");
    *out = nullptr;
    if (hbm_budget < 256) return fail(ISING_EINVAL, "ising_server_create: budget too small");
    if (max_slots < 1 || max_slots > (1 << 20)) return fail(ISING_EINVAL, "ising_server_create: max_slots in [1, 2^20]");
    if (quantum_sweeps < 1 || quantum_sweeps > 100000)
        return fail(ISING_EINVAL, "ising_server_create: quantum_sweeps in [1, 100000]");
    ising_server* s = new (std::nothrow) ising_server(hbm_budget, max_slots, quantum_sweeps);
    if (!s) return fail(ISING_ENOMEM, "ising_server_create: host allocation failed");
    s->stream = (hipStream_t)stream;
    s->h_state.resize(max_slots);
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipMalloc(&s->arena, s->sched.budget());
    if (e != hipSuccess) {
        s->arena = nullptr;
        release(s);
        return fail(ISING_ENOMEM, "ising_server_create: arena of %zu bytes: %s", hbm_budget, hipGetErrorString(e));
    }
    e = hipMalloc(&s->d_desc, sizeof(LatticeDesc) * max_slots);
    if (e == hipSuccess) e = hipMalloc(&s->d_state, sizeof(LatticeState) * max_slots);
    if (e == hipSuccess) e = hipMalloc(&s->d_ids, sizeof(int32_t) * max_slots);
    if (e == hipSuccess) e = hipMalloc(&s->d_fin, sizeof(int32_t) * max_slots);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_desc, sizeof(LatticeDesc) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_ids, sizeof(int32_t) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_fin, sizeof(int32_t) * max_slots, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_state, 0, sizeof(LatticeState) * max_slots, s->stream);
    if (e != hipSuccess) {
        release(s);
        return hip_fail(e, "ising_server_create");
    }
    s->lds_limit = resident_lds_limit(s->device);
    *out = s;
    return ISING_OK;
}

int ising_server_submit(ising_server* s, uint64_t req_id, int32_t L, double T, int64_t sweeps, uint64_t seed,
                        int32_t init) {
    if (!s) return fail(ISING_EINVAL, "ising_server_submit: null handle");
    if (!valid_L(L)) return fail(ISING_EINVAL, "ising_server_submit: L = %d invalid", L);
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_server_submit: T must be finite and > 0");
    if (sweeps < 0 || sweeps > 0x7FFFFFFF) return fail(ISING_EINVAL, "ising_server_submit: sweeps out of range");
    if (init != ISING_COLD && init != ISING_HOT) return fail(ISING_EINVAL, "ising_server_submit: init must be 0 or 1");
    Request r;
    r.id = req_id;
    r.L = L;
    r.T = T;
    r.sweeps = sweeps;
    r.seed = seed;
    r.init = init;
    r.bytes = ising_required_bytes(L);
    r.t_submit = now_s();
    if (!s->sched.submit(r))
        return fail(ISING_EINVAL, "ising_server_submit: lattice of %zu bytes exceeds the budget", r.bytes);
    return ISING_OK;
}

int ising_server_step(ising_server* s, int32_t* active) {
    if (!s) return fail(ISING_EINVAL, "ising_server_step: null handle");
    if (s->inflight) {
        ISING_HIP(hipStreamSynchronize(s->stream));
        s->sched.complete_quantum();
        s->inflight = false;
        s->staged = false;
    }
    // finished requests leave first so their memory and slots can be reused
    int rc = prepare_quantum(s);
    if (rc == ISING_OK) rc = retire_finished(s);
    if (rc == ISING_OK) rc = admit_queued(s);
    if (rc == ISING_OK) rc = prepare_quantum(s);
    if (rc == ISING_OK) rc = retire_finished(s);  // zero-sweep requests finish at once
    if (rc == ISING_OK) rc = launch_quantum(s);
    if (active) *active = s->sched.active();
    return rc;
}

int ising_server_poll(ising_server* s, ising_result* out, int32_t cap, int32_t* n) {
    if (!s || !n || (cap > 0 && !out)) return fail(ISING_EINVAL, "ising_server_poll: null argument");
    const int32_t k = std::min<int32_t>(cap, (int32_t)s->done.size());
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return ISING_OK;
}

int ising_server_stats(ising_server* s, int32_t* queued, int32_t* resident, int32_t* finished, size_t* bytes_in_use) {
    if (!s) return fail(ISING_EINVAL, "ising_server_stats: null handle");
    if (queued) *queued = (int32_t)s->sched.queued();
    if (resident) *resident = s->sched.active();
    if (finished) *finished = (int32_t)s->done.size();
    if (bytes_in_use) *bytes_in_use = s->sched.bytes_in_use();
    return ISING_OK;
}

int ising_server_destroy(ising_server* s) {
    if (!s) return ISING_OK;
    hipError_t e = hipStreamSynchronize(s->stream);
    release(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ISING_OK;
}

}  // extern "C"

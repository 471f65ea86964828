// Continuous-batching server: requests of different L, T and sweep counts
// share the GPU.  Their packed lattices and sweep counters stay resident in
// one device arena; every quantum advances all resident lattices together
// (tiled lattices in shared half-sweep launches, small ones one workgroup
// each), and requests join and leave between quanta.  Admission is by
// memory footprint (first-fit in the arena) and free slots, in arrival order.
//
// Pipelining: the host plans, uploads and enqueues quantum q+1 while quantum
// q runs (at most two quanta in flight).  Bookkeeping counts sweeps when they
// are enqueued; a request whose last quantum has been enqueued has its E/M
// reduction and read-back enqueued right behind it into a pinned ring entry,
// and its slot and arena range are reused at once (stream order puts any
// later use after the read-back).  Results are harvested when their event
// has completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <vector>

#include "ising_host.hpp"
#include "ising_launch.hpp"
#include "ising_sched.hpp"

using namespace ising;

namespace {

constexpr int kServerWpt = 1;  // words per thread of the server's kernels
constexpr int kStages = 2;     // quanta in flight = staging buffer sets
constexpr int kRing = 4;       // read-back ring entries

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Host staging of one quantum's tables (pinned), reusable once `done` fired.
struct Stage {
    LatticeDesc* desc = nullptr;
    WaveItem* waves = nullptr;
    int64_t waves_cap = 0;
    int32_t* ids = nullptr;
    hipEvent_t done = nullptr;  // recorded after the quantum's kernels
    bool used = false;
};

// One batch of finished requests whose E/M read-back is in flight.
struct Readback {
    int32_t* ids = nullptr;  // pinned: slot ids uploaded for the reduction
    int64_t* em = nullptr;   // pinned: (E, M) per listed slot
    hipEvent_t done = nullptr;
    bool pending = false;
    std::vector<ising_result> meta;  // request data; E, M and t_done filled at harvest
};

}  // namespace

struct ising_server {
    Scheduler sched;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;  // resident (small-lattice) work runs beside the tiled launches
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    int device = 0;
    uint8_t* arena = nullptr;
    LatticeDesc* d_desc = nullptr;
    LatticeState* d_state = nullptr;
    WaveItem* d_waves = nullptr;
    int64_t d_waves_cap = 0;
    int32_t* d_ids = nullptr;  // resident ids of the current quantum
    int32_t* d_fin = nullptr;  // ids of a read-back batch
    int64_t* d_em = nullptr;   // (E, M) of a read-back batch
    Stage stage[kStages];
    int next_stage = 0;
    std::deque<hipEvent_t> inflight;  // quantum events, oldest first
    Readback ring[kRing];
    int next_ring = 0;  // entry the next batch uses = oldest entry
    size_t lds_limit = 0;
    int32_t resident_max_L = 256;
    std::vector<ising_result> done;

    ising_server(size_t budget, int32_t slots, int32_t quantum) : sched(budget, slots, quantum) {}
};

namespace {

void release(ising_server* s) {
    if (!s) return;
    if (s->arena) (void)hipFree(s->arena);
    if (s->d_desc) (void)hipFree(s->d_desc);
    if (s->d_state) (void)hipFree(s->d_state);
    if (s->d_waves) (void)hipFree(s->d_waves);
    if (s->d_ids) (void)hipFree(s->d_ids);
    if (s->d_fin) (void)hipFree(s->d_fin);
    if (s->d_em) (void)hipFree(s->d_em);
    for (Stage& st : s->stage) {
        if (st.desc) (void)hipHostFree(st.desc);
        if (st.waves) (void)hipHostFree(st.waves);
        if (st.ids) (void)hipHostFree(st.ids);
        if (st.done) (void)hipEventDestroy(st.done);
    }
    for (Readback& r : s->ring) {
        if (r.ids) (void)hipHostFree(r.ids);
        if (r.em) (void)hipHostFree(r.em);
        if (r.done) (void)hipEventDestroy(r.done);
    }
    for (hipEvent_t e : s->inflight) (void)hipEventDestroy(e);
    if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
    if (s->join_ev) (void)hipEventDestroy(s->join_ev);
    if (s->side) (void)hipStreamDestroy(s->side);
    delete s;
}

// Move a completed read-back batch into the finished list.  wait: block on
// its event; otherwise only if it has already completed.
int harvest(ising_server* s, Readback& r, bool wait) {
    if (!r.pending) return ISING_OK;
    if (wait) {
        ISING_HIP(hipEventSynchronize(r.done));
    } else {
        const hipError_t e = hipEventQuery(r.done);
        if (e == hipErrorNotReady) return ISING_OK;
        if (e != hipSuccess) return hip_fail(e, "hipEventQuery");
    }
    const double t = now_s();
    for (size_t k = 0; k < r.meta.size(); ++k) {
        ising_result res = r.meta[k];
        res.E = r.em[2 * k];
        res.M = r.em[2 * k + 1];
        res.t_done_s = t;
        s->done.push_back(res);
    }
    r.meta.clear();
    r.pending = false;
    return ISING_OK;
}

// Harvest in submission order (oldest ring entry first); stop at the first
// batch that is not ready unless `wait`.
int harvest_all(ising_server* s, bool wait) {
    for (int k = 0; k < kRing; ++k) {
        Readback& r = s->ring[(s->next_ring + k) % kRing];
        int rc = harvest(s, r, wait);
        if (rc != ISING_OK) return rc;
        if (r.pending) break;
    }
    return ISING_OK;
}

int grow_waves(ising_server* s, Stage& st, int64_t need) {
    if (need > st.waves_cap) {
        const int64_t cap = std::max<int64_t>(need, 2 * st.waves_cap);
        if (st.waves) (void)hipHostFree(st.waves);
        st.waves = nullptr;
        st.waves_cap = 0;
        ISING_HIP(hipHostMalloc(&st.waves, sizeof(WaveItem) * cap, hipHostMallocDefault));
        st.waves_cap = cap;
    }
    if (need > s->d_waves_cap) {
        // earlier quanta read the device table: let them finish before replacing it
        ISING_HIP(hipStreamSynchronize(s->stream));
        const int64_t cap = std::max<int64_t>(need, 2 * s->d_waves_cap);
        if (s->d_waves) (void)hipFree(s->d_waves);
        s->d_waves = nullptr;
        s->d_waves_cap = 0;
        ISING_HIP(hipMalloc(&s->d_waves, sizeof(WaveItem) * cap));
        s->d_waves_cap = cap;
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

bool is_resident(const ising_server* s, const Geometry& g) {
    return g.L <= s->resident_max_L && (size_t)g.N * g.L * 8 <= s->lds_limit;
}

// Plan the next quantum, upload its tables through a staging set and enqueue
// its kernels.  Descriptors cover every active slot (those already done with
// zero sweeps, so the read-back that follows can use them).
int enqueue_quantum(ising_server* s) {
    Scheduler& sc = s->sched;
    sc.plan_quantum();
    const int32_t slots = (int32_t)sc.slots().size();
    Stage& st = s->stage[s->next_stage];
    s->next_stage = (s->next_stage + 1) % kStages;
    if (st.used) ISING_HIP(hipEventSynchronize(st.done));  // its previous copies have been read
    int64_t n_waves = 0;
    for (int32_t i = 0; i < slots; ++i) {
        const Slot& sl = sc.slots()[i];
        if (!sl.active || sl.planned <= 0) continue;
        const Geometry g = make_geometry(sl.req.L);
        if (!is_resident(s, g)) n_waves += waves_per_colour(g, kServerWpt);
    }
    int rc = grow_waves(s, st, std::max<int64_t>(n_waves, 1));
    if (rc != ISING_OK) return rc;
    int32_t n_res = 0, K = 0;
    size_t lds = 0;
    bool off32 = true;
    n_waves = 0;
    for (int32_t i = 0; i < slots; ++i) {
        const Slot& sl = sc.slots()[i];
        LatticeDesc& d = st.desc[i];
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
        d.segs = segments_per_row(g.L, kServerWpt);
        d.sweep_limit = (int32_t)sl.planned;
        if (sl.planned <= 0) continue;
        K = std::max<int32_t>(K, (int32_t)sl.planned);
        if (is_resident(s, g)) {
            d.resident = 1;
            st.ids[n_res++] = i;
            lds = std::max(lds, (size_t)g.N * g.L * 8);
        } else {
            d.units = units_per_colour(g, kServerWpt);
            off32 = off32 && fits_off32(g);
            d.part_begin = (int32_t)n_waves;
            for (int32_t I = 0; I < g.N; ++I)
                for (int32_t s0 = 0; s0 < d.segs; s0 += 64) st.waves[n_waves++] = {i, I, s0};
            d.part_count = (int32_t)(n_waves - d.part_begin);
        }
    }
    ISING_HIP(hipMemcpyAsync(s->d_desc, st.desc, sizeof(LatticeDesc) * slots, hipMemcpyHostToDevice, s->stream));
    if (n_waves)
        ISING_HIP(hipMemcpyAsync(s->d_waves, st.waves, sizeof(WaveItem) * n_waves, hipMemcpyHostToDevice, s->stream));
    if (n_res) ISING_HIP(hipMemcpyAsync(s->d_ids, st.ids, sizeof(int32_t) * n_res, hipMemcpyHostToDevice, s->stream));
    if (K > 0) {
        const int block = 64, rblock = 256;
        if (n_res) {
            // the resident lattices (one workgroup each) run on the side
            // stream, overlapping the tiled launches of the other lattices
            ISING_HIP(set_resident_lds(kServerWpt, lds));
            ISING_HIP(hipEventRecord(s->fork_ev, s->stream));
            ISING_HIP(hipStreamWaitEvent(s->side, s->fork_ev, 0));
            ISING_HIP(launch_resident(kServerWpt, rblock, s->d_desc, s->d_state, s->d_ids, n_res, K, 0, lds, s->side));
            ISING_HIP(hipEventRecord(s->join_ev, s->side));
        }
        for (int32_t k = 0; k < K && n_waves; ++k) {
            ISING_HIP(launch_halfsweep_multi(kServerWpt, block, s->d_desc, s->d_state, s->d_waves, n_waves, 0,
                                             (uint32_t)k, nullptr, nullptr, 0, off32, s->stream));
            ISING_HIP(launch_halfsweep_multi(kServerWpt, block, s->d_desc, s->d_state, s->d_waves, n_waves, 1,
                                             (uint32_t)k, nullptr, nullptr, 0, off32, s->stream));
        }
        if (n_res) ISING_HIP(hipStreamWaitEvent(s->stream, s->join_ev, 0));
        ISING_HIP(launch_chunk_end(s->d_desc, s->d_state, slots, nullptr, 0, (uint32_t)K, s->stream));
    }
    ISING_HIP(hipEventRecord(st.done, s->stream));
    st.used = true;
    sc.complete_quantum();
    return ISING_OK;
}

// Enqueue E/M and read-back of every request whose sweeps are all enqueued,
// then free their slots and memory.
int enqueue_retirements(ising_server* s) {
    const std::vector<int32_t> fin = s->sched.finished();
    if (fin.empty()) return ISING_OK;
    Readback& r = s->ring[s->next_ring];
    int rc = harvest(s, r, true);  // the entry's previous batch must have landed
    if (rc != ISING_OK) return rc;
    s->next_ring = (s->next_ring + 1) % kRing;
    const int32_t nf = (int32_t)fin.size();
    for (int32_t k = 0; k < nf; ++k) {
        const Slot& sl = s->sched.slots()[fin[k]];
        r.ids[k] = fin[k];
        ising_result m;
        m.req_id = sl.req.id;
        m.L = sl.req.L;
        m.status = ISING_OK;
        m.T = sl.req.T;
        m.sweeps = sl.req.sweeps;
        m.E = m.M = 0;
        m.t_submit_s = sl.req.t_submit;
        m.t_admit_s = sl.t_admit;
        m.t_done_s = 0;
        r.meta.push_back(m);
    }
    ISING_HIP(hipMemcpyAsync(s->d_fin, r.ids, sizeof(int32_t) * nf, hipMemcpyHostToDevice, s->stream));
    ISING_HIP(launch_observe_multi(s->d_desc, s->d_state, s->d_fin, nf, s->d_em, s->stream));
    ISING_HIP(hipMemcpyAsync(r.em, s->d_em, sizeof(int64_t) * 2 * nf, hipMemcpyDeviceToHost, s->stream));
    ISING_HIP(hipEventRecord(r.done, s->stream));
    r.pending = true;
    for (int32_t i : fin) s->sched.retire(i);
    return ISING_OK;
}

int wait_idle(ising_server* s) {
    while (!s->inflight.empty()) {
        hipEvent_t e = s->inflight.front();
        s->inflight.pop_front();
        const hipError_t he = hipEventSynchronize(e);
        (void)hipEventDestroy(e);
        if (he != hipSuccess) return hip_fail(he, "hipEventSynchronize");
    }
    return harvest_all(s, true);
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
    if (e == hipSuccess) e = hipMalloc(&s->d_em, sizeof(int64_t) * 2 * max_slots);
    for (Stage& st : s->stage) {
        if (e == hipSuccess) e = hipHostMalloc(&st.desc, sizeof(LatticeDesc) * max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&st.ids, sizeof(int32_t) * max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
    }
    for (Readback& r : s->ring) {
        if (e == hipSuccess) e = hipHostMalloc(&r.ids, sizeof(int32_t) * max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&r.em, sizeof(int64_t) * 2 * max_slots, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming);
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
    int rc = harvest_all(s, false);
    // at most kStages quanta in flight: wait for the oldest before adding one
    while (rc == ISING_OK && (int)s->inflight.size() >= kStages) {
        hipEvent_t e = s->inflight.front();
        s->inflight.pop_front();
        const hipError_t he = hipEventSynchronize(e);
        (void)hipEventDestroy(e);
        if (he != hipSuccess) rc = hip_fail(he, "hipEventSynchronize");
        if (rc == ISING_OK) rc = harvest_all(s, false);
    }
    if (rc == ISING_OK) rc = admit_queued(s);
    if (rc == ISING_OK && s->sched.active() > 0) {
        rc = enqueue_quantum(s);
        if (rc == ISING_OK) rc = enqueue_retirements(s);
        if (rc == ISING_OK) {
            hipEvent_t e = nullptr;
            hipError_t he = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (he == hipSuccess) he = hipEventRecord(e, s->stream);
            if (he != hipSuccess) {
                if (e) (void)hipEventDestroy(e);
                rc = hip_fail(he, "quantum event");
            } else {
                s->inflight.push_back(e);
            }
        }
    }
    // nothing resident or queued: let every pending read-back land
    if (rc == ISING_OK && s->sched.active() == 0 && s->sched.queued() == 0) rc = wait_idle(s);
    if (active) *active = s->sched.active();
    return rc;
}

int ising_server_poll(ising_server* s, ising_result* out, int32_t cap, int32_t* n) {
    if (!s || !n || (cap > 0 && !out)) return fail(ISING_EINVAL, "ising_server_poll: null argument");
    int rc = harvest_all(s, false);
    if (rc != ISING_OK) return rc;
    const int32_t k = std::max<int32_t>(0, std::min<int32_t>(cap, (int32_t)s->done.size()));
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

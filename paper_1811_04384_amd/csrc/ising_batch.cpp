// Batch engine: many independent lattices of mixed L and T advanced together.
//
// Three execution paths, chosen per lattice by the plan (results never depend
// on it because every random number is a function of (seed, sweep, site)):
//  - half-sweep launches: per half-sweep, one launch over a table of
//    wavefronts covering every such lattice (each wavefront belongs to one
//    lattice);
//  - resident: one workgroup per lattice runs all sweeps of a chunk inside
//    one launch, colours separated by workgroup barriers, the lattice kept in
//    LDS when it fits;
//  - multi-sweep tiles: several sweeps per launch on LDS tiles of word
//    columns with redundant halos, one workgroup per tile, tiles of all such
//    lattices in one launch.
// A chunk of sweeps is captured once into a hipGraph (the half-sweep
// launches on one branch, resident and tile work on the other) and
// replayed; per-call parameters live in device memory so replays need no
// re-capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ising_host.hpp"
#include "ising_launch.hpp"

using namespace ising;

struct ising_batch {
    int32_t n = 0;
    std::vector<Geometry> geo;
    std::vector<uint64_t> seed;
    std::vector<size_t> offset;  // byte offset of each lattice in the arena
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;  // caller's stream
    hipStream_t cap = nullptr;     // private capture stream
    hipStream_t side = nullptr;    // second branch of a captured chunk
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, stage_ev = nullptr;
    bool stage_pending = false;
    int device = 0;
    std::string arch;
    LatticeDesc* d_desc = nullptr;
    LatticeState* d_state = nullptr;
    LatticeDesc* h_desc = nullptr;  // pinned staging of the descriptors
    std::vector<uint64_t> t_host;
    ising_batch_plan plan{};
    // derived from the plan
    std::vector<int32_t> resident;  // 0 half-sweep launches, 1 resident in LDS, 2 resident in global memory, 3 tiles,
                                    // 4 resident tiles, 5 codes drawn chip-wide
    std::vector<int64_t> units;
    std::vector<int32_t> part_begin, part_count;
    WaveItem* d_waves = nullptr;
    int64_t n_waves = 0;
    Partial* d_partials = nullptr;
    int32_t* d_ids_lds = nullptr;
    int32_t n_lds = 0;
    size_t lds_bytes = 0;
    int32_t* d_ids_glb = nullptr;
    int32_t n_glb = 0;
    int32_t n_tiled = 0;  // lattices advanced by half-sweep launches
    bool off32 = true;  // every such lattice < 4 GiB
    // multi-sweep tiles
    TileWork* d_tiles = nullptr;
    int32_t n_tiles = 0;
    Partial* d_tile_part = nullptr;  // kTileMaxSweeps x n_tiles
    uint64_t* d_halo = nullptr;      // n_tiles x halo_stride: halo copies of the tiles narrower than their lattice
    int64_t halo_stride = 0;
    int32_t* d_ids_tile = nullptr;
    int32_t n_tile_lat = 0;
    std::vector<std::pair<Geometry, int32_t>> tile_shapes;  // distinct (geometry, tile width) of the tiles
    // resident tiles trading boundary words (plan.tile_exchange)
    PersistTile* d_res = nullptr;
    int32_t n_res = 0;
    size_t res_lds = 0;
    uint64_t* d_exch = nullptr;
    int64_t exch_tile_words = 0;
    uint64_t* d_flags = nullptr;
    uint32_t* d_err = nullptr;
    Partial* d_res_part = nullptr;  // sweeps_per_graph x n_res
    int32_t* d_ids_res = nullptr;
    int32_t n_res_lat = 0;
    // small resident lattices whose codes are drawn chip-wide (plan.draw_sweeps)
    DrawLat* d_draw = nullptr;
    int32_t n_draw = 0;
    int32_t draw_max_items = 0;  // largest n_draw of the list
    int32_t draw_S = 0;          // sweeps per draw pass
    int32_t draw_wmax = 0;       // words of a colour per thread of an apply workgroup
    size_t draw_lds = 0;
    uint64_t* d_codes = nullptr;
    uint8_t* d_stage = nullptr;  // spin output staging, spin_stage_bytes of the largest L
    size_t stage_bytes = 0;
    std::map<std::pair<int32_t, int32_t>, hipGraphExec_t> graphs;  // (sweeps, every) -> executable
};

namespace {

template <class T>
void free_dev(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void drop_graphs(ising_batch* b) {
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

void release(ising_batch* b) {
    if (!b) return;
    drop_graphs(b);
    free_dev(b->arena);
    free_dev(b->d_desc);
    free_dev(b->d_state);
    free_dev(b->d_waves);
    free_dev(b->d_partials);
    free_dev(b->d_ids_lds);
    free_dev(b->d_ids_glb);
    free_dev(b->d_stage);
    free_dev(b->d_tiles);
    free_dev(b->d_tile_part);
    free_dev(b->d_halo);
    free_dev(b->d_ids_tile);
    free_dev(b->d_res);
    free_dev(b->d_exch);
    free_dev(b->d_flags);
    free_dev(b->d_err);
    free_dev(b->d_res_part);
    free_dev(b->d_ids_res);
    free_dev(b->d_draw);
    free_dev(b->d_codes);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->join_ev) (void)hipEventDestroy(b->join_ev);
    if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
}

size_t lattice_bytes(const Geometry& g) { return (size_t)g.N * (size_t)g.L * sizeof(uint64_t); }

// Largest L a plan may mark resident (one workgroup per lattice).  The
// lattices of the largest such size (N = 196, 6.4 MB) no longer fit in LDS
// and are already far slower with one workgroup each than tiled; larger ones
// would put a multi-gigabyte lattice on a single workgroup.
constexpr int32_t kResidentMaxL = 4096;
// Sweeps per chip-wide draw pass, and the largest code buffer it may use.
constexpr int32_t kMaxDrawSweeps = 4096;
constexpr size_t kMaxDrawBytes = size_t(256) << 20;

int check_plan(const ising_batch_plan& p) {
    if (p.resident_max_L < 0 || p.resident_max_L > kResidentMaxL)
        return fail(ISING_EINVAL, "plan: resident_max_L must be in [0, %d] (got %d)", kResidentMaxL, p.resident_max_L);
    if (!valid_block(p.resident_block, 1024)) return fail(ISING_EINVAL, "plan: resident_block must be a multiple of 64 in [64, 1024]");
    if (p.words_per_thread != 1 && p.words_per_thread != 2 && p.words_per_thread != 4)
        return fail(ISING_EINVAL, "plan: words_per_thread must be 1, 2 or 4");
    if (!valid_block(p.tiled_block, 256)) return fail(ISING_EINVAL, "plan: tiled_block must be a multiple of 64 in [64, 256]");
    if (p.sweeps_per_graph < 1 || p.sweeps_per_graph > 100000) return fail(ISING_EINVAL, "plan: sweeps_per_graph must be in [1, 100000]");
    if (p.tile_max_L < 0 || p.tile_max_L > kMaxL) return fail(ISING_EINVAL, "plan: tile_max_L must be in [0, %d]", kMaxL);
    if (p.draw_sweeps < 0 || p.draw_sweeps > kMaxDrawSweeps)
        return fail(ISING_EINVAL, "plan: draw_sweeps must be in [0, %d]", kMaxDrawSweeps);
    if (p.tile_max_L > 0) {
        if (p.tile_sweeps < 1 || p.tile_sweeps > kTileMaxSweeps)
            return fail(ISING_EINVAL, "plan: tile_sweeps must be in [1, %d]", kTileMaxSweeps);
        if (p.tile_cols < 2 || p.tile_cols % 2) return fail(ISING_EINVAL, "plan: tile_cols must be even and >= 2");
        if (!valid_block(p.tile_block, 1024)) return fail(ISING_EINVAL, "plan: tile_block must be a multiple of 64 in [64, 1024]");
        if (p.tile_exchange != 0 && p.tile_exchange != 1) return fail(ISING_EINVAL, "plan: tile_exchange must be 0 or 1");
    }
    return ISING_OK;
}

// Interior width of lattice g's tiles under plan p (g.L: the whole lattice
// in one workgroup), or 0 if its tiles do not fit in LDS.
int32_t tile_width(const Geometry& g, const ising_batch_plan& p, size_t lds_limit) {
    int32_t w = p.tile_cols >= g.L ? g.L : p.tile_cols;
    if (w < g.L && w + 4 * p.tile_sweeps > g.L) w = g.L;  // the halos would overlap: whole lattice
    return tile_lds_bytes(g.L, g.N, w, p.tile_sweeps) <= lds_limit ? w : 0;
}

// Threads per apply workgroup of the lattices whose codes are drawn chip-wide.
int32_t apply_block(const ising_batch_plan& p) { return std::min(p.resident_block, 256); }

size_t tile_launch_lds(const ising_batch* b, int32_t K) {
    size_t m = 0;
    for (const auto& gw : b->tile_shapes) m = std::max(m, tile_lds_bytes(gw.first.L, gw.first.N, gw.second, K));
    return m;
}

// Upload the descriptors (pinned staging; the previous upload must have
// completed before the staging buffer is rewritten).
int upload_descs(ising_batch* b, const double* T, int64_t* dev_E, int64_t* dev_M, int64_t samples_per_lattice) {
    if (b->stage_pending) {
        ISING_HIP(hipEventSynchronize(b->stage_ev));
        b->stage_pending = false;
    }
    for (int32_t i = 0; i < b->n; ++i) {
        LatticeDesc& d = b->h_desc[i];
        const Geometry& g = b->geo[i];
        d.W = reinterpret_cast<uint64_t*>(b->arena + b->offset[i]);
        d.L = g.L;
        d.N = g.N;
        d.istar = g.istar;
        d.sh_star = g.sh_star;
        d.k0 = (uint32_t)b->seed[i];
        d.k1 = (uint32_t)(b->seed[i] >> 32);
        if (T) thresholds_of(T[i], &d.t4, &d.t8);
        else d.t4 = d.t8 = 0;
        d.units = b->units.empty() ? 0 : b->units[i];
        d.segs = segments_per_row(g.L, b->plan.words_per_thread);
        d.resident = b->resident.empty() ? 0 : (b->resident[i] != 0);
        d.part_begin = b->part_begin.empty() ? 0 : b->part_begin[i];
        d.part_count = b->part_count.empty() ? 0 : b->part_count[i];
        d.sweep_limit = 0x7FFFFFFF;
        d.pad_ = 0;
        d.series_E = dev_E ? dev_E + (int64_t)i * samples_per_lattice : nullptr;
        d.series_M = dev_M ? dev_M + (int64_t)i * samples_per_lattice : nullptr;
    }
    ISING_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(LatticeDesc) * b->n, hipMemcpyHostToDevice, b->stream));
    ISING_HIP(hipEventRecord(b->stage_ev, b->stream));
    b->stage_pending = true;
    return ISING_OK;
}

int apply_plan(ising_batch* b, const ising_batch_plan& p) {
    int rc = check_plan(p);
    if (rc != ISING_OK) return rc;
    ISING_HIP(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    free_dev(b->d_waves);
    free_dev(b->d_partials);
    free_dev(b->d_ids_lds);
    free_dev(b->d_ids_glb);
    free_dev(b->d_tiles);
    free_dev(b->d_tile_part);
    free_dev(b->d_halo);
    free_dev(b->d_ids_tile);
    free_dev(b->d_res);
    free_dev(b->d_exch);
    free_dev(b->d_flags);
    free_dev(b->d_res_part);
    free_dev(b->d_ids_res);
    free_dev(b->d_draw);
    free_dev(b->d_codes);
    b->n_draw = 0;
    b->n_res = 0;
    b->n_res_lat = 0;
    b->res_lds = 0;
    b->tile_shapes.clear();
    b->plan = p;
    const size_t res_limit = persist_lds_limit(b->device);
    std::vector<int32_t> ids_res;
    std::vector<PersistTile> res_tiles;
    int32_t res_max_N = 0;
    const size_t lds_limit = resident_lds_limit(b->device);
    const size_t tile_limit = tile_lds_limit(b->device);
    std::vector<int32_t> ids_tile;
    std::vector<TileWork> tiles;
    int64_t halo_stride = 0;
    b->resident.assign(b->n, 0);
    b->units.assign(b->n, 0);
    b->part_begin.assign(b->n, 0);
    b->part_count.assign(b->n, 0);
    std::vector<int32_t> ids_lds, ids_glb, ids_draw;
    std::vector<WaveItem> waves;
    size_t max_lds = 0;
    b->off32 = true;
    for (int32_t i = 0; i < b->n; ++i) {
        const Geometry& g = b->geo[i];
        if (g.L <= p.resident_max_L) {
            if (p.draw_sweeps > 0 && wave_apply_words_per_thread(g.L, g.N, apply_block(p)) > 0 &&
                wave_apply_lds_bytes(g.N * g.L, p.draw_sweeps) <= lds_limit) {
                b->resident[i] = 5;
                ids_draw.push_back(i);
            } else if (lattice_bytes(g) <= lds_limit) {
                b->resident[i] = 1;
                ids_lds.push_back(i);
                max_lds = std::max(max_lds, lattice_bytes(g));
            } else {
                b->resident[i] = 2;
                ids_glb.push_back(i);
            }
            continue;
        }
        if (g.L <= p.tile_max_L && p.tile_exchange) {
            // resident tiles, as long as all of them fit on the device at once
            const int32_t w = p.tile_cols >= g.L ? g.L : p.tile_cols;
            const size_t lds = persist_lds_bytes(g.L, g.N, w, p.tile_block);
            int64_t capacity = 0;
            if (lds <= res_limit) ISING_HIP(persist_capacity(p.tile_block, std::max(lds, b->res_lds), b->device, &capacity));
            const int32_t nt = (g.L + w - 1) / w;
            if (lds <= res_limit && (int64_t)res_tiles.size() + nt <= capacity) {
                b->resident[i] = 4;
                ids_res.push_back(i);
                b->part_begin[i] = (int32_t)res_tiles.size();
                b->part_count[i] = nt;
                const int32_t base = (int32_t)res_tiles.size();
                for (int32_t t = 0; t < nt; ++t) {
                    const int32_t c0 = t * w;
                    res_tiles.push_back({i, c0, std::min(w, g.L - c0), base + (t + nt - 1) % nt, base + (t + 1) % nt,
                                         base + t});
                }
                b->res_lds = std::max(b->res_lds, lds);
                res_max_N = std::max(res_max_N, g.N);
                continue;
            }
        }
        const int32_t tw = g.L <= p.tile_max_L && !p.tile_exchange ? tile_width(g, p, tile_limit) : 0;
        if (tw > 0) {
            b->resident[i] = 3;
            ids_tile.push_back(i);
            b->part_begin[i] = (int32_t)tiles.size();
            for (int32_t c0 = 0; c0 < g.L; c0 += tw)
                tiles.push_back({i, c0, std::min(tw, g.L - c0), (int32_t)tiles.size()});
            if (tw < g.L) halo_stride = std::max(halo_stride, tile_halo_stride(g.N, p.tile_sweeps));
            b->part_count[i] = (int32_t)tiles.size() - b->part_begin[i];
            bool seen = false;
            for (const auto& gw : b->tile_shapes) seen = seen || (gw.first.L == g.L && gw.second == tw);
            if (!seen) b->tile_shapes.push_back({g, tw});
            continue;
        }
        const int64_t u = units_per_colour(g, p.words_per_thread);
        b->units[i] = u;
        b->off32 = b->off32 && fits_off32(g);
        b->part_begin[i] = (int32_t)waves.size();
        const int32_t segs = segments_per_row(g.L, p.words_per_thread);
        for (int32_t I = 0; I < g.N; ++I)
            for (int32_t s0 = 0; s0 < segs; s0 += 64) waves.push_back({i, I, s0});
        b->part_count[i] = (int32_t)waves.size() - b->part_begin[i];
    }
    b->n_waves = (int64_t)waves.size();
    b->n_lds = (int32_t)ids_lds.size();
    b->n_glb = (int32_t)ids_glb.size();
    b->n_tile_lat = (int32_t)ids_tile.size();
    b->n_tiles = (int32_t)tiles.size();
    b->halo_stride = halo_stride;
    b->n_res_lat = (int32_t)ids_res.size();
    b->n_res = (int32_t)res_tiles.size();
    b->n_draw = (int32_t)ids_draw.size();
    b->n_tiled = b->n - b->n_lds - b->n_glb - b->n_tile_lat - b->n_res_lat - b->n_draw;
    b->lds_bytes = max_lds;
    if (!waves.empty()) {
        ISING_HIP(hipMalloc(&b->d_waves, sizeof(WaveItem) * waves.size()));
        ISING_HIP(hipMemcpy(b->d_waves, waves.data(), sizeof(WaveItem) * waves.size(), hipMemcpyHostToDevice));
        ISING_HIP(hipMalloc(&b->d_partials, sizeof(Partial) * waves.size()));
    }
    if (!ids_lds.empty()) {
        ISING_HIP(hipMalloc(&b->d_ids_lds, sizeof(int32_t) * ids_lds.size()));
        ISING_HIP(hipMemcpy(b->d_ids_lds, ids_lds.data(), sizeof(int32_t) * ids_lds.size(), hipMemcpyHostToDevice));
        ISING_HIP(set_resident_lds(p.words_per_thread, max_lds));
    }
    if (!ids_glb.empty()) {
        ISING_HIP(hipMalloc(&b->d_ids_glb, sizeof(int32_t) * ids_glb.size()));
        ISING_HIP(hipMemcpy(b->d_ids_glb, ids_glb.data(), sizeof(int32_t) * ids_glb.size(), hipMemcpyHostToDevice));
    }
    if (!res_tiles.empty()) {
        // consecutive workgroups go to the 8 XCDs in turn: with a tile count
        // that is a multiple of 8, give every XCD a run of consecutive tiles
        // (neighbours then trade words inside one XCD except at run ends)
        const int32_t n = (int32_t)res_tiles.size();
        if (n % 8 == 0) {
            const int32_t m = n / 8;
            auto block_of = [&](int32_t t) { return 8 * (t % m) + t / m; };
            std::vector<PersistTile> by_block(n);
            for (int32_t t = 0; t < n; ++t) {
                PersistTile q = res_tiles[t];
                q.left = block_of(q.left);
                q.right = block_of(q.right);
                by_block[block_of(t)] = q;
            }
            res_tiles.swap(by_block);
        }
        ISING_HIP(allow_persist_lds(b->device));
        b->exch_tile_words = 4 * (int64_t)res_max_N;
        ISING_HIP(hipMalloc(&b->d_res, sizeof(PersistTile) * res_tiles.size()));
        ISING_HIP(hipMemcpy(b->d_res, res_tiles.data(), sizeof(PersistTile) * res_tiles.size(), hipMemcpyHostToDevice));
        ISING_HIP(hipMalloc(&b->d_exch, sizeof(uint64_t) * (size_t)b->exch_tile_words * res_tiles.size()));
        ISING_HIP(hipMalloc(&b->d_flags, sizeof(uint64_t) * res_tiles.size()));
        ISING_HIP(hipMemset(b->d_flags, 0, sizeof(uint64_t) * res_tiles.size()));
        if (!b->d_err) {
            ISING_HIP(hipMalloc(&b->d_err, sizeof(uint32_t)));
            ISING_HIP(hipMemset(b->d_err, 0, sizeof(uint32_t)));
        }
        ISING_HIP(hipMalloc(&b->d_res_part, sizeof(Partial) * res_tiles.size() * (size_t)p.sweeps_per_graph));
        ISING_HIP(hipMalloc(&b->d_ids_res, sizeof(int32_t) * ids_res.size()));
        ISING_HIP(hipMemcpy(b->d_ids_res, ids_res.data(), sizeof(int32_t) * ids_res.size(), hipMemcpyHostToDevice));
    }
    if (!ids_draw.empty()) {
        // codes of draw_S sweeps of every such lattice per draw pass
        std::vector<DrawLat> dl;
        int64_t words = 0;
        int32_t max_NL = 0;
        b->draw_max_items = 0;
        b->draw_wmax = 1;
        for (int32_t i : ids_draw) {
            const Geometry& g = b->geo[i];
            dl.push_back({i, 2 * g.N * ((g.L + 7) / 8), 0});
            words += (int64_t)g.N * g.L;
            max_NL = std::max(max_NL, g.N * g.L);
            b->draw_max_items = std::max(b->draw_max_items, dl.back().n_draw);
            b->draw_wmax = std::max(b->draw_wmax, wave_apply_words_per_thread(g.L, g.N, apply_block(p)));
        }
        b->draw_S = (int32_t)std::min<int64_t>(p.draw_sweeps, std::max<int64_t>(1, (int64_t)(kMaxDrawBytes / 8) / words));
        int64_t base = 0;
        for (auto& e : dl) {
            e.base = base;
            base += (int64_t)b->draw_S * b->geo[e.lat].N * b->geo[e.lat].L;
        }
        b->draw_lds = wave_apply_lds_bytes(max_NL, b->draw_S);
        ISING_HIP(allow_wave_apply_lds(b->device));
        ISING_HIP(hipMalloc(&b->d_draw, sizeof(DrawLat) * dl.size()));
        ISING_HIP(hipMemcpy(b->d_draw, dl.data(), sizeof(DrawLat) * dl.size(), hipMemcpyHostToDevice));
        ISING_HIP(hipMalloc(&b->d_codes, sizeof(uint64_t) * (size_t)base));
    }
    if (!tiles.empty()) {
        ISING_HIP(allow_tile_lds(b->device));
        ISING_HIP(hipMalloc(&b->d_tiles, sizeof(TileWork) * tiles.size()));
        ISING_HIP(hipMemcpy(b->d_tiles, tiles.data(), sizeof(TileWork) * tiles.size(), hipMemcpyHostToDevice));
        ISING_HIP(hipMalloc(&b->d_tile_part, sizeof(Partial) * tiles.size() * kTileMaxSweeps));
        if (halo_stride > 0) ISING_HIP(hipMalloc(&b->d_halo, sizeof(uint64_t) * tiles.size() * (size_t)halo_stride));
        ISING_HIP(hipMalloc(&b->d_ids_tile, sizeof(int32_t) * ids_tile.size()));
        ISING_HIP(hipMemcpy(b->d_ids_tile, ids_tile.data(), sizeof(int32_t) * ids_tile.size(), hipMemcpyHostToDevice));
    }
    return upload_descs(b, nullptr, nullptr, nullptr, 0);
}

// Enqueue one chunk of k sweeps (sample after local sweeps s with
// (s + 1) % every == 0) on stream s0, resident work on stream s1.
int enqueue_chunk(ising_batch* b, int32_t k, int32_t every, hipStream_t s0, hipStream_t s1) {
    const ising_batch_plan& p = b->plan;
    const bool fork =
        (b->n_lds + b->n_glb + b->n_tile_lat + b->n_res_lat + b->n_draw) > 0 && b->n_tiled > 0 && s1 != nullptr;
    hipStream_t rs = fork ? s1 : s0;
    if (fork) {
        ISING_HIP(hipEventRecord(b->fork_ev, s0));
        ISING_HIP(hipStreamWaitEvent(s1, b->fork_ev, 0));
    }
    if (b->n_lds)
        ISING_HIP(launch_resident(p.words_per_thread, p.resident_block, b->d_desc, b->d_state, b->d_ids_lds, b->n_lds,
                                  k, every, b->lds_bytes, rs));
    if (b->n_glb)
        ISING_HIP(launch_resident(p.words_per_thread, p.resident_block, b->d_desc, b->d_state, b->d_ids_glb, b->n_glb,
                                  k, every, 0, rs));
    // codes drawn chip-wide, then applied, draw_S sweeps at a time
    for (int32_t done = 0; b->n_draw && done < k; done += b->draw_S) {
        const int32_t S = std::min(b->draw_S, k - done);
        ISING_HIP(launch_draw_codes(b->d_desc, b->d_state, b->d_draw, b->n_draw, b->draw_max_items, b->d_codes, done,
                                    S, rs));
        ISING_HIP(launch_wave_apply(b->draw_wmax, apply_block(p), b->d_desc, b->d_state, b->d_draw, b->n_draw,
                                    b->d_codes, done, S, every, b->draw_lds, rs));
    }
    // A measured sweep s is finalized by the next launch on s0: the colour-0
    // half-sweep of sweep s + 1, or the chunk's end.
    auto measured = [&](int32_t s) { return every > 0 && s >= 0 && (s + 1) % every == 0; };
    // resident tiles: the whole chunk in one launch, its samples finalized
    // right behind it on the same branch (chunks hold a multiple of `every`
    // sweeps, so chunk-local sampling is the call's)
    if (b->n_res_lat) {
        PersistLaunch a = {};
        a.tiles = b->d_res;
        a.descs = b->d_desc;
        a.states = b->d_state;
        a.sweep_off = 0;
        a.K = k;
        a.every = every;
        a.sample_base = 0;
        a.n_tiles = b->n_res;
        a.partials = b->d_res_part;
        a.exch = b->d_exch;
        a.exch_tile_words = b->exch_tile_words;
        a.flags = b->d_flags;
        a.error = b->d_err;
        a.wait_ticks = 100000000ull;  // one second of the 100 MHz clock
        ISING_HIP(launch_persist(a, b->n_res, p.tile_block, b->res_lds, rs));
        if (every > 0)
            ISING_HIP(launch_finalize_resident(b->d_desc, b->d_state, b->d_ids_res, b->n_res_lat, b->d_res_part,
                                               b->n_res, k / every, rs));
    }
    // tiles: up to tile_sweeps sweeps per launch, the launch's samples
    // finalized right behind it on the same branch
    for (int32_t done = 0; b->n_tile_lat && done < k;) {
        const int32_t kb = std::min(p.tile_sweeps, k - done);
        uint32_t mask = 0;
        for (int32_t j = 0; j < kb; ++j)
            if (measured(done + j)) mask |= 1u << j;
        TileLaunch a = {};
        a.tiles = b->d_tiles;
        a.descs = b->d_desc;
        a.states = b->d_state;
        a.sweep_off = (uint32_t)done;
        a.K = kb;
        a.sample_mask = mask;
        a.n_tiles = b->n_tiles;
        a.partials = b->d_tile_part;
        ISING_HIP(launch_tiles(a, b->n_tiles, p.tile_block, tile_launch_lds(b, kb), b->d_halo, b->halo_stride, rs));
        ISING_HIP(launch_finalize_tiles(b->d_desc, b->d_state, b->d_ids_tile, b->n_tile_lat, b->d_tile_part,
                                        b->n_tiles, mask, (uint32_t)done, rs));
        done += kb;
    }
    if (b->n_tiled) {
        for (int32_t s = 0; s < k; ++s) {
            ISING_HIP(launch_halfsweep_multi(p.words_per_thread, p.tiled_block, b->d_desc, b->d_state, b->d_waves,
                                             b->n_waves, 0, (uint32_t)s, nullptr,
                                             measured(s - 1) ? b->d_partials : nullptr, (uint32_t)(s - 1), b->off32,
                                             s0));
            ISING_HIP(launch_halfsweep_multi(p.words_per_thread, p.tiled_block, b->d_desc, b->d_state, b->d_waves,
                                             b->n_waves, 1, (uint32_t)s, measured(s) ? b->d_partials : nullptr,
                                             nullptr, 0, b->off32, s0));
        }
    }
    if (fork) {
        ISING_HIP(hipEventRecord(b->join_ev, s1));
        ISING_HIP(hipStreamWaitEvent(s0, b->join_ev, 0));
    }
    const bool fin_last = b->n_tiled > 0 && measured(k - 1);
    ISING_HIP(launch_chunk_end(b->d_desc, b->d_state, b->n, fin_last ? b->d_partials : nullptr, (uint32_t)(k - 1),
                               (uint32_t)k, s0));
    return ISING_OK;
}

int get_graph(ising_batch* b, int32_t k, int32_t every, hipGraphExec_t* out) {
    auto it = b->graphs.find({k, every});
    if (it != b->graphs.end()) {
        *out = it->second;
        return ISING_OK;
    }
    ISING_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_chunk(b, k, every, b->cap, b->side);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (rc != ISING_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    b->graphs[{k, every}] = exec;
    *out = exec;
    return ISING_OK;
}

int32_t chunk_sweeps(const ising_batch* b, int32_t every) {
    int32_t K = b->plan.sweeps_per_graph;
    if (every > 0) K = std::max(every, (K / every) * every);
    return K;
}

int sweep_impl(ising_batch* b, const double* T, int64_t n, int32_t every, int64_t* dev_E, int64_t* dev_M) {
    if (!b || !T) return fail(ISING_EINVAL, "ising_batch_sweep: null argument");
    if (n < 0) return fail(ISING_EINVAL, "ising_batch_sweep: n_sweeps must be >= 0");
    if (every < 0) return fail(ISING_EINVAL, "ising_batch_sweep: every must be >= 0");
    if ((dev_E || dev_M) && every == 0) return fail(ISING_EINVAL, "ising_batch_sweep: series need every >= 1");
    for (int32_t i = 0; i < b->n; ++i)
        if (!valid_T(T[i])) return fail(ISING_EINVAL, "ising_batch_sweep: T[%d] must be finite and > 0", i);
    const int64_t samples = every > 0 ? n / every : 0;
    int rc = upload_descs(b, T, dev_E, dev_M, samples);
    if (rc != ISING_OK) return rc;
    ISING_HIP(launch_begin_call(b->d_state, b->n, b->stream));
    const int32_t K = chunk_sweeps(b, every);
    for (int64_t done = 0; done < n;) {
        const int32_t k = (int32_t)std::min<int64_t>(K, n - done);
        hipGraphExec_t g = nullptr;
        rc = get_graph(b, k, every, &g);
        if (rc != ISING_OK) return rc;
        if (b->n_res > 0)  // the chunk holds resident tiles
            ISING_HIP(resident_gate(b->device, b->stream, [&] { return hipGraphLaunch(g, b->stream); }));
        else
            ISING_HIP(hipGraphLaunch(g, b->stream));
        done += k;
    }
    for (auto& t : b->t_host) t += (uint64_t)n;
    return ISING_OK;
}

int create_impl(int32_t n, const int32_t* L, const uint64_t* seed, const int32_t* init, void* stream,
                ising_batch** out, const ising_batch_plan* plan) {
    if (!out) return fail(ISING_EINVAL, "ising_batch_create: null output");
    *out = nullptr;
    if (n < 1 || !L || !seed || !init) return fail(ISING_EINVAL, "ising_batch_create: need n >= 1 and non-null arrays");
    for (int32_t i = 0; i < n; ++i) {
        if (!valid_L(L[i])) return fail(ISING_EINVAL, "ising_batch_create: L[%d] = %d invalid (even, 4..%d)", i, L[i], kMaxL);
        if (init[i] != ISING_COLD && init[i] != ISING_HOT) return fail(ISING_EINVAL, "ising_batch_create: init[%d] must be 0 or 1", i);
    }
    ising_batch* b = new (std::nothrow) ising_batch();
    if (!b) return fail(ISING_ENOMEM, "ising_batch_create: host allocation failed");
    b->n = n;
    b->stream = (hipStream_t)stream;
    b->geo.resize(n);
    b->seed.assign(seed, seed + n);
    b->offset.resize(n);
    b->t_host.assign(n, 0);
    size_t off = 0;
    for (int32_t i = 0; i < n; ++i) {
        b->geo[i] = make_geometry(L[i]);
        b->offset[i] = off;
        off += (lattice_bytes(b->geo[i]) + 255) & ~(size_t)255;
    }
    b->arena_bytes = off;
    hipError_t e = hipGetDevice(&b->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, b->device);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "ising_batch_create: device query");
    }
    b->arch = prop.gcnArchName;
    b->arch = b->arch.substr(0, b->arch.find(':'));
    e = hipMalloc(&b->arena, b->arena_bytes);
    if (e != hipSuccess) {
        b->arena = nullptr;
        release(b);
        return fail(ISING_ENOMEM, "ising_batch_create: hipMalloc of %zu bytes failed", off);
    }
    for (int32_t i = 0; i < n; ++i) b->stage_bytes = std::max(b->stage_bytes, spin_stage_bytes(L[i]));
    if (e == hipSuccess) e = hipMalloc(&b->d_stage, b->stage_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_desc, sizeof(LatticeDesc) * n);
    if (e == hipSuccess) e = hipMalloc(&b->d_state, sizeof(LatticeState) * n);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_desc, sizeof(LatticeDesc) * n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_state, 0, sizeof(LatticeState) * n, b->stream);
    for (int32_t i = 0; i < n && e == hipSuccess; ++i)
        e = launch_init(reinterpret_cast<uint64_t*>(b->arena + b->offset[i]), b->geo[i], seed[i], init[i], b->stream);
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "ising_batch_create");
    }
    ising_batch_plan p;
    if (plan) {
        p = *plan;
    } else {
        // default: lattices that fit in one workgroup's LDS are resident
        const size_t lim = resident_lds_limit(b->device);
        p.resident_max_L = 0;
        for (int32_t i = 0; i < n; ++i)
            if (lattice_bytes(b->geo[i]) <= lim && b->geo[i].L <= 256) p.resident_max_L = std::max(p.resident_max_L, b->geo[i].L);
        p.resident_block = 256;
        p.words_per_thread = 1;
        p.tiled_block = 64;  // fastest measured for small and large batches alike
        p.sweeps_per_graph = 50;
        p.tile_max_L = 0;
        p.tile_sweeps = 2;
        p.tile_cols = 16;
        p.tile_block = 256;
        p.tile_exchange = 0;
        // the smallest lattices (up to 1024 words of a colour) have their
        // codes drawn chip-wide; a batch of nothing else runs 500 sweeps per
        // graph (8 x L = 64 to 2048 x L = 64 measured 2-4x faster than
        // drawing in each lattice's workgroup)
        p.draw_sweeps = 0;
        bool all_drawn = true;
        for (int32_t i = 0; i < n; ++i) {
            const Geometry& g = b->geo[i];
            const bool drawn = g.L <= p.resident_max_L && wave_apply_words_per_thread(g.L, g.N, 256) > 0 &&
                               wave_apply_lds_bytes(g.N * g.L, 500) <= lim;
            if (drawn) p.draw_sweeps = 500;
            all_drawn = all_drawn && drawn;
        }
        if (all_drawn) p.sweeps_per_graph = 500;
    }
    int rc = apply_plan(b, p);
    if (rc != ISING_OK) {
        release(b);
        return rc;
    }
    *out = b;
    return ISING_OK;
}

std::string cache_key(const ising_batch* b) {
    std::map<int32_t, int32_t> hist;
    for (const auto& g : b->geo) hist[g.L] += 1;
    std::ostringstream os;
    os << b->arch << "|plan4|";
    bool first = true;
    for (auto& kv : hist) {
        os << (first ? "" : ",") << kv.first << "x" << kv.second;
        first = false;
    }
    return os.str();
}

bool cache_lookup(const char* path, const std::string& key, ising_batch_plan* p) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string want = "\"" + key + "\":";
    while (std::getline(f, line)) {
        const size_t at = line.find(want);
        if (at == std::string::npos) continue;
        ising_batch_plan q;
        if (std::sscanf(line.c_str() + at + want.size(),
                        " {\"resident_max_L\": %d, \"resident_block\": %d, \"words_per_thread\": %d, \"tiled_block\": %d, "
                        "\"sweeps_per_graph\": %d, \"tile_max_L\": %d, \"tile_sweeps\": %d, \"tile_cols\": %d, "
                        "\"tile_block\": %d, \"tile_exchange\": %d, \"draw_sweeps\": %d",
                        &q.resident_max_L, &q.resident_block, &q.words_per_thread, &q.tiled_block, &q.sweeps_per_graph,
                        &q.tile_max_L, &q.tile_sweeps, &q.tile_cols, &q.tile_block, &q.tile_exchange,
                        &q.draw_sweeps) == 11) {
            *p = q;
            return true;
        }
    }
    return false;
}

void cache_store(const char* path, const std::string& key, const ising_batch_plan& p, double ms) {
    if (!path) return;
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line)) {
            if (line.find("\"" + key + "\":") != std::string::npos) continue;
            if (line.find("\":") == std::string::npos) continue;  // braces
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            lines.push_back(line);
        }
    }
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "\"%s\": {\"resident_max_L\": %d, \"resident_block\": %d, \"words_per_thread\": %d, \"tiled_block\": "
                  "%d, \"sweeps_per_graph\": %d, \"tile_max_L\": %d, \"tile_sweeps\": %d, \"tile_cols\": %d, "
                  "\"tile_block\": %d, \"tile_exchange\": %d, \"draw_sweeps\": %d, \"ms_per_sweep\": %.6f}",
                  key.c_str(), p.resident_max_L, p.resident_block, p.words_per_thread, p.tiled_block, p.sweeps_per_graph,
                  p.tile_max_L, p.tile_sweeps, p.tile_cols, p.tile_block, p.tile_exchange, p.draw_sweeps, ms);
    lines.push_back(buf);
    std::ofstream f(path, std::ios::trunc);
    f << "{\n";
    for (size_t i = 0; i < lines.size(); ++i) f << lines[i] << (i + 1 < lines.size() ? ",\n" : "\n");
    f << "}\n";
}

// Time `sweeps` sweeps of a scratch batch under plan p: best of two runs
// after a warm-up that captures the chunk graphs; ms per sweep.
int time_plan(ising_batch* s, const ising_batch_plan& p, const double* T, int32_t sweeps, double* ms_per_sweep,
              int32_t every = 0) {
    int rc = apply_plan(s, p);
    if (rc != ISING_OK) return rc;
    rc = sweep_impl(s, T, sweeps, every, nullptr, nullptr);  // captures every chunk length used below
    if (rc != ISING_OK) return rc;
    hipEvent_t e0, e1;
    ISING_HIP(hipEventCreate(&e0));
    ISING_HIP(hipEventCreate(&e1));
    double best = 1e300;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 2 && rc == ISING_OK && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s->stream);
        if (e == hipSuccess) rc = sweep_impl(s, T, sweeps, every, nullptr, nullptr);
        if (e == hipSuccess && rc == ISING_OK) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess && rc == ISING_OK) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && rc == ISING_OK) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rc == ISING_OK) best = std::min(best, (double)ms / sweeps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ISING_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *ms_per_sweep = best;
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_batch_create(int32_t n, const int32_t* L, const uint64_t* seed, const int32_t* init, void* stream,
                       ising_batch** out) {
    return create_impl(n, L, seed, init, stream, out, nullptr);
}

int ising_batch_destroy(ising_batch* b) {
    if (!b) return ISING_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    release(b);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ISING_OK;
}

int ising_batch_sweep(ising_batch* b, const double* T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                      int64_t* dev_M) {
    return sweep_impl(b, T, n_sweeps, every, dev_E, dev_M);
}

// Error left by a resident-tile launch (read after the stream has been
// synchronised); cleared once reported.
static int resident_error(ising_batch* b) {
    if (!b->d_err) return ISING_OK;
    uint32_t err = 0;
    ISING_HIP(hipMemcpy(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost));
    if (!err) return ISING_OK;
    ISING_HIP(hipMemset(b->d_err, 0, sizeof err));
    return fail(ISING_EHIP, "batch: a resident-tile launch waited too long for a neighbour tile and was abandoned; "
                            "the states of its lattices are undefined");
}

int ising_batch_results(ising_batch* b, int64_t* E, int64_t* M, int64_t* sum_E, int64_t* sum_absM,
                        int64_t* n_samples) {
    if (!b) return fail(ISING_EINVAL, "ising_batch_results: null handle");
    if (E || M) ISING_HIP(launch_observe_multi(b->d_desc, b->d_state, nullptr, b->n, nullptr, b->stream));
    std::vector<LatticeState> st(b->n);
    ISING_HIP(hipMemcpyAsync(st.data(), b->d_state, sizeof(LatticeState) * b->n, hipMemcpyDeviceToHost, b->stream));
    ISING_HIP(hipStreamSynchronize(b->stream));
    const int rc = resident_error(b);
    if (rc != ISING_OK) return rc;
    for (int32_t i = 0; i < b->n; ++i) {
        if (E) E[i] = st[i].last_E;
        if (M) M[i] = st[i].last_M;
        if (sum_E) sum_E[i] = st[i].mom.sum_E;
        if (sum_absM) sum_absM[i] = st[i].mom.sum_absM;
        if (n_samples) n_samples[i] = st[i].mom.n;
    }
    return ISING_OK;
}

int ising_batch_reset_sums(ising_batch* b) {
    if (!b) return fail(ISING_EINVAL, "ising_batch_reset_sums: null handle");
    ISING_HIP(launch_reset_sums(b->d_state, b->n, b->stream));
    return ISING_OK;
}

int ising_batch_moments(ising_batch* b, ising_moments* out) {
    if (!b || !out) return fail(ISING_EINVAL, "ising_batch_moments: null argument");
    std::vector<LatticeState> st(b->n);
    ISING_HIP(hipMemcpyAsync(st.data(), b->d_state, sizeof(LatticeState) * b->n, hipMemcpyDeviceToHost, b->stream));
    ISING_HIP(hipStreamSynchronize(b->stream));
    const int rc = resident_error(b);
    if (rc != ISING_OK) return rc;
    for (int32_t i = 0; i < b->n; ++i) std::memcpy(&out[i], &st[i].mom, sizeof(ising_moments));
    return ISING_OK;
}

int ising_batch_scan(ising_batch* b, int32_t n_T, const double* T, int64_t therm, int64_t meas, int32_t every,
                     ising_moments* out) {
    if (!b) return fail(ISING_EINVAL, "ising_batch_scan: null handle");
    if (n_T < 0 || therm < 0 || meas < 0 || every < 1)
        return fail(ISING_EINVAL, "ising_batch_scan: need n_T, therm, meas >= 0 and every >= 1");
    if (n_T > 0 && (!T || !out)) return fail(ISING_EINVAL, "ising_batch_scan: null array");
    for (int64_t k = 0; k < (int64_t)n_T * b->n; ++k)
        if (!valid_T(T[k])) return fail(ISING_EINVAL, "ising_batch_scan: T[%lld] = %g is not finite and > 0",
                                        (long long)k, T[k]);
    for (int32_t j = 0; j < n_T; ++j) {
        const double* Tj = T + (size_t)j * b->n;
        int rc = sweep_impl(b, Tj, therm, 0, nullptr, nullptr);
        if (rc != ISING_OK) return rc;
        ISING_HIP(launch_reset_sums(b->d_state, b->n, b->stream));
        rc = sweep_impl(b, Tj, meas, every, nullptr, nullptr);
        if (rc != ISING_OK) return rc;
        rc = ising_batch_moments(b, out + (size_t)j * b->n);
        if (rc != ISING_OK) return rc;
    }
    return ISING_OK;
}

int ising_batch_get_spins_region(ising_batch* b, int32_t i, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols,
                                 uint8_t* host) {
    if (!b || !host) return fail(ISING_EINVAL, "ising_batch_get_spins_region: null argument");
    if (i < 0 || i >= b->n) return fail(ISING_EINVAL, "ising_batch_get_spins_region: index %d out of range", i);
    const Geometry& g = b->geo[i];
    const int32_t L = g.L;
    if (nrows < 1 || ncols < 1 || nrows > L || ncols > L)
        return fail(ISING_EINVAL, "ising_batch_get_spins_region: window %dx%d outside 1..L=%d", nrows, ncols, L);
    const int32_t rr = (int32_t)(((int64_t)r0 % L + L) % L), cc = (int32_t)(((int64_t)c0 % L + L) % L);
    return read_spin_window(reinterpret_cast<const uint64_t*>(b->arena + b->offset[i]), g, rr, cc, nrows, ncols, host,
                            b->d_stage, b->stage_bytes, b->stream);
}

int ising_batch_get_spins(ising_batch* b, int32_t i, uint8_t* host) {
    if (!b || !host) return fail(ISING_EINVAL, "ising_batch_get_spins: null argument");
    if (i < 0 || i >= b->n) return fail(ISING_EINVAL, "ising_batch_get_spins: index %d out of range", i);
    const Geometry& g = b->geo[i];
    return read_spin_window(reinterpret_cast<const uint64_t*>(b->arena + b->offset[i]), g, 0, 0, g.L, g.L, host,
                            b->d_stage, b->stage_bytes, b->stream);
}

int ising_batch_get_sweep_count(ising_batch* b, int32_t i, uint64_t* t) {
    if (!b || !t) return fail(ISING_EINVAL, "ising_batch_get_sweep_count: null argument");
    if (i < 0 || i >= b->n) return fail(ISING_EINVAL, "ising_batch_get_sweep_count: index %d out of range", i);
    *t = b->t_host[i];
    return ISING_OK;
}

int ising_batch_check_plan(const ising_batch_plan* plan) {
    if (!plan) return fail(ISING_EINVAL, "ising_batch_check_plan: null plan");
    return check_plan(*plan);
}

int ising_batch_set_plan(ising_batch* b, const ising_batch_plan* plan) {
    if (!b || !plan) return fail(ISING_EINVAL, "ising_batch_set_plan: null argument");
    return apply_plan(b, *plan);
}

int ising_batch_get_plan(ising_batch* b, ising_batch_plan* plan) {
    if (!b || !plan) return fail(ISING_EINVAL, "ising_batch_get_plan: null argument");
    *plan = b->plan;
    return ISING_OK;
}

int ising_batch_autotune(ising_batch* b, const double* T, const char* cache_path, ising_batch_plan* chosen) {
    if (!b || !T) return fail(ISING_EINVAL, "ising_batch_autotune: null argument");
    for (int32_t i = 0; i < b->n; ++i)
        if (!valid_T(T[i])) return fail(ISING_EINVAL, "ising_batch_autotune: T[%d] must be finite and > 0", i);
    const std::string key = cache_key(b);
    ising_batch_plan best;
    if (cache_lookup(cache_path, key, &best)) {
        int rc = apply_plan(b, best);
        if (rc == ISING_OK && chosen) *chosen = best;
        return rc;
    }
    // scratch batch of the same shapes (hot start, seeds = index)
    std::vector<int32_t> L(b->n), init(b->n, ISING_HOT);
    std::vector<uint64_t> seeds(b->n);
    double total_spins = 0;
    std::vector<int32_t> distinct;
    for (int32_t i = 0; i < b->n; ++i) {
        L[i] = b->geo[i].L;
        seeds[i] = (uint64_t)i;
        total_spins += (double)L[i] * L[i];
        distinct.push_back(L[i]);
    }
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    ISING_HIP(hipStreamSynchronize(b->stream));
    ising_batch* s = nullptr;
    ising_batch_plan p0 = b->plan;
    int rc = create_impl(b->n, L.data(), seeds.data(), init.data(), b->stream, &s, &p0);
    if (rc != ISING_OK) return rc;
    // about 50 ms of work per timing at ~2 attempts/ps, at least 20 sweeps
    const int32_t sweeps = (int32_t)std::max(20.0, std::min(2000.0, 1e11 / std::max(total_spins, 1.0)));
    double best_ms = 1e300;
    best = p0;
    std::vector<std::pair<double, ising_batch_plan>> seen;
    auto consider = [&](const ising_batch_plan& p) -> int {
        double ms = 0;
        int r = time_plan(s, p, T, sweeps, &ms);
        if (r != ISING_OK) return r;
        seen.push_back({ms, p});
        if (ms < best_ms) {
            best_ms = ms;
            best = p;
        }
        return ISING_OK;
    };
    // 1) tiled shape with everything tiled
    for (int wpt : {1, 2, 4})
        for (int blk : {64, 128, 256}) {
            if (rc != ISING_OK) break;
            ising_batch_plan p = best;
            p.resident_max_L = 0;
            p.tile_max_L = 0;
            p.words_per_thread = wpt;
            p.tiled_block = blk;
            p.sweeps_per_graph = std::min(sweeps, 20);
            rc = consider(p);
        }
    // 1b) multi-sweep tiles for every lattice (sweeps per launch, tile
    // width, workgroup size), then the largest L that stays on tiles
    const int32_t max_L = distinct.back();
    const ising_batch_plan half_best = best;
    for (int K : {1, 2, 4})
        for (int cols : {16, 32, 64})
            for (int blk : {256, 512}) {
                if (rc != ISING_OK) break;
                ising_batch_plan p = half_best;
                p.resident_max_L = 0;
                p.tile_max_L = max_L;
                p.tile_exchange = 0;
                p.tile_sweeps = K;
                p.tile_cols = cols;
                p.tile_block = blk;
                p.sweeps_per_graph = std::max(K, (std::min(sweeps, 20) / K) * K);
                rc = consider(p);
            }
    // 1c) resident tiles trading boundary words (tile width, workgroup size)
    for (int cols : {16, 32, 64})
        for (int blk : {256, 512, 1024}) {
            if (rc != ISING_OK) break;
            ising_batch_plan p = half_best;
            p.resident_max_L = 0;
            p.tile_max_L = max_L;
            p.tile_exchange = 1;
            p.tile_sweeps = 1;
            p.tile_cols = cols;
            p.tile_block = blk;
            p.sweeps_per_graph = std::min(sweeps, 50);
            rc = consider(p);
        }
    {
        const ising_batch_plan tile_best = best;
        if (tile_best.tile_max_L > 0)
            for (int32_t Lt : distinct) {
                if (rc != ISING_OK || Lt >= max_L) break;
                ising_batch_plan p = tile_best;
                p.tile_max_L = Lt;
                rc = consider(p);
            }
    }
    // 2) which sizes go resident, and the resident workgroup size: only sizes
    // whose lattice fits one workgroup's LDS are tried
    const ising_batch_plan tiled_best = best;
    const size_t lds_limit = resident_lds_limit(b->device);
    for (int32_t Lr : distinct)
        for (int rb : {256, 512, 1024}) {
            if (lattice_bytes(make_geometry(Lr)) > lds_limit) break;
            if (rc != ISING_OK) break;
            ising_batch_plan p = tiled_best;
            p.resident_max_L = Lr;
            p.resident_block = rb;
            rc = consider(p);
        }
    // 2b) the smallest lattices with their codes drawn chip-wide
    {
        const ising_batch_plan res_best = best;
        int32_t Ld = 0;
        for (int32_t L0 : distinct) {
            const Geometry g = make_geometry(L0);
            if (wave_apply_words_per_thread(g.L, g.N, 256) > 0 && wave_apply_lds_bytes(g.N * g.L, 1000) <= lds_limit)
                Ld = L0;
        }
        if (Ld > 0)
            for (int rb : {64, 128, 256})
                for (int ds : {100, 1000}) {
                    if (rc != ISING_OK) break;
                    ising_batch_plan p = res_best;
                    p.resident_max_L = std::max(res_best.resident_max_L, Ld);
                    p.resident_block = rb;
                    p.draw_sweeps = ds;
                    p.sweeps_per_graph = std::min(sweeps, 1000);
                    rc = consider(p);
                }
    }
    // 3) sweeps per graph
    const ising_batch_plan shape_best = best;
    for (int k : {10, 50, 100, 250, 1000}) {
        if (rc != ISING_OK) break;
        ising_batch_plan p = shape_best;
        p.sweeps_per_graph = std::min(k, sweeps);
        rc = consider(p);
    }
    // 4) the three fastest distinct plans again, three times as long and
    // sampling every 10 sweeps as a measured run does (a sampled sweep costs
    // the resident and the tiled kernels differently); short trials differ
    // by a few per cent of noise
    if (rc == ISING_OK) {
        std::stable_sort(seen.begin(), seen.end(),
                         [](const std::pair<double, ising_batch_plan>& x, const std::pair<double, ising_batch_plan>& y) {
                             return x.first < y.first;
                         });
        auto same = [](const ising_batch_plan& x, const ising_batch_plan& y) {
            return std::memcmp(&x, &y, sizeof x) == 0;
        };
        std::vector<ising_batch_plan> top;
        for (const auto& c : seen) {
            bool dup = false;
            for (const auto& q : top) dup = dup || same(q, c.second);
            if (!dup) top.push_back(c.second);
            if (top.size() == 3) break;
        }
        const int32_t every = 10;
        const int32_t long_sweeps = ((3 * sweeps + every - 1) / every) * every;
        double confirm_ms = 1e300;
        for (const auto& q : top) {
            double ms = 0;
            rc = time_plan(s, q, T, long_sweeps, &ms, every);
            if (rc != ISING_OK) break;
            if (ms < confirm_ms) {
                confirm_ms = ms;
                best = q;
                best_ms = ms;
            }
        }
    }
    ising_batch_destroy(s);
    if (rc != ISING_OK) return rc;
    rc = apply_plan(b, best);
    if (rc != ISING_OK) return rc;
    cache_store(cache_path, key, best, best_ms);
    if (chosen) *chosen = best;
    return ISING_OK;
}

}  // extern "C"

// sph_internal.h -- internal declarations of the MI355X SPH sweep library.
// Device helpers, the context object and the launch wrappers shared by the
// translation units of the library.  Nothing here is part of the C interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sph.h"

namespace sphmi {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kGroup = 64;         // sink group: one wavefront, one particle per lane
constexpr int kStackCap = 768;     // walk stack (node ids) of one wave
constexpr int kCandCap = 256;      // per-wave candidate-bucket list in LDS
constexpr int kMaxRow = 4096;      // longest neighbour row sph_neighbors can sort

// Device counters of the most recent call (all 64-bit, summed with integer
// atomics so totals do not depend on scheduling).
enum Counter {
    C_PAIRS_D = 0, C_PAIRS_F, C_CAND_D, C_CAND_F, C_NR_ITER_MAX, C_NR_SCANS,
    C_NOCONV, C_REWALK, C_OVERFLOW, C_ROWLONG,
    C_ITERLIM, C_NONFINITE,               // the status word (adjacent: copied together)
    C_RETEST,                             // mixed pairs re-tested in FP64 (exact membership)
    C_SLOTS_D, C_SLOTS_F,                 // candidate slots loaded (interaction-list lengths)
    C_LEV0, C_LEV1, C_LEV2, C_LEV3,       // force-pass sink groups per bucket level
    C_FGMISS,                             // FastGas: force pairs with a stale neighbour density
    C_WALKED,                             // sink groups left to the walking sweep kernels
    C_NTRANSIENT,                         // counters above are cleared by every call
    C_PAIRS_D_TOT = C_NTRANSIENT,         // running totals since the context was made
    C_PAIRS_F_TOT,
    C_NCOUNTERS
};

// Dynamic bucket sizing: level h of a bucket size (buckets of 8 2^h, h <= 3).
inline int base_level(int bucket) {
    int h = 0;
    while ((8 << h) < bucket && h < 3) ++h;
    return h;
}

// The counters are accumulated in kCntShards copies, each on a 256-byte line
// of its own (sink group g adds to copy g mod kCntShards): the sweeps end
// every wave with a handful of 64-bit atomics, which on a single line
// serialise in the L2 and hold the finishing waves back (measured: a third
// of the density pass at 2M particles).  A fold kernel sums the copies into
// the summary block the host reads (maximum for C_NR_ITER_MAX).
constexpr int kCntShards = 16;
constexpr int kCntStride = 32;   // 64-bit counters per copy
// Workgroups are dealt to the XCDs in turn; the persistent sweep launch keeps
// one queue counter per XCD, each on its own 256-byte line
constexpr int kXcds = 8;
constexpr int kQueueStride = 64;   // uint32 per queue counter
// Stored interaction lists (the walk kernels): up to kListChunks chunks of at
// most kCandCap refined buckets per sink group, and a header of kWalkWords:
// [0] chunks, [1] the chunks' minimum-image flags (a bit each), [2] kList*
// flags, [3 + c] the bucket count of chunk c
constexpr int kListChunks = 16;
constexpr int kListCap = kListChunks * kCandCap;
constexpr int kWalkWords = 3 + kListChunks;
static_assert(kListChunks <= 32, "minimum-image flags: one bit per chunk");
constexpr int kListLong = 1;       // more than kListChunks chunks: not stored
constexpr int kListLinear = 2;     // the walk outgrew its stack and ran as the linear test
static_assert(C_NCOUNTERS <= kCntStride, "counter copy too small");
__host__ __device__ inline int64_t cnt_shard(int64_t g) { return (g % kCntShards) * kCntStride; }

// A lane's value after a DPP move within its row of 16 lanes (CTRL: the DPP
// control word: 0xB1 and 0x4E swap neighbours and pairs of a quad, 0x141
// mirrors each half row, 0x140 the row).  The two halves of a double move
// separately.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    // (a lane whose source is not valid keeps its own value, which leaves a
    // minimum or maximum unchanged)
    const int l0 = (int)(b & 0xffffffffll), h0 = (int)(b >> 32);
    const int lo = __builtin_amdgcn_update_dpp(l0, l0, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(h0, h0, CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Minimum (MAX: maximum) over aligned segments of B lanes (B = 8, 16, 32 or
// 64), left in every lane of the segment: within a quad by two swaps, then
// each half row with its mirror (lane i meets lane 7 - i of the other quad),
// each row with its mirror, then across rows by lane shuffles.
template <bool MAX>
__device__ __forceinline__ double seg_reduce(double v, int B) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
    v = op(v, dpp_move<0xB1>(v));
    v = op(v, dpp_move<0x4E>(v));
    v = op(v, dpp_move<0x141>(v));
    if (B >= 16) v = op(v, dpp_move<0x140>(v));
    if (B >= 32) v = op(v, __shfl_xor(v, 16));
    if (B >= 64) v = op(v, __shfl_xor(v, 32));
    return v;
}

// Timing events recorded around the phases when timing is on.
enum TimingEvent {
    E_BEGIN = 0, E_TREE0, E_TREE1, E_DWALK0, E_DEN0, E_DEN1, E_FWALK0, E_FOR0, E_FOR1, E_END,
    E_NEVENTS
};

// FP64 results of the last step (device), copied into sph_stats.
struct StepReport {
    double momentum[3];
    double e_kin, e_int;
    double dt_next;   // min_i dt_i of the last force pass, capped by dt_max
    double dt_used;   // dt of the last step
    double pad;
};

// Individual time steps: the time T and the next step boundary in units of
// dt_max 2^-rung_max, the active and density-pass particle counts.
struct RungState {
    long long T, Tnext, nact, ndens;
};

// Per-set geometry shared by all kernels (device array, one entry per set).
struct SetGeom {
    double lo[3];     // box low corner (periodic) or key box (open)
    double L[3];      // box lengths (periodic) or key-box lengths (open)
    double halfL[3];  // L/2 (exact)
    int64_t p0, p1;   // particle range [p0, p1) (sorted order == caller set range)
    int64_t b0;       // first global bucket of the set
    int64_t g0;       // first global sink group of the set
    int64_t node0;    // node slot of heap index 0 (slots node0 + 1 .. node0 + 2*nbp - 1)
    int32_t nb;       // buckets in the set
    int32_t nbp;      // nb rounded up to a power of two (leaf count of the heap)
    int32_t depth;    // log2(nbp)
    int32_t pad;
};

// One tree node: cell bound (AABB of positions), box-of-balls (AABB of the
// kernel balls) and ball-of-balls (an enclosing sphere of the kernel balls),
// Sec. 2.3.2 and Fig. 1.  Empty nodes have clo > chi.
struct alignas(16) Node {
    double clo[3], chi[3];
    double blo[3], bhi[3];
    double bc[3], br;
};

struct Ctx {
    sph_params prm{};
    int32_t nsets = 1;
    std::vector<int64_t> set_off;   // host, nsets+1
    std::vector<double> set_box;    // host, 6*nsets (empty = params box)
    int32_t bucket = 32;
    int32_t topo_bucket = 0;        // bucket size the current allocation was laid out for
    int64_t n = 0;                  // particles of the current allocation
    int64_t nbuckets = 0, ngroups = 0, nnodes = 0;
    int32_t max_depth = 0;
    int32_t key_passes = 0;         // radix passes of 8 bits
    int32_t set_bits = 0;
    bool have_tree = false, have_forces = false;
    std::string err;
    hipStream_t last_stream = nullptr;

    // topology (device)
    SetGeom *d_sets = nullptr;
    int32_t *d_grp_set = nullptr;   // per group: set id
    int32_t *d_bkt_set = nullptr;   // per bucket: set id
    int64_t *d_level_pref = nullptr;// (max_depth+1) x (nsets+1) prefix of nodes per height
    std::vector<int64_t> level_total;

    // sort
    uint64_t *d_key[2] = {nullptr, nullptr};
    uint32_t *d_perm[2] = {nullptr, nullptr};
    uint32_t *d_hist = nullptr;     // 256 x sort blocks
    int64_t sort_blocks = 0;
    double *d_bbox = nullptr;       // per set: open-boundary key box (6 doubles)

    // sorted particle data (FP64)
    double *xs = nullptr, *ys = nullptr, *zs = nullptr, *ms = nullptr, *Hs = nullptr;
    double *vxs = nullptr, *vys = nullptr, *vzs = nullptr, *us = nullptr;
    double *rhos = nullptr, *oms = nullptr, *As = nullptr, *css = nullptr, *Ps = nullptr;
    // mixed path: FP32 force-pass records of every particle, written by the EOS
    // pass in sorted order: (vx vy vz H), (1/H A c rho), m
    float *frec1 = nullptr, *frec2 = nullptr, *fm = nullptr;
    // FP64 path: the same records in FP64, (vx vy vz H), (1/H A c rho)
    double *drec1 = nullptr, *drec2 = nullptr;
    double *axs = nullptr, *ays = nullptr, *azs = nullptr, *dus = nullptr, *dts = nullptr;
    // FP32 bucket-relative offsets for the mixed path

    Node *nodes = nullptr;

    // predictor scratch (caller order) for the step
    double *vpx = nullptr, *vpy = nullptr, *vpz = nullptr, *upred = nullptr;
    double *hprev = nullptr;   // caller order: converged H of the step before (0 = none)
    double *d_h0 = nullptr;    // caller order: the autotuner's copy of the first guess of H
    double *rho_old = nullptr; // caller order: density of the last step (entropy-conserving update)
    double *rho_pred = nullptr;// caller order: predicted density (evolved density)
    double *rho_sum = nullptr; // caller order: summed density of a step (evolved density)
    double *drs = nullptr;     // sorted: continuity rate of the force pass (evolved density)
    // interface correction (sorted): material ids, imbalance, averages
    double *mats = nullptr, *imbs = nullptr, *tbar = nullptr, *pbar = nullptr;
    // dynamic bucket sizing: the tree is built over buckets of 8; each group's
    // level h (buckets of 8 2^h) follows its list lengths from step to step
    bool dyn = false;
    int32_t base_bucket = 32;  // bucket size the levels start from
    double *levc = nullptr;    // caller order: level of each particle's group
    double *levs = nullptr;    // sorted
    double *d_levref = nullptr;// mean list length per pair of the last force pass (one value;
                               // kept off the counters' cache line, which the sweeps' atomics
                               // keep busy)
    // individual time steps (device): time, next boundary, active and
    // density counts; sorted rungs, packed rungs, sink lists and marks
    RungState *d_rung = nullptr;
    double *rungs = nullptr;   // sorted: rung
    double *nbmax = nullptr;   // sorted: largest rung over F_i (force pass)
    int32_t *rpack = nullptr;  // sorted: rung | 256 when the density is not of this substep
    int64_t *rflags = nullptr; // n + 1: compaction flags, then their exclusive scan
    uint32_t *sinks = nullptr, *dsinks = nullptr;   // active sinks, density sinks (sorted)
    uint32_t *mark = nullptr;  // sorted: FastGas marks
    double *nbmax_c = nullptr; // caller order: nbmax of the active particles
    bool rungs_on = false;
    // what the next sweep launches take: a sink list and its device length
    // (null: all particles), the packed rungs (null: no rung maximum)
    const uint32_t *sweep_sinks = nullptr;
    const long long *sweep_nsinks = nullptr;
    bool sweep_rpack = false;
    bool rpack_ready = false;   // sph_init: the desired rungs are packed (limiter pass)
    // sweep launch shape (SPH_LAUNCH_*), the persistent launch's per-XCD queue
    // counters, the device's CUs; shape and workgroups of the last force launch
    int32_t launch = SPH_LAUNCH_GROUPS;
    uint32_t *d_queue = nullptr;
    int32_t ncu = 0;
    int32_t sweep_launch = SPH_LAUNCH_GROUPS;
    int64_t sweep_workgroups = 0;
    bool mats_has = false;     // the caller gave material ids
    uint32_t *d_wstack = nullptr;   // sweep walk stacks, kStackCap node ids per sink group
    // stored interaction lists of the sweeps (kListCap buckets and a header of
    // kWalkWords per sink group; one pass at a time) and the per-group flag of
    // the groups left to the walking kernels; null: the sweeps walk themselves
    uint32_t *d_wlist = nullptr;
    int32_t *d_whdr = nullptr;
    int32_t *d_defer = nullptr;

    // scan scratch
    int64_t *d_scan_tmp = nullptr;
    int64_t scan_tmp_len = 0;

    // counters, step report, reduction partials
    unsigned long long *d_cnt = nullptr;    // kCntShards copies of the counters
    unsigned long long *d_csum = nullptr;   // their sums (C_NCOUNTERS), what the host reads
    StepReport *d_rep = nullptr;
    double *d_dt = nullptr;         // per set: step size used by the kick kernels
    double *d_set_dtnext = nullptr; // per set: min_i dt_i of the last force pass
    double *d_part = nullptr;       // reduction partials
    unsigned long long *h_cnt = nullptr; // pinned host mirrors
    StepReport *h_rep = nullptr;
    // status word of the last call: C_ITERLIM and C_NONFINITE copied into
    // pinned memory at the end of every enqueuing call, then status_ev; the
    // next call reads them once the event has completed (never waits for it)
    unsigned long long *h_flags = nullptr;
    hipEvent_t status_ev = nullptr;
    bool status_pending = false;

    // phase timing (hipEvents on the call's stream; off during graph capture)
    bool timing = false;
    bool capturing = false;
    hipEvent_t ev[E_NEVENTS] = {};
    unsigned ev_mask = 0;           // events recorded by the last call

    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    std::vector<void *> allocs;
};

// ---------------------------------------------------------------- launches
// Tree (sph_tree.hip)
hipError_t launch_tree_build(Ctx *c, const sph_particles *p, hipStream_t s);
hipError_t launch_refit(Ctx *c, hipStream_t s);
hipError_t launch_init_nodes(Ctx *c, hipStream_t s);
hipError_t launch_scan_i64(Ctx *c, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
int64_t scan_tmp_needed(int64_t n);
int64_t sort_blocks_needed(int64_t n);
int key_bits_per_axis();

// Sweep (sph_sweep.hip)
hipError_t launch_density(Ctx *c, hipStream_t s);
hipError_t launch_forces(Ctx *c, hipStream_t s);
hipError_t launch_neighbors(Ctx *c, int mode, int64_t *row_count_caller, const int64_t *offsets,
                            int32_t *idx, hipStream_t s);
hipError_t launch_sort_rows(Ctx *c, const int64_t *offsets, int32_t *idx, hipStream_t s);
hipError_t launch_interface_sums(Ctx *c, int mode, hipStream_t s);   // 0 imbalance, 1 averages

// Elementwise, step, reductions (sph_kdk.hip)
constexpr int kMaxCols = 8;
struct Cols {
    const double *src[kMaxCols];
    double *dst[kMaxCols];
    int n;
};
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
// zero counters [0, last) of every copy; fold the copies into d_csum
hipError_t launch_reset_counters(Ctx *c, int last, hipStream_t s);
// individual time steps (Sec. 2.3.6)
hipError_t launch_rung_open(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_rung_drift(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_rung_lists(Ctx *c, bool fastgas, hipStream_t s);
hipError_t launch_rung_dens_list(Ctx *c, hipStream_t s);
hipError_t launch_rung_close(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_rung_finish(Ctx *c, hipStream_t s);
hipError_t launch_rung_desired(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_rung_limit_init(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_rung_pack(Ctx *c, hipStream_t s);
hipError_t launch_scatter_sinks(Ctx *c, const Cols &cols, hipStream_t s);   // active sinks only
hipError_t launch_mark(Ctx *c, hipStream_t s);
hipError_t launch_rung_pack_init(Ctx *c, hipStream_t s);   // no FastGas flags
hipError_t launch_fold_counters(Ctx *c, hipStream_t s);
hipError_t launch_gather(Ctx *c, const Cols &cols, hipStream_t s);   // dst[k] = src[perm[k]]
hipError_t launch_scatter(Ctx *c, const Cols &cols, hipStream_t s);  // dst[perm[k]] = src[k]
hipError_t launch_eos(Ctx *c, const double *u_sorted, double *P_caller, double *c_caller,
                      hipStream_t s);
hipError_t launch_kick_drift(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_closing_kick(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_isentrope(Ctx *c, sph_particles *p, hipStream_t s);
hipError_t launch_ic_correct(Ctx *c, double *P_caller, double *c_caller, double *imb_caller,
                             double *rho_caller, hipStream_t s);
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);
hipError_t launch_reduce(Ctx *c, const sph_particles *p, hipStream_t s);
hipError_t launch_set_dt(Ctx *c, double dt, hipStream_t s);
hipError_t launch_set_dtnext(Ctx *c, const sph_particles *p, hipStream_t s);
int reduce_partials();

// Records timing event e on stream s when timing is on (no-op otherwise).
inline void mark(Ctx *c, int e, hipStream_t s) {
    if (c->timing && !c->capturing && c->ev[e]) {
        if (hipEventRecord(c->ev[e], s) == hipSuccess) c->ev_mask |= 1u << e;
    }
}

}  // namespace sphmi

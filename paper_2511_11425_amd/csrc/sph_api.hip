// sph_api.hip -- the C interface (include/sph.h): context, device memory,
// call sequencing, counters, graph capture and the bucket-size autotuner.
#include "sph_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstddef>
#include <climits>
#include <new>

using namespace sphmi;

struct sph_ctx {
    Ctx c;
};

namespace {

const char kVersion[] = "sph-mi355x 0.1 (gfx950)";

sph_status fail(sph_ctx *x, sph_status st, const char *msg) {
    if (x) x->c.err = msg;
    return st;
}

sph_status hip_fail(sph_ctx *x, hipError_t e, const char *where) {
    if (x) {
        x->c.err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return SPH_ERR_HIP;
}

#define HIPCHK(x, expr, where)                                  \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail((x), e_, where);  \
    } while (0)

template <typename T>
hipError_t dalloc(Ctx &c, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (count > 0 ? count : 1));
    if (e != hipSuccess) return e;
    c.allocs.push_back(q);
    *p = reinterpret_cast<T *>(q);
    return hipSuccess;
}

void free_events(Ctx &c) {
    for (int e = 0; e < E_NEVENTS; ++e)
        if (c.ev[e]) { (void)hipEventDestroy(c.ev[e]); c.ev[e] = nullptr; }
}

void free_all(Ctx &c) {
    if (c.graph_exec) { (void)hipGraphExecDestroy(c.graph_exec); c.graph_exec = nullptr; }
    if (c.graph) { (void)hipGraphDestroy(c.graph); c.graph = nullptr; }
    for (void *q : c.allocs) (void)hipFree(q);
    c.allocs.clear();
    c.frec1 = c.frec2 = c.fm = nullptr;
    c.drec1 = c.drec2 = nullptr;
    c.rho_old = c.rho_pred = c.rho_sum = c.drs = nullptr;
    c.mats = c.imbs = c.tbar = c.pbar = nullptr;
    c.levc = c.levs = c.d_levref = nullptr;
    c.d_queue = nullptr;
    c.d_wlist = nullptr; c.d_whdr = nullptr; c.d_defer = nullptr;
    c.d_rung = nullptr; c.rungs = c.nbmax = c.nbmax_c = nullptr; c.rpack = nullptr;
    c.rflags = nullptr; c.sinks = c.dsinks = c.mark = nullptr;
    if (c.h_cnt) { (void)hipHostFree(c.h_cnt); c.h_cnt = nullptr; }
    if (c.h_rep) { (void)hipHostFree(c.h_rep); c.h_rep = nullptr; }
    if (c.h_flags) { (void)hipHostFree(c.h_flags); c.h_flags = nullptr; }
    c.status_pending = false;
    c.n = 0;
    c.have_tree = false;
    c.have_forces = false;
}

bool valid_params(const sph_params *p, std::string &why) {
    if (!p) { why = "params is NULL"; return false; }
    if (p->kernel < 0 || p->kernel > 3) { why = "kernel must be 0..3"; return false; }
    if (p->precision != SPH_PREC_FP64 && p->precision != SPH_PREC_MIXED) {
        why = "precision must be SPH_PREC_FP64 or SPH_PREC_MIXED"; return false;
    }
    if (p->eos != SPH_EOS_IDEAL && p->eos != SPH_EOS_STIFFENED) { why = "bad eos"; return false; }
    static const double sig43[4] = {32.0 / 3.0, 14.0, 165.0 / 8.0, 455.0 / 16.0};
    if (!(p->n_ngb > sig43[p->kernel])) { why = "n_ngb must exceed (4 pi/3) sigma of the kernel"; return false; }
    if (p->periodic) {
        for (int a = 0; a < 3; ++a)
            if (!(p->box_hi[a] > p->box_lo[a])) { why = "empty periodic box"; return false; }
    }
    if (!(p->h_max > 0)) { why = "h_max must be positive"; return false; }
    if (!(p->oversel >= 1.0)) { why = "oversel must be >= 1"; return false; }
    if (!(p->gamma > 1.0)) { why = "gamma must exceed 1"; return false; }
    if (p->nr_maxit < 1) { why = "nr_maxit must be >= 1"; return false; }
    if (p->bucket != 0 && p->bucket != 8 && p->bucket != 16 && p->bucket != 32 && p->bucket != 64) {
        why = "bucket must be 0, 8, 16, 32 or 64"; return false;
    }
    if (p->stack_limit != 0 && (p->stack_limit < 2 || p->stack_limit > kStackCap)) {
        why = "stack_limit must be 0 or 2..768"; return false;
    }
    if (p->flags & ~(SPH_FLAG_ENTROPY | SPH_FLAG_EVOLVED | SPH_FLAG_INTERFACE | SPH_FLAG_DYNAMIC |
                     SPH_FLAG_RUNGS)) {
        why = "unknown flags"; return false;
    }
    if ((p->flags & SPH_FLAG_INTERFACE) && (p->flags & SPH_FLAG_EVOLVED)) {
        why = "the interface correction applies to the summed density (not SPH_FLAG_EVOLVED)";
        return false;
    }
    if ((p->flags & SPH_FLAG_INTERFACE) && !(p->ic_alpha > 0.0)) {
        why = "ic_alpha must be positive"; return false;
    }
    if ((p->flags & SPH_FLAG_ENTROPY) && (p->flags & SPH_FLAG_EVOLVED)) {
        why = "the entropy-conserving update needs the summed density (not SPH_FLAG_EVOLVED)";
        return false;
    }
    if (p->launch != SPH_LAUNCH_GROUPS && p->launch != SPH_LAUNCH_PERSISTENT &&
        p->launch != SPH_LAUNCH_WALK) {
        why = "launch must be SPH_LAUNCH_GROUPS, SPH_LAUNCH_PERSISTENT or SPH_LAUNCH_WALK";
        return false;
    }
    if ((p->flags & SPH_FLAG_RUNGS) && p->launch == SPH_LAUNCH_PERSISTENT) {
        why = "SPH_FLAG_RUNGS launches one workgroup per sink group"; return false;
    }
    if (p->flags & SPH_FLAG_RUNGS) {
        if (p->flags != SPH_FLAG_RUNGS) {
            why = "SPH_FLAG_RUNGS is not combined with the other flags"; return false;
        }
        if (p->rung_max < 0 || p->rung_max > 20) { why = "rung_max must be 0..20"; return false; }
        if (!(p->dt_max > 0.0)) { why = "dt_max must be positive"; return false; }
        if (!(p->fastgas >= 0.0 && p->fastgas <= 1.0)) {
            why = "fastgas must be in [0, 1]"; return false;
        }
    }
    return true;
}

// Topology of buckets, groups and tree nodes for n particles and bucket size B.
struct Topology {
    std::vector<SetGeom> sets;
    std::vector<int32_t> grp_set, bkt_set;
    std::vector<int64_t> pref;        // (max_depth+1) x (nsets+1): prefix of nodes per height
    std::vector<int64_t> level_total;
    int64_t nbuckets = 0, ngroups = 0, nnodes = 0;
    int max_depth = 0;
};

bool make_topology(const Ctx &c, int B, Topology &t, std::string &why) {
    const int ns = c.nsets;
    t.sets.assign(ns, SetGeom{});
    t.grp_set.clear();
    t.bkt_set.clear();
    int64_t b0 = 0, g0 = 0, node0 = 0;
    int max_depth = 0;
    for (int q = 0; q < ns; ++q) {
        SetGeom &g = t.sets[q];
        g.p0 = c.set_off[q];
        g.p1 = c.set_off[q + 1];
        int64_t np = g.p1 - g.p0;
        int64_t nb = (np + B - 1) / B;
        int64_t nbp = 1;
        int depth = 0;
        while (nbp < nb) { nbp <<= 1; ++depth; }
        if (nbp > (int64_t)1 << 30) { why = "set too large"; return false; }
        g.nb = (int32_t)nb;
        g.nbp = (int32_t)nbp;
        g.depth = depth;
        g.b0 = b0;
        g.g0 = g0;
        g.node0 = node0;
        const double *lo = c.set_box.empty() ? c.prm.box_lo : &c.set_box[6 * q];
        const double *hi = c.set_box.empty() ? c.prm.box_hi : &c.set_box[6 * q + 3];
        for (int a = 0; a < 3; ++a) {
            g.lo[a] = lo[a];
            g.L[a] = hi[a] - lo[a];
            g.halfL[a] = 0.5 * g.L[a];
        }
        int64_t ng = (np + kGroup - 1) / kGroup;
        for (int64_t k = 0; k < ng; ++k) t.grp_set.push_back(q);
        for (int64_t k = 0; k < nb; ++k) t.bkt_set.push_back(q);
        b0 += nb;
        g0 += ng;
        node0 += 2 * nbp;
        max_depth = std::max(max_depth, depth);
    }
    t.nbuckets = b0;
    t.ngroups = g0;
    t.nnodes = node0;
    t.max_depth = max_depth;
    // nodes per height d: nbp >> d for sets with depth >= d
    t.pref.assign((size_t)(max_depth + 1) * (ns + 1), 0);
    t.level_total.assign(max_depth + 1, 0);
    for (int d = 0; d <= max_depth; ++d) {
        int64_t acc = 0;
        for (int q = 0; q < ns; ++q) {
            t.pref[(size_t)d * (ns + 1) + q] = acc;
            if (t.sets[q].depth >= d && t.sets[q].nb > 0) acc += (int64_t)(t.sets[q].nbp >> d);
        }
        t.pref[(size_t)d * (ns + 1) + ns] = acc;
        t.level_total[d] = acc;
    }
    return true;
}

// Copies the topology of the context's current bucket size to the device
// (the allocation holds the largest one, that of the smallest bucket size).
sph_status upload_topology(sph_ctx *x, const Topology &t, hipStream_t s) {
    Ctx &c = x->c;
    const int ns = c.nsets;
    c.nbuckets = t.nbuckets;
    c.ngroups = t.ngroups;
    c.nnodes = t.nnodes;
    c.max_depth = t.max_depth;
    c.level_total = t.level_total;
    HIPCHK(x, hipMemcpyAsync(c.d_sets, t.sets.data(), sizeof(SetGeom) * ns, hipMemcpyHostToDevice, s),
           "sets");
    if (!t.grp_set.empty())
        HIPCHK(x, hipMemcpyAsync(c.d_grp_set, t.grp_set.data(), sizeof(int32_t) * t.grp_set.size(),
                                 hipMemcpyHostToDevice, s), "groups");
    if (!t.bkt_set.empty())
        HIPCHK(x, hipMemcpyAsync(c.d_bkt_set, t.bkt_set.data(), sizeof(int32_t) * t.bkt_set.size(),
                                 hipMemcpyHostToDevice, s), "buckets");
    HIPCHK(x, hipMemcpyAsync(c.d_level_pref, t.pref.data(), sizeof(int64_t) * t.pref.size(),
                             hipMemcpyHostToDevice, s), "levels");
    HIPCHK(x, launch_init_nodes(&c, s), "init nodes");
    // host pages of the topology vectors must outlive the copies
    HIPCHK(x, hipStreamSynchronize(s), "topology sync");
    c.topo_bucket = c.bucket;
    c.have_tree = false;
    c.have_forces = false;
    return SPH_OK;
}

// Dynamic bucket sizing: every particle starts at the level of the base
// bucket size (buckets of 8 2^h).
hipError_t reset_levels(Ctx &c, double *dst, int64_t n, hipStream_t s) {
    const double v = (double)base_level(c.base_bucket);
    unsigned long long bits;
    std::memcpy(&bits, &v, sizeof(bits));
    return launch_fill_u64(reinterpret_cast<unsigned long long *>(dst), n, bits, s);
}

// Device memory for n particles.  Every bucket-size-dependent array is sized
// for the smallest bucket size (8), so a change of the bucket size (the
// autotuner's trials) only rewrites the topology: after the first call at a
// given n nothing is allocated.
sph_status setup(sph_ctx *x, int64_t n, hipStream_t s) {
    Ctx &c = x->c;
    std::string why;
    Topology t;
    if (c.n == n && c.allocs.size() > 0) {
        if (c.topo_bucket == c.bucket) return SPH_OK;
        if (!make_topology(c, c.bucket, t, why)) return fail(x, SPH_ERR_INVALID, "set too large");
        return upload_topology(x, t, s);
    }
    free_all(c);
    const int ns = c.nsets;
    Topology tmax;   // the largest topology (bucket size 8) sizes the allocation
    if (!make_topology(c, 8, tmax, why) || !make_topology(c, c.bucket, t, why))
        return fail(x, SPH_ERR_INVALID, "set too large");
    const int64_t cap_buckets = tmax.nbuckets, cap_nodes = tmax.nnodes;
    const size_t cap_pref = tmax.pref.size();
    c.ngroups = t.ngroups;
    c.set_bits = 0;
    while ((1 << c.set_bits) < ns) ++c.set_bits;
    int key_bits = 3 * key_bits_per_axis() + c.set_bits;
    c.key_passes = (key_bits + 7) / 8;
    c.sort_blocks = sort_blocks_needed(n);
    int64_t scan_len = std::max<int64_t>(n + 1, 256 * std::max<int64_t>(c.sort_blocks, 1));
    c.scan_tmp_len = scan_tmp_needed(scan_len);

    hipError_t e = hipSuccess;
    const char *what = "";
#define A(ptr, cnt) if (e == hipSuccess) { what = #ptr; e = dalloc(c, &(ptr), (cnt)); }
    A(c.d_sets, ns);
    A(c.d_grp_set, t.grp_set.size());
    A(c.d_bkt_set, cap_buckets);
    A(c.d_level_pref, cap_pref);
    A(c.d_key[0], n); A(c.d_key[1], n);
    A(c.d_perm[0], n); A(c.d_perm[1], n);
    A(c.d_hist, 2 * 256 * std::max<int64_t>(c.sort_blocks, 1));  // int64 view
    A(c.d_bbox, 6 * ns);
    A(c.xs, n); A(c.ys, n); A(c.zs, n); A(c.ms, n); A(c.Hs, n);
    A(c.vxs, n); A(c.vys, n); A(c.vzs, n); A(c.us, n);
    A(c.rhos, n); A(c.oms, n); A(c.As, n); A(c.css, n); A(c.Ps, n);
    if (c.prm.precision == SPH_PREC_MIXED) { A(c.frec1, 4 * n); A(c.frec2, 4 * n); A(c.fm, n); }
    else { A(c.drec1, 4 * n); A(c.drec2, 4 * n); }
    A(c.axs, n); A(c.ays, n); A(c.azs, n); A(c.dus, n); A(c.dts, n);
    A(c.nodes, cap_nodes);
    A(c.vpx, n); A(c.vpy, n); A(c.vpz, n); A(c.upred, n);
    A(c.hprev, n);
    A(c.d_h0, n);
    if (c.prm.flags & SPH_FLAG_ENTROPY) A(c.rho_old, n);
    if (c.prm.flags & SPH_FLAG_EVOLVED) { A(c.rho_pred, n); A(c.rho_sum, n); A(c.drs, n); }
    if (c.prm.flags & SPH_FLAG_INTERFACE) { A(c.mats, n); A(c.imbs, n); A(c.tbar, n); A(c.pbar, n); }
    if (c.dyn) { A(c.levc, n); A(c.levs, n); A(c.d_levref, 1); }
    if (c.rungs_on) {
        A(c.d_rung, 1); A(c.rungs, n); A(c.nbmax, n); A(c.nbmax_c, n); A(c.rpack, n);
        A(c.rflags, n + 1); A(c.sinks, n); A(c.dsinks, n);
        if (c.prm.fastgas > 0.0) A(c.mark, n + 2);
    }
    A(c.d_wstack, (size_t)std::max<int64_t>(c.ngroups, 1) * kStackCap);
    A(c.d_wlist, (size_t)std::max<int64_t>(c.ngroups, 1) * kListCap);
    A(c.d_whdr, (size_t)std::max<int64_t>(c.ngroups, 1) * kWalkWords);
    A(c.d_defer, (size_t)std::max<int64_t>(c.ngroups, 1));
    A(c.d_queue, kXcds * kQueueStride);
    A(c.d_scan_tmp, c.scan_tmp_len);
    A(c.d_cnt, kCntShards * kCntStride);
    A(c.d_csum, C_NCOUNTERS);
    A(c.d_rep, 1);
    A(c.d_dt, ns);
    A(c.d_set_dtnext, ns);
    A(c.d_part, 6 * reduce_partials());
#undef A
    if (e != hipSuccess) {
        free_all(c);
        x->c.err = std::string("device allocation failed (") + what + "): " + hipGetErrorString(e);
        return SPH_ERR_OOM;
    }
    if (hipHostMalloc((void **)&c.h_cnt, sizeof(unsigned long long) * C_NCOUNTERS) != hipSuccess ||
        hipHostMalloc((void **)&c.h_rep, sizeof(StepReport)) != hipSuccess ||
        hipHostMalloc((void **)&c.h_flags, 2 * sizeof(unsigned long long)) != hipSuccess) {
        free_all(c);
        return fail(x, SPH_ERR_OOM, "pinned allocation failed");
    }
    c.h_flags[0] = c.h_flags[1] = 0;
    if (!c.status_ev)
        HIPCHK(x, hipEventCreateWithFlags(&c.status_ev, hipEventDisableTiming), "status event");
    HIPCHK(x, launch_fill_u64(c.d_cnt, kCntShards * kCntStride, 0ull, s), "counters");
    HIPCHK(x, launch_fill_u64(c.d_csum, C_NCOUNTERS, 0ull, s), "counter sums");
    HIPCHK(x, launch_fill_u64(reinterpret_cast<unsigned long long *>(c.d_rep),
                              sizeof(StepReport) / 8, 0ull, s), "report");
    if (c.dyn) {
        HIPCHK(x, reset_levels(c, c.levc, n, s), "levels");
        HIPCHK(x, launch_fill_u64(reinterpret_cast<unsigned long long *>(c.d_levref), 1, 0ull, s),
               "level reference");
    }
    sph_status st = upload_topology(x, t, s);
    if (st != SPH_OK) return st;
    c.n = n;
    return SPH_OK;
}

sph_status check_particles(sph_ctx *x, const sph_particles *p, bool outputs, int64_t n) {
    if (!p) return fail(x, SPH_ERR_INVALID, "particles is NULL");
    if (n == 0) return SPH_OK;  // empty columns may be NULL
    if (!p->x || !p->y || !p->z || !p->vx || !p->vy || !p->vz || !p->m || !p->u || !p->H)
        return fail(x, SPH_ERR_INVALID, "a state array is NULL");
    if (outputs && (!p->rho || !p->omega || !p->P || !p->c || !p->ax || !p->ay || !p->az ||
                    !p->dudt || !p->dt))
        return fail(x, SPH_ERR_INVALID, "an output array is NULL");
    if (outputs && x && (x->c.prm.flags & SPH_FLAG_EVOLVED) && !p->drhodt)
        return fail(x, SPH_ERR_INVALID, "drhodt is NULL (evolved density)");
    if (x && (x->c.prm.flags & SPH_FLAG_RUNGS) && !p->rung)
        return fail(x, SPH_ERR_INVALID, "rung is NULL (individual time steps)");
    return SPH_OK;
}

// The device status word of a finished call, as an sph_status.
sph_status flags_status(const unsigned long long *f) {
    if (f[1]) return SPH_ERR_NONFINITE;
    if (f[0]) return SPH_ERR_NOCONV;
    return SPH_OK;
}

// Start of a call: the status of the previous call, once the device has
// finished it (never waits).  A non-OK status is returned by this call, which
// then enqueues nothing; it is reported once.
sph_status take_status(sph_ctx *x) {
    Ctx &c = x->c;
    if (!c.status_pending || !c.status_ev) return SPH_OK;
    if (hipEventQuery(c.status_ev) != hipSuccess) return SPH_OK;   // not finished yet
    c.status_pending = false;
    const sph_status st = flags_status(c.h_flags);
    if (st == SPH_ERR_NOCONV)
        return fail(x, st, "the previous call left a smoothing-length iteration at nr_maxit");
    if (st == SPH_ERR_NONFINITE)
        return fail(x, st, "the previous call produced a non-finite result");
    return SPH_OK;
}

// End of an enqueuing call: the status word goes to pinned memory behind the
// call's work, followed by the status event (skipped while capturing a graph;
// sph_graph_launch posts it after the replay).
hipError_t post_status(Ctx &c, hipStream_t s) {
    if (c.d_cnt) {
        // (the sums the host reads: also inside a captured graph)
        hipError_t e = launch_fold_counters(&c, s);
        if (e != hipSuccess) return e;
    }
    if (c.capturing || !c.h_flags || !c.status_ev) return hipSuccess;
    hipError_t e = hipMemcpyAsync(c.h_flags, c.d_csum + C_ITERLIM, 2 * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(c.status_ev, s);
    if (e == hipSuccess) c.status_pending = true;
    return e;
}

hipError_t reset_counters(Ctx &c, hipStream_t s) {
    c.ev_mask = 0;
    mark(&c, E_BEGIN, s);
    return launch_reset_counters(&c, C_NTRANSIENT, s);
}

Cols cols0() {
    Cols k;
    std::memset(&k, 0, sizeof(k));
    return k;
}

// Density pass on the current tree; H first guess from the caller.  Inside a
// step with the evolved density the summed density goes to scratch: the
// caller's rho is then a state variable.
sph_status do_density(sph_ctx *x, sph_particles *p, hipStream_t s, bool in_step = false) {
    Ctx &c = x->c;
    Cols g = cols0();
    g.src[0] = p->H; g.dst[0] = c.Hs; g.n = 1;
    if (c.dyn) { g.src[1] = c.levc; g.dst[1] = c.levs; g.n = 2; }
    if (c.rungs_on && in_step) {
        // (with FastGas the particles outside the density pass keep theirs)
        g.src[g.n] = p->rho; g.dst[g.n] = c.rhos; ++g.n;
        g.src[g.n] = p->omega; g.dst[g.n] = c.oms; ++g.n;
    }
    HIPCHK(x, launch_gather(&c, g, s), "gather H");
    HIPCHK(x, launch_density(&c, s), "density");
    const bool keep_rho = in_step && (c.prm.flags & SPH_FLAG_EVOLVED);
    Cols o = cols0();
    o.src[0] = c.Hs; o.dst[0] = p->H;
    o.src[1] = c.rhos; o.dst[1] = keep_rho ? c.rho_sum : p->rho;
    o.src[2] = c.oms; o.dst[2] = p->omega;
    o.n = 3;
    HIPCHK(x, launch_scatter(&c, o, s), "scatter density");
    HIPCHK(x, launch_refit(&c, s), "refit");
    return SPH_OK;
}

// Force pass; velocities and u from the given columns (caller order).  The
// density comes from the density pass, from the caller (gather_density) or,
// with the evolved density inside a step, from the predicted density.
sph_status do_forces(sph_ctx *x, sph_particles *p, const double *vx, const double *vy,
                     const double *vz, const double *u, bool gather_density, hipStream_t s,
                     bool in_step = false) {
    Ctx &c = x->c;
    const bool evolved = (c.prm.flags & SPH_FLAG_EVOLVED) != 0;
    Cols g = cols0();
    g.src[0] = vx; g.dst[0] = c.vxs;
    g.src[1] = vy; g.dst[1] = c.vys;
    g.src[2] = vz; g.dst[2] = c.vzs;
    g.src[3] = u; g.dst[3] = c.us;
    g.n = 4;
    auto col = [&g](const double *src, double *dst) {
        g.src[g.n] = src; g.dst[g.n] = dst; ++g.n;
    };
    if (in_step && evolved) col(c.rho_pred, c.rhos);
    if (gather_density) {
        col(p->H, c.Hs);
        col(p->rho, c.rhos);
        col(p->omega, c.oms);
    }
    // (inside a step the density pass has gathered the levels)
    if (c.dyn && !in_step) col(c.levc, c.levs);
    HIPCHK(x, launch_gather(&c, g, s), "gather force inputs");
    if (gather_density) HIPCHK(x, launch_refit(&c, s), "refit");
    const bool ic = (c.prm.flags & SPH_FLAG_INTERFACE) != 0;
    if (ic) {
        // interface correction (Sec. 2.3.4): materials in sorted order, the
        // kernel imbalance, EOS, the averages, the corrected fluid values
        c.mats_has = p->mat != nullptr;
        if (c.mats_has) {
            Cols mcol = cols0();
            mcol.src[0] = p->mat; mcol.dst[0] = c.mats; mcol.n = 1;
            HIPCHK(x, launch_gather(&c, mcol, s), "gather materials");
        }
        HIPCHK(x, launch_interface_sums(&c, 0, s), "kernel imbalance");
    }
    HIPCHK(x, launch_eos(&c, c.us, p->P, p->c, s), "eos");
    if (ic) {
        HIPCHK(x, launch_interface_sums(&c, 1, s), "interface averages");
        HIPCHK(x, launch_ic_correct(&c, p->P, p->c, p->imb, p->rhoc, s), "interface correction");
    }
    const bool sub = c.rungs_on && in_step;   // a substep: the active sinks only
    if (sub) {
        c.sweep_sinks = c.sinks;
        c.sweep_nsinks = reinterpret_cast<const long long *>(
            reinterpret_cast<const char *>(c.d_rung) + offsetof(RungState, nact));
    }
    c.sweep_rpack = c.rungs_on && (in_step || c.rpack_ready);
    const hipError_t fe = launch_forces(&c, s);
    c.sweep_sinks = nullptr;
    c.sweep_nsinks = nullptr;
    c.sweep_rpack = false;
    HIPCHK(x, fe, "forces");
    Cols o = cols0();
    o.src[0] = c.axs; o.dst[0] = p->ax;
    o.src[1] = c.ays; o.dst[1] = p->ay;
    o.src[2] = c.azs; o.dst[2] = p->az;
    o.src[3] = c.dus; o.dst[3] = p->dudt;
    o.src[4] = c.dts; o.dst[4] = p->dt;
    o.n = 5;
    if (c.rungs_on && (in_step || c.rpack_ready)) {
        o.src[o.n] = c.nbmax; o.dst[o.n] = c.nbmax_c;
        o.n += 1;
    }
    if (sub) {
        HIPCHK(x, launch_scatter_sinks(&c, o, s), "scatter forces");
        return SPH_OK;
    }
    if (evolved) {
        o.src[o.n] = c.drs; o.dst[o.n] = p->drhodt;
        o.n += 1;
    }
    if (c.dyn) {
        o.src[o.n] = c.levs; o.dst[o.n] = c.levc;
        o.n += 1;
    }
    HIPCHK(x, launch_scatter(&c, o, s), "scatter forces");
    return SPH_OK;
}

// Individual time steps: the device length of a sink list inside RungState.
const long long *rung_count(const Ctx &c, size_t off) {
    return reinterpret_cast<const long long *>(reinterpret_cast<const char *>(c.d_rung) + off);
}

hipError_t reset_rung_state(Ctx &c, hipStream_t s) {
    unsigned long long *w = reinterpret_cast<unsigned long long *>(c.d_rung);
    hipError_t e = launch_fill_u64(w, 4, 0ull, s);
    if (e == hipSuccess) e = launch_fill_u64(w + 1, 1, (unsigned long long)LLONG_MAX, s);
    if (e == hipSuccess) e = launch_fill_u64(w + 2, 2, (unsigned long long)c.n, s);
    return e;
}

// Rungs at T = 0 (after the initial force pass): desired rungs from dt, then
// a second force pass over them for the largest neighbour rung, then the
// limiter (the forces of the second pass equal the first's).
sph_status init_rungs(sph_ctx *x, sph_particles *p, hipStream_t s) {
    Ctx &c = x->c;
    HIPCHK(x, reset_rung_state(c, s), "rung state");
    HIPCHK(x, launch_rung_desired(&c, p, s), "desired rungs");
    Cols g = cols0();
    g.src[0] = p->rung; g.dst[0] = c.rungs; g.n = 1;
    HIPCHK(x, launch_gather(&c, g, s), "gather rungs");
    HIPCHK(x, launch_rung_pack_init(&c, s), "pack rungs");
    c.rpack_ready = true;
    sph_status st = do_forces(x, p, p->vx, p->vy, p->vz, p->u, false, s);
    c.rpack_ready = false;
    if (st != SPH_OK) return st;
    HIPCHK(x, launch_rung_limit_init(&c, p, s), "limiter");
    return SPH_OK;
}

// One substep (Sec. 2.3.6): opening kick of the particles at a step
// boundary, drift of all to the next boundary T', tree, density (all
// particles, or with FastGas those on the active particles' lists), EOS and
// forces of the active particles with v and u predicted at T', their closing
// kick and new rung.
sph_status do_substep(sph_ctx *x, sph_particles *p, hipStream_t s) {
    Ctx &c = x->c;
    HIPCHK(x, reset_counters(c, s), "counters");
    HIPCHK(x, launch_rung_open(&c, p, s), "opening kick");
    HIPCHK(x, launch_rung_drift(&c, p, s), "drift");
    HIPCHK(x, launch_tree_build(&c, p, s), "tree");
    Cols g = cols0();
    g.src[0] = p->rung; g.dst[0] = c.rungs; g.n = 1;
    HIPCHK(x, launch_gather(&c, g, s), "gather rungs");
    HIPCHK(x, launch_rung_lists(&c, false, s), "active sinks");
    const bool fg = c.prm.fastgas > 0.0;
    if (fg) {
        HIPCHK(x, launch_fill_u64(reinterpret_cast<unsigned long long *>(c.mark), (c.n + 2) / 2, 0ull,
                                  s), "marks");
        c.sweep_sinks = c.sinks;
        c.sweep_nsinks = rung_count(c, offsetof(RungState, nact));
        const hipError_t e = launch_mark(&c, s);
        c.sweep_sinks = nullptr;
        c.sweep_nsinks = nullptr;
        HIPCHK(x, e, "FastGas marks");
        HIPCHK(x, launch_rung_dens_list(&c, s), "density sinks");
        c.sweep_sinks = c.dsinks;
        c.sweep_nsinks = rung_count(c, offsetof(RungState, ndens));
    }
    sph_status st = do_density(x, p, s, true);
    c.sweep_sinks = nullptr;
    c.sweep_nsinks = nullptr;
    if (st != SPH_OK) return st;
    HIPCHK(x, launch_rung_pack(&c, s), "pack rungs");
    st = do_forces(x, p, c.vpx, c.vpy, c.vpz, c.upred, false, s, true);
    if (st != SPH_OK) return st;
    HIPCHK(x, launch_rung_close(&c, p, s), "closing kick");
    HIPCHK(x, launch_rung_finish(&c, s), "substep end");
    HIPCHK(x, launch_reduce(&c, p, s), "reduce");
    mark(&c, E_END, s);
    return SPH_OK;
}

sph_status do_step(sph_ctx *x, sph_particles *p, double dt, hipStream_t s) {
    Ctx &c = x->c;
    HIPCHK(x, reset_counters(c, s), "counters");
    HIPCHK(x, launch_set_dt(&c, dt, s), "dt");
    HIPCHK(x, launch_kick_drift(&c, p, s), "kick-drift");
    HIPCHK(x, launch_tree_build(&c, p, s), "tree");
    sph_status st = do_density(x, p, s, true);
    if (st != SPH_OK) return st;
    if (c.prm.flags & SPH_FLAG_ENTROPY) HIPCHK(x, launch_isentrope(&c, p, s), "isentrope");
    st = do_forces(x, p, c.vpx, c.vpy, c.vpz, c.upred, false, s, true);
    if (st != SPH_OK) return st;
    HIPCHK(x, launch_closing_kick(&c, p, s), "closing kick");
    HIPCHK(x, launch_reduce(&c, p, s), "reduce");
    HIPCHK(x, launch_set_dtnext(&c, p, s), "set dt");
    mark(&c, E_END, s);
    return SPH_OK;
}

// ---------------------------------------------------------------- allocation-free start-up
//
// sph_init_noalloc runs the start-up pass of sph_init (tree build, density,
// forces) with every work array carved out of one file-scope device array,
// `scratch`, instead of device allocations: for callers that cannot
// allocate.  Each GPU the library runs on holds its own copy of the array
// (kNoAllocBytes) until the process ends; the host keeps its device address,
// obtained once per device with hipGetSymbolAddress, and passes that address
// (never the array's host-side name) to every launch.  All calls on one GPU
// share the array, which keeps the last call's contents: everything a call
// reads is written or cleared by that call first, and calls that overlap on
// one GPU race.
constexpr int64_t kNoAllocMaxN = 65536;          // particles per call
constexpr size_t kNoAllocBytes = 32ull << 20;    // 32 MiB per GPU
constexpr int kNoAllocDevices = 16;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

unsigned char *g_scratch[kNoAllocDevices] = {};   // device address of `scratch` per GPU
sph_ctx g_noalloc[kNoAllocDevices];               // host state per GPU (no allocation)

// Bump allocator over the scratch array (256-byte aligned pieces).
struct Carve {
    unsigned char *base;
    size_t off, cap;
    bool ok;
    template <typename T> void take(T **p, size_t count) {
        const size_t bytes = (sizeof(T) * (count > 0 ? count : 1) + 255) & ~(size_t)255;
        if (!ok || off + bytes > cap) { ok = false; *p = nullptr; return; }
        *p = reinterpret_cast<T *>(base + off);
        off += bytes;
    }
};

// Topology of one set written on the device (no host-to-device copies).
__global__ void k_one_set_topology(SetGeom *sets, int32_t *grp_set, int64_t ng, int32_t *bkt_set,
                                   int64_t nb, int64_t *pref, int max_depth, SetGeom g) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) sets[0] = g;
    if (t < ng) grp_set[t] = 0;
    if (t < nb) bkt_set[t] = 0;
    if (t <= max_depth) {
        pref[2 * t] = 0;
        pref[2 * t + 1] = g.nb > 0 ? (int64_t)(g.nbp >> t) : 0;
    }
}

}  // namespace

extern "C" {

void sph_default_params(sph_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->kernel = SPH_KERNEL_M4;
    p->precision = SPH_PREC_FP64;
    p->eos = SPH_EOS_IDEAL;
    p->periodic = 1;
    p->n_ngb = 64.0;
    for (int a = 0; a < 3; ++a) { p->box_lo[a] = 0.0; p->box_hi[a] = 1.0; }
    p->gamma = 5.0 / 3.0;
    p->P0 = 0.0;
    p->alpha = 1.0;
    p->beta = 2.0;
    p->eps_av = 0.01;
    p->eta_c = 0.3;
    p->eta_a = 0.2;
    p->dt_max = 1.0;
    p->h_max = 0.25;
    p->oversel = 1.1;
    p->nr_tol = 0.0;
    p->nr_maxit = 64;
    p->bucket = 32;
    p->ic_alpha = 10.0;
    p->rung_max = 8;
    p->fastgas = 0.0;
}

const char *sph_version(void) { return kVersion; }

const char *sph_last_error(const sph_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

sph_status sph_create_batch(const sph_params *params, int32_t nsets, const int64_t *set_offsets,
                            const double *set_box, sph_ctx **out) {
    if (!out) return SPH_ERR_INVALID;
    *out = nullptr;
    std::string why;
    if (!valid_params(params, why)) return SPH_ERR_INVALID;
    if (nsets < 1 || nsets > 4096) return SPH_ERR_INVALID;
    if (nsets > 1 && !set_offsets) return SPH_ERR_INVALID;
    if (nsets > 1 && (params->flags & SPH_FLAG_RUNGS)) return SPH_ERR_INVALID;
    if (set_offsets) {
        if (set_offsets[0] != 0) return SPH_ERR_INVALID;
        for (int q = 0; q < nsets; ++q)
            if (set_offsets[q + 1] < set_offsets[q]) return SPH_ERR_INVALID;
        if (set_offsets[nsets] > ((int64_t)1 << 31) - 1) return SPH_ERR_INVALID;
    }
    if (set_box) {
        for (int q = 0; q < nsets; ++q)
            for (int a = 0; a < 3; ++a)
                if (params->periodic && !(set_box[6 * q + 3 + a] > set_box[6 * q + a]))
                    return SPH_ERR_INVALID;
    }
    sph_ctx *x = new (std::nothrow) sph_ctx();
    if (!x) return SPH_ERR_OOM;
    Ctx &c = x->c;
    c.prm = *params;
    if (!(c.prm.nr_tol > 0))
        c.prm.nr_tol = c.prm.precision == SPH_PREC_MIXED ? 1e-5 : 1e-14;
    c.dyn = (c.prm.flags & SPH_FLAG_DYNAMIC) != 0;
    c.rungs_on = (c.prm.flags & SPH_FLAG_RUNGS) != 0;
    c.base_bucket = c.prm.bucket == 0 ? 32 : c.prm.bucket;
    c.bucket = c.dyn ? 8 : c.base_bucket;   // (dynamic sizing: the tree's buckets are the finest)
    if (c.prm.stack_limit == 0) c.prm.stack_limit = kStackCap;
    c.launch = c.prm.launch;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&c.ncu, hipDeviceAttributeMultiprocessorCount, dev);
    c.nsets = nsets;
    if (set_offsets) c.set_off.assign(set_offsets, set_offsets + nsets + 1);
    if (set_box) c.set_box.assign(set_box, set_box + 6 * nsets);
    *out = x;
    return SPH_OK;
}

sph_status sph_create(const sph_params *params, sph_ctx **out) {
    return sph_create_batch(params, 1, nullptr, nullptr, out);
}

void sph_destroy(sph_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    free_all(ctx->c);
    free_events(ctx->c);
    if (ctx->c.status_ev) (void)hipEventDestroy(ctx->c.status_ev);
    delete ctx;
}

sph_status sph_build_tree(sph_ctx *ctx, const sph_particles *p, int64_t n, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    sph_status st = check_particles(ctx, p, false, n);
    if (st != SPH_OK) return st;
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(ctx, SPH_ERR_INVALID, "bad n");
    if (c.nsets == 1) {
        c.set_off.assign({0, n});
    } else if (c.set_off.back() != n) {
        return fail(ctx, SPH_ERR_INVALID, "n differs from the batch total");
    }
    st = setup(ctx, n, s);
    if (st != SPH_OK) return st;
    c.last_stream = s;
    if (n > 0) HIPCHK(ctx, launch_tree_build(&c, p, s), "tree build");
    c.have_tree = true;
    return SPH_OK;
}

sph_status sph_neighbors(sph_ctx *ctx, const sph_particles *p, int32_t mode, int64_t *offsets,
                         int32_t *idx, int64_t capacity, int64_t *needed, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    if (!c.have_tree) return fail(ctx, SPH_ERR_STATE, "no tree: call sph_build_tree first");
    if (!offsets || !needed || (mode != SPH_MODE_GATHER && mode != SPH_MODE_FORCE))
        return fail(ctx, SPH_ERR_INVALID, "bad neighbour arguments");
    (void)p;
    {
        sph_status st = take_status(ctx);
        if (st != SPH_OK) return st;
    }
    c.last_stream = s;
    HIPCHK(ctx, reset_counters(c, s), "counters");
    // counts into offsets[0..n-1], offsets[n] = 0, then exclusive scan in place
    HIPCHK(ctx, launch_fill_u64(reinterpret_cast<unsigned long long *>(offsets), c.n + 1, 0ull, s),
           "fill");
    HIPCHK(ctx, launch_neighbors(&c, mode, offsets, nullptr, nullptr, s), "count");
    HIPCHK(ctx, launch_scan_i64(&c, offsets, offsets, c.n + 1, s), "scan");
    int64_t total = 0;
    HIPCHK(ctx, hipMemcpyAsync(&total, offsets + c.n, sizeof(int64_t), hipMemcpyDeviceToHost, s),
           "total");
    HIPCHK(ctx, hipStreamSynchronize(s), "sync");
    *needed = total;
    if (total > capacity || (!idx && total > 0))
        return fail(ctx, SPH_ERR_CAPACITY, "idx capacity below the number of pairs");
    if (total > 0) {
        HIPCHK(ctx, launch_neighbors(&c, mode, nullptr, offsets, idx, s), "fill");
        HIPCHK(ctx, launch_sort_rows(&c, offsets, idx, s), "sort rows");
    }
    HIPCHK(ctx, launch_fold_counters(&c, s), "fold counters");
    HIPCHK(ctx, hipMemcpyAsync(c.h_cnt, c.d_csum, sizeof(unsigned long long) * C_NCOUNTERS,
                               hipMemcpyDeviceToHost, s), "counters");
    HIPCHK(ctx, hipStreamSynchronize(s), "sync");
    if (c.h_cnt[C_ROWLONG]) return fail(ctx, SPH_ERR_CAPACITY, "a row exceeds 4096 entries");
    return SPH_OK;
}

sph_status sph_density(sph_ctx *ctx, sph_particles *p, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    if (!c.have_tree) return fail(ctx, SPH_ERR_STATE, "no tree: call sph_build_tree first");
    sph_status st = check_particles(ctx, p, true, c.n);
    if (st != SPH_OK) return st;
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    c.last_stream = s;
    HIPCHK(ctx, reset_counters(c, s), "counters");
    st = do_density(ctx, p, s);
    mark(&c, E_END, s);
    if (st == SPH_OK) HIPCHK(ctx, post_status(c, s), "status");
    return st;
}

sph_status sph_forces(sph_ctx *ctx, sph_particles *p, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    if (!c.have_tree) return fail(ctx, SPH_ERR_STATE, "no tree: call sph_build_tree first");
    sph_status st = check_particles(ctx, p, true, c.n);
    if (st != SPH_OK) return st;
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    c.last_stream = s;
    HIPCHK(ctx, reset_counters(c, s), "counters");
    st = do_forces(ctx, p, p->vx, p->vy, p->vz, p->u, true, s);
    if (st != SPH_OK) return st;
    HIPCHK(ctx, launch_reduce(&c, p, s), "reduce");
    HIPCHK(ctx, launch_set_dtnext(&c, p, s), "set dt");
    mark(&c, E_END, s);
    HIPCHK(ctx, post_status(c, s), "status");
    c.have_forces = true;
    return SPH_OK;
}

sph_status sph_init(sph_ctx *ctx, sph_particles *p, int64_t n, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    sph_status st = check_particles(ctx, p, true, n);
    if (st != SPH_OK) return st;
    st = sph_build_tree(ctx, p, n, stream);   // (takes the previous status)
    if (st != SPH_OK) return st;
    HIPCHK(ctx, launch_reset_counters(&c, C_NTRANSIENT, s), "counters");
    HIPCHK(ctx, launch_fill_u64(reinterpret_cast<unsigned long long *>(c.hprev), c.n, 0ull, s),
           "H history");
    if (c.dyn) {
        HIPCHK(ctx, reset_levels(c, c.levc, c.n, s), "levels");
        HIPCHK(ctx, launch_fill_u64(reinterpret_cast<unsigned long long *>(c.d_levref), 1, 0ull,
                                    s), "level reference");
    }
    st = do_density(ctx, p, s);
    if (st != SPH_OK) return st;
    if (c.prm.flags & SPH_FLAG_ENTROPY)
        HIPCHK(ctx, launch_copy(c.rho_old, p->rho, c.n, s), "rho_old");
    st = do_forces(ctx, p, p->vx, p->vy, p->vz, p->u, false, s);
    if (st != SPH_OK) return st;
    if (c.rungs_on) {
        st = init_rungs(ctx, p, s);
        if (st != SPH_OK) return st;
    }
    HIPCHK(ctx, launch_reduce(&c, p, s), "reduce");
    HIPCHK(ctx, launch_set_dtnext(&c, p, s), "set dt");
    mark(&c, E_END, s);
    HIPCHK(ctx, post_status(c, s), "status");
    c.have_forces = true;
    return SPH_OK;
}

sph_status sph_step(sph_ctx *ctx, sph_particles *p, double dt, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    if (!c.have_forces) return fail(ctx, SPH_ERR_STATE, "call sph_init before sph_step");
    sph_status st = check_particles(ctx, p, true, c.n);
    if (st != SPH_OK) return st;
    if (!(dt == dt)) return fail(ctx, SPH_ERR_INVALID, "dt is NaN");
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    c.last_stream = s;
    if (c.rungs_on && dt > 0.0)
        return fail(ctx, SPH_ERR_INVALID, "with individual time steps dt must be <= 0");
    st = c.rungs_on ? do_substep(ctx, p, s) : do_step(ctx, p, dt, s);
    if (st == SPH_OK) HIPCHK(ctx, post_status(c, s), "status");
    return st;
}

sph_status sph_graph_capture_step(sph_ctx *ctx, sph_particles *p, double dt, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    if (!c.have_forces) return fail(ctx, SPH_ERR_STATE, "call sph_init before capturing a step");
    if (c.rungs_on)
        return fail(ctx, SPH_ERR_INVALID, "individual time steps are not captured as a graph");
    sph_status st = check_particles(ctx, p, true, c.n);
    if (st != SPH_OK) return st;
    if (!s) return fail(ctx, SPH_ERR_INVALID, "graph capture needs a non-null stream");
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    if (c.graph_exec) { (void)hipGraphExecDestroy(c.graph_exec); c.graph_exec = nullptr; }
    if (c.graph) { (void)hipGraphDestroy(c.graph); c.graph = nullptr; }
    HIPCHK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    c.capturing = true;
    st = do_step(ctx, p, dt, s);
    c.capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != SPH_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    c.graph = g;
    HIPCHK(ctx, hipGraphInstantiate(&c.graph_exec, g, nullptr, nullptr, 0), "instantiate");
    return SPH_OK;
}

sph_status sph_graph_launch(sph_ctx *ctx, void *stream) {
    if (!ctx) return SPH_ERR_INVALID;
    Ctx &c = ctx->c;
    if (!c.graph_exec) return fail(ctx, SPH_ERR_STATE, "no captured graph");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    sph_status st = take_status(ctx);
    if (st != SPH_OK) return st;
    c.last_stream = s;
    HIPCHK(ctx, hipGraphLaunch(c.graph_exec, s), "graph launch");
    HIPCHK(ctx, post_status(c, s), "status");
    return SPH_OK;
}

sph_status sph_get_stats(sph_ctx *ctx, sph_stats *out) {
    if (!ctx || !out) return SPH_ERR_INVALID;
    Ctx &c = ctx->c;
    std::memset(out, 0, sizeof(*out));
    out->n = c.n;
    if (!c.d_cnt) return SPH_OK;
    HIPCHK(ctx, hipStreamSynchronize(c.last_stream), "sync");
    HIPCHK(ctx, hipMemcpy(c.h_cnt, c.d_csum, sizeof(unsigned long long) * C_NCOUNTERS,
                          hipMemcpyDeviceToHost), "counters");
    HIPCHK(ctx, hipMemcpy(c.h_rep, c.d_rep, sizeof(StepReport), hipMemcpyDeviceToHost), "report");
    out->pairs_density = (int64_t)c.h_cnt[C_PAIRS_D];
    out->pairs_force = (int64_t)c.h_cnt[C_PAIRS_F];
    out->cand_density = (int64_t)c.h_cnt[C_CAND_D];
    out->cand_force = (int64_t)c.h_cnt[C_CAND_F];
    out->nr_iter_max = (int64_t)c.h_cnt[C_NR_ITER_MAX];
    out->nr_scans = (int64_t)c.h_cnt[C_NR_SCANS];
    out->n_noconv = (int64_t)c.h_cnt[C_NOCONV];
    out->n_rewalk = (int64_t)c.h_cnt[C_REWALK];
    out->n_overflow = (int64_t)c.h_cnt[C_OVERFLOW];
    for (int a = 0; a < 3; ++a) out->momentum[a] = c.h_rep->momentum[a];
    out->e_kin = c.h_rep->e_kin;
    out->e_int = c.h_rep->e_int;
    out->dt_next = c.h_rep->dt_next;
    out->dt_used = c.h_rep->dt_used;
    out->pairs_density_total = (int64_t)c.h_cnt[C_PAIRS_D_TOT];
    out->pairs_force_total = (int64_t)c.h_cnt[C_PAIRS_F_TOT];
    out->n_iter_limit = (int64_t)c.h_cnt[C_ITERLIM];
    out->n_nonfinite = (int64_t)c.h_cnt[C_NONFINITE];
    out->n_retest = (int64_t)c.h_cnt[C_RETEST];
    out->status = (int32_t)flags_status(&c.h_cnt[C_ITERLIM]);
    out->slots_density = (int64_t)c.h_cnt[C_SLOTS_D];
    out->slots_force = (int64_t)c.h_cnt[C_SLOTS_F];
    for (int q = 0; q < 4; ++q) out->groups_by_level[q] = (int64_t)c.h_cnt[C_LEV0 + q];
    out->n_active = c.n;
    out->n_dens = c.n;
    if (c.rungs_on && c.d_rung) {
        RungState rs;
        HIPCHK(ctx, hipMemcpy(&rs, c.d_rung, sizeof(rs), hipMemcpyDeviceToHost), "rung state");
        out->t_units = rs.T;
        out->n_active = rs.nact;
        out->n_dens = c.prm.fastgas > 0.0 ? rs.ndens : c.n;
        out->n_fastgas_miss = (int64_t)c.h_cnt[C_FGMISS];
    }
    out->launch = c.sweep_launch;
    out->workgroups_force = c.sweep_workgroups;
    c.status_pending = false;   // reported here, not again by the next call
    auto span = [&](int a, int b) -> double {
        if (!((c.ev_mask >> a) & 1u) || !((c.ev_mask >> b) & 1u)) return -1.0;
        float ms = -1.0f;
        if (hipEventElapsedTime(&ms, c.ev[a], c.ev[b]) != hipSuccess) return -1.0;
        return (double)ms;
    };
    out->t_tree_ms = span(E_TREE0, E_TREE1);
    out->t_density_ms = span(E_DEN0, E_DEN1);
    out->t_forces_ms = span(E_FOR0, E_FOR1);
    out->t_force_walk_ms = span(E_FWALK0, E_FOR0);
    out->t_density_walk_ms = span(E_DWALK0, E_DEN0);
    out->groups_walked = (int64_t)c.h_cnt[C_WALKED];
    out->t_total_ms = span(E_BEGIN, E_END);
    return SPH_OK;
}

sph_status sph_set_timing(sph_ctx *ctx, int32_t enable) {
    if (!ctx) return SPH_ERR_INVALID;
    Ctx &c = ctx->c;
    if (enable && !c.ev[0]) {
        for (int e = 0; e < E_NEVENTS; ++e)
            HIPCHK(ctx, hipEventCreate(&c.ev[e]), "event create");
    }
    c.timing = enable != 0;
    c.ev_mask = 0;
    return SPH_OK;
}

sph_status sph_autotune(sph_ctx *ctx, sph_particles *p, int32_t *bucket, void *stream) {
    if (!ctx || !bucket) return SPH_ERR_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Ctx &c = ctx->c;
    const int64_t n = c.nsets > 1 ? c.set_off.back() : c.n;
    if (c.nsets == 1 && !c.have_tree)
        return fail(ctx, SPH_ERR_STATE, "sph_autotune needs a previous sph_build_tree or sph_init");
    sph_status st = check_particles(ctx, p, true, n);
    if (st != SPH_OK) return st;
    st = take_status(ctx);
    if (st != SPH_OK) return st;
    if (n == 0) { *bucket = c.dyn ? c.base_bucket : c.bucket; return SPH_OK; }
    // every trial starts from the same first guess of H (kept in the context's
    // scratch column, so the trials allocate nothing)
    st = setup(ctx, n, s);
    if (st != SPH_OK) return st;
    double *const H0 = c.d_h0;
    hipError_t e = hipMemcpyAsync(H0, p->H, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    const bool timing = c.timing;
    st = sph_set_timing(ctx, 1);
    const int cands[4] = {8, 16, 32, 64};
    int best = c.dyn ? c.base_bucket : c.bucket;
    int best_launch = c.launch;
    double tbest = 1e300;
    // every bucket size with every launch shape (substeps of individual time
    // steps launch one walking workgroup per group only)
    const int shapes[3] = {SPH_LAUNCH_GROUPS, SPH_LAUNCH_WALK, SPH_LAUNCH_PERSISTENT};
    const int nlaunch = c.rungs_on ? 2 : 3;
    for (int q = 0; q < 4 * nlaunch && st == SPH_OK && e == hipSuccess; ++q) {
        // (dynamic sizing: the tree keeps buckets of 8; the trials set the
        // level the groups start from)
        if (c.dyn) c.base_bucket = cands[q % 4];
        else c.bucket = cands[q % 4];
        c.launch = shapes[q / 4];
        double t = 1e300;
        for (int rep = 0; rep < 2 && st == SPH_OK && e == hipSuccess; ++rep) {
            e = hipMemcpyAsync(p->H, H0, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) break;
            st = sph_init(ctx, p, n, stream);
            // timed: a density and a force pass from the converged H, as in a
            // step (sph_init's own density pass starts from the first guess),
            // each with its walk kernel (smaller buckets shorten the sweeps'
            // lists but lengthen the walks)
            sph_stats ss;
            double td = -1.0, tf = -1.0;
            if (c.rungs_on) {
                if (st == SPH_OK) st = sph_get_stats(ctx, &ss);
                if (st == SPH_OK) { td = ss.t_density_ms; tf = ss.t_forces_ms; }
            } else {
                if (st == SPH_OK) st = sph_density(ctx, p, stream);
                if (st == SPH_OK) st = sph_get_stats(ctx, &ss);
                if (st == SPH_OK && ss.t_density_ms >= 0)
                    td = ss.t_density_ms + std::max(ss.t_density_walk_ms, 0.0);
                if (st == SPH_OK) st = sph_forces(ctx, p, stream);
                if (st == SPH_OK) st = sph_get_stats(ctx, &ss);
                if (st == SPH_OK && ss.t_forces_ms >= 0)
                    tf = ss.t_forces_ms + std::max(ss.t_force_walk_ms, 0.0);
            }
            if (td >= 0 && tf >= 0) t = std::min(t, td + tf);
        }
        if (t < tbest) { tbest = t; best = cands[q % 4]; best_launch = c.launch; }
    }
    c.launch = best_launch;
    if (st == SPH_OK && e == hipSuccess) {
        if (c.dyn) c.base_bucket = best;
        else c.bucket = best;
        e = hipMemcpyAsync(p->H, H0, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) st = sph_init(ctx, p, n, stream);
    }
    (void)hipStreamSynchronize(s);
    c.timing = timing;
    if (e != hipSuccess) return hip_fail(ctx, e, "autotune");
    if (st != SPH_OK) return st;
    *bucket = best;
    return SPH_OK;
}

sph_status sph_init_noalloc(const sph_params *params, sph_particles *p, int64_t n, void *stream) {
    std::string why;
    if (!valid_params(params, why)) return SPH_ERR_INVALID;
    if (params->flags & SPH_FLAG_RUNGS) return SPH_ERR_INVALID;   // (a global step only)
    if (n < 0) return SPH_ERR_INVALID;
    if (n > kNoAllocMaxN) return SPH_ERR_CAPACITY;   // beyond the static work space
    if (check_particles(nullptr, p, true, n) != SPH_OK) return SPH_ERR_INVALID;
    if ((params->flags & SPH_FLAG_EVOLVED) && n > 0 && !p->drhodt) return SPH_ERR_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPH_ERR_HIP;
    if (dev < 0 || dev >= kNoAllocDevices) return SPH_ERR_INVALID;
    if (!g_scratch[dev]) {
        // once per GPU, with that GPU current: the device address of its copy
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPH_ERR_HIP;
        g_scratch[dev] = static_cast<unsigned char *>(ptr);
        g_noalloc[dev].c.level_total.reserve(64);   // host bookkeeping, sized once
    }
    sph_ctx *const x = &g_noalloc[dev];
    Ctx &c = x->c;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c.prm = *params;
    if (!(c.prm.nr_tol > 0)) c.prm.nr_tol = c.prm.precision == SPH_PREC_MIXED ? 1e-5 : 1e-14;
    if (c.prm.stack_limit == 0) c.prm.stack_limit = kStackCap;
    c.dyn = (c.prm.flags & SPH_FLAG_DYNAMIC) != 0;
    c.base_bucket = c.prm.bucket == 0 ? 32 : c.prm.bucket;
    c.bucket = c.dyn ? 8 : c.base_bucket;
    c.launch = SPH_LAUNCH_WALK;   // (the static work space holds no queue and no lists)
    c.nsets = 1;
    c.timing = false;
    c.capturing = false;
    c.last_stream = s;
    if (n == 0) return SPH_OK;

    // topology of one set of n particles
    const int B = c.bucket;
    SetGeom g{};
    g.p0 = 0;
    g.p1 = n;
    const int64_t nb = (n + B - 1) / B;
    int64_t nbp = 1;
    int depth = 0;
    while (nbp < nb) { nbp <<= 1; ++depth; }
    g.nb = (int32_t)nb;
    g.nbp = (int32_t)nbp;
    g.depth = depth;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = c.prm.box_lo[a];
        g.L[a] = c.prm.box_hi[a] - c.prm.box_lo[a];
        g.halfL[a] = 0.5 * g.L[a];
    }
    c.n = n;
    c.nbuckets = nb;
    c.ngroups = (n + kGroup - 1) / kGroup;
    c.nnodes = 2 * nbp;
    c.max_depth = depth;
    c.level_total.assign(depth + 1, 0);   // within the reserved capacity
    for (int d = 0; d <= depth; ++d) c.level_total[d] = nbp >> d;
    c.set_bits = 0;
    c.key_passes = (3 * key_bits_per_axis() + 7) / 8;
    c.sort_blocks = sort_blocks_needed(n);
    c.scan_tmp_len = scan_tmp_needed(std::max<int64_t>(n + 1, 256 * std::max<int64_t>(c.sort_blocks, 1)));

    Carve cv{g_scratch[dev], 0, kNoAllocBytes, true};
    int64_t *pref = nullptr;
    cv.take(&c.d_sets, 1);
    cv.take(&c.d_grp_set, c.ngroups);
    cv.take(&c.d_bkt_set, nb);
    cv.take(&pref, 2 * (depth + 1));
    c.d_level_pref = pref;
    cv.take(&c.d_key[0], n); cv.take(&c.d_key[1], n);
    cv.take(&c.d_perm[0], n); cv.take(&c.d_perm[1], n);
    cv.take(&c.d_hist, 2 * 256 * std::max<int64_t>(c.sort_blocks, 1));
    cv.take(&c.d_bbox, 6);
    cv.take(&c.xs, n); cv.take(&c.ys, n); cv.take(&c.zs, n); cv.take(&c.ms, n); cv.take(&c.Hs, n);
    cv.take(&c.vxs, n); cv.take(&c.vys, n); cv.take(&c.vzs, n); cv.take(&c.us, n);
    cv.take(&c.rhos, n); cv.take(&c.oms, n); cv.take(&c.As, n); cv.take(&c.css, n); cv.take(&c.Ps, n);
    c.frec1 = c.frec2 = c.fm = nullptr;
    c.drec1 = c.drec2 = nullptr;
    if (c.prm.precision == SPH_PREC_MIXED) {
        cv.take(&c.frec1, 4 * n); cv.take(&c.frec2, 4 * n); cv.take(&c.fm, n);
    } else {
        cv.take(&c.drec1, 4 * n); cv.take(&c.drec2, 4 * n);
    }
    cv.take(&c.axs, n); cv.take(&c.ays, n); cv.take(&c.azs, n); cv.take(&c.dus, n); cv.take(&c.dts, n);
    cv.take(&c.nodes, c.nnodes);
    c.drs = nullptr;
    if (c.prm.flags & SPH_FLAG_EVOLVED) cv.take(&c.drs, n);
    c.mats = c.imbs = c.tbar = c.pbar = nullptr;
    c.levc = c.levs = c.d_levref = nullptr;
    if (c.dyn) { cv.take(&c.levc, n); cv.take(&c.levs, n); cv.take(&c.d_levref, 1); }
    if (c.prm.flags & SPH_FLAG_INTERFACE) {
        cv.take(&c.mats, n); cv.take(&c.imbs, n); cv.take(&c.tbar, n); cv.take(&c.pbar, n);
    }
    cv.take(&c.d_wstack, (size_t)c.ngroups * kStackCap);
    cv.take(&c.d_scan_tmp, c.scan_tmp_len);
    cv.take(&c.d_cnt, kCntShards * kCntStride);
    cv.take(&c.d_csum, C_NCOUNTERS);
    if (!cv.ok) return SPH_ERR_CAPACITY;

    const int64_t nt = std::max<int64_t>(std::max<int64_t>(c.ngroups, nb), depth + 1);
    k_one_set_topology<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(
        c.d_sets, c.d_grp_set, c.ngroups, c.d_bkt_set, nb, pref, depth, g);
    if (hipGetLastError() != hipSuccess) return SPH_ERR_HIP;
    if (launch_init_nodes(&c, s) != hipSuccess) return SPH_ERR_HIP;
    if (launch_fill_u64(c.d_cnt, kCntShards * kCntStride, 0ull, s) != hipSuccess ||
        launch_fill_u64(c.d_csum, C_NCOUNTERS, 0ull, s) != hipSuccess)
        return SPH_ERR_HIP;
    if (c.dyn && (reset_levels(c, c.levc, n, s) != hipSuccess ||
                  launch_fill_u64(reinterpret_cast<unsigned long long *>(c.d_levref), 1, 0ull, s) !=
                      hipSuccess))
        return SPH_ERR_HIP;
    if (launch_tree_build(&c, p, s) != hipSuccess) return SPH_ERR_HIP;
    sph_status st = do_density(x, p, s);
    if (st != SPH_OK) return st;
    return do_forces(x, p, p->vx, p->vy, p->vz, p->u, false, s);
}

}  // extern "C"

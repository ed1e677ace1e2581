// sph_sweep.hip -- the neighbour-interaction sweep on gfx950.
//
//   walk      one wavefront per sink group of 64 consecutive (Hilbert-ordered)
//             particles walks its set's bucket tree with the bound-overlap
//             tests of Sec. 2.3.2 / Fig. 1: gather = sink box-of-balls AND
//             sink ball-of-balls overlap the source cell bound; scatter =
//             source box-of-balls AND ball-of-balls overlap the sink cell
//             bound.  Up to 64 nodes are tested per step (one per lane);
//             accepted children are pushed on the group's stack (global
//             memory) and accepted buckets appended to an LDS candidate list
//             by ballot + popcount compaction.  The list holds whole buckets
//             (Sec. 2.3.2: lists are not pruned pairwise during the walk); a
//             per-sink refinement (FP32, conservative) then drops buckets
//             that no sink of the group needs.
//   tiles     candidates are staged 64 at a time into LDS, each tile taking
//             runs of 2 slots spread over the whole list; each lane (one
//             sink) tests its distance to every staged candidate, the
//             accepted pairs go through a small LDS ring and are evaluated
//             one pair per lane (see "pair compaction").
//   density   the pairs add m f, m q f' and m (2 q f' + q^2 f'') to per-sink
//             sums (eq:Density_estimate and its H derivatives); a Halley
//             iteration on the constant kernel mass (Sec. 2.3.3) re-scans the
//             same candidate list (the walk used oversel*H so H can grow; a
//             group whose H outgrows it is re-walked).
//   forces    same structure over the gather-or-scatter list with the
//             symmetrised pressure force, PdV du/dt, Monaghan viscosity and
//             the time-step limits (Sec. 2.3.5, 2.3.6).
//
// Precision: FP64 path = every pair operation in FP64 with the pair distance
// evaluated as (dx*dx + dy*dy) + dz*dz without contraction, so neighbour
// sets are reproducible bit for bit.  Mixed path = pair arithmetic in FP32 on
// coordinates relative to the sink group's centre (formed in FP64, rounded
// once per staged candidate); the FP32 pair terms are summed in FP64 per
// sink; H iteration bookkeeping, positions and outputs stay FP64.
#include "sph_internal.h"

#include <cfloat>
#include <type_traits>

namespace sphmi {

namespace {

// ---------------------------------------------------------------- kernels
constexpr double kPi = 3.14159265358979323846;

template <int K> __device__ __forceinline__ double sigma_of() {
    return K == 0 ? 8.0 / kPi : K == 1 ? 21.0 / (2.0 * kPi) : K == 2 ? 495.0 / (32.0 * kPi)
                                                                   : 1365.0 / (64.0 * kPi);
}

// f(q) and q f'(q) on 0 <= q <= 1 (s clamped so rounding at q ~ 1 stays harmless).
template <int K, typename R>
__device__ __forceinline__ void shape_f_qfp(R q, R &f, R &qfp) {
    R s = R(1) - q;
    s = s > R(0) ? s : R(0);
    if constexpr (K == 0) {
        if (q < R(0.5)) {
            f = R(1) + q * q * (R(6) * q - R(6));
            qfp = q * q * (R(18) * q - R(12));
        } else {
            f = R(2) * s * s * s;
            qfp = R(-6) * q * s * s;
        }
    } else if constexpr (K == 1) {
        R s3 = s * s * s;
        f = s3 * s * (R(1) + R(4) * q);
        qfp = R(-20) * q * q * s3;
    } else if constexpr (K == 2) {
        R s2 = s * s, s5 = s2 * s2 * s;
        f = s5 * s * (R(1) + q * (R(6) + q * R(35.0 / 3.0)));
        qfp = R(-56.0 / 3.0) * q * q * s5 * (R(1) + R(5) * q);
    } else {
        R s2 = s * s, s4 = s2 * s2, s7 = s4 * s2 * s;
        f = s7 * s * (R(1) + q * (R(8) + q * (R(25) + q * R(32))));
        qfp = R(-22) * q * q * s7 * (R(1) + q * (R(7) + q * R(16)));
    }
}

// f, t1 = q f'(q) and t2 = 2 q f'(q) + q^2 f''(q): with S0 = sum m f,
// T1 = sum m t1, T2 = sum m t2 over r < H, d S0/dH = -T1/H and
// d^2 S0/dH^2 = T2/H^2 (the smoothing-length iteration uses both).
template <int K, typename R>
__device__ __forceinline__ void shape_f_t1_t2(R q, R &f, R &t1, R &t2) {
    R s = R(1) - q;
    s = s > R(0) ? s : R(0);
    const R q2 = q * q;
    if constexpr (K == 0) {
        if (q < R(0.5)) {
            f = R(1) + q2 * (R(6) * q - R(6));
            t1 = q2 * (R(18) * q - R(12));
            t2 = R(36) * q2 * (R(2) * q - R(1));
        } else {
            f = R(2) * s * s * s;
            t1 = R(-6) * q * s * s;
            t2 = R(12) * q * s * (R(2) * q - R(1));
        }
    } else if constexpr (K == 1) {
        const R s2 = s * s, s3 = s2 * s;
        f = s3 * s * (R(1) + R(4) * q);
        t1 = R(-20) * q2 * s3;
        t2 = R(60) * q2 * s2 * (R(2) * q - R(1));
    } else if constexpr (K == 2) {
        const R s2 = s * s, s4 = s2 * s2, s5 = s4 * s;
        f = s5 * s * (R(1) + q * (R(6) + q * R(35.0 / 3.0)));
        t1 = R(-56.0 / 3.0) * q2 * s5 * (R(1) + R(5) * q);
        t2 = R(56) * q2 * s4 * (q * (R(15) * q - R(4)) - R(1));
    } else {
        const R s2 = s * s, s4 = s2 * s2, s6 = s4 * s2, s7 = s6 * s;
        f = s7 * s * (R(1) + q * (R(8) + q * (R(25) + q * R(32))));
        t1 = R(-22) * q2 * s7 * (R(1) + q * (R(7) + q * R(16)));
        t2 = R(66) * q2 * s6 * (q * (q * (R(64) * q - R(1)) - R(6)) - R(1));
    }
}

// g(q) = f'(q)/q.  The outer cubic-spline piece (q >= 1/2, so r > 0) needs
// 1/q = H/r; it is formed only in that branch.
template <int K, typename R>
__device__ __forceinline__ R shape_g(R q, R H, R r) {
    R s = R(1) - q;
    s = s > R(0) ? s : R(0);
    if constexpr (K == 0) {
        if (q < R(0.5)) return R(18) * q - R(12);
        return R(-6) * s * s * (H / r);
    } else if constexpr (K == 1) {
        return R(-20) * s * s * s;
    } else if constexpr (K == 2) {
        R s2 = s * s;
        return R(-56.0 / 3.0) * s2 * s2 * s * (R(1) + R(5) * q);
    } else {
        R s2 = s * s, s4 = s2 * s2;
        return R(-22) * s4 * s2 * s * (R(1) + q * (R(7) + q * R(16)));
    }
}

// ---------------------------------------------------------------- geometry

__device__ __forceinline__ double min_image(double d, double L, double hL) {
    if (d > hL) return d - L;
    if (d < -hL) return d + L;
    return d;
}

// r^2 = (dx*dx + dy*dy) + dz*dz without FMA contraction (reproducible membership).
__device__ __forceinline__ double r2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    return r2;
}

// Wave-uniform value moved to scalar registers (the reductions below leave
// the same value in every lane; saying so frees vector registers).
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_min(double v) { return uniform(seg_reduce<false>(v, 64)); }
__device__ __forceinline__ double wave_max(double v) { return uniform(seg_reduce<true>(v, 64)); }
__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct Sink {
    double clo[3], chi[3];  // cell bound of the group
    double blo[3], bhi[3];  // box of the balls of radius Hw
    double bc[3], br;       // enclosing sphere of the balls
};

__device__ inline void sink_bounds(bool act, const double *x, double Hw, Sink &sk) {
    for (int a = 0; a < 3; ++a) {
        sk.clo[a] = wave_min(act ? x[a] : DBL_MAX);
        sk.chi[a] = wave_max(act ? x[a] : -DBL_MAX);
        sk.blo[a] = wave_min(act ? x[a] - Hw : DBL_MAX);
        sk.bhi[a] = wave_max(act ? x[a] + Hw : -DBL_MAX);
        sk.bc[a] = uniform(0.5 * (sk.clo[a] + sk.chi[a]));
    }
    double r = 0.0;
    if (act) {
        double dx = x[0] - sk.bc[0], dy = x[1] - sk.bc[1], dz = x[2] - sk.bc[2];
        r = sqrt(dx * dx + dy * dy + dz * dz) + Hw;
    }
    sk.br = wave_max(r) * (1.0 + 1e-12);
}

// Distance between interval centres along one axis (minimum image when periodic).
__device__ __forceinline__ double cdist(double ca, double cb, double L, double hL, bool per) {
    double d = cb - ca;
    if (per) d = min_image(d, L, hL);
    return fabs(d);
}

__device__ __forceinline__ bool box_box(const double *alo, const double *ahi, const double *blo,
                                        const double *bhi, const SetGeom &g, bool per, double slop) {
    for (int a = 0; a < 3; ++a) {
        if (!(blo[a] <= bhi[a]) || !(alo[a] <= ahi[a])) return false;
        double ca = 0.5 * (alo[a] + ahi[a]), wa = 0.5 * (ahi[a] - alo[a]);
        double cb = 0.5 * (blo[a] + bhi[a]), wb = 0.5 * (bhi[a] - blo[a]);
        if (cdist(ca, cb, g.L[a], g.halfL[a], per) - wa - wb > slop) return false;
    }
    return true;
}

__device__ __forceinline__ bool ball_box(const double *c, double R, const double *blo,
                                         const double *bhi, const SetGeom &g, bool per, double slop) {
    if (!(R >= 0.0)) return false;
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!(blo[a] <= bhi[a])) return false;
        double cb = 0.5 * (blo[a] + bhi[a]), wb = 0.5 * (bhi[a] - blo[a]);
        double gap = cdist(c[a], cb, g.L[a], g.halfL[a], per) - wb;
        gap = gap > 0.0 ? gap : 0.0;
        d2 += gap * gap;
    }
    double Rs = R + slop;
    return d2 <= Rs * Rs;
}

// Walk state lives in the stack (global memory for the density and force
// kernels, LDS for the neighbour lists), the LDS candidate list and
// wave-uniform registers.
// In tree mode `lin` is -1; a group whose stack would overflow restarts in
// linear mode, where `lin` is the next bucket of the set to test (every bucket
// is tested once with the same bound tests, so the result does not depend on
// the stack size).  `nstack > 0` means "more candidates to come" in both modes.
struct WalkState {
    int nstack;
    int ncand;
    int lin;
    int cap;       // stack entries in use (<= kStackCap)
    bool overflow;
    bool far;      // after refine: a kept bucket may need the periodic image
};

// The walk starts from all nodes of one level of the heap (up to 64, one per
// lane) instead of the root: a node's bounds contain its children's, so the
// skipped ancestors could only have accepted what their descendants accept,
// and the first, nearly empty steps of the walk are saved.
__device__ __forceinline__ void walk_reset(uint32_t *stack, WalkState &w, bool linear,
                                           const SetGeom &g) {
    int d0 = g.depth < 6 ? g.depth : 6;
    while (d0 > 0 && (2 << d0) > w.cap) --d0;
    const int nstart = 1 << d0;
    if ((int)threadIdx.x < nstart) stack[threadIdx.x] = (uint32_t)(nstart + (int)threadIdx.x);
    w.nstack = nstart;
    w.ncand = 0;
    w.lin = linear ? 0 : -1;
    w.overflow = false;
    __syncthreads();
}

// Continue the walk until the stack is empty or the candidate list is nearly
// full (the caller consumes it and calls again).  The walk and the refinement
// run at a raised wave priority: each of their steps waits on memory, and
// letting them issue ahead of the other waves' tile arithmetic overlaps that
// wait with it (FP64 sweeps 4 % faster at 2M; the mixed ones unchanged).
template <bool SCATTER>
__device__ void walk(const SetGeom &g, bool per, double slop, const Node *__restrict__ nodes,
                     const Sink &sk, uint32_t *stack, uint32_t *cand, WalkState &w) {
    __builtin_amdgcn_s_setprio(2);
    const int lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;
    if (w.lin >= 0) {
        while (w.lin < g.nb && w.ncand <= kCandCap - kWave) {
            const int b = w.lin + lane;
            bool ok = false;
            if (b < g.nb) {
                const Node *nd = nodes + g.node0 + g.nbp + b;
                double clo[3] = {nd->clo[0], nd->clo[1], nd->clo[2]};
                double chi[3] = {nd->chi[0], nd->chi[1], nd->chi[2]};
                ok = box_box(sk.blo, sk.bhi, clo, chi, g, per, slop) &&
                     ball_box(sk.bc, sk.br, clo, chi, g, per, slop);
                if (SCATTER && !ok) {
                    double blo[3] = {nd->blo[0], nd->blo[1], nd->blo[2]};
                    double bhi[3] = {nd->bhi[0], nd->bhi[1], nd->bhi[2]};
                    double bc[3] = {nd->bc[0], nd->bc[1], nd->bc[2]};
                    ok = box_box(blo, bhi, sk.clo, sk.chi, g, per, slop) &&
                         ball_box(bc, nd->br, sk.clo, sk.chi, g, per, slop);
                }
            }
            const uint64_t m = __ballot(ok);
            if (ok) cand[w.ncand + __popcll(m & lt)] = (uint32_t)(g.b0 + b);
            w.ncand += __popcll(m);
            w.lin += kWave;
        }
        w.nstack = w.lin < g.nb ? 1 : 0;
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        return;
    }
    while (w.nstack > 0 && w.ncand <= kCandCap - kWave) {
        int k = w.nstack < kWave ? w.nstack : kWave;
        if (w.nstack + k > w.cap) k = w.cap - w.nstack;
        if (k <= 0) { w.overflow = true; w.nstack = 0; break; }
        const int base = w.nstack - k;
        uint32_t h = lane < k ? stack[base + lane] : 0u;
        __syncthreads();
        bool ok = false;
        if (lane < k) {
            // all bounds of the node are read at once: each step of the walk
            // then waits for one round trip to memory, not two
            const Node nd = nodes[g.node0 + h];
            ok = box_box(sk.blo, sk.bhi, nd.clo, nd.chi, g, per, slop) &&
                 ball_box(sk.bc, sk.br, nd.clo, nd.chi, g, per, slop);
            if (SCATTER) {
                const bool sc = box_box(nd.blo, nd.bhi, sk.clo, sk.chi, g, per, slop) &&
                                ball_box(nd.bc, nd.br, sk.clo, sk.chi, g, per, slop);
                ok = ok || sc;
            }
        }
        const bool leaf = h >= (uint32_t)g.nbp;
        const bool inner_ok = ok && !leaf;
        const bool leaf_ok = ok && leaf && (h - (uint32_t)g.nbp) < (uint32_t)g.nb;
        const uint64_t m1 = __ballot(inner_ok);
        const uint64_t m2 = __ballot(leaf_ok);
        if (inner_ok) {
            int p = __popcll(m1 & lt);
            stack[base + 2 * p] = 2u * h;
            stack[base + 2 * p + 1] = 2u * h + 1u;
        }
        if (leaf_ok) {
            int p = __popcll(m2 & lt);
            cand[w.ncand + p] = (uint32_t)(g.b0 + (int64_t)(h - (uint32_t)g.nbp));
        }
        w.nstack = base + 2 * __popcll(m1);
        w.ncand += __popcll(m2);
        __syncthreads();
    }
    __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ float wrap_f(float d, float L, float hL) {
    if (d > hL) return d - L;
    if (d < -hL) return d + L;
    return d;
}

__device__ __forceinline__ bool group_needs_wrap(bool per, const SetGeom &g, const double *gext,
                                                 double reach) {
    if (!per) return false;
    for (int a = 0; a < 3; ++a)
        if (gext[a] + reach >= 0.5 * g.L[a] * (1.0 - 1e-6)) return true;
    return false;
}

// Four values staged together so one LDS instruction moves them.
template <typename R> struct alignas(4 * sizeof(R)) V4 { R x, y, z, w; };

// Four consecutive entries of an LDS array (one 128-bit read for FP32).
template <typename R>
__device__ __forceinline__ V4<R> ld4(const R *p) { return *reinterpret_cast<const V4<R> *>(p); }

// Per-sink refinement of the candidate buckets: the group-level bounds of the
// walk accept a bucket when it may hold a neighbour of ANY sink; here every
// lane tests its own ball (gather) and, for the force pass, whether it lies
// inside the bucket's box-of-balls and ball-of-balls (scatter).  Buckets that
// no lane needs are dropped (order kept), so the tiles carry fewer candidates.
// Dropping a bucket is the only decision made here: keeping one too many costs
// time, never results.
//
// The tests run branch-free in FP32 on bounds relative to the group centre
// gc.  The lane that loads a bucket (kRefineBatch at a time, one per lane)
// turns each bound into a centre offset from gc (its minimum image when
// periodic) and a half width or radius, widened by 1e-5 of the bound's reach
// plus the set's slop; FP32 rounds these values and the sinks' offsets to
// within 6e-8 of their size, so the widened tests keep every bucket the exact
// FP64 tests would.  A bound that comes within the group's reach of half a
// box from gc has no image common to all sinks; such a bucket is kept
// untested.  The records (kRefineRec floats each) go to an LDS stage.
// `w.far` reports whether any kept bucket reaches within the group's extent
// gext of half a box from gc on some axis, i.e. whether one of its particles
// may need the minimum image (a superset of `needs_image`, as every particle
// lies inside its bucket's cell bound).
constexpr int kRefineBatch = 32;
constexpr int kRefineRec = 20;   // cell centre + half width (6), keep flag, box of balls (6), ball (4)
constexpr int kRefineStageBytes = kRefineBatch * kRefineRec * (int)sizeof(float);

template <bool SCATTER>
__device__ void refine(const SetGeom &g, bool per, double slop, const Node *__restrict__ nodes,
                       const double *xi, double R, double Rmax, bool act, const double *gc,
                       const double *gext, uint32_t *cand, float *stage, WalkState &w) {
    const int lane = threadIdx.x;
    constexpr int NB = kRefineBatch;
    __builtin_amdgcn_s_setprio(2);   // (see walk)
    float q[3];   // the sink's offset from gc
    for (int c = 0; c < 3; ++c)
        q[c] = (float)(per ? min_image(xi[c] - gc[c], g.L[c], g.halfL[c]) : xi[c] - gc[c]);
    const double Rw = R * (1.0 + 1e-5) + slop;
    const float R2 = act ? (float)(Rw * Rw) * (1.0f + 1e-6f) : -1.0f;
    const double gmax = fmax(gext[0], fmax(gext[1], gext[2]));
    int kept = 0;
    bool far = false;
    for (int t0 = 0; t0 < w.ncand; t0 += NB) {
        const int nb = min(NB, w.ncand - t0);
        uint32_t bl = 0;
        int bfar = 0;
        if (lane < nb) {
            bl = cand[t0 + lane];
            const Node nd = nodes[g.node0 + g.nbp + ((int64_t)bl - g.b0)];
            float *rec = stage + lane * kRefineRec;
            bool keep = false;
            double smax = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double lo = nd.clo[c], hi = nd.chi[c];
                if (per && fmax(fabs(lo - gc[c]), fabs(hi - gc[c])) + gext[c] >= 0.999 * g.halfL[c])
                    bfar = 1;
                double cc = 0.5 * (lo + hi) - gc[c];
                const double hw = 0.5 * (hi - lo);
                if (per) cc = min_image(cc, g.L[c], g.halfL[c]);
                if (!(hw >= 0.0) || (per && fabs(cc) + hw + gext[c] + Rmax >= 0.499 * g.L[c]))
                    keep = true;
                rec[c] = (float)cc;
                rec[3 + c] = (float)(hw + 1e-5 * (fabs(cc) + hw + gext[c] + Rmax) + slop);
                if (SCATTER) {
                    double bcc = 0.5 * (nd.blo[c] + nd.bhi[c]) - gc[c];
                    const double bw = 0.5 * (nd.bhi[c] - nd.blo[c]);
                    if (per) bcc = min_image(bcc, g.L[c], g.halfL[c]);
                    if (!(bw >= 0.0) || (per && fabs(bcc) + bw + gext[c] >= 0.499 * g.L[c]))
                        keep = true;
                    rec[8 + c] = (float)bcc;
                    rec[11 + c] = (float)(bw + 1e-5 * (fabs(bcc) + bw + gext[c]) + slop);
                    double sc = nd.bc[c] - gc[c];
                    if (per) sc = min_image(sc, g.L[c], g.halfL[c]);
                    if (per && fabs(sc) + nd.br + gext[c] >= 0.499 * g.L[c]) keep = true;
                    rec[16 + c] = (float)sc;
                    smax = fmax(smax, fabs(sc));
                }
            }
            rec[6] = keep ? 1.0f : 0.0f;
            if (SCATTER) {
                if (!(nd.br >= 0.0)) rec[6] = 1.0f;
                const double rr = nd.br + 1e-5 * (smax + nd.br + gmax) + slop;
                rec[19] = (float)(rr * rr) * (1.0f + 1e-6f);
            }
        }
        __syncthreads();
        for (int u = 0; u < nb; ++u) {
            const float *rec = stage + u * kRefineRec;
            const V4<float> r0 = ld4(rec), r1 = ld4(rec + 4);
            const float gx = fmaxf(fabsf(q[0] - r0.x) - r0.w, 0.0f);
            const float gy = fmaxf(fabsf(q[1] - r0.y) - r1.x, 0.0f);
            const float gz = fmaxf(fabsf(q[2] - r0.z) - r1.y, 0.0f);
            bool ok = r1.z != 0.0f || fmaf(gx, gx, fmaf(gy, gy, gz * gz)) <= R2;
            if (SCATTER) {
                const V4<float> r2 = ld4(rec + 8), r3 = ld4(rec + 12), r4 = ld4(rec + 16);
                const float ex = fabsf(q[0] - r2.x) - r2.w;
                const float ey = fabsf(q[1] - r2.y) - r3.x;
                const float ez = fabsf(q[2] - r2.z) - r3.y;
                const float sx = q[0] - r4.x, sy = q[1] - r4.y, sz = q[2] - r4.z;
                ok = ok || (fmaxf(ex, fmaxf(ey, ez)) <= 0.0f &&
                            fmaf(sx, sx, fmaf(sy, sy, sz * sz)) <= r4.w);
            }
            ok = ok && act;
            if (__any(ok)) {
                if (lane == 0) cand[kept] = (uint32_t)__builtin_amdgcn_readlane((int)bl, u);
                far = far || __builtin_amdgcn_readlane(bfar, u) != 0;
                ++kept;
            }
        }
        __syncthreads();
    }
    w.ncand = kept;
    w.far = far;
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
}

// Per-sink sums are accumulated in FP64 in both paths: the pair terms of the
// mixed path are FP32, their sum is not.  (LDS atomic adds are native for
// FP64 on gfx950; the FP32 form was measured several times slower, and a
// wider accumulator also replaces a compensated FP32 sum.)  The largest
// signal term is a maximum of non-negative values, kept as the integer
// maximum of their bit patterns.
__device__ __forceinline__ void lds_max_nonneg(uint32_t *p, float v) {
    atomicMax(p, __float_as_uint(v));
}
__device__ __forceinline__ void lds_max_nonneg(unsigned long long *p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ float bits_to_real(uint32_t b) { return __uint_as_float(b); }
__device__ __forceinline__ double bits_to_real(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD b mod
// 8), and each XCD has its own L2.  Sink groups are numbered along the
// Hilbert curve, so neighbouring groups share most of their candidates; this
// permutation gives every XCD one contiguous range of groups, so those shared
// candidates are fetched into one L2 instead of eight.
__device__ __forceinline__ int64_t xcd_group(int64_t b, int64_t n) {
    const int64_t q = n / kXcds, r = n % kXcds;
    const int64_t x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Persistent launch: as many workgroups as the CUs hold at once, each taking
// sink groups until none is left.  The groups are split into the same kXcds
// contiguous ranges that xcd_group deals out, one queue counter per range (on
// its own 256-byte line); a wave takes the next group of its own XCD's range
// and, once that is empty, of the following ranges in turn, so an XCD that
// finishes early helps the others.  Returns -1 once every range is empty: each
// call either returns a group or moves k on, so every wave exits after at
// most ngroups + kXcds fetches.  The counters start at zero (cleared before
// the launch).
__device__ __forceinline__ int64_t next_group(uint32_t *queue, int64_t n, int &k) {
    const int x0 = (int)(blockIdx.x % kXcds);
    const int64_t q = n / kXcds, r = n % kXcds;
    while (k < kXcds) {
        const int x = (x0 + k) % kXcds;
        const int64_t len = q + (x < r ? 1 : 0);
        uint32_t t = 0;
        if (threadIdx.x == 0) t = atomicAdd(&queue[x * kQueueStride], 1u);
        // (all 64 lanes are active here: lane 0's value, as a scalar, so that
        // the group index and all that follows from it stay in SGPRs)
        t = __builtin_amdgcn_readfirstlane(t);
        if ((int64_t)t < len) return x * q + (x < r ? x : r) + (int64_t)t;
        ++k;
    }
    return -1;
}

struct SweepArgs {
    const SetGeom *sets;
    const int32_t *grp_set;
    const Node *nodes;
    const uint32_t *perm;
    const double *xs, *ys, *zs, *ms;
    double *Hs, *rhos, *oms;
    const double *vxs, *vys, *vzs, *As, *css;
    const float *frec1, *frec2, *fm;   // mixed force records (see the EOS pass)
    const double *drec1, *drec2;       // FP64 force records
    double *ax, *ay, *az, *du, *dt;
    double *drho;           // evolved density: continuity rate (sorted), else null
    // interface correction (sorted): material ids (null: one material),
    // imbalance, u and P of the EOS pass, the averages, normalisation alpha
    const double *mats;
    double *imb;
    const double *us, *Ps_;
    double *tbar, *pbar;
    double ic_alpha;
    int entropy;            // du/dt without the PdV term (entropy-conserving update)
    unsigned long long *cnt;
    int B;                  // bucket size of the tree (the finest with dynamic sizing)
    const double *levs;     // dynamic bucket sizing: per sorted particle, the level h of
    double *levs_out;       //   its group (buckets of B 2^h); null when off
    int lev_max;            //   largest level (B 2^lev_max <= 64)
    const double *lev_ref;  //   mean list length per pair of the previous force pass
    int periodic;
    double oversel, tol, h_max, n_ngb;
    int maxit;
    int stack_limit;
    double alpha, beta, eps, eta_a, eta_c, dt_max;
    // neighbour lists
    int64_t *row_count;     // caller order (count pass)
    const int64_t *offsets; // caller order (fill pass)
    int32_t *idx;
    uint32_t *wstack;       // walk stacks of the sweeps (kStackCap per sink group)
    // individual time steps: sink lists (sorted indices of the sinks; null: a
    // group is a run of 64 consecutive particles) and their lengths (device),
    // each particle's rung packed with a FastGas flag (rung | 256 when its
    // density is not of this substep), the largest rung over F_i (out), marks
    const uint32_t *sinks;
    const long long *nsinks;
    const int32_t *rpack;
    double *nbmax;
    uint32_t *mark;
    double fastgas;         // active fraction below which FastGas marks
    // persistent launch: per-XCD queue counters (null: one workgroup per
    // sink group) and the number of sink groups
    uint32_t *queue;
    int64_t ngroups;
    // stored interaction lists (k_walk; kListCap buckets and a header of
    // kWalkWords per group) and the flags of the groups left to the walking
    // kernels (null in a walking launch: every group)
    const uint32_t *wlist;
    const int32_t *whdr;
    int32_t *defer;
    uint32_t *wlist_out;
    int32_t *whdr_out;
};

// The sinks of group grp: sorted indices i (one per lane) and whether the
// lane holds one.  With a sink list the groups are its runs of 64 entries;
// groups past its end have no sinks (the caller returns before any barrier).
__device__ __forceinline__ bool group_sinks(const SweepArgs &a, const SetGeom &g, int64_t grp,
                                            int64_t &i, bool &act) {
    const int lane = threadIdx.x;
    if (a.sinks) {
        const int64_t kb = grp * kGroup;
        const int64_t ns = *a.nsinks;
        if (kb >= ns) return false;
        act = kb + lane < ns;
        i = (int64_t)a.sinks[act ? kb + lane : kb];
        return true;
    }
    i = g.p0 + (grp - g.g0) * kGroup + lane;
    act = i < g.p1;
    return true;
}

// Sorted index of the sink of lane s of group grp (band re-tests).
__device__ __forceinline__ int64_t sink_index(const SweepArgs &a, const SetGeom &g, int64_t grp,
                                              int s) {
    if (a.sinks) return (int64_t)a.sinks[grp * kGroup + s];
    return g.p0 + (grp - g.g0) * kGroup + s;
}

__device__ __forceinline__ double set_slop(const SetGeom &g) {
    return 1e-9 * (g.L[0] + g.L[1] + g.L[2]);
}
__device__ __forceinline__ double set_hcap(const SetGeom &g, bool per, double h_max) {
    if (!per) return h_max;
    double lm = fmin(g.L[0], fmin(g.L[1], g.L[2]));
    return fmin(h_max, 0.5 * lm);
}

// Dynamic bucket sizing (Sec. 2.3.2, last paragraph).  The tree is built
// over buckets of B particles (the finest size); a group at level h walks it
// only down to the nodes of height h, which are contiguous runs of B 2^h
// particles, and treats those as its buckets.  The copy of the set's
// geometry is adjusted to that level (leaf count, bucket count, depth) and
// the group's bucket size returned.  A group's level is the smallest level
// any of its particles carries from the previous step (the most refined
// wins), so a region whose lists blew up keeps small buckets after the
// particles are re-sorted.
__device__ __forceinline__ int group_bucket(const SweepArgs &a, SetGeom &g, int64_t i, bool act,
                                            int &level) {
    int B = a.B;
    level = 0;
    if (!a.levs) return B;
    int h = (int)wave_min(act ? a.levs[i] : 1e30);
    h = h < 0 ? 0 : h;
    h = h > a.lev_max ? a.lev_max : h;
    h = h > g.depth ? g.depth : h;
    level = h;
    g.nbp >>= h;
    g.nb = (g.nb + (1 << h) - 1) >> h;
    g.depth -= h;
    return B << h;
}

// Stage 64 candidate slots starting at candidate-list position t0 (64/B
// buckets).  Returns the sorted particle index of this lane's slot or -1.
__device__ __forceinline__ int64_t slot_index(const SetGeom &g, const uint32_t *cand, int ncand,
                                              int t0, int B) {
    const int lane = threadIdx.x;
    int bi = t0 + lane / B;
    int off = lane % B;
    if (bi >= ncand) return -1;
    int64_t b = cand[bi];
    int64_t start = g.p0 + (b - g.b0) * B;
    int64_t j = start + off;
    return j < g.p1 ? j : -1;
}

// Tile composition of the density and force sweeps.  The candidate slots of a
// list (ncand buckets of B) are cut into runs of kRun; tile t of the T =
// ceil(ncand B / 64) tiles takes runs t, T + t, 2T + t, ... (lane kRun c + e
// holds slot kRun (cT + t) + e).  Each tile thus samples the whole
// neighbourhood of the group instead of 64/B adjacent buckets, so the sinks'
// hit counts per tile are even and the compaction, whose rounds number the
// largest count of any sink, needs about half as many rounds.  (Runs of 2
// and 4 measure alike; single slots cost more in staging, runs of 8 more
// compaction rounds.)  An FP64
// tile takes the minimum-image path as soon as one of its candidates may need
// it, which interleaved tiles of a group near the box edge nearly all would;
// such lists (refine's `far`) keep adjacent buckets per tile (slot_index).
// Returns the sorted particle index or -1.
__device__ __forceinline__ int sweep_tiles(int ncand, int B) {
    return (ncand * B + kWave - 1) / kWave;
}
__device__ __forceinline__ int64_t sweep_slot(const SetGeom &g, const uint32_t *cand, int ncand,
                                              int t, int T, int lb) {
    constexpr int kRun = 2;
    const int lane = threadIdx.x;
    const int p = kRun * ((lane / kRun) * T + t) + (lane % kRun);
    const int bi = p >> lb;
    if (bi >= ncand) return -1;
    const int64_t j = g.p0 + ((int64_t)cand[bi] - g.b0) * ((int64_t)1 << lb) + (p & ((1 << lb) - 1));
    return j < g.p1 ? j : -1;
}

// ================================================================ pair compaction
//
// A staged tile holds 64 candidates; a wave holds 64 sinks.  Evaluating the
// full 64 x 64 block with one sink per lane executes the interaction maths for
// every candidate that ANY lane accepts, i.e. for nearly all of them, while
// only ~10% of the (sink, candidate) pairs are neighbours.  The sweep
// therefore separates, per tile:
//   test     lane = sink, candidates by LDS broadcast, distance test only,
//            giving a 64-bit hit mask per lane;
//   compact  in rounds: round r appends the r-th accepted candidate of every
//            lane that has one to a small LDS ring of pairs (so entries of a
//            round have distinct sinks), and the rounds stop after as many as
//            the largest per-lane count, typically far fewer than 64;
//   interact lane = pair: whenever U x 64 pairs are pending, they are
//            fetched together (their LDS latencies overlap) and their
//            contributions added to the sinks' LDS accumulators with LDS
//            float atomics (one wave per workgroup, so the order of the adds
//            is fixed).  The remainder is drained at the end of the tile.
//            The sweeps use U = 1: at four or five waves per SIMD the other
//            waves hide the fetch latency, and a second chunk's registers
//            would spill (measured 2 % faster than U = 2).
// Each sink then folds the tile's partial sums into its own accumulators.
// The ring never holds more than U x 64 - 1 + 64 pairs, so the pair list
// costs kRing x 2 bytes of LDS instead of one entry per possible pair (U = 1:
// 127 pending pairs at most, so 128 entries).  The workgroup is one wave,
// whose LDS instructions execute in issue order, so ring writes and reads
// need only a compiler-level ordering point (a workgroup barrier would also
// wait for every outstanding LDS atomic).
constexpr int kRing = 128;

// Candidate queue of the sweeps: a ring of two tiles.  A load of 64 slots
// appends at most 64 candidates to fewer than 64 queued ones, and every time
// 64 are queued the half they start in is processed as a tile.
constexpr int kQueue = 2 * kWave;

// Hit bits are collected most significant first: `push_hit(acc, a, b)` is
// 2 acc + (a < b), one compare whose lane mask is the carry-in of one add, in
// place of a compare, a select and a merge per candidate.  (The carry-out
// overwrites the mask; nothing else reads it.)
__device__ __forceinline__ uint32_t push_hit(uint32_t acc, float a, float b) {
    asm("v_cmp_lt_f32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(acc) : "v"(a), "v"(b) : "vcc");
    return acc;
}
__device__ __forceinline__ uint32_t push_hit(uint32_t acc, double a, double b) {
    asm("v_cmp_lt_f64 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %0, %0, vcc"
        : "+v"(acc) : "v"(a), "v"(b) : "vcc");
    return acc;
}

// `hit8(k0, acc)` pushes the hits of candidates k0..k0+7 of this lane, in
// that order, onto acc (push_hit); candidate c of the tile ends at bit 63 - c
// of the lane's mask.  `fetch(s, k)` loads the operands of pair (sink s,
// candidate k) and `apply(d, valid, decided)` adds its contributions when
// `valid`; with `decided` false it may instead return true ("defer"): the
// pair lies in the band where only an FP64 test decides membership (mixed
// path).  Deferred pairs of a chunk are compacted into the ring slots that
// chunk has just consumed, `exact(s, k, act)` decides each of them (lanes
// with `act`; called by the whole wave), and those
// inside are applied again with `decided` true.  This rare path stays out of
// the hot pair terms, whose register budget it would otherwise share.
template <int U, class Hit8, class Fetch, class Apply, class Exact>
__device__ __forceinline__ void tile_pairs(uint16_t *ring, Hit8 hit8, Fetch fetch, Apply apply,
                                           Exact exact, int &hits) {
    static_assert(U * kWave + kWave <= kRing, "pair ring too small");
    static_assert(U == 1, "deferred pairs reuse the slots of a single chunk");
    const int lane = threadIdx.x;
    uint32_t first = 0, second = 0;   // candidates 0..31, 32..63
#pragma unroll 1
    for (int k0 = 0; k0 < kWave / 2; k0 += 8) first = hit8(k0, first);
#pragma unroll 1
    for (int k0 = kWave / 2; k0 < kWave; k0 += 8) second = hit8(k0, second);
    uint64_t m = ((uint64_t)first << 32) | second;
    hits += __popcll(m);
    int produced = 0, consumed = 0;
    auto run = [&](int n) {   // pairs consumed .. consumed + n - 1, n <= 64
        const uint16_t p = ring[(consumed + (lane < n ? lane : 0)) & (kRing - 1)];
        const bool defer = apply(fetch((int)(p >> 6), (int)(p & 63)), lane < n, false);
        const uint64_t bm = __ballot(defer);
        if (bm != 0ull) {
            __builtin_amdgcn_wave_barrier();
            if (defer)
                ring[__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bm,
                                                                         (uint32_t)consumed)) &
                     (kRing - 1)] = p;
            __builtin_amdgcn_wave_barrier();
            const int nb = __popcll(bm);
            const uint16_t q = ring[(consumed + (lane < nb ? lane : 0)) & (kRing - 1)];
            const bool in = exact((int)(q >> 6), (int)(q & 63), lane < nb);
            apply(fetch((int)(q >> 6), (int)(q & 63)), in, true);
            __builtin_amdgcn_wave_barrier();
        }
        consumed += n;
    };
    for (;;) {
        const bool h = m != 0ull;
        const uint64_t bal = __ballot(h);
        if (bal == 0ull) break;
        // ring slot: `produced` plus the entries of lower lanes in this round
        const uint32_t slot = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, (uint32_t)produced));
        if (h) ring[slot & (kRing - 1)] = (uint16_t)(((lane << 6) | 63) - __builtin_ctzll(m));
        m &= m - 1ull;   // (0 stays 0)
        produced += __popcll(bal);
        if (produced - consumed >= U * kWave) {
            __builtin_amdgcn_wave_barrier();
            run(U * kWave);
            __builtin_amdgcn_wave_barrier();
        }
    }
    __builtin_amdgcn_wave_barrier();
    while (produced > consumed) run(min(U * kWave, produced - consumed));
}


// Square root of the pair distance: the hardware instruction in FP32 (within
// one ulp, the mixed path's tolerance is far wider), IEEE in FP64.
__device__ __forceinline__ float pair_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double pair_sqrt(double x) { return sqrt(x); }
// Reciprocal in the force pair terms: the hardware instruction in FP32 (about
// one ulp), a correctly rounded division in FP64.
__device__ __forceinline__ float pair_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double pair_rcp(double x) { return 1.0 / x; }

// Pair difference d = x_k - x_i (candidate minus sink).  FP64: absolute
// coordinates, minimum image in tiles that may need it (WRAP), distance
// without contraction (the sets are bit-exact).  Mixed: FP32 coordinates
// relative to the group centre, re-wrapped (WRAP) only when the group is too
// wide for the single image chosen at staging; r^2 with fused multiply-adds
// (the same expression for the test and the interaction, symmetric in i, j).
template <bool MIXED, bool WRAP, typename R>
__device__ __forceinline__ R pair_r2(R xk, R yk, R zk, R xi, R yi, R zi, bool per,
                                     const SetGeom &g, const R *Lf, const R *hLf,
                                     R &dx, R &dy, R &dz) {
    dx = xk - xi; dy = yk - yi; dz = zk - zi;
    if constexpr (MIXED) {
        if constexpr (WRAP) {
            dx = wrap_f(dx, Lf[0], hLf[0]);
            dy = wrap_f(dy, Lf[1], hLf[1]);
            dz = wrap_f(dz, Lf[2], hLf[2]);
        }
        return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    } else {
        if (WRAP && per) {
            dx = min_image(dx, g.L[0], g.halfL[0]);
            dy = min_image(dy, g.L[1], g.halfL[1]);
            dz = min_image(dz, g.L[2], g.halfL[2]);
        }
        return r2_exact(dx, dy, dz);
    }
}

// ================================================================ exact membership (mixed path)
//
// The mixed path decides r^2 < T (T = H_i^2 for the gather set, max(H_i,
// H_j)^2 for the force set) in FP32 on coordinates relative to the group
// centre gc, so near the boundary its answer may differ from the FP64 one
// that defines the sets.  Bound of the difference: with A = x_j - gc and
// B = x_i - gc (each rounded once to FP32) and t = A - B, every FP32
// difference d has |d - t| <= u (|A| + |B| + |t|) per axis (u = 2^-24), and
// near the boundary |A| <= |B| + sqrt(T), |B| <= G (the group's largest
// offset from gc), so |d^2 - t^2| <= 2 u sqrt(T) |E| + 3 u T with
// |E| <= 2 sqrt(3) (2 G + sqrt(T)) (plus sqrt(3) L when the FP32 difference is
// re-wrapped by a box length L).  Relative to T, with sqrt(T) >= Hmin (the
// smallest sink H of the group), the error stays below
//   beta_r = u (4 sqrt(3) (2 G/Hmin + 1 + L/Hmin) + 3);
// `guard_band` returns band = 2 beta_r plus 16 u for the roundings of the
// thresholds themselves.  The FP32 test then accepts r^2 < T (1 + band), a
// superset of the FP64 set, and the interaction re-tests in FP64 every
// accepted pair with r >= sqrt(T) (1 - band): exactly the FP64 sets, at the
// cost of a few FP64 tests per thousand sinks.
__device__ __forceinline__ double guard_band(double G, double Hmin, double Lwrap) {
    const double u = 0x1p-24;
    return 2.0 * u * (4.0 * 1.7320508075688772 * ((2.0 * G + Lwrap) / Hmin + 1.0) + 3.0) +
           16.0 * u;
}

// FP64 decision r_ij^2 < T for sorted particles i and j: the same expression
// as the FP64 path (minimum image per axis, no contraction).
__device__ __forceinline__ bool exact_inside(const double *xs, const double *ys, const double *zs,
                                             int64_t i, int64_t j, double T, bool per,
                                             const SetGeom &g) {
    double dx = xs[j] - xs[i], dy = ys[j] - ys[i], dz = zs[j] - zs[i];
    if (per) {
        dx = min_image(dx, g.L[0], g.halfL[0]);
        dy = min_image(dy, g.L[1], g.halfL[1]);
        dz = min_image(dz, g.L[2], g.halfL[2]);
    }
    return r2_exact(dx, dy, dz) < T;
}

// One candidate slot of the fill loop: sorted index (-1: empty) and FP64
// position plus one more column (m for the density pass, H for the force pass).
struct Slot {
    int64_t j;
    double x, y, z, w;
};

// ================================================================ candidate filter
//
// The walk and the refinement keep whole buckets; within a kept bucket most
// particles are still out of reach of every sink.  Before a candidate enters
// the queue that the distance tests read, it is tested once (one lane per
// candidate, not per pair) against bounds of the whole group, relative to
// the group centre gc: the box of the sinks' kernel balls and a ball around
// gc that encloses them (the gather test of Sec. 2.3.2 applied to a single
// particle), or, in the force pass, also whether the candidate's own ball
// reaches the box of the sink positions (the scatter test).  The bounds are
// widened by 1e-5 of the group's reach, far beyond the rounding of either
// precision and the mixed path's membership band, so the filter drops only
// candidates that no sink can accept.  A candidate whose offset from gc comes
// within the group's extent of half a box may need another periodic image
// for some sink; it is kept untested.
struct GroupFilter {
    float blo[3], bhi[3];   // box of the sinks' balls
    float clo[3], chi[3];   // box of the sink positions
    float R2;               // squared radius of the ball around gc holding every sink ball
    float lim[3];           // per axis: offsets beyond this may need another image
    float eps;              // absolute widening
    bool per;

    __device__ __forceinline__ bool ambiguous(float d0, float d1, float d2) const {
        return per && (fabsf(d0) >= lim[0] || fabsf(d1) >= lim[1] || fabsf(d2) >= lim[2]);
    }
    // gather: some sink's ball may hold the candidate
    __device__ __forceinline__ bool gather(float d0, float d1, float d2) const {
        return d0 >= blo[0] && d0 <= bhi[0] && d1 >= blo[1] && d1 <= bhi[1] && d2 >= blo[2] &&
               d2 <= bhi[2] && fmaf(d0, d0, fmaf(d1, d1, d2 * d2)) <= R2;
    }
    __device__ __forceinline__ bool inside(float d0, float d1, float d2) const {
        return ambiguous(d0, d1, d2) || gather(d0, d1, d2);
    }
    // force set: gather, or the candidate's ball of radius Hj reaches a sink
    __device__ __forceinline__ bool inside_fs(float d0, float d1, float d2, float Hj) const {
        const float e0 = fmaxf(fmaxf(clo[0] - d0, d0 - chi[0]), 0.0f);
        const float e1 = fmaxf(fmaxf(clo[1] - d1, d1 - chi[1]), 0.0f);
        const float e2 = fmaxf(fmaxf(clo[2] - d2, d2 - chi[2]), 0.0f);
        const float rj = fmaf(Hj, 1.0f + 1e-5f, eps);
        return ambiguous(d0, d1, d2) || gather(d0, d1, d2) ||
               fmaf(e0, e0, fmaf(e1, e1, e2 * e2)) <= rj * rj;
    }
};

__device__ __forceinline__ float uniform_f(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The filter of a group whose sinks (lanes with `act`) sit at xi with support
// radius H.  Bounds are reduced in FP64 and rounded to FP32 with their
// widening (1e-5 of the reach, against FP32's 6e-8), the candidate offsets
// they are compared with are the FP32 roundings of the FP64 ones.
__device__ inline GroupFilter group_filter(bool act, const double *xi, const double *gc, double H,
                                           bool per, const SetGeom &g, const double *gext) {
    GroupFilter f;
    f.per = per;
    double q[3];
    for (int c = 0; c < 3; ++c) {
        const double d = xi[c] - gc[c];
        q[c] = act ? (per ? min_image(d, g.L[c], g.halfL[c]) : d) : 0.0;
    }
    const double Hmax = wave_max(act ? H : 0.0);
    const double gm = fmax(gext[0], fmax(gext[1], gext[2]));
    const double eps = 1e-5 * (gm + Hmax);
    f.eps = uniform_f((float)eps);
    const double Hw = H * (1.0 + 1e-5);
    for (int c = 0; c < 3; ++c) {
        f.blo[c] = uniform_f((float)(wave_min(act ? q[c] - Hw : DBL_MAX) - eps));
        f.bhi[c] = uniform_f((float)(wave_max(act ? q[c] + Hw : -DBL_MAX) + eps));
        f.clo[c] = uniform_f((float)(wave_min(act ? q[c] : DBL_MAX) - eps));
        f.chi[c] = uniform_f((float)(wave_max(act ? q[c] : -DBL_MAX) + eps));
        f.lim[c] = uniform_f((float)(0.499 * g.L[c] - gext[c]));
    }
    const double R = wave_max(act ? sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) + Hw : 0.0) + eps;
    f.R2 = uniform_f((float)(R * R));
    return f;
}

// FP64 tiles: the minimum image is the identity for every pair of the tile
// when each candidate lies within half a box minus the group's extent of the
// group centre on every axis (|x_j - x_i| <= |x_j - gc| + |gc - x_i|), so such
// tiles skip it and keep bit-identical distances.
__device__ __forceinline__ bool needs_image(bool per, const SetGeom &g, const double *gc,
                                            const double *gext, double x, double y, double z) {
    if (!per) return false;
    return fabs(x - gc[0]) + gext[0] >= 0.999 * g.halfL[0] ||
           fabs(y - gc[1]) + gext[1] >= 0.999 * g.halfL[1] ||
           fabs(z - gc[2]) + gext[2] >= 0.999 * g.halfL[2];
}

// ================================================================ density

// Occupancy of the density kernels.  The walk stack lives in global memory
// (one per sink group, as for the force kernels), leaving 6-7 KiB of LDS; the
// mixed kernel is held to 96 VGPRs, five waves per SIMD, the FP64 one to 128,
// four waves.  The values that then spill to scratch cost less than the
// latency the extra waves hide (measured at 2M with the walk inside: mixed
// 2.48 ms at three waves, 2.21 at four, 2.13 at five; FP64 7.29 at three,
// 6.83 at four; with stored lists: mixed 1.48 ms at five waves, 1.59 at
// four; FP64 5.24 at four, 5.59 at three).
template <int K, bool MIXED, bool LISTED>
__device__ __forceinline__ void density_group(const SweepArgs &a, const int64_t grp) {
    typedef typename std::conditional<MIXED, float, double>::type R;
    __shared__ uint32_t cand[kCandCap];
    __shared__ uint16_t ring[kRing];
    // candidate queue (x y z m, a ring of kQueue entries; tiles are its
    // halves) and, in the mixed path, the candidates' squared offsets from
    // the group centre and sorted indices, per-sink counts of pairs the FP64
    // re-test rejected and the sinks' FP64 H (exact membership); while the
    // walk refines its list the same LDS holds the refinement stage
    constexpr int kTileBytes =
        4 * kQueue * (int)sizeof(R) + (MIXED ? kQueue * 8 + kWave * 12 : 0);
    __shared__ alignas(16) unsigned char tile_buf[kTileBytes > kRefineStageBytes ? kTileBytes
                                                                                  : kRefineStageBytes];
    R *const qx_ = reinterpret_cast<R *>(tile_buf);
    R *const qy_ = qx_ + kQueue;
    R *const qz_ = qy_ + kQueue;
    R *const qm_ = qz_ + kQueue;
    R *const qc_ = qm_ + kQueue;   // (mixed)
    int32_t *const qj_ = reinterpret_cast<int32_t *>(qm_ + (MIXED ? 2 : 1) * kQueue);
    int32_t *const srej = qj_ + kQueue;
    double *const sH = reinterpret_cast<double *>(srej + kWave);
    float *const stage = reinterpret_cast<float *>(tile_buf);
    __shared__ V4<R> sp[kWave];   // sink: position, 1/H
    __shared__ double acc0[kWave], acc1[kWave], acc2[kWave];

    const int lane = threadIdx.x;
    unsigned long long *const ctr = a.cnt + cnt_shard(grp);   // this group's counter copy
    uint32_t *const stack = a.wstack + grp * kStackCap;
    const int sid = a.grp_set[grp];
    SetGeom g = a.sets[sid];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    const double cap = set_hcap(g, per, a.h_max);
    int64_t i;
    bool act;
    if (!group_sinks(a, g, grp, i, act)) return;
    // a walking launch after a listed one: only the groups it left
    if (!LISTED && a.defer && a.defer[grp] == 0) return;
    int level;
    const int Bg = group_bucket(a, g, i, act, level);   // this group's bucket size
    const int lb = 31 - __builtin_clz((unsigned)Bg);     // Bg = 2^lb
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    const double mi = act ? a.ms[i] : 0.0;
    double H = act ? a.Hs[i] : 0.0;
    if (!(H > 0.0)) H = 0.01 * cap;
    if (H > cap) H = cap;
    const double target = a.n_ngb * mi;
    const double sig = sigma_of<K>();
    const double c43 = 4.0 * kPi / 3.0;

    double lo = 0.0, hi = 0.0;
    bool hi_ok = false;
    bool done = !act;
    bool noconv = false;
    double Hw = fmin(a.oversel * H, cap);
    double rho = 0.0, om = 1.0;
    int cnt_out = 0;

    // group centre (reference point of the mixed path's FP32 coordinates)
    double gc[3];
    for (int q = 0; q < 3; ++q) {
        double mn = wave_min(act ? xi[q] : DBL_MAX), mx = wave_max(act ? xi[q] : -DBL_MAX);
        gc[q] = 0.5 * (mn + mx);
    }
    double gext[3];
    for (int q = 0; q < 3; ++q) gext[q] = wave_max(act ? fabs(xi[q] - gc[q]) : 0.0);
    const double gmax = fmax(gext[0], fmax(gext[1], gext[2]));
    const double Lmax = fmax(g.L[0], fmax(g.L[1], g.L[2]));
    const R Lf[3] = {(R)g.L[0], (R)g.L[1], (R)g.L[2]};
    const R hLf[3] = {(R)g.halfL[0], (R)g.halfL[1], (R)g.halfL[2]};
    R qx, qy, qz;
    if constexpr (MIXED) {
        qx = (R)(per ? min_image(xi[0] - gc[0], g.L[0], g.halfL[0]) : xi[0] - gc[0]);
        qy = (R)(per ? min_image(xi[1] - gc[1], g.L[1], g.halfL[1]) : xi[1] - gc[1]);
        qz = (R)(per ? min_image(xi[2] - gc[2], g.L[2], g.halfL[2]) : xi[2] - gc[2]);
    } else {
        qx = xi[0]; qy = xi[1]; qz = xi[2];
    }
    sp[lane] = V4<R>{qx, qy, qz, R(0)};
    acc0[lane] = 0; acc1[lane] = 0; acc2[lane] = 0;

    bool wrapf = false;

    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    Sink sk;
    bool list_complete = false;
    bool linear = false;
    int overflows = 0;
    int scans = 0, rewalks = 0;
    int retests = 0;   // pairs the wave re-tested in FP64 (mixed)
    unsigned long long cand_tested = 0;
    unsigned long long slots = 0;   // candidate slots loaded (before the filter)
    bool need_walk = true;
    // LISTED: the list at Hw comes from k_walk in chunks; a list too long to
    // store, or a root beyond Hw (a new walk), leaves the group to the
    // walking kernel, which redoes it from the start
    const int32_t *const hdr = LISTED ? a.whdr + grp * kWalkWords : nullptr;
    int nch = 0, farm = 0;
    auto load_chunk = [&](int c) {
        ws.ncand = hdr[3 + c];
        ws.far = ((farm >> c) & 1) != 0;
        const uint32_t *src = a.wlist + grp * kListCap + c * kCandCap;
        for (int t = lane; t < ws.ncand; t += kWave) cand[t] = src[t];
        __syncthreads();
    };
    auto defer_group = [&]() {
        if (lane == 0) {
            a.defer[grp] = 1;
            atomicAdd(&ctr[C_WALKED], 1ull);
        }
    };

    while (true) {
        if (need_walk && LISTED) {
            const int flags = hdr[2];
            if (flags & kListLong) { defer_group(); return; }
            if (lane == 0) a.defer[grp] = 0;
            if (flags & kListLinear) ++overflows;
            nch = hdr[0];
            farm = hdr[1];
            list_complete = nch <= 1;
            ws.ncand = 0;
            ws.nstack = 0;
            if (nch == 1) load_chunk(0);
            need_walk = false;
            if constexpr (MIXED) wrapf = group_needs_wrap(per, g, gext, wave_max(act ? Hw : 0.0));
        }
        if (!LISTED && need_walk) {
            sink_bounds(act, xi, Hw, sk);
            walk_reset(stack, ws, linear, g);
            walk<false>(g, per, slop, a.nodes, sk, stack, cand, ws);
            if (ws.overflow) {
                ++overflows;
                linear = true;
                walk_reset(stack, ws, true, g);
                walk<false>(g, per, slop, a.nodes, sk, stack, cand, ws);
            }
            refine<false>(g, per, slop, a.nodes, xi, Hw, wave_max(act ? Hw : 0.0), act, gc, gext, cand,
                          stage, ws);
            list_complete = (ws.nstack == 0);
            need_walk = false;
            if constexpr (MIXED) wrapf = group_needs_wrap(per, g, gext, wave_max(act ? Hw : 0.0));
        }
        // ---- one scan over the candidate list at the lanes' current H.  The
        // particle meets itself (r = 0: f = 1, q f' = 0), which is the self
        // term of the density; it is not counted as a neighbour.
        double S0 = 0.0, T1 = 0.0, T2 = 0.0;
        int cnt = 0;
        const R Hr = (R)H;
        const R Hinv = R(1) / Hr;
        // mixed: the FP32 test accepts r^2 < H^2 (1 + band), pairs with
        // q >= 1 - band are re-tested in FP64 (see guard_band)
        const double band =
            MIXED ? guard_band(gmax, wave_min(act ? H : DBL_MAX), wrapf ? Lmax : 0.0) : 0.0;
        const R H2 = MIXED ? (R)(H * H * (1.0 + band)) : (R)(H * H);
        const R qlo = (R)(1.0 - band);
        // mixed, tiles without re-wrapping: the distance test in expanded
        // form, |A|^2 - 2 A.B < H2' - |B|^2 for candidate A and sink B (both
        // offsets from the group centre), three FMAs per candidate.  Its
        // rounding error stays below u (6 |A|^2 + 6 |A||B| + 4 |B|^2) + u H2'
        // (u = 2^-24), with |B| <= sqrt(3) G and, for a pair the difference
        // form r^2 < H2 accepts, |A| <= |B| + 1.01 H; H2' = H2 (1 + loose),
        // loose twice that bound over H^2 plus the difference form's own
        // 4.2 u, so it accepts every pair the difference form accepts.  The
        // few it accepts beyond lie past the band and go to the FP64 re-test,
        // which rejects them: the sets stay exact.
        R m2qx = R(0), m2qy = R(0), m2qz = R(0), TsX = R(0);
        if constexpr (MIXED) {
            const double S = 1.7320508075688772 * gmax / (act ? H : 1.0);
            const double A_ = S + 1.01;
            const double loose = 0x1p-23 * (6.0 * A_ * A_ + 6.0 * A_ * S + 4.0 * S * S + 8.0);
            m2qx = -2.0f * qx; m2qy = -2.0f * qy; m2qz = -2.0f * qz;
            TsX = (R)((double)H2 * (1.0 + loose)) - fmaf(qx, qx, fmaf(qy, qy, qz * qz));
        }
        sp[lane].w = Hinv;
        // the group's bounds at this scan's H (candidate filter)
        const GroupFilter fil = group_filter(act, xi, gc, H, per, g, gext);
        int qb = 0, qn = 0;   // candidate queue: first entry, entries
        bool first_chunk = true;
        int chunk = 0;
        while (true) {
            if (LISTED && !list_complete) {
                load_chunk(chunk);
                ++chunk;
            } else if (!LISTED && (!first_chunk || !list_complete)) {
                if (!first_chunk) {
                    ws.ncand = 0;
                    walk<false>(g, per, slop, a.nodes, sk, stack, cand, ws);
                } else {
                    walk_reset(stack, ws, linear, g);
                    walk<false>(g, per, slop, a.nodes, sk, stack, cand, ws);
                }
                if (ws.overflow) {
                    // restart this scan with the linear bucket test
                    ++overflows;
                    linear = true;
                    S0 = T1 = T2 = 0.0;
                    cnt = 0;
                    first_chunk = true;
                    continue;
                }
                refine<false>(g, per, slop, a.nodes, xi, Hw, wave_max(act ? Hw : 0.0), act, gc, gext, cand,
                          stage, ws);
            }
            const int nload = sweep_tiles(ws.ncand, Bg);
            if constexpr (MIXED) {
                // (after the refinement, which shares this LDS)
                sH[lane] = H;
                srej[lane] = 0;
            }
            // One tile: the 64 queue entries from qb (nv of them valid).
            auto run_tile = [&](int nv) {
                R *const tx = qx_ + qb, *const ty = qy_ + qb, *const tz = qz_ + qb,
                         *const tm = qm_ + qb, *const tc = qc_ + qb;
                const int32_t *const tj = qj_ + qb;
                if (lane >= nv) {
                    tx[lane] = (R)NAN; ty[lane] = R(0); tz[lane] = R(0); tm[lane] = R(0);
                    if constexpr (MIXED) tc[lane] = (R)NAN;
                }
                if constexpr (!MIXED)
                    wrapf = __any(lane < nv && needs_image(per, g, gc, gext, (double)tx[lane],
                                                           (double)ty[lane], (double)tz[lane]));
                cand_tested += (unsigned long long)nv;
                __syncthreads();
                auto tile = [&](auto wrap_tag) {
                    constexpr bool WRAP = decltype(wrap_tag)::value;
                    auto r2of = [&](R x, R y, R z) -> R {
                        R dx, dy, dz;
                        return pair_r2<MIXED, WRAP, R>(x, y, z, qx, qy, qz, per, g, Lf, hLf,
                                                       dx, dy, dz);
                    };
                    struct PD { int s; R x, y, z, m; V4<R> si; };
                    tile_pairs<1>(ring, [&](int k0, uint32_t b) {
#pragma unroll
                        for (int h = 0; h < 8; h += 4) {
                            const V4<R> X = ld4(tx + k0 + h), Y = ld4(ty + k0 + h),
                                        Z = ld4(tz + k0 + h);
                            if constexpr (MIXED && !WRAP) {
                                const V4<R> C = ld4(tc + k0 + h);
                                auto ex = [&](R x, R y, R z, R c) -> R {
                                    return fmaf(x, m2qx, fmaf(y, m2qy, fmaf(z, m2qz, c)));
                                };
                                b = push_hit(b, ex(X.x, Y.x, Z.x, C.x), TsX);
                                b = push_hit(b, ex(X.y, Y.y, Z.y, C.y), TsX);
                                b = push_hit(b, ex(X.z, Y.z, Z.z, C.z), TsX);
                                b = push_hit(b, ex(X.w, Y.w, Z.w, C.w), TsX);
                            } else {
                                b = push_hit(b, r2of(X.x, Y.x, Z.x), H2);
                                b = push_hit(b, r2of(X.y, Y.y, Z.y), H2);
                                b = push_hit(b, r2of(X.z, Y.z, Z.z), H2);
                                b = push_hit(b, r2of(X.w, Y.w, Z.w), H2);
                            }
                        }
                        return b;
                    }, [&](int s, int k) {
                        return PD{s, tx[k], ty[k], tz[k], tm[k], sp[s]};
                    }, [&](const PD &d, bool valid, bool decided) -> bool {
                        R ex, ey, ez;
                        const R r2 = pair_r2<MIXED, WRAP, R>(d.x, d.y, d.z, d.si.x, d.si.y,
                                                             d.si.z, per, g, Lf, hLf, ex, ey, ez);
                        const R q = pair_sqrt(r2) * d.si.w;
                        // near the boundary the FP64 test decides (mixed, rare)
                        if (MIXED && !decided && valid && q >= qlo) return true;
                        R f, t1, t2;
                        shape_f_t1_t2<K, R>(q, f, t1, t2);
                        if (valid) {
                            atomicAdd(&acc0[d.s], (double)(d.m * f));
                            atomicAdd(&acc1[d.s], (double)(d.m * t1));
                            atomicAdd(&acc2[d.s], (double)(d.m * t2));
                        }
                        return false;
                    }, [&](int s_, int k_, bool act_) -> bool {
                        bool in = false;
                        if (act_) {
                            const double Hs = sH[s_];
                            in = exact_inside(a.xs, a.ys, a.zs, sink_index(a, g, grp, s_),
                                              (int64_t)tj[k_], Hs * Hs, per, g);
                            if (!in) atomicAdd(&srej[s_], 1);
                        }
                        retests += __popcll(__ballot(act_));
                        return in;
                    }, cnt);
                };
                if (wrapf) tile(std::true_type{});
                else tile(std::false_type{});
                __syncthreads();
                S0 += acc0[lane];
                T1 += acc1[lane];
                T2 += acc2[lane];
                acc0[lane] = 0; acc1[lane] = 0; acc2[lane] = 0;
                if constexpr (MIXED) {
                    cnt -= srej[lane];
                    srej[lane] = 0;
                }
            };
            // Candidates are loaded 64 slots at a time; those the group's
            // bounds at this scan's H rule out for every sink are dropped, the
            // rest appended to the queue, and each full half of it is a tile.
            // (one call site of the tile code: the loop flushes the last
            // partial tile itself, before the walk refines again, whose stage
            // shares this LDS, or the scan ends)
            // (fetching the next slot during this one's filter, as the force
            // pass does, costs the density kernel more in spilled registers
            // at five waves per SIMD than it hides: 2.16 -> 2.32 ms at 2M)
            for (int t = 0;;) {
              if (t < nload) {
                const int64_t j = (MIXED || !ws.far) ? sweep_slot(g, cand, ws.ncand, t, nload, lb)
                                                     : slot_index(g, cand, ws.ncand, t << (6 - lb), Bg);
                const Slot cur = j >= 0 ? Slot{j, a.xs[j], a.ys[j], a.zs[j], a.ms[j]}
                                        : Slot{-1, 0.0, 0.0, 0.0, 0.0};
                slots += (unsigned long long)__popcll(__ballot(j >= 0));
                ++t;
                R px = R(0), py = R(0), pz = R(0), pm = R(0);
                bool keep = false;
                if (j >= 0) {
                    double d0 = cur.x - gc[0], d1 = cur.y - gc[1], d2 = cur.z - gc[2];
                    // (no kept bucket of this chunk reaches near half a box
                    // from gc unless ws.far: the image is then the identity)
                    if (per && ws.far) {
                        d0 = min_image(d0, g.L[0], g.halfL[0]);
                        d1 = min_image(d1, g.L[1], g.halfL[1]);
                        d2 = min_image(d2, g.L[2], g.halfL[2]);
                    }
                    keep = fil.inside((float)d0, (float)d1, (float)d2);
                    pm = (R)cur.w;
                    if constexpr (MIXED) {
                        px = (R)d0; py = (R)d1; pz = (R)d2;
                    } else {
                        px = cur.x; py = cur.y; pz = cur.z;
                    }
                }
                const uint64_t kb = __ballot(keep);
                if (keep) {
                    const int at = (qb + qn + (int)__builtin_amdgcn_mbcnt_hi(
                                                   (uint32_t)(kb >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u))) &
                                   (kQueue - 1);
                    qx_[at] = px; qy_[at] = py; qz_[at] = pz; qm_[at] = pm;
                    if constexpr (MIXED) {
                        qj_[at] = (int32_t)j;
                        qc_[at] = fmaf(px, px, fmaf(py, py, pz * pz));
                    }
                }
                qn += __popcll(kb);
              }
              if (qn >= kWave || (t >= nload && qn > 0)) {
                const int nv = qn < kWave ? qn : kWave;
                run_tile(nv);
                qb ^= kWave;
                qn -= nv;
              }
              if (t >= nload && qn == 0) break;
            }
            first_chunk = false;
            if (LISTED ? (list_complete || chunk == nch) : ws.nstack == 0) break;  // list finished
        }
        ++scans;
        // ---- Halley update per lane, safeguarded by a bracket (Sec. 2.3.3:
        // Newton-Raphson on the constant kernel mass; the second derivative
        // of the same sums makes the update cubically convergent).
        //   F = (4 pi/3) sigma S0 - n_ngb m,  F' = -(4 pi/3) sigma T1 / H,
        //   F'' = (4 pi/3) sigma T2 / H^2,  rho = sigma S0 / H^3,
        //   Omega = 1 + H rho'/(3 rho) = -T1 / (3 S0).
        bool want_walk = false;
        if (!done) {
            const double H3 = H * H * H;
            const double c0 = c43 * sig;
            const double F = c0 * S0 - target;
            const double dF = -c0 * T1 / H;
            const double d2F = c0 * T2 / (H * H);
            rho = sig * S0 / H3;
            om = -T1 / (3.0 * S0);
            cnt_out = cnt - 1;
            if (F < 0.0) lo = H; else { hi = H; hi_ok = true; }
            // Newton step for the stopping test (before the bracket safeguard:
            // a step below the spacing of doubles leaves H - step == H)
            const double newton = dF > 0.0 ? F / dF : NAN;
            const double den = 2.0 * dF * dF - F * d2F;
            const double step = (dF > 0.0 && den > 0.0) ? 2.0 * F * dF / den : newton;
            // a small Halley step is taken without another scan: it leaves an
            // O((step/H)^3) error in H and, through the second-order Taylor
            // step of S0, in rho; Omega's first-order step of T1 leaves
            // O((step/H)^2), so FP64 accepts steps up to sqrt(tol) H
            const double accept = MIXED ? 2e-3 : sqrt(a.tol);
            if (F == 0.0 || (!MIXED && fabs(newton) <= a.tol * H)) {
                done = true;
            } else if (fabs(step) <= accept * H && H - step <= cap) {
                // the sums at the new H follow from their derivatives
                // (S0'' = T2/H^2, T1' = -(T2-T1)/H)
                done = true;
                const double dH = -step;
                const double S0n = S0 - T1 / H * dH + 0.5 * T2 / (H * H) * dH * dH;
                const double T1n = T1 - (T2 - T1) / H * dH;
                H = H + dH;
                rho = sig * S0n / (H * H * H);
                om = -T1n / (3.0 * S0n);
            } else if (F < 0.0 && H >= cap) {
                done = true;   // the root lies beyond the cap
                noconv = true;
            } else {
                double Hn = H - step;
                if (hi_ok) {
                    if (!(Hn > lo && Hn < hi)) Hn = 0.5 * (lo + hi);
                } else {
                    if (!(Hn > H)) Hn = 2.0 * H;
                    if (Hn > cap) Hn = cap;
                    if (Hn > Hw) {
                        if (H < Hw) Hn = Hw;           // probe the search radius first
                        else want_walk = true;         // root lies beyond the list
                    }
                }
                if (want_walk) Hw = fmin(cap, a.oversel * Hn);
                H = Hn;
            }
        }
        if (__all(done)) break;
        if (scans >= a.maxit) break;
        if (__any(want_walk)) {
            if constexpr (LISTED) { defer_group(); return; }
            need_walk = true;
            ++rewalks;
        }
    }
    // status word: the iteration limit reached, a non-finite result
    const bool iterlim = act && !done;
    const bool nonfinite = act && !(isfinite(H) && isfinite(rho) && isfinite(om));
    if (act) {
        if (!done) noconv = true;
        a.Hs[i] = H;
        a.rhos[i] = rho;
        a.oms[i] = om;
    }
    // counters
    int pairs_n = wave_sum_i(act ? cnt_out : 0);
    int bad = wave_sum_i((act && noconv) ? 1 : 0);
    int nact = wave_sum_i(act ? 1 : 0);
    const int nlim = wave_sum_i(iterlim ? 1 : 0);
    const int nnan = wave_sum_i(nonfinite ? 1 : 0);
    const int nret = retests;   // (a wave total)
    if (lane == 0) {
        if (nlim) atomicAdd(&ctr[C_ITERLIM], (unsigned long long)nlim);
        if (nnan) atomicAdd(&ctr[C_NONFINITE], (unsigned long long)nnan);
        if (nret) atomicAdd(&ctr[C_RETEST], (unsigned long long)nret);
        atomicAdd(&ctr[C_SLOTS_D], slots);
        atomicAdd(&ctr[C_PAIRS_D], (unsigned long long)pairs_n);
        atomicAdd(&ctr[C_PAIRS_D_TOT], (unsigned long long)pairs_n);
        atomicAdd(&ctr[C_CAND_D], cand_tested * (unsigned long long)nact);
        atomicMax(&ctr[C_NR_ITER_MAX], (unsigned long long)scans);
        atomicAdd(&ctr[C_NR_SCANS], (unsigned long long)scans);
        if (bad) atomicAdd(&ctr[C_NOCONV], (unsigned long long)bad);
        if (rewalks) atomicAdd(&ctr[C_REWALK], (unsigned long long)rewalks);
        if (overflows) atomicAdd(&ctr[C_OVERFLOW], (unsigned long long)overflows);
    }
}

// Sweep kernel launch modes: a walking kernel (one workgroup per sink group,
// each walking the tree itself), a listed one (the lists from k_walk), and a
// listed one on a persistent grid taking groups from the per-XCD queues.
// The listed kernels hold no walk code, which frees registers: at 2M, mixed
// density spills 47 values instead of 152 and the mixed force kernel none
// instead of 21.
constexpr int kLmWalk = 0, kLmListed = 1, kLmPersistent = 2;

template <int K, bool MIXED, int LM>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(MIXED ? 5 : 4))) void k_density(SweepArgs a) {
    if constexpr (LM == kLmPersistent) {
        int k = 0;
        for (int64_t grp; (grp = next_group(a.queue, a.ngroups, k)) >= 0;)
            density_group<K, MIXED, true>(a, grp);
    } else {
        density_group<K, MIXED, LM == kLmListed>(a, xcd_group(blockIdx.x, gridDim.x));
    }
}

// ================================================================ forces

// Occupancy of the force kernels.  Their walk stack lives in global memory
// (one per sink group, in L2 while the group runs).  Both run three waves per
// SIMD with up to 168 VGPRs: once the candidate filter had halved the
// distance tests, the fourth wave of the mixed kernel (128 VGPRs, 52 of its
// values spilled to scratch) cost more than it hid (2M mixed forces 3.81 ms
// at four waves, 3.24 at three).  Without the walk code (stored lists) the
// mixed kernel needs 135 VGPRs and spills nothing at three waves; at four it
// spills 5 and measured 3.07 ms against 2.90.
// EV: room for the evolved density's continuity sum (a fifth per-sink
// accumulator).  Without it the FP64 kernel's LDS admits twelve workgroups
// per CU instead of eleven (2M FP64 forces 4.85 -> 4.72 ms).
template <int K, bool MIXED, bool RUNGS, bool LISTED, bool EV>
__device__ __forceinline__ void forces_group(const SweepArgs &a, const int64_t grp) {
    typedef typename std::conditional<MIXED, float, double>::type R;
    // (the listed FP64 kernel reads its chunk of the stored list in place:
    // the kilobyte of LDS it saves lets it, whose LDS limits its occupancy,
    // hold eleven workgroups per CU instead of ten; FP64 forces at 2M 5.07 ->
    // 4.86 ms.  The mixed kernel, limited by its registers, copies the chunk
    // to LDS: read in place it took 2.93 ms against 2.87.)
    __shared__ uint32_t cand_lds[(LISTED && !MIXED) ? 1 : kCandCap];
    const uint32_t *cand_rd = cand_lds;
    __shared__ uint16_t ring[kRing];
    // candidate queue (a ring of kQueue entries; tiles are its halves): what
    // the distance test reads, x y z and H^2, and the sorted index through
    // which the interaction reads the candidate's force record (m, v, H, 1/H,
    // A, c, rho; written once per particle by the EOS pass, and shared by the
    // tile's pairs in the L1 cache); while the walk refines its list the same
    // LDS holds the refinement stage
    constexpr int kTileBytes = 4 * kQueue * (int)sizeof(R) + kQueue * 4;
    __shared__ alignas(16) unsigned char tile_buf[kTileBytes > kRefineStageBytes ? kTileBytes
                                                                                  : kRefineStageBytes];
    R *const qx_ = reinterpret_cast<R *>(tile_buf);
    R *const qy_ = qx_ + kQueue;
    R *const qz_ = qy_ + kQueue;
    R *const qh2_ = qz_ + kQueue;
    int32_t *const qj_ = reinterpret_cast<int32_t *>(qh2_ + kQueue);
    float *const stage = reinterpret_cast<float *>(tile_buf);
    const V4<R> *const rec1 = reinterpret_cast<const V4<R> *>(MIXED ? (const void *)a.frec1
                                                                     : (const void *)a.drec1);
    const V4<R> *const rec2 = reinterpret_cast<const V4<R> *>(MIXED ? (const void *)a.frec2
                                                                     : (const void *)a.drec2);
    // mixed: the tile's force records are staged in LDS (one round trip per
    // tile instead of one per chunk of pairs); the FP64 kernel, whose LDS
    // already limits its occupancy, reads them per pair through the L1 cache
    __shared__ V4<R> trec1[MIXED ? kWave : 1], trec2[MIXED ? kWave : 1];
    __shared__ R trm[MIXED ? kWave : 1];
    __shared__ V4<R> sp[kWave], sv[kWave], sq[kWave];  // sink: (x H) (v 1/H) (A c rho sigma/H^5)
    typedef typename std::conditional<MIXED, uint32_t, unsigned long long>::type Bits;
    __shared__ double acc[EV ? 5 : 4][kWave];   // a_x a_y a_z du/dt, sum m (v_ij . x_ij) G_i
    __shared__ Bits amu[kWave];   // bits of max(0, -mu) (non-negative, so integer order)
    // individual time steps: largest rung over F_i, sorted index of each sink,
    // pairs whose neighbour's density is not of this substep (FastGas)
    __shared__ int armax[RUNGS ? kWave : 1], asidx[RUNGS ? kWave : 1], amiss[1];

    const int lane = threadIdx.x;
    unsigned long long *const ctr = a.cnt + cnt_shard(grp);   // this group's counter copy
    uint32_t *const stack = a.wstack + grp * kStackCap;
    const int sid = a.grp_set[grp];
    SetGeom g = a.sets[sid];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    int64_t i;
    bool act;
    if (!group_sinks(a, g, grp, i, act)) return;
    if (!LISTED && a.defer && a.defer[grp] == 0) return;
    int level;
    const int Bg = group_bucket(a, g, i, act, level);   // this group's bucket size
    const int lb = 31 - __builtin_clz((unsigned)Bg);     // Bg = 2^lb
    const double lref = a.levs_out ? *a.lev_ref : 0.0;    // (for the level rule at the end)
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    const double Hd = act ? a.Hs[i] : 0.0;
    const R sig = (R)sigma_of<K>();

    double gc[3];
    for (int q = 0; q < 3; ++q) {
        double mn = wave_min(act ? xi[q] : DBL_MAX), mx = wave_max(act ? xi[q] : -DBL_MAX);
        gc[q] = 0.5 * (mn + mx);
    }
    double gext[3];
    for (int q = 0; q < 3; ++q) gext[q] = wave_max(act ? fabs(xi[q] - gc[q]) : 0.0);
    const R Lf[3] = {(R)g.L[0], (R)g.L[1], (R)g.L[2]};
    const R hLf[3] = {(R)g.halfL[0], (R)g.halfL[1], (R)g.halfL[2]};
    const double Hsink_max = wave_max(act ? Hd : 0.0);
    // mixed: the FP32 test accepts r^2 < max(H_i, H_j)^2 (1 + band), pairs with
    // r >= max(H_i, H_j) (1 - band) are re-tested in FP64 (see guard_band).
    // A group that needs the re-wrapped differences gets the wider band.
    double band = 0.0, bandw = 0.0;
    if constexpr (MIXED) {
        const double gmax = fmax(gext[0], fmax(gext[1], gext[2]));
        const double Lmax = fmax(g.L[0], fmax(g.L[1], g.L[2]));
        const double hmin = wave_min(act ? Hd : DBL_MAX);
        band = guard_band(gmax, hmin, 0.0);
        bandw = guard_band(gmax, hmin, Lmax);
    }
    const R band1 = (R)(1.0 + band), qlo = (R)(1.0 - band);
    const R band1w = (R)(1.0 + bandw), qlow = (R)(1.0 - bandw);

    R qx, qy, qz;
    if constexpr (MIXED) {
        qx = (R)(per ? min_image(xi[0] - gc[0], g.L[0], g.halfL[0]) : xi[0] - gc[0]);
        qy = (R)(per ? min_image(xi[1] - gc[1], g.L[1], g.halfL[1]) : xi[1] - gc[1]);
        qz = (R)(per ? min_image(xi[2] - gc[2], g.L[2], g.halfL[2]) : xi[2] - gc[2]);
    } else {
        qx = xi[0]; qy = xi[1]; qz = xi[2];
    }
    const R Hi = (R)Hd;
    const R Hi2 = MIXED ? (R)(Hd * Hd * (1.0 + band)) : (R)(Hd * Hd);
    const R Hi2w = MIXED ? (R)(Hd * Hd * (1.0 + bandw)) : Hi2;
    const R wfac = (R)((1.0 + bandw) / (1.0 + band));   // staged H^2 of a wrapped tile
    const GroupFilter fil = group_filter(act, xi, gc, Hd, per, g, gext);
    const R Ai = (R)(act ? a.As[i] : 0.0);
    const R ci = (R)(act ? a.css[i] : 0.0);
    // sink data for the interaction phase
    sp[lane] = V4<R>{qx, qy, qz, Hi};
    sv[lane] = V4<R>{(R)(act ? a.vxs[i] : 0.0), (R)(act ? a.vys[i] : 0.0),
                     (R)(act ? a.vzs[i] : 0.0), act ? R(1) / Hi : R(0)};
    const double hinv_i = act ? 1.0 / Hd : 0.0, h2_i = hinv_i * hinv_i;
    sq[lane] = V4<R>{Ai, ci, (R)(act ? a.rhos[i] : 1.0), (R)(sigma_of<K>() * h2_i * h2_i * hinv_i)};
    for (int q = 0; q < (EV ? 5 : 4); ++q) acc[q][lane] = 0;
    amu[lane] = 0;
    if constexpr (RUNGS) {
        armax[lane] = -1;
        asidx[lane] = act ? (int)i : -1;
        if (lane == 0) amiss[0] = 0;
    }
    const R alpha = (R)a.alpha, beta = (R)a.beta, eps = (R)a.eps;
    const R pdv = a.entropy ? R(0) : R(1);   // PdV part of du/dt (off: entropy-conserving)
    const bool evolved = a.drho != nullptr;

    Sink sk;
    sink_bounds(act, xi, Hd, sk);
    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    bool linear = false;
    int overflows = 0;

    double acc_d[5] = {0, 0, 0, 0, 0};
    int cnt = 0;
    int rej = 0;       // accepted pairs that the FP64 re-test rejected (wave total)
    int retests = 0;   // pairs the wave re-tested in FP64
    unsigned long long cand_tested = 0;
    unsigned long long slots = 0;   // candidate slots loaded (before the filter)
    // LISTED: the refined list comes from k_walk in chunks; a list too long
    // to store leaves the group to the walking kernel
    const int32_t *const hdr = LISTED ? a.whdr + grp * kWalkWords : nullptr;
    int nch = 0, farm = 0, chunk = 0;
    if constexpr (LISTED) {
        const int flags = hdr[2];
        if (flags & kListLong) {
            if (lane == 0) {
                a.defer[grp] = 1;
                atomicAdd(&ctr[C_WALKED], 1ull);
            }
            return;
        }
        if (lane == 0) a.defer[grp] = 0;
        if (flags & kListLinear) overflows = 1;
        nch = hdr[0];
        farm = hdr[1];
    } else {
        walk_reset(stack, ws, linear, g);
    }

    while (true) {
      if constexpr (LISTED) {
        if (chunk == nch) break;
        ws.ncand = hdr[3 + chunk];
        ws.far = ((farm >> chunk) & 1) != 0;
        const uint32_t *src = a.wlist + grp * kListCap + chunk * kCandCap;
        if constexpr (MIXED) {
            for (int t = lane; t < ws.ncand; t += kWave) cand_lds[t] = src[t];
            __syncthreads();
        } else {
            cand_rd = src;
        }
        ++chunk;
      } else {
        walk<true>(g, per, slop, a.nodes, sk, stack, cand_lds, ws);
        if (ws.overflow) {
            // restart the whole pass with the linear bucket test
            ++overflows;
            linear = true;
            for (int q = 0; q < 5; ++q) acc_d[q] = 0;
            cnt = 0;
            rej = 0;
            retests = 0;
            cand_tested = 0;
            slots = 0;
            amu[lane] = 0;
            walk_reset(stack, ws, true, g);
            continue;
        }
        refine<true>(g, per, slop, a.nodes, xi, Hd, Hsink_max, act, gc, gext, cand_lds, stage, ws);
      }
        const int nload = sweep_tiles(ws.ncand, Bg);
        int qb = 0, qn = 0;   // candidate queue: first entry, entries
        // One tile: the 64 queue entries from qb (nv of them valid).
        auto run_tile = [&](int nv) {
            R *const tx = qx_ + qb, *const ty = qy_ + qb, *const tz = qz_ + qb;
            R *const th2 = qh2_ + qb;
            const int32_t *const tj = qj_ + qb;
            if (lane >= nv) {
                tx[lane] = (R)NAN; ty[lane] = R(0); tz[lane] = R(0); th2[lane] = R(0);
            }
            bool wrapf = false;
            if constexpr (MIXED) {
                // (the staged H^2 carry the band's 1 + band, within the 1e-6 margin)
                const double reach =
                    fmax(Hsink_max, sqrt(wave_max(lane < nv ? (double)th2[lane] : 0.0)));
                wrapf = group_needs_wrap(per, g, gext, reach);
            } else {
                wrapf = __any(lane < nv &&
                              needs_image(per, g, gc, gext, tx[lane], ty[lane], tz[lane]));
            }
            if constexpr (MIXED) {
                if (lane < nv) {
                    const int32_t j = tj[lane];
                    trec1[lane] = rec1[j];
                    trec2[lane] = rec2[j];
                    trm[lane] = a.fm[j];
                }
            }
            cand_tested += (unsigned long long)nv;
            __syncthreads();
            auto tile = [&](auto wrap_tag) {
                constexpr bool WRAP = decltype(wrap_tag)::value;
                // r = 0 pairs (the particle itself, or a coincident one) count as
                // neighbours but exert no force and no heating (x_ij = 0): they
                // are accepted here and skipped in the interaction
                const R hi2 = WRAP ? Hi2w : Hi2;
                auto in = [&](uint32_t b, R x, R y, R z, R h2) -> uint32_t {
                    R dx, dy, dz;
                    const R r2 = pair_r2<MIXED, WRAP, R>(x, y, z, qx, qy, qz, per, g, Lf, hLf,
                                                         dx, dy, dz);
                    if (MIXED && WRAP) h2 *= wfac;
                    return push_hit(b, r2, hi2 > h2 ? hi2 : h2);
                };
                struct PF { int s; R x, y, z, m; V4<R> cv, cq, ip, iv, iq; int j, rp; };
                tile_pairs<1>(ring, [&](int k0, uint32_t b) {
#pragma unroll
                    for (int h = 0; h < 8; h += 4) {
                        const V4<R> X = ld4(tx + k0 + h), Y = ld4(ty + k0 + h),
                                    Z = ld4(tz + k0 + h), W = ld4(th2 + k0 + h);
                        b = in(b, X.x, Y.x, Z.x, W.x);
                        b = in(b, X.y, Y.y, Z.y, W.y);
                        b = in(b, X.z, Y.z, Z.z, W.z);
                        b = in(b, X.w, Y.w, Z.w, W.w);
                    }
                    return b;
                }, [&](int s, int k) {
                    int jr = 0, rp = 0;
                    if constexpr (RUNGS) { jr = tj[k]; rp = a.rpack[jr]; }
                    if constexpr (MIXED)
                        return PF{s, tx[k], ty[k], tz[k], trm[k], trec1[k], trec2[k], sp[s], sv[s],
                                  sq[s], jr, rp};
                    const int32_t j = tj[k];
                    return PF{s, tx[k], ty[k], tz[k], (R)a.ms[j], rec1[j], rec2[j], sp[s], sv[s],
                              sq[s], jr, rp};
                }, [&](const PF &d, bool valid, bool decided) -> bool {
                    const int s = d.s;
                    const V4<R> &cv = d.cv, &cq = d.cq, &ip = d.ip, &iv = d.iv, &iq = d.iq;
                    R ex, ey, ez;
                    const R r2 = pair_r2<MIXED, WRAP, R>(d.x, d.y, d.z, ip.x, ip.y, ip.z,
                                                         per, g, Lf, hLf, ex, ey, ez);
                    const R r = pair_sqrt(r2);
                    const R Hs_ = ip.w, Hj = cv.w;
                    // near the boundary the FP64 test decides (mixed, rare)
                    if (MIXED && !decided && valid &&
                        r >= (Hs_ > Hj ? Hs_ : Hj) * (WRAP ? qlow : qlo))
                        return true;
                    R Gi = 0, Gj = 0;
                    // (the sink's sigma / H^5 is prepared once, in its record)
                    if constexpr (K == 0) {
                        if (r2 < Hs_ * Hs_) Gi = iq.w * shape_g<K, R>(r * iv.w, Hs_, r);
                        if (r2 < Hj * Hj) {
                            const R hinv = cq.x;
                            const R h2 = hinv * hinv;
                            Gj = sig * shape_g<K, R>(r * hinv, Hj, r) * (h2 * h2 * hinv);
                        }
                    } else {
                        // the Wendland shapes vanish for q >= 1 through their
                        // clamped (1 - q), so no branch on the support is needed
                        // (2M mixed forces 3.41 -> 3.33 ms)
                        Gi = iq.w * shape_g<K, R>(r * iv.w, Hs_, r);
                        const R hinv = cq.x;
                        const R h2 = hinv * hinv;
                        Gj = sig * shape_g<K, R>(r * hinv, Hj, r) * (h2 * h2 * hinv);
                    }
                    // x_ij = x_i - x_j = -d ; v_ij = v_i - v_j
                    const R xx = -ex, xy = -ey, xz = -ez;
                    const R wx = iv.x - cv.x, wy = iv.y - cv.y, wz = iv.z - cv.z;
                    const R vdotx = wx * xx + wy * xy + wz * xz;
                    const R hbar = R(0.25) * (Hs_ + Hj);
                    const R mu = hbar * vdotx * pair_rcp(r2 + eps * hbar * hbar);
                    R Pi = 0;
                    if (vdotx < R(0)) {
                        const R cbar = R(0.5) * (iq.y + cq.z);
                        const R rbar = R(0.5) * (iq.z + cq.w);
                        Pi = (-alpha * cbar * mu + beta * mu * mu) * pair_rcp(rbar);
                    }
                    const R Gbar = R(0.5) * (Gi + Gj);
                    const R mj = d.m;
                    const R sc_ = mj * (iq.x * Gi + cq.y * Gj + Pi * Gbar);
                    if (valid && r2 > R(0)) {
                        atomicAdd(&acc[0][s], (double)(-sc_ * xx));
                        atomicAdd(&acc[1][s], (double)(-sc_ * xy));
                        atomicAdd(&acc[2][s], (double)(-sc_ * xz));
                        // du/dt: A_i m_j G_i v.x + (1/2) m_j Pi Gbar v.x (A_i is the sink's)
                        atomicAdd(&acc[3][s],
                                  (double)(mj * vdotx * (pdv * iq.x * Gi + R(0.5) * Pi * Gbar)));
                        if constexpr (EV) {
                            if (evolved) atomicAdd(&acc[EV ? 4 : 0][s], (double)(mj * vdotx * Gi));
                        }
                        if (mu < R(0)) lds_max_nonneg(&amu[s], -mu);
                    }
                    if constexpr (RUNGS) {
                        // F_i without i itself (a coincident j counts)
                        if (valid && d.j != asidx[s]) {
                            atomicMax(&armax[s], d.rp & 255);
                            if (d.rp >> 8) atomicAdd(&amiss[0], 1);
                        }
                    }
                    return false;
                }, [&](int s_, int k_, bool act_) -> bool {
                    bool in = false;
                    if (act_) {
                        const int64_t jj = (int64_t)tj[k_];
                        const int64_t si_ = sink_index(a, g, grp, s_);
                        const double hi_ = a.Hs[si_], hj_ = a.Hs[jj];
                        in = exact_inside(a.xs, a.ys, a.zs, si_, jj,
                                          fmax(hi_ * hi_, hj_ * hj_), per, g);
                    }
                    retests += __popcll(__ballot(act_));
                    rej += __popcll(__ballot(act_ && !in));
                    return in;
                }, cnt);
            };
            if (wrapf) tile(std::true_type{});
            else tile(std::false_type{});
            __syncthreads();
            for (int q = 0; q < ((EV && evolved) ? 5 : 4); ++q) {
                acc_d[q] += acc[q][lane];
                acc[q][lane] = 0;
            }
        };
        // Candidates are loaded 64 slots at a time; those that no sink's ball
        // reaches and whose own ball reaches no sink are dropped, the rest
        // appended to the queue, and each full half of it is a tile (one call
        // site of the tile code: the loop flushes the last partial tile
        // itself, before the walk refines again, whose stage shares this LDS).
        // the next load's slot is fetched while this one is filtered
        auto load_slot = [&](int t) -> Slot {
            const uint32_t *const cl = (LISTED && !MIXED) ? cand_rd : cand_lds;
            const int64_t j = (MIXED || !ws.far) ? sweep_slot(g, cl, ws.ncand, t, nload, lb)
                                                 : slot_index(g, cl, ws.ncand, t << (6 - lb), Bg);
            if (j < 0) return Slot{-1, 0.0, 0.0, 0.0, 0.0};
            return Slot{j, a.xs[j], a.ys[j], a.zs[j], a.Hs[j]};
        };
        Slot nxt = nload > 0 ? load_slot(0) : Slot{-1, 0.0, 0.0, 0.0, 0.0};
        for (int t = 0;;) {
          if (t < nload) {
            const Slot cur = nxt;
            const int64_t j = cur.j;
            slots += (unsigned long long)__popcll(__ballot(j >= 0));
            ++t;
            if (t < nload) nxt = load_slot(t);
            R px = R(0), py = R(0), pz = R(0), ph2 = R(0);
            bool keep = false;
            if (j >= 0) {
                double d0 = cur.x - gc[0], d1 = cur.y - gc[1], d2 = cur.z - gc[2];
                if (per && ws.far) {   // (see the density pass)
                    d0 = min_image(d0, g.L[0], g.halfL[0]);
                    d1 = min_image(d1, g.L[1], g.halfL[1]);
                    d2 = min_image(d2, g.L[2], g.halfL[2]);
                }
                const double Hj = cur.w;
                keep = fil.inside_fs((float)d0, (float)d1, (float)d2, (float)Hj);
                if constexpr (MIXED) {
                    px = (R)d0; py = (R)d1; pz = (R)d2;
                    const R hj = (R)Hj;
                    ph2 = hj * hj * band1;
                } else {
                    px = cur.x; py = cur.y; pz = cur.z;
                    ph2 = Hj * Hj;
                }
            }
            const uint64_t kb = __ballot(keep);
            if (keep) {
                const int at = (qb + qn + (int)__builtin_amdgcn_mbcnt_hi(
                                               (uint32_t)(kb >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u))) &
                               (kQueue - 1);
                qx_[at] = px; qy_[at] = py; qz_[at] = pz; qh2_[at] = ph2;
                qj_[at] = (int32_t)j;
            }
            qn += __popcll(kb);
          }
          if (qn >= kWave || (t >= nload && qn > 0)) {
            const int nv = qn < kWave ? qn : kWave;
            run_tile(nv);
            qb ^= kWave;
            qn -= nv;
          }
          if (t >= nload && qn == 0) break;
        }
        if constexpr (!LISTED) {
            if (ws.nstack == 0) break;
            ws.ncand = 0;
        }
    }
    __syncthreads();
    const R mumax = bits_to_real(amu[lane]);
    bool nonfinite = false;
    if (act) {
        const double axv = acc_d[0], ayv = acc_d[1], azv = acc_d[2];
        a.ax[i] = axv;
        a.ay[i] = ayv;
        a.az[i] = azv;
        a.du[i] = acc_d[3];
        double amag = sqrt(axv * axv + ayv * ayv + azv * azv);
        double den = (1.0 + 0.6 * a.alpha) * (double)ci + 0.6 * a.beta * (double)mumax;
        double dtv = a.dt_max;
        if (amag > 0.0) dtv = fmin(dtv, a.eta_a * sqrt(Hd / amag));
        if (den > 0.0) dtv = fmin(dtv, a.eta_c * 0.5 * Hd / den);
        // a non-finite |a| or signal speed gives no limit: the step is NaN
        // (fmin would otherwise drop it) and the status word says so
        if (!isfinite(amag) || !isfinite(den)) dtv = NAN;
        a.dt[i] = dtv;
        nonfinite = !isfinite(dtv) || !isfinite(acc_d[3]);
        if (evolved) a.drho[i] = acc_d[4] / a.oms[i];
        if constexpr (RUNGS) a.nbmax[i] = (double)armax[lane];
    }
    // the particle itself passed the distance test once (r = 0)
    int pairs_n = wave_sum_i(act ? cnt - 1 : 0) - rej;
    int nact = wave_sum_i(act ? 1 : 0);
    const int nnan = wave_sum_i(nonfinite ? 1 : 0);
    const int nret = retests;   // (a wave total)
    if (a.levs_out) {
        // next step's level from this pass's list length r (candidate slots
        // loaded per neighbour pair of an average sink), against the mean r
        // of the previous force pass: a list more than 1.5 times as long as
        // the mean halves the group's buckets, one shorter than the mean
        // doubles them again, up to the base size (the first pass keeps the
        // levels)
        const double pps = nact > 0 ? (double)pairs_n / nact : 0.0;
        const double r = (double)slots / (pps > 1.0 ? pps : 1.0);
        int hn = level;
        if (lref > 0.0) hn += r > 1.5 * lref ? -1 : (r < lref ? 1 : 0);
        hn = hn < 0 ? 0 : (hn > a.lev_max ? a.lev_max : hn);
        if (act) a.levs_out[i] = (double)hn;
    }
    if (lane == 0) {
        if (RUNGS && amiss[0]) atomicAdd(&ctr[C_FGMISS], (unsigned long long)amiss[0]);
        atomicAdd(&ctr[C_SLOTS_F], slots);
        atomicAdd(&ctr[C_LEV0 + level], 1ull);
        if (nnan) atomicAdd(&ctr[C_NONFINITE], (unsigned long long)nnan);
        if (nret) atomicAdd(&ctr[C_RETEST], (unsigned long long)nret);
        atomicAdd(&ctr[C_PAIRS_F], (unsigned long long)pairs_n);
        atomicAdd(&ctr[C_PAIRS_F_TOT], (unsigned long long)pairs_n);
        atomicAdd(&ctr[C_CAND_F], cand_tested * (unsigned long long)nact);
        if (overflows) atomicAdd(&ctr[C_OVERFLOW], (unsigned long long)overflows);
    }
}

template <int K, bool MIXED, bool RUNGS, int LM, bool EV = true>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void k_forces(SweepArgs a) {
    if constexpr (LM == kLmPersistent) {
        int k = 0;
        for (int64_t grp; (grp = next_group(a.queue, a.ngroups, k)) >= 0;)
            forces_group<K, MIXED, RUNGS, true, EV>(a, grp);
    } else {
        forces_group<K, MIXED, RUNGS, LM == kLmListed, EV>(a, xcd_group(blockIdx.x, gridDim.x));
    }
}

// The interaction list of each sink group for one sweep, as a kernel of its
// own before the sweep: the walk (gather test at the search radius Hw of the
// density pass, or the gather-or-scatter test at H of the force pass) and the
// per-sink refinement, chunk after chunk, with the same code and inputs as
// the walking sweep kernels use, hence the same chunks.  Each step of the
// walk waits on memory; here (84 VGPRs, five waves per SIMD) the waits of
// more groups overlap than in the sweep kernels, and those then hold no walk
// code.  A list of more than kListChunks chunks is marked long and left to
// the walking kernel.
template <bool SCATTER>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(5))) void k_walk(SweepArgs a) {
    __shared__ uint32_t cand[kCandCap];
    __shared__ alignas(16) float stage[kRefineStageBytes / 4];
    const int lane = threadIdx.x;
    const int64_t grp = xcd_group(blockIdx.x, gridDim.x);
    uint32_t *const stack = a.wstack + grp * kStackCap;
    const int sid = a.grp_set[grp];
    SetGeom g = a.sets[sid];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    int64_t i;
    bool act;
    if (!group_sinks(a, g, grp, i, act)) return;
    int level;
    (void)group_bucket(a, g, i, act, level);
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    // the radius the sweep walks with (density: its first search radius)
    double Rw;
    if constexpr (SCATTER) {
        Rw = act ? a.Hs[i] : 0.0;
    } else {
        const double cap = set_hcap(g, per, a.h_max);
        double H = act ? a.Hs[i] : 0.0;
        if (!(H > 0.0)) H = 0.01 * cap;
        if (H > cap) H = cap;
        Rw = fmin(a.oversel * H, cap);
    }
    double gc[3];
    for (int q = 0; q < 3; ++q) {
        double mn = wave_min(act ? xi[q] : DBL_MAX), mx = wave_max(act ? xi[q] : -DBL_MAX);
        gc[q] = 0.5 * (mn + mx);
    }
    double gext[3];
    for (int q = 0; q < 3; ++q) gext[q] = wave_max(act ? fabs(xi[q] - gc[q]) : 0.0);
    const double Rmax = wave_max(act ? Rw : 0.0);
    Sink sk;
    sink_bounds(act, xi, Rw, sk);
    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    walk_reset(stack, ws, false, g);
    uint32_t *const out = a.wlist_out + grp * kListCap;
    int32_t *const h = a.whdr_out + grp * kWalkWords;
    int nch = 0, farm = 0, flags = 0;
    while (true) {
        walk<SCATTER>(g, per, slop, a.nodes, sk, stack, cand, ws);
        if (ws.overflow) {
            // the stack was too small: the whole list again as the linear test
            flags |= kListLinear;
            nch = 0;
            farm = 0;
            walk_reset(stack, ws, true, g);
            continue;
        }
        refine<SCATTER>(g, per, slop, a.nodes, xi, Rw, Rmax, act, gc, gext, cand, stage, ws);
        if (ws.ncand > 0) {
            if (nch == kListChunks) { flags |= kListLong; break; }
            for (int t = lane; t < ws.ncand; t += kWave) out[nch * kCandCap + t] = cand[t];
            if (lane == 0) h[3 + nch] = ws.ncand;
            farm |= (ws.far ? 1 : 0) << nch;
            ++nch;
        }
        if (ws.nstack == 0) break;
        ws.ncand = 0;
    }
    if (lane == 0) {
        h[0] = nch;
        h[1] = farm;
        h[2] = flags;
    }
}

// ================================================================ interface correction
//
// Two gather sums at the converged H for the interface correction (Sec.
// 2.3.4), with the density pass's walk, refinement, candidate filter, queue
// and pair compaction (one scan, no iteration):
//   MODE 0, kernel imbalance (eq:Kernel_imbalance): per sink, over G_i and i,
//     D = sum m_j f(q),  N = sum kappa_ij m_j f(q) (x_j - x_i),
//     I = alpha |N| / (h D) with h = H/2 (the factor sigma/H^3 of W cancels);
//   MODE 1, averages: w_ij = exp(-I_j^2) f(q), Tbar = sum w T_j / sum w,
//     Pbar = sum w P_j / sum w.
// Both sums vanish continuously at the support (f(1) = 0), so the mixed path
// needs no FP64 re-test near it.
template <int K, bool MIXED, int MODE>
__global__ __launch_bounds__(kWave) void k_gather_sums(SweepArgs a) {
    typedef typename std::conditional<MIXED, float, double>::type R;
    __shared__ uint32_t cand[kCandCap];
    __shared__ uint16_t ring[kRing];
    // queue: x y z and three payload columns (MODE 0: m, material; MODE 1:
    // exp(-I^2), T, P)
    constexpr int kTileBytes = 6 * kQueue * (int)sizeof(R);
    __shared__ alignas(16) unsigned char tile_buf[kTileBytes > kRefineStageBytes ? kTileBytes
                                                                                  : kRefineStageBytes];
    R *const qx_ = reinterpret_cast<R *>(tile_buf);
    R *const qy_ = qx_ + kQueue;
    R *const qz_ = qy_ + kQueue;
    R *const q1_ = qz_ + kQueue;
    R *const q2_ = q1_ + kQueue;
    R *const q3_ = q2_ + kQueue;
    float *const stage = reinterpret_cast<float *>(tile_buf);
    __shared__ V4<R> sp[kWave];   // sink: position, 1/H
    __shared__ R smat[kWave];     // sink: material (MODE 0)
    __shared__ double acc[4][kWave];

    const int lane = threadIdx.x;
    const int64_t grp = xcd_group(blockIdx.x, gridDim.x);
    uint32_t *const stack = a.wstack + grp * kStackCap;
    const int sid = a.grp_set[grp];
    SetGeom g = a.sets[sid];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    const int64_t i = g.p0 + (grp - g.g0) * kGroup + lane;
    const bool act = i < g.p1;
    int level;
    const int Bg = group_bucket(a, g, i, act, level);
    const int lb = 31 - __builtin_clz((unsigned)Bg);
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    const double H = act ? a.Hs[i] : 0.0;

    double gc[3];
    for (int q = 0; q < 3; ++q) {
        const double mn = wave_min(act ? xi[q] : DBL_MAX), mx = wave_max(act ? xi[q] : -DBL_MAX);
        gc[q] = 0.5 * (mn + mx);
    }
    double gext[3];
    for (int q = 0; q < 3; ++q) gext[q] = wave_max(act ? fabs(xi[q] - gc[q]) : 0.0);
    const R Lf[3] = {(R)g.L[0], (R)g.L[1], (R)g.L[2]};
    const R hLf[3] = {(R)g.halfL[0], (R)g.halfL[1], (R)g.halfL[2]};
    R qx, qy, qz;
    if constexpr (MIXED) {
        qx = (R)(per ? min_image(xi[0] - gc[0], g.L[0], g.halfL[0]) : xi[0] - gc[0]);
        qy = (R)(per ? min_image(xi[1] - gc[1], g.L[1], g.halfL[1]) : xi[1] - gc[1]);
        qz = (R)(per ? min_image(xi[2] - gc[2], g.L[2], g.halfL[2]) : xi[2] - gc[2]);
    } else {
        qx = xi[0]; qy = xi[1]; qz = xi[2];
    }
    const R Hr = (R)H;
    sp[lane] = V4<R>{qx, qy, qz, act ? R(1) / Hr : R(0)};
    if (MODE == 0) smat[lane] = (R)(act && a.mats ? a.mats[i] : 0.0);
    for (int q = 0; q < 4; ++q) acc[q][lane] = 0.0;
    const R H2 = MIXED ? Hr * Hr : (R)(H * H);
    bool wrapf = MIXED && group_needs_wrap(per, g, gext, wave_max(act ? H : 0.0));
    const GroupFilter fil = group_filter(act, xi, gc, H, per, g, gext);

    Sink sk;
    sink_bounds(act, xi, H, sk);
    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    bool linear = false;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt = 0;
    walk_reset(stack, ws, linear, g);
    while (true) {
        walk<false>(g, per, slop, a.nodes, sk, stack, cand, ws);
        if (ws.overflow) {
            // restart with the linear bucket test
            linear = true;
            for (int q = 0; q < 4; ++q) sums[q] = 0.0;
            walk_reset(stack, ws, true, g);
            continue;
        }
        refine<false>(g, per, slop, a.nodes, xi, H, wave_max(act ? H : 0.0), act, gc, gext, cand,
                      stage, ws);
        const int nload = sweep_tiles(ws.ncand, Bg);
        int qb = 0, qn = 0;
        auto run_tile = [&](int nv) {
            R *const tx = qx_ + qb, *const ty = qy_ + qb, *const tz = qz_ + qb;
            R *const t1 = q1_ + qb, *const t2 = q2_ + qb, *const t3 = q3_ + qb;
            if (lane >= nv) {
                tx[lane] = (R)NAN; ty[lane] = R(0); tz[lane] = R(0);
                t1[lane] = R(0); t2[lane] = R(0); t3[lane] = R(0);
            }
            if constexpr (!MIXED)
                wrapf = __any(lane < nv && needs_image(per, g, gc, gext, (double)tx[lane],
                                                       (double)ty[lane], (double)tz[lane]));
            __syncthreads();
            auto tile = [&](auto wrap_tag) {
                constexpr bool WRAP = decltype(wrap_tag)::value;
                struct PG { int s; R x, y, z, p1, p2, p3; V4<R> si; };
                tile_pairs<1>(ring, [&](int k0, uint32_t b) {
#pragma unroll
                    for (int h = 0; h < 8; h += 4) {
                        const V4<R> X = ld4(tx + k0 + h), Y = ld4(ty + k0 + h),
                                    Z = ld4(tz + k0 + h);
                        R dx, dy, dz;
                        b = push_hit(b, pair_r2<MIXED, WRAP, R>(X.x, Y.x, Z.x, qx, qy, qz, per, g,
                                                                Lf, hLf, dx, dy, dz), H2);
                        b = push_hit(b, pair_r2<MIXED, WRAP, R>(X.y, Y.y, Z.y, qx, qy, qz, per, g,
                                                                Lf, hLf, dx, dy, dz), H2);
                        b = push_hit(b, pair_r2<MIXED, WRAP, R>(X.z, Y.z, Z.z, qx, qy, qz, per, g,
                                                                Lf, hLf, dx, dy, dz), H2);
                        b = push_hit(b, pair_r2<MIXED, WRAP, R>(X.w, Y.w, Z.w, qx, qy, qz, per, g,
                                                                Lf, hLf, dx, dy, dz), H2);
                    }
                    return b;
                }, [&](int s, int k) {
                    return PG{s, tx[k], ty[k], tz[k], t1[k], t2[k], t3[k], sp[s]};
                }, [&](const PG &d, bool valid, bool) -> bool {
                    R ex, ey, ez;
                    const R r2 = pair_r2<MIXED, WRAP, R>(d.x, d.y, d.z, d.si.x, d.si.y, d.si.z,
                                                         per, g, Lf, hLf, ex, ey, ez);
                    R f, qfp;
                    shape_f_qfp<K, R>(pair_sqrt(r2) * d.si.w, f, qfp);
                    if (valid) {
                        if constexpr (MODE == 0) {
                            const R w = d.p1 * f;
                            const R kw = d.p2 == smat[d.s] ? w : -w;
                            atomicAdd(&acc[0][d.s], (double)w);
                            atomicAdd(&acc[1][d.s], (double)(kw * ex));
                            atomicAdd(&acc[2][d.s], (double)(kw * ey));
                            atomicAdd(&acc[3][d.s], (double)(kw * ez));
                        } else {
                            const R w = d.p1 * f;
                            atomicAdd(&acc[0][d.s], (double)w);
                            atomicAdd(&acc[1][d.s], (double)(w * d.p2));
                            atomicAdd(&acc[2][d.s], (double)(w * d.p3));
                        }
                    }
                    return false;
                }, [&](int, int, bool) -> bool { return false; }, cnt);
            };
            if (wrapf) tile(std::true_type{});
            else tile(std::false_type{});
            __syncthreads();
            for (int q = 0; q < 4; ++q) {
                sums[q] += acc[q][lane];
                acc[q][lane] = 0.0;
            }
        };
        for (int t = 0;;) {
          if (t < nload) {
            const int64_t j = (MIXED || !ws.far) ? sweep_slot(g, cand, ws.ncand, t, nload, lb)
                                                 : slot_index(g, cand, ws.ncand, t << (6 - lb), Bg);
            ++t;
            R px = R(0), py = R(0), pz = R(0), p1 = R(0), p2 = R(0), p3 = R(0);
            bool keep = false;
            if (j >= 0) {
                double d0 = a.xs[j] - gc[0], d1 = a.ys[j] - gc[1], d2 = a.zs[j] - gc[2];
                if (per) {
                    d0 = min_image(d0, g.L[0], g.halfL[0]);
                    d1 = min_image(d1, g.L[1], g.halfL[1]);
                    d2 = min_image(d2, g.L[2], g.halfL[2]);
                }
                keep = fil.inside((float)d0, (float)d1, (float)d2);
                if constexpr (MIXED) {
                    px = (R)d0; py = (R)d1; pz = (R)d2;
                } else {
                    px = a.xs[j]; py = a.ys[j]; pz = a.zs[j];
                }
                if constexpr (MODE == 0) {
                    p1 = (R)a.ms[j];
                    p2 = (R)(a.mats ? a.mats[j] : 0.0);
                } else {
                    const double Ij = a.imb[j];
                    p1 = (R)exp(-Ij * Ij);
                    p2 = (R)a.us[j];
                    p3 = (R)a.Ps_[j];
                }
            }
            const uint64_t kb = __ballot(keep);
            if (keep) {
                const int at = (qb + qn + (int)__builtin_amdgcn_mbcnt_hi(
                                               (uint32_t)(kb >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u))) &
                               (kQueue - 1);
                qx_[at] = px; qy_[at] = py; qz_[at] = pz;
                q1_[at] = p1; q2_[at] = p2; q3_[at] = p3;
            }
            qn += __popcll(kb);
          }
          if (qn >= kWave || (t >= nload && qn > 0)) {
            const int nv = qn < kWave ? qn : kWave;
            run_tile(nv);
            qb ^= kWave;
            qn -= nv;
          }
          if (t >= nload && qn == 0) break;
        }
        if (ws.nstack == 0) break;
        ws.ncand = 0;
    }
    if (act) {
        if constexpr (MODE == 0) {
            const double nrm = sqrt(sums[1] * sums[1] + sums[2] * sums[2] + sums[3] * sums[3]);
            a.imb[i] = a.ic_alpha * nrm / (0.5 * H * sums[0]);
        } else {
            a.tbar[i] = sums[1] / sums[0];
            a.pbar[i] = sums[2] / sums[0];
        }
    }
}

// ================================================================ neighbour lists

template <bool FORCE, bool FILL>
__global__ __launch_bounds__(kWave) void k_neighbors(SweepArgs a) {
    __shared__ uint32_t stack[kStackCap];
    __shared__ uint32_t cand[kCandCap];
    __shared__ double tx[kWave], ty[kWave], tz[kWave], tH[kWave];
    __shared__ int32_t tid[kWave];

    const int lane = threadIdx.x;
    const int64_t grp = xcd_group(blockIdx.x, gridDim.x);
    unsigned long long *const ctr = a.cnt + cnt_shard(grp);   // this group's counter copy
    const int sid = a.grp_set[grp];
    const SetGeom g = a.sets[sid];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    const int64_t i = g.p0 + (grp - g.g0) * kGroup + lane;
    const bool act = i < g.p1;
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    const double Hd = act ? a.Hs[i] : 0.0;
    const double Hi2 = Hd * Hd;
    const int64_t orig = act ? (int64_t)a.perm[i] : 0;
    int64_t wpos = (FILL && act) ? a.offsets[orig] : 0;

    Sink sk;
    sink_bounds(act, xi, Hd, sk);
    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    walk_reset(stack, ws, false, g);
    int64_t cnt = 0;
    int overflows = 0;
    while (true) {
        walk<FORCE>(g, per, slop, a.nodes, sk, stack, cand, ws);
        if (ws.overflow) {
            ++overflows;
            cnt = 0;
            walk_reset(stack, ws, true, g);
            continue;
        }
        for (int t0 = 0; t0 < ws.ncand; t0 += kWave / a.B) {
            int64_t j = slot_index(g, cand, ws.ncand, t0, a.B);
            tx[lane] = j >= 0 ? a.xs[j] : NAN;
            ty[lane] = j >= 0 ? a.ys[j] : 0.0;
            tz[lane] = j >= 0 ? a.zs[j] : 0.0;
            tH[lane] = j >= 0 ? a.Hs[j] : 0.0;
            tid[lane] = j >= 0 ? (int32_t)j : -1;
            __syncthreads();
            for (int k = 0; k < kWave; ++k) {
                const int32_t jj = tid[k];
                double dx = tx[k] - xi[0], dy = ty[k] - xi[1], dz = tz[k] - xi[2];
                if (per) {
                    dx = min_image(dx, g.L[0], g.halfL[0]);
                    dy = min_image(dy, g.L[1], g.halfL[1]);
                    dz = min_image(dz, g.L[2], g.halfL[2]);
                }
                double r2 = r2_exact(dx, dy, dz);
                double Hs2 = Hi2;
                if (FORCE) {
                    double Hj2 = tH[k] * tH[k];
                    Hs2 = Hs2 > Hj2 ? Hs2 : Hj2;
                }
                if (act && jj >= 0 && (int64_t)jj != i && r2 < Hs2) {
                    if (FILL) a.idx[wpos + cnt] = (int32_t)a.perm[jj];
                    ++cnt;
                }
            }
            __syncthreads();
        }
        if (ws.nstack == 0) break;
        ws.ncand = 0;
    }
    if (!FILL && act) a.row_count[orig] = cnt;
    if (lane == 0 && overflows) atomicAdd(&ctr[C_OVERFLOW], (unsigned long long)overflows);
}

// One workgroup per row: bitonic sort in LDS (rows up to kMaxRow entries).
__global__ __launch_bounds__(256) void k_sort_rows(const int64_t *__restrict__ offsets,
                                                   int32_t *__restrict__ idx,
                                                   unsigned long long *cnt) {
    __shared__ int32_t v[kMaxRow];
    const int64_t row = blockIdx.x;
    const int64_t b = offsets[row], e = offsets[row + 1];
    const int64_t len = e - b;
    if (len <= 1) return;
    if (len > kMaxRow) {
        if (threadIdx.x == 0) atomicAdd(&cnt[cnt_shard(blockIdx.x) + C_ROWLONG], 1ull);
        return;
    }
    int P = 1;
    while (P < len) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x) v[t] = t < len ? idx[b + t] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int t = threadIdx.x; t < P; t += blockDim.x) {
                int u = t ^ jj;
                if (u > t) {
                    bool up = (t & k) == 0;
                    int32_t x = v[t], y = v[u];
                    if ((x > y) == up) { v[t] = y; v[u] = x; }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < len; t += blockDim.x) idx[b + t] = v[t];
}


// FastGas marking (Sec. 2.3.6, last paragraph), below fastgas n active
// particles: every particle of a bucket on the interaction list of an active
// sink group is marked, and so are the sinks; the density pass then runs for
// the marked particles only.  The lists are taken with the sinks' balls
// widened to oversel H and their cell bound by (oversel - 1) times their
// largest H, so that the smoothing lengths of this substep's density pass,
// which move little over a substep, keep the force sets of the active
// particles inside them (the force pass counts any neighbour left out).
__global__ __launch_bounds__(kWave) void k_mark(SweepArgs a) {
    __shared__ uint32_t cand[kCandCap];
    const int lane = threadIdx.x;
    const int64_t grp = xcd_group(blockIdx.x, gridDim.x);
    if (!((double)*a.nsinks < a.fastgas * (double)(a.sets[0].p1 - a.sets[0].p0))) return;
    uint32_t *const stack = a.wstack + grp * kStackCap;
    const SetGeom g = a.sets[0];
    const bool per = a.periodic != 0;
    const double slop = set_slop(g);
    int64_t i;
    bool act;
    if (!group_sinks(a, g, grp, i, act)) return;
    const double xi[3] = {act ? a.xs[i] : 0.0, act ? a.ys[i] : 0.0, act ? a.zs[i] : 0.0};
    const double Hd = act ? a.Hs[i] : 0.0;
    if (act) a.mark[i] = 1u;
    Sink sk;
    sink_bounds(act, xi, a.oversel * Hd, sk);
    const double grow = (a.oversel - 1.0) * wave_max(act ? Hd : 0.0);
    for (int q = 0; q < 3; ++q) { sk.clo[q] -= grow; sk.chi[q] += grow; }
    WalkState ws{0, 0, -1, a.stack_limit, false, false};
    walk_reset(stack, ws, false, g);
    while (true) {
        walk<true>(g, per, slop, a.nodes, sk, stack, cand, ws);
        if (ws.overflow) {
            walk_reset(stack, ws, true, g);
            continue;
        }
        for (int t0 = 0; t0 < ws.ncand; t0 += kWave / a.B) {
            const int64_t j = slot_index(g, cand, ws.ncand, t0, a.B);
            if (j >= 0) a.mark[j] = 1u;
        }
        __syncthreads();   // (the next walk step rewrites cand)
        if (ws.nstack == 0) break;
        ws.ncand = 0;
    }
}

// ---------------------------------------------------------------- dispatch

inline SweepArgs base_args(Ctx *c) {
    SweepArgs a{};
    a.sets = c->d_sets;
    a.grp_set = c->d_grp_set;
    a.nodes = c->nodes;
    a.perm = c->d_perm[0];
    a.xs = c->xs; a.ys = c->ys; a.zs = c->zs; a.ms = c->ms;
    a.Hs = c->Hs; a.rhos = c->rhos; a.oms = c->oms;
    a.vxs = c->vxs; a.vys = c->vys; a.vzs = c->vzs; a.As = c->As; a.css = c->css;
    a.frec1 = c->frec1; a.frec2 = c->frec2; a.fm = c->fm;
    a.drec1 = c->drec1; a.drec2 = c->drec2;
    a.wstack = c->d_wstack;
    a.cnt = c->d_cnt;
    a.B = c->bucket;
    a.levs = c->dyn ? c->levs : nullptr;
    a.levs_out = c->dyn ? c->levs : nullptr;
    a.lev_max = c->dyn ? base_level(c->base_bucket) : 0;
    a.lev_ref = c->d_levref;
    a.periodic = c->prm.periodic;
    a.oversel = c->prm.oversel;
    a.tol = c->prm.nr_tol;
    a.h_max = c->prm.h_max;
    a.n_ngb = c->prm.n_ngb;
    a.maxit = c->prm.nr_maxit;
    a.stack_limit = c->prm.stack_limit;
    a.alpha = c->prm.alpha; a.beta = c->prm.beta; a.eps = c->prm.eps_av;
    a.eta_a = c->prm.eta_a; a.eta_c = c->prm.eta_c; a.dt_max = c->prm.dt_max;
    a.sinks = c->sweep_sinks;
    a.nsinks = c->sweep_nsinks;
    a.rpack = c->sweep_rpack ? c->rpack : nullptr;
    a.nbmax = c->nbmax;
    a.mark = c->mark;
    a.fastgas = c->prm.fastgas;
    return a;
}

// Clears the persistent launch's queue counters (a kernel rather than a
// memset, so the clear can be captured in a graph).
__global__ void k_queue_reset(uint32_t *queue) {
    if (threadIdx.x < kXcds) queue[threadIdx.x * kQueueStride] = 0u;
}

// Workgroups of a persistent launch: what the CUs hold at once (occupancy
// from the kernel's registers and LDS), at most one per sink group.  The
// count is taken once per kernel instance.
template <typename F>
unsigned persistent_grid(Ctx *c, F kernel, int &cache) {
    if (cache <= 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        cache = per_cu;
    }
    const int64_t cap = c->ncu > 0 ? (int64_t)cache * c->ncu : c->ngroups;
    return (unsigned)(c->ngroups < cap ? c->ngroups : cap);
}

// The launches of one sweep.  With stored lists (a context that holds the
// buffers; not in the substeps of individual time steps) the listed sweep
// kernel, one workgroup per group or persistent, then the walking kernel for
// the groups the listed one left (the others return at once); else the
// walking kernel for every group.
template <int K, bool MIXED>
void launch_density_k(Ctx *c, SweepArgs &a, hipStream_t s) {
    const unsigned ng = (unsigned)c->ngroups;
    if (!a.defer) {
        k_density<K, MIXED, kLmWalk><<<ng, kWave, 0, s>>>(a);
        return;
    }
    if (a.queue) {
        static int occ = 0;
        const unsigned grid = persistent_grid(c, k_density<K, MIXED, kLmPersistent>, occ);
        k_density<K, MIXED, kLmPersistent><<<grid, kWave, 0, s>>>(a);
    } else {
        k_density<K, MIXED, kLmListed><<<ng, kWave, 0, s>>>(a);
    }
    k_density<K, MIXED, kLmWalk><<<ng, kWave, 0, s>>>(a);
}

template <int K, bool MIXED>
void launch_forces_k(Ctx *c, SweepArgs &a, hipStream_t s) {
    const unsigned ng = (unsigned)c->ngroups;
    c->sweep_workgroups = c->ngroups;
    c->sweep_launch = SPH_LAUNCH_GROUPS;
    if (a.rpack) {
        // individual time steps: one workgroup per group of the sink list
        // (with the rung maximum over F_i)
        if (!a.defer) {
            c->sweep_launch = SPH_LAUNCH_WALK;
            k_forces<K, MIXED, true, kLmWalk><<<ng, kWave, 0, s>>>(a);
            return;
        }
        k_forces<K, MIXED, true, kLmListed><<<ng, kWave, 0, s>>>(a);
        k_forces<K, MIXED, true, kLmWalk><<<ng, kWave, 0, s>>>(a);
        return;
    }
    if (!a.defer) {
        c->sweep_launch = SPH_LAUNCH_WALK;
        k_forces<K, MIXED, false, kLmWalk><<<ng, kWave, 0, s>>>(a);
        return;
    }
    // (the listed FP64 kernels without the evolved density take four
    // accumulators; every other kernel five)
    auto listed = [&](auto ev_tag) {
        constexpr bool EV = decltype(ev_tag)::value;
        if (a.queue) {
            static int occ = 0;
            const unsigned grid =
                persistent_grid(c, k_forces<K, MIXED, false, kLmPersistent, EV>, occ);
            c->sweep_workgroups = grid;
            c->sweep_launch = SPH_LAUNCH_PERSISTENT;
            k_forces<K, MIXED, false, kLmPersistent, EV><<<grid, kWave, 0, s>>>(a);
        } else {
            k_forces<K, MIXED, false, kLmListed, EV><<<ng, kWave, 0, s>>>(a);
        }
    };
    if constexpr (MIXED) {
        listed(std::true_type{});
    } else {
        if (a.drho) listed(std::true_type{});
        else listed(std::false_type{});
    }
    k_forces<K, MIXED, false, kLmWalk><<<ng, kWave, 0, s>>>(a);
}

// With stored lists: the walk kernel of the sweep writes them (and the
// sweep's launches read them).
template <bool SCATTER>
hipError_t launch_walk(Ctx *c, SweepArgs &a, hipStream_t s) {
    a.wlist = a.wlist_out = c->d_wlist;
    a.whdr = a.whdr_out = c->d_whdr;
    a.defer = c->d_defer;
    k_walk<SCATTER><<<(unsigned)c->ngroups, kWave, 0, s>>>(a);
    return hipGetLastError();
}

// The launch shape of the context: a persistent launch clears its queue
// counters first.
inline hipError_t set_launch(Ctx *c, SweepArgs &a, bool rungs, hipStream_t s) {
    a.ngroups = c->ngroups;
    a.queue = (c->launch == SPH_LAUNCH_PERSISTENT && c->d_queue && !rungs) ? c->d_queue : nullptr;
    if (a.queue) {
        k_queue_reset<<<1, kWave, 0, s>>>(a.queue);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <bool MIXED>
hipError_t density_dispatch(Ctx *c, SweepArgs a, hipStream_t s) {
    switch (c->prm.kernel) {
    case 0: launch_density_k<0, MIXED>(c, a, s); break;
    case 1: launch_density_k<1, MIXED>(c, a, s); break;
    case 2: launch_density_k<2, MIXED>(c, a, s); break;
    default: launch_density_k<3, MIXED>(c, a, s); break;
    }
    return hipGetLastError();
}

template <bool MIXED>
hipError_t forces_dispatch(Ctx *c, SweepArgs a, hipStream_t s) {
    switch (c->prm.kernel) {
    case 0: launch_forces_k<0, MIXED>(c, a, s); break;
    case 1: launch_forces_k<1, MIXED>(c, a, s); break;
    case 2: launch_forces_k<2, MIXED>(c, a, s); break;
    default: launch_forces_k<3, MIXED>(c, a, s); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_density(Ctx *c, hipStream_t s) {
    if (c->ngroups == 0) return hipSuccess;
    SweepArgs a = base_args(c);
    hipError_t e = set_launch(c, a, c->sweep_sinks != nullptr, s);
    if (e != hipSuccess) return e;
    if (c->d_wlist && c->launch != SPH_LAUNCH_WALK) {
        mark(c, E_DWALK0, s);
        e = launch_walk<false>(c, a, s);
        if (e != hipSuccess) return e;
    }
    mark(c, E_DEN0, s);
    e = c->prm.precision == SPH_PREC_MIXED ? density_dispatch<true>(c, a, s)
                                           : density_dispatch<false>(c, a, s);
    mark(c, E_DEN1, s);
    return e;
}

// Mean list length per pair of the force pass just run (the reference of the
// next pass's level rule): slots per group over pairs per particle.
__global__ void k_level_ref(const unsigned long long *cnt, int64_t ngroups, int64_t n,
                            double *ref) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long pairs = 0, slots = 0;
    for (int q = 0; q < kCntShards; ++q) {
        pairs += cnt[q * kCntStride + C_PAIRS_F];
        slots += cnt[q * kCntStride + C_SLOTS_F];
    }
    const double pps = (double)pairs / (double)(n > 0 ? n : 1);
    *ref = (double)slots / (double)(ngroups > 0 ? ngroups : 1) / (pps > 1.0 ? pps : 1.0);
}

hipError_t launch_forces(Ctx *c, hipStream_t s) {
    if (c->ngroups == 0) return hipSuccess;
    SweepArgs a = base_args(c);
    a.ax = c->axs; a.ay = c->ays; a.az = c->azs; a.du = c->dus; a.dt = c->dts;
    a.drho = (c->prm.flags & SPH_FLAG_EVOLVED) ? c->drs : nullptr;
    a.entropy = (c->prm.flags & SPH_FLAG_ENTROPY) ? 1 : 0;
    hipError_t e = set_launch(c, a, a.rpack != nullptr, s);
    if (e != hipSuccess) return e;
    if (c->d_wlist && c->launch != SPH_LAUNCH_WALK) {
        mark(c, E_FWALK0, s);
        e = launch_walk<true>(c, a, s);
        if (e != hipSuccess) return e;
    }
    mark(c, E_FOR0, s);
    e = c->prm.precision == SPH_PREC_MIXED ? forces_dispatch<true>(c, a, s)
                                           : forces_dispatch<false>(c, a, s);
    mark(c, E_FOR1, s);
    if (e == hipSuccess && c->dyn) {
        k_level_ref<<<1, 64, 0, s>>>(c->d_cnt, c->ngroups, c->n, c->d_levref);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_mark(Ctx *c, hipStream_t s) {
    if (c->ngroups == 0) return hipSuccess;
    SweepArgs a = base_args(c);
    k_mark<<<(unsigned)c->ngroups, kWave, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_interface_sums(Ctx *c, int mode, hipStream_t s) {
    if (c->ngroups == 0) return hipSuccess;
    SweepArgs a = base_args(c);
    a.mats = c->mats_has ? c->mats : nullptr;
    a.imb = c->imbs;
    a.us = c->us;
    a.Ps_ = c->Ps;
    a.tbar = c->tbar;
    a.pbar = c->pbar;
    a.ic_alpha = c->prm.ic_alpha;
    dim3 grid((unsigned)c->ngroups), block(kWave);
    const bool mixed = c->prm.precision == SPH_PREC_MIXED;
#define GS(KK)                                                                              \
    if (mode == 0) {                                                                        \
        if (mixed) k_gather_sums<KK, true, 0><<<grid, block, 0, s>>>(a);                    \
        else k_gather_sums<KK, false, 0><<<grid, block, 0, s>>>(a);                         \
    } else {                                                                                \
        if (mixed) k_gather_sums<KK, true, 1><<<grid, block, 0, s>>>(a);                    \
        else k_gather_sums<KK, false, 1><<<grid, block, 0, s>>>(a);                         \
    }
    switch (c->prm.kernel) {
    case 0: GS(0); break;
    case 1: GS(1); break;
    case 2: GS(2); break;
    default: GS(3); break;
    }
#undef GS
    return hipGetLastError();
}

hipError_t launch_neighbors(Ctx *c, int mode, int64_t *row_count_caller, const int64_t *offsets,
                            int32_t *idx, hipStream_t s) {
    if (c->ngroups == 0) return hipSuccess;
    SweepArgs a = base_args(c);
    a.row_count = row_count_caller;
    a.offsets = offsets;
    a.idx = idx;
    dim3 grid((unsigned)c->ngroups), block(kWave);
    bool fill = idx != nullptr;
    if (mode == SPH_MODE_FORCE) {
        if (fill) k_neighbors<true, true><<<grid, block, 0, s>>>(a);
        else k_neighbors<true, false><<<grid, block, 0, s>>>(a);
    } else {
        if (fill) k_neighbors<false, true><<<grid, block, 0, s>>>(a);
        else k_neighbors<false, false><<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_sort_rows(Ctx *c, const int64_t *offsets, int32_t *idx, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_sort_rows<<<(unsigned)c->n, 256, 0, s>>>(offsets, idx, c->d_cnt);
    return hipGetLastError();
}

}  // namespace sphmi

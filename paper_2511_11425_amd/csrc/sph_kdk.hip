// sph_kdk.hip -- elementwise passes of the step: gathers into and scatters out
// of Hilbert order, the equation of state (Sec. 2.3.1), the kick-drift-kick
// integrator with the velocity/energy predictor (Sec. 2.3.6), and the FP64
// reductions of momentum, energy and the global time step.  All of these are
// HBM-bound streams; they are kept separate from the sweep so the same
// kernels serve the single-call interface and the captured step.
#include "sph_internal.h"

#include <cfloat>
#include <climits>
#include <cstddef>

namespace sphmi {

namespace {

constexpr int kThreads = 256;
constexpr int kRedBlocks = 512;

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__device__ inline int find_set_k(const SetGeom *sets, int nsets, int64_t i) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sets[mid].p0 <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_reset_counters(unsigned long long *cnt, int last) {
    const int t = threadIdx.x;
    if (t < kCntShards * kCntStride && t % kCntStride < last) cnt[t] = 0ull;
}

__global__ void k_fold_counters(const unsigned long long *__restrict__ cnt,
                                unsigned long long *__restrict__ sum) {
    const int k = threadIdx.x;
    if (k >= C_NCOUNTERS) return;
    unsigned long long v = 0;
    for (int q = 0; q < kCntShards; ++q) {
        const unsigned long long w = cnt[q * kCntStride + k];
        v = k == C_NR_ITER_MAX ? (w > v ? w : v) : v + w;
    }
    sum[k] = v;
}

__global__ void k_gather_cols(const uint32_t *__restrict__ perm, int64_t n, Cols c) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
#pragma unroll
    for (int q = 0; q < kMaxCols; ++q)
        if (q < c.n) c.dst[q][k] = c.src[q][i];
}

__global__ void k_scatter_cols(const uint32_t *__restrict__ perm, int64_t n, Cols c) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
#pragma unroll
    for (int q = 0; q < kMaxCols; ++q)
        if (q < c.n) c.dst[q][i] = c.src[q][k];
}

// EOS on sorted arrays: P, c and A = P / (Omega rho^2); P and c also go to
// the caller's arrays.
struct ForceRecords {   // per-particle records the force pass reads (one path's are null)
    const double *m, *H, *vx, *vy, *vz;
    float *rec1, *rec2, *fm;     // mixed path
    double *drec1, *drec2;       // FP64 path
};

__global__ void k_eos(const uint32_t *__restrict__ perm, int64_t n, int eos, double gam, double P0,
                      const double *__restrict__ rho, const double *__restrict__ u,
                      const double *__restrict__ om, double *__restrict__ Ps,
                      double *__restrict__ cs, double *__restrict__ As,
                      double *__restrict__ Pc, double *__restrict__ cc, ForceRecords fr) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double r = rho[k], uu = u[k];
    double P, c2;
    if (eos == SPH_EOS_IDEAL) {
        P = (gam - 1.0) * r * uu;
        c2 = gam * (gam - 1.0) * uu;
    } else {
        P = (gam - 1.0) * r * uu - gam * P0;
        c2 = gam * (P + P0) / r;
    }
    double c = c2 > 0.0 ? sqrt(c2) : 0.0;
    const double A = P / (om[k] * r * r);
    Ps[k] = P;
    cs[k] = c;
    As[k] = A;
    if (fr.rec1) {
        const double H = fr.H[k];
        float4 *r1 = reinterpret_cast<float4 *>(fr.rec1);
        float4 *r2 = reinterpret_cast<float4 *>(fr.rec2);
        r1[k] = make_float4((float)fr.vx[k], (float)fr.vy[k], (float)fr.vz[k], (float)H);
        r2[k] = make_float4((float)(1.0 / H), (float)A, (float)c, (float)r);
        fr.fm[k] = (float)fr.m[k];
    }
    if (fr.drec1) {
        const double H = fr.H[k];
        double4 *r1 = reinterpret_cast<double4 *>(fr.drec1);
        double4 *r2 = reinterpret_cast<double4 *>(fr.drec2);
        r1[k] = make_double4(fr.vx[k], fr.vy[k], fr.vz[k], H);
        r2[k] = make_double4(1.0 / H, A, c, r);
    }
    uint32_t i = perm[k];
    Pc[i] = P;
    cc[i] = c;
}

// Interface correction (Sec. 2.3.4), after the EOS pass and the two gather
// sums, in sorted order: with e = exp(-I^2) and T = u (c_v = 1),
//   P~ = e P + (1 - e) Pbar,  T~ = e T + (1 - e) Tbar,
//   rho~ = rho_EOS(T~, P~): ideal P~/((gamma-1) T~), stiffened
//          (P~ + gamma P0)/((gamma-1) T~); the uncorrected rho where that is
//          not a positive number;
//   c~ from the EOS at (rho~, T~), A = P~/(Omega rho~^2).
// The force pass then reads rho~, P~, c~ and A (and their FP32 or FP64
// records); the caller gets P~, c~, I and rho~.
__global__ void k_ic_correct(const uint32_t *__restrict__ perm, int64_t n, int eos, double gam,
                             double P0, double *rho, const double *__restrict__ u,
                             const double *__restrict__ om, double *Ps, double *cs, double *As,
                             const double *__restrict__ imb, const double *__restrict__ tbar,
                             const double *__restrict__ pbar, double *Pc, double *cc,
                             double *imb_c, double *rho_c, ForceRecords fr) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double I = imb[k];
    const double e = exp(-I * I);
    const double P = e * Ps[k] + (1.0 - e) * pbar[k];
    const double T = e * u[k] + (1.0 - e) * tbar[k];
    double r = eos == SPH_EOS_IDEAL ? P / ((gam - 1.0) * T) : (P + gam * P0) / ((gam - 1.0) * T);
    if (!(r > 0.0) || !isfinite(r)) r = rho[k];
    const double c2 = eos == SPH_EOS_IDEAL ? gam * (gam - 1.0) * T : gam * (P + P0) / r;
    const double c = c2 > 0.0 ? sqrt(c2) : 0.0;
    const double A = P / (om[k] * r * r);
    rho[k] = r;
    Ps[k] = P;
    cs[k] = c;
    As[k] = A;
    if (fr.rec1) {
        float4 *r2 = reinterpret_cast<float4 *>(fr.rec2);
        r2[k] = make_float4((float)(1.0 / fr.H[k]), (float)A, (float)c, (float)r);
    }
    if (fr.drec1) {
        double4 *r2 = reinterpret_cast<double4 *>(fr.drec2);
        r2[k] = make_double4(1.0 / fr.H[k], A, c, r);
    }
    const uint32_t i = perm[k];
    Pc[i] = P;
    cc[i] = c;
    if (imb_c) imb_c[i] = I;
    if (rho_c) rho_c[i] = r;
}

// Step size of every set: the given dt, else the set's smallest per-particle
// limit from its last force pass (independent sets keep independent steps).
__global__ void k_set_dt(double dt_in, double dt_max, const double *set_dtnext, int nsets,
                         double *d_dt, StepReport *rep) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsets) return;
    double dt = dt_in > 0.0 ? dt_in : fmin(set_dtnext[s], dt_max);
    d_dt[s] = dt;
    if (s == 0) rep->dt_used = dt;
}

__device__ inline long long dbits(double v) { return __double_as_longlong(v); }

__global__ void k_fill_f64(double *p, int n, double v) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Per-set minimum of dt (dt >= 0, so the bit patterns order like the values).
// Per-set minimum of the particle steps.  A block reduces 2048 consecutive
// particles; a block inside one set (the usual case) issues one atomic, a
// block across a set boundary one per particle.
constexpr int kMinItems = 8;

__global__ __launch_bounds__(kThreads) void k_set_min_dt(const double *__restrict__ dt, int64_t n,
                                                         const SetGeom *sets, int nsets,
                                                         double *set_min) {
    __shared__ double wmin[kThreads / 64];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kThreads * kMinItems;
    const int64_t end = base + (int64_t)kThreads * kMinItems < n ? base + (int64_t)kThreads * kMinItems : n;
    const int s0 = nsets == 1 ? 0 : find_set_k(sets, nsets, base);
    const bool one_set = nsets == 1 || end <= sets[s0].p1;
    long long *dst = reinterpret_cast<long long *>(set_min);
    if (one_set) {
        double v = DBL_MAX;
        for (int it = 0; it < kMinItems; ++it) {
            const int64_t i = base + (int64_t)it * kThreads + tid;
            if (i < end) v = fmin(v, dt[i]);
        }
        for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
        if ((tid & 63) == 0) wmin[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            for (int w = 1; w < kThreads / 64; ++w) v = fmin(v, wmin[w]);
            if (v < DBL_MAX) atomicMin(&dst[s0], dbits(v));
        }
    } else {
        for (int it = 0; it < kMinItems; ++it) {
            const int64_t i = base + (int64_t)it * kThreads + tid;
            if (i < end) atomicMin(&dst[find_set_k(sets, nsets, i)], dbits(dt[i]));
        }
    }
}

// Opening kick, predictor and drift in caller order (Sec. 2.3.6):
//   v_half = v + (dt/2) a,  u_half = u + (dt/2) du      (stored in v, u)
//   v_pred = v_half + (dt/2) a,  u_pred likewise          (scratch)
//   x     += dt v_half, wrapped into the periodic box
//   evolved density: rho_half = rho + (dt/2) drho (stored in rho),
//                    rho_pred = rho_half + (dt/2) drho (scratch)
struct KickArgs {
    double *x, *y, *z, *vx, *vy, *vz, *u;
    double *H, *Hprev;
    const double *ax, *ay, *az, *du;
    double *vpx, *vpy, *vpz, *up;
    double *rho, *rhop;          // evolved density only (else null)
    const double *drho;
    const SetGeom *sets;
    int nsets;
    int periodic;
    const double *dt;
    int64_t n;
};

__device__ __forceinline__ double wrap_box(double v, double lo, double L) {
#pragma clang fp contract(off)
    double t = floor((v - lo) / L);
    double s = L * t;
    return v - s;
}

__global__ void k_kick_drift(KickArgs a) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int sid = a.nsets == 1 ? 0 : find_set_k(a.sets, a.nsets, i);
    const double dt = a.dt[sid];
    const double hdt = 0.5 * dt;
    double ax = a.ax[i], ay = a.ay[i], az = a.az[i], du = a.du[i];
    double vhx = a.vx[i] + hdt * ax;
    double vhy = a.vy[i] + hdt * ay;
    double vhz = a.vz[i] + hdt * az;
    double uh = a.u[i] + hdt * du;
    a.vx[i] = vhx; a.vy[i] = vhy; a.vz[i] = vhz; a.u[i] = uh;
    a.vpx[i] = vhx + hdt * ax;
    a.vpy[i] = vhy + hdt * ay;
    a.vpz[i] = vhz + hdt * az;
    a.up[i] = uh + hdt * du;
    if (a.rho) {
        const double dr = a.drho[i];
        const double rh = a.rho[i] + hdt * dr;
        a.rho[i] = rh;
        a.rhop[i] = rh + hdt * dr;
    }
    double nx = a.x[i] + dt * vhx;
    double ny = a.y[i] + dt * vhy;
    double nz = a.z[i] + dt * vhz;
    if (a.periodic) {
        const SetGeom &g = a.sets[sid];
        nx = wrap_box(nx, g.lo[0], g.L[0]);
        ny = wrap_box(ny, g.lo[1], g.L[1]);
        nz = wrap_box(nz, g.lo[2], g.L[2]);
    }
    a.x[i] = nx; a.y[i] = ny; a.z[i] = nz;
    // First guess of the density pass's smoothing-length iteration: the
    // converged H extrapolated by its change over the last step (ratio held
    // to [0.95, 1.05]).  The iteration converges to the same root from any
    // guess; a closer guess saves a scan of the candidates (Sec. 2.3.3).
    const double Hn = a.H[i], Hp = a.Hprev[i];
    a.Hprev[i] = Hn;
    if (Hp > 0.0 && Hn > 0.0) a.H[i] = Hn * fmin(fmax(Hn / Hp, 0.95), 1.05);
}

// Closing kick: v = v_half + (dt/2) a_new, u likewise (and rho with the
// evolved density).
__global__ void k_closing_kick(int64_t n, const SetGeom *sets, int nsets,
                               const double *__restrict__ dtp, double *vx, double *vy,
                               double *vz, double *u, const double *__restrict__ ax,
                               const double *__restrict__ ay, const double *__restrict__ az,
                               const double *__restrict__ du, double *rho,
                               const double *__restrict__ drho) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hdt = 0.5 * dtp[nsets == 1 ? 0 : find_set_k(sets, nsets, i)];
    vx[i] = vx[i] + hdt * ax[i];
    vy[i] = vy[i] + hdt * ay[i];
    vz[i] = vz[i] + hdt * az[i];
    u[i] = u[i] + hdt * du[i];
    if (rho) rho[i] = rho[i] + hdt * drho[i];
}

// Entropy-conserving update (Sec. 2.3.5), after the density pass of a step:
// the half-step u moves along the adiabat from the last step's density to
// the new one, u(rho_new, s(rho_old, u)); ideal gas: u scales as
// rho^(gamma-1) (Springel & Hernquist 2002); stiffened gas: u - P0/rho does
// ((P + P0)/rho^gamma is its adiabatic invariant).  Then rho_old moves on and
// the prediction of u is redone from the new half-step value.
__global__ void k_isentrope(int64_t n, const SetGeom *sets, int nsets, const double *dtp,
                            int eos, double gam, double P0, double *u, double *rho_old,
                            const double *__restrict__ rho_new, const double *__restrict__ du,
                            double *up) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double hdt = 0.5 * dtp[nsets == 1 ? 0 : find_set_k(sets, nsets, i)];
    const double r0 = rho_old[i], r1 = rho_new[i];
    const double ratio = pow(r1 / r0, gam - 1.0);
    const double uh = eos == SPH_EOS_IDEAL ? u[i] * ratio : (u[i] - P0 / r0) * ratio + P0 / r1;
    u[i] = uh;
    up[i] = uh + hdt * du[i];
    rho_old[i] = r1;
}

__global__ void k_copy_f64(double *dst, const double *__restrict__ src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Deterministic two-stage FP64 reduction: fixed grid, fixed tree order.
__global__ __launch_bounds__(kThreads) void k_reduce_part(int64_t n, const double *__restrict__ m,
                                                          const double *__restrict__ vx,
                                                          const double *__restrict__ vy,
                                                          const double *__restrict__ vz,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ dt,
                                                          double *__restrict__ part) {
    __shared__ double sh[6][kThreads];
    double acc[5] = {0, 0, 0, 0, 0};
    double mn = DBL_MAX;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)kRedBlocks * kThreads) {
        double mm = m[i], a = vx[i], b = vy[i], c = vz[i];
        acc[0] += mm * a;
        acc[1] += mm * b;
        acc[2] += mm * c;
        acc[3] += 0.5 * mm * (a * a + b * b + c * c);
        acc[4] += mm * u[i];
        mn = fmin(mn, dt[i]);
    }
    for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] = acc[q];
    sh[5][threadIdx.x] = mn;
    __syncthreads();
    for (int st = kThreads / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
            sh[5][threadIdx.x] = fmin(sh[5][threadIdx.x], sh[5][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedBlocks) void k_reduce_final(const double *__restrict__ part,
                                                             double dt_max, StepReport *rep) {
    __shared__ double sh[6][kRedBlocks];
    for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] = part[threadIdx.x * 6 + q];
    __syncthreads();
    for (int st = kRedBlocks / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int q = 0; q < 5; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + st];
            sh[5][threadIdx.x] = fmin(sh[5][threadIdx.x], sh[5][threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rep->momentum[0] = sh[0][0];
        rep->momentum[1] = sh[1][0];
        rep->momentum[2] = sh[2][0];
        rep->e_kin = sh[3][0];
        rep->e_int = sh[4][0];
        rep->dt_next = fmin(sh[5][0], dt_max);
    }
}


// ---- individual time steps (Sec. 2.3.6) ---------------------------------------
// Time is counted in units of delta = dt_max 2^-R (R = rung_max); a particle
// on rung r steps L = 2^(R-r) units and its steps start at multiples of L.
// Caller order unless noted; the arithmetic follows the oracle's order.

__device__ __forceinline__ long long rung_step(double r, int R) {
    int k = (int)r;
    k = k < 0 ? 0 : (k > R ? R : k);
    return 1ll << (R - k);
}

// The smallest rung whose step dt_max 2^-r fits under dt; R when none does
// (NaN included).
__device__ __forceinline__ int desired_rung(double dt, double dt0, int R) {
    for (int k = 0; k <= R; ++k)
        if (dt >= ldexp(dt0, -k)) return k;
    return R;
}

// Opening kick of the particles at a step boundary, v_half = v + (L/2) delta a
// (u likewise), and the next step boundary of any particle (one atomic
// minimum per wave).
__global__ void k_rung_open(int64_t n, int R, double delta, RungState *rs,
                            const double *__restrict__ rung, double *vx, double *vy, double *vz,
                            double *u, const double *__restrict__ ax, const double *__restrict__ ay,
                            const double *__restrict__ az, const double *__restrict__ du) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long nxt = LLONG_MAX;
    if (i < n) {
        const long long T = rs->T;
        const long long L = rung_step(rung[i], R);
        if (T % L == 0) {
            const double h = 0.5 * (double)L * delta;
            vx[i] = vx[i] + h * ax[i];
            vy[i] = vy[i] + h * ay[i];
            vz[i] = vz[i] + h * az[i];
            u[i] = u[i] + h * du[i];
        }
        nxt = T - T % L + L;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const long long w = __shfl_xor(nxt, o);
        nxt = w < nxt ? w : nxt;
    }
    if ((threadIdx.x & 63) == 0 && nxt != LLONG_MAX)
        atomicMin(reinterpret_cast<unsigned long long *>(&rs->Tnext), (unsigned long long)nxt);
}

// Drift of every particle to the next boundary T', x += (T' - T) delta v
// (wrapped), and the prediction at T': v_pred = v + ((T' - Tb) - L/2) delta a
// with Tb the start of the particle's current step (u likewise).
__global__ void k_rung_drift(int64_t n, int R, double delta, const RungState *rs,
                             const double *__restrict__ rung, double *x, double *y, double *z,
                             const double *__restrict__ vx, const double *__restrict__ vy,
                             const double *__restrict__ vz, const double *__restrict__ u,
                             const double *__restrict__ ax, const double *__restrict__ ay,
                             const double *__restrict__ az, const double *__restrict__ du,
                             double *vpx, double *vpy, double *vpz, double *up, int periodic,
                             const SetGeom *sets) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long T = rs->T, Tn = rs->Tnext;
    const double dx = (double)(Tn - T) * delta;
    double nx = x[i] + dx * vx[i];
    double ny = y[i] + dx * vy[i];
    double nz = z[i] + dx * vz[i];
    if (periodic) {
        const SetGeom &g = sets[0];
        nx = wrap_box(nx, g.lo[0], g.L[0]);
        ny = wrap_box(ny, g.lo[1], g.L[1]);
        nz = wrap_box(nz, g.lo[2], g.L[2]);
    }
    x[i] = nx; y[i] = ny; z[i] = nz;
    const long long L = rung_step(rung[i], R);
    const long long Tb = (Tn % L == 0) ? Tn - L : Tn - Tn % L;
    const double cf = ((double)(Tn - Tb) - 0.5 * (double)L) * delta;
    vpx[i] = vx[i] + cf * ax[i];
    vpy[i] = vy[i] + cf * ay[i];
    vpz[i] = vz[i] + cf * az[i];
    up[i] = u[i] + cf * du[i];
}

// Sorted order: the active sinks (whose step ends at T') in ascending order.
__global__ void k_rung_flags(int64_t n, int R, const RungState *rs, const double *__restrict__ rungs,
                             int64_t *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) flags[k] = (rs->Tnext % rung_step(rungs[k], R) == 0) ? 1 : 0;
    else if (k == n) flags[k] = 0;
}
__global__ void k_rung_compact(int64_t n, int R, RungState *rs, const double *__restrict__ rungs,
                               const int64_t *__restrict__ offs, uint32_t *sinks) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && rs->Tnext % rung_step(rungs[k], R) == 0) sinks[offs[k]] = (uint32_t)k;
    if (k == n) rs->nact = offs[n];
}

// FastGas: below fastgas n active particles the density sinks are the marked
// particles, else all of them.
__global__ void k_dens_flags(int64_t n, double thr, const RungState *rs,
                             const uint32_t *__restrict__ mark, int64_t *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool fg = (double)rs->nact < thr * (double)n;
    if (k < n) flags[k] = (!fg || mark[k]) ? 1 : 0;
    else if (k == n) flags[k] = 0;
}
__global__ void k_dens_compact(int64_t n, double thr, RungState *rs,
                               const uint32_t *__restrict__ mark, const int64_t *__restrict__ offs,
                               uint32_t *sinks) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool fg = (double)rs->nact < thr * (double)n;
    if (k < n && (!fg || mark[k])) sinks[offs[k]] = (uint32_t)k;
    if (k == n) rs->ndens = offs[n];
}

// Sorted order: rung | 256 for particles whose density is not of this substep.
__global__ void k_rung_pack(int64_t n, const double *__restrict__ rungs,
                            const uint32_t *__restrict__ mark, double thr, const RungState *rs,
                            int32_t *rpack) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    bool fresh = true;
    if (mark) fresh = !((double)rs->nact < thr * (double)n) || mark[k] != 0;
    rpack[k] = (int32_t)rungs[k] | (fresh ? 0 : 256);
}

// Closing kick of the active particles, v = v_half + (L/2) delta a_new (u
// likewise), then the new rung: desired, raised to max_{F_i} r_j - 2, capped at
// R, and when longer than the old step, the lowest rung whose step divides T'.
__global__ void k_rung_close(int64_t n, int R, double dt0, double delta, const RungState *rs,
                             double *rung, double *vx, double *vy, double *vz, double *u,
                             const double *__restrict__ ax, const double *__restrict__ ay,
                             const double *__restrict__ az, const double *__restrict__ du,
                             const double *__restrict__ dt, const double *__restrict__ nbmax) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long Tn = rs->Tnext;
    const long long L = rung_step(rung[i], R);
    if (Tn % L != 0) return;
    const double h = 0.5 * (double)L * delta;
    vx[i] = vx[i] + h * ax[i];
    vy[i] = vy[i] + h * ay[i];
    vz[i] = vz[i] + h * az[i];
    u[i] = u[i] + h * du[i];
    const int r_old = (int)rung[i];
    int r = desired_rung(dt[i], dt0, R);
    const int lim = (int)nbmax[i] - 2;
    r = r > lim ? r : lim;
    r = r < R ? r : R;
    if (r < r_old)
        while (Tn % rung_step((double)r, R) != 0) ++r;
    rung[i] = (double)r;
}

// End of a substep: its length into the report, T = T', next boundary unset.
__global__ void k_rung_finish(RungState *rs, double delta, StepReport *rep) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    rep->dt_used = (double)(rs->Tnext - rs->T) * delta;
    rs->T = rs->Tnext;
    rs->Tnext = LLONG_MAX;
}

// Initial rungs: desired ones, then the limiter against the neighbours'
// desired rungs (nbmax from a force pass over the desired rungs).
__global__ void k_rung_desired(int64_t n, int R, double dt0, const double *__restrict__ dt,
                               double *rung) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rung[i] = (double)desired_rung(dt[i], dt0, R);
}
__global__ void k_rung_limit_init(int64_t n, int R, double dt0, const double *__restrict__ dt,
                                  const double *__restrict__ nbmax, double *rung) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = desired_rung(dt[i], dt0, R);
    const int lim = (int)nbmax[i] - 2;
    r = r > lim ? r : lim;
    rung[i] = (double)(r < R ? r : R);
}

// Sorted-order columns of the listed sinks into caller order.
__global__ void k_scatter_sinks(const uint32_t *__restrict__ perm, const uint32_t *__restrict__ sinks,
                                const long long *__restrict__ nsinks, Cols c) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *nsinks) return;
    const uint32_t i = sinks[k];
    const uint32_t o = perm[i];
    for (int q = 0; q < kMaxCols; ++q)
        if (q < c.n) c.dst[q][o] = c.src[q][i];
}
}  // namespace

int reduce_partials() { return kRedBlocks; }

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<nblk(n, kThreads), kThreads, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_reset_counters(Ctx *c, int last, hipStream_t s) {
    k_reset_counters<<<1, kCntShards * kCntStride, 0, s>>>(c->d_cnt, last);
    return hipGetLastError();
}

hipError_t launch_fold_counters(Ctx *c, hipStream_t s) {
    k_fold_counters<<<1, kCntStride, 0, s>>>(c->d_cnt, c->d_csum);
    return hipGetLastError();
}

hipError_t launch_gather(Ctx *c, const Cols &cols, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_gather_cols<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->d_perm[0], c->n, cols);
    return hipGetLastError();
}

hipError_t launch_scatter(Ctx *c, const Cols &cols, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_scatter_cols<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->d_perm[0], c->n, cols);
    return hipGetLastError();
}

hipError_t launch_eos(Ctx *c, const double *u_sorted, double *P_caller, double *c_caller,
                      hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    ForceRecords fr{c->ms, c->Hs, c->vxs, c->vys, c->vzs, c->frec1, c->frec2, c->fm,
                    c->drec1, c->drec2};
    k_eos<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->d_perm[0], c->n, c->prm.eos, c->prm.gamma,
                                                    c->prm.P0, c->rhos, u_sorted, c->oms, c->Ps,
                                                    c->css, c->As, P_caller, c_caller, fr);
    return hipGetLastError();
}

hipError_t launch_ic_correct(Ctx *c, double *P_caller, double *c_caller, double *imb_caller,
                             double *rho_caller, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    ForceRecords fr{c->ms, c->Hs, c->vxs, c->vys, c->vzs, c->frec1, c->frec2, c->fm,
                    c->drec1, c->drec2};
    k_ic_correct<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->d_perm[0], c->n, c->prm.eos, c->prm.gamma, c->prm.P0, c->rhos, c->us, c->oms, c->Ps,
        c->css, c->As, c->imbs, c->tbar, c->pbar, P_caller, c_caller, imb_caller, rho_caller, fr);
    return hipGetLastError();
}

hipError_t launch_set_dt(Ctx *c, double dt, hipStream_t s) {
    k_set_dt<<<nblk(c->nsets, 64), 64, 0, s>>>(dt, c->prm.dt_max, c->d_set_dtnext, c->nsets,
                                                c->d_dt, c->d_rep);
    return hipGetLastError();
}

hipError_t launch_set_dtnext(Ctx *c, const sph_particles *p, hipStream_t s) {
    k_fill_f64<<<nblk(c->nsets, 64), 64, 0, s>>>(c->d_set_dtnext, c->nsets, c->prm.dt_max);
    if (c->n > 0)
        k_set_min_dt<<<nblk(c->n, kThreads * kMinItems), kThreads, 0, s>>>(
            p->dt, c->n, c->d_sets, c->nsets, c->d_set_dtnext);
    return hipGetLastError();
}

hipError_t launch_kick_drift(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    KickArgs a;
    a.x = p->x; a.y = p->y; a.z = p->z; a.vx = p->vx; a.vy = p->vy; a.vz = p->vz; a.u = p->u;
    a.H = p->H; a.Hprev = c->hprev;
    a.ax = p->ax; a.ay = p->ay; a.az = p->az; a.du = p->dudt;
    a.vpx = c->vpx; a.vpy = c->vpy; a.vpz = c->vpz; a.up = c->upred;
    const bool evolved = (c->prm.flags & SPH_FLAG_EVOLVED) != 0;
    a.rho = evolved ? p->rho : nullptr;
    a.rhop = evolved ? c->rho_pred : nullptr;
    a.drho = evolved ? p->drhodt : nullptr;
    a.sets = c->d_sets; a.nsets = c->nsets; a.periodic = c->prm.periodic;
    a.dt = c->d_dt; a.n = c->n;
    k_kick_drift<<<nblk(c->n, kThreads), kThreads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_closing_kick(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    const bool evolved = (c->prm.flags & SPH_FLAG_EVOLVED) != 0;
    k_closing_kick<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->d_sets, c->nsets, c->d_dt, p->vx, p->vy, p->vz, p->u, p->ax, p->ay, p->az,
        p->dudt, evolved ? p->rho : nullptr, evolved ? p->drhodt : nullptr);
    return hipGetLastError();
}

hipError_t launch_isentrope(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_isentrope<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->d_sets, c->nsets, c->d_dt, c->prm.eos, c->prm.gamma, c->prm.P0, p->u,
        c->rho_old, p->rho, p->dudt, c->upred);
    return hipGetLastError();
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_copy_f64<<<nblk(n, kThreads), kThreads, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

hipError_t launch_reduce(Ctx *c, const sph_particles *p, hipStream_t s) {
    k_reduce_part<<<kRedBlocks, kThreads, 0, s>>>(c->n, p->m, p->vx, p->vy, p->vz, p->u, p->dt,
                                                   c->d_part);
    k_reduce_final<<<1, kRedBlocks, 0, s>>>(c->d_part, c->prm.dt_max, c->d_rep);
    return hipGetLastError();
}


// ---- individual time steps: launchers ------------------------------------------

namespace {
inline double rung_delta(const Ctx *c) { return ldexp(c->prm.dt_max, -c->prm.rung_max); }
}  // namespace

hipError_t launch_rung_open(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_open<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->prm.rung_max, rung_delta(c), c->d_rung, p->rung, p->vx, p->vy, p->vz, p->u,
        p->ax, p->ay, p->az, p->dudt);
    return hipGetLastError();
}

hipError_t launch_rung_drift(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_drift<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->prm.rung_max, rung_delta(c), c->d_rung, p->rung, p->x, p->y, p->z, p->vx, p->vy,
        p->vz, p->u, p->ax, p->ay, p->az, p->dudt, c->vpx, c->vpy, c->vpz, c->upred,
        c->prm.periodic, c->d_sets);
    return hipGetLastError();
}

hipError_t launch_rung_lists(Ctx *c, bool fastgas, hipStream_t s) {
    (void)fastgas;
    const int64_t n = c->n;
    k_rung_flags<<<nblk(n + 1, kThreads), kThreads, 0, s>>>(n, c->prm.rung_max, c->d_rung,
                                                           c->rungs, c->rflags);
    hipError_t e = launch_scan_i64(c, c->rflags, c->rflags, n + 1, s);
    if (e != hipSuccess) return e;
    k_rung_compact<<<nblk(n + 1, kThreads), kThreads, 0, s>>>(n, c->prm.rung_max, c->d_rung,
                                                             c->rungs, c->rflags, c->sinks);
    return hipGetLastError();
}

hipError_t launch_rung_dens_list(Ctx *c, hipStream_t s) {
    const int64_t n = c->n;
    k_dens_flags<<<nblk(n + 1, kThreads), kThreads, 0, s>>>(n, c->prm.fastgas, c->d_rung, c->mark,
                                                           c->rflags);
    hipError_t e = launch_scan_i64(c, c->rflags, c->rflags, n + 1, s);
    if (e != hipSuccess) return e;
    k_dens_compact<<<nblk(n + 1, kThreads), kThreads, 0, s>>>(n, c->prm.fastgas, c->d_rung,
                                                             c->mark, c->rflags, c->dsinks);
    return hipGetLastError();
}

hipError_t launch_rung_pack(Ctx *c, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    const bool fg = c->prm.fastgas > 0.0 && c->mark;
    k_rung_pack<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->n, c->rungs, fg ? c->mark : nullptr,
                                                         c->prm.fastgas, c->d_rung, c->rpack);
    return hipGetLastError();
}

hipError_t launch_rung_close(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_close<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->prm.rung_max, c->prm.dt_max, rung_delta(c), c->d_rung, p->rung, p->vx, p->vy,
        p->vz, p->u, p->ax, p->ay, p->az, p->dudt, p->dt, c->nbmax_c);
    return hipGetLastError();
}

hipError_t launch_rung_finish(Ctx *c, hipStream_t s) {
    k_rung_finish<<<1, 64, 0, s>>>(c->d_rung, rung_delta(c), c->d_rep);
    return hipGetLastError();
}

hipError_t launch_rung_desired(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_desired<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->n, c->prm.rung_max,
                                                            c->prm.dt_max, p->dt, p->rung);
    return hipGetLastError();
}

hipError_t launch_rung_limit_init(Ctx *c, sph_particles *p, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_limit_init<<<nblk(c->n, kThreads), kThreads, 0, s>>>(
        c->n, c->prm.rung_max, c->prm.dt_max, p->dt, c->nbmax_c, p->rung);
    return hipGetLastError();
}

hipError_t launch_rung_pack_init(Ctx *c, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    k_rung_pack<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->n, c->rungs, nullptr, 0.0, c->d_rung,
                                                         c->rpack);
    return hipGetLastError();
}

hipError_t launch_scatter_sinks(Ctx *c, const Cols &cols, hipStream_t s) {
    if (c->n == 0) return hipSuccess;
    const long long *nact = reinterpret_cast<const long long *>(
        reinterpret_cast<const char *>(c->d_rung) + offsetof(RungState, nact));
    k_scatter_sinks<<<nblk(c->n, kThreads), kThreads, 0, s>>>(c->d_perm[0], c->sinks, nact, cols);
    return hipGetLastError();
}

}  // namespace sphmi

// sph_tree.hip -- tree build over particle buckets (Sec. 2.1: storage reordered
// so each cell is a contiguous range; Sec. 2.3.2 and Fig. 1: cell bound,
// box-of-balls and ball-of-balls combined bottom-up).
//
// MI355X design: instead of a top-down recursive bisection, particles are
// ordered along a Hilbert curve (10 bits per axis, set id in the high bits) by
// a hand-written stable LSD radix sort, cut into buckets of B consecutive
// particles, and an implicit binary tree (heap layout) is laid over the
// buckets of each set.  Fixed-size runs of a space-filling order are compact
// only if the curve has no long jumps: on a Morton curve a run that crosses
// the boundary of a large octant spans far-apart regions, and once particles
// drift off their lattice cells most runs are unaligned.  Consecutive Hilbert
// cells always share a face, so every bucket and every sink group stays a
// connected, compact region.  Every node is then a contiguous particle range, as in
// the paper, and bounds are combined level by level with one launch per
// tree height across all sets (the small top heights in one launch).
// 10 bits per axis give 2^30 cells per set, far more than particles even at
// 10^8 per set, so cells shared by two particles are rare and harmless (their
// order is the caller's); the 30-bit keys sort in 4 radix passes instead of 6.
#include "sph_internal.h"

#include <cfloat>

namespace sphmi {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kKeyBits = 10;

__device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Hilbert index of a cell with integer coordinates X[0..2] (kKeyBits each),
// after J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707
// (2004): the coordinates are transformed in place into the "transposed"
// index (bit j of X[0], X[1], X[2] are the index bits 3j+2, 3j+1, 3j), which
// is then interleaved.
__device__ inline uint64_t hilbert_key(uint32_t X[3]) {
    for (uint32_t Q = 1u << (kKeyBits - 1); Q > 1u; Q >>= 1) {
        const uint32_t P = Q - 1u;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                       // invert the low bits of X[0]
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;   // swap low bits of X[0], X[i]
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];                                // Gray encode
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = 1u << (kKeyBits - 1); Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    return (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
}

__device__ inline int find_set(const SetGeom *sets, int nsets, int64_t i) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sets[mid].p0 <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Order-preserving map of a double to a signed 64-bit integer (for min/max atomics).
__device__ inline long long dkey(double v) {
    long long b = __double_as_longlong(v);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffll);
}
__device__ inline double dval(long long k) {
    long long b = k >= 0 ? k : (k ^ 0x7fffffffffffffffll);
    return __longlong_as_double(b);
}

__global__ void k_bbox_init(long long *enc, int nsets) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nsets * 6) enc[t] = (t % 6) < 3 ? LLONG_MAX : LLONG_MIN;
}

// Open boundary: the key box of each set is the bounding box of its particles.
// A block reduces kBoxItems x 256 consecutive particles; a block inside one set
// (the usual case) issues one atomic per bound, a block across a set boundary
// one per particle and bound.
constexpr int kBoxItems = 16;

__global__ __launch_bounds__(256) void k_bbox(const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z, int64_t n,
                                              const SetGeom *sets, int nsets, long long *enc) {
    __shared__ double red[6][4];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 256 * kBoxItems;
    const int64_t end = base + 256 * kBoxItems < n ? base + 256 * kBoxItems : n;
    const int s0 = nsets == 1 ? 0 : find_set(sets, nsets, base);
    const bool one_set = nsets == 1 || end <= sets[s0].p1;
    if (one_set) {
        double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
        for (int it = 0; it < kBoxItems; ++it) {
            const int64_t i = base + (int64_t)it * 256 + tid;
            if (i < end) {
                const double v[3] = {x[i], y[i], z[i]};
                for (int a = 0; a < 3; ++a) { mn[a] = fmin(mn[a], v[a]); mx[a] = fmax(mx[a], v[a]); }
            }
        }
        for (int a = 0; a < 3; ++a) {
            for (int o = 32; o > 0; o >>= 1) {
                mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
                mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
            }
        }
        if ((tid & 63) == 0) {
            for (int a = 0; a < 3; ++a) { red[a][tid >> 6] = mn[a]; red[3 + a][tid >> 6] = mx[a]; }
        }
        __syncthreads();
        if (tid < 6) {
            double r = red[tid][0];
            for (int w = 1; w < 4; ++w) r = tid < 3 ? fmin(r, red[tid][w]) : fmax(r, red[tid][w]);
            if (tid < 3) atomicMin(&enc[s0 * 6 + tid], dkey(r));
            else atomicMax(&enc[s0 * 6 + tid], dkey(r));
        }
    } else {
        for (int it = 0; it < kBoxItems; ++it) {
            const int64_t i = base + (int64_t)it * 256 + tid;
            if (i < end) {
                const int s = find_set(sets, nsets, i);
                const double v[3] = {x[i], y[i], z[i]};
                for (int a = 0; a < 3; ++a) {
                    atomicMin(&enc[s * 6 + a], dkey(v[a]));
                    atomicMax(&enc[s * 6 + 3 + a], dkey(v[a]));
                }
            }
        }
    }
}

// Open-boundary key boxes into the per-set geometry (padded so the extreme
// particles map inside the key range).
__global__ void k_bbox_finish(const long long *enc, SetGeom *sets, int nsets) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsets) return;
    for (int a = 0; a < 3; ++a) {
        double lo = dval(enc[s * 6 + a]), hi = dval(enc[s * 6 + 3 + a]);
        if (!(hi >= lo)) { lo = 0.0; hi = 1.0; }
        double pad = 1e-9 * (fabs(lo) + fabs(hi)) + 1e-300;
        lo -= pad; hi += pad;
        double L = hi - lo;
        if (!(L > 0)) L = 1.0;
        sets[s].lo[a] = lo;
        sets[s].L[a] = L;
        sets[s].halfL[a] = 0.5 * L;
    }
}

__global__ void k_sfc_keys(const double *__restrict__ x, const double *__restrict__ y,
                         const double *__restrict__ z, int64_t n, const SetGeom *sets, int nsets,
                         uint64_t *keys, uint32_t *perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int s = nsets == 1 ? 0 : find_set(sets, nsets, i);
    const SetGeom &g = sets[s];
    double v[3] = {x[i], y[i], z[i]};
    uint32_t X[3];
    const double scale = (double)(1u << kKeyBits);
    for (int a = 0; a < 3; ++a) {
        double t = floor((v[a] - g.lo[a]) / g.L[a] * scale);
        if (!(t >= 0.0)) t = 0.0;
        if (t > scale - 1.0) t = scale - 1.0;
        X[a] = (uint32_t)t;
    }
    keys[i] = ((uint64_t)s << (3 * kKeyBits)) | hilbert_key(X);
    perm[i] = (uint32_t)i;
}

// ---- stable LSD radix sort, 8-bit digits -------------------------------------

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                             int64_t n, int shift, int64_t nblk,
                                                             int64_t *__restrict__ hist) {
    __shared__ unsigned int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + (int64_t)it * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, int64_t nblk, const int64_t *__restrict__ offs) {
    __shared__ unsigned int run[256];
    __shared__ unsigned int wcnt[kSortThreads / kWave][256];
    __shared__ int64_t goff[256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    run[tid] = 0;
    goff[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    for (int q = 0; q < kSortThreads / kWave; ++q) wcnt[q][tid] = 0;
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        int64_t i = base + (int64_t)it * kSortThreads + tid;
        bool ok = i < n;
        uint64_t k = ok ? kin[i] : 0;
        uint32_t v = ok ? vin[i] : 0;
        unsigned d = ok ? (unsigned)((k >> shift) & 255u) : 0u;
        // lanes holding the same digit
        uint64_t same = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? bal : ~bal;
        }
        unsigned rank = (unsigned)__popcll(same & lt);
        if (ok && rank == 0) wcnt[w][d] = (unsigned)__popcll(same);
        __syncthreads();
        if (ok) {
            unsigned pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            int64_t dst = goff[d] + pos;
            kout[dst] = k;
            vout[dst] = v;
        }
        __syncthreads();
        unsigned add = 0;
        for (int q = 0; q < kSortThreads / kWave; ++q) { add += wcnt[q][tid]; wcnt[q][tid] = 0; }
        run[tid] += add;
        __syncthreads();
    }
}

// ---- exclusive scan of int64 ----------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int64_t wave_incl_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total in *tot.
template <int NT>
__device__ inline int64_t block_excl_scan(int64_t v, int64_t *tot) {
    __shared__ int64_t wsum[NT / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int64_t off = 0, all = 0;
    for (int q = 0; q < NT / 64; ++q) {
        if (q < w) off += wsum[q];
        all += wsum[q];
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(const int64_t *__restrict__ in,
                                                              int64_t *__restrict__ out, int64_t n,
                                                              int64_t *__restrict__ bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t off = block_excl_scan<kScanThreads>(s, &tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_single(int64_t *__restrict__ v, int64_t n) {
    int64_t carry = 0;
    for (int64_t b = 0; b < n; b += 1024) {
        int64_t i = b + threadIdx.x;
        int64_t x = i < n ? v[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan<1024>(x, &tot);
        if (i < n) v[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int64_t *__restrict__ out, int64_t n,
                                                           const int64_t *__restrict__ bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t add = bsum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) out[base + k] += add;
}

// ---- gather into sorted order ---------------------------------------------

__global__ void k_gather(const uint32_t *__restrict__ perm, int64_t n, const double *__restrict__ x,
                         const double *__restrict__ y, const double *__restrict__ z,
                         const double *__restrict__ m, const double *__restrict__ H,
                         double *__restrict__ xs, double *__restrict__ ys, double *__restrict__ zs,
                         double *__restrict__ ms, double *__restrict__ Hs) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
    xs[k] = x[i]; ys[k] = y[i]; zs[k] = z[i]; ms[k] = m[i]; Hs[k] = H[i];
}

// ---- bounds ----------------------------------------------------------------

__device__ inline void node_empty(Node &o) {
    for (int a = 0; a < 3; ++a) {
        o.clo[a] = DBL_MAX; o.chi[a] = -DBL_MAX;
        o.blo[a] = DBL_MAX; o.bhi[a] = -DBL_MAX;
        o.bc[a] = 0.0;
    }
    o.br = -1.0;
}

__global__ void k_nodes_empty(Node *nodes, int64_t nn) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nn) node_empty(nodes[t]);
}

// Leaf bounds, one lane per particle: the B lanes of a bucket form an aligned
// segment of the wave (B divides 64, B >= 8) and reduce the cell bound, the
// box of the balls and the enclosing sphere inside it (segment reductions:
// DPP moves inside each row of 16 lanes, lane shuffles across rows).
__global__ __launch_bounds__(256) void k_leaf_bounds(const SetGeom *__restrict__ sets,
                                                     const int32_t *__restrict__ bkt_set,
                                                     int64_t nbk, int B,
                                                     const double *__restrict__ xs,
                                                     const double *__restrict__ ys,
                                                     const double *__restrict__ zs,
                                                     const double *__restrict__ Hs,
                                                     Node *__restrict__ nodes) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = t / B;
    const int off = (int)(t - b * B);
    const bool inb = b < nbk;
    const int s = inb ? bkt_set[b] : 0;
    const SetGeom &g = sets[s];
    const int64_t lb = b - g.b0;
    const int64_t k = g.p0 + lb * B + off;
    const bool act = inb && k < g.p1;
    double v[3] = {0.0, 0.0, 0.0}, H = 0.0;
    if (act) { v[0] = xs[k]; v[1] = ys[k]; v[2] = zs[k]; H = Hs[k]; }
    double clo[3], chi[3], blo[3], bhi[3];
    for (int a = 0; a < 3; ++a) {
        clo[a] = act ? v[a] : DBL_MAX;
        chi[a] = act ? v[a] : -DBL_MAX;
        blo[a] = act ? v[a] - H : DBL_MAX;
        bhi[a] = act ? v[a] + H : -DBL_MAX;
    }
    for (int a = 0; a < 3; ++a) {
        clo[a] = seg_reduce<false>(clo[a], B);
        chi[a] = seg_reduce<true>(chi[a], B);
        blo[a] = seg_reduce<false>(blo[a], B);
        bhi[a] = seg_reduce<true>(bhi[a], B);
    }
    double c[3];
    for (int a = 0; a < 3; ++a) c[a] = 0.5 * (clo[a] + chi[a]);
    double R = -1.0;
    if (act) {
        const double dx = v[0] - c[0], dy = v[1] - c[1], dz = v[2] - c[2];
        R = sqrt(dx * dx + dy * dy + dz * dz) + H;
    }
    R = seg_reduce<true>(R, B);
    if (inb && off == 0) {
        Node o;
        for (int a = 0; a < 3; ++a) {
            o.clo[a] = clo[a]; o.chi[a] = chi[a];
            o.blo[a] = blo[a]; o.bhi[a] = bhi[a];
            o.bc[a] = R >= 0.0 ? c[a] : 0.0;
        }
        o.br = R >= 0.0 ? R * (1.0 + 1e-12) : -1.0;
        nodes[g.node0 + g.nbp + lb] = o;
    }
}

// Smallest sphere enclosing two spheres (not required to be minimal for a
// node; combining pairwise is what the paper does, Fig. 1 centre).
__device__ inline void ball_union(const double *c1, double r1, const double *c2, double r2,
                                  double *c, double *r) {
    if (r1 < 0) { for (int a = 0; a < 3; ++a) c[a] = c2[a]; *r = r2; return; }
    if (r2 < 0) { for (int a = 0; a < 3; ++a) c[a] = c1[a]; *r = r1; return; }
    double d[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dist + r2 <= r1) { for (int a = 0; a < 3; ++a) c[a] = c1[a]; *r = r1; return; }
    if (dist + r1 <= r2) { for (int a = 0; a < 3; ++a) c[a] = c2[a]; *r = r2; return; }
    double R = 0.5 * (dist + r1 + r2);
    double t = (R - r1) / dist;
    for (int a = 0; a < 3; ++a) c[a] = c1[a] + t * d[a];
    // cover the rounding of the centre
    *r = R * (1.0 + 1e-12) + 1e-12 * (fabs(c[0]) + fabs(c[1]) + fabs(c[2]));
}

// A node's bounds from its two children's.
__device__ __forceinline__ void combine_nodes(const Node &a, const Node &b, Node &o) {
    for (int q = 0; q < 3; ++q) {
        o.clo[q] = fmin(a.clo[q], b.clo[q]); o.chi[q] = fmax(a.chi[q], b.chi[q]);
        o.blo[q] = fmin(a.blo[q], b.blo[q]); o.bhi[q] = fmax(a.bhi[q], b.bhi[q]);
    }
    ball_union(a.bc, a.br, b.bc, b.br, o.bc, &o.br);
}

// The set holding node t of a height whose per-set node counts have the
// prefix pref (t counts the nodes of that height over all sets, in set order).
__device__ __forceinline__ int set_of_node(const int64_t *__restrict__ pref, int nsets, int64_t t) {
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Node t of height d from its two children.
__device__ __forceinline__ void combine_one(const SetGeom *__restrict__ sets, int nsets,
                                            const int64_t *__restrict__ pref, int64_t t, int d,
                                            Node *__restrict__ nodes) {
    const int lo = set_of_node(pref, nsets, t);
    const SetGeom &g = sets[lo];
    int64_t h = (int64_t)(g.nbp >> d) + (t - pref[lo]);
    Node o;
    combine_nodes(nodes[g.node0 + 2 * h], nodes[g.node0 + 2 * h + 1], o);
    nodes[g.node0 + h] = o;
}

__global__ void k_combine(const SetGeom *__restrict__ sets, int nsets,
                          const int64_t *__restrict__ pref, int64_t total, int d,
                          Node *__restrict__ nodes) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) combine_one(sets, nsets, pref, t, d, nodes);
}

// The small top heights d0..d1 (at most kTopThreads nodes each) in one
// workgroup, one thread per node, height after height, instead of one launch
// per height.  Each height's nodes stay in LDS (in the order of t) for the
// next one, so only height d0 reads its children from global memory (a round
// trip per height otherwise: 36 us for the eleven top heights at 2M).
constexpr int kTopThreads = 512;
__global__ __launch_bounds__(kTopThreads) void k_combine_top(const SetGeom *__restrict__ sets,
                                                             int nsets,
                                                             const int64_t *__restrict__ pref_all,
                                                             int d0, int d1, Node *__restrict__ nodes) {
    __shared__ Node lv[kTopThreads];   // 64 KiB
    const int64_t t = threadIdx.x;
    for (int d = d0; d <= d1; ++d) {
        const int64_t *pref = pref_all + (int64_t)d * (nsets + 1);
        const bool have = t < pref[nsets];
        Node o;
        if (have) {
            const int lo = set_of_node(pref, nsets, t);
            const SetGeom &g = sets[lo];
            const int64_t j = t - pref[lo];
            const int64_t h = (int64_t)(g.nbp >> d) + j;
            if (d == d0) {
                combine_nodes(nodes[g.node0 + 2 * h], nodes[g.node0 + 2 * h + 1], o);
            } else {
                // the children: nodes 2j and 2j + 1 of this set at height d - 1
                const int64_t c = pref_all[(int64_t)(d - 1) * (nsets + 1) + lo] + 2 * j;
                combine_nodes(lv[c], lv[c + 1], o);
            }
            nodes[g.node0 + h] = o;
        }
        __syncthreads();   // (every read of height d - 1 is done)
        if (have) lv[t] = o;
        __syncthreads();
    }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_scan_i64(Ctx *c, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (c->scan_tmp_len < nb) return hipErrorInvalidValue;
    k_scan_blocks<<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, c->d_scan_tmp);
    k_scan_single<<<1, 1024, 0, s>>>(c->d_scan_tmp, nb);
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, s>>>(out, n, c->d_scan_tmp);
    return hipGetLastError();
}

int64_t scan_tmp_needed(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }
int64_t sort_blocks_needed(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
int key_bits_per_axis() { return kKeyBits; }

hipError_t launch_init_nodes(Ctx *c, hipStream_t s) {
    k_nodes_empty<<<nblk(c->nnodes, 256), 256, 0, s>>>(c->nodes, c->nnodes);
    return hipGetLastError();
}

hipError_t launch_refit(Ctx *c, hipStream_t s) {
    if (c->nbuckets == 0) return hipSuccess;
    k_leaf_bounds<<<nblk(c->nbuckets * c->bucket, 256), 256, 0, s>>>(
        c->d_sets, c->d_bkt_set, c->nbuckets, c->bucket, c->xs, c->ys, c->zs, c->Hs, c->nodes);
    int d = 1;
    for (; d <= c->max_depth && c->level_total[d] > kTopThreads; ++d)
        k_combine<<<nblk(c->level_total[d], 128), 128, 0, s>>>(
            c->d_sets, c->nsets, c->d_level_pref + (int64_t)d * (c->nsets + 1), c->level_total[d],
            d, c->nodes);
    if (d <= c->max_depth)
        k_combine_top<<<1, kTopThreads, 0, s>>>(c->d_sets, c->nsets, c->d_level_pref, d,
                                                c->max_depth, c->nodes);
    return hipGetLastError();
}

hipError_t launch_tree_build(Ctx *c, const sph_particles *p, hipStream_t s) {
    const int64_t n = c->n;
    mark(c, E_TREE0, s);
    if (!c->prm.periodic) {
        long long *enc = reinterpret_cast<long long *>(c->d_bbox);
        k_bbox_init<<<nblk(6 * c->nsets, 256), 256, 0, s>>>(enc, c->nsets);
        if (n > 0)
            k_bbox<<<nblk(n, 256 * kBoxItems), 256, 0, s>>>(p->x, p->y, p->z, n, c->d_sets,
                                                            c->nsets, enc);
        k_bbox_finish<<<nblk(c->nsets, 64), 64, 0, s>>>(enc, c->d_sets, c->nsets);
    }
    k_sfc_keys<<<nblk(n, 256), 256, 0, s>>>(p->x, p->y, p->z, n, c->d_sets, c->nsets, c->d_key[0],
                                          c->d_perm[0]);
    int cur = 0;
    const int64_t nb = c->sort_blocks;
    for (int pass = 0; pass < c->key_passes; ++pass) {
        int shift = 8 * pass;
        k_radix_hist<<<(unsigned)nb, kSortThreads, 0, s>>>(c->d_key[cur], n, shift, nb,
                                                           reinterpret_cast<int64_t *>(c->d_hist));
        hipError_t e = launch_scan_i64(c, reinterpret_cast<int64_t *>(c->d_hist),
                                       reinterpret_cast<int64_t *>(c->d_hist), 256 * nb, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<(unsigned)nb, kSortThreads, 0, s>>>(
            c->d_key[cur], c->d_perm[cur], c->d_key[cur ^ 1], c->d_perm[cur ^ 1], n, shift, nb,
            reinterpret_cast<const int64_t *>(c->d_hist));
        cur ^= 1;
    }
    if (cur != 0) {
        hipError_t e = hipMemcpyAsync(c->d_perm[0], c->d_perm[1], sizeof(uint32_t) * n,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    k_gather<<<nblk(n, 256), 256, 0, s>>>(c->d_perm[0], n, p->x, p->y, p->z, p->m, p->H, c->xs,
                                          c->ys, c->zs, c->ms, c->Hs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_refit(c, s);
    mark(c, E_TREE1, s);
    return e;
}

}  // namespace sphmi

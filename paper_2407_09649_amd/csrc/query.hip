// query.hip -- distance, gradient and variance of the L-GPDF at query points.
//
// Per (query, cluster) pair (Sec. III-A):
//   o      = sum_i alpha_i k(|x - x_i|)                     Eq. (1)
//   u      = 1 - |W k|^2, W = L^{-1}                         Eq. (2), minus sign
//   d      = r(o_c), o_c = clamp(o, occ_min, occ_max)        Eq. (3), footnote 1
//   v      = Lambda^2 u, Lambda = dr/do at o_c               Eq. (4)
//   grad d = Lambda grad o                                   Eq. (5) + chain rule
// combined over the selected clusters by the smooth minimum of Eq. (10)
// (weights exp(-lambda (d_q - d_min))) or the closest node, and signed from
// the sensor origin by the side of the nearest training point.
//
// Layout of the work: queries are grouped by cell (the cluster cell they fall
// in), so that all lanes of a wavefront share one neighbour list.  One lane
// evaluates one query; cluster points, alpha and W are wave-uniform and come
// through scalar loads.  The kernel vector k of a pair stays in VGPRs
// (compile-time unrolled size classes n <= 8, 16, 32); larger clusters
// stream W in 32-row panels and recompute the kernel values left of each
// panel's diagonal block.  The same kernels are instantiated in FP32 (the
// product path) and FP64.  FP32 results carry a running first-order error
// estimate; queries whose estimate exceeds the tolerance are regrouped by
// cell and re-evaluated by the FP64 instance.
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <utility>

namespace gpdf {

namespace {

constexpr int kQT = 256;            // threads per workgroup of the helper kernels
// evaluation kernels: one wavefront per workgroup, so that a finished
// wavefront's slot is refilled at once (waves of one workgroup end at
// different times)
constexpr int kEvalT = 64;
constexpr int kWaves = kEvalT / 64;
constexpr int kListStride = kCellListStride;
// combination variants, fixed per launch: smooth minimum with the weighted
// gradient, smooth minimum with the plain gradient mean, closest node
constexpr int kModeSmooth = 0, kModeMean = 1, kModeHard = 2;
constexpr int kMaxKnn = 16;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kEps = 5.9604645e-08f;  // 2^-24

inline unsigned blocks_for(int64_t n, int t = kQT) {
    int64_t g = (n + t - 1) / t;
    return unsigned(g < 1 ? 1 : g);
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// The template argument KERN carries the kernel (GPDF_KERNEL_*) and, in the
// bit kNoGrad, that the call asked for no gradient: the FP32 instances then
// leave out the gradient sums, its reverting and its error estimate.
constexpr int kNoGrad = 8;
// the bit kProp: the model carries a surface property and the call asks for
// it (Eq. (6)): one more product k . beta per point and its combination
constexpr int kProp = 16;
constexpr int kern_kind(int k) { return k & 7; }
constexpr bool kern_grad(int k) { return (k & kNoGrad) == 0; }
constexpr bool kern_prop(int k) { return (k & kProp) != 0; }

// Data that no kernel of a launch writes (model arrays, cell lists, chunk
// table, counts) is read through the constant address space.  That tells
// the compiler that no store of the kernel can change it, so its uniform
// loads stay scalar loads also inside loops that store (the persistent
// instances), where it could not otherwise prove it.
// Vector types are read component by component (their copy constructors
// cannot bind to the constant address space); the compiler merges the
// components back into one wide load.
template <typename T>
using ro_ptr = const __attribute__((address_space(4))) T *;
__device__ __forceinline__ float ld_ro(const float *p) { return *(ro_ptr<float>)p; }
__device__ __forceinline__ double ld_ro(const double *p) { return *(ro_ptr<double>)p; }
__device__ __forceinline__ uint32_t ld_ro(const uint32_t *p) { return *(ro_ptr<uint32_t>)p; }
__device__ __forceinline__ float4 ld_ro(const float4 *p) {
    const ro_ptr<float> f = (ro_ptr<float>)p;
    return make_float4(f[0], f[1], f[2], f[3]);
}
__device__ __forceinline__ int4 ld_ro(const int4 *p) {
    const ro_ptr<int> f = (ro_ptr<int>)p;
    return make_int4(f[0], f[1], f[2], f[3]);
}
__device__ __forceinline__ uint2 ld_ro(const uint2 *p) {
    const ro_ptr<uint32_t> f = (ro_ptr<uint32_t>)p;
    return make_uint2(f[0], f[1]);
}
template <typename T>
struct RoPtr {
    const T *p;
    __device__ __forceinline__ T operator[](int64_t i) const { return ld_ro(p + i); }
    __device__ __forceinline__ T operator*() const { return ld_ro(p); }
};
template <typename T>
__device__ __forceinline__ RoPtr<T> ro(const T *p) { return RoPtr<T>{p}; }

// workgroup -> work item, XCD-aware: workgroups are dispatched round-robin
// over the 8 XCDs, so the first n items are handed out as 8 contiguous
// ranges, one per XCD, and neighbouring items share one XCD's L2.  A
// bijection from [0, nb) onto [0, nb), nb = min(gridDim.x, n rounded up to 8);
// workgroups at or past nb get nb (no item).
__device__ __forceinline__ uint32_t xcd_item(uint32_t n) {
    const uint32_t nb = min(gridDim.x, (n + 7u) & ~7u), b = blockIdx.x;
    if (b >= nb) return nb;
    const uint32_t q = nb / 8, r = nb % 8, x = b % 8;
    return x * q + min(x, r) + b / 8;
}

// elementary functions per precision: raw hardware approximations in FP32,
// the device math library in FP64
template <typename T> struct RT;
template <> struct RT<float> {
    static __device__ __forceinline__ float expn(float t) { return fexp2(-t * kLog2e); }
    static __device__ __forceinline__ float sqrt(float x) { return fsqrt(x); }
    static __device__ __forceinline__ float rcp(float x) { return frcp(x); }
    static __device__ __forceinline__ float log(float x) { return flog(x); }
};
template <> struct RT<double> {
    static __device__ __forceinline__ double expn(double t) { return ::exp(-t); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
};

// the cell (cluster coordinates) a point falls in; false if not finite / out of range
__device__ inline bool query_cell(const float *x, int voxel_mode, double hv, double hc, int64_t c[3]) {
    for (int a = 0; a < 3; ++a) {
        int64_t v;
        if (voxel_mode) {
            if (!cell_coord(x[a], hv, v)) return false;
            c[a] = floor_div8(v);
        } else {
            if (!cell_coord(x[a], hc, v)) return false;
            c[a] = v;
        }
    }
    return true;
}

__device__ inline void write_invalid(uint32_t qi, float *dist, float *grad, float *var,
                                     uint8_t *valid, float *aux, float *prop, float *prop_var) {
    dist[qi] = INFINITY;
    valid[qi] = 0;
    if (grad) { grad[3 * qi] = 0.f; grad[3 * qi + 1] = 0.f; grad[3 * qi + 2] = 0.f; }
    if (var) var[qi] = INFINITY;
    if (aux) { aux[3 * qi] = 0.f; aux[3 * qi + 1] = 0.f; aux[3 * qi + 2] = 0.f; }
    if (prop) prop[qi] = 0.f;
    if (prop_var) prop_var[qi] = INFINITY;
}

// ---------------------------------------------------------------------------
// grouping of queries by cell
// ---------------------------------------------------------------------------
__global__ void k_qcells(const float *__restrict__ q, int64_t mb, const uint32_t *__restrict__ dm, int voxel_mode,
                         double hv, double hc, HashView qh, uint32_t *__restrict__ cnt, int32_t *__restrict__ qslot,
                         uint32_t *__restrict__ qrank, float *dist, float *grad, float *var,
                         uint8_t *valid, float *aux, float *prop, float *prop_var,
                         unsigned long long *__restrict__ stat) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t m = dev_count(mb, dm);
    if (int64_t(blockIdx.x) * blockDim.x >= m) return;  // whole block past the end
    int64_t c[3];
    const bool in = i < m;
    const bool okc = in && query_cell(q + 3 * i, voxel_mode, hv, hc, c);
    // the queries of one wavefront mostly share a few cells: the lanes form
    // groups of equal cell key (ballots only), then the first lane of every
    // group probes the table and adds its group's size to the cell count,
    // all groups at once, so the wavefront waits for one probe and one
    // atomic instead of one per cell
    const int lane = int(threadIdx.x & 63);
    const unsigned long long key = okc ? pack_key(c[0], c[1], c[2]) : 0ull;
    int leader = lane;
    uint64_t group = 0;
    for (uint64_t todo = __ballot(okc); todo;) {
        const int l0 = __ffsll((long long)todo) - 1;
        const unsigned long long k0 = __shfl(key, l0, 64);
        const uint64_t grp = __ballot(okc && key == k0) & todo;
        if ((grp >> lane) & 1ull) { leader = l0; group = grp; }
        todo &= ~grp;
    }
    int64_t s0 = -1;
    uint32_t base = 0;
    if (okc && leader == lane) {
        bool ins;
        s0 = hash_insert(qh, key, &ins);
        if (s0 >= 0) base = atomicAdd(&cnt[s0], uint32_t(__popcll(group)));
    }
    const int64_t s = okc ? __shfl(s0, leader, 64) : int64_t(-1);
    const uint32_t rank = __shfl(base, leader, 64) + uint32_t(__popcll(group & lanes_below()));
    wave_count(&stat[ST_NONFINITE_Q], in && !okc);
    wave_count(&stat[ST_HASH_FULL], okc && s < 0);
    if (!in) return;
    if (s < 0) {
        qslot[i] = -1;
        write_invalid(uint32_t(i), dist, grad, var, valid, aux, prop, prop_var);
        return;
    }
    qslot[i] = int32_t(s);
    qrank[i] = rank;
}

__global__ __launch_bounds__(256) void k_cells_compact(
    const unsigned long long *__restrict__ keys, const uint32_t *__restrict__ cnt, int64_t cap,
    const uint32_t *__restrict__ tile_off, int64_t ntiles, int32_t *__restrict__ cell_of_slot,
    uint64_t *__restrict__ cell_key, uint32_t *__restrict__ cell_cnt,
    uint32_t *__restrict__ cell_chunks, unsigned long long *__restrict__ stat, uint32_t *__restrict__ ncells) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stat[ST_CELLS] = tile_off[ntiles];
        *ncells = tile_off[ntiles];
    }
    for_occupied_in_tile(keys, cap, tile_off[blockIdx.x], [&](int64_t s, unsigned long long k, uint32_t id) {
        cell_of_slot[s] = int32_t(id);
        cell_key[id] = k;
        const uint32_t n = cnt[s];
        cell_cnt[id] = n;
        cell_chunks[id] = (n + 63) / 64;
    });
}

__global__ void k_cell_lists(int64_t ncb, const uint32_t *__restrict__ dnc, const uint64_t *__restrict__ cell_key,
                             const unsigned long long *__restrict__ chash, uint32_t cmask,
                             const int32_t *__restrict__ chash_val, const uint8_t *__restrict__ pd,
                             const int32_t *__restrict__ coff, const int64_t *__restrict__ woff,
                             int4 *__restrict__ lists) {
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(ncb, dnc)) return;
    int64_t cc[3];
    unpack_key(cell_key[c], cc);
    int4 *L = lists + c * kListStride;
    int nsel = 0;
    // ascending key order: x offset outermost, z innermost.  The nine cells
    // of one x offset are looked up together: their first probes are loaded
    // at once (a key mostly sits in its first slot or meets an empty one),
    // only the others probe on, then the clusters' records are loaded at once
    // A neighbour cell outside the 21-bit key range holds no cluster; its
    // packed key would alias another cell's (or the empty-slot marker).
    auto in_range = [](int64_t v) { return v >= -kBias && v < kBias; };
    for (int dx = -1; dx <= 1; ++dx) {
        uint64_t key[9];
        unsigned long long k0[9];
        uint32_t s0[9];
        bool inr[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int64_t nx = cc[0] + dx, ny = cc[1] + t / 3 - 1, nz = cc[2] + t % 3 - 1;
            inr[t] = in_range(nx) && in_range(ny) && in_range(nz);
            key[t] = inr[t] ? pack_key(nx, ny, nz) : 0ull;
            s0[t] = uint32_t(mix64(key[t]) & cmask);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) k0[t] = chash[s0[t]];
        int32_t id[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int64_t sl = !inr[t] ? int64_t(-1)
                               : k0[t] == key[t] ? int64_t(s0[t])
                               : k0[t] == kNoKey ? int64_t(-1) : hash_find(chash, cmask, key[t]);
            id[t] = sl < 0 ? -1 : chash_val[sl];
        }
        int32_t b[9], e[9];
        uint8_t ok[9];
        int64_t wo[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int32_t j = id[t] < 0 ? 0 : id[t];
            b[t] = coff[j];
            e[t] = coff[j + 1];
            ok[t] = pd[j];
            wo[t] = woff[j];
        }
#pragma unroll
        for (int t = 0; t < 9; ++t)
            if (id[t] >= 0 && ok[t] && e[t] > b[t]) L[1 + nsel++] = make_int4(id[t], b[t], e[t] - b[t], int32_t(wo[t]));
    }
    L[0] = make_int4(nsel, 0, 0, 0);
}

// chunk table: (cell, first query) for every 64-query chunk of every cell
__global__ void k_chunk_table(int64_t ncb, const uint32_t *__restrict__ dnc, const uint32_t *__restrict__ cell_chunks,
                              const uint32_t *__restrict__ chunk_off, uint2 *__restrict__ chunk) {
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(ncb, dnc)) return;
    const uint32_t o = chunk_off[c];
    for (uint32_t j = 0; j < cell_chunks[c]; ++j) chunk[o + j] = make_uint2(uint32_t(c), j * 64u);
}

__global__ void k_scatter_order(const int32_t *__restrict__ qslot, const uint32_t *__restrict__ qrank,
                                int64_t mb, const uint32_t *__restrict__ dm, const int32_t *__restrict__ cell_of_slot,
                                const uint32_t *__restrict__ cell_off, uint32_t *__restrict__ order) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= dev_count(mb, dm)) return;
    const int32_t s = qslot[i];
    if (s < 0) return;
    order[cell_off[cell_of_slot[s]] + qrank[i]] = uint32_t(i);
}

__global__ void k_all_invalid(int64_t m, float *dist, float *grad, float *var, uint8_t *valid,
                              float *aux, float *prop, float *prop_var) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) write_invalid(uint32_t(i), dist, grad, var, valid, aux, prop, prop_var);
}

// refine records (cell, query) -> counting sort by cell
// (grid-stride: the records are a small share of the queries that bound the
// grid)
__global__ void k_refine_count(const uint2 *__restrict__ rec, const unsigned long long *__restrict__ nrec,
                               int64_t cap, uint32_t *__restrict__ rcnt, uint32_t *__restrict__ rrank) {
    const int64_t n = min(int64_t(*nrec), cap);
    for (int64_t b = int64_t(blockIdx.x) * blockDim.x; b < n; b += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = b + threadIdx.x;
        const uint32_t r = wave_rank(rcnt, i < n ? int64_t(rec[i].x) : int64_t(-1));
        if (i < n) rrank[i] = r;
    }
}

// re-evaluation chunks per cell, 64 refined queries each
__global__ void k_refine_chunks(int64_t ncb, const uint32_t *__restrict__ dnc, const uint32_t *__restrict__ rcnt,
                                uint32_t *__restrict__ rchunks) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(ncb, dnc)) return;
    rchunks[c] = (rcnt[c] + 63) / 64;
}

__global__ void k_refine_scatter(const uint2 *__restrict__ rec, const unsigned long long *__restrict__ nrec,
                                 int64_t cap, const uint32_t *__restrict__ rrank,
                                 const uint32_t *__restrict__ roff, uint32_t *__restrict__ rorder,
                                 uint32_t *__restrict__ rcell) {
    const int64_t n = min(int64_t(*nrec), cap);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t p = roff[rec[i].x] + rrank[i];
        rorder[p] = rec[i].y;
        rcell[p] = rec[i].x;
    }
}

// ---------------------------------------------------------------------------
// pair evaluation (T = float: the product path; T = double: re-evaluation)
// ---------------------------------------------------------------------------
template <typename T>
struct PairRaw {
    T o, gx, gy, gz;
    T ss;
    float S;   // sum of squared term scales (FP32 error estimate)
    T c;       // property k . beta (Eq. (6))
    float Sc;  // its sum of squared term scales
};

template <typename T>
struct Acc {
    T m, sw, swd, swv, sgx, sgy, sgz;      // smooth-min sums, scaled by exp(-lambda (. - m))
    T pgx, pgy, pgz;                       // plain gradient sum
    T hd, hv, hgx, hgy, hgz, ho, hu;       // closest node
    float A1, A2, B1, C1;                  // error-estimate sums (smooth-min scaled, FP32 only)
    float Ggx, Ggy, Ggz, G2;               // sum w e_d g and w e_d |g|^2
    float hed, heg, hev, sum_eg;           // closest node estimates, plain sum of e_g
    T swc, swu, hc;                        // property and latent variance: weighted sums, closest node
    float Cc1, Mc1, Mc2, hec;              // property error sums: w e_c, w e_d c, w e_d c^2; closest node
    int nq, ntot;
    float best;                            // nearest training point (FP32 decision)
    int bidx;
};

template <typename T>
__device__ inline void acc_init(Acc<T> &A) {
    A.m = T(INFINITY);
    A.sw = A.swd = A.swv = A.sgx = A.sgy = A.sgz = T(0);
    A.pgx = A.pgy = A.pgz = T(0);
    A.hd = T(INFINITY); A.hv = A.hgx = A.hgy = A.hgz = A.ho = A.hu = T(0);
    A.A1 = A.A2 = A.B1 = A.C1 = 0.f;
    A.Ggx = A.Ggy = A.Ggz = A.G2 = 0.f;
    A.hed = A.heg = A.hev = A.sum_eg = 0.f;
    A.swc = A.swu = A.hc = T(0);
    A.Cc1 = A.Mc1 = A.Mc2 = A.hec = 0.f;
    A.nq = 0; A.ntot = 0;
    A.best = INFINITY; A.bidx = -1;
}

struct QueryPoint {
    float fx, fy, fz;  // the FP32 query (for the FP32 nearest-point decision)
};

// one point: kernel value k, the factor e multiplying alpha (x - x_i) in the
// gradient sum, and the point's contribution to the running sums
//
// live == false marks a row loaded past the end of the cluster (batched FP32
// loads): its alpha is taken as 0 and it takes no part in the nearest-point
// decision, so every sum is left bitwise unchanged.
template <typename T, int KERN>
__device__ __forceinline__ T point_eval(const float4 p, T alpha, const QueryPoint &Q, int gidx,
                                        const QueryConsts &C, PairRaw<T> &r, Acc<T> &A,
                                        bool live = true, T beta = T(0)) {
    // nearest training point, decided in FP32 in a fixed order
    {
        const float ex = Q.fx - p.x, ey = Q.fy - p.y, ez = Q.fz - p.z;
        const float r2f = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
        if (live && r2f < A.best) { A.best = r2f; A.bidx = gidx; }
    }
    alpha = live ? alpha : T(0);
    T dx, dy, dz;
    if constexpr (std::is_same<T, float>::value) {
        dx = Q.fx - p.x; dy = Q.fy - p.y; dz = Q.fz - p.z;
    } else {
        dx = double(Q.fx) - double(p.x); dy = double(Q.fy) - double(p.y); dz = double(Q.fz) - double(p.z);
    }
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    T k, e, t;
    if (kern_kind(KERN) == GPDF_KERNEL_MATERN32) {
        t = RT<T>::sqrt(r2) * T(std::is_same<T, float>::value ? C.a : C.ad);  // sqrt(3) r / l
        e = RT<T>::expn(t);
        k = fma(t, e, e);                   // (1 + t) e^{-t}
    } else {
        t = r2 * T(std::is_same<T, float>::value ? C.a : C.ad);              // r^2 / 2 l^2
        k = RT<T>::expn(t);
        e = k;
    }
    r.o = fma(alpha, k, r.o);
    if constexpr (kern_grad(KERN)) {
        const T cg = alpha * e;
        r.gx = fma(cg, dx, r.gx);
        r.gy = fma(cg, dy, r.gy);
        r.gz = fma(cg, dz, r.gz);
    }
    if constexpr (std::is_same<T, float>::value) {
        // root-sum-square scale of the rounding errors of the terms alpha k,
        // whose relative error grows like (1 + t) through the exponent
        const float akt = fabsf(alpha) * fmaf(k, t, k);
        r.S = fmaf(akt, akt, r.S);
    }
    if constexpr (kern_prop(KERN)) {
        // the property GP shares the kernel values (Eq. (6))
        const T bl = live ? beta : T(0);
        r.c = fma(bl, k, r.c);
        if constexpr (std::is_same<T, float>::value) {
            const float bkt = fabsf(bl) * fmaf(k, t, k);
            r.Sc = fmaf(bkt, bkt, r.Sc);
        }
    }
    return k;
}

// beta of point i of a cluster (FP64 array), 0 when the launch has no property
template <typename T, int KERN>
__device__ __forceinline__ T beta_of(const double *__restrict__ b64, int i) {
    if constexpr (kern_prop(KERN)) return T(b64[i]);
    else return T(0);
}

template <typename T>
__device__ __forceinline__ T alpha_of(const float4 &p, const double *__restrict__ a64, int i) {
    if constexpr (std::is_same<T, float>::value) return p.w;
    else return a64[i];
}

// n <= NMAX: k in registers, W rows packed (row i at i (i + 1) / 2).  The
// rows are generated at compile time (index sequences), so every k_j index is
// a constant and the vector lives in VGPRs.
// kernel value only (a point already summed in another panel)
template <typename T, int KERN>
__device__ __forceinline__ T point_k(const float4 p, const QueryPoint &Q, const QueryConsts &C) {
    T dx, dy, dz;
    if constexpr (std::is_same<T, float>::value) {
        dx = Q.fx - p.x; dy = Q.fy - p.y; dz = Q.fz - p.z;
    } else {
        dx = double(Q.fx) - double(p.x); dy = double(Q.fy) - double(p.y); dz = double(Q.fz) - double(p.z);
    }
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (kern_kind(KERN) == GPDF_KERNEL_MATERN32) {
        const T t = RT<T>::sqrt(r2) * T(std::is_same<T, float>::value ? C.a : C.ad);
        const T e = RT<T>::expn(t);
        return fma(t, e, e);
    } else {
        return RT<T>::expn(r2 * T(std::is_same<T, float>::value ? C.a : C.ad));
    }
}

// n <= NMAX <= 32: k in registers, W rows packed (row i at i (i + 1) / 2).
// The rows are generated at compile time (index sequences), so every k_j
// index is a constant and the vector lives in VGPRs.
template <typename T, typename PW, int... J>
__device__ __forceinline__ T row_dot(PW Wi, const T *kr, std::integer_sequence<int, J...>) {
    T t[2] = {T(0), T(0)};
    ((t[J & 1] = fma(Wi[J], kr[J], t[J & 1])), ...);
    return t[0] + t[1];
}

template <typename T, int KERN, int NMAX, int I>
__device__ __forceinline__ void small_rows(const float4 *__restrict__ P, const double *__restrict__ a64,
                                           const double *__restrict__ b64,
                                           const T *__restrict__ W, int n, int pbase,
                                           const QueryPoint &Q, const QueryConsts &C, PairRaw<T> &r,
                                           Acc<T> &A, T *kr) {
    if constexpr (I < NMAX) {
        if (I >= n) return;
        const float4 p = ro(P)[I];
        kr[I] = point_eval<T, KERN>(p, alpha_of<T>(p, a64, I), Q, pbase + I, C, r, A, true,
                                    beta_of<T, KERN>(b64, I));
        const T t = row_dot<T>(ro(W + (I * (I + 1)) / 2), kr, std::make_integer_sequence<int, I + 1>{});
        r.ss = fma(t, t, r.ss);
        small_rows<T, KERN, NMAX, I + 1>(P, a64, b64, W, n, pbase, Q, C, r, A, kr);
    }
}

// FP32: the points and factor rows of a group of rows are loaded as one
// batch of scalar loads, so the wavefront waits once per group instead of
// once per row.  Scalar loads may return out of order, so a wait always
// covers every load in flight; batching is the way to overlap them.  Rows of
// the last group at or past n are loaded but masked (point_eval with
// live == false, their squared products dropped); the point and factor
// arrays carry a tail pad so that these loads stay inside the allocation.
constexpr int f32_group(int i) { return i < 8 ? 4 : 2; }   // rows per batch

template <int KERN, int I, int WO>
__device__ __forceinline__ void group_row_f32(const float4 pp, float bb, const float *w, int n, int pbase,
                                              const QueryPoint &Q, const QueryConsts &C,
                                              PairRaw<float> &r, Acc<float> &A, float *kr) {
    const bool live = I < n;
    kr[I] = point_eval<float, KERN>(pp, pp.w, Q, pbase + I, C, r, A, live, bb);
    const float t = row_dot<float>(w + WO, kr, std::make_integer_sequence<int, I + 1>{});
    r.ss = live ? fmaf(t, t, r.ss) : r.ss;
}

template <int KERN, int I0, int... R>
__device__ __forceinline__ void group_rows_f32(const float4 *p, const float *b, const float *w, int n, int pbase,
                                               const QueryPoint &Q, const QueryConsts &C,
                                               PairRaw<float> &r, Acc<float> &A, float *kr,
                                               std::integer_sequence<int, R...>) {
    // row I0 + R starts at R I0 + R (R + 1) / 2 inside the batch
    (group_row_f32<KERN, I0 + R, R * I0 + R * (R + 1) / 2>(p[R], b[R], w, n, pbase, Q, C, r, A, kr), ...);
}

template <int KERN, int NMAX, int I0>
__device__ __forceinline__ void small_groups_f32(const float4 *__restrict__ P, const float *__restrict__ B,
                                                 const float *__restrict__ W,
                                                 int n, int pbase, const QueryPoint &Q,
                                                 const QueryConsts &C, PairRaw<float> &r,
                                                 Acc<float> &A, float *kr) {
    if constexpr (I0 < NMAX) {
        if (I0 >= n) return;
        constexpr int G = f32_group(I0);
        constexpr int WB = I0 * (I0 + 1) / 2;        // first element of row I0
        constexpr int WL = G * I0 + G * (G + 1) / 2;  // elements of rows I0 .. I0 + G - 1
        float4 p[G];
        float b[G];
        float w[WL];
#pragma unroll
        for (int i = 0; i < G; ++i) p[i] = ro(P)[I0 + i];
#pragma unroll
        for (int i = 0; i < G; ++i) b[i] = kern_prop(KERN) ? ro(B)[I0 + i] : 0.f;
#pragma unroll
        for (int i = 0; i < WL; ++i) w[i] = ro(W)[WB + i];
        group_rows_f32<KERN, I0>(p, b, w, n, pbase, Q, C, r, A, kr, std::make_integer_sequence<int, G>{});
        small_groups_f32<KERN, NMAX, I0 + G>(P, B, W, n, pbase, Q, C, r, A, kr);
    }
}

// B: beta in FP32 (the FP32 path), b64: in FP64; read only when KERN
// carries kProp
template <typename T, int KERN, int NMAX>
__device__ __forceinline__ void eval_small(const float4 *__restrict__ P, const double *__restrict__ a64,
                                           const float *__restrict__ B, const double *__restrict__ b64,
                                           const T *__restrict__ W, int n, int pbase,
                                           const QueryPoint &Q, const QueryConsts &C, PairRaw<T> &r,
                                           Acc<T> &A) {
    T kr[NMAX];
    if constexpr (std::is_same<T, float>::value)
        small_groups_f32<KERN, NMAX, 0>(P, B, W, n, pbase, Q, C, r, A, kr);
    else
        small_rows<T, KERN, NMAX, 0>(P, a64, b64, W, n, pbase, Q, C, r, A, kr);
}

// t[R0 + R] += col[R0 + R] k_j for R = 0 .. kPanel - 1 - R0
template <typename T, int R0, typename PC, int... R>
__device__ __forceinline__ void panel_update(T *t, PC col, T kj, std::integer_sequence<int, R...>) {
    ((t[R0 + R] = fma(col[R0 + R], kj, t[R0 + R])), ...);
}

// diagonal block of a panel: column J holds rows J .. kPanel - 1 (lower
// triangle), so the update starts at row J; its points are summed here
template <typename T, int KERN, int J>
__device__ __forceinline__ void diag_cols(const float4 *__restrict__ P, const double *__restrict__ a64,
                                          const double *__restrict__ b64,
                                          const T *__restrict__ D, int nrem, int pbase,
                                          const QueryPoint &Q, const QueryConsts &C, PairRaw<T> &r,
                                          Acc<T> &A, T *t) {
    if constexpr (J < kPanel) {
        if (J >= nrem) return;
        const float4 p = ro(P)[J];
        const T kj = point_eval<T, KERN>(p, alpha_of<T>(p, a64, J), Q, pbase + J, C, r, A, true,
                                         beta_of<T, KERN>(b64, J));
        panel_update<T, J>(t, ro(D + J * kPanel), kj, std::make_integer_sequence<int, kPanel - J>{});
        diag_cols<T, KERN, J + 1>(P, a64, b64, D, nrem, pbase, Q, C, r, A, t);
    }
}

// FP32 diagonal block, two columns per batch of scalar loads; the second
// column of the last pair may lie past the cluster and is then masked.  The
// kernel values go to the lane's column of kc (stride 64), which the next
// panel reads instead of recomputing them.
template <int KERN, int J>
__device__ __forceinline__ void diag_pairs_f32(const float4 *__restrict__ P, const float *__restrict__ B,
                                               const float *__restrict__ D,
                                               int nrem, int pbase, const QueryPoint &Q,
                                               const QueryConsts &C, PairRaw<float> &r, Acc<float> &A,
                                               float *t, float *kc) {
    if constexpr (J < kPanel) {
        if (J >= nrem) return;
        const float4 p0 = ro(P)[J], p1 = ro(P)[J + 1];
        const float b0 = kern_prop(KERN) ? ro(B)[J] : 0.f, b1 = kern_prop(KERN) ? ro(B)[J + 1] : 0.f;
        float a[kPanel - J], b[kPanel - J - 1];
#pragma unroll
        for (int i = 0; i < kPanel - J; ++i) a[i] = ro(D)[J * kPanel + J + i];
#pragma unroll
        for (int i = 0; i < kPanel - J - 1; ++i) b[i] = ro(D)[(J + 1) * kPanel + J + 1 + i];
        const float k0 = point_eval<float, KERN>(p0, p0.w, Q, pbase + J, C, r, A, true, b0);
#pragma unroll
        for (int i = 0; i < kPanel - J; ++i) t[J + i] = fmaf(a[i], k0, t[J + i]);
        const bool live = J + 1 < nrem;
        const float k1 = point_eval<float, KERN>(p1, p1.w, Q, pbase + J + 1, C, r, A, live, b1);
#pragma unroll
        for (int i = 0; i < kPanel - J - 1; ++i) t[J + 1 + i] = live ? fmaf(b[i], k1, t[J + 1 + i]) : t[J + 1 + i];
        if (kc) {
            kc[J * 64] = k0;
            kc[(J + 1) * 64] = k1;
        }
        diag_pairs_f32<KERN, J + 2>(P, B, D, nrem, pbase, Q, C, r, A, t, kc);
    }
}

// n > 32: W in 32-row panels (column-major inside).  Panel r needs k_j for
// every column j < 32 (r + 1): the columns left of its diagonal block belong
// to points summed in earlier panels and only their kernel values are
// needed; the diagonal block sums its own points.  Given kc (the FP32 query
// kernel: the lane's column of an 8 KB LDS array per wavefront), the kernel
// values of the previous panel's diagonal block are kept there and the
// earlier ones recomputed; otherwise all are recomputed.
template <typename T, int KERN>
__device__ __forceinline__ void eval_panels(const float4 *__restrict__ P, const double *__restrict__ a64,
                                            const float *__restrict__ B, const double *__restrict__ b64,
                                            const T *__restrict__ W, int n, int pbase,
                                            const QueryPoint &Q, const QueryConsts &C, PairRaw<T> &r,
                                            Acc<T> &A, float *kc) {
    const T *Pn = W;
    for (int c0 = 0; c0 < n; c0 += kPanel) {
        T t[kPanel];
#pragma unroll
        for (int q = 0; q < kPanel; ++q) t[q] = T(0);
        if constexpr (std::is_same<T, float>::value) {
            // c0 is a multiple of the panel height: columns go in pairs; the
            // last panel's columns come from the cache, the earlier ones are
            // recomputed
            for (int j = 0; j < c0; j += 2) {
                const float4 p0 = ro(P)[j], p1 = ro(P)[j + 1];
                float a[kPanel], b[kPanel];
#pragma unroll
                for (int i = 0; i < kPanel; ++i) { a[i] = ro(Pn)[j * kPanel + i]; b[i] = ro(Pn)[(j + 1) * kPanel + i]; }
                float k0, k1;
                if (kc && j >= c0 - kPanel) {
                    k0 = kc[(j - (c0 - kPanel)) * 64];
                    k1 = kc[(j + 1 - (c0 - kPanel)) * 64];
                } else {
                    k0 = point_k<float, KERN>(p0, Q, C);
                    k1 = point_k<float, KERN>(p1, Q, C);
                }
                panel_update<float, 0>(t, a, k0, std::make_integer_sequence<int, kPanel>{});
                panel_update<float, 0>(t, b, k1, std::make_integer_sequence<int, kPanel>{});
            }
            diag_pairs_f32<KERN, 0>(P + c0, B + c0, Pn + c0 * kPanel, n - c0, pbase + c0, Q, C, r, A, t, kc);
        } else {
            for (int j = 0; j < c0; ++j) {
                const T kj = point_k<T, KERN>(ro(P)[j], Q, C);
                panel_update<T, 0>(t, ro(Pn + j * kPanel), kj, std::make_integer_sequence<int, kPanel>{});
            }
            diag_cols<T, KERN, 0>(P + c0, a64 + c0, b64 + c0, Pn + c0 * kPanel, n - c0, pbase + c0, Q, C, r, A, t);
        }
#pragma unroll
        for (int q = 0; q < kPanel; ++q) r.ss = fma(t[q], t[q], r.ss);
        Pn += int64_t(min(c0 + kPanel, n)) * kPanel;
    }
}

// Matern-3/2 reverting: t >= 0 with (1 + t) e^{-t} = o.  Seed from the
// branch-point series of W_{-1} (Corless et al. 1996) in s = sqrt(2 (1 - o)),
// eight terms in FP32 and four in FP64, for o > 1/2, from the asymptote t = y + log(1 + t),
// y = -log o, below; then Newton steps on f(t) = (1 + t) e^{-t} - o (three in
// FP32, five in FP64).  Near o = 1 the residual f cancels, and in FP32 the
// Newton steps would lose accuracy the series keeps (1 - o is exact there):
// above o = 0.95 the FP32 result is the series itself (relative error below
// 1e-6 against 6e-6 to 4e-3 after the steps).
template <typename T>
__device__ __forceinline__ T matern_t(T o) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const T s = RT<T>::sqrt(T(2) * (T(1) - o));
    T p = T(43) / T(540);
    if constexpr (f32) {
        p = fma(s, T(1963) / T(204120), T(680863) / T(43545600));
        p = fma(s, p, T(221) / T(8505));
        p = fma(s, p, T(769) / T(17280));
        p = fma(s, p, T(43) / T(540));
    }
    p = fma(s, p, T(11) / T(72));
    p = fma(s, p, T(1) / T(3));
    const T ta = s * fma(s, p, T(1));
    const T y = -RT<T>::log(o);
    T tb = y + RT<T>::log(T(1) + y);
    tb = y + RT<T>::log(T(1) + tb);
    T t = o > T(0.5) ? ta : tb;
    constexpr int kIt = f32 ? 3 : 5;
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const T E = RT<T>::expn(t);
        const T f = fma(t, E, E) - o;
        t = fma(f, RT<T>::rcp(t * E), t);
    }
    if constexpr (f32) return o > 0.95f ? ta : t;
    return t;
}

// one pair's outputs: distance, variance, gradient, latent occupancy and
// variance, and (FP32) the first-order error estimates of d, grad d and v
template <typename T>
struct PairOut {
    T d, v, gx, gy, gz, o, u;
    float ed, eg, ev, gn;
    T c;        // property (Eq. (6))
    float ec;   // its FP32 error estimate
};

template <typename T, int KERN>
__device__ __forceinline__ PairOut<T> pair_out(const PairRaw<T> &r, int n, const QueryConsts &C) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const T o = r.o;
    const T u = fmin(fmax(T(1) - r.ss, T(0)), T(1));
    const T omin = f32 ? T(C.omin) : T(C.omind), omax = f32 ? T(C.omax) : T(C.omaxd);
    const T oc = fmin(fmax(o, omin), omax);
    const T cc = f32 ? T(C.c) : T(C.cd), aa = f32 ? T(C.a) : T(C.ad);
    T d, lam, gsc;    // distance, Lambda, gradient scale
    float sens;       // |d ln(gsc) / d o| (error estimate)
    if (kern_kind(KERN) == GPDF_KERNEL_MATERN32) {
        const T t = matern_t<T>(oc);
        const T E = RT<T>::expn(t);
        const T tE = t * E;
        d = cc * t;
        lam = -cc * RT<T>::rcp(tE);          // -(l / sqrt3) e^t / t
        gsc = aa * RT<T>::rcp(tE);           // grad d = a G / (t e^{-t})
        sens = float(fabs(t - T(1)) * RT<T>::rcp(t * tE));
    } else {
        const T L = -RT<T>::log(oc);
        d = cc * RT<T>::sqrt(T(2) * L);      // l sqrt(-2 log o)
        lam = -cc * cc * RT<T>::rcp(oc * d); // -l^2 / (o d)
        gsc = RT<T>::rcp(oc * d);            // grad d = G / (o d)
        sens = float(RT<T>::rcp(oc) + fabs(lam) * RT<T>::rcp(d));
    }
    // at a cap the distance, Lambda and the gradient scale are the constants
    // of that cap, evaluated once in FP64 (in FP32, 1 - occ_max itself would
    // carry a relative error of ~1e-2); below the lower cap the returned
    // distance is the constant r(occ_min) and its gradient is zero, at the
    // upper cap Lambda(occ_max) grad o is kept
    if (o >= omax) {
        d = f32 ? T(C.cap_hi[0]) : T(C.cap_hid[0]);
        lam = f32 ? T(C.cap_hi[1]) : T(C.cap_hid[1]);
        gsc = f32 ? T(C.cap_hi[2]) : T(C.cap_hid[2]);
    } else if (o <= omin) {
        d = f32 ? T(C.cap_lo[0]) : T(C.cap_lod[0]);
        lam = f32 ? T(C.cap_lo[1]) : T(C.cap_lod[1]);
        gsc = f32 ? T(C.cap_lo[2]) : T(C.cap_lod[2]);
    }
    constexpr bool grad = kern_grad(KERN);
    const T gs = o < omin ? T(0) : gsc;
    const T gx = grad ? gs * r.gx : T(0), gy = grad ? gs * r.gy : T(0), gz = grad ? gs * r.gz : T(0);
    const T v = lam * lam * u;
    float ed = 0.f, eg = 0.f, ev = 0.f, gn = 0.f;
    if constexpr (f32) {
        // first-order error estimates of this pair's distance, gradient and
        // relative variance: the error of o is the root-sum-square of the
        // term errors plus the reverting solve, which settles at ~ eps o
        const float sS = fsqrt(r.S);
        const float dO = C.err_c * kEps * sS + 2.f * kEps * oc;
        if constexpr (grad) gn = fsqrt(fmaf(gz, gz, fmaf(gy, gy, gx * gx)));
        // o clearly beyond a cap (by more than its error): d, Lambda and v are
        // the constants of the cap and do not see the error of o; below the
        // lower cap the gradient is exactly zero
        const bool low = o < omin - 4.f * dO, high = o > omax + 4.f * dO;
        const float dOe = (low || high) ? 0.f : dO;
        ed = fabsf(lam) * dOe + 4.f * kEps * d;
        if constexpr (grad)
            eg = low ? 0.f : gsc * C.err_c * kEps * sS * frcp(C.a) + gn * sens * dOe + 8.f * kEps * gn;
        ev = 2.f * sens * dOe + 4.f * kEps * float(n) * frcp(fmaxf(u, 1e-30f)) + 8.f * kEps;
        // o within its error of the lower cap: the FP32 decision that switches
        // the gradient off is not reliable, and the gradient is either zero
        // or about gsc |grad o|
        if (grad && fabsf(o - omin) <= 4.f * dO) {
            const float go = fsqrt(fmaf(float(r.gz), float(r.gz), fmaf(float(r.gy), float(r.gy), float(r.gx) * float(r.gx))));
            eg += float(gsc) * go;
        }
    }
    float ec = 0.f;
    if constexpr (f32 && kern_prop(KERN)) ec = C.err_c * kEps * fsqrt(r.Sc) + 2.f * kEps * fabsf(r.c);
    return PairOut<T>{d, v, gx, gy, gz, o, u, ed, eg, ev, gn, kern_prop(KERN) ? r.c : T(0), ec};
}

// accumulation of one pair into the combination of its query (closest node,
// online smooth minimum, plain gradient sum, counts)
template <typename T, bool GRAD = true, bool PROP = false>
__device__ __forceinline__ void pair_accumulate(const PairOut<T> &P, int n, const QueryConsts &C, Acc<T> &A) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const T d = P.d, v = P.v, gx = P.gx, gy = P.gy, gz = P.gz, o = P.o, u = P.u;
    const float ed = P.ed, eg = P.eg, ev = P.ev, gn = P.gn;
    // closest node (strict <: the first in ascending key order wins ties)
    if (d < A.hd) {
        A.hd = d; A.hv = v; A.ho = o; A.hu = u;
        A.hed = ed; A.hev = ev;
        if constexpr (GRAD) { A.hgx = gx; A.hgy = gy; A.hgz = gz; A.heg = eg; }
        if constexpr (PROP) { A.hc = P.c; A.hec = P.ec; }
    }
    // smooth minimum, online: rescale the sums when the minimum moves
    const T delta = d - A.m;
    const T lamw = f32 ? T(C.lam) : T(C.lamd);
    const T ex = RT<T>::expn(lamw * fabs(delta));
    const bool newmin = delta < T(0);
    const T so = newmin ? ex : T(1);
    const T w = newmin ? T(1) : ex;
    if constexpr (f32) {
        const float shift = newmin ? float(A.m - d) : 0.f;  // A2 is relative to the minimum
        A.A2 = so * fmaf(shift, A.A1, A.A2) + w * ed * (newmin ? 0.f : float(delta));
        if (!(A.m < INFINITY)) A.A2 = 0.f;
        A.A1 = fmaf(so, A.A1, w * ed);
        A.C1 = fmaf(so, A.C1, w * v * ev);
        if constexpr (GRAD) {
            A.B1 = fmaf(so, A.B1, w * eg);
            const float wed = w * ed;
            A.Ggx = fmaf(so, A.Ggx, wed * gx);
            A.Ggy = fmaf(so, A.Ggy, wed * gy);
            A.Ggz = fmaf(so, A.Ggz, wed * gz);
            A.G2 = fmaf(so, A.G2, wed * gn * gn);
            A.sum_eg += eg;
        }
        if constexpr (PROP) {
            const float wed = w * ed, cf = float(P.c);
            A.Cc1 = fmaf(so, A.Cc1, w * P.ec);
            A.Mc1 = fmaf(so, A.Mc1, wed * cf);
            A.Mc2 = fmaf(so, A.Mc2, wed * cf * cf);
        }
    }
    A.sw = fma(so, A.sw, w);
    A.swd = fma(so, A.swd, w * d);
    A.swv = fma(so, A.swv, w * v);
    if constexpr (PROP) {
        A.swc = fma(so, A.swc, w * P.c);
        A.swu = fma(so, A.swu, w * u);
    }
    if constexpr (GRAD) {
        A.sgx = fma(so, A.sgx, w * gx);
        A.sgy = fma(so, A.sgy, w * gy);
        A.sgz = fma(so, A.sgz, w * gz);
        A.pgx += gx; A.pgy += gy; A.pgz += gz;
    }
    A.m = fmin(A.m, d);
    A.nq += 1;
    A.ntot += n;
}

template <typename T, int KERN>
__device__ __forceinline__ void finish_pair(const PairRaw<T> &r, int n, const QueryConsts &C, Acc<T> &A) {
    pair_accumulate<T, kern_grad(KERN), kern_prop(KERN)>(pair_out<T, KERN>(r, n, C), n, C, A);
}

struct Outputs {
    float *dist, *grad, *var, *aux;
    uint8_t *valid;
    uint2 *refine;              // FP32 pass: (cell, query) records to redo in FP64
    unsigned long long *stat;   // the refine record counter (its value is used)
    unsigned long long *spread; // every other per-wavefront count (spread_add)
    float *prop, *prop_var;     // surface property and its variance (kProp launches)
};

// final combination, sign, error test and stores for one lane
template <typename T, int MODE, bool PROP = false>
__device__ inline void finish_query(const Acc<T> &A, uint32_t qi, uint32_t cell, bool active,
                                    const QueryPoint &Q, const float4 *__restrict__ pts,
                                    const QueryConsts &C, const Outputs &O) {
    constexpr bool f32 = std::is_same<T, float>::value;
    bool bad = false, bd = false, bg = false, bv = false;
    if (active && A.nq == 0)
        write_invalid(qi, O.dist, O.grad, O.var, O.valid, O.aux, PROP ? O.prop : nullptr,
                      PROP ? O.prop_var : nullptr);
    if (active && A.nq > 0) {
        T D, V, Gx, Gy, Gz, Cp = T(0), Wp = T(0);
        float Ed = 0.f, Eg = 0.f, Ev = 0.f, Ec = 0.f;
        if constexpr (MODE == kModeHard) {
            D = A.hd; V = A.hv; Gx = A.hgx; Gy = A.hgy; Gz = A.hgz;
            Ed = A.hed; Eg = A.heg; Ev = A.hev;
            if constexpr (PROP) { Cp = A.hc; Wp = A.hu; Ec = A.hec; }
        } else {
            const T iw = T(1) / A.sw;
            D = A.swd * iw;
            V = A.swv * iw;
            if constexpr (PROP) { Cp = A.swc * iw; Wp = A.swu * iw; }
            if constexpr (MODE == kModeMean) {
                const T iq = T(1) / T(A.nq);
                Gx = A.pgx * iq; Gy = A.pgy * iq; Gz = A.pgz * iq;
            } else {
                Gx = A.sgx * iw; Gy = A.sgy * iw; Gz = A.sgz * iw;
            }
            if constexpr (f32) {
                const float Gn = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
                const float lam = C.lam;
                Ed = (A.A1 * (1.f + lam * (D - A.m)) + lam * A.A2) * iw;
                // weight errors move G by lambda sum (w/W) e_d |g_q - G|,
                // bounded by Cauchy-Schwarz through the online moments of g
                const float Q2 = A.G2 - 2.f * (Gx * A.Ggx + Gy * A.Ggy + Gz * A.Ggz) + Gn * Gn * A.A1;
                Eg = (A.B1 + lam * sqrtf(fmaxf(A.A1 * Q2, 0.f))) * iw;
                if constexpr (MODE == kModeMean) Eg = A.sum_eg / float(A.nq) + Eg;
                Ev = A.C1 / A.swv;
                if constexpr (PROP) {
                    // as the gradient: the pair errors plus the weight errors,
                    // lambda sum (w/W) e_d |c_q - C| by Cauchy-Schwarz
                    const float Cf = float(Cp);
                    const float Q2c = A.Mc2 - 2.f * Cf * A.Mc1 + Cf * Cf * A.A1;
                    Ec = (A.Cc1 + lam * sqrtf(fmaxf(A.A1 * Q2c, 0.f))) * iw;
                }
            }
        }
        if (C.signed_ && A.bidx >= 0) {
            // sensor side of the nearest training point, decided in FP32
            const float4 p = pts[A.bidx];
            const float ax = Q.fx - p.x, ay = Q.fy - p.y, az = Q.fz - p.z;
            const float ox = C.d_origin ? C.d_origin[0] : C.ox, oy = C.d_origin ? C.d_origin[1] : C.oy,
                        oz = C.d_origin ? C.d_origin[2] : C.oz;
            const float bx = ox - p.x, by = oy - p.y, bz = oz - p.z;
            const float dot = fmaf(az, bz, fmaf(ay, by, ax * bx));
            if (!(dot >= 0.f)) { D = -D; Gx = -Gx; Gy = -Gy; Gz = -Gz; }
        }
        O.dist[qi] = float(D);
        O.valid[qi] = 1;
        if (O.grad) { O.grad[3 * qi] = float(Gx); O.grad[3 * qi + 1] = float(Gy); O.grad[3 * qi + 2] = float(Gz); }
        if (O.var) O.var[qi] = float(V);
        if (O.aux) { O.aux[3 * qi] = float(A.ho); O.aux[3 * qi + 1] = float(A.hu); O.aux[3 * qi + 2] = float(A.ntot); }
        if constexpr (PROP) {
            if (O.prop) O.prop[qi] = float(Cp);
            if (O.prop_var) O.prop_var[qi] = float(Wp);
        }
        if constexpr (f32) {
            // an output the caller did not ask for is not refined for; the
            // property variance is the latent variance, whose error the
            // relative variance estimate covers
            bd = !(Ed <= C.tau_d);
            bg = O.grad && !(Eg <= C.tau_g);
            bv = (O.var || (PROP && O.prop_var)) && !(Ev <= C.tau_v);
            bad = bd || bg || bv;
            if constexpr (PROP) bad = bad || (O.prop && !(Ec <= C.tau_c));
        }
    }
    // one atomic per wavefront for the valid count and the refine records
    const int lane = threadIdx.x & 63;
    if constexpr (f32) {
        const uint64_t nv = __ballot(active && A.nq > 0);
        if (lane == 0 && nv) spread_add(O.spread, ST_VALID_Q, (unsigned long long)__popcll(nv));
        const uint64_t mb = __ballot(bad);
        if (mb) {
            const uint64_t b1 = __ballot(bd), b2 = __ballot(bg), b3 = __ballot(bv);
            if (lane == 0) {
                spread_add(O.spread, ST_REF_D, (unsigned long long)__popcll(b1));
                spread_add(O.spread, ST_REF_G, (unsigned long long)__popcll(b2));
                spread_add(O.spread, ST_REF_V, (unsigned long long)__popcll(b3));
            }
        }
        if (mb && O.refine) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&O.stat[ST_REFINE], (unsigned long long)__popcll(mb));
            base = __shfl(base, 0, 64);
            if (bad) {
                const uint64_t lt = lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
                O.refine[base + __popcll(mb & lt)] = make_uint2(cell, qi);
            }
        }
    } else if (O.refine) {
        // FP64 instance: a null refine buffer marks the re-evaluation pass,
        // whose queries the FP32 pass already counted; otherwise this is the
        // FP64 evaluation of every query and counts them here
        const uint64_t nv = __ballot(active && A.nq > 0);
        if (lane == 0 && nv) spread_add(O.spread, ST_VALID_Q, (unsigned long long)__popcll(nv));
    }
}

template <typename T>
__device__ __forceinline__ const T *factor_base(const float *W32, const double *W64, int64_t off) {
    if constexpr (std::is_same<T, float>::value) return W32 + off;
    else return W64 + off;
}

template <typename T, int KERN>
__device__ __forceinline__ void eval_cluster(int base, int n, int64_t woff, const float4 *__restrict__ pts,
                                             const double *__restrict__ alpha64,
                                             const float *__restrict__ beta32,
                                             const double *__restrict__ beta64,
                                             const float *__restrict__ W32,
                                             const double *__restrict__ W64, const QueryPoint &Q,
                                             const QueryConsts &C, Acc<T> &A, float *kc = nullptr) {
    const float4 *P = pts + base;
    const double *a64 = alpha64 + base;
    const float *B = beta32 + base;
    const double *b64 = beta64 + base;
    const T *W = factor_base<T>(W32, W64, woff);
    PairRaw<T> r{T(0), T(0), T(0), T(0), T(0), 0.f, T(0), 0.f};
    if (n <= 8) eval_small<T, KERN, 8>(P, a64, B, b64, W, n, base, Q, C, r, A);
    else if (n <= 16) eval_small<T, KERN, 16>(P, a64, B, b64, W, n, base, Q, C, r, A);
    else if (n <= kPanel) eval_small<T, KERN, kPanel>(P, a64, B, b64, W, n, base, Q, C, r, A);
    else eval_panels<T, KERN>(P, a64, B, b64, W, n, base, Q, C, r, A, kc);
    finish_pair<T, KERN>(r, n, C, A);
}

struct Grouping {
    const uint2 *chunk;        // (cell, first query)
    const uint32_t *nchunks;   // device-side chunk count
    const uint32_t *cell_cnt;  // queries per cell
    const uint32_t *cell_off;  // first query of each cell in order[]
    const uint32_t *order;     // query indices grouped by cell
};

struct ModelView {
    const float4 *pts;
    const double *alpha64;
    const float *beta32;     // property right-hand side (Eq. (6)), read only by kProp launches;
    const double *beta64;    // never null (without a property they alias unread arrays)
    const int32_t *coff;
    const int64_t *woff;
    const float *W32;
    const double *W64;
    const uint64_t *ckey;
    const uint8_t *pd;
    int64_t ncl;
    double edge;
    const unsigned long long *chash;   // cluster hash (key -> slot)
    const int32_t *chash_val;          // slot -> cluster
    uint32_t cmask;
};

// NEIGHBOR27: one wavefront per (cell, 64-query chunk).  The cell's list
// holds a descriptor (cluster, first point, size, factor offset) per
// selected cluster; the next descriptor is loaded while the current cluster
// is evaluated.
template <typename T, int KERN, int MODE>
__device__ __forceinline__ void cells_chunk(uint32_t wave, const float *__restrict__ q, const Grouping &G,
                                            const int4 *__restrict__ lists, const ModelView &Mo,
                                            const QueryConsts &C, const Outputs &O) {
    const int lane = threadIdx.x & 63;
    const uint2 ch = ro(G.chunk)[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(ro(G.cell_cnt)[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = G.order[ro(G.cell_off)[cell] + start + (active ? lane : 0)];
    const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
    const RoPtr<int4> L = ro(lists + size_t(cell) * kListStride);
    const int nsel = int(uniform(uint32_t(L[0].x)));
    Acc<T> A;
    acc_init(A);
    // FP32: the kernel values of the previous panel (clusters above one
    // panel), one column of 32 per lane, column-major over the lanes
    [[maybe_unused]] float *kc = nullptr;
    if constexpr (std::is_same<T, float>::value) {
        __shared__ float kcache[kPanel * 64];
        kc = kcache + lane;
    }
    uint32_t sum_n = 0, sum_tri = 0;
    int4 nxt = L[1];
    for (int s = 0; s < nsel; ++s) {
        const int4 d = nxt;
        if (s + 1 < nsel) nxt = L[2 + s];
        const int base = int(uniform(uint32_t(d.y))), n = int(uniform(uint32_t(d.z)));
        const int64_t woff = int64_t(uniform(uint32_t(d.w)));
        eval_cluster<T, KERN>(base, n, woff, Mo.pts, Mo.alpha64, Mo.beta32, Mo.beta64, Mo.W32, Mo.W64, Q, C, A,
                              kc);
        sum_n += uint32_t(n);
        sum_tri += uint32_t(n * (n + 1) / 2);
    }
    finish_query<T, MODE, kern_prop(KERN)>(A, qi, cell, active, Q, Mo.pts, C, O);
    // algorithmic work of this wavefront (active lanes), one atomic each
    if (std::is_same<T, float>::value && lane == 0 && nsel > 0) {
        spread_add(O.spread, ST_PAIRS, (unsigned long long)nsel * cnt);
        spread_add(O.spread, ST_POINTS, (unsigned long long)sum_n * cnt);
        spread_add(O.spread, ST_TRI, (unsigned long long)sum_tri * cnt);
    }
}

// PERSIST == false: one wavefront (workgroup) per chunk, XCD-aware order.
// PERSIST: a fixed set of wavefronts takes chunks from the counter *work
// (zero at launch) until none is left.  Two instances, so that each keeps
// the register allocation of a single chunk body.
// the persistent FP32 instance is held to the occupancy of the one-chunk
// instance (four wavefronts per SIMD); left alone, the compiler keeps far more
// live across the chunk loop.  The FP32 one-chunk instances without gradient
// (the fusion's test voxels) are held to five, measured faster there (the
// ones with gradient measured slower at five)
template <typename T, int KERN, bool PERSIST>
constexpr int eval_min_waves() {
    return !std::is_same<T, float>::value ? 1 : PERSIST ? 4 : (KERN & kNoGrad) ? 5 : 1;
}

// REC (one-chunk instance of a captured frame): block 0 writes the number of
// chunks the launch takes, min(grid, chunks), to *work and the chunk count to
// *aux (pinned host memory).  The persistent instance takes the chunks from
// *aux on when aux is given (from 0 otherwise).  aux is the last argument, so
// that the instances without it lay out the others as before.
template <typename T, int KERN, int MODE, bool PERSIST, bool REC = false>
__global__ __launch_bounds__(kEvalT, (eval_min_waves<T, KERN, PERSIST>())) void k_query_cells(const float *__restrict__ q, Grouping G,
                                                     const int4 *__restrict__ lists, ModelView Mo,
                                                     QueryConsts C, Outputs O, uint32_t *work,
                                                     uint32_t *aux) {
    const uint32_t nch = *ro(G.nchunks);
    if constexpr (!PERSIST) {
        // the chunks this launch takes are 0 .. min(grid, chunks) - 1
        if constexpr (REC) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                *work = min(gridDim.x, nch);
                *aux = nch;
            }
        }
        const uint32_t wave = xcd_item(nch);
        if (wave < nch) cells_chunk<T, KERN, MODE>(wave, q, G, lists, Mo, C, O);
    } else {
        // The chunks form kXcds contiguous ranges, one per XCD (workgroups
        // are dispatched round-robin over the XCDs), each taken through its
        // own counter (zero at launch, one cache line each).  A wavefront
        // drains the range of its XCD, then those of the following XCDs:
        // neighbouring chunks share an L2 and the load still balances.  The
        // next index is requested before the current chunk is evaluated, so
        // the round trip of the counter overlaps the work.
        // Chunks below *aux (when given) are another launch's.
        const bool lead = (threadIdx.x & 63) == 0;
        const uint32_t f = aux ? min(uniform(*ro(aux)), nch) : 0u;
        const uint32_t per = (nch - f + kXcds - 1) / kXcds;
        const uint32_t x0 = blockIdx.x % kXcds;
        for (uint32_t r = 0; r < uint32_t(kXcds); ++r) {
            const uint32_t x = (x0 + r) % kXcds;
            const uint32_t lo = f + x * per, hi = min(nch, lo + per);
            if (lo >= hi) continue;
            uint32_t *ctr = work + x * kCtrStride;
            uint32_t i = 0;
            if (lead) i = atomicAdd(ctr, 1u);
            i = uniform(uint32_t(__shfl(int(i), 0, 64)));
            while (i < hi - lo) {
                uint32_t nx = 0;
                if (lead) nx = atomicAdd(ctr, 1u);
                cells_chunk<T, KERN, MODE>(lo + i, q, G, lists, Mo, C, O);
                i = uniform(uint32_t(__shfl(int(nx), 0, 64)));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Cluster-major FP64 re-evaluation.  The refined queries are a small, sparse
// share of a call (under 1 % of a LiDAR band), spread over thousands of
// cells; grouped per cell or per cluster they fill few lanes of a wavefront.
// So the pairs (refined query, cluster of at most kBigMaxN points) of all
// cells are counting-sorted by cluster, the clusters of at most one panel
// first, and evaluated densely:
//   n <= 32   one lane per pair, 64 consecutive pairs of the sorted list per
//             wavefront (neighbouring lanes mostly share a cluster, so their
//             loads coalesce): the FP64 small-cluster evaluation of the query
//             kernel;
//   n > 32    items of up to 16 queries of one cluster, a workgroup of four
//             wavefronts: kernel values into LDS, then the product W K on
//             FP64 MFMA (v_mfma_f64_16x16x4f64), the 16-row tiles of W shared
//             out over the wavefronts, each factor element read once per item.
// The pairs are reverted where they are evaluated (Eq. (3)-(5), one lane per
// pair) and go to a buffer with their nearest point; a combination pass with
// one lane per refined query combines them in list order.  Counts and offsets stay on the
// device; when a call's pairs exceed the buffers, or a cluster exceeds
// kBigMaxN points, a device flag hands every refined query to the FP64 query
// kernel instead.
//
// Indexing: a cell reserves one run of slots per selected cluster,
// cbase[cell, s], in the cluster's run; refined query p of the cell (its
// rank) sits at off[cluster] + cbase + p of the sorted pair list.  cbase
// lives at the cell's first re-evaluation chunk index (rchunk_off).  The
// reverted pair of the refined query at refine position r and descriptor s
// of its cell's list is stored at s * cap_ref + r, so that the combination
// reads consecutive records in consecutive lanes.
// ---------------------------------------------------------------------------
constexpr int kBigB = 16;                 // queries per item, clusters above one panel
constexpr int kBigMaxN = 256;             // larger clusters: the FP64 query kernel
constexpr int kBigStride = kListStride - 1;
constexpr int kBigT = 256;                // threads per large-cluster item

// a reverted pair (the FP64 PairOut without the FP32 error estimates), its
// nearest training point and the cluster size
struct BigOut {
    double d, v, gx, gy, gz, o, u, c;
    float best;
    int bidx;
    int n, pad;
};
static_assert(sizeof(BigOut) == 80, "BigOut layout");

template <int KERN>
__device__ __forceinline__ BigOut big_out(const PairRaw<double> &r, int n, const QueryConsts &C, float best, int bidx) {
    const PairOut<double> p = pair_out<double, KERN>(r, n, C);
    return BigOut{p.d, p.v, p.gx, p.gy, p.gz, p.o, p.u, p.c, best, bidx, n, 0};
}

struct BigView {
    const BigOut *res;      // [descriptor s][refine position]
    int64_t cap_ref;        // refine positions per descriptor
};

__device__ __forceinline__ bool cm_cluster(int n) { return n <= kBigMaxN; }

// pairs per cluster; each cell with refined queries reserves a run per
// selected cluster.  One thread per (first re-evaluation chunk of a cell,
// list slot); the chunk table is in cell order, so the cell's first chunk
// index is w.
__global__ void k_cm_count(const uint2 *__restrict__ chunk, const uint32_t *__restrict__ nchunks, int64_t cap_ch,
                           const uint32_t *__restrict__ rcnt, const int4 *__restrict__ lists,
                           uint32_t *__restrict__ bcnt, uint32_t *__restrict__ cbase) {
    const uint32_t nch = *nchunks;
    if (int64_t(nch) > cap_ch) return;
    const uint32_t total = nch * uint32_t(kBigStride);
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const uint32_t w = idx / kBigStride, s = idx - w * kBigStride;
        const uint2 ch = chunk[w];
        if (ch.y != 0) continue;
        const int4 *L = lists + size_t(ch.x) * kListStride;
        if (int(s) >= L[0].x) continue;
        const int4 d = L[1 + s];
        if (cm_cluster(d.z)) cbase[size_t(w) * kBigStride + s] = atomicAdd(&bcnt[d.x], rcnt[ch.x]);
    }
}

// the counts by size class, and the items of the larger clusters
__global__ void k_cm_split(int64_t ncb, const uint32_t *__restrict__ dncl, const int32_t *__restrict__ coff,
                           const uint32_t *__restrict__ bcnt, uint32_t *__restrict__ bcs,
                           uint32_t *__restrict__ bcb, uint32_t *__restrict__ nits, uint32_t *__restrict__ nit) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(ncb, dncl)) return;
    const int n = coff[c + 1] - coff[c];
    const uint32_t k = bcnt[c];
    const bool big = n > kPanel && n <= kBigMaxN;
    bcs[c] = n <= kPanel ? k : 0u;
    bcb[c] = big ? k : 0u;
    nits[c] = n <= kPanel ? (k + 63) / 64 : 0u;
    nit[c] = big ? (k + kBigB - 1) / kBigB : 0u;
}

// per cluster, once the counts are scanned: the run offsets (the clusters of
// at most one panel first, then the others) and the items of both size
// classes, when the pairs fit the buffers.  The first thread also records
// the decision: ok (the pairs fit), and the refined queries for the
// combination when every selected cluster has at most kBigMaxN points, else
// the chunks for the FP64 query kernel.
struct CmTotals {
    const uint32_t *nchunks, *nps, *npb, *maxn;
    const unsigned long long *nrec;
    int64_t cap_ch, cap_pairs, cap_rec, cap_ref;
};

__device__ __forceinline__ bool cm_fit(const CmTotals &T, int64_t nr) {
    return int64_t(*T.nchunks) <= T.cap_ch && int64_t(*T.nps) + int64_t(*T.npb) <= T.cap_pairs && nr <= T.cap_ref;
}

__global__ void k_cm_finish(int64_t ncb, const uint32_t *__restrict__ dncl, const int32_t *__restrict__ coff,
                            CmTotals T, const uint32_t *__restrict__ boffs, const uint32_t *__restrict__ boffb,
                            const uint32_t *__restrict__ nits, const uint32_t *__restrict__ ioffs,
                            const uint32_t *__restrict__ nit, const uint32_t *__restrict__ ioff,
                            uint32_t *__restrict__ boff, uint2 *__restrict__ items_s, uint2 *__restrict__ item,
                            uint32_t *__restrict__ ok, uint32_t *__restrict__ nref_fast,
                            uint32_t *__restrict__ nch_slow) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nr = min(int64_t(*T.nrec), T.cap_rec);
    const bool fit = cm_fit(T, nr);
    if (c == 0) {
        const bool all = fit && *T.maxn <= uint32_t(kBigMaxN);
        *ok = fit ? 1u : 0u;
        *nref_fast = all ? uint32_t(nr) : 0u;
        *nch_slow = all ? 0u : *T.nchunks;
    }
    if (!fit || c >= dev_count(ncb, dncl)) return;
    const int n = coff[c + 1] - coff[c];
    boff[c] = n <= kPanel ? boffs[c] : *T.nps + boffb[c];
    for (uint32_t i = 0; i < nits[c]; ++i) items_s[ioffs[c] + i] = make_uint2(uint32_t(c), i * 64u);
    for (uint32_t i = 0; i < nit[c]; ++i) item[ioff[c] + i] = make_uint2(uint32_t(c), i * kBigB);
}

// the query and result slot of every pair: one thread per (refine record,
// list slot)
__global__ void k_cm_fill(const uint2 *__restrict__ rec, const unsigned long long *__restrict__ nrec, int64_t cap,
                          const uint32_t *__restrict__ rrank, const uint32_t *__restrict__ roff,
                          const uint32_t *__restrict__ rchunk_off, const int4 *__restrict__ lists,
                          const uint32_t *__restrict__ cbase, const uint32_t *__restrict__ boff,
                          const uint32_t *__restrict__ ok, int64_t cap_ref, uint32_t *__restrict__ bq,
                          uint32_t *__restrict__ bdst) {
    if (*ok == 0) return;
    const uint32_t nr = uint32_t(min(int64_t(*nrec), cap));
    const uint32_t total = nr * uint32_t(kBigStride);
    for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const uint32_t i = idx / kBigStride, s = idx - i * kBigStride;
        const uint2 r = rec[i];
        const int4 *L = lists + size_t(r.x) * kListStride;
        if (int(s) >= L[0].x) continue;
        const int4 d = L[1 + s];
        if (!cm_cluster(d.z)) continue;
        const uint32_t p = rrank[i];
        const uint32_t pos = boff[d.x] + cbase[size_t(rchunk_off[r.x]) * kBigStride + s] + p;
        bq[pos] = r.y;
        bdst[pos] = uint32_t(int64_t(s) * cap_ref + roff[r.x] + p);
    }
}

// the FP64 small-cluster rows of the query kernel, on the cluster's data
// staged in LDS (the same arithmetic in the same order)
template <int KERN, int NMAX, int I>
__device__ __forceinline__ void cm_rows(const float4 *P, const double *a64, const double *b64, const double *W,
                                        int n, int pbase, const QueryPoint &Q, const QueryConsts &C,
                                        PairRaw<double> &r, Acc<double> &A, double *kr) {
    if constexpr (I < NMAX) {
        if (I >= n) return;
        const float4 p = P[I];
        kr[I] = point_eval<double, KERN>(p, a64[I], Q, pbase + I, C, r, A, true, beta_of<double, KERN>(b64, I));
        const double t = row_dot<double>(W + (I * (I + 1)) / 2, kr, std::make_integer_sequence<int, I + 1>{});
        r.ss = fma(t, t, r.ss);
        cm_rows<KERN, NMAX, I + 1>(P, a64, b64, W, n, pbase, Q, C, r, A, kr);
    }
}

constexpr int kSmallB = 64;   // queries per item, clusters of at most one panel
constexpr int kSmallW = kPanel * (kPanel + 1) / 2;

// clusters of at most one panel: one wavefront per item (up to 64 queries of
// one cluster), one query per lane.  The cluster's packed factor, points,
// alpha and beta are staged in LDS by the whole wavefront, every load issued
// before the first store, so that the item waits for memory once.
template <int KERN>
__global__ __launch_bounds__(64, 3) void k_cm_small(const float *__restrict__ q, const uint2 *__restrict__ items,
                                                    const uint32_t *__restrict__ nitems,
                                                    const uint32_t *__restrict__ bcnt,
                                                    const uint32_t *__restrict__ boff,
                                                    const uint32_t *__restrict__ bq,
                                                    const uint32_t *__restrict__ bdst, ModelView Mo, QueryConsts C,
                                                    const uint32_t *__restrict__ ok, BigOut *__restrict__ res) {
    __shared__ double sW[kSmallW + 64];
    __shared__ float4 sP[kPanel];
    __shared__ double sA[kPanel], sB[kPanel];
    if (uniform(*ro(ok)) == 0) return;
    const uint32_t ni = *ro(nitems);
    const int lane = int(threadIdx.x & 63);
    for (uint32_t w = blockIdx.x; w < ni; w += gridDim.x) {
        const uint2 it = ro(items)[w];
        const uint32_t cl = uniform(it.x), first = uniform(it.y);
        const int cnt = int(uniform(min(ro(bcnt)[cl] - first, uint32_t(kSmallB))));
        const uint32_t pos0 = uniform(ro(boff)[cl] + first);
        const int base = int(uniform(uint32_t(Mo.coff[cl])));
        const int n = int(uniform(uint32_t(Mo.coff[cl + 1]))) - base;
        const int nw = n * (n + 1) / 2;
        const double *W = Mo.W64 + int64_t(uniform(uint32_t(Mo.woff[cl])));
        const bool act = lane < cnt;
        const uint32_t pos = pos0 + uint32_t(act ? lane : 0);
        const uint32_t qi = bq[pos];
        // staging: all loads first
        double wv[(kSmallW + 63) / 64];
#pragma unroll
        for (int u = 0; u < (kSmallW + 63) / 64; ++u) {
            const int i = lane + 64 * u;
            wv[u] = i < nw ? W[i] : 0.0;
        }
        float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
        double av = 0.0, bv = 0.0;
        if (lane < n) {
            pv = Mo.pts[base + lane];
            av = Mo.alpha64[base + lane];
            if constexpr (kern_prop(KERN)) bv = Mo.beta64[base + lane];
        }
        const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
#pragma unroll
        for (int u = 0; u < (kSmallW + 63) / 64; ++u) sW[lane + 64 * u] = wv[u];
        if (lane < kPanel) {
            sP[lane] = pv;
            sA[lane] = av;
            sB[lane] = bv;
        }
        __syncthreads();  // the cluster's data in LDS
        PairRaw<double> r{0.0, 0.0, 0.0, 0.0, 0.0, 0.f, 0.0, 0.f};
        Acc<double> A;
        acc_init(A);
        double kr[kPanel];
        if (n <= 8) cm_rows<KERN, 8, 0>(sP, sA, sB, sW, n, base, Q, C, r, A, kr);
        else if (n <= 16) cm_rows<KERN, 16, 0>(sP, sA, sB, sW, n, base, Q, C, r, A, kr);
        else cm_rows<KERN, kPanel, 0>(sP, sA, sB, sW, n, base, Q, C, r, A, kr);
        const BigOut b = big_out<KERN>(r, n, C, A.best, A.bidx);
        if (act) res[bdst[pos]] = b;
        __syncthreads();  // the LDS is rewritten by the next item
    }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// W(i, j) of a cluster above one panel (32-row panels, column-major inside;
// panel r starts at 512 r (r + 1): every panel before the last is full);
// 0 above the diagonal and outside the cluster
__device__ __forceinline__ double w64_panel_at(const double *__restrict__ W, int n, int i, int j) {
    if (i >= n || j > i) return 0.0;
    const int r = i >> 5;
    return W[int64_t(512) * r * (r + 1) + int64_t(j) * kPanel + (i - (r << 5))];
}

// clusters of 33 to kBigMaxN points: one workgroup of four wavefronts per
// item.  Kernel values: thread t takes query t % 16 and the points
// j = t / 16 + 16 m; the partial sums of a query are added over the four
// lane groups of a wavefront by shuffles and over the wavefronts in LDS, in a
// fixed order.  Product: wavefront v takes the 16-row tiles v, v + 4, ...;
// per tile the k-steps of four columns accumulate on MFMA (A = W tile from
// memory, B = kernel values from LDS) in four independent accumulators,
// whose sum is squared into the lane's query (column) sum; the factor loads
// of 16 k-steps are in flight at a time.
// MFMA lane layout (lane l, lr = l % 16, lg = l / 16): A[m][k] lane m + 16 k,
// B[k][n] lane n + 16 k, D[m][n] lane n + 16 (m / 4), element m % 4.
template <int KERN>
__global__ __launch_bounds__(kBigT, 4) void k_cm_big(const float *__restrict__ q, const uint2 *__restrict__ items,
                                                  const uint32_t *__restrict__ nitems,
                                                  const uint32_t *__restrict__ bcnt,
                                                  const uint32_t *__restrict__ boff, const uint32_t *__restrict__ bq,
                                                  const uint32_t *__restrict__ bdst, ModelView Mo, QueryConsts C,
                                                  const uint32_t *__restrict__ ok, BigOut *__restrict__ res) {
    extern __shared__ double kb[];   // [rows rounded up to 4][kBigB]
    __shared__ float4 sP[kBigMaxN];
    __shared__ double sA[kBigMaxN], sB[kBigMaxN];
    __shared__ double part[4][kBigB][6];
    __shared__ float pbest[4][kBigB];
    __shared__ int pidx[4][kBigB];
    __shared__ double pss[4][kBigB];
    if (uniform(*ro(ok)) == 0) return;
    const uint32_t ni = *ro(nitems);
    const int t = int(threadIdx.x), lane = t & 63, wv = t >> 6;
    for (uint32_t w = blockIdx.x; w < ni; w += gridDim.x) {
    const uint2 it = ro(items)[w];
    const uint32_t cl = uniform(it.x), first = uniform(it.y);
    const int cnt = int(uniform(min(ro(bcnt)[cl] - first, uint32_t(kBigB))));
    const uint32_t pos0 = uniform(ro(boff)[cl] + first);
    const int base = int(uniform(uint32_t(Mo.coff[cl])));
    const int n = int(uniform(uint32_t(Mo.coff[cl + 1]))) - base;
    const int rows = (n + 3) & ~3;
    const double *W = Mo.W64 + int64_t(uniform(uint32_t(Mo.woff[cl])));
    // the cluster's points, alpha and beta staged in LDS (one round of loads)
    if (t < n) {
        sP[t] = Mo.pts[base + t];
        sA[t] = Mo.alpha64[base + t];
        if constexpr (kern_prop(KERN)) sB[t] = Mo.beta64[base + t];
    }
    __syncthreads();
    // kernel values and sums
    {
        const int a = t & 15, ph = t >> 4;
        const bool act = a < cnt;
        const uint32_t qi = ro(bq)[pos0 + uint32_t(act ? a : 0)];
        const float fx = q[3 * qi], fy = q[3 * qi + 1], fz = q[3 * qi + 2];
        double o = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, cp = 0.0;
        float best = INFINITY;
        int bidx = 0x7fffffff;
        for (int j = ph; j < rows; j += 16) {
            double k = 0.0;
            if (j < n) {
                const float4 p = sP[j];
                const double al = sA[j];
                const float ex = fx - p.x, ey = fy - p.y, ez = fz - p.z;
                const float r2f = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
                if (r2f < best) { best = r2f; bidx = base + j; }
                const double dx = double(fx) - double(p.x), dy = double(fy) - double(p.y),
                             dz = double(fz) - double(p.z);
                const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                double e;
                if (kern_kind(KERN) == GPDF_KERNEL_MATERN32) {
                    const double tt = ::sqrt(r2) * C.ad;
                    e = ::exp(-tt);
                    k = fma(tt, e, e);
                } else {
                    k = ::exp(-(r2 * C.ad));
                    e = k;
                }
                o = fma(al, k, o);
                if constexpr (kern_prop(KERN)) cp = fma(sB[j], k, cp);
                const double cg = al * e;
                gx = fma(cg, dx, gx);
                gy = fma(cg, dy, gy);
                gz = fma(cg, dz, gz);
            }
            kb[j * kBigB + a] = act ? k : 0.0;
        }
#pragma unroll
        for (int m = 16; m <= 32; m <<= 1) {
            o += __shfl_xor(o, m, 64);
            gx += __shfl_xor(gx, m, 64);
            gy += __shfl_xor(gy, m, 64);
            gz += __shfl_xor(gz, m, 64);
            if constexpr (kern_prop(KERN)) cp += __shfl_xor(cp, m, 64);
            const float b2 = __shfl_xor(best, m, 64);
            const int i2 = __shfl_xor(bidx, m, 64);
            if (b2 < best || (b2 == best && i2 < bidx)) { best = b2; bidx = i2; }
        }
        if (lane < kBigB) {
            part[wv][lane][0] = o; part[wv][lane][1] = gx; part[wv][lane][2] = gy;
            part[wv][lane][3] = gz; part[wv][lane][4] = cp;
            pbest[wv][lane] = best;
            pidx[wv][lane] = bidx;
        }
    }
    __syncthreads();  // kernel values and partial sums visible
    // product W K on MFMA
    const int lr = lane & 15, lg = lane >> 4;
    const int ntile = (n + 15) >> 4;
    double ssq = 0.0;
    for (int tile = wv; tile < ntile; tile += 4) {
        const int i = 16 * tile + lr;
        const int ksteps = (min(16 * tile + 16, n) + 3) >> 2;   // columns up to the tile's last row
        f64x4 acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
        // 16 k-steps of factor loads in flight at a time
        for (int s0 = 0; s0 < ksteps; s0 += 16) {
            double av[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int j = 4 * (s0 + u) + lg;
                av[u] = s0 + u < ksteps ? w64_panel_at(W, n, i, j) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int j = min(4 * (s0 + u) + lg, rows - 1);
                acc[u & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], kb[j * kBigB + lr], acc[u & 3], 0, 0, 0);
            }
        }
        const f64x4 d = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        ssq = fma(d[0], d[0], ssq);
        ssq = fma(d[1], d[1], ssq);
        ssq = fma(d[2], d[2], ssq);
        ssq = fma(d[3], d[3], ssq);
    }
    ssq += __shfl_xor(ssq, 16, 64);
    ssq += __shfl_xor(ssq, 32, 64);
    if (lane < kBigB) pss[wv][lane] = ssq;
    __syncthreads();
    if (t < cnt) {
        double sm[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) sm[k] = ((part[0][t][k] + part[1][t][k]) + part[2][t][k]) + part[3][t][k];
        float best = pbest[0][t];
        int bidx = pidx[0][t];
#pragma unroll
        for (int v = 1; v < 4; ++v)
            if (pbest[v][t] < best || (pbest[v][t] == best && pidx[v][t] < bidx)) { best = pbest[v][t]; bidx = pidx[v][t]; }
        const double ss = ((pss[0][t] + pss[1][t]) + pss[2][t]) + pss[3][t];
        // the raw sums; k_cm_revert reverts them (o, grad o, |W k|^2 in u, c)
        res[bdst[pos0 + uint32_t(t)]] = BigOut{0.0, 0.0, sm[1], sm[2], sm[3], sm[0], ss, sm[4], best, bidx, n, 0};
    }
    __syncthreads();  // kb and the partial sums are rewritten by the next item
    }
}

// the pairs of the larger clusters: the raw sums the item kernel stored (o,
// grad o, |W k|^2 in u, c) reverted in place, one lane per pair
template <int KERN>
__global__ __launch_bounds__(64) void k_cm_revert(const uint32_t *__restrict__ nps, const uint32_t *__restrict__ npb,
                                                  const uint32_t *__restrict__ bdst, QueryConsts C,
                                                  const uint32_t *__restrict__ ok, BigOut *__restrict__ res) {
    if (uniform(*ro(ok)) == 0) return;
    const uint32_t s0 = *ro(nps), nb = *ro(npb);
    for (uint32_t i = blockIdx.x * 64u + threadIdx.x; i < nb; i += gridDim.x * 64u) {
        BigOut *b = res + bdst[s0 + i];
        const BigOut raw = *b;
        const PairRaw<double> r{raw.o, raw.gx, raw.gy, raw.gz, raw.u, 0.f, raw.c, 0.f};
        *b = big_out<KERN>(r, raw.n, C, raw.best, raw.bidx);
    }
}

// The combination of the re-evaluated queries: one lane per refined query,
// 64 consecutive queries of the refine order (grouped by cell) per
// wavefront; each lane takes its cell's selected clusters in list order as
// the query kernel does and combines every reverted pair from the
// cluster-major buffer.  The next pair is loaded while the current one is
// combined.  Grid-stride over the windows.
template <int KERN, int MODE>
__global__ __launch_bounds__(kEvalT) void k_cm_combine(const float *__restrict__ q,
                                                       const uint32_t *__restrict__ nref,
                                                       const uint32_t *__restrict__ rorder,
                                                       const uint32_t *__restrict__ rcell,
                                                       const int4 *__restrict__ lists, ModelView Mo, QueryConsts C,
                                                       Outputs O, BigView BV) {
    const int lane = threadIdx.x & 63;
    const uint32_t nr = *ro(nref), nwin = (nr + 63) / 64;
    for (uint32_t w = blockIdx.x; w < nwin; w += gridDim.x) {
        const uint32_t p = 64 * w + uint32_t(lane);
        const bool active = p < nr;
        const uint32_t pp = active ? p : 64 * w;
        const uint32_t qi = rorder[pp], cell = rcell[pp];
        const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
        const int nsel = lists[size_t(cell) * kListStride].x;
        const BigOut *R = BV.res + pp;
        Acc<double> A;
        acc_init(A);
        // two pairs in flight ahead of the one combined
        BigOut b0{}, b1{};
        if (nsel > 0) b0 = R[0];
        if (nsel > 1) b1 = R[BV.cap_ref];
        for (int s = 0; s < nsel; ++s) {
            const BigOut b = b0;
            b0 = b1;
            if (s + 2 < nsel) b1 = R[int64_t(s + 2) * BV.cap_ref];
            const PairOut<double> po{b.d, b.v, b.gx, b.gy, b.gz, b.o, b.u, 0.f, 0.f, 0.f, 0.f, b.c, 0.f};
            pair_accumulate<double, kern_grad(KERN), kern_prop(KERN)>(po, b.n, C, A);
            if (b.best < A.best) { A.best = b.best; A.bidx = b.bidx; }
        }
        finish_query<double, MODE, kern_prop(KERN)>(A, qi, cell, active, Q, Mo.pts, C, O);
    }
}

template <int KERN>
void launch_cm_combine(unsigned grid, hipStream_t s, const float *q, const uint32_t *nref, const uint32_t *rorder,
                       const uint32_t *rcell, const int4 *lists, const ModelView &Mo, const QueryConsts &C,
                       const Outputs &O, const BigView &BV) {
    if (C.combine == GPDF_COMB_HARDMIN)
        hipLaunchKernelGGL((k_cm_combine<KERN, kModeHard>), dim3(grid), dim3(kEvalT), 0, s, q, nref, rorder, rcell,
                           lists, Mo, C, O, BV);
    else if (C.grad_mode == GPDF_GRAD_PAPER_MEAN)
        hipLaunchKernelGGL((k_cm_combine<KERN, kModeMean>), dim3(grid), dim3(kEvalT), 0, s, q, nref, rorder, rcell,
                           lists, Mo, C, O, BV);
    else
        hipLaunchKernelGGL((k_cm_combine<KERN, kModeSmooth>), dim3(grid), dim3(kEvalT), 0, s, q, nref, rorder,
                           rcell, lists, Mo, C, O, BV);
}

// ---------------------------------------------------------------------------
// BF16 precision: the variance product W k of a 64-query chunk and one
// cluster runs on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation) as
// C = W K^T.  Kernel values, the occupancy o = k . alpha and its gradient sum,
// reverting and the combination stay FP32: o is an O(n) sum beside the kernel
// values, and near the surface the reverting scale 1/t (Eq. (3)-(5)) turns a
// BF16 error in o into a gradient wrong by tens of times.
// Lane layout of the 16x16x32 MFMA (lane l, lr = l % 16, lg = l / 16):
//   A[m][k] lane m + 16 (k / 8), element k % 8; B[k][n] lane n + 16 (k / 8),
//   element k % 8; D[m][n] lane n + 16 (m / 4), element m % 4.
// W is kept per cluster in BF16, row-major, rows padded to 16 and columns to
// 32 (zero above the diagonal).  Clusters above kBfMaxN points use the FP32
// path.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kBfMaxN = 256;

__host__ __device__ inline int bf_rows(int n) { return (n + 15) & ~15; }
__host__ __device__ inline int bf_cols(int n) { return (n + 31) & ~31; }

// index of W(i, j), j <= i, in the FP32 query layout
__device__ inline int64_t w_index(int n, int i, int j) {
    if (n <= kPanel) return int64_t(i) * (i + 1) / 2 + j;
    const int r = i / kPanel;
    return w32_panel_offset(n, r) + int64_t(j) * kPanel + (i - r * kPanel);
}

// one workgroup per cluster: BF16 W from the FP32 factor
__global__ void k_pack_bf16(const int32_t *__restrict__ coff, const int64_t *__restrict__ woff,
                            const int64_t *__restrict__ bfoff, const uint8_t *__restrict__ pd,
                            const float *__restrict__ W32, const float4 *__restrict__ pts,
                            __bf16 *__restrict__ M) {
    const int c = blockIdx.x;
    const int base = coff[c], n = coff[c + 1] - base;
    if (n > kBfMaxN || !pd[c]) return;
    const int rows = bf_rows(n), cols = bf_cols(n);
    __bf16 *Mc = M + bfoff[c];
    const float *W = W32 + woff[c];
    for (int idx = threadIdx.x; idx < rows * cols; idx += blockDim.x) {
        const int i = idx / cols, j = idx - i * cols;
        float v = 0.f;
        if (i < n && j <= i) v = W[w_index(n, i, j)];
        Mc[idx] = (__bf16)v;
    }
}

// one point of the BF16 path: kernel value (returned), occupancy and gradient
// sums and the nearest-point decision, FP32
template <int KERN>
__device__ __forceinline__ float point_eval_b(const float4 p, const QueryPoint &Q, int gidx,
                                              const QueryConsts &C, PairRaw<float> &r, Acc<float> &A) {
    const float dx = Q.fx - p.x, dy = Q.fy - p.y, dz = Q.fz - p.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (r2 < A.best) { A.best = r2; A.bidx = gidx; }
    float k, e, t;
    if (kern_kind(KERN) == GPDF_KERNEL_MATERN32) {
        t = fsqrt(r2) * C.a;
        e = fexp2(-t * kLog2e);
        k = fmaf(t, e, e);
    } else {
        t = r2 * C.a;
        k = fexp2(-t * kLog2e);
        e = k;
    }
    r.o = fmaf(p.w, k, r.o);
    // error scale of the term alpha k, as in the FP32 path
    const float akt = fabsf(p.w) * fmaf(k, t, k);
    r.S = fmaf(akt, akt, r.S);
    const float cg = p.w * e;
    r.gx = fmaf(cg, dx, r.gx);
    r.gy = fmaf(cg, dy, r.gy);
    r.gz = fmaf(cg, dz, r.gz);
    return k;
}

__device__ __forceinline__ float pick4(const float (&v)[4], int i) {
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}

template <int KERN>
__device__ void eval_cluster_bf16(int base, int n, int64_t bfo, const float4 *__restrict__ pts,
                                  const __bf16 *__restrict__ Mall, __bf16 *Kt, int kts,
                                  const QueryPoint &Q, const QueryConsts &C, Acc<float> &A) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    PairRaw<float> r{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int cols = bf_cols(n), rows = n;
    const float4 *P = pts + base;
    // this lane's kernel vector, BF16, as row `lane` of K (LDS)
    __bf16 *kr = Kt + lane * kts;
    for (int j = 0; j < cols; ++j) {
        float k = 0.f;
        if (j < n) k = point_eval_b<KERN>(P[j], Q, base + j, C, r, A);
        kr[j] = (__bf16)k;
    }
    __syncthreads();
    const __bf16 *M = Mall + bfo;
    float ssp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < rows; p0 += 64) {
        f32x4 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // columns this panel needs: up to its last W row
        const int kend = min(cols, (p0 + 64 + 31) & ~31);
        for (int k0 = 0; k0 < kend; k0 += 32) {
            bf16x8 b[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                b[nt] = *reinterpret_cast<const bf16x8 *>(Kt + (16 * nt + lr) * kts + k0 + 8 * lg);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int row0 = p0 + 16 * mt;
                if (row0 >= rows) break;
                // blocks above the diagonal of W are zero
                if (k0 > row0 + 15) continue;
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(M + int64_t(row0 + lr) * cols + k0 + 8 * lg);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nt], acc[mt][nt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = p0 + 16 * mt + 4 * lg + e;
                    const float v = acc[mt][nt][e];
                    if (i < n) ssp[nt] = fmaf(v, v, ssp[nt]);
                }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        ssp[nt] += __shfl_xor(ssp[nt], 16, 64);
        ssp[nt] += __shfl_xor(ssp[nt], 32, 64);
    }
    // query of this lane: column lr of tile lg
    r.ss = pick4(ssp, lg);
    __syncthreads();  // K is rewritten by the next cluster
    finish_pair<float, KERN>(r, n, C, A);
}

// ---------------------------------------------------------------------------
// FP32 on MFMA: the variance product W k of a 64-query chunk and one cluster
// as C = W K^T with v_mfma_f32_16x16x4_f32, FP32 operands and accumulation.
// Everything else is the FP32 path (kernel values, sums, reverting, error
// estimate and the FP64 re-evaluation of every output).
// Lane layout (lane l, lr = l % 16, lg = l / 16): A[m][k] lane m + 16 k,
// B[k][n] lane n + 16 k, D[m][n] lane n + 16 (m / 4), element m % 4
// (checked on the device).  W is read from the FP32 factor in the query
// layout; the kernel values sit in LDS, one row of kts floats per query (kts
// odd, so that the 16 rows one MFMA operand reads lie in distinct banks).
// Clusters above kF32mMaxN points use the VALU path.
// ---------------------------------------------------------------------------
constexpr int kF32mMaxN = 248;

template <int KERN>
__device__ void eval_cluster_f32m(int base, int n, int64_t woff, const float4 *__restrict__ pts,
                                  const float *__restrict__ W32, float *Kt, int kts, const QueryPoint &Q,
                                  const QueryConsts &C, Acc<float> &A) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    PairRaw<float> r{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int cols = (n + 3) & ~3;
    const float4 *P = pts + base;
    float *kr = Kt + lane * kts;
    for (int j = 0; j < cols; ++j) {
        float k = 0.f;
        if (j < n) {
            const float4 p = P[j];
            k = point_eval<float, KERN>(p, p.w, Q, base + j, C, r, A);
        }
        kr[j] = k;
    }
    __syncthreads();
    const float *W = W32 + woff;
    float ssp[4] = {0.f, 0.f, 0.f, 0.f};
    for (int p0 = 0; p0 < n; p0 += 64) {
        f32x4 acc[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // columns this row panel needs: up to its last row
        const int kend = min(cols, (p0 + 64 + 3) & ~3);
        for (int k0 = 0; k0 < kend; k0 += 4) {
            float b[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) b[nt] = Kt[(16 * nt + lr) * kts + k0 + lg];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int row0 = p0 + 16 * mt;
                if (row0 >= n) break;
                // blocks above the diagonal of W are zero
                if (k0 > row0 + 15) continue;
                const int i = row0 + lr, j = k0 + lg;
                const float a = (i < n && j <= i) ? W[w_index(n, i, j)] : 0.f;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[nt], acc[mt][nt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = p0 + 16 * mt + 4 * lg + e;
                    const float v = acc[mt][nt][e];
                    if (i < n) ssp[nt] = fmaf(v, v, ssp[nt]);
                }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        ssp[nt] += __shfl_xor(ssp[nt], 16, 64);
        ssp[nt] += __shfl_xor(ssp[nt], 32, 64);
    }
    // query of this lane: column lr of tile lg
    r.ss = pick4(ssp, lg);
    __syncthreads();  // K is rewritten by the next cluster
    finish_pair<float, KERN>(r, n, C, A);
}

// min_n: clusters of min_n to kF32mMaxN points take the MFMA product, the
// others the VALU path (the size bucket boundary the autotuner picks)
template <int KERN, int MODE>
__global__ __launch_bounds__(kEvalT) void k_query_cells_f32m(const float *__restrict__ q, Grouping G,
                                                             const int4 *__restrict__ lists, ModelView Mo, int kts,
                                                             int min_n, QueryConsts C, Outputs O) {
    extern __shared__ float Kf[];
    const uint32_t nch = *ro(G.nchunks);
    const uint32_t wave = xcd_item(nch);
    const int lane = threadIdx.x & 63;
    if (wave >= nch) return;
    const uint2 ch = ro(G.chunk)[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(ro(G.cell_cnt)[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = G.order[ro(G.cell_off)[cell] + start + (active ? lane : 0)];
    const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
    const RoPtr<int4> L = ro(lists + size_t(cell) * kListStride);
    const int nsel = int(uniform(uint32_t(L[0].x)));
    Acc<float> A;
    acc_init(A);
    uint32_t sum_n = 0, sum_tri = 0;
    for (int s = 0; s < nsel; ++s) {
        const int4 d = L[1 + s];
        const int base = int(uniform(uint32_t(d.y))), n = int(uniform(uint32_t(d.z)));
        const int64_t woff = int64_t(uniform(uint32_t(d.w)));
        if (n >= min_n && n <= kF32mMaxN)
            eval_cluster_f32m<KERN>(base, n, woff, Mo.pts, Mo.W32, Kf, kts, Q, C, A);
        else
            eval_cluster<float, KERN>(base, n, woff, Mo.pts, Mo.alpha64, Mo.beta32, Mo.beta64, Mo.W32, Mo.W64, Q, C, A);
        sum_n += uint32_t(n);
        sum_tri += uint32_t(n * (n + 1) / 2);
    }
    finish_query<float, MODE>(A, qi, cell, active, Q, Mo.pts, C, O);
    if (lane == 0 && nsel > 0) {
        spread_add(O.spread, ST_PAIRS, (unsigned long long)nsel * cnt);
        spread_add(O.spread, ST_POINTS, (unsigned long long)sum_n * cnt);
        spread_add(O.spread, ST_TRI, (unsigned long long)sum_tri * cnt);
    }
}

template <int KERN, int MODE>
__global__ __launch_bounds__(kEvalT) void k_query_cells_bf16(const float *__restrict__ q, Grouping G,
                                                             const int4 *__restrict__ lists, ModelView Mo,
                                                             const __bf16 *__restrict__ Mbf,
                                                             const int64_t *__restrict__ bfoff, int kts,
                                                             QueryConsts C, Outputs O) {
    extern __shared__ __bf16 Kt[];
    const uint32_t nch = *ro(G.nchunks);
    const uint32_t wave = xcd_item(nch);
    const int lane = threadIdx.x & 63;
    if (wave >= nch) return;
    const uint2 ch = ro(G.chunk)[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(ro(G.cell_cnt)[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = G.order[ro(G.cell_off)[cell] + start + (active ? lane : 0)];
    const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
    const RoPtr<int4> L = ro(lists + size_t(cell) * kListStride);
    const int nsel = int(uniform(uint32_t(L[0].x)));
    Acc<float> A;
    acc_init(A);
    uint32_t sum_n = 0, sum_tri = 0;
    for (int s = 0; s < nsel; ++s) {
        const int4 d = L[1 + s];
        const int cid = int(uniform(uint32_t(d.x)));
        const int base = int(uniform(uint32_t(d.y))), n = int(uniform(uint32_t(d.z)));
        if (n <= kBfMaxN)
            eval_cluster_bf16<KERN>(base, n, bfoff[cid], Mo.pts, Mbf, Kt, kts, Q, C, A);
        else
            eval_cluster<float, KERN>(base, n, int64_t(uniform(uint32_t(d.w))), Mo.pts, Mo.alpha64, Mo.beta32,
                                      Mo.beta64, Mo.W32, Mo.W64, Q, C, A);
        sum_n += uint32_t(n);
        sum_tri += uint32_t(n * (n + 1) / 2);
    }
    finish_query<float, MODE>(A, qi, cell, active, Q, Mo.pts, C, O);
    if (lane == 0 && nsel > 0) {
        spread_add(O.spread, ST_PAIRS, (unsigned long long)nsel * cnt);
        spread_add(O.spread, ST_POINTS, (unsigned long long)sum_n * cnt);
        spread_add(O.spread, ST_TRI, (unsigned long long)sum_tri * cnt);
    }
}

// squared FP64 distance from x to the centre of cell key k, no contraction,
// accumulated over x, y, z in that order
__device__ inline double centre_d2(const QueryPoint &Q, uint64_t k, double edge) {
    int64_t c[3];
    unpack_key(k, c);
    const float x[3] = {Q.fx, Q.fy, Q.fz};
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ctr = __dmul_rn(__dadd_rn(double(c[a]), 0.5), edge);
        const double dd = __dsub_rn(double(x[a]), ctr);
        d2 = __dadd_rn(d2, __dmul_rn(dd, dd));
    }
    return d2;
}

__device__ inline int wave_min_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// the Q nearest usable clusters of a query by FP64 distance from the query to
// the cell centre, ties to the smaller key (= smaller index): bd/bi hold the
// best Q as (distance^2, index) in ascending order (index 0x7fffffff for an
// empty place)
__device__ inline void knn_insert(double d2, int ci, int Qn, double *bd, int *bi, double &worst) {
    if (d2 > worst) return;   // an equal distance may still enter by its smaller index
    double cd = d2;
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) {
        // keep (distance, index) order; an equal distance stays behind the
        // smaller index
        if (j < Qn && (cd < bd[j] || (cd == bd[j] && ci < bi[j]))) {
            const double td = bd[j];
            const int ti = bi[j];
            bd[j] = cd;
            bi[j] = ci;
            cd = td;
            ci = ti;
        }
    }
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j)
        if (j == Qn - 1) worst = bd[j];
}

// Shells of cells at Chebyshev distance r = 0, 1, 2, ... around the query's
// cell, looked up in the cluster hash.  A cell of shell r + 1 has its centre
// at least (r + 1/2) edge from the query along one axis, so the search ends
// once Q clusters are held and the Q-th is nearer than that (with a margin
// for the FP64 rounding of the squared distances).  Beyond kKnnShells shells
// (fewer than Q clusters nearby) every cluster is scanned.  The result is the
// brute-force selection.
constexpr int kKnnShells = 8;
__device__ inline void knn_select(const QueryPoint &Q, const ModelView &Mo, const QueryConsts &C, int Qn, double *bd,
                                  int *bi) {
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) { bd[j] = INFINITY; bi[j] = 0x7fffffff; }
    double worst = INFINITY;
    int64_t cq[3];
    const float xq[3] = {Q.fx, Q.fy, Q.fz};
    bool done = false;
    if (query_cell(xq, C.hv > 0.0 ? 1 : 0, C.hv, C.hc, cq)) {
        auto in_range = [](int64_t v) { return v >= -kBias && v < kBias; };
        for (int r = 0; r <= kKnnShells && !done; ++r) {
            for (int dx = -r; dx <= r; ++dx)
                for (int dy = -r; dy <= r; ++dy)
                    for (int dz = -r; dz <= r; ++dz) {
                        if (max(abs(dx), max(abs(dy), abs(dz))) != r) continue;
                        const int64_t nx = cq[0] + dx, ny = cq[1] + dy, nz = cq[2] + dz;
                        if (!(in_range(nx) && in_range(ny) && in_range(nz))) continue;
                        const int64_t sl = hash_find(Mo.chash, Mo.cmask, pack_key(nx, ny, nz));
                        if (sl < 0) continue;
                        const int c = Mo.chash_val[sl];
                        if (!Mo.pd[c] || Mo.coff[c + 1] == Mo.coff[c]) continue;
                        knn_insert(centre_d2(Q, Mo.ckey[c], Mo.edge), c, Qn, bd, bi, worst);
                    }
            const double b = (double(r) + 0.5) * Mo.edge;
            done = worst < b * b * (1.0 - 1e-12);
        }
    }
    if (!done) {
        // a non-finite query keeps no cluster (as the brute-force scan, whose
        // distances are then NaN); otherwise scan every cluster
#pragma unroll
        for (int j = 0; j < kMaxKnn; ++j) { bd[j] = INFINITY; bi[j] = 0x7fffffff; }
        worst = INFINITY;
        for (int64_t c = 0; c < Mo.ncl; ++c) {
            if (!Mo.pd[c] || Mo.coff[c + 1] == Mo.coff[c]) continue;
            knn_insert(centre_d2(Q, Mo.ckey[c], Mo.edge), int(c), Qn, bd, bi, worst);
        }
    }
}

// lazy training: mark the clusters that the queries select and that are not
// trained yet (the Q nearest of each query)
__global__ void k_lazy_mark_knn(const float *__restrict__ q, int64_t m, ModelView Mo, QueryConsts C,
                                const uint8_t *__restrict__ trained, uint8_t *__restrict__ need) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const QueryPoint Q{q[3 * j], q[3 * j + 1], q[3 * j + 2]};
    double bd[kMaxKnn];
    int bi[kMaxKnn];
    knn_select(Q, Mo, C, C.knn_q, bd, bi);
#pragma unroll
    for (int k = 0; k < kMaxKnn; ++k)
        if (k < C.knn_q && bi[k] != 0x7fffffff && !trained[bi[k]]) need[bi[k]] = 1;
}

// ... and the clusters of the 27 cells around each query cell
__global__ void k_lazy_mark_cells(int64_t ncb, const uint32_t *__restrict__ dnc,
                                  const uint64_t *__restrict__ cell_key, ModelView Mo,
                                  const uint8_t *__restrict__ trained, uint8_t *__restrict__ need) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(ncb, dnc)) return;
    int64_t cc[3];
    unpack_key(cell_key[c], cc);
    auto in_range = [](int64_t v) { return v >= -kBias && v < kBias; };
    for (int t = 0; t < 27; ++t) {
        const int64_t nx = cc[0] + t / 9 - 1, ny = cc[1] + (t / 3) % 3 - 1, nz = cc[2] + t % 3 - 1;
        if (!(in_range(nx) && in_range(ny) && in_range(nz))) continue;
        const int64_t sl = hash_find(Mo.chash, Mo.cmask, pack_key(nx, ny, nz));
        if (sl < 0) continue;
        const int id = Mo.chash_val[sl];
        if (Mo.pd[id] && Mo.coff[id + 1] > Mo.coff[id] && !trained[id]) need[id] = 1;
    }
}

// KNN: each lane picks its Q nearest clusters by cell-centre distance (ties
// to the smaller key); the wavefront walks the union of the lanes' lists in
// ascending cluster order and each lane evaluates exactly its own clusters
template <typename T, int KERN, int MODE>
__global__ __launch_bounds__(kEvalT) void k_query_knn(const float *__restrict__ q, Grouping G,
                                                   ModelView Mo, QueryConsts C, Outputs O) {
    __shared__ int32_t lst[kWaves][kMaxKnn][64];
    const int wv = threadIdx.x >> 6;
    const uint32_t wave = blockIdx.x * kWaves + wv;
    const int lane = threadIdx.x & 63;
    if (wave >= *ro(G.nchunks)) return;
    const uint2 ch = ro(G.chunk)[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(ro(G.cell_cnt)[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = G.order[ro(G.cell_off)[cell] + start + (active ? lane : 0)];
    const QueryPoint Q{q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
    const int Qn = C.knn_q;
    double bd[kMaxKnn];
    int bi[kMaxKnn];
    knn_select(Q, Mo, C, Qn, bd, bi);
    // ascending cluster index (= ascending key)
#pragma unroll
    for (int a = 1; a < kMaxKnn; ++a)
#pragma unroll
        for (int b = kMaxKnn - 1; b >= a; --b)
            if (bi[b] < bi[b - 1]) { const int t = bi[b]; bi[b] = bi[b - 1]; bi[b - 1] = t; }
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) lst[wv][j][lane] = bi[j];
    Acc<T> A;
    acc_init(A);
    int ptr = 0;
    while (true) {
        const int mine = (active && ptr < Qn) ? lst[wv][ptr][lane] : 0x7fffffff;
        const int c = int(uniform(uint32_t(wave_min_i32(mine))));
        if (c == 0x7fffffff) break;
        if (mine == c) {
            ++ptr;
            const int base = int(uniform(uint32_t(Mo.coff[c])));
            const int n = int(uniform(uint32_t(Mo.coff[c + 1]))) - base;
            eval_cluster<T, KERN>(base, n, Mo.woff[c], Mo.pts, Mo.alpha64, Mo.beta32, Mo.beta64, Mo.W32, Mo.W64, Q, C, A);
        }
    }
    finish_query<T, MODE, kern_prop(KERN)>(A, qi, cell, active, Q, Mo.pts, C, O);
}

// grid: one workgroup per chunk (an upper bound); with work != NULL the
// persistent grid
template <typename T, int KERN, int MODE>
void launch_query(bool knn, unsigned grid, hipStream_t s, const float *q, const Grouping &G,
                  const int4 *lists, const ModelView &Mo, const QueryConsts &C, const Outputs &O,
                  uint32_t *work, uint32_t *covered = nullptr, uint32_t *aux = nullptr) {
    // property launches: NEIGHBOR27 (the caller rejects the other
    // combinations), one workgroup per chunk, or persistent given a counter
    if constexpr (kern_prop(KERN)) {
        if (work)
            hipLaunchKernelGGL((k_query_cells<T, KERN, MODE, true>), dim3(grid), dim3(kEvalT), 0, s, q, G, lists,
                               Mo, C, O, work, nullptr);
        else
            hipLaunchKernelGGL((k_query_cells<T, KERN, MODE, false>), dim3(grid), dim3(kEvalT), 0, s, q, G, lists,
                               Mo, C, O, nullptr, nullptr);
    } else if (knn) {
        hipLaunchKernelGGL((k_query_knn<T, KERN, MODE>), dim3(grid), dim3(kEvalT), 0, s, q, G, Mo, C, O);
    } else if (work) {
        hipLaunchKernelGGL((k_query_cells<T, KERN, MODE, true>), dim3(grid), dim3(kEvalT), 0, s, q, G, lists,
                           Mo, C, O, work, aux);
    } else {
        // covered: the one-chunk instance that records its share (a captured
        // frame's FP32 evaluation without gradient, the only one it has)
        if constexpr (std::is_same<T, float>::value && !kern_grad(KERN)) {
            if (covered) {
                hipLaunchKernelGGL((k_query_cells<T, KERN, MODE, false, true>), dim3(grid), dim3(kEvalT), 0, s, q, G,
                                   lists, Mo, C, O, covered, aux);
                return;
            }
        }
        hipLaunchKernelGGL((k_query_cells<T, KERN, MODE, false>), dim3(grid), dim3(kEvalT), 0, s, q, G, lists,
                           Mo, C, O, work, nullptr);
    }
}

template <typename T, int KERN>
void launch_query_m(bool knn, unsigned grid, hipStream_t s, const float *q, const Grouping &G,
                    const int4 *lists, const ModelView &Mo, const QueryConsts &C, const Outputs &O,
                    uint32_t *work, uint32_t *covered = nullptr, uint32_t *aux = nullptr) {
    if (C.combine == GPDF_COMB_HARDMIN)
        launch_query<T, KERN, kModeHard>(knn, grid, s, q, G, lists, Mo, C, O, work, covered, aux);
    else if (C.grad_mode == GPDF_GRAD_PAPER_MEAN)
        launch_query<T, KERN, kModeMean>(knn, grid, s, q, G, lists, Mo, C, O, work, covered, aux);
    else
        launch_query<T, KERN, kModeSmooth>(knn, grid, s, q, G, lists, Mo, C, O, work, covered, aux);
}

template <int KERN>
void launch_bf16_m(unsigned grid, size_t lds, hipStream_t s, const float *q, const Grouping &G, const int4 *lists,
                   const ModelView &Mo, const __bf16 *Mbf, const int64_t *bfoff, int kts, const QueryConsts &C,
                   const Outputs &O) {
    if (C.combine == GPDF_COMB_HARDMIN)
        hipLaunchKernelGGL((k_query_cells_bf16<KERN, kModeHard>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists, Mo,
                           Mbf, bfoff, kts, C, O);
    else if (C.grad_mode == GPDF_GRAD_PAPER_MEAN)
        hipLaunchKernelGGL((k_query_cells_bf16<KERN, kModeMean>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists, Mo,
                           Mbf, bfoff, kts, C, O);
    else
        hipLaunchKernelGGL((k_query_cells_bf16<KERN, kModeSmooth>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists,
                           Mo, Mbf, bfoff, kts, C, O);
}

template <typename T, int PF>
void launch_query_kf(int kernel, bool knn, unsigned grid, hipStream_t s, const float *q, const Grouping &G,
                     const int4 *lists, const ModelView &Mo, const QueryConsts &C, const Outputs &O,
                     uint32_t *work, uint32_t *covered = nullptr, uint32_t *aux = nullptr) {
    if constexpr (std::is_same<T, float>::value) {
        if (!O.grad) {
            if (kernel == GPDF_KERNEL_MATERN32)
                launch_query_m<T, GPDF_KERNEL_MATERN32 | kNoGrad | PF>(knn, grid, s, q, G, lists, Mo, C, O, work,
                                                                       covered, aux);
            else
                launch_query_m<T, GPDF_KERNEL_SE | kNoGrad | PF>(knn, grid, s, q, G, lists, Mo, C, O, work, covered,
                                                                 aux);
            return;
        }
    }
    if (kernel == GPDF_KERNEL_MATERN32)
        launch_query_m<T, GPDF_KERNEL_MATERN32 | PF>(knn, grid, s, q, G, lists, Mo, C, O, work);
    else
        launch_query_m<T, GPDF_KERNEL_SE | PF>(knn, grid, s, q, G, lists, Mo, C, O, work);
}

template <int KERN>
void launch_f32m_m(unsigned grid, size_t lds, hipStream_t s, const float *q, const Grouping &G, const int4 *lists,
                   const ModelView &Mo, int kts, int min_n, const QueryConsts &C, const Outputs &O) {
    if (C.combine == GPDF_COMB_HARDMIN)
        hipLaunchKernelGGL((k_query_cells_f32m<KERN, kModeHard>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists, Mo,
                           kts, min_n, C, O);
    else if (C.grad_mode == GPDF_GRAD_PAPER_MEAN)
        hipLaunchKernelGGL((k_query_cells_f32m<KERN, kModeMean>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists, Mo,
                           kts, min_n, C, O);
    else
        hipLaunchKernelGGL((k_query_cells_f32m<KERN, kModeSmooth>), dim3(grid), dim3(kEvalT), lds, s, q, G, lists,
                           Mo, kts, min_n, C, O);
}

template <typename T>
void launch_query_k(gpdf_ctx *c, int kernel, bool knn, unsigned grid, hipStream_t s, const float *q,
                    const Grouping &G, const int4 *lists, const ModelView &Mo,
                    const QueryConsts &C, const Outputs &O, int slot) {
    if (O.prop || O.prop_var) {
        launch_query_kf<T, kProp>(kernel, knn, grid, s, q, G, lists, Mo, C, O, nullptr);
        return;
    }
    uint32_t *work = nullptr;
    // In a captured graph the FP32 evaluation is one workgroup per chunk
    // over the first g chunks, g set before each replay from the chunk count
    // of the last one (the node's grid; the graph runs no count back to the
    // host), then the persistent instance over the chunks from g on (none
    // unless the count grew).  The first launch writes how many chunks it
    // took, where the second starts, so the split holds whatever grid a
    // replay runs with, and the chunk count to pinned host memory.  The persistent instance alone costs more: the loop around the
    // chunk keeps the launch's arguments in scalar registers and spills them.
    if (std::is_same<T, float>::value && c->capturing && c->d_gfirst && !knn && !O.grad &&
        c->tune.eval_persistent == 0 && !c->geval_node) {
        work = c->d_work + int64_t(slot) * kWorkSlot;
        fill_u32(work, 0u, kWorkSlot, s);
        const unsigned g0 = std::min<unsigned>(grid, kGraphEvalGrid0);
        launch_query_kf<T, 0>(kernel, knn, g0, s, q, G, lists, Mo, C, O, nullptr, c->d_gfirst, c->d_gchunks);
        hipStreamCaptureStatus cs;
        const hipGraphNode_t *deps = nullptr;
        size_t nd = 0;
        if (hipStreamGetCaptureInfo_v2(s, &cs, nullptr, nullptr, &deps, &nd) == hipSuccess && nd == 1) {
            c->geval_node = deps[0];
            c->geval_grid0 = g0;
            c->geval_gridmax = grid;
        }
        launch_query_kf<T, 0>(kernel, knn, std::min<unsigned>(grid, 1024u), s, q, G, lists, Mo, C, O, work, nullptr,
                              c->d_gfirst);
        return;
    }
    // persistent when tuned so, and always in a captured graph otherwise;
    // the FP32 instance holds four wavefronts per SIMD
    const int per = c->tune.eval_persistent > 0 ? c->tune.eval_persistent : (c->capturing ? 4 : 0);
    if (per > 0 && !knn) {
        // 256 CUs x 4 SIMDs x the wavefronts per SIMD
        work = c->d_work + int64_t(slot) * kWorkSlot;
        fill_u32(work, 0u, kWorkSlot, s);
        grid = std::min<unsigned>(grid, 1024u * unsigned(per));
    }
    launch_query_kf<T, 0>(kernel, knn, grid, s, q, G, lists, Mo, C, O, work);
}

}  // namespace

// ---------------------------------------------------------------------------
// Per-cell cluster lists of gpdf_query_distance_noalloc: a fixed array in
// device memory instead of the context's buffer (which a call grows when it
// meets more cells than before), for callers that cannot allocate.  Each GPU
// holds one copy of the array for the life of the process, shared by every
// call on that GPU.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int4 scratch[size_t(kNoAllocCells) * kCellListStride];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int4 *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's copy of `scratch`, taken once per device with
// that device current (the host-side name is not a device address).
gpdf_status scratch_setup(gpdf_ctx *c) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(c, e, "scratch: device");
    if (dev < 0 || dev >= kMaxDevices) return fail(c, GPDF_E_INVALID_ARG, "scratch: device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail(c, e, "scratch: symbol address");
        g_scratch_ptr[dev] = static_cast<int4 *>(ptr);
    }
    c->scratch_lists = g_scratch_ptr[dev];
    return GPDF_OK;
}

QueryConsts make_consts(const gpdf_params &p, const float *origin, const float *d_origin) {
    QueryConsts C{};
    const bool matern = p.kernel == GPDF_KERNEL_MATERN32;
    C.ad = matern ? 1.7320508075688772935 / p.length_scale : 1.0 / (2.0 * p.length_scale * p.length_scale);
    C.cd = matern ? p.length_scale / 1.7320508075688772935 : p.length_scale;
    C.l = float(p.length_scale);
    C.a = float(C.ad);
    C.c = float(C.cd);
    C.lam = float(p.smooth_min_lambda);
    C.omin = float(p.occ_min);
    C.omax = float(p.occ_max);
    // thresholds 5x inside the distance (1e-4 m) and gradient (1e-3)
    // tolerances; relative variance held to 1e-3.  err_c scales the
    // root-sum-square rounding estimate (a probabilistic, not worst-case,
    // estimate); at 2 the results left in FP32 stay at least 4x inside the
    // tolerances on the sphere, LiDAR and planar-patch workloads
    C.tau_d = 2e-5f;
    C.tau_g = 2e-4f;
    C.tau_v = 1e-3f;
    // surface property: 2e-5 in the property's own units (intensities and
    // colour channels in [0, 1]), 5x inside a 1e-4 tolerance, as the distance
    C.tau_c = 2e-5f;
    C.err_c = 2.f;
    C.kernel = p.kernel;
    C.combine = p.combine;
    C.grad_mode = p.grad_mode;
    C.knn_q = p.selection == GPDF_SEL_KNN ? p.knn_q : 0;
    C.signed_ = origin != nullptr || d_origin != nullptr;
    if (origin) { C.ox = origin[0]; C.oy = origin[1]; C.oz = origin[2]; }
    C.d_origin = d_origin;
    // distance, Lambda and gradient scale at the two caps, in FP64
    auto cap = [&](double o, double *out) {
        if (matern) {
            // t >= 0 with (1 + t) e^{-t} = o: Newton from the branch-point
            // series (o near 1) or the asymptote t = y + log(1 + t), y = -log o
            const double y = -std::log(o);
            double t = o > 0.5 ? std::sqrt(2.0 * (1.0 - o)) : y + std::log(1.0 + y + std::log(1.0 + y));
            for (int it = 0; it < 60; ++it) {
                const double E = std::exp(-t), f = (1.0 + t) * E - o;
                const double tn = t + f / (t * E);
                if (tn == t) break;
                t = tn;
            }
            const double tE = t * std::exp(-t);
            out[0] = C.cd * t;
            out[1] = -C.cd / tE;
            out[2] = C.ad / tE;
        } else {
            const double dd = C.cd * std::sqrt(-2.0 * std::log(o));
            out[0] = dd;
            out[1] = -C.cd * C.cd / (o * dd);
            out[2] = 1.0 / (o * dd);
        }
    };
    cap(p.occ_max, C.cap_hid);
    cap(p.occ_min, C.cap_lod);
    for (int k = 0; k < 3; ++k) {
        C.cap_hi[k] = float(C.cap_hid[k]);
        C.cap_lo[k] = float(C.cap_lod[k]);
    }
    C.ld = p.length_scale;
    C.sd = p.noise_sigma;
    C.hv = p.voxel_size;
    C.hc = p.cluster_size;
    C.lamd = p.smooth_min_lambda;
    C.omind = p.occ_min;
    C.omaxd = p.occ_max;
    return C;
}

// per-cell cluster lists for at least cap cells (reallocated when larger)
hipError_t ensure_cell_lists(gpdf_ctx *c, int64_t cap) {
    if (cap <= c->cap_cells) return hipSuccess;
    hipError_t e;
    if (c->d_cell_list && (e = hipFree(c->d_cell_list)) != hipSuccess) return e;
    c->d_cell_list = nullptr;
    c->cap_cells = 0;
    if ((e = hipMalloc((void **)&c->d_cell_list, sizeof(int4) * size_t(cap) * kCellListStride)) != hipSuccess)
        return e;
    c->cap_cells = cap;
    return hipSuccess;
}

// BF16 copies of [W; alpha] for the current model (once per training)
gpdf_status build_bf16(gpdf_ctx *c) {
    Model &M = c->model;
    if (M.bf16_ready) return GPDF_OK;
    hipStream_t s = c->stream;
    hipError_t e;
    const int64_t ncl = M.nclusters;
    std::vector<int32_t> coff(size_t(ncl) + 1);
    if ((e = hipMemcpyAsync(coff.data(), c->d_coff, sizeof(int32_t) * (size_t(ncl) + 1), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(c, e, "bf16: read offsets");
    std::vector<int64_t> &off = c->h_bfoff;
    off.assign(size_t(ncl), 0);
    int64_t tot = 0;
    for (int64_t i = 0; i < ncl; ++i) {
        const int n = coff[size_t(i) + 1] - coff[size_t(i)];
        off[size_t(i)] = tot;
        if (n <= kBfMaxN) tot += int64_t(bf_rows(n)) * bf_cols(n);
    }
    if (tot > c->cap_bfM) {
        if (c->d_bfM && (e = hipFree(c->d_bfM)) != hipSuccess) return hip_fail(c, e, "bf16: free");
        c->d_bfM = nullptr;
        c->cap_bfM = 0;
        const int64_t cap = tot + tot / 4 + 4096;
        if ((e = hipMalloc(&c->d_bfM, sizeof(__bf16) * size_t(cap))) != hipSuccess) return hip_fail(c, e, "bf16: alloc");
        c->cap_bfM = cap;
    }
    if (ncl > c->cap_bfoff) {
        if (c->d_bfoff && (e = hipFree(c->d_bfoff)) != hipSuccess) return hip_fail(c, e, "bf16: free");
        c->d_bfoff = nullptr;
        c->cap_bfoff = 0;
        if ((e = hipMalloc((void **)&c->d_bfoff, sizeof(int64_t) * size_t(ncl))) != hipSuccess)
            return hip_fail(c, e, "bf16: alloc");
        c->cap_bfoff = ncl;
    }
    if ((e = hipMemcpyAsync(c->d_bfoff, off.data(), sizeof(int64_t) * size_t(ncl), hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return hip_fail(c, e, "bf16: offsets");
    hipLaunchKernelGGL(k_pack_bf16, dim3(unsigned(ncl)), dim3(256), 0, s, c->d_coff, c->d_woff, c->d_bfoff, c->d_pd,
                       c->d_W32, c->d_pts, static_cast<__bf16 *>(c->d_bfM));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "bf16: pack");
    M.bf16_ready = true;
    return GPDF_OK;
}

// the cluster bound of the cluster-major pass (the device count is the exact one)
static int64_t cm_cluster_bound(const gpdf_ctx *c, const Model &M) {
    return std::max<int64_t>(M.host_counts ? M.nclusters : c->p.max_clusters, 1);
}

// The cluster-major FP64 pass over the refine records and chunk table just
// built: pair counts per cluster, run offsets (clusters of at most one panel
// first), the items of both size classes, each pair's query and result
// slot, then the evaluation kernels.  bcnt is cleared by the caller.
static BigView refine_cm(gpdf_ctx *c, const Model &M, hipStream_t s, const float *d_q, const int4 *lists,
                         const ModelView &Mo, const QueryConsts &C, int64_t m, bool want_prop) {
    uint32_t *cnt = c->d_cnt;
    const int64_t ncl = cm_cluster_bound(c, M);
    const uint32_t *dncl = cnt + CNT_CL;
    const unsigned long long *nrec = c->d_stat + ST_REFINE;
    hipLaunchKernelGGL(k_cm_count, dim3(1024), dim3(kQT), 0, s, c->d_rchunk, cnt + CNT_RCHUNKS, c->cap_bchunks,
                       c->d_rcnt, lists, c->d_bcnt, c->d_bbase);
    hipLaunchKernelGGL(k_cm_split, dim3(blocks_for(ncl)), dim3(kQT), 0, s, ncl, dncl, c->d_coff, c->d_bcnt,
                       c->d_bcs, c->d_bcb, c->d_bnits, c->d_bnit);
    ScanList SL;
    SL.add(c->d_bcs, c->d_boffs, cnt + CNT_BPAIRS_S);
    SL.add(c->d_bcb, c->d_boffb, cnt + CNT_BPAIRS_B);
    SL.add(c->d_bnits, c->d_bioffs, cnt + CNT_BITEMS_S);
    SL.add(c->d_bnit, c->d_bioff, cnt + CNT_BITEMS);
    exclusive_scan_u32_multi(SL, ncl, c->d_part, s, dncl, c->capturing);
    const CmTotals T{cnt + CNT_RCHUNKS, cnt + CNT_BPAIRS_S, cnt + CNT_BPAIRS_B, cnt + CNT_MAXN, nrec,
                     c->cap_bchunks, c->cap_bpairs, m, c->cap_bref};
    hipLaunchKernelGGL(k_cm_finish, dim3(blocks_for(ncl)), dim3(kQT), 0, s, ncl, dncl, c->d_coff, T, c->d_boffs,
                       c->d_boffb, c->d_bnits, c->d_bioffs, c->d_bnit, c->d_bioff, c->d_boff, c->d_bitems,
                       c->d_bitem, cnt + CNT_BIGOK, cnt + CNT_NREF_FAST, cnt + CNT_RCH_SLOW);
    hipLaunchKernelGGL(k_cm_fill, dim3(1024), dim3(kQT), 0, s, c->d_refine,
                       nrec, m, c->d_rrank, c->d_roff, c->d_rchunk_off, lists, c->d_bbase, c->d_boff,
                       cnt + CNT_BIGOK, c->cap_bref, c->d_bq, c->d_bdst);
    // kernel values of the largest cluster the large-cluster pass takes
    const int64_t nmax = M.host_counts ? std::min<int64_t>(std::max<int64_t>(M.max_n, 4), kBigMaxN) : kBigMaxN;
    const size_t lds = size_t((nmax + 3) & ~int64_t(3)) * kBigB * sizeof(double);
    BigOut *res = static_cast<BigOut *>(c->d_bres);
    const int kern = c->p.kernel;
#define GPDF_CM(K)                                                                                              \
    do {                                                                                                        \
        hipLaunchKernelGGL((k_cm_small<K>), dim3(3072), dim3(64), 0, s, d_q, c->d_bitems, cnt + CNT_BITEMS_S,    \
                           c->d_bcnt, c->d_boff, c->d_bq, c->d_bdst, Mo, C, cnt + CNT_BIGOK, res);              \
        hipLaunchKernelGGL((k_cm_big<K>), dim3(1024), dim3(kBigT), lds, s, d_q, c->d_bitem, cnt + CNT_BITEMS,    \
                           c->d_bcnt, c->d_boff, c->d_bq, c->d_bdst, Mo, C, cnt + CNT_BIGOK, res);              \
        hipLaunchKernelGGL((k_cm_revert<K>), dim3(2048), dim3(64), 0, s, cnt + CNT_BPAIRS_S, cnt + CNT_BPAIRS_B, \
                           c->d_bdst, C, cnt + CNT_BIGOK, res);                                                 \
    } while (0)
    if (want_prop) {
        if (kern == GPDF_KERNEL_MATERN32) GPDF_CM(GPDF_KERNEL_MATERN32 | kProp);
        else GPDF_CM(GPDF_KERNEL_SE | kProp);
    } else if (kern == GPDF_KERNEL_MATERN32) {
        GPDF_CM(GPDF_KERNEL_MATERN32);
    } else {
        GPDF_CM(GPDF_KERNEL_SE);
    }
#undef GPDF_CM
    return BigView{res, c->cap_bref};
}

gpdf_status query(gpdf_ctx *c, const float *d_q, int64_t m, const float *origin, float *dist,
                  float *grad, float *var, uint8_t *valid, float *aux, int32_t correct, const uint32_t *dm,
                  const float *d_origin, bool noalloc, float *prop, float *prop_var) {
    if (noalloc) {
        // nothing below may allocate: the BF16 copy of the factors is built
        // (and its buffer sized) on the first BF16 query of a training
        if (c->p.precision == GPDF_PREC_BF16)
            return fail(c, GPDF_E_INVALID_ARG, "query_distance_noalloc: BF16 precision is not supported");
        if (!c->scratch_lists) return fail(c, GPDF_E_INVALID_ARG, "query_distance_noalloc: no scratch on this device");
    }
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "query: join");
    hipStream_t s = c->stream;
    const Model &M = c->model;
    const bool eager = dm == nullptr;
    if (!M.trained) return fail(c, GPDF_E_NOT_TRAINED, "query before training");
    if (m < 0 || m > c->p.max_queries) return fail(c, GPDF_E_CAPACITY, "query: m exceeds max_queries");
    if (m > 0 && (!dist || !valid || !d_q)) return fail(c, GPDF_E_INVALID_ARG, "query: null buffer");
    if (origin && !(std::isfinite(origin[0]) && std::isfinite(origin[1]) && std::isfinite(origin[2])))
        return fail(c, GPDF_E_INVALID_ARG, "query: non-finite origin");
    const bool want_prop = prop || prop_var;
    if (want_prop) {
        if (!M.props) return fail(c, GPDF_E_INVALID_ARG, "query: the model was trained without a property");
        if (c->p.precision == GPDF_PREC_BF16 || c->p.precision == GPDF_PREC_FP32_MFMA ||
            c->p.selection != GPDF_SEL_NEIGHBOR27 || noalloc || correct)
            return fail(c, GPDF_E_INVALID_ARG,
                        "query: the property needs FP32 or FP64 precision, NEIGHBOR27 selection, no correction");
    }
    c->last_queries = m;
    uint32_t *cnt = c->d_cnt;
    // per-call counters
    FillList F;
    F.u64(c->d_stat + ST_NONFINITE_Q, 0ull, 1);
    F.u64(c->d_stat + ST_VALID_Q, 0ull, 1);
    F.u64(c->d_stat + ST_REFINE, 0ull, 1);
    F.u64(c->d_stat + ST_CELLS, 0ull, 1);
    F.u64(c->d_stat + ST_PAIRS, 0ull, 3);
    F.u64(c->d_stat + ST_REF_D, 0ull, 3);
    F.u32(cnt + CNT_CELLS, 0u, 3);  // cells, chunks, re-evaluation chunks
    if (m == 0) {
        (void)fill_multi(F, s);
        return GPDF_OK;
    }
    hipError_t e;
    if (M.host_counts && M.nclusters == 0) {
        // nothing to select: every query is invalid
        (void)fill_multi(F, s);
        hipLaunchKernelGGL(k_all_invalid, dim3(blocks_for(m)), dim3(kQT), 0, s, m, dist, grad, var,
                           valid, aux, prop, prop_var);
        return (e = hipGetLastError()) == hipSuccess ? GPDF_OK : hip_fail(c, e, "query launch");
    }
    const QueryConsts C = make_consts(c->p, origin, d_origin);
    const bool vox = c->p.voxel_size > 0.0;
    const bool knn = C.knn_q > 0;
    if (!eager && (knn || c->p.precision == GPDF_PREC_BF16 || c->p.precision == GPDF_PREC_FP32_MFMA || correct)) {
        (void)fill_multi(F, s);
        return fail(c, GPDF_E_INVALID_ARG, "query with device counts: NEIGHBOR27, FP32/FP64, no correction");
    }
    const double edge = vox ? 8.0 * c->p.voxel_size : c->p.cluster_size;
    const int kern = c->p.kernel;
    // without a property the beta pointers alias arrays that no launch reads
    const float *b32 = c->d_beta32 ? c->d_beta32 : c->d_W32;
    const double *b64 = c->d_beta64 ? c->d_beta64 : c->d_alpha64;
    const ModelView Mo{c->d_pts, c->d_alpha64, b32, b64, c->d_coff, c->d_woff, c->d_W32, c->d_W64,
                       c->d_ckey, c->d_pd, M.nclusters, edge, c->d_chash, c->d_chash_val, c->chash_mask};
    // 1. group by cell
    stage_begin(c, GPDF_MS_GROUP);
    // at most m distinct cells (far fewer in practice): a table of 1.25m to
    // 2.5m slots, within the allocation; it is cleared and compacted per call
    const uint32_t qmask = std::min(c->qhash_mask, pow2_mask(m + m / 4 + 1));
    const int64_t qcap = int64_t(qmask) + 1;
    F.u64(c->d_qhash, (unsigned long long)kNoKey, qcap);
    F.u32(c->d_qhash_cnt, 0u, qcap);
    if ((e = fill_multi(F, s)) != hipSuccess) return hip_fail(c, e, "query: clear");
    HashView qh{c->d_qhash, qmask};
    hipLaunchKernelGGL(k_qcells, dim3(blocks_for(m)), dim3(kQT), 0, s, d_q, m, dm, vox ? 1 : 0,
                       c->p.voxel_size, c->p.cluster_size, qh, c->d_qhash_cnt, c->d_qslot, c->d_qrank,
                       dist, grad, var, valid, aux, prop, prop_var, c->d_stat);
    count_occupied(c->d_qhash, qcap, c->d_tile_cnt, c->d_tile_off, c->d_part, s);
    const int64_t ntiles = compact_tiles(qcap);
    hipLaunchKernelGGL(k_cells_compact, dim3(unsigned(ntiles)), dim3(256), 0, s, c->d_qhash,
                       c->d_qhash_cnt, qcap, c->d_tile_off, ntiles, c->d_qhash_cell, c->d_cell_key,
                       c->d_cell_cnt, c->d_cell_chunks, c->d_stat, cnt + CNT_CELLS);
    // the number of cells: read back (eager), else bounded by the queries
    int64_t nc = std::min<int64_t>(m, qcap);
    if (eager) {
        ReadList R;
        R.u32(cnt + CNT_CELLS);
        if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "query: read cell count");
        const uint32_t ncells = uint32_t(c->h_read[0]);
        if (ncells == 0) return GPDF_OK;
        nc = int64_t(ncells);
    }
    const uint32_t *dnc = cnt + CNT_CELLS;
    ScanList CL;
    CL.add(c->d_cell_cnt, c->d_cell_off, nullptr);
    CL.add(c->d_cell_chunks, c->d_chunk_off, cnt + CNT_CHUNKS);
    exclusive_scan_u32_multi(CL, nc, c->d_part, s, dnc, c->capturing);
    hipLaunchKernelGGL(k_chunk_table, dim3(blocks_for(nc)), dim3(kQT), 0, s, nc, dnc, c->d_cell_chunks,
                       c->d_chunk_off, c->d_chunk);
    // lazy training: factor the clusters these queries select, until a
    // round trains none (a cluster found not positive definite leaves the
    // selection, which may then take another)
    if (M.lazy) {
        if (!eager) return fail(c, GPDF_E_INVALID_ARG, "query with device counts on a lazily trained model");
        for (int round = 0; round < 8; ++round) {
            if (knn)
                hipLaunchKernelGGL(k_lazy_mark_knn, dim3(blocks_for(m)), dim3(kQT), 0, s, d_q, m, Mo, C,
                                   c->d_trained, c->d_need);
            else
                hipLaunchKernelGGL(k_lazy_mark_cells, dim3(blocks_for(nc)), dim3(kQT), 0, s, nc, dnc, c->d_cell_key,
                                   Mo, c->d_trained, c->d_need);
            int64_t k = 0;
            const gpdf_status st = lazy_train_round(c, &k);
            if (st != GPDF_OK) return st;
            if (k == 0) break;
        }
    }
    int4 *lists = noalloc ? c->scratch_lists : c->d_cell_list;
    if (!knn && noalloc && nc > kNoAllocCells)
        return fail(c, GPDF_E_CAPACITY,
                    "query_distance_noalloc: the queries fall in " + std::to_string(nc) +
                        " cells, more than the " + std::to_string(kNoAllocCells) + " cell lists of the fixed scratch");
    if (!knn && !noalloc && nc > c->cap_cells) {
        if (!eager) return fail(c, GPDF_E_CAPACITY, "query: cell lists not allocated for the bound");
        // grow the per-cell cluster lists (one reallocation per new maximum)
        const int64_t cap = std::min<int64_t>(c->p.max_queries + 1, nc + nc / 4 + 1024);
        if ((e = ensure_cell_lists(c, cap)) != hipSuccess) return hip_fail(c, e, "query: cell lists");
        lists = c->d_cell_list;
    }
    if (!knn)
        hipLaunchKernelGGL(k_cell_lists, dim3(blocks_for(nc)), dim3(kQT), 0, s, nc, dnc, c->d_cell_key,
                           c->d_chash, c->chash_mask, c->d_chash_val, c->d_pd, c->d_coff,
                           c->d_woff, lists);
    hipLaunchKernelGGL(k_scatter_order, dim3(blocks_for(m)), dim3(kQT), 0, s, c->d_qslot, c->d_qrank, m, dm,
                       c->d_qhash_cell, c->d_cell_off, c->d_order);
    stage_end(c, GPDF_MS_GROUP);
    // 2. evaluation; the chunk count stays on the device (grid is an upper bound)
    const int64_t max_chunks = nc + (m + 63) / 64;
    const unsigned grid = blocks_for(max_chunks * 64, kEvalT);
    const Grouping G{c->d_chunk, cnt + CNT_CHUNKS, c->d_cell_cnt, c->d_cell_off, c->d_order};
    Outputs O{dist, grad, var, aux, valid, c->d_refine, c->d_stat, c->d_spread, prop, prop_var};
    if (c->p.precision == GPDF_PREC_FP64) {
        stage_begin(c, GPDF_MS_EVAL);
        launch_query_k<double>(c, kern, knn, grid, s, d_q, G, lists, Mo, C, O, 0);
        stage_end(c, GPDF_MS_EVAL);
    } else {
        stage_begin(c, GPDF_MS_EVAL);
        if (c->p.precision == GPDF_PREC_BF16) {
            // the variance product on BF16 MFMA; distance and gradient keep
            // the FP32 path's error estimate and FP64 re-evaluation, the
            // variance keeps its BF16 error (never refined for)
            const gpdf_status st = build_bf16(c);
            if (st != GPDF_OK) return st;
            const int kts = bf_cols(int(std::min<int64_t>(M.max_n, kBfMaxN))) + 8;
            const size_t lds = size_t(64) * kts * sizeof(__bf16);
            QueryConsts Cb = C;
            Cb.tau_v = INFINITY;
            const __bf16 *Mbf = static_cast<const __bf16 *>(c->d_bfM);
            if (kern == GPDF_KERNEL_MATERN32)
                launch_bf16_m<GPDF_KERNEL_MATERN32>(grid, lds, s, d_q, G, lists, Mo, Mbf, c->d_bfoff, kts, Cb,
                                                    O);
            else
                launch_bf16_m<GPDF_KERNEL_SE>(grid, lds, s, d_q, G, lists, Mo, Mbf, c->d_bfoff, kts, Cb, O);
        } else if (c->p.precision == GPDF_PREC_FP32_MFMA ||
                   (c->tune.mfma_min_n > 0 && eager && !knn && !want_prop)) {
            // the variance product on FP32 MFMA for the clusters of
            // mfma_min_n to 248 points (FP32_MFMA precision: every cluster up
            // to 248 unless tuned otherwise), the VALU path for the others;
            // every output keeps the FP32 error estimate and FP64
            // re-evaluation.  The LDS row of a query holds the largest
            // cluster's kernel values (odd stride).
            const int min_n = c->tune.mfma_min_n > 0 ? c->tune.mfma_min_n : 1;
            const int kts = ((int(std::min<int64_t>(std::max<int64_t>(M.max_n, 1), kF32mMaxN)) + 3) & ~3) + 1;
            const size_t lds = size_t(64) * kts * sizeof(float);
            if (kern == GPDF_KERNEL_MATERN32)
                launch_f32m_m<GPDF_KERNEL_MATERN32>(grid, lds, s, d_q, G, lists, Mo, kts, min_n, C, O);
            else
                launch_f32m_m<GPDF_KERNEL_SE>(grid, lds, s, d_q, G, lists, Mo, kts, min_n, C, O);
        } else {
            launch_query_k<float>(c, kern, knn, grid, s, d_q, G, lists, Mo, C, O, 0);
        }
        stage_end(c, GPDF_MS_EVAL);
        // 3. queries whose FP32 estimate is too large: regroup by cell
        //    (counting sort of the records) and redo them in FP64
        stage_begin(c, GPDF_MS_REFINE);
        // records (grid-stride over a bounded grid: they are a small share
        // of the queries)
        const unsigned rgrid = std::min<unsigned>(blocks_for(m), 1024u);
        {
            FillList F2;
            F2.u32(c->d_rcnt, 0u, nc);
            if (!knn) {
                F2.u32(c->d_bcnt, 0u, cm_cluster_bound(c, M));
                F2.u32(c->d_work, 0u, kWorkSlot);
            }
            if ((e = fill_multi(F2, s)) != hipSuccess) return hip_fail(c, e, "query: refine clear");
        }
        hipLaunchKernelGGL(k_refine_count, dim3(rgrid), dim3(kQT), 0, s, c->d_refine,
                           c->d_stat + ST_REFINE, m, c->d_rcnt, c->d_rrank);
        hipLaunchKernelGGL(k_refine_chunks, dim3(blocks_for(nc)), dim3(kQT), 0, s, nc, dnc, c->d_rcnt,
                           c->d_rchunks);
        ScanList RL;
        RL.add(c->d_rcnt, c->d_roff, nullptr);
        RL.add(c->d_rchunks, c->d_rchunk_off, cnt + CNT_RCHUNKS);
        exclusive_scan_u32_multi(RL, nc, c->d_part, s, dnc, c->capturing);
        hipLaunchKernelGGL(k_chunk_table, dim3(blocks_for(nc)), dim3(kQT), 0, s, nc, dnc, c->d_rchunks,
                           c->d_rchunk_off, c->d_rchunk);
        hipLaunchKernelGGL(k_refine_scatter, dim3(rgrid), dim3(kQT), 0, s, c->d_refine,
                           c->d_stat + ST_REFINE, m, c->d_rrank, c->d_roff, c->d_rorder, c->d_rcell);
        const Grouping R{c->d_rchunk, cnt + CNT_RCHUNKS, c->d_rcnt, c->d_roff, c->d_rorder};
        Outputs O64 = O;
        O64.refine = nullptr;
        if (knn) {
            launch_query_k<double>(c, kern, knn, grid, s, d_q, R, lists, Mo, C, O64, 1);
        } else {
            // cluster-major evaluation of the pairs, then their combination;
            // the FP64 query kernel (persistent, on the evaluation's counter
            // slot, cleared above) takes the chunks instead when the pass
            // could not take every pair
            const BigView BV = refine_cm(c, M, s, d_q, lists, Mo, C, m, want_prop);
            // grid-stride launches: the items are of even size, and one
            // shared work counter would serialise on its atomics
            const unsigned rg = unsigned(std::min<int64_t>(2048, (m + 63) / 64));
            const Grouping Rs{c->d_rchunk, cnt + CNT_RCH_SLOW, c->d_rcnt, c->d_roff, c->d_rorder};
            const uint32_t *nrf = cnt + CNT_NREF_FAST;
#define GPDF_CMB(K) \
    launch_cm_combine<K>(rg, s, d_q, nrf, c->d_rorder, c->d_rcell, lists, Mo, C, O64, BV)
            if (want_prop) {
                if (kern == GPDF_KERNEL_MATERN32) GPDF_CMB(GPDF_KERNEL_MATERN32 | kProp);
                else GPDF_CMB(GPDF_KERNEL_SE | kProp);
            } else if (kern == GPDF_KERNEL_MATERN32) {
                GPDF_CMB(GPDF_KERNEL_MATERN32);
            } else {
                GPDF_CMB(GPDF_KERNEL_SE);
            }
#undef GPDF_CMB
            if (want_prop) launch_query_kf<double, kProp>(kern, false, 1024, s, d_q, Rs, lists, Mo, C, O64, c->d_work);
            else launch_query_kf<double, 0>(kern, false, 1024, s, d_q, Rs, lists, Mo, C, O64, c->d_work);
        }
        stage_end(c, GPDF_MS_REFINE);
    }
    fold_stats(c->d_spread, c->d_stat, s);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "query launch");
    if (correct) return mlp_apply(c, dist, var, grad, aux, valid, m, dist);
    return GPDF_OK;
}

}  // namespace gpdf

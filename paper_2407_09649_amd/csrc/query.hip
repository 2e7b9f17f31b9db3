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
// (templates for n <= 16, 32, 64); larger clusters stream W in 64-row panels.
// FP32 results carry a running error bound; queries whose bound exceeds the
// tolerance are re-evaluated by a wave-per-query FP64 kernel.
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>
#include <utility>

namespace gpdf {

namespace {

constexpr int kQT = 256;            // threads per workgroup (4 wavefronts)
constexpr int kWaves = kQT / 64;
constexpr int kListStride = 28;     // count + 27 cluster ids
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
                                     uint8_t *valid, float *aux) {
    dist[qi] = INFINITY;
    valid[qi] = 0;
    if (grad) { grad[3 * qi] = 0.f; grad[3 * qi + 1] = 0.f; grad[3 * qi + 2] = 0.f; }
    if (var) var[qi] = INFINITY;
    if (aux) { aux[3 * qi] = 0.f; aux[3 * qi + 1] = 0.f; aux[3 * qi + 2] = 0.f; }
}

// ---------------------------------------------------------------------------
// grouping of queries by cell
// ---------------------------------------------------------------------------
__global__ void k_qcells(const float *__restrict__ q, int64_t m, int voxel_mode, double hv, double hc,
                         HashView qh, uint32_t *__restrict__ cnt, int32_t *__restrict__ qslot,
                         uint32_t *__restrict__ qrank, float *dist, float *grad, float *var,
                         uint8_t *valid, float *aux, unsigned long long *__restrict__ stat) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t c[3];
    if (!query_cell(q + 3 * i, voxel_mode, hv, hc, c)) {
        qslot[i] = -1;
        write_invalid(uint32_t(i), dist, grad, var, valid, aux);
        atomicAdd(&stat[ST_NONFINITE_Q], 1ull);
        return;
    }
    bool ins;
    int64_t s = hash_insert(qh, pack_key(c[0], c[1], c[2]), &ins);
    if (s < 0) {
        qslot[i] = -1;
        write_invalid(uint32_t(i), dist, grad, var, valid, aux);
        atomicAdd(&stat[ST_HASH_FULL], 1ull);
        return;
    }
    qslot[i] = int32_t(s);
    qrank[i] = atomicAdd(&cnt[s], 1u);
}

__global__ void k_cells_compact(const unsigned long long *__restrict__ keys,
                                const uint32_t *__restrict__ cnt, int64_t cap,
                                int32_t *__restrict__ cell_of_slot, uint64_t *__restrict__ cell_key,
                                uint32_t *__restrict__ cell_cnt, uint32_t *__restrict__ cell_chunks,
                                unsigned long long *__restrict__ stat) {
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    const unsigned long long k = keys[s];
    if (k == kNoKey) return;
    const uint32_t id = uint32_t(atomicAdd(&stat[ST_CELLS], 1ull));
    cell_of_slot[s] = int32_t(id);
    cell_key[id] = k;
    const uint32_t n = cnt[s];
    cell_cnt[id] = n;
    cell_chunks[id] = (n + 63) / 64;
}

__global__ void k_chunks_and_lists(int64_t ncells, const uint64_t *__restrict__ cell_key,
                                   const uint32_t *__restrict__ cell_chunks,
                                   const uint32_t *__restrict__ chunk_off, uint2 *__restrict__ chunk,
                                   const unsigned long long *__restrict__ chash, uint32_t cmask,
                                   const int32_t *__restrict__ chash_val,
                                   const uint8_t *__restrict__ pd, const int32_t *__restrict__ coff,
                                   int32_t *__restrict__ lists) {
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const uint32_t o = chunk_off[c];
    for (uint32_t j = 0; j < cell_chunks[c]; ++j) chunk[o + j] = make_uint2(uint32_t(c), j * 64);
    int64_t cc[3];
    unpack_key(cell_key[c], cc);
    int32_t *L = lists + c * kListStride;
    int nsel = 0;
    // ascending key order: x offset outermost, z innermost
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int64_t s = hash_find(chash, cmask, pack_key(cc[0] + dx, cc[1] + dy, cc[2] + dz));
                if (s < 0) continue;
                const int32_t id = chash_val[s];
                if (pd[id] && coff[id + 1] > coff[id]) L[1 + nsel++] = id;
            }
    L[0] = nsel;
}

__global__ void k_all_invalid(int64_t m, float *dist, float *grad, float *var, uint8_t *valid,
                              float *aux) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) write_invalid(uint32_t(i), dist, grad, var, valid, aux);
}

__global__ void k_scatter_order(const int32_t *__restrict__ qslot, const uint32_t *__restrict__ qrank,
                                int64_t m, const int32_t *__restrict__ cell_of_slot,
                                const uint32_t *__restrict__ cell_off, uint32_t *__restrict__ order) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t s = qslot[i];
    if (s < 0) return;
    order[cell_off[cell_of_slot[s]] + qrank[i]] = uint32_t(i);
}

// ---------------------------------------------------------------------------
// FP32 pair evaluation
// ---------------------------------------------------------------------------
struct PairRaw {
    float o, gx, gy, gz, S, ss;
};

struct Acc {
    float m, sw, swd, swv, sgx, sgy, sgz;   // smooth-min sums, scaled by exp(-lambda (. - m))
    float pgx, pgy, pgz;                    // plain gradient sum
    float hd, hv, hgx, hgy, hgz, ho, hu;    // closest node
    float A1, A2, B1, C1;                   // error-estimate sums (smooth-min scaled)
    float Ggx, Ggy, Ggz, G2;                // sum w e_d g and w e_d |g|^2
    float hed, heg, hev, sum_eg;            // closest node estimates, plain sum of e_g
    int nq, ntot;
    float best;
    int bidx;
};

__device__ inline void acc_init(Acc &A) {
    A.m = INFINITY;
    A.sw = A.swd = A.swv = A.sgx = A.sgy = A.sgz = 0.f;
    A.pgx = A.pgy = A.pgz = 0.f;
    A.hd = INFINITY; A.hv = A.hgx = A.hgy = A.hgz = A.ho = A.hu = 0.f;
    A.A1 = A.A2 = A.B1 = A.C1 = 0.f;
    A.Ggx = A.Ggy = A.Ggz = A.G2 = 0.f;
    A.hed = A.heg = A.hev = A.sum_eg = 0.f;
    A.nq = 0; A.ntot = 0;
    A.best = INFINITY; A.bidx = -1;
}

// one point: kernel value k, the factor e multiplying alpha (x - x_i) in the
// gradient sum, and the point's contribution to the running sums
template <int KERN>
__device__ __forceinline__ float point_eval(const float4 p, float qx, float qy, float qz, int gidx,
                                            const QueryConsts &C, PairRaw &r, Acc &A) {
    const float dx = qx - p.x, dy = qy - p.y, dz = qz - p.z;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (r2 < A.best) { A.best = r2; A.bidx = gidx; }
    float k, e, t;
    if (KERN == GPDF_KERNEL_MATERN32) {
        t = fsqrt(r2) * C.a;                 // sqrt(3) r / l
        e = fexp2(-t * kLog2e);
        k = fmaf(t, e, e);                   // (1 + t) e^{-t}
    } else {
        t = r2 * C.a;                        // r^2 / 2 l^2
        k = fexp2(-t * kLog2e);
        e = k;
    }
    r.o = fmaf(p.w, k, r.o);
    const float cg = p.w * e;
    r.gx = fmaf(cg, dx, r.gx);
    r.gy = fmaf(cg, dy, r.gy);
    r.gz = fmaf(cg, dz, r.gz);
    // root-sum-square scale of the rounding errors of the terms alpha k,
    // whose relative error grows like (1 + t) through the exponent
    const float akt = fabsf(p.w) * fmaf(k, t, k);
    r.S = fmaf(akt, akt, r.S);
    return k;
}

// n <= NMAX: k in registers, W rows packed (row i at i (i + 1) / 2).  The
// rows are generated at compile time (index sequences), so every k_j index is
// a constant and the vector lives in VGPRs.
template <int... J>
__device__ __forceinline__ float row_dot(const float *__restrict__ Wi, const float *kr,
                                         std::integer_sequence<int, J...>) {
    float t[2] = {0.f, 0.f};
    ((t[J & 1] = fmaf(Wi[J], kr[J], t[J & 1])), ...);
    return t[0] + t[1];
}

template <int KERN, int NMAX, int I>
__device__ __forceinline__ void small_rows(const float4 *__restrict__ P, const float *__restrict__ W,
                                           int n, int pbase, float qx, float qy, float qz,
                                           const QueryConsts &C, PairRaw &r, Acc &A, float *kr) {
    if constexpr (I < NMAX) {
        if (I >= n) return;
        kr[I] = point_eval<KERN>(P[I], qx, qy, qz, pbase + I, C, r, A);
        const float t = row_dot(W + (I * (I + 1)) / 2, kr, std::make_integer_sequence<int, I + 1>{});
        r.ss = fmaf(t, t, r.ss);
        small_rows<KERN, NMAX, I + 1>(P, W, n, pbase, qx, qy, qz, C, r, A, kr);
    }
}

template <int KERN, int NMAX>
__device__ __forceinline__ void eval_small(const float4 *__restrict__ P, const float *__restrict__ W,
                                           int n, int pbase, float qx, float qy, float qz,
                                           const QueryConsts &C, PairRaw &r, Acc &A) {
    float kr[NMAX];
    small_rows<KERN, NMAX, 0>(P, W, n, pbase, qx, qy, qz, C, r, A, kr);
}

template <int... Q>
__device__ __forceinline__ void panel_update(float *t, const float *__restrict__ col, float kj,
                                             std::integer_sequence<int, Q...>) {
    ((t[Q] = fmaf(col[Q], kj, t[Q])), ...);
}

// n > 64: point sums in one pass, then W k by 64-row panels with k recomputed
template <int KERN>
__device__ __forceinline__ void eval_big(const float4 *__restrict__ P, const float *__restrict__ W, int n,
                                      int pbase, float qx, float qy, float qz, const QueryConsts &C,
                                      PairRaw &r, Acc &A) {
    for (int i = 0; i < n; ++i) point_eval<KERN>(P[i], qx, qy, qz, pbase + i, C, r, A);
    const int nb = (n + kPanel - 1) / kPanel;
    PairRaw dummy{};
    Acc dA;
    dA.best = -1.f;  // never updated: r2 < -1 is false
    dA.bidx = 0;
    const float *Pn = W;
    for (int rb = 0; rb < nb; ++rb) {
        float t[kPanel];
#pragma unroll
        for (int q = 0; q < kPanel; ++q) t[q] = 0.f;
        const int ncol = min((rb + 1) * kPanel, n);
        for (int j = 0; j < ncol; ++j) {
            const float kj = point_eval<KERN>(P[j], qx, qy, qz, 0, C, dummy, dA);
            panel_update(t, Pn + j * kPanel, kj, std::make_integer_sequence<int, kPanel>{});
        }
#pragma unroll
        for (int q = 0; q < kPanel; ++q) r.ss = fmaf(t[q], t[q], r.ss);
        Pn += ncol * kPanel;
    }
}

// Matern-3/2 reverting in FP32: t >= 0 with (1 + t) e^{-t} = o.  Seed from the
// branch-point series of W_{-1} (Corless et al. 1996) for o > 1/2, from the
// asymptote t = y + log(1 + t), y = -log o, below; then three Newton steps.
__device__ __forceinline__ float matern_t32(float o) {
    const float s = fsqrt(2.f * (1.f - o));
    const float ta = s * fmaf(s, fmaf(s, fmaf(s, 43.f / 540.f, 11.f / 72.f), 1.f / 3.f), 1.f);
    const float y = -flog(o);
    float tb = y + flog(1.f + y);
    tb = y + flog(1.f + tb);
    float t = o > 0.5f ? ta : tb;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        const float E = fexp2(-t * kLog2e);
        const float f = fmaf(t, E, E) - o;
        t = fmaf(f, frcp(t * E), t);
    }
    return t;
}

template <int KERN>
__device__ __forceinline__ void finish_pair(const PairRaw &r, int n, const QueryConsts &C, Acc &A) {
    const float o = r.o;
    const float u = fminf(fmaxf(1.f - r.ss, 0.f), 1.f);
    const float oc = fminf(fmaxf(o, C.omin), C.omax);
    const float sS = fsqrt(r.S);
    // estimated error of o: root-sum-square of the term errors, plus the
    // FP32 reverting solve, which settles where its residual is ~ eps o
    const float dO = C.err_c * kEps * sS + 2.f * kEps * oc;
    float d, lam, gsc, sens;  // distance, Lambda, gradient scale, |d ln gsc / d o|
    if (KERN == GPDF_KERNEL_MATERN32) {
        const float t = matern_t32(oc);
        const float E = fexp2(-t * kLog2e);
        const float tE = t * E;
        d = C.c * t;
        lam = -C.c * frcp(tE);               // -(l / sqrt3) e^t / t
        gsc = C.a * frcp(tE);                // grad d = a G / (t e^{-t})
        sens = fabsf(t - 1.f) * frcp(t * tE);
    } else {
        const float L = -flog(oc);
        d = C.c * fsqrt(2.f * L);            // l sqrt(-2 log o)
        lam = -C.c * C.c * frcp(oc * d);     // -l^2 / (o d)
        gsc = frcp(oc * d);                  // grad d = G / (o d)
        sens = frcp(oc) + fabsf(lam) * frcp(d);
    }
    const float gx = gsc * r.gx, gy = gsc * r.gy, gz = gsc * r.gz;
    const float v = lam * lam * u;
    const float gn = fsqrt(fmaf(gz, gz, fmaf(gy, gy, gx * gx)));
    // first-order error estimates of this pair's distance, gradient and
    // (relative) variance from the error of o and of the variance sum
    const float ed = fabsf(lam) * dO + 4.f * kEps * d;
    const float eg = gsc * C.err_c * kEps * sS * frcp(C.a) + gn * sens * dO + 8.f * kEps * gn;
    const float ev = 2.f * sens * dO + 4.f * kEps * float(n) * frcp(fmaxf(u, 1e-30f)) + 8.f * kEps;
    // closest node (strict <: the first in ascending key order wins ties)
    if (d < A.hd) {
        A.hd = d; A.hv = v; A.hgx = gx; A.hgy = gy; A.hgz = gz; A.ho = o; A.hu = u;
        A.hed = ed; A.heg = eg; A.hev = ev;
    }
    // smooth minimum, online: rescale the sums when the minimum moves
    const float delta = d - A.m;
    const float ex = fexp2(-C.lam * kLog2e * fabsf(delta));
    const bool newmin = delta < 0.f;
    const float so = newmin ? ex : 1.f;
    const float w = newmin ? 1.f : ex;
    const float shift = newmin ? (A.m - d) : 0.f;  // A2 is relative to the minimum
    A.A2 = so * fmaf(shift, A.A1, A.A2) + w * ed * (newmin ? 0.f : delta);
    if (!(A.m < INFINITY)) A.A2 = 0.f;
    A.A1 = fmaf(so, A.A1, w * ed);
    A.B1 = fmaf(so, A.B1, w * eg);
    const float wed = w * ed;
    A.Ggx = fmaf(so, A.Ggx, wed * gx);
    A.Ggy = fmaf(so, A.Ggy, wed * gy);
    A.Ggz = fmaf(so, A.Ggz, wed * gz);
    A.G2 = fmaf(so, A.G2, wed * gn * gn);
    A.C1 = fmaf(so, A.C1, w * v * ev);
    A.sw = fmaf(so, A.sw, w);
    A.swd = fmaf(so, A.swd, w * d);
    A.swv = fmaf(so, A.swv, w * v);
    A.sgx = fmaf(so, A.sgx, w * gx);
    A.sgy = fmaf(so, A.sgy, w * gy);
    A.sgz = fmaf(so, A.sgz, w * gz);
    A.m = fminf(A.m, d);
    A.pgx += gx; A.pgy += gy; A.pgz += gz;
    A.sum_eg += eg;
    A.nq += 1;
    A.ntot += n;
}

struct Outputs {
    float *dist, *grad, *var, *aux;
    uint8_t *valid;
    uint32_t *refine;
    unsigned long long *stat;
    int refine_all;  // FP64 mode: every valid query is redone
};

// final combination, sign, error test and stores for one lane
__device__ inline void finish_query(const Acc &A, uint32_t qi, bool active, float qx, float qy,
                                    float qz, const float4 *__restrict__ pts, const QueryConsts &C,
                                    const Outputs &O) {
    if (!active) return;
    if (A.nq == 0) {
        write_invalid(qi, O.dist, O.grad, O.var, O.valid, O.aux);
        return;
    }
    float D, V, Gx, Gy, Gz, Ed, Eg, Ev;
    if (C.combine == GPDF_COMB_HARDMIN) {
        D = A.hd; V = A.hv; Gx = A.hgx; Gy = A.hgy; Gz = A.hgz; Ed = A.hed; Eg = A.heg; Ev = A.hev;
    } else {
        const float iw = 1.f / A.sw;
        D = A.swd * iw;
        V = A.swv * iw;
        if (C.grad_mode == GPDF_GRAD_PAPER_MEAN) {
            const float iq = 1.f / float(A.nq);
            Gx = A.pgx * iq; Gy = A.pgy * iq; Gz = A.pgz * iq;
        } else {
            Gx = A.sgx * iw; Gy = A.sgy * iw; Gz = A.sgz * iw;
        }
        const float Gn = sqrtf(Gx * Gx + Gy * Gy + Gz * Gz);
        Ed = (A.A1 * (1.f + C.lam * (D - A.m)) + C.lam * A.A2) * iw;
        // weight errors move G by lambda sum (w/W) e_d |g_q - G|, bounded by
        // Cauchy-Schwarz through the online moments of g
        const float Q2 = A.G2 - 2.f * (Gx * A.Ggx + Gy * A.Ggy + Gz * A.Ggz) + Gn * Gn * A.A1;
        Eg = (A.B1 + C.lam * sqrtf(fmaxf(A.A1 * Q2, 0.f))) * iw;
        if (C.grad_mode == GPDF_GRAD_PAPER_MEAN) Eg = A.sum_eg / float(A.nq) + Eg;
        Ev = A.C1 / A.swv;
    }
    if (C.signed_ && A.bidx >= 0) {
        // sensor side of the nearest training point, decided in FP32
        const float4 p = pts[A.bidx];
        const float ax = qx - p.x, ay = qy - p.y, az = qz - p.z;
        const float bx = C.ox - p.x, by = C.oy - p.y, bz = C.oz - p.z;
        const float dot = fmaf(az, bz, fmaf(ay, by, ax * bx));
        if (!(dot >= 0.f)) { D = -D; Gx = -Gx; Gy = -Gy; Gz = -Gz; }
    }
    O.dist[qi] = D;
    O.valid[qi] = 1;
    if (O.grad) { O.grad[3 * qi] = Gx; O.grad[3 * qi + 1] = Gy; O.grad[3 * qi + 2] = Gz; }
    if (O.var) O.var[qi] = V;
    if (O.aux) { O.aux[3 * qi] = A.ho; O.aux[3 * qi + 1] = A.hu; O.aux[3 * qi + 2] = float(A.ntot); }
    const bool bad = O.refine_all || !(Ed <= C.tau_d) || !(Eg <= C.tau_g) || !(Ev <= C.tau_v);
    if (bad) {
        const unsigned long long pos = atomicAdd(&O.stat[ST_REFINE], 1ull);
        O.refine[pos] = qi;
    }
}

template <int KERN>
__device__ __forceinline__ void eval_cluster(int32_t cid, const float4 *__restrict__ pts,
                                             const int32_t *__restrict__ coff,
                                             const int64_t *__restrict__ woff32,
                                             const float *__restrict__ W32, float qx, float qy,
                                             float qz, const QueryConsts &C, Acc &A) {
    const int base = coff[cid];
    const int n = coff[cid + 1] - base;
    const float4 *P = pts + base;
    const float *W = W32 + woff32[cid];
    PairRaw r{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (n <= 16) eval_small<KERN, 16>(P, W, n, base, qx, qy, qz, C, r, A);
    else if (n <= 32) eval_small<KERN, 32>(P, W, n, base, qx, qy, qz, C, r, A);
    else if (n <= 64) eval_small<KERN, 64>(P, W, n, base, qx, qy, qz, C, r, A);
    else eval_big<KERN>(P, W, n, base, qx, qy, qz, C, r, A);
    finish_pair<KERN>(r, n, C, A);
}

// NEIGHBOR27: one wavefront per (cell, 64-query chunk)
template <int KERN>
__global__ __launch_bounds__(kQT) void k_query32(
    const float *__restrict__ q, const uint2 *__restrict__ chunk,
    const uint32_t *__restrict__ chunk_total, const uint32_t *__restrict__ cell_cnt,
    const uint32_t *__restrict__ cell_off, const uint32_t *__restrict__ order,
    const int32_t *__restrict__ lists, const float4 *__restrict__ pts,
    const int32_t *__restrict__ coff, const int64_t *__restrict__ woff32,
    const float *__restrict__ W32, QueryConsts C, Outputs O) {
    const uint32_t wave = blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= *chunk_total) return;
    const uint2 ch = chunk[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(cell_cnt[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = order[cell_off[cell] + start + (active ? lane : 0)];
    const float qx = q[3 * qi], qy = q[3 * qi + 1], qz = q[3 * qi + 2];
    const int32_t *L = lists + size_t(cell) * kListStride;
    const int nsel = int(uniform(uint32_t(L[0])));
    Acc A;
    acc_init(A);
    for (int s = 0; s < nsel; ++s) {
        const int32_t cid = int32_t(uniform(uint32_t(L[1 + s])));
        eval_cluster<KERN>(cid, pts, coff, woff32, W32, qx, qy, qz, C, A);
    }
    finish_query(A, qi, active, qx, qy, qz, pts, C, O);
    const uint64_t nv = __ballot(active && A.nq > 0);
    if (lane == 0 && nv) atomicAdd(&O.stat[ST_VALID_Q], (unsigned long long)__popcll(nv));
}

// squared FP64 distance from x to the centre of cell key k, no contraction,
// in the same order as the oracle (x, y, z)
__device__ inline double centre_d2(const float *x, uint64_t k, double edge) {
    int64_t c[3];
    unpack_key(k, c);
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

// KNN: each lane picks its Q nearest clusters by cell-centre distance (ties
// to the smaller key); the wavefront walks the union of the lanes' lists in
// ascending cluster order and each lane evaluates exactly its own clusters
template <int KERN>
__global__ __launch_bounds__(kQT) void k_query32_knn(
    const float *__restrict__ q, const uint2 *__restrict__ chunk,
    const uint32_t *__restrict__ chunk_total, const uint32_t *__restrict__ cell_cnt,
    const uint32_t *__restrict__ cell_off, const uint32_t *__restrict__ order,
    const uint64_t *__restrict__ ckey, const uint8_t *__restrict__ pd, int64_t ncl,
    double edge, const float4 *__restrict__ pts, const int32_t *__restrict__ coff,
    const int64_t *__restrict__ woff32, const float *__restrict__ W32, QueryConsts C, Outputs O) {
    __shared__ int32_t lst[kWaves][kMaxKnn][64];
    const int wv = threadIdx.x >> 6;
    const uint32_t wave = blockIdx.x * kWaves + wv;
    const int lane = threadIdx.x & 63;
    if (wave >= *chunk_total) return;
    const uint2 ch = chunk[wave];
    const uint32_t cell = uniform(ch.x), start = uniform(ch.y);
    const uint32_t cnt = uniform(min(cell_cnt[cell] - start, 64u));
    const bool active = uint32_t(lane) < cnt;
    const uint32_t qi = order[cell_off[cell] + start + (active ? lane : 0)];
    const float x[3] = {q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
    const int Q = C.knn_q;
    double bd[kMaxKnn];
    int bi[kMaxKnn];
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) { bd[j] = INFINITY; bi[j] = 0x7fffffff; }
    for (int64_t c = 0; c < ncl; ++c) {
        if (!pd[c] || coff[c + 1] == coff[c]) continue;
        const double d2 = centre_d2(x, ckey[c], edge);
        if (!(d2 < bd[Q - 1])) continue;
        // insert keeping (distance, index) order; equal distance keeps the earlier
        double cd = d2;
        int ci = int(c);
#pragma unroll
        for (int j = 0; j < kMaxKnn; ++j) {
            if (j < Q && cd < bd[j]) {
                const double td = bd[j]; const int ti = bi[j];
                bd[j] = cd; bi[j] = ci; cd = td; ci = ti;
            }
        }
    }
    // ascending cluster index (= ascending key)
#pragma unroll
    for (int a = 1; a < kMaxKnn; ++a)
#pragma unroll
        for (int b = kMaxKnn - 1; b >= a; --b)
            if (bi[b] < bi[b - 1]) { const int t = bi[b]; bi[b] = bi[b - 1]; bi[b - 1] = t; }
#pragma unroll
    for (int j = 0; j < kMaxKnn; ++j) lst[wv][j][lane] = bi[j];
    Acc A;
    acc_init(A);
    int ptr = 0;
    while (true) {
        const int mine = (active && ptr < Q) ? lst[wv][ptr][lane] : 0x7fffffff;
        const int c = int(uniform(uint32_t(wave_min_i32(mine))));
        if (c == 0x7fffffff) break;
        if (mine == c) {
            ++ptr;
            eval_cluster<KERN>(c, pts, coff, woff32, W32, x[0], x[1], x[2], C, A);
        }
    }
    finish_query(A, qi, active, x[0], x[1], x[2], pts, C, O);
    const uint64_t nv = __ballot(active && A.nq > 0);
    if (lane == 0 && nv) atomicAdd(&O.stat[ST_VALID_Q], (unsigned long long)__popcll(nv));
}

// ---------------------------------------------------------------------------
// FP64 evaluation, one wavefront per query
// ---------------------------------------------------------------------------
__device__ inline double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// t - log(1 + t), with the alternating series below t = 0.1
__device__ inline double phi64(double t) {
    if (t >= 0.1) return t - log1p(t);
    double s = 0.0, pw = t * t;
    for (int k = 2; k <= 24; ++k) {
        s += ((k & 1) ? -pw : pw) / double(k);
        pw *= t;
    }
    return s;
}

// Matern reverting in FP64: solve t - log(1 + t) = -log o by safeguarded Newton
__device__ inline double matern_t64(double o) {
    if (!(o < 1.0)) return 0.0;
    const double y = o > 0.5 ? -log1p(o - 1.0) : -log(o);
    double lo = 0.0, hi = 1.0;
    while (phi64(hi) < y) hi *= 2.0;
    double t = o > 0.5 ? sqrt(2.0 * y) : y + log1p(y);
    if (!(t > lo && t < hi)) t = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        const double f = phi64(t) - y;
        if (f < 0.0) lo = t; else hi = t;
        double tn = t - f * (1.0 + t) / t;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - t) <= 1e-17 * t) { t = tn; break; }
        t = tn;
        if (hi - lo <= 1e-17 * t) break;
    }
    return t;
}

template <int KERN>
__global__ __launch_bounds__(kQT) void k_query64(
    const float *__restrict__ q, const uint32_t *__restrict__ recs,
    const unsigned long long *__restrict__ nrec_ptr, int64_t nrec_host, int use_host_count,
    int voxel_mode, const unsigned long long *__restrict__ chash, uint32_t cmask,
    const int32_t *__restrict__ chash_val, const uint64_t *__restrict__ ckey,
    const uint8_t *__restrict__ pd, int64_t ncl, double edge, const float4 *__restrict__ pts,
    const double *__restrict__ alpha64, const int32_t *__restrict__ coff,
    const int64_t *__restrict__ woff64, const double *__restrict__ W64, QueryConsts C, Outputs O) {
    extern __shared__ double kb_all[];
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    double *kb = kb_all + size_t(wv) * 1024;
    const int64_t nrec = use_host_count ? nrec_host : int64_t(*nrec_ptr);
    const int64_t total_waves = int64_t(gridDim.x) * kWaves;
    const bool matern = KERN == GPDF_KERNEL_MATERN32;
    const double l = C.ld;
    const double a = matern ? 1.7320508075688772935 / l : 0.0;
    for (int64_t rix = int64_t(blockIdx.x) * kWaves + wv; rix < nrec; rix += total_waves) {
        const uint32_t qi = recs ? recs[rix] : uint32_t(rix);
        const float xf[3] = {q[3 * qi], q[3 * qi + 1], q[3 * qi + 2]};
        const double x[3] = {double(xf[0]), double(xf[1]), double(xf[2])};
        // ---- selection
        int32_t sel[32];
        int nsel = 0;
        int64_t cc[3];
        bool ok = query_cell(xf, voxel_mode, C.hv, C.hc, cc);
        if (ok && C.knn_q == 0) {
            int32_t mine = -1;
            if (lane < 27) {
                const int dx = lane / 9 - 1, dy = (lane / 3) % 3 - 1, dz = lane % 3 - 1;
                const int64_t s = hash_find(chash, cmask, pack_key(cc[0] + dx, cc[1] + dy, cc[2] + dz));
                if (s >= 0) {
                    const int32_t id = chash_val[s];
                    if (pd[id] && coff[id + 1] > coff[id]) mine = id;
                }
            }
            uint64_t msk = __ballot(mine >= 0);
            while (msk) {
                const int b = __ffsll((long long)msk) - 1;
                msk &= msk - 1;
                sel[nsel++] = __shfl(mine, b, 64);
            }
        } else if (ok) {
            // Q nearest: per-lane candidates over a strided share, then Q
            // rounds of a wave argmin on (distance, index)
            const int Q = C.knn_q;
            double bd[kMaxKnn];
            int bi[kMaxKnn];
            for (int j = 0; j < kMaxKnn; ++j) { bd[j] = INFINITY; bi[j] = 0x7fffffff; }
            for (int64_t c = lane; c < ncl; c += 64) {
                if (!pd[c] || coff[c + 1] == coff[c]) continue;
                double cd = centre_d2(xf, ckey[c], edge);
                int ci = int(c);
                for (int j = 0; j < Q; ++j) {
                    if (cd < bd[j] || (cd == bd[j] && ci < bi[j])) {
                        const double td = bd[j]; const int ti = bi[j];
                        bd[j] = cd; bi[j] = ci; cd = td; ci = ti;
                    }
                }
            }
            int head = 0;
            for (int r = 0; r < Q; ++r) {
                double hd = head < Q ? bd[head] : INFINITY;
                int hi = head < Q ? bi[head] : 0x7fffffff;
                for (int o = 32; o > 0; o >>= 1) {
                    const double od = __shfl_xor(hd, o, 64);
                    const int oi = __shfl_xor(hi, o, 64);
                    if (od < hd || (od == hd && oi < hi)) { hd = od; hi = oi; }
                }
                if (hi == 0x7fffffff) break;
                if (head < Q && bi[head] == hi) ++head;
                sel[nsel++] = hi;
            }
            for (int i2 = 1; i2 < nsel; ++i2) {
                const int32_t v = sel[i2];
                int j = i2;
                while (j > 0 && sel[j - 1] > v) { sel[j] = sel[j - 1]; --j; }
                sel[j] = v;
            }
        }
        if (nsel == 0) {
            if (lane == 0) write_invalid(qi, O.dist, O.grad, O.var, O.valid, O.aux);
            continue;
        }
        // ---- pairs
        double m = INFINITY, sw = 0, swd = 0, swv = 0, sg[3] = {0, 0, 0}, pg[3] = {0, 0, 0};
        double hd = INFINITY, hv = 0, hg[3] = {0, 0, 0}, ho = 0, hu = 0;
        double dlist[32], vlist[32], glist[32][3];
        int ntot = 0;
        float best = INFINITY;
        int bidx = 0x7fffffff;
        for (int s = 0; s < nsel; ++s) {
            const int cid = sel[s];
            const int base = coff[cid], n = coff[cid + 1] - base;
            double o = 0, g[3] = {0, 0, 0};
            for (int i = lane; i < n; i += 64) {
                const float4 p = pts[base + i];
                const float ex = xf[0] - p.x, ey = xf[1] - p.y, ez = xf[2] - p.z;
                const float r2f = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
                if (r2f < best) { best = r2f; bidx = base + i; }
                const double dx = x[0] - double(p.x), dy = x[1] - double(p.y), dz = x[2] - double(p.z);
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                double k, gc;
                if (matern) {
                    const double e = exp(-a * r);
                    k = (1.0 + a * r) * e;
                    gc = -a * a * e;
                } else {
                    k = exp(-r * r / (2.0 * l * l));
                    gc = -k / (l * l);
                }
                kb[i] = k;
                const double al = alpha64[base + i];
                o += al * k;
                g[0] += al * gc * dx; g[1] += al * gc * dy; g[2] += al * gc * dz;
            }
            o = wsum(o);
            g[0] = wsum(g[0]); g[1] = wsum(g[1]); g[2] = wsum(g[2]);
            __builtin_amdgcn_wave_barrier();
            const double *Wc = W64 + woff64[cid];
            double ss = 0.0;
            for (int i = lane; i < n; i += 64) {
                double t = 0.0;
                for (int j = 0; j <= i; ++j) t += Wc[int64_t(j) * n - int64_t(j) * (j - 1) / 2 + (i - j)] * kb[j];
                ss += t * t;
            }
            ss = wsum(ss);
            __builtin_amdgcn_wave_barrier();
            double u = 1.0 - ss;
            u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
            double oc = o < C.omind ? C.omind : o;
            oc = oc > C.omaxd ? C.omaxd : oc;
            double d, lam;
            if (matern) {
                const double t = matern_t64(oc);
                const double cl = l / 1.7320508075688772935;
                d = cl * t;
                lam = -cl * exp(t) / t;
            } else {
                const double gg = sqrt(-2.0 * log(oc));
                d = l * gg;
                lam = -l / (oc * gg);
            }
            const double v = lam * lam * u;
            const double gd[3] = {lam * g[0], lam * g[1], lam * g[2]};
            dlist[s] = d; vlist[s] = v;
            glist[s][0] = gd[0]; glist[s][1] = gd[1]; glist[s][2] = gd[2];
            if (d < hd) { hd = d; hv = v; hg[0] = gd[0]; hg[1] = gd[1]; hg[2] = gd[2]; ho = o; hu = u; }
            if (d < m) m = d;
            ntot += n;
        }
        for (int s = 0; s < nsel; ++s) {
            const double w = exp(-C.lamd * (dlist[s] - m));
            sw += w; swd += w * dlist[s]; swv += w * vlist[s];
            for (int k = 0; k < 3; ++k) { sg[k] += w * glist[s][k]; pg[k] += glist[s][k]; }
        }
        double D, V, G[3];
        if (C.combine == GPDF_COMB_HARDMIN) {
            D = hd; V = hv; G[0] = hg[0]; G[1] = hg[1]; G[2] = hg[2];
        } else {
            D = swd / sw; V = swv / sw;
            for (int k = 0; k < 3; ++k)
                G[k] = C.grad_mode == GPDF_GRAD_PAPER_MEAN ? pg[k] / double(nsel) : sg[k] / sw;
        }
        // nearest training point: wave argmin on (FP32 distance, index)
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            const float ob = __shfl_xor(best, o2, 64);
            const int oi = __shfl_xor(bidx, o2, 64);
            if (ob < best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
        }
        if (C.signed_ && bidx != 0x7fffffff) {
            const float4 p = pts[bidx];
            const float ax = xf[0] - p.x, ay = xf[1] - p.y, az = xf[2] - p.z;
            const float bx = C.ox - p.x, by = C.oy - p.y, bz = C.oz - p.z;
            const float dot = fmaf(az, bz, fmaf(ay, by, ax * bx));
            if (!(dot >= 0.f)) { D = -D; G[0] = -G[0]; G[1] = -G[1]; G[2] = -G[2]; }
        }
        if (lane == 0) {
            O.dist[qi] = float(D);
            O.valid[qi] = 1;
            if (O.grad) { O.grad[3 * qi] = float(G[0]); O.grad[3 * qi + 1] = float(G[1]); O.grad[3 * qi + 2] = float(G[2]); }
            if (O.var) O.var[qi] = float(V);
            if (O.aux) { O.aux[3 * qi] = float(ho); O.aux[3 * qi + 1] = float(hu); O.aux[3 * qi + 2] = float(ntot); }
        }
    }
}

}  // namespace

QueryConsts make_consts(const gpdf_params &p, const float *origin) {
    QueryConsts C{};
    const bool matern = p.kernel == GPDF_KERNEL_MATERN32;
    C.l = float(p.length_scale);
    C.a = matern ? float(1.7320508075688772935 / p.length_scale)
                 : float(1.0 / (2.0 * p.length_scale * p.length_scale));
    C.c = matern ? float(p.length_scale / 1.7320508075688772935) : float(p.length_scale);
    C.lam = float(p.smooth_min_lambda);
    C.omin = float(p.occ_min);
    C.omax = float(p.occ_max);
    // thresholds 5x inside the distance (1e-4 m) and gradient (1e-3)
    // tolerances; relative variance held to 1e-3.  err_c scales the
    // root-sum-square rounding estimate (a probabilistic, not worst-case,
    // estimate); at 2 the results left in FP32 stay at least 6x inside the
    // tolerances on the sphere, LiDAR and planar-patch workloads
    C.tau_d = 2e-5f;
    C.tau_g = 2e-4f;
    C.tau_v = 1e-3f;
    C.err_c = 2.f;
    C.kernel = p.kernel;
    C.combine = p.combine;
    C.grad_mode = p.grad_mode;
    C.knn_q = p.selection == GPDF_SEL_KNN ? p.knn_q : 0;
    C.signed_ = origin != nullptr;
    if (origin) { C.ox = origin[0]; C.oy = origin[1]; C.oz = origin[2]; }
    C.ld = p.length_scale;
    C.sd = p.noise_sigma;
    C.hv = p.voxel_size;
    C.hc = p.cluster_size;
    C.lamd = p.smooth_min_lambda;
    C.omind = p.occ_min;
    C.omaxd = p.occ_max;
    return C;
}

gpdf_status query(gpdf_ctx *c, const float *d_q, int64_t m, const float *origin, float *dist,
                  float *grad, float *var, uint8_t *valid, float *aux, int32_t correct) {
    hipStream_t s = c->stream;
    const Model &M = c->model;
    if (!M.trained) return fail(c, GPDF_E_NOT_TRAINED, "query before training");
    if (m < 0 || m > c->p.max_queries) return fail(c, GPDF_E_CAPACITY, "query: m exceeds max_queries");
    if (!dist || !valid || (m > 0 && !d_q)) return fail(c, GPDF_E_INVALID_ARG, "query: null buffer");
    if (origin && !(std::isfinite(origin[0]) && std::isfinite(origin[1]) && std::isfinite(origin[2])))
        return fail(c, GPDF_E_INVALID_ARG, "query: non-finite origin");
    c->last_queries = m;
    // per-call counters
    fill_u64(c->d_stat + ST_NONFINITE_Q, 0ull, 1, s);
    fill_u64(c->d_stat + ST_VALID_Q, 0ull, 1, s);
    fill_u64(c->d_stat + ST_REFINE, 0ull, 1, s);
    fill_u64(c->d_stat + ST_CELLS, 0ull, 1, s);
    if (m == 0) return GPDF_OK;
    const QueryConsts C = make_consts(c->p, origin);
    const bool vox = c->p.voxel_size > 0.0;
    const double edge = vox ? 8.0 * c->p.voxel_size : c->p.cluster_size;
    const bool matern = c->p.kernel == GPDF_KERNEL_MATERN32;
    Outputs O{dist, grad, var, aux, valid, c->d_refine, c->d_stat, 0};
    hipError_t e;
    const size_t lds64 = sizeof(double) * 1024 * kWaves;
    if (M.nclusters == 0) {
        // nothing to select: every query is invalid
        hipLaunchKernelGGL(k_all_invalid, dim3(blocks_for(m)), dim3(kQT), 0, s, m, dist, grad, var,
                           valid, aux);
        return (e = hipGetLastError()) == hipSuccess ? GPDF_OK : hip_fail(c, e, "query launch");
    }
    if (c->p.precision == GPDF_PREC_FP64) {
        // every query on the FP64 path, one wavefront each
        hipLaunchKernelGGL(matern ? k_query64<GPDF_KERNEL_MATERN32> : k_query64<GPDF_KERNEL_SE>,
                           dim3(std::min<int64_t>(blocks_for(m * 64), 8192)), dim3(kQT), lds64, s,
                           d_q, (const uint32_t *)nullptr, (const unsigned long long *)nullptr, m, 1,
                           vox ? 1 : 0, c->d_chash, c->chash_mask, c->d_chash_val, c->d_ckey, c->d_pd,
                           M.nclusters, edge, c->d_pts, c->d_alpha64, c->d_coff, c->d_woff64,
                           c->d_W64, C, O);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "query64 launch");
        if (correct) return mlp_apply(c, dist, var, grad, aux, valid, m, dist);
        return GPDF_OK;
    }
    // 1. group by cell
    const int64_t qcap = int64_t(c->qhash_mask) + 1;
    fill_u64(c->d_qhash, (unsigned long long)kNoKey, qcap, s);
    fill_u32(c->d_qhash_cnt, 0u, qcap, s);
    HashView qh{c->d_qhash, c->qhash_mask};
    hipLaunchKernelGGL(k_qcells, dim3(blocks_for(m)), dim3(kQT), 0, s, d_q, m, vox ? 1 : 0,
                       c->p.voxel_size, c->p.cluster_size, qh, c->d_qhash_cnt, c->d_qslot, c->d_qrank,
                       dist, grad, var, valid, aux, c->d_stat);
    hipLaunchKernelGGL(k_cells_compact, dim3(blocks_for(qcap)), dim3(kQT), 0, s, c->d_qhash,
                       c->d_qhash_cnt, qcap, c->d_qhash_cell, c->d_cell_key, c->d_cell_cnt,
                       c->d_cell_chunks, c->d_stat);
    unsigned long long ncells = 0;
    if ((e = hipMemcpyAsync(&ncells, c->d_stat + ST_CELLS, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(c, e, "query: read cell count");
    if (ncells == 0) return GPDF_OK;
    exclusive_scan_u32(c->d_cell_cnt, c->d_cell_off, int64_t(ncells), c->d_part, s);
    exclusive_scan_u32(c->d_cell_chunks, c->d_chunk_off, int64_t(ncells), c->d_part, s);
    hipLaunchKernelGGL(k_chunks_and_lists, dim3(blocks_for(ncells)), dim3(kQT), 0, s, int64_t(ncells),
                       c->d_cell_key, c->d_cell_chunks, c->d_chunk_off, c->d_chunk, c->d_chash,
                       c->chash_mask, c->d_chash_val, c->d_pd, c->d_coff, c->d_cell_list);
    hipLaunchKernelGGL(k_scatter_order, dim3(blocks_for(m)), dim3(kQT), 0, s, c->d_qslot, c->d_qrank, m,
                       c->d_qhash_cell, c->d_cell_off, c->d_order);
    // 2. FP32 evaluation; the chunk count stays on the device (grid is an upper bound)
    const int64_t max_chunks = int64_t(ncells) + (m + 63) / 64;
    const unsigned grid = blocks_for(max_chunks * 64);
    const uint32_t *d_nchunks = c->d_chunk_off + ncells;
    if (C.knn_q == 0) {
        hipLaunchKernelGGL(matern ? k_query32<GPDF_KERNEL_MATERN32> : k_query32<GPDF_KERNEL_SE>,
                           dim3(grid), dim3(kQT), 0, s, d_q, c->d_chunk, d_nchunks, c->d_cell_cnt,
                           c->d_cell_off, c->d_order, c->d_cell_list, c->d_pts, c->d_coff,
                           c->d_woff32, c->d_W32, C, O);
    } else {
        hipLaunchKernelGGL(matern ? k_query32_knn<GPDF_KERNEL_MATERN32> : k_query32_knn<GPDF_KERNEL_SE>,
                           dim3(grid), dim3(kQT), 0, s, d_q, c->d_chunk, d_nchunks, c->d_cell_cnt,
                           c->d_cell_off, c->d_order, c->d_ckey, c->d_pd, M.nclusters, edge, c->d_pts,
                           c->d_coff, c->d_woff32, c->d_W32, C, O);
    }
    // 3. FP64 re-evaluation of the queries whose FP32 bound is too loose
    hipLaunchKernelGGL(matern ? k_query64<GPDF_KERNEL_MATERN32> : k_query64<GPDF_KERNEL_SE>, dim3(2048),
                       dim3(kQT), lds64, s, d_q, c->d_refine, c->d_stat + ST_REFINE, int64_t(0), 0,
                       vox ? 1 : 0, c->d_chash, c->chash_mask, c->d_chash_val, c->d_ckey, c->d_pd,
                       M.nclusters, edge, c->d_pts, c->d_alpha64, c->d_coff, c->d_woff64, c->d_W64, C,
                       O);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "query launch");
    if (correct) return mlp_apply(c, dist, var, grad, aux, valid, m, dist);
    return GPDF_OK;
}

}  // namespace gpdf

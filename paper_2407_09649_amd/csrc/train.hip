// train.hip -- the local GPs of one frame (L-GPDF, Sec. IV-A).
//
//   keys      voxel or cell coordinates floor(x / h) in FP64
//   sort      stable radix sort by (cluster, voxel) or (cluster, input index)
//   clusters  unique voxels -> centres (voxel mode), runs of equal cluster key
//   train     per cluster, FP64: A = K + s^2 I (Eq. (1)), L = chol(A),
//             W = L^{-1}, alpha = W^T W 1; W also kept in FP32 for queries
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>

namespace gpdf {

namespace {

constexpr int kT = 256;

inline unsigned blocks_for(int64_t n, int t = kT) {
    int64_t g = (n + t - 1) / t;
    return unsigned(g < 1 ? 1 : g);
}

// voxel mode: composite key = (cluster cell: 3 x 18-bit offset binary) << 9 | local voxel
// raw mode: key = packed cell of size h_c, value = input index
// points at or past the count (dn, a device count bounded by n) are absent
__global__ void k_point_keys(const float *__restrict__ xyz, int64_t n, const uint32_t *__restrict__ dn,
                             int voxel_mode, double h, uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                             uint32_t *__restrict__ flag, unsigned long long *__restrict__ stat) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i >= dev_count(n, dn)) {
        flag[i] = 0;
        key[i] = kNoKey;
        val[i] = uint32_t(i);
        return;
    }
    int64_t c[3];
    bool ok = cell_coord(xyz[3 * i], h, c[0]) && cell_coord(xyz[3 * i + 1], h, c[1]) &&
              cell_coord(xyz[3 * i + 2], h, c[2]);
    if (!ok) {
        atomicAdd(&stat[ST_SKIPPED_POINTS], 1ull);
        flag[i] = 0;
        key[i] = kNoKey;
        val[i] = uint32_t(i);
        return;
    }
    uint64_t k;
    if (voxel_mode) {
        const int64_t b18 = int64_t(1) << 17;
        int64_t cl[3] = {floor_div8(c[0]), floor_div8(c[1]), floor_div8(c[2])};
        uint64_t local = uint64_t(((c[0] - 8 * cl[0]) << 6) | ((c[1] - 8 * cl[1]) << 3) |
                                  (c[2] - 8 * cl[2]));
        k = (((uint64_t(cl[0] + b18) << 36) | (uint64_t(cl[1] + b18) << 18) |
              uint64_t(cl[2] + b18))
             << 9) |
            local;
    } else {
        k = pack_key(c[0], c[1], c[2]);
    }
    key[i] = k;
    val[i] = uint32_t(i);
    flag[i] = 1;
}

__global__ void k_compact_pairs(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                                int64_t n, uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    kout[pos[i]] = kin[i];
    vout[pos[i]] = vin[i];
}

// keys past the valid count sort last
__global__ void k_pad_keys(uint64_t *__restrict__ key, uint32_t *__restrict__ val, int64_t n,
                           const uint32_t *__restrict__ dvalid) {
    const int64_t nv = dev_count(n, dvalid);
    for (int64_t i = nv + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        key[i] = kNoKey;
        val[i] = 0;
    }
}

// flag[i] = 1 where (key >> sh) starts a new run among the first dn keys;
// 0 up to the bound n
__global__ void k_run_flags(const uint64_t *__restrict__ key, int64_t n, const uint32_t *__restrict__ dn, int sh,
                            uint32_t *__restrict__ flag) {
    const int64_t na = dev_count(n, dn);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        flag[i] = (i < na && (i == 0 || (key[i] >> sh) != (key[i - 1] >> sh))) ? 1u : 0u;
}

__global__ void k_compact_unique(const uint64_t *__restrict__ key, int64_t n,
                                 const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                                 uint64_t *__restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        if (flag[i]) out[pos[i]] = key[i];
}

// Surface property of each training point (Eq. (6)).  Voxel mode: the mean
// of the properties of the voxel's raw points, summed in FP64 in input order
// (the sort is stable, so a voxel's run holds its points by ascending input
// index); flag marks the first entry of each voxel run and pos is its voxel
// index.  Raw mode (flag == NULL): the point's own property.
__global__ void k_point_prop(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val, int64_t n,
                             const uint32_t *__restrict__ dn, const uint32_t *__restrict__ flag,
                             const uint32_t *__restrict__ pos, const float *__restrict__ prop,
                             double *__restrict__ cprop) {
    const int64_t na = dev_count(n, dn);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < na;
         i += int64_t(gridDim.x) * blockDim.x) {
        if (!flag) {
            cprop[i] = double(prop[val[i]]);
            continue;
        }
        if (!flag[i]) continue;
        const uint64_t k = key[i];
        double sum = double(prop[val[i]]);
        int64_t e = i + 1;
        while (e < na && key[e] == k) {
            sum += double(prop[val[e]]);
            ++e;
        }
        cprop[pos[i]] = sum / double(e - i);
    }
}

// beta = W^T (W c) = (K + s^2 I)^{-1} c per cluster (Eq. (6)): the property
// right-hand side on the trained factor W = L^{-1}, read in the query layout
// (packed rows for n <= 32, 32-row column-major panels above).  One
// workgroup per cluster; a cluster that is not positive definite gets 0.
__device__ __forceinline__ int64_t w_at(int n, int i, int j) {
    if (n <= kPanel) return int64_t(i) * (i + 1) / 2 + j;
    const int r = i / kPanel;
    return w32_panel_offset(n, r) + int64_t(j) * kPanel + (i - r * kPanel);
}

__global__ __launch_bounds__(256) void k_beta(const int32_t *__restrict__ coff, int64_t Cb,
                                              const uint32_t *__restrict__ dncl, const int64_t *__restrict__ woff,
                                              const double *__restrict__ W64, const uint8_t *__restrict__ pd,
                                              const double *__restrict__ cprop, double *__restrict__ beta64,
                                              float *__restrict__ beta32) {
    __shared__ double y[1024];   // the largest cluster (max_cluster_points <= 1024)
    const int64_t C = dev_count(Cb, dncl);
    for (int64_t c = blockIdx.x; c < C; c += gridDim.x) {
        const int base = coff[c], n = coff[c + 1] - base;
        const bool ok = pd[c] != 0;
        const double *W = W64 + woff[c];
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            double t = 0.0;
            if (ok)
                for (int j = 0; j <= i; ++j) t = fma(W[w_at(n, i, j)], cprop[base + j], t);
            y[i] = t;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double t = 0.0;
            if (ok)
                for (int i = j; i < n; ++i) t = fma(W[w_at(n, i, j)], y[i], t);
            beta64[base + j] = t;
            beta32[base + j] = float(t);
        }
        __syncthreads();
    }
}

// clusters: offsets, keys and training points.  voxel_mode: keys are the
// unique composite keys; raw mode: keys are cell keys, vals input indices.
__global__ void k_clusters(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val,
                           int64_t nbound, const uint32_t *__restrict__ dn, const uint32_t *__restrict__ flag,
                           const uint32_t *__restrict__ pos, int voxel_mode, double hv,
                           const float *__restrict__ xyz, float4 *__restrict__ pts,
                           int32_t *__restrict__ coff, uint64_t *__restrict__ ckey,
                           int64_t cap, uint32_t *__restrict__ ncl_out,
                           unsigned long long *__restrict__ stat) {
    const int64_t n = dev_count(nbound, dn);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const uint64_t k = key[i];
        if (voxel_mode) {
            const int64_t b18 = int64_t(1) << 17;
            const uint64_t ck = k >> 9;
            int64_t cl[3] = {int64_t((ck >> 36) & 0x3FFFF) - b18, int64_t((ck >> 18) & 0x3FFFF) - b18,
                             int64_t(ck & 0x3FFFF) - b18};
            int64_t v[3] = {8 * cl[0] + int64_t((k >> 6) & 7), 8 * cl[1] + int64_t((k >> 3) & 7),
                            8 * cl[2] + int64_t(k & 7)};
            // voxel centre (c + 1/2) h, formed in FP64 and rounded once
            pts[i] = make_float4(float((double(v[0]) + 0.5) * hv), float((double(v[1]) + 0.5) * hv),
                                 float((double(v[2]) + 0.5) * hv), 0.0f);
            if (flag[i] && int64_t(pos[i]) < cap) {
                const uint32_t c = pos[i];
                coff[c] = int32_t(i);
                ckey[c] = pack_key(cl[0], cl[1], cl[2]);
            } else if (flag[i] && int64_t(pos[i]) == cap) {
                coff[cap] = int32_t(i);  // the last kept cluster ends where the first dropped one starts
            }
        } else {
            const uint32_t s = val[i];
            pts[i] = make_float4(xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2], 0.0f);
            if (flag[i] && int64_t(pos[i]) < cap) {
                const uint32_t c = pos[i];
                coff[c] = int32_t(i);
                ckey[c] = k;
            } else if (flag[i] && int64_t(pos[i]) == cap) {
                coff[cap] = int32_t(i);  // the last kept cluster ends where the first dropped one starts
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t ncl = pos[n];
        if (int64_t(ncl) <= cap) coff[ncl] = int32_t(n);
        *ncl_out = uint32_t(min(int64_t(ncl), cap));
        if (int64_t(ncl) > cap) atomicAdd(&stat[ST_CAPACITY], 1ull);
    }
}

// ---------------------------------------------------------------------------
// FP64 training of one cluster per workgroup
// ---------------------------------------------------------------------------
__device__ inline double kernel64(int kernel, double r, double l) {
    if (kernel == GPDF_KERNEL_MATERN32) {
        const double a = 1.7320508075688772935 * r / l;
        return (1.0 + a) * exp(-a);
    }
    return exp(-r * r / (2.0 * l * l));
}

constexpr int kMaxClusterN = 1024;
constexpr int kBlockLdsN = 176;                          // packed triangle in LDS up to here
constexpr int kBlockLdsElems = kBlockLdsN * (kBlockLdsN + 1) / 2;

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// One workgroup of T threads per cluster (n > 64).  The lower triangle of
// A = K + s^2 I is packed by rows, in LDS up to n = 176 (124.6 KB), else in
// the FP64 workspace.  Cholesky and the inverse W = L^{-1} run together in
// place: after step k, columns 0..k of the triangle hold W (rows k+1.. as
// partial sums R) and columns k+1.. the trailing part of A.  Step k:
//   l = sqrt(A(k,k)), L(i,k) = A(i,k) / l for i > k (kept in LDS),
//   row k of W  = R(k, 0..k-1) / l, W(k,k) = 1 / l,
//   for i > k:  R(i,j) -= L(i,k) W(k,j)   (j < k),   W(i,k) = -L(i,k) / l,
//               A(i,j) -= L(i,k) L(j,k)    (k < j <= i).
// The elements of rows k+1..n-1 are contiguous in the packed triangle, so a
// step is one range split evenly over the workgroup: two barriers per step,
// consecutive threads on consecutive elements.  A pivot at or below
// 1e-10 (1 + s^2) marks the cluster non positive definite.  alpha = W^T (W 1).
__device__ __forceinline__ int tri_row(int p) {
    int i = int((sqrtf(8.f * float(p) + 1.f) - 1.f) * 0.5f);
    if ((i + 1) * (i + 2) / 2 <= p) ++i;
    if (i * (i + 1) / 2 > p) --i;
    return i;
}

// the body, inlined once with A in LDS and once with A in global memory, so
// that every access compiles to LDS or global instructions (a pointer that
// may be either would compile to flat accesses)
template <int T, int MAXC>
__device__ __forceinline__ void train_block_body(double *__restrict__ A, double *__restrict__ craw,
                                                 double *__restrict__ piv,
                                                 int c, int base, int n,
                                                 float4 *__restrict__ pts, const int64_t *__restrict__ woff,
                                                 double *__restrict__ W64all, float *__restrict__ W32all,
                                                 double *__restrict__ alpha64, uint8_t *__restrict__ pd, int kernel,
                                                 double l, double s2, unsigned long long *__restrict__ stat) {
    constexpr int kW = T / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // A = K + s^2 I (lower triangle)
    for (int i = wv; i < n; i += kW) {
        const float4 pi = pts[base + i];
        for (int j = lane; j <= i; j += 64) {
            const float4 pj = pts[base + j];
            const double dx = double(pi.x) - double(pj.x), dy = double(pi.y) - double(pj.y),
                         dz = double(pi.z) - double(pj.z);
            double v = kernel64(kernel, sqrt(dx * dx + dy * dy + dz * dz), l);
            if (i == j) v += s2;
            A[tri(i, j)] = v;
        }
    }
    const double thr = 1e-10 * (1.0 + s2);
    const int end = n * (n + 1) / 2;
    // Step k needs row k left of the pivot and column k below it, unscaled:
    // both live in one vector x (x[j] = A(k, j) for j < k, A(j, k) for
    // j > k), double-buffered with the pivot.  The wavefront that updates
    // row k + 1 in step k stages that row and the next pivot; the lane that
    // updates element (i, k + 1) of a lower row stages it, so one barrier per
    // step suffices.  With inv = 1 / sqrt(pivot) every element of row i takes
    // l_i = x_i inv^2 and becomes -l_i in column k, A(i, j) - l_i x_j elsewhere.
    __syncthreads();  // A assembled
    for (int i = 1 + tid; i < n; i += T) craw[i] = A[tri(i, 0)];
    if (tid == 0) piv[0] = A[0];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int b = k & 1;
        const double *x = craw + b * kMaxClusterN;
        double *xn = craw + (b ^ 1) * kMaxClusterN;
        const double d = piv[b];
        if (!(d > thr)) {
            for (int i = tid; i < n; i += T) {
                alpha64[base + i] = 0.0;
                pts[base + i].w = 0.0f;
            }
            if (tid == 0) {
                pd[c] = 0;
                atomicAdd(&stat[ST_NONPD], 1ull);
            }
            return;
        }
        const double inv = 1.0 / sqrt(d);
        const double inv2 = inv * inv;
        // row k of W (nobody reads row k during this step)
        for (int j = tid; j < k; j += T) A[tri(k, j)] = x[j] * inv;
        if (tid == 0) A[tri(k, k)] = inv;
        // rows below k: a packed row (contiguous) per wavefront, its columns
        // over the lanes
        for (int i = k + 1 + wv; i < n; i += kW) {
            double *Ai = A + tri(i, 0);
            const double lii = x[i] * inv2;
            if (i == k + 1) {
                for (int j = lane; j <= i; j += 64) {
                    const double a = j == k ? -lii : Ai[j] - lii * x[j];
                    Ai[j] = a;
                    if (j <= k) xn[j] = a;
                    else piv[b ^ 1] = a;
                }
            } else {
                // both loads unconditional (x[k] is read and then not used), so
                // that column k costs a select instead of a branch; with A in
                // LDS a row has at most MAXC chunks of 64 columns, unrolled so
                // that their loads are issued together
                if constexpr (MAXC > 0) {
#pragma unroll
                    for (int cc = 0; cc < MAXC; ++cc) {
                        const int j = lane + 64 * cc;
                        if (j <= i) {
                            const double aij = Ai[j], xj = x[j];
                            const double t = aij - lii * xj;
                            Ai[j] = j == k ? -lii : t;
                        }
                    }
                } else {
                    for (int j = lane; j <= i; j += 64) {
                        const double aij = Ai[j], xj = x[j];
                        const double t = aij - lii * xj;
                        Ai[j] = j == k ? -lii : t;
                    }
                }
                if (lane == ((k + 1) & 63)) xn[i] = Ai[k + 1];  // this lane's own update
            }
        }
        __syncthreads();
    }
    // y = W 1 (row sums), alpha = W^T y
    for (int i = tid; i < n; i += T) {
        const double *Wi = A + tri(i, 0);
        double s0 = 0.0, s1 = 0.0;
        int j = 0;
        for (; j + 1 <= i; j += 2) { s0 += Wi[j]; s1 += Wi[j + 1]; }
        if (j <= i) s0 += Wi[j];
        craw[i] = s0 + s1;
    }
    __syncthreads();
    for (int j = tid; j < n; j += T) {
        double a = 0.0;
        for (int i = j; i < n; ++i) a += A[tri(i, j)] * craw[i];
        alpha64[base + j] = a;
        pts[base + j].w = float(a);
    }
    // W in the query layout (FP32 and FP64): packed rows for n <= 32 (the
    // order of the packed triangle), 32-row panels above that, column-major
    // inside and zero above the diagonal
    float *W32 = W32all + woff[c];
    double *W64 = W64all + woff[c];
    if (n <= kPanel) {
        for (int idx = tid; idx < end; idx += T) {
            W32[idx] = float(A[idx]);
            W64[idx] = A[idx];
        }
        if (tid == 0) pd[c] = 1;
        return;
    }
    const int nb = (n + kPanel - 1) / kPanel;
    for (int r = 0; r < nb; ++r) {
        const int64_t po = w32_panel_offset(n, r);
        const int ncol = min((r + 1) * kPanel, n);
        for (int idx = tid; idx < ncol * kPanel; idx += T) {
            const int j = idx / kPanel, rr = idx - j * kPanel;
            const int i = r * kPanel + rr;
            const double v = (i < n && j <= i) ? A[tri(i, j)] : 0.0;
            W32[po + idx] = float(v);
            W64[po + idx] = v;
        }
    }
    if (tid == 0) pd[c] = 1;
}

// persistent: each workgroup takes the next cluster of the bucket from the
// counter *work (zero at launch) until none is left
template <int T>
__global__ __launch_bounds__(T) void k_train_block(
    const int32_t *__restrict__ list, const uint32_t *__restrict__ dcnt, uint32_t *__restrict__ work,
    float4 *__restrict__ pts, const int32_t *__restrict__ coff,
    const int64_t *__restrict__ aoff, const int64_t *__restrict__ woff, double *__restrict__ Aall,
    double *__restrict__ W64all, float *__restrict__ W32all, double *__restrict__ alpha64,
    uint8_t *__restrict__ pd, int kernel, double l, double s2, unsigned long long *__restrict__ stat) {
    __shared__ double sA[kBlockLdsElems];
    __shared__ double craw[2 * kMaxClusterN];
    __shared__ double piv[2];
    __shared__ uint32_t item;
    const uint32_t cnt = *dcnt;
    while (true) {
        __syncthreads();  // the previous cluster is done with the LDS and item
        if (threadIdx.x == 0) item = atomicAdd(work, 1u);
        __syncthreads();
        const uint32_t b = item;
        if (b >= cnt) break;
        const int c = list[b];
        const int base = coff[c];
        const int n = coff[c + 1] - base;
        if (n <= kBlockLdsN)
            train_block_body<T, (kBlockLdsN + 63) / 64>(sA, craw, piv, c, base, n, pts, woff, W64all, W32all, alpha64, pd, kernel,
                                l, s2, stat);
        else
            train_block_body<T, 0>(Aall + aoff[c], craw, piv, c, base, n, pts, woff, W64all, W32all, alpha64,
                                pd, kernel, l, s2, stat);
    }
}

// ---------------------------------------------------------------------------
// Blocked FP64 training on 16 x 16 tiles with FP64 MFMA (65 to 256 points)
//
// A = K + s^2 I is padded to T = ceil(n / 16) tiles per edge with an identity
// block (so the padded factor is block diagonal with I and changes nothing),
// and its lower tiles are kept in LDS (n <= 192) or in the FP64 workspace.
// Right-looking Cholesky by tile columns p = 0 .. T - 1:
//   one wavefront factors the diagonal tile, L_pp = chol(A_pp), and inverts
//   it, V_p = L_pp^{-1} (16 steps in registers, column c in lane c), which
//   replaces A_pp (L_pp is not read again);
//   L_ip = A_ip V_p^T                for the tiles below (i > p);
//   A_ij -= L_ip L_jp^T              for the trailing tiles (p < j <= i),
// then W = L^{-1} in place by tile columns j = T - 1 .. 0 (the blocked
// triangular inverse): M_kj = L_kj V_j, W_ij = -sum_{k=j+1..i} W_ik M_kj,
// with W_jj = V_j already in place.  Every tile product is four
// v_mfma_f64_16x16x4f64.  Finally
// alpha = W^T (W 1) and W in the query layout.  A pivot at or below
// 1e-10 (1 + s^2) marks the cluster non positive definite.
// Lane layout of v_mfma_f64_16x16x4f64 (lane l, r = l % 16, g = l / 16):
//   A[m][k] lane m + 16 k; B[k][n] lane n + 16 k; D[m][n] lane n + 16 (m % 4),
//   element m / 4 (checked on the device).
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kTb = 16;                                  // tile edge
constexpr int kTileElems = kTb * kTb;                    // 2 KB of FP64
constexpr int kMfmaMaxN = 256;                           // largest cluster of this trainer
constexpr int kMfmaLdsT = 12;                            // tiles per edge held in LDS at most (n <= 192)
__host__ __device__ inline int mfma_tiles(int n) { return (n + kTb - 1) / kTb; }
// FP64 workspace of a cluster: its lower tiles
__host__ __device__ inline int64_t mfma_ws(int n) {
    const int64_t T = mfma_tiles(n);
    return T * (T + 1) / 2 * kTileElems;
}
// element (r, c) of a tile: rows of 16, the column XOR-swizzled by the row,
// so that 16 lanes reading one column, or one row, meet 16 distinct bank
// pairs of the LDS
__device__ __forceinline__ int tel(int r, int c) { return r * kTb + (c ^ r); }
__device__ __forceinline__ int tlow(int ti, int tj) { return (ti * (ti + 1) / 2 + tj) * kTileElems; }

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// acc += s X Y^T (X, Y tiles)
__device__ __forceinline__ f64x4 tile_xyt(const double *X, const double *Y, f64x4 acc, double sgn, int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < kTb; k0 += 4) acc = mfma64(sgn * X[tel(r, k0 + g)], Y[tel(r, k0 + g)], acc);
    return acc;
}
// acc += X Y
__device__ __forceinline__ f64x4 tile_xy(const double *X, const double *Y, f64x4 acc, int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int k0 = 0; k0 < kTb; k0 += 4) acc = mfma64(X[tel(r, k0 + g)], Y[tel(k0 + g, r)], acc);
    return acc;
}
// the accumulator of a lane: rows g, g + 4, g + 8, g + 12 (g = lane / 16) of
// column lane % 16
__device__ __forceinline__ f64x4 tile_get(const double *X, int lane) {
    const int g = lane >> 4, c = lane & 15;
    return f64x4{X[tel(g, c)], X[tel(g + 4, c)], X[tel(g + 8, c)], X[tel(g + 12, c)]};
}
__device__ __forceinline__ void tile_put(double *X, f64x4 v, int lane) {
    const int g = lane >> 4, c = lane & 15;
    X[tel(g, c)] = v[0];
    X[tel(g + 4, c)] = v[1];
    X[tel(g + 8, c)] = v[2];
    X[tel(g + 12, c)] = v[3];
}
__device__ __forceinline__ double bcast(double v, int lane) {
    return __builtin_bit_cast(double, (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(__builtin_bit_cast(uint64_t, v) >> 32), lane))) << 32) |
                                          uint64_t(uint32_t(__builtin_amdgcn_readlane(int(__builtin_bit_cast(uint64_t, v)), lane))));
}

// Cholesky and inverse of the diagonal tile D (one wavefront).  Lane c
// (c = lane % 16; the four groups of 16 lanes repeat the same work) holds
// column c of A in registers, which is also row c as A is symmetric, and
// column c of R = I, which becomes V = L^{-1}.  Step k broadcasts the
// pivot A(k, k) and the column A(r, k), r > k, from lane k by readlane; with
// L(k, k) = sqrt(A(k, k)) and L(r, k) = A(r, k) / L(k, k):
//   V(k, c) = R(k, c) / L(k, k),
//   A(r, c) -= A(r, k) A(k, c) / A(k, k),   R(r, c) -= L(r, k) V(k, c)   (r > k).
// No LDS and no branch: the columns c <= k of A are finished and take
// updates nobody reads, and R(k, c) = 0 for c > k keeps V(k, c) = 0 there.
// Writes V over D (zero above the diagonal): L_pp itself is not needed;
// false if a pivot is not above thr.
__device__ __forceinline__ bool diag_factor(double *D, double thr, int lane) {
    const int c = lane & 15;
    double a[kTb], w[kTb];
#pragma unroll
    for (int r = 0; r < kTb; ++r) {
        a[r] = D[tel(r, c)];
        w[r] = r == c ? 1.0 : 0.0;
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < kTb; ++k) {
        const double piv = bcast(a[k], k);
        ok = ok && piv > thr;
        // 1 / sqrt(pivot): the hardware estimate and two Newton steps
        // y <- y (3 - x y^2) / 2, each doubling the correct bits
        const double x = ok ? piv : 1.0;
        double inv = __builtin_amdgcn_rsq(x);
        inv = inv * fma(-0.5 * x * inv, inv, 1.5);
        inv = inv * fma(-0.5 * x * inv, inv, 1.5);
        const double t = a[k] * (inv * inv);   // A(k, c) / A(k, k)
        const double v = w[k] * inv;           // V(k, c)
        w[k] = v;
        const double vi = v * inv;
#pragma unroll
        for (int r = k + 1; r < kTb; ++r) {
            const double ark = bcast(a[r], k);  // read before this step's update of a[r]
            w[r] = fma(-ark, vi, w[r]);
            a[r] = fma(-ark, t, a[r]);
            // the update of R stays here: nothing else depends on it before
            // the store, and sunk there it would hold every broadcast value
            asm volatile("" : "+v"(w[r]));
        }
    }
    if (lane < kTb) {
#pragma unroll
        for (int r = 0; r < kTb; ++r) D[tel(r, c)] = c <= r ? w[r] : 0.0;
    }
    return ok;
}

// two independent tile products with all operand loads issued first:
// acc1 += s X1 Y1^T and acc2 += s X2 Y2^T
__device__ __forceinline__ void tile_xyt2(const double *X1, const double *Y1, f64x4 &acc1, const double *X2,
                                          const double *Y2, f64x4 &acc2, double sgn, int lane) {
    const int r = lane & 15, g = lane >> 4;
    double a1[4], b1[4], a2[4], b2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a1[q] = X1[tel(r, 4 * q + g)];
        b1[q] = Y1[tel(r, 4 * q + g)];
        a2[q] = X2[tel(r, 4 * q + g)];
        b2[q] = Y2[tel(r, 4 * q + g)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc1 = mfma64(sgn * a1[q], b1[q], acc1);
        acc2 = mfma64(sgn * a2[q], b2[q], acc2);
    }
}
// acc1 += X1 Y1 and acc2 += X2 Y2, loads first
__device__ __forceinline__ void tile_xy2(const double *X1, const double *Y1, f64x4 &acc1, const double *X2,
                                         const double *Y2, f64x4 &acc2, int lane) {
    const int r = lane & 15, g = lane >> 4;
    double a1[4], b1[4], a2[4], b2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        a1[q] = X1[tel(r, 4 * q + g)];
        b1[q] = Y1[tel(4 * q + g, r)];
        a2[q] = X2[tel(r, 4 * q + g)];
        b2[q] = Y2[tel(4 * q + g, r)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc1 = mfma64(a1[q], b1[q], acc1);
        acc2 = mfma64(a2[q], b2[q], acc2);
    }
}

// the body of one cluster (NT threads), the tiles in LDS or in the workspace
template <int NT>
__device__ __forceinline__ void train_mfma_body(double *__restrict__ A, double *__restrict__ ybuf,
                                                int *flag, int *next,
                                                int c, int base, int n, float4 *__restrict__ pts,
                                                const int64_t *__restrict__ woff, double *__restrict__ W64all,
                                                float *__restrict__ W32all, double *__restrict__ alpha64,
                                                uint8_t *__restrict__ pd, int kernel, double l, double s2,
                                                unsigned long long *__restrict__ stat) {
    // the thread index passes through an empty asm once per cluster: every
    // address derived from it is then formed inside the cluster's work, not
    // hoisted out of the persistent loop and held in registers throughout
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int kW = NT / 64;
    const int T = mfma_tiles(n);
    // A = K + s^2 I, padded with the identity; a tile per wavefront, lane l
    // on column l % 16 of rows l / 16 + 4 e, the five point loads together
    const int ntl = T * (T + 1) / 2;
    for (int t = wv; t < ntl; t += kW) {
        int ti = int((sqrtf(8.f * float(t) + 1.f) - 1.f) * 0.5f);
        if ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        if (ti * (ti + 1) / 2 > t) --ti;
        const int tj = t - ti * (ti + 1) / 2;
        const int g = lane >> 4, cc = lane & 15;
        const int j = tj * kTb + cc;
        const float4 pj = pts[base + min(j, n - 1)];
        float4 pi[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) pi[e] = pts[base + min(ti * kTb + g + 4 * e, n - 1)];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int rr = g + 4 * e, i = ti * kTb + rr;
            double v;
            if (i < n && j < n) {
                const double dx = double(pi[e].x) - double(pj.x), dy = double(pi[e].y) - double(pj.y),
                             dz = double(pi[e].z) - double(pj.z);
                v = kernel64(kernel, sqrt(dx * dx + dy * dy + dz * dz), l);
                if (i == j) v += s2;
            } else {
                v = i == j ? 1.0 : 0.0;
            }
            A[tlow(ti, tj) + tel(rr, cc)] = v;
        }
    }
    if (tid == 0) *flag = 1;
    __syncthreads();
    const double thr = 1e-10 * (1.0 + s2);
    // the diagonal tile of the next column is factored by wavefront 0 inside
    // the trailing update of the current one (its own update comes first)
    if (wv == 0 && !diag_factor(A, thr, lane) && lane == 0) *flag = 0;
    __syncthreads();
    for (int p = 0; p < T; ++p) {
        if (!*flag) break;
        // L_ip = A_ip V_p^T
        const double *Vp = A + tlow(p, p);
        for (int i = p + 1 + wv; i < T; i += kW) {
            double *X = A + tlow(i, p);
            const f64x4 acc = tile_xyt(X, Vp, f64x4{0.0, 0.0, 0.0, 0.0}, 1.0, lane);
            tile_put(X, acc, lane);
        }
        if (tid == 0) *next = 1;
        __syncthreads();
        // A_ij -= L_ip L_jp^T.  Trailing tile 0, the next diagonal tile, is
        // updated and factored by wavefront 0 first (look-ahead); the others
        // go in pairs (the second repeats the first when none is left and is
        // then not stored) to whichever wavefront takes the next pair from
        // the LDS counter, so wavefront 0 joins once it has factored
        const int m = T - 1 - p, nt = m * (m + 1) / 2;
        auto trail_tile = [&](int t, int &i, int &j) {
            int a = int((sqrtf(8.f * float(t) + 1.f) - 1.f) * 0.5f);
            if ((a + 1) * (a + 2) / 2 <= t) ++a;
            if (a * (a + 1) / 2 > t) --a;
            i = p + 1 + a;
            j = p + 1 + (t - a * (a + 1) / 2);
        };
        if (wv == 0 && nt > 0) {
            double *Y = A + tlow(p + 1, p + 1);
            const f64x4 acc = tile_xyt(A + tlow(p + 1, p), A + tlow(p + 1, p), tile_get(Y, lane), -1.0, lane);
            tile_put(Y, acc, lane);
            if (!diag_factor(Y, thr, lane) && lane == 0) *flag = 0;
        }
        while (true) {
            int t0 = 0;
            if (lane == 0) t0 = atomicAdd(next, 2);
            const int t = __builtin_amdgcn_readfirstlane(t0);
            if (t >= nt) break;
            const bool two = t + 1 < nt;
            int i1, j1, i2, j2;
            trail_tile(t, i1, j1);
            trail_tile(two ? t + 1 : t, i2, j2);
            double *Y1 = A + tlow(i1, j1), *Y2 = A + tlow(i2, j2);
            f64x4 acc1 = tile_get(Y1, lane), acc2 = tile_get(Y2, lane);
            tile_xyt2(A + tlow(i1, p), A + tlow(j1, p), acc1, A + tlow(i2, p), A + tlow(j2, p), acc2, -1.0, lane);
            tile_put(Y1, acc1, lane);
            if (two) tile_put(Y2, acc2, lane);
        }
        __syncthreads();
    }
    if (!*flag) {
        for (int i = tid; i < n; i += NT) {
            alpha64[base + i] = 0.0;
            pts[base + i].w = 0.0f;
        }
        if (tid == 0) {
            pd[c] = 0;
            atomicAdd(&stat[ST_NONPD], 1ull);
        }
        return;
    }
    // W = L^{-1} by tile columns, right to left
    for (int j = T - 1; j >= 0; --j) {
        const double *Vj = A + tlow(j, j);
        // M_kj = L_kj V_j
        for (int k = j + 1 + wv; k < T; k += kW) {
            double *X = A + tlow(k, j);
            const f64x4 acc = tile_xy(X, Vj, f64x4{0.0, 0.0, 0.0, 0.0}, lane);
            tile_put(X, acc, lane);
        }
        __syncthreads();
        // W_ij = -sum_k W_ik M_kj (i > j), kept in registers until every
        // product of the column has read its M tiles
        constexpr int kMaxOut = (kMfmaMaxN / kTb + kW - 1) / kW;
        f64x4 out[kMaxOut];
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o) {
            const int i = j + 1 + wv + o * kW;
            out[o] = f64x4{0.0, 0.0, 0.0, 0.0};
            if (i < T) {
                // two chains (k even and odd offsets) with their loads together
                f64x4 odd = f64x4{0.0, 0.0, 0.0, 0.0};
                int k = j + 1;
                for (; k + 1 <= i; k += 2)
                    tile_xy2(A + tlow(i, k), A + tlow(k, j), out[o], A + tlow(i, k + 1), A + tlow(k + 1, j), odd,
                             lane);
                if (k <= i) out[o] = tile_xy(A + tlow(i, k), A + tlow(k, j), out[o], lane);
                out[o] += odd;
            }
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < kMaxOut; ++o) {
            const int i = j + 1 + wv + o * kW;
            if (i < T) tile_put(A + tlow(i, j), -out[o], lane);
        }
        __syncthreads();
    }
    // y = W 1, alpha = W^T y
    for (int i = tid; i < n; i += NT) {
        const int ti = i / kTb, rr = i - ti * kTb;
        double s0 = 0.0;
        for (int tj = 0; tj <= ti; ++tj) {
            const double *X = A + tlow(ti, tj);
#pragma unroll
            for (int cc = 0; cc < kTb; ++cc) s0 += X[tel(rr, cc)];
        }
        ybuf[i] = s0;
    }
    __syncthreads();
    for (int j = tid; j < n; j += NT) {
        const int tj = j / kTb, cc = j - tj * kTb;
        // rows at or above j in the diagonal tile and the padded rows
        // contribute zeros (W is lower triangular, its padding block I
        // meets no real column)
        double a = 0.0;
        for (int ti = tj; ti < T; ++ti) {
            const double *X = A + tlow(ti, tj);
            double v[kTb];
#pragma unroll
            for (int rr = 0; rr < kTb; ++rr) v[rr] = X[tel(rr, cc)];
#pragma unroll
            for (int rr = 0; rr < kTb; ++rr) {
                const int i = ti * kTb + rr;
                if (i >= j && i < n) a += v[rr] * ybuf[i];
            }
        }
        alpha64[base + j] = a;
        pts[base + j].w = float(a);
    }
    // W in the query layout: 32-row panels, column-major inside, zero above
    // the diagonal
    float *W32 = W32all + woff[c];
    double *W64 = W64all + woff[c];
    const int nb = (n + kPanel - 1) / kPanel;
    for (int rp = 0; rp < nb; ++rp) {
        const int64_t po = w32_panel_offset(n, rp);
        const int ncol = min((rp + 1) * kPanel, n);
        for (int idx = tid; idx < ncol * kPanel; idx += NT) {
            const int jj = idx / kPanel, rr = idx - jj * kPanel;
            const int i = rp * kPanel + rr;
            double v = 0.0;
            if (i < n && jj <= i) {
                const int ti = i / kTb, tj = jj / kTb;
                v = A[tlow(ti, tj) + tel(i - ti * kTb, jj - tj * kTb)];
            }
            W32[po + idx] = float(v);
            W64[po + idx] = v;
        }
    }
    if (tid == 0) pd[c] = 1;
}

// persistent: each workgroup takes the next cluster of its bucket from the
// counter *work (zero at launch) until none is left.  LT > 0: the bucket's
// clusters have at most LT tile rows and keep their tiles in LDS, sized for
// LT, so that two or three small GPs share a CU; LT = 0: the tiles are in the
// FP64 workspace and the LDS holds only y.  WPE, the wavefronts per SIMD
// that the registers must allow, is the GPs per CU times NT / 256
template <int LT, int NT, int WPE, int NL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_train_mfma(
    const int32_t *__restrict__ list, const uint32_t *__restrict__ dcnt, int64_t lstride, uint32_t *__restrict__ work,
    float4 *__restrict__ pts, const int32_t *__restrict__ coff, const int64_t *__restrict__ aoff,
    const int64_t *__restrict__ woff, double *__restrict__ Aall, double *__restrict__ W64all,
    float *__restrict__ W32all, double *__restrict__ alpha64, uint8_t *__restrict__ pd, int kernel, double l,
    double s2, unsigned long long *__restrict__ stat) {
    static_assert(LT <= kMfmaLdsT, "LDS tiles beyond the bucket bound");
    __shared__ double sA[LT > 0 ? LT * (LT + 1) / 2 * kTileElems : 1];
    __shared__ double ybuf[LT > 0 ? LT * kTb : kMfmaMaxN];
    __shared__ int flag, next;
    __shared__ uint32_t item;
    // NL lists (lstride apart) with their counts at dcnt[0 .. NL - 1], taken
    // one after the other
    uint32_t lcnt[NL], cnt = 0;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        lcnt[k] = dcnt[k];
        cnt += lcnt[k];
    }
    while (true) {
        __syncthreads();  // the previous cluster is done with the LDS and item
        if (threadIdx.x == 0) item = atomicAdd(work, 1u);
        __syncthreads();
        uint32_t b = item;
        if (b >= cnt) break;
        int64_t lo = 0;
#pragma unroll
        for (int k = 0; k + 1 < NL; ++k) {
            if (lo == int64_t(k) * lstride && b >= lcnt[k]) {
                b -= lcnt[k];
                lo += lstride;
            }
        }
        const int c = list[lo + b];
        const int base = coff[c];
        const int n = coff[c + 1] - base;
        if constexpr (LT > 0) {
            if (mfma_tiles(n) > LT) continue;  // not of this bucket (the plan never puts it here)
            train_mfma_body<NT>(sA, ybuf, &flag, &next, c, base, n, pts, woff, W64all, W32all, alpha64, pd, kernel,
                                l, s2, stat);
        } else {
            train_mfma_body<NT>(Aall + aoff[c], ybuf, &flag, &next, c, base, n, pts, woff, W64all, W32all, alpha64,
                                pd, kernel, l, s2, stat);
        }
    }
}

// ---------------------------------------------------------------------------
// size buckets: n <= 8 one lane per cluster (registers), n <= 64 one
// wavefront per cluster (LDS), larger one workgroup per cluster (above)
// ---------------------------------------------------------------------------
constexpr int kTinyN = 8;
constexpr int kWaveN = 64;
// the bucket of a cluster of n points, 0 .. kBuckets - 1: one lane (n <= 8),
// one wavefront (n <= 64), the blocked trainer by tile rows T (T <= 6, 8, 12
// with the tiles in LDS; T = 16, 15, 14, 13 in the workspace, one list each
// so that its trainer takes the longest GPs first), one workgroup (larger)
__device__ inline int size_bucket(int n) {
    if (n <= kTinyN) return 0;
    if (n <= kWaveN) return 1;
    if (n > kMfmaMaxN) return CNT_HUGE - CNT_TINY;
    const int T = mfma_tiles(n);
    return T <= 6 ? 2 : T <= 8 ? 3 : T <= kMfmaLdsT ? 4 : 5 + (16 - T);
}
static_assert(kBuckets == 10 && CNT_BIG6 - CNT_TINY == 2 && CNT_T16 - CNT_TINY == 5 && CNT_T13 - CNT_TINY == 8 &&
                  kMfmaMaxN == 16 * kTb,
              "size buckets");
// appends cluster c to list b (lists of C entries, counts from CNT_TINY);
// b < 0 appends nothing (every lane of the wavefront calls it)
__device__ inline void bucket_append(int b, int64_t c, int32_t *__restrict__ list, int64_t C,
                                     uint32_t *__restrict__ cnt) {
#pragma unroll
    for (int k = 0; k < kBuckets; ++k) {
        const uint32_t r = wave_count32(&cnt[CNT_TINY + k], b == k);
        if (b == k) list[k * C + r] = int32_t(c);
    }
}

// store W (FP32 and FP64, packed rows), alpha and the positive-definite flag
__device__ inline void put_w(float *W32, double *W64, int64_t off, int idx, double w) {
    W32[off + idx] = float(w);
    W64[off + idx] = w;
}

__global__ __launch_bounds__(64) void k_train_tiny(
    const int32_t *__restrict__ list, const uint32_t *__restrict__ dcnt, float4 *__restrict__ pts,
    const int32_t *__restrict__ coff, const int64_t *__restrict__ woff, double *__restrict__ W64all,
    float *__restrict__ W32all, double *__restrict__ alpha64, uint8_t *__restrict__ pd, int kernel,
    double l, double s2, unsigned long long *__restrict__ stat) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(*dcnt)) return;
    const int c = list[t];
    const int base = coff[c];
    const int n = coff[c + 1] - base;
    double px[kTinyN], py[kTinyN], pz[kTinyN];
#pragma unroll
    for (int i = 0; i < kTinyN; ++i) {
        float4 p = i < n ? pts[base + i] : make_float4(0.f, 0.f, 0.f, 0.f);
        px[i] = p.x; py[i] = p.y; pz[i] = p.z;
    }
    // A = K + s^2 I, lower triangle packed by rows
    double L[kTinyN * (kTinyN + 1) / 2];
#pragma unroll
    for (int i = 0; i < kTinyN; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const double dx = px[i] - px[j], dy = py[i] - py[j], dz = pz[i] - pz[j];
            double v = kernel64(kernel, sqrt(dx * dx + dy * dy + dz * dz), l);
            if (i == j) v += s2;
            L[i * (i + 1) / 2 + j] = v;
        }
    // Cholesky, left-looking (the pivot test uses the original diagonal)
    const double thr = 1e-10 * (1.0 + s2);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kTinyN; ++j) {
        if (j < n) {
            double d = L[j * (j + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) d -= L[j * (j + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            ok = ok && (d > thr);
            const double ljj = sqrt(fmax(d, thr));
            L[j * (j + 1) / 2 + j] = ljj;
#pragma unroll
            for (int i = j + 1; i < kTinyN; ++i) {
                if (i < n) {
                    double sum = L[i * (i + 1) / 2 + j];
#pragma unroll
                    for (int k = 0; k < j; ++k) sum -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
                    L[i * (i + 1) / 2 + j] = sum / ljj;
                }
            }
        }
    }
    if (!ok) {
        for (int i = 0; i < n; ++i) { alpha64[base + i] = 0.0; pts[base + i].w = 0.0f; }
        pd[c] = 0;
        atomicAdd(&stat[ST_NONPD], 1ull);
        return;
    }
    // W = L^{-1} (packed rows), y = W 1, alpha = W^T y
    double W[kTinyN * (kTinyN + 1) / 2];
#pragma unroll
    for (int i = 0; i < kTinyN; ++i) {
        const double inv = 1.0 / L[i * (i + 1) / 2 + i];
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double sum = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int m = j; m < i; ++m) sum -= L[i * (i + 1) / 2 + m] * W[m * (m + 1) / 2 + j];
            W[i * (i + 1) / 2 + j] = sum * inv;
        }
    }
    double y[kTinyN];
#pragma unroll
    for (int i = 0; i < kTinyN; ++i) {
        double sum = 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) sum += (i < n) ? W[i * (i + 1) / 2 + j] : 0.0;
        y[i] = sum;
    }
    const int64_t off = woff[c];
#pragma unroll
    for (int j = 0; j < kTinyN; ++j) {
        if (j < n) {
            double a = 0.0;
#pragma unroll
            for (int i = j; i < kTinyN; ++i) a += (i < n) ? W[i * (i + 1) / 2 + j] * y[i] : 0.0;
            alpha64[base + j] = a;
            pts[base + j].w = float(a);
        }
    }
#pragma unroll
    for (int i = 0; i < kTinyN; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
            if (i < n) put_w(W32all, W64all, off, i * (i + 1) / 2 + j, W[i * (i + 1) / 2 + j]);
    pd[c] = 1;
}

// one wavefront per cluster, 8 < n <= 64; lane i owns row i of A in LDS
// (row stride 65 doubles: column reads by different lanes hit different
// banks); W = L^{-1} kept by packed columns, lane j owning column j
__global__ __launch_bounds__(64) void k_train_wave(
    const int32_t *__restrict__ list, const uint32_t *__restrict__ dcnt, float4 *__restrict__ pts,
    const int32_t *__restrict__ coff,
    const int64_t *__restrict__ woff, double *__restrict__ W64all, float *__restrict__ W32all,
    double *__restrict__ alpha64, uint8_t *__restrict__ pd, int kernel, double l, double s2,
    unsigned long long *__restrict__ stat) {
    constexpr int S = kWaveN + 1;
    __shared__ float sp[3][kWaveN];
    __shared__ double A[kWaveN * S];
    __shared__ double Wc[kWaveN * (kWaveN + 1) / 2];
    __shared__ double sy[kWaveN];
    const int lane = threadIdx.x;
    const int cnt = int(*dcnt);
    // persistent: workgroup b takes clusters b, b + gridDim.x, ...
    for (int b = blockIdx.x; b < cnt; b += gridDim.x) {
    __syncthreads();  // the previous cluster is done with the LDS
    const int c = list[b];
    const int base = coff[c];
    const int n = coff[c + 1] - base;
    if (lane < n) {
        const float4 p = pts[base + lane];
        sp[0][lane] = p.x; sp[1][lane] = p.y; sp[2][lane] = p.z;
    }
    __syncthreads();
    if (lane < n) {
        const double xi = sp[0][lane], yi = sp[1][lane], zi = sp[2][lane];
        for (int j = 0; j <= lane; ++j) {
            const double dx = xi - double(sp[0][j]), dy = yi - double(sp[1][j]), dz = zi - double(sp[2][j]);
            double v = kernel64(kernel, sqrt(dx * dx + dy * dy + dz * dz), l);
            if (j == lane) v += s2;
            A[lane * S + j] = v;
        }
    }
    __syncthreads();
    // right-looking Cholesky: lane i updates its own row
    const double thr = 1e-10 * (1.0 + s2);
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        int good = 1;
        if (lane == k) {
            const double d = A[k * S + k];
            good = d > thr;
            A[k * S + k] = sqrt(fmax(d, thr));
        }
        good = __shfl(good, k, 64);
        if (!good) { ok = false; break; }
        __syncthreads();
        const double lkk = A[k * S + k];
        if (lane > k && lane < n) A[lane * S + k] /= lkk;
        __syncthreads();
        if (lane > k && lane < n) {
            // four columns at a time, their loads before their stores: the
            // row elements (lane, j > k) written here are never the column
            // elements (j, k) read here (S > kWaveN), so they do not alias
            const double lik = A[lane * S + k];
            double *Ar = A + lane * S;
            int j = k + 1;
            for (; j + 3 <= lane; j += 4) {
                const double c0 = A[j * S + k], c1 = A[(j + 1) * S + k], c2 = A[(j + 2) * S + k],
                             c3 = A[(j + 3) * S + k];
                const double r0 = Ar[j], r1 = Ar[j + 1], r2 = Ar[j + 2], r3 = Ar[j + 3];
                Ar[j] = r0 - lik * c0;
                Ar[j + 1] = r1 - lik * c1;
                Ar[j + 2] = r2 - lik * c2;
                Ar[j + 3] = r3 - lik * c3;
            }
            for (; j <= lane; ++j) Ar[j] -= lik * A[j * S + k];
        }
    }
    if (!ok) {
        if (lane < n) { alpha64[base + lane] = 0.0; pts[base + lane].w = 0.0f; }
        if (lane == 0) { pd[c] = 0; atomicAdd(&stat[ST_NONPD], 1ull); }
        continue;
    }
    __syncthreads();
    // column j of W: W(j, j) = 1 / L(j, j), W(i, j) = -sum_{m=j}^{i-1} L(i, m) W(m, j) / L(i, i)
    if (lane < n) {
        const int j = lane;
        double *Wj = Wc + (j * n - j * (j - 1) / 2) - j;  // Wj[i] = W(i, j)
        Wj[j] = 1.0 / A[j * S + j];
        for (int i = j + 1; i < n; ++i) {
            const double *Li = A + i * S;
            double s0 = 0.0, s1 = 0.0;
            int m = j;
            for (; m + 1 < i; m += 2) { s0 += Li[m] * Wj[m]; s1 += Li[m + 1] * Wj[m + 1]; }
            if (m < i) s0 += Li[m] * Wj[m];
            Wj[i] = -(s0 + s1) / Li[i];
        }
    }
    __syncthreads();
    if (lane < n) {
        double sum = 0.0;
        for (int j = 0; j <= lane; ++j) sum += Wc[j * n - j * (j - 1) / 2 + (lane - j)];
        sy[lane] = sum;
    }
    __syncthreads();
    if (lane < n) {
        const int j = lane;
        const double *Wj = Wc + (j * n - j * (j - 1) / 2) - j;
        double a = 0.0;
        for (int i = j; i < n; ++i) a += Wj[i] * sy[i];
        alpha64[base + j] = a;
        pts[base + j].w = float(a);
    }
    // W in the query layout: packed rows up to 32 points, 32-row panels
    // (column-major inside, zero above the diagonal) above that
    const int64_t off = woff[c];
    if (n <= kPanel) {
        const int tot = n * (n + 1) / 2;
        for (int idx = lane; idx < tot; idx += 64) {
            int i = int((sqrt(8.0 * double(idx) + 1.0) - 1.0) * 0.5);
            while ((i + 1) * (i + 2) / 2 <= idx) ++i;
            while (i * (i + 1) / 2 > idx) --i;
            const int j = idx - i * (i + 1) / 2;
            put_w(W32all, W64all, off, idx, Wc[j * n - j * (j - 1) / 2 + (i - j)]);
        }
    } else {
        const int nb = (n + kPanel - 1) / kPanel;
        for (int r = 0; r < nb; ++r) {
            const int64_t po = off + w32_panel_offset(n, r);
            const int ncol = min((r + 1) * kPanel, n);
            for (int idx = lane; idx < ncol * kPanel; idx += 64) {
                const int j = idx / kPanel, i = r * kPanel + (idx - j * kPanel);
                const double w = (i < n && j <= i) ? Wc[j * n - j * (j - 1) / 2 + (i - j)] : 0.0;
                put_w(W32all, W64all, po, idx, w);
            }
        }
    }
    if (lane == 0) pd[c] = 1;
    }
}

// per-cluster storage: factor elements in the query layout and, above the
// LDS limit of the workgroup trainer, the packed FP64 workspace
__global__ void k_cluster_sizes(const int32_t *__restrict__ coff, int64_t nbound, const uint32_t *__restrict__ dcl,
                                uint32_t *__restrict__ wsz, uint32_t *__restrict__ asz, int max_cp,
                                uint32_t *__restrict__ maxn) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(nbound, dcl)) return;
    const int n = coff[c + 1] - coff[c];
    const bool ok = n <= max_cp && n <= kMaxClusterN;
    wsz[c] = ok ? uint32_t(w32_size(n)) : 0u;
    // FP64 workspace: tiles of the MFMA trainer above its LDS limit, the
    // packed triangle of the workgroup trainer above 256 points
    asz[c] = !ok ? 0u
             : n > kMfmaMaxN ? uint32_t(n * (n + 1) / 2)
             : (n > kWaveN && mfma_tiles(n) > kMfmaLdsT) ? uint32_t(mfma_ws(n)) : 0u;
    atomicMax(maxn, uint32_t(n));
}

// offsets and size buckets: n <= 8 to list[0..], n <= 64 to list[C..],
// n <= 256 to list[2C..], larger to list[3C..]; clusters that exceed a
// capacity are not trained (pd = 0) and counted
__global__ void k_cluster_plan(const int32_t *__restrict__ coff, int64_t nbound, const uint32_t *__restrict__ dcl,
                               const uint32_t *__restrict__ wsz, const uint32_t *__restrict__ asz,
                               const uint32_t *__restrict__ wo, const uint32_t *__restrict__ ao, int64_t cap_w,
                               int64_t cap_a, int max_cp, int64_t *__restrict__ woff, int64_t *__restrict__ aoff,
                               int32_t *__restrict__ list, int64_t C, uint32_t *__restrict__ cnt,
                               uint8_t *__restrict__ pd, unsigned long long *__restrict__ stat,
                               uint8_t *__restrict__ trained, int lazy) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = c < dev_count(nbound, dcl);
    int n = 0;
    bool ok = false;
    if (in) {
        n = coff[c + 1] - coff[c];
        ok = n <= max_cp && n <= kMaxClusterN && int64_t(wo[c]) + wsz[c] <= cap_w &&
             int64_t(ao[c]) + asz[c] <= cap_a;
        woff[c] = wo[c];
        aoff[c] = ao[c];
        if (!ok) {
            pd[c] = 0;
            atomicAdd(&stat[ST_CAPACITY], 1ull);
        }
        // lazy: selectable until a query's selection trains it
        if (lazy) {
            trained[c] = 0;
            if (ok) pd[c] = 1;
        }
    }
    if (lazy) return;
    bucket_append(in && ok ? size_bucket(n) : -1, c, list, C, cnt);
}

// lazy training: the marked clusters that are not trained yet into the size
// buckets (as k_cluster_plan), marked trained
__global__ void k_lazy_plan(const int32_t *__restrict__ coff, int64_t ncl, uint8_t *__restrict__ need,
                            uint8_t *__restrict__ trained, const uint8_t *__restrict__ pd,
                            int32_t *__restrict__ list, int64_t C, uint32_t *__restrict__ cnt) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool take = false;
    int n = 0;
    if (c < ncl && need[c]) {
        need[c] = 0;
        take = !trained[c] && pd[c];
        if (take) trained[c] = 1;
        n = coff[c + 1] - coff[c];
    }
    bucket_append(take ? size_bucket(n) : -1, c, list, C, cnt);
}

__global__ void k_copy_count(uint32_t *__restrict__ cnt, int dst, int src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) cnt[dst] = cnt[src];
}

__global__ void k_chash_insert(const uint64_t *__restrict__ ckey, int64_t nbound, const uint32_t *__restrict__ dn,
                               HashView h, int32_t *__restrict__ hval,
                               unsigned long long *__restrict__ stat) {
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= dev_count(nbound, dn)) return;
    bool ins;
    int64_t s = hash_insert(h, ckey[c], &ins);
    if (s < 0) {
        atomicAdd(&stat[ST_HASH_FULL], 1ull);
        return;
    }
    hval[s] = int32_t(c);
}

}  // namespace

// The trainers of the four size buckets (lists and counts from the plan):
// the two small-cluster trainers on s, the large-cluster ones on sb (forked
// from s; join_ev marks their end)
hipError_t launch_trainers(gpdf_ctx *c, int64_t C, hipStream_t s, hipStream_t sb) {
    hipError_t e;
    uint32_t *cnt = c->d_cnt;
    const double l = c->p.length_scale, s2 = c->p.noise_sigma * c->p.noise_sigma;
    // work counters: the workgroup trainer in slot 2, the four blocked
    // trainers on their own lines of slot 3, cleared before the fork
    fill_u32(c->d_work + 2 * kWorkSlot, 0u, 2 * kWorkSlot, s);
    // the blocked trainer with its tiles in the workspace on sb, those with
    // their tiles in LDS and the workgroup trainer on sb2 beside it, so that
    // each fills the CUs that the end of the other leaves idle (an LDS
    // trainer's workgroup cannot share a CU with one of 9-12 tile rows, so
    // the smaller buckets follow that one); sb2 joins sb
    hipStream_t sb2 = sb == s ? s : c->side2;
    if (sb != s) {
        if ((e = hipEventRecord(c->fork_ev, s)) != hipSuccess || (e = hipStreamWaitEvent(sb, c->fork_ev, 0)) != hipSuccess ||
            (e = hipStreamWaitEvent(sb2, c->fork_ev, 0)) != hipSuccess)
            return e;
    }
    {
        // grids: a CU holds three GPs of <= 6 tile rows, two of <= 8, one of
        // <= 12 (their LDS) and two with the tiles in the workspace (their
        // registers); the smaller GPs take four wavefronts each, the others
        // eight; a bucket never takes more workgroups than clusters
        uint32_t *w3 = c->d_work + 3 * kWorkSlot;
        const unsigned g1 = unsigned(std::min<int64_t>(C, 256)), g2 = unsigned(std::min<int64_t>(C, 512)),
                       g3 = unsigned(std::min<int64_t>(C, 768));
#define GPDF_TRAIN_MFMA(LT, NT, WPE, NL, G, B, K, ST)                                                           \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_train_mfma<LT, NT, WPE, NL>), dim3(G), dim3(NT), 0, ST, c->d_blist + (B - CNT_TINY) * C, \
                       cnt + B, C, w3 + K * kCtrStride, c->d_pts, c->d_coff, c->d_aoff, c->d_woff, c->d_A, c->d_W64,   \
                       c->d_W32, c->d_alpha64, c->d_pd, c->p.kernel, l, s2, c->d_stat)
        // largest first on each stream, so that the long GPs start early
        GPDF_TRAIN_MFMA(0, 256, 2, 4, g2, CNT_T16, 3, sb);
        GPDF_TRAIN_MFMA(12, 512, 2, 1, g1, CNT_BIG12, 2, sb2);
        GPDF_TRAIN_MFMA(8, 256, 2, 1, g2, CNT_BIG8, 1, sb2);
        GPDF_TRAIN_MFMA(6, 256, 3, 1, g3, CNT_BIG6, 0, sb2);
#undef GPDF_TRAIN_MFMA
    }
    {
        const unsigned gb = unsigned(std::min<int64_t>(C, 256));
#define GPDF_TRAIN_BLOCK(T)                                                                                    \
    hipLaunchKernelGGL(k_train_block<T>, dim3(gb), dim3(T), 0, sb2, c->d_blist + (CNT_HUGE - CNT_TINY) * C, cnt + CNT_HUGE, c->d_work + 2 * kWorkSlot, \
                       c->d_pts, c->d_coff, c->d_aoff, c->d_woff, c->d_A, c->d_W64, c->d_W32, c->d_alpha64,     \
                       c->d_pd, c->p.kernel, l, s2, c->d_stat)
        if (c->tune.train_threads == 512) GPDF_TRAIN_BLOCK(512);
        else if (c->tune.train_threads == 256) GPDF_TRAIN_BLOCK(256);
        else GPDF_TRAIN_BLOCK(1024);
#undef GPDF_TRAIN_BLOCK
    }
    if (sb != s && ((e = hipEventRecord(c->join2_ev, sb2)) != hipSuccess || (e = hipStreamWaitEvent(sb, c->join2_ev, 0)) != hipSuccess ||
                    (e = hipEventRecord(c->join_ev, sb)) != hipSuccess))
        return e;
    hipLaunchKernelGGL(k_train_tiny, dim3(blocks_for(C, 64)), dim3(64), 0, s, c->d_blist, cnt + CNT_TINY,
                       c->d_pts, c->d_coff, c->d_woff, c->d_W64, c->d_W32, c->d_alpha64, c->d_pd, c->p.kernel, l,
                       s2, c->d_stat);
    hipLaunchKernelGGL(k_train_wave, dim3(unsigned(std::min<int64_t>(C, 2048))), dim3(64), 0, s, c->d_blist + C,
                       cnt + CNT_WAVE, c->d_pts, c->d_coff, c->d_woff, c->d_W64, c->d_W32, c->d_alpha64, c->d_pd,
                       c->p.kernel, l, s2, c->d_stat);
    return hipGetLastError();
}

// Training of one frame.  Every count stays on the device (DevCount):
// grids are sized by the number of input points n and the capacities.  With
// dn (a device count of input points, at most n) nothing is read back, so the
// sequence can be captured in a graph; otherwise the counts and the
// capacity counter are read back once at the end.
gpdf_status train(gpdf_ctx *c, const float *d_xyz, int64_t n, const uint32_t *dn, const float *d_prop) {
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "train: join");
    hipStream_t s = c->stream;
    Model &M = c->model;
    const bool eager = dn == nullptr;
    if (n < 0 || n > c->p.max_points)
        return fail(c, GPDF_E_CAPACITY, "train: n exceeds max_points");
    M = Model();
    M.trained = true;
    if (d_prop && !c->d_cprop) return fail(c, GPDF_E_INVALID_ARG, "train: properties are off in the parameters");
    if (d_prop && (c->p.lazy_train || !eager))
        return fail(c, GPDF_E_INVALID_ARG, "train: a property needs eager, non-lazy training");
    M.props = d_prop != nullptr;
    uint32_t *cnt = c->d_cnt;
    FillList F;
    F.u32(cnt + CNT_VALID, 0u, CNT_MAXN - CNT_VALID + 1);
    F.u64(c->d_stat + ST_CAPACITY, 0ull, 1);
    F.u64(c->d_chash, (unsigned long long)kNoKey, int64_t(c->chash_mask) + 1);
    if (hipError_t fe = fill_multi(F, s); fe != hipSuccess) return hip_fail(c, fe, "train: clear");
    if (n == 0) {
        M.host_counts = true;
        return GPDF_OK;
    }
    const bool vox = c->p.voxel_size > 0.0;
    const double h = vox ? c->p.voxel_size : c->p.cluster_size;
    const int64_t C = std::min<int64_t>(n, c->p.max_clusters);  // bound of the cluster count
    hipError_t e;
    // 1. keys of the finite points, compacted in input order; the rest sorts last
    hipLaunchKernelGGL(k_point_keys, dim3(blocks_for(n)), dim3(kT), 0, s, d_xyz, n, dn, vox ? 1 : 0, h,
                       c->d_key, c->d_val, c->d_flag, c->d_stat);
    exclusive_scan_u32(c->d_flag, c->d_scan, n, c->d_part, s, nullptr, cnt + CNT_VALID);
    hipLaunchKernelGGL(k_compact_pairs, dim3(blocks_for(n)), dim3(kT), 0, s, c->d_key, c->d_val,
                       c->d_flag, c->d_scan, n, c->d_key2, c->d_val2);
    const unsigned g = std::min<unsigned>(blocks_for(n), 4096);
    hipLaunchKernelGGL(k_pad_keys, dim3(g), dim3(kT), 0, s, c->d_key2, c->d_val2, n, cnt + CNT_VALID);
    // 2. stable sort by key over all eight digits
    uint64_t *k = c->d_key2, *ka = c->d_key;
    uint32_t *v = c->d_val2, *va = c->d_val;
    radix_sort_pairs(k, ka, v, va, n, ~uint64_t(0), c->d_hist, c->d_part, s);
    // 3. unique voxels (voxel mode) and cluster runs
    uint64_t *keys = k;
    if (vox) {
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, k, n, cnt + CNT_VALID, 0, c->d_flag);
        exclusive_scan_u32(c->d_flag, c->d_scan, n, c->d_part, s, nullptr, cnt + CNT_PTS);
        hipLaunchKernelGGL(k_compact_unique, dim3(g), dim3(kT), 0, s, k, n, c->d_flag, c->d_scan, ka);
        if (d_prop)
            hipLaunchKernelGGL(k_point_prop, dim3(g), dim3(kT), 0, s, k, v, n, cnt + CNT_VALID, c->d_flag,
                               c->d_scan, d_prop, c->d_cprop);
        keys = ka;
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, keys, n, cnt + CNT_PTS, 9, c->d_flag);
    } else {
        hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, s, cnt, int(CNT_PTS), int(CNT_VALID));
        if (d_prop)
            hipLaunchKernelGGL(k_point_prop, dim3(g), dim3(kT), 0, s, keys, v, n, cnt + CNT_VALID, nullptr,
                               nullptr, d_prop, c->d_cprop);
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, keys, n, cnt + CNT_VALID, 0, c->d_flag);
    }
    exclusive_scan_u32(c->d_flag, c->d_scan, n, c->d_part, s);
    hipLaunchKernelGGL(k_clusters, dim3(g), dim3(kT), 0, s, keys, v, n, cnt + CNT_PTS, c->d_flag, c->d_scan,
                       vox ? 1 : 0, c->p.voxel_size, d_xyz, c->d_pts, c->d_coff, c->d_ckey, c->p.max_clusters,
                       cnt + CNT_CL, c->d_stat);
    // 4. factor storage (scans of the per-cluster sizes) and size buckets
    hipLaunchKernelGGL(k_cluster_sizes, dim3(blocks_for(C)), dim3(kT), 0, s, c->d_coff, C, cnt + CNT_CL,
                       c->d_wsz, c->d_asz, int(c->p.max_cluster_points), cnt + CNT_MAXN);
    exclusive_scan_u32(c->d_wsz, c->d_wo32, C, c->d_part, s, cnt + CNT_CL, cnt + CNT_WTOT);
    exclusive_scan_u32(c->d_asz, c->d_ao32, C, c->d_part, s, cnt + CNT_CL, cnt + CNT_ATOT);
    hipLaunchKernelGGL(k_cluster_plan, dim3(blocks_for(C)), dim3(kT), 0, s, c->d_coff, C, cnt + CNT_CL, c->d_wsz,
                       c->d_asz, c->d_wo32, c->d_ao32, c->cap_w, c->cap_a, int(c->p.max_cluster_points),
                       c->d_woff, c->d_aoff, c->d_blist, C, cnt, c->d_pd, c->d_stat, c->d_trained,
                       c->p.lazy_train);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return hip_fail(c, e2, "train: launch");
    if (!c->p.lazy_train) {
        // 5. FP64 training, one persistent launch per size bucket.  The
        //    large-cluster trainers (few workgroups, each for long) run on a
        //    second stream beside the other two; the buckets are disjoint.
        //    eager: the join is left to the first operation that needs the
        //    model (the test voxels of a fusion, which need only the points,
        //    run beside the trainer); a captured frame joins here (left to
        //    the query, its replays measured slower)
        if ((e = launch_trainers(c, C, s, c->side)) != hipSuccess) return hip_fail(c, e, "train: trainers");
        if (eager && !d_prop) c->join_pending = true;
        else if ((e = hipStreamWaitEvent(s, c->join_ev, 0)) != hipSuccess) return hip_fail(c, e, "train: join");
        // the property right-hand side on every factor (Eq. (6))
        if (d_prop)
            hipLaunchKernelGGL(k_beta, dim3(unsigned(std::min<int64_t>(C, 4096))), dim3(256), 0, s, c->d_coff, C,
                               cnt + CNT_CL, c->d_woff, c->d_W64, c->d_pd, c->d_cprop, c->d_beta64, c->d_beta32);
    }
    // 6. cluster hash
    HashView hv{c->d_chash, c->chash_mask};
    hipLaunchKernelGGL(k_chash_insert, dim3(blocks_for(C)), dim3(kT), 0, s, c->d_ckey, C, cnt + CNT_CL, hv,
                       c->d_chash_val, c->d_stat);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "train: launch");
    if (!eager) return GPDF_OK;
    // counts of the model and capacity check: one read-back
    static_assert(kCnt + 1 <= ReadList::kMax, "read-back list too short");
    ReadList R;
    R.u32(cnt, kCnt);
    R.u64(c->d_stat + ST_CAPACITY);
    if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "train: read counts");
    uint32_t hc[kCnt];
    for (int k = 0; k < kCnt; ++k) hc[k] = uint32_t(c->h_read[k]);
    const unsigned long long capx = c->h_read[kCnt];
    M.host_counts = true;
    M.lazy = c->p.lazy_train != 0;
    M.skipped = n - int64_t(hc[CNT_VALID]);
    M.npoints = hc[CNT_PTS];
    M.nclusters = hc[CNT_CL];
    M.ntrained = M.lazy ? 0 : M.nclusters;
    M.max_n = hc[CNT_MAXN];
    if (capx) {
        M.trained = false;
        return fail(c, GPDF_E_CAPACITY,
                    "train: capacity exceeded (max_clusters, max_cluster_points or max_factor_elems)");
    }
    return GPDF_OK;
}

}  // namespace gpdf

namespace gpdf {

gpdf_status lazy_train_round(gpdf_ctx *c, int64_t *ntrained) {
    hipStream_t s = c->stream;
    const Model &M = c->model;
    uint32_t *cnt = c->d_cnt;
    const int64_t C = std::max<int64_t>(M.nclusters, 1);
    hipError_t e;
    FillList F;
    F.u32(cnt + CNT_TINY, 0u, CNT_HUGE - CNT_TINY + 1);
    if ((e = fill_multi(F, s)) != hipSuccess) return hip_fail(c, e, "lazy: clear");
    hipLaunchKernelGGL(k_lazy_plan, dim3(blocks_for(M.nclusters)), dim3(kT), 0, s, c->d_coff, M.nclusters, c->d_need,
                       c->d_trained, c->d_pd, c->d_blist, C, cnt);
    ReadList R;
    for (int k = CNT_TINY; k <= CNT_HUGE; ++k) R.u32(cnt + k);
    if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "lazy: counts");
    int64_t tot = 0;
    for (int k = 0; k <= CNT_HUGE - CNT_TINY; ++k) tot += int64_t(c->h_read[k]);
    *ntrained = tot;
    c->model.ntrained += tot;
    if (tot == 0) return GPDF_OK;
    if ((e = launch_trainers(c, C, s, s)) != hipSuccess) return hip_fail(c, e, "lazy: trainers");
    return GPDF_OK;
}

}  // namespace gpdf

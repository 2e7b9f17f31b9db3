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
__global__ void k_point_keys(const float *__restrict__ xyz, int64_t n, int voxel_mode, double h,
                             uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                             uint32_t *__restrict__ flag, unsigned long long *__restrict__ stat) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
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

// OR over (key ^ key[0]): the bits that vary among the valid keys
__global__ void k_varying_bits(const uint64_t *__restrict__ key, const uint32_t *__restrict__ cnt,
                               unsigned long long *__restrict__ out) {
    const uint32_t n = *cnt;
    uint64_t acc = 0;
    if (n > 0) {
        const uint64_t k0 = key[0];
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
             i += int64_t(gridDim.x) * blockDim.x)
            acc |= key[i] ^ k0;
    }
    for (int o = 32; o > 0; o >>= 1) acc |= __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr(out, (unsigned long long)acc);
}

// flag[i] = 1 where (key >> sh) starts a new run
__global__ void k_run_flags(const uint64_t *__restrict__ key, int64_t n, int sh,
                            uint32_t *__restrict__ flag) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        flag[i] = (i == 0 || (key[i] >> sh) != (key[i - 1] >> sh)) ? 1u : 0u;
}

__global__ void k_compact_unique(const uint64_t *__restrict__ key, int64_t n,
                                 const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                                 uint64_t *__restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        if (flag[i]) out[pos[i]] = key[i];
}

// clusters: offsets, keys and training points.  voxel_mode: keys are the
// unique composite keys; raw mode: keys are cell keys, vals input indices.
__global__ void k_clusters(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val,
                           int64_t n, const uint32_t *__restrict__ flag,
                           const uint32_t *__restrict__ pos, int voxel_mode, double hv,
                           const float *__restrict__ xyz, float4 *__restrict__ pts,
                           int32_t *__restrict__ coff, uint64_t *__restrict__ ckey,
                           int64_t cap, uint32_t *__restrict__ ncl_out) {
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
            }
        } else {
            const uint32_t s = val[i];
            pts[i] = make_float4(xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2], 0.0f);
            if (flag[i] && int64_t(pos[i]) < cap) {
                const uint32_t c = pos[i];
                coff[c] = int32_t(i);
                ckey[c] = k;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t ncl = pos[n];
        if (int64_t(ncl) <= cap) coff[ncl] = int32_t(n);
        *ncl_out = ncl;
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

constexpr int kMaxLdsN = 64;
constexpr int kMaxClusterN = 1024;

__global__ __launch_bounds__(kT) void k_train_clusters(
    float4 *__restrict__ pts, const int32_t *__restrict__ coff, const int64_t *__restrict__ aoff,
    const int64_t *__restrict__ woff, const int64_t *__restrict__ wtoff, double *__restrict__ Aall,
    double *__restrict__ Wtall, double *__restrict__ W64all, float *__restrict__ W32all,
    double *__restrict__ alpha64,
    uint8_t *__restrict__ pd, int kernel, double l, double s2, unsigned long long *__restrict__ stat) {
    __shared__ float sx[kMaxClusterN], sy[kMaxClusterN], sz[kMaxClusterN];
    __shared__ double sA[kMaxLdsN * kMaxLdsN];
    __shared__ double sy1[kMaxClusterN];
    __shared__ int s_ok;
    const int c = blockIdx.x;
    const int base = coff[c];
    const int n = coff[c + 1] - base;
    const int tid = threadIdx.x;
    double *A = (n <= kMaxLdsN) ? sA : Aall + aoff[c];
    double *W = Wtall + wtoff[c];
    for (int i = tid; i < n; i += kT) {
        float4 p = pts[base + i];
        sx[i] = p.x; sy[i] = p.y; sz[i] = p.z;
    }
    __syncthreads();
    // A = K + s^2 I
    for (int64_t idx = tid; idx < int64_t(n) * n; idx += kT) {
        const int i = int(idx / n), j = int(idx - int64_t(i) * n);
        const double dx = double(sx[i]) - double(sx[j]);
        const double dy = double(sy[i]) - double(sy[j]);
        const double dz = double(sz[i]) - double(sz[j]);
        double v = kernel64(kernel, sqrt(dx * dx + dy * dy + dz * dz), l);
        if (i == j) v += s2;
        A[idx] = v;
    }
    // Cholesky, right-looking; a pivot at or below 1e-10 of the original
    // diagonal 1 + s^2 marks the cluster non positive definite
    const double thr = 1e-10 * (1.0 + s2);
    if (tid == 0) s_ok = 1;
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        if (tid == 0) {
            const double d = A[int64_t(k) * n + k];
            if (!(d > thr)) s_ok = 0;
            else A[int64_t(k) * n + k] = sqrt(d);
        }
        __syncthreads();
        if (!s_ok) break;
        const double lkk = A[int64_t(k) * n + k];
        for (int i = k + 1 + tid; i < n; i += kT) A[int64_t(i) * n + k] /= lkk;
        __syncthreads();
        for (int j = k + 1 + tid; j < n; j += kT) {
            const double ljk = A[int64_t(j) * n + k];
            for (int i = j; i < n; ++i) A[int64_t(i) * n + j] -= A[int64_t(i) * n + k] * ljk;
        }
    }
    __syncthreads();
    if (!s_ok) {
        for (int i = tid; i < n; i += kT) {
            alpha64[base + i] = 0.0;
            pts[base + i].w = 0.0f;
        }
        if (tid == 0) {
            pd[c] = 0;
            atomicAdd(&stat[ST_NONPD], 1ull);
        }
        return;
    }
    // W = L^{-1}, one column per thread; packed column-major storage:
    // column j holds rows j..n-1 starting at j n - j (j - 1) / 2
    for (int j = tid; j < n; j += kT) {
        double *Wj = W + (int64_t(j) * n - int64_t(j) * (j - 1) / 2) - j;  // Wj[i] = W(i, j)
        Wj[j] = 1.0 / A[int64_t(j) * n + j];
        for (int i = j + 1; i < n; ++i) {
            const double *Li = A + int64_t(i) * n;
            double s = 0.0;
            for (int m = j; m < i; ++m) s += Li[m] * Wj[m];
            Wj[i] = -s / Li[i];
        }
    }
    __threadfence_block();
    __syncthreads();
    // y = W 1 (row sums), alpha = W^T y
    for (int i = tid; i < n; i += kT) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += W[int64_t(j) * n - int64_t(j) * (j - 1) / 2 + (i - j)];
        sy1[i] = s;
    }
    __syncthreads();
    for (int j = tid; j < n; j += kT) {
        const double *Wj = W + (int64_t(j) * n - int64_t(j) * (j - 1) / 2) - j;
        double s = 0.0;
        for (int i = j; i < n; ++i) s += Wj[i] * sy1[i];
        alpha64[base + j] = s;
        pts[base + j].w = float(s);
    }
    // W in the query layout, FP32 and FP64: packed rows for n <= 64, 64-row
    // panels (column-major inside, zero above the diagonal) above that
    float *W32 = W32all + woff[c];
    double *W64 = W64all + woff[c];
    if (n <= kPanel) {
        for (int64_t idx = tid; idx < int64_t(n) * (n + 1) / 2; idx += kT) {
            // row i holds entries i (i + 1) / 2 .. i (i + 1) / 2 + i
            int i = int((sqrt(8.0 * double(idx) + 1.0) - 1.0) * 0.5);
            while (int64_t(i + 1) * (i + 2) / 2 <= idx) ++i;
            while (int64_t(i) * (i + 1) / 2 > idx) --i;
            const int j = int(idx - int64_t(i) * (i + 1) / 2);
            const double w = W[int64_t(j) * n - int64_t(j) * (j - 1) / 2 + (i - j)];
            W32[idx] = float(w);
            W64[idx] = w;
        }
    } else {
        const int nb = (n + kPanel - 1) / kPanel;
        for (int r = 0; r < nb; ++r) {
            const int64_t po = w32_panel_offset(n, r);
            const int ncol = std::min((r + 1) * kPanel, n);
            for (int idx = tid; idx < ncol * kPanel; idx += kT) {
                const int j = idx / kPanel, rr = idx - j * kPanel;
                const int i = r * kPanel + rr;
                double v = 0.0;
                if (i < n && j <= i) v = W[int64_t(j) * n - int64_t(j) * (j - 1) / 2 + (i - j)];
                W32[po + idx] = float(v);
                W64[po + idx] = v;
            }
        }
    }
    if (tid == 0) pd[c] = 1;
}

__global__ void k_chash_insert(const uint64_t *__restrict__ ckey, int64_t ncl, HashView h,
                               int32_t *__restrict__ hval, unsigned long long *__restrict__ stat) {
    int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncl) return;
    bool ins;
    int64_t s = hash_insert(h, ckey[c], &ins);
    if (s < 0) {
        atomicAdd(&stat[ST_HASH_FULL], 1ull);
        return;
    }
    hval[s] = int32_t(c);
}

}  // namespace

gpdf_status train(gpdf_ctx *c, const float *d_xyz, int64_t n) {
    hipStream_t s = c->stream;
    Model &M = c->model;
    if (n < 0 || n > c->p.max_points)
        return fail(c, GPDF_E_CAPACITY, "train: n exceeds max_points");
    M = Model();
    M.trained = true;
    if (n == 0) return GPDF_OK;
    const bool vox = c->p.voxel_size > 0.0;
    const double h = vox ? c->p.voxel_size : c->p.cluster_size;
    hipError_t e;
    // 1. keys of valid points, compacted in input order
    hipLaunchKernelGGL(k_point_keys, dim3(blocks_for(n)), dim3(kT), 0, s, d_xyz, n, vox ? 1 : 0, h,
                       c->d_key, c->d_val, c->d_flag, c->d_stat);
    exclusive_scan_u32(c->d_flag, c->d_scan, n, c->d_part, s);
    hipLaunchKernelGGL(k_compact_pairs, dim3(blocks_for(n)), dim3(kT), 0, s, c->d_key, c->d_val,
                       c->d_flag, c->d_scan, n, c->d_key2, c->d_val2);
    fill_u64(reinterpret_cast<unsigned long long *>(c->d_red), 0ull, 1, s);
    hipLaunchKernelGGL(k_varying_bits, dim3(256), dim3(kT), 0, s, c->d_key2, c->d_scan + n,
                       (unsigned long long *)c->d_red);
    uint32_t nvalid = 0;
    uint64_t vbits = 0;
    if ((e = hipMemcpyAsync(&nvalid, c->d_scan + n, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&vbits, c->d_red, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(c, e, "train: read counts");
    M.skipped = n - int64_t(nvalid);
    if (nvalid == 0) return GPDF_OK;
    // 2. stable sort by key
    uint64_t *k = c->d_key2, *ka = c->d_key;
    uint32_t *v = c->d_val2, *va = c->d_val;
    radix_sort_pairs(k, ka, v, va, nvalid, vbits, c->d_hist, c->d_part, s);
    // 3. unique voxels (voxel mode) and cluster runs
    uint64_t *keys = k;
    const unsigned g = std::min<unsigned>(blocks_for(nvalid), 4096);
    uint32_t npts = nvalid;
    if (vox) {
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, k, int64_t(nvalid), 0, c->d_flag);
        exclusive_scan_u32(c->d_flag, c->d_scan, nvalid, c->d_part, s);
        hipLaunchKernelGGL(k_compact_unique, dim3(g), dim3(kT), 0, s, k, int64_t(nvalid), c->d_flag,
                           c->d_scan, ka);
        keys = ka;
        if ((e = hipMemcpyAsync(&npts, c->d_scan + nvalid, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return hip_fail(c, e, "train: read voxel count");
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, keys, int64_t(npts), 9, c->d_flag);
    } else {
        hipLaunchKernelGGL(k_run_flags, dim3(g), dim3(kT), 0, s, keys, int64_t(npts), 0, c->d_flag);
    }
    exclusive_scan_u32(c->d_flag, c->d_scan, npts, c->d_part, s);
    uint32_t *d_ncl = reinterpret_cast<uint32_t *>(c->d_red) + 2;
    hipLaunchKernelGGL(k_clusters, dim3(g), dim3(kT), 0, s, keys, v, int64_t(npts), c->d_flag,
                       c->d_scan, vox ? 1 : 0, c->p.voxel_size, d_xyz, c->d_pts, c->d_coff,
                       c->d_ckey, c->p.max_clusters, d_ncl);
    uint32_t ncl = 0;
    if ((e = hipMemcpyAsync(&ncl, d_ncl, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(c, e, "train: read cluster count");
    if (int64_t(ncl) > c->p.max_clusters) {
        M.trained = false;
        return fail(c, GPDF_E_CAPACITY, "train: cluster count exceeds max_clusters");
    }
    // 4. factor storage offsets (host)
    std::vector<int32_t> off(ncl + 1);
    if ((e = hipMemcpyAsync(off.data(), c->d_coff, sizeof(int32_t) * (ncl + 1), hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(c, e, "train: read offsets");
    // kept in the context: the uploads below read them asynchronously
    std::vector<int64_t> &o32 = c->h_o32, &o64 = c->h_o64, &oa = c->h_oa;
    o32.assign(ncl, 0); o64.assign(ncl, 0); oa.assign(ncl, 0);
    int64_t s32 = 0, s64 = 0, sa = 0, maxn = 0;
    M.h_n.resize(ncl);
    for (uint32_t i = 0; i < ncl; ++i) {
        const int64_t nc = off[i + 1] - off[i];
        M.h_n[i] = int32_t(nc);
        maxn = std::max(maxn, nc);
        o32[i] = s32; s32 += w32_size(nc);
        o64[i] = s64; s64 += nc * (nc + 1) / 2;
        oa[i] = sa; if (nc > kMaxLdsN) sa += nc * nc;
    }
    if (maxn > c->p.max_cluster_points || maxn > kMaxClusterN) {
        M.trained = false;
        return fail(c, GPDF_E_CAPACITY, "train: a cluster exceeds max_cluster_points");
    }
    if (s32 > c->cap_w || s64 > c->cap_w || sa > c->cap_a) {
        M.trained = false;
        return fail(c, GPDF_E_CAPACITY, "train: factor storage exceeds max_factor_elems");
    }
    if ((e = hipMemcpyAsync(c->d_woff, o32.data(), 8 * ncl, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(c->d_wtoff, o64.data(), 8 * ncl, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(c->d_aoff, oa.data(), 8 * ncl, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(c, e, "train: upload offsets");
    // 5. FP64 training
    const double l = c->p.length_scale, s2 = c->p.noise_sigma * c->p.noise_sigma;
    hipLaunchKernelGGL(k_train_clusters, dim3(ncl), dim3(kT), 0, s, c->d_pts, c->d_coff, c->d_aoff,
                       c->d_woff, c->d_wtoff, c->d_A, c->d_Wt, c->d_W64, c->d_W32, c->d_alpha64, c->d_pd,
                       c->p.kernel, l, s2, c->d_stat);
    // 6. cluster hash
    fill_u64(c->d_chash, (unsigned long long)kNoKey, int64_t(c->chash_mask) + 1, s);
    HashView hv{c->d_chash, c->chash_mask};
    hipLaunchKernelGGL(k_chash_insert, dim3(blocks_for(ncl)), dim3(kT), 0, s, c->d_ckey, int64_t(ncl),
                       hv, c->d_chash_val, c->d_stat);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(c, e, "train: launch");
    M.nclusters = ncl;
    M.npoints = npts;
    M.max_n = maxn;
    return GPDF_OK;
}

}  // namespace gpdf

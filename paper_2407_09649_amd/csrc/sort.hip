// sort.hip -- device-wide exclusive scan, stable LSD radix sort of
// (uint64 key, uint32 value) pairs, and fill kernels.
//
// The radix sort is what makes every result-bearing order deterministic:
// clusters come out in ascending key order and members keep ascending voxel
// key (voxel mode) or input index (raw mode), independent of hash-slot races.
#include "gpdf_internal.hpp"

namespace gpdf {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096 elements per block

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// block-wide exclusive scan of one value per thread; returns the block total
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds_wave, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) lds_wave[wave] = inc;
    __syncthreads();
    uint32_t wave_off = 0, tot = 0;
    for (int w = 0; w < nwaves; ++w) {
        uint32_t s = lds_wave[w];
        if (w < wave) wave_off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return wave_off + inc - v;
}

// element count: the bound n, or the device count *dn when given (never
// above the bound)
__device__ __forceinline__ int64_t scan_count(int64_t n, const uint32_t *dn) {
    return dn ? min(n, int64_t(*dn)) : n;
}

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int64_t nb_, const uint32_t *__restrict__ dn,
                              uint32_t *__restrict__ partials) {
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t n = scan_count(nb_, dn);
    const int64_t base = int64_t(blockIdx.x) * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + int64_t(i) * kScanThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    uint32_t tot;
    block_exclusive_scan(s, lds, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// single block: exclusive scan of the block partials (any count)
__global__ void k_scan_partials(uint32_t *__restrict__ partials, int64_t nb) {
    __shared__ uint32_t lds[kScanThreads / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        int64_t idx = base + threadIdx.x;
        uint32_t v = idx < nb ? partials[idx] : 0;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, lds, tot);
        uint32_t c = carry;
        if (idx < nb) partials[idx] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

// each thread owns kScanItems consecutive elements
__global__ void k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                            int64_t nb_, const uint32_t *__restrict__ dn, const uint32_t *__restrict__ partials,
                            uint32_t *__restrict__ total_out) {
    __shared__ uint32_t lds[kScanThreads / 64];
    const int64_t n = scan_count(nb_, dn);
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot) + partials[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    // the total lands one past the end: written by the thread whose range
    // holds index n, or by the last thread when n fills the final tile
    const bool last = blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1;
    if ((base <= n && n < base + kScanItems) || (last && n == base + kScanItems)) {
        out[n] = run;
        if (total_out) *total_out = run;
    }
}

// one block for inputs up to a few tiles: the whole scan in one launch (most
// scans here are over per-cell, per-cluster or per-tile counts).  A tile is
// read and written with coalesced accesses through LDS; in LDS each thread
// owns kScan1Items consecutive elements (one pad word per kScan1Items keeps
// the strided accesses off a single bank).  Tiles run in order with a carry;
// a tile is read whole before it is written, so in place is fine.
constexpr int kScan1Threads = 1024;
constexpr int kScan1Items = 16;
constexpr int64_t kScan1Tile = int64_t(kScan1Threads) * kScan1Items;
constexpr int64_t kScan1Max = 4 * kScan1Tile;

__device__ __forceinline__ int scan1_pad(int j) { return j + j / kScan1Items; }

__device__ __forceinline__ void scan_single(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                            int64_t n, uint32_t *__restrict__ total_out) {
    __shared__ uint32_t lds[kScan1Threads / 64];
    __shared__ uint32_t buf[kScan1Tile + kScan1Tile / kScan1Items];
    const int t = int(threadIdx.x);
    uint32_t carry = 0;
    // the next tile's loads are issued before the current tile is scanned
    uint32_t nx[kScan1Items];
#pragma unroll
    for (int i = 0; i < kScan1Items; ++i) {
        const int j = i * kScan1Threads + t;
        nx[i] = j < n ? in[j] : 0u;
    }
    for (int64_t t0 = 0; t0 < n; t0 += kScan1Tile) {
#pragma unroll
        for (int i = 0; i < kScan1Items; ++i) buf[scan1_pad(i * kScan1Threads + t)] = nx[i];
        const int64_t t1 = t0 + kScan1Tile;
#pragma unroll
        for (int i = 0; i < kScan1Items; ++i) {
            const int64_t j = t1 + i * kScan1Threads + t;
            nx[i] = j < n ? in[j] : 0u;
        }
        __syncthreads();
        uint32_t v[kScan1Items];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kScan1Items; ++i) {
            v[i] = buf[scan1_pad(t * kScan1Items + i)];
            s += v[i];
        }
        uint32_t tot;
        uint32_t run = block_exclusive_scan(s, lds, tot) + carry;  // ends with a barrier
#pragma unroll
        for (int i = 0; i < kScan1Items; ++i) {
            buf[scan1_pad(t * kScan1Items + i)] = run;
            run += v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScan1Items; ++i) {
            const int j = i * kScan1Threads + t;
            if (t0 + j < n) out[t0 + j] = buf[scan1_pad(j)];
        }
        __syncthreads();  // buf is refilled by the next tile
        carry += tot;
    }
    if (t == 0) {
        out[n] = carry;
        if (total_out) *total_out = carry;
    }
}

__global__ __launch_bounds__(kScan1Threads) void k_scan_single(const uint32_t *__restrict__ in,
                                                               uint32_t *__restrict__ out, int64_t nb_,
                                                               const uint32_t *__restrict__ dn,
                                                               uint32_t *__restrict__ total_out) {
    scan_single(in, out, scan_count(nb_, dn), total_out);
}

// several independent scans of one length, one block each
__global__ __launch_bounds__(kScan1Threads) void k_scan_multi(ScanList L, int64_t nb_,
                                                              const uint32_t *__restrict__ dn) {
    const int k = int(blockIdx.x);
    scan_single(L.in[k], L.out[k], scan_count(nb_, dn), L.total[k]);
}

// ---------------------------------------------------------------------------
// radix sort, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsItems = 4;  // rounds per block: short serial chains, many blocks
constexpr int kRsTile = kRsThreads * kRsItems;
static_assert(kRsTile == kRsTileKeys, "histogram sizing");
constexpr int64_t kRsRawBlocks = 64;  // up to this many blocks the scatter scans the counts itself

__global__ void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                          uint32_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kRsTile;
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        int64_t idx = base + int64_t(r) * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = h[threadIdx.x];
}

// hist: the exclusive scan of the digit-major counts, or (raw != 0, for a
// few blocks) the counts themselves, from which each block forms its own
// offsets: the digits below d in all blocks plus digit d in the blocks before
__global__ void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                             uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n,
                             int shift, const uint32_t *__restrict__ hist, int64_t nblocks, int raw) {
    constexpr int W = kRsThreads / 64;
    __shared__ uint32_t base_d[256];
    __shared__ uint32_t wcnt[W][256];
    __shared__ uint32_t lds_w[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (raw) {
        uint32_t tot = 0, before = 0;
#pragma unroll 16
        for (int64_t b = 0; b < nblocks; ++b) {
            const uint32_t h = hist[int64_t(threadIdx.x) * nblocks + b];
            tot += h;
            before += b < int64_t(blockIdx.x) ? h : 0u;
        }
        uint32_t all;
        base_d[threadIdx.x] = block_exclusive_scan(tot, lds_w, all) + before;
    } else {
        base_d[threadIdx.x] = hist[int64_t(threadIdx.x) * nblocks + blockIdx.x];
    }
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t tile = int64_t(blockIdx.x) * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
#pragma unroll
        for (int w = 0; w < W; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t idx = tile + int64_t(r) * kRsThreads + threadIdx.x;
        const bool ok = idx < n;
        uint64_t k = ok ? kin[idx] : 0;
        uint32_t v = ok ? vin[idx] : 0;
        uint32_t d = uint32_t(k >> shift) & 0xFF;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const uint32_t below = __popcll(peers & lt);
        if (ok && below == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (ok) {
            uint32_t off = base_d[d] + below;
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            kout[off] = k;
            vout[off] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) add += wcnt[w][threadIdx.x];
        base_d[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void k_fill_multi(FillList L) {
    const FillOp o = L.op[blockIdx.y];
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < o.n; i += int64_t(gridDim.x) * blockDim.x) {
        if (o.bytes == 8) static_cast<unsigned long long *>(o.p)[i] = o.v;
        else static_cast<uint32_t *>(o.p)[i] = uint32_t(o.v);
    }
}

__global__ void k_read_words(ReadList L, unsigned long long *out) {
    const int i = int(threadIdx.x);
    if (i < L.count)
        out[i] = L.bytes[i] == 8 ? *static_cast<const unsigned long long *>(L.src[i])
                                 : (unsigned long long)(*static_cast<const uint32_t *>(L.src[i]));
    __threadfence_system();
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g > 65536) g = 65536;
    return unsigned(g < 1 ? 1 : g);
}

}  // namespace

void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                        hipStream_t s, const uint32_t *dn, uint32_t *total_out, bool by_count) {
    if (n <= kScan1Max || (by_count && dn)) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScan1Threads), 0, s, in, out, n, dn, total_out);
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, in, n, dn, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, in, out, n, dn,
                       partials, total_out);
}

void exclusive_scan_u32_multi(const ScanList &L, int64_t n, uint32_t *partials, hipStream_t s,
                              const uint32_t *dn, bool by_count) {
    if (n <= kScan1Max || (by_count && dn)) {
        hipLaunchKernelGGL(k_scan_multi, dim3(unsigned(L.count)), dim3(kScan1Threads), 0, s, L, n, dn);
        return;
    }
    for (int k = 0; k < L.count; ++k) exclusive_scan_u32(L.in[k], L.out[k], n, partials, s, dn, L.total[k]);
}

// Stable sort by key over the 8-bit digits that contain varying bits; the
// result ends in (keys, vals) (pointers are swapped as needed).  hist needs
// 256 * ceil(n / kRsTileKeys) entries, partials ceil(256 * ceil(n / kRsTileKeys) / 4096) + 1.
void radix_sort_pairs(uint64_t *&keys, uint64_t *&keys_alt, uint32_t *&vals, uint32_t *&vals_alt,
                      int64_t n, uint64_t varying_bits, uint32_t *hist, uint32_t *partials,
                      hipStream_t s) {
    if (n <= 1) return;
    const int64_t nb = (n + kRsTile - 1) / kRsTile;
    for (int shift = 0; shift < 64; shift += 8) {
        if (((varying_bits >> shift) & 0xFF) == 0) continue;
        hipLaunchKernelGGL(k_rs_hist, dim3(unsigned(nb)), dim3(kRsThreads), 0, s, keys, n, shift,
                           hist, nb);
        const int raw = nb <= kRsRawBlocks ? 1 : 0;
        if (!raw) exclusive_scan_u32(hist, hist, 256 * nb, partials, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(unsigned(nb)), dim3(kRsThreads), 0, s, keys, vals,
                           keys_alt, vals_alt, n, shift, hist, nb, raw);
        std::swap(keys, keys_alt);
        std::swap(vals, vals_alt);
    }
}

__global__ __launch_bounds__(256) void k_count_occupied(const unsigned long long *__restrict__ keys,
                                                        int64_t cap, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t wsum[4];
    const int64_t t0 = int64_t(blockIdx.x) * kCompactTile;
    uint32_t n = 0;
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t s = t0 + r * 256 + threadIdx.x;
        n += uint32_t(__popcll(__ballot(s < cap && keys[s] != kNoKey)));
    }
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

void count_occupied(const unsigned long long *keys, int64_t cap, uint32_t *tile_cnt,
                    uint32_t *tile_off, uint32_t *partials, hipStream_t s) {
    const int64_t nt = compact_tiles(cap);
    hipLaunchKernelGGL(k_count_occupied, dim3(unsigned(nt)), dim3(256), 0, s, keys, cap, tile_cnt);
    exclusive_scan_u32(tile_cnt, tile_off, nt, partials, s);
}

void fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
}
hipError_t read_back(gpdf_ctx *c, const ReadList &L, hipStream_t s) {
    if (L.overflow) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_read_words, dim3(1), dim3(ReadList::kMax), 0, s, L, c->h_read);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : hipStreamSynchronize(s);
}

hipError_t fill_multi(const FillList &L, hipStream_t s) {
    if (L.overflow) return hipErrorInvalidValue;
    if (L.count <= 0) return hipSuccess;
    int64_t nmax = 1;
    for (int k = 0; k < L.count; ++k) nmax = std::max(nmax, L.op[k].n);
    hipLaunchKernelGGL(k_fill_multi, dim3(std::min<unsigned>(grid_for(nmax, 256), 4096), unsigned(L.count)),
                       dim3(256), 0, s, L);
    return hipGetLastError();
}

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
}

// one thread per counter: sum its spread rows into the statistics array and
// clear them (stream-ordered after the kernels that added to them)
__global__ __launch_bounds__(64) void k_fold_stats(unsigned long long *sp, unsigned long long *stat) {
    const int st = int(threadIdx.x);
    if (st >= ST_COUNT) return;
    unsigned long long sum = 0;
    for (int r = 0; r < kSpread; ++r) {
        unsigned long long &x = sp[size_t(r) * kSpreadStride + st];
        sum += x;
        x = 0;
    }
    if (sum) atomicAdd(&stat[st], sum);
}

void fold_stats(unsigned long long *spread, unsigned long long *stat, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, s, spread, stat);
}

}  // namespace gpdf

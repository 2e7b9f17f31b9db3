// gpdf_internal.hpp -- internal declarations shared by the HIP sources of
// libvdbgpdf.so.  Not installed; the public interface is include/vdbgpdf.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vdbgpdf.h"

namespace gpdf {

// ---------------------------------------------------------------------------
// keys: integer cell coordinates c = floor(x / h) taken in FP64, packed as
// three 21-bit offset-binary fields (x high).  ~0 marks "no key".
// ---------------------------------------------------------------------------
constexpr int64_t kBias = int64_t(1) << 20;
constexpr uint64_t kNoKey = ~uint64_t(0);

__host__ __device__ inline uint64_t pack_key(int64_t cx, int64_t cy, int64_t cz) {
    return (uint64_t(cx + kBias) << 42) | (uint64_t(cy + kBias) << 21) | uint64_t(cz + kBias);
}
__host__ __device__ inline void unpack_key(uint64_t k, int64_t c[3]) {
    c[0] = int64_t((k >> 42) & 0x1FFFFF) - kBias;
    c[1] = int64_t((k >> 21) & 0x1FFFFF) - kBias;
    c[2] = int64_t(k & 0x1FFFFF) - kBias;
}
// floor(x / h) in FP64 with IEEE division; false for non-finite or out of range
__device__ inline bool cell_coord(float x, double h, int64_t &c) {
    if (!isfinite(x)) return false;
    double f = floor(__ddiv_rn(double(x), h));
    if (f < -double(kBias) || f >= double(kBias)) return false;
    c = int64_t(f);
    return true;
}
__host__ __device__ inline int64_t floor_div8(int64_t a) {  // arithmetic shift = floor
    return a >> 3;
}

// 64-bit finaliser of MurmurHash3 (Appleby), a bijective mixer
__host__ __device__ inline uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

// open-addressing table of 64-bit keys, linear probing, capacity 2^k
// One slot of the global grid: the voxel key and its fused D and V in one
// 16-byte record, so that a group of 8 slots fills one 128-byte line.
struct GSlot {
    unsigned long long key;    // kNoKey = empty
    float D, V;
};

struct HashView {
    unsigned long long *keys;  // kNoKey = empty
    uint32_t mask;             // capacity - 1
};

// find-or-insert; returns the slot or -1 if the probe sequence is exhausted.
// Within a launch a slot only goes from empty to a key, so a plain read that
// already shows the key (or another key) settles the probe without an
// atomic; only empty slots are claimed with compare-and-swap.
__device__ inline int64_t hash_insert(HashView h, uint64_t key, bool *inserted) {
    uint64_t s = mix64(key) & h.mask;
    for (uint32_t p = 0; p <= h.mask; ++p) {
        unsigned long long cur = __hip_atomic_load(&h.keys[s], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) { *inserted = false; return int64_t(s); }
        if (cur == kNoKey) {
            cur = atomicCAS(&h.keys[s], (unsigned long long)kNoKey, (unsigned long long)key);
            if (cur == kNoKey) { *inserted = true; return int64_t(s); }
            if (cur == key) { *inserted = false; return int64_t(s); }
        }
        s = (s + 1) & h.mask;
    }
    *inserted = false;
    return -1;
}

// Voxel tables hashed by 2x2x2 mini-brick: the key with the lowest bit of
// each coordinate cleared picks a group of 8 consecutive slots, the voxel's
// position in the brick (the three low bits) its slot in the group, and
// probing moves by whole groups (every voxel keeps one probe sequence).
// Neighbouring voxels then share cache lines.  The mask is at least 1023.
constexpr uint64_t kBrickLowBits = (1ull << 42) | (1ull << 21) | 1ull;
__device__ __forceinline__ uint64_t brick_slot(uint64_t key, uint32_t mask) {
    const uint64_t local = ((key >> 40) & 4ull) | ((key >> 20) & 2ull) | (key & 1ull);
    return ((mix64(key & ~kBrickLowBits) << 3) | local) & mask;
}

// hash_insert with the mini-brick probe sequence
__device__ inline int64_t brick_insert(HashView h, uint64_t key, bool *inserted) {
    uint64_t s = brick_slot(key, h.mask);
    const uint32_t ngroups = (h.mask >> 3) + 1;
    for (uint32_t p = 0; p < ngroups; ++p) {
        unsigned long long cur = __hip_atomic_load(&h.keys[s], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) { *inserted = false; return int64_t(s); }
        if (cur == kNoKey) {
            cur = atomicCAS(&h.keys[s], (unsigned long long)kNoKey, (unsigned long long)key);
            if (cur == kNoKey) { *inserted = true; return int64_t(s); }
            if (cur == key) { *inserted = false; return int64_t(s); }
        }
        s = (s + 8) & h.mask;
    }
    *inserted = false;
    return -1;
}

__device__ inline int64_t hash_find(const unsigned long long *__restrict__ keys, uint32_t mask,
                                    uint64_t key) {
    uint64_t s = mix64(key) & mask;
    for (uint32_t p = 0; p <= mask; ++p) {
        unsigned long long k = keys[s];
        if (k == key) return int64_t(s);
        if (k == kNoKey) return -1;
        s = (s + 1) & mask;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// wavefront-aggregated atomics: one atomic per wavefront (or per distinct
// address in the wavefront) instead of one per lane
// ---------------------------------------------------------------------------
__device__ inline uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// adds pred ? 1 : 0 per lane to *ctr; returns this lane's slot (valid when pred)
__device__ inline unsigned long long wave_count(unsigned long long *ctr, bool pred) {
    const uint64_t mb = __ballot(pred);
    if (!mb) return 0;
    const int leader = __ffsll((long long)mb) - 1;
    unsigned long long base = 0;
    if ((threadIdx.x & 63) == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(mb));
    base = __shfl(base, leader, 64);
    return base + __popcll(mb & lanes_below());
}

// per-lane increment of cnt[slot] returning the lane's rank, aggregated over
// the lanes of the wavefront that share a slot (slot < 0: no increment)
__device__ inline uint32_t wave_rank(uint32_t *cnt, int64_t slot) {
    uint32_t rank = 0;
    uint64_t todo = __ballot(slot >= 0);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int64_t s0 = __shfl(slot, leader, 64);
        const uint64_t grp = __ballot(slot == s0) & todo;
        uint32_t base = 0;
        if ((threadIdx.x & 63) == leader) base = atomicAdd(&cnt[s0], uint32_t(__popcll(grp)));
        base = __shfl(base, leader, 64);
        if (slot == s0) rank = base + uint32_t(__popcll(grp & lanes_below()));
        todo &= ~grp;
    }
    return rank;
}

// ---------------------------------------------------------------------------
// slot-ordered compaction of an open-addressing table: a block of 256 threads
// owns a tile of kCompactTile consecutive slots; count_occupied() gives each
// tile's first output index, for_occupied_in_tile() numbers the occupied
// slots of the calling block's tile in slot order (deterministic output, one
// pass over the keys each, no global atomics)
// ---------------------------------------------------------------------------
constexpr int kCellListStride = 28;  // int4 entries per cell list: count + 27 descriptors
// cells of the fixed cell-list scratch of the allocation-free query (28 MiB)
constexpr int64_t kNoAllocCells = int64_t(1) << 16;
constexpr int kCompactItems = 16;
constexpr int kCompactTile = 256 * kCompactItems;

// mask of the smallest power-of-two table (at least 1024 slots) holding want
inline uint32_t pow2_mask(int64_t want) {
    uint64_t cap = 1024;
    while (int64_t(cap) < want) cap <<= 1;
    return uint32_t(cap - 1);
}

inline int64_t compact_tiles(int64_t cap) { return (cap + kCompactTile - 1) / kCompactTile; }

template <class Body>
__device__ __forceinline__ void for_occupied_in_tile(const unsigned long long *__restrict__ keys,
                                                     int64_t cap, uint32_t base, Body body) {
    __shared__ uint32_t wsum[4];
    const int w = threadIdx.x >> 6;
    const int64_t t0 = int64_t(blockIdx.x) * kCompactTile;
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t s = t0 + r * 256 + threadIdx.x;
        const unsigned long long k = s < cap ? keys[s] : kNoKey;
        const uint64_t b = __ballot(k != kNoKey);
        if ((threadIdx.x & 63) == 0) wsum[w] = uint32_t(__popcll(b));
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int i = 0; i < 4; ++i) {
            before += i < w ? wsum[i] : 0u;
            tot += wsum[i];
        }
        if (k != kNoKey) body(s, k, base + before + uint32_t(__popcll(b & lanes_below())));
        __syncthreads();
        base += tot;
    }
}

// ---------------------------------------------------------------------------
// counts that stay on the device (u32), so that a whole frame can run
// without a host round trip
// ---------------------------------------------------------------------------
enum DevCount : int {
    CNT_IN = 0,   // points of the frame (graph input)
    CNT_VALID,    // finite points
    CNT_PTS,      // training points (unique voxels or valid points)
    CNT_CL,       // clusters
    CNT_TINY,     // size buckets: n <= 8, n <= 64, then by 16-row tiles T:
    CNT_WAVE,     // T <= 6, T <= 8, T <= 12, then T = 16, 15, 14, 13 (tiles
    CNT_BIG6,     // in the workspace, one trainer launch over the four lists,
    CNT_BIG8,     // longest first), larger than 256 points
    CNT_BIG12,
    CNT_T16,
    CNT_T15,
    CNT_T14,
    CNT_T13,
    CNT_HUGE,
    CNT_WTOT,     // factor elements
    CNT_ATOT,     // FP64 workspace elements
    CNT_MAXN,     // largest cluster
    CNT_CELLS,    // query cells
    CNT_CHUNKS,   // query chunks
    CNT_RCHUNKS,  // re-evaluation chunks
    CNT_TEST,     // test voxels (clamped to max_queries)
    CNT_FRAME,    // frame stamp (graph input)
    CNT_M,        // query count read by the kernels (graph)
    CNT_BPAIRS_S, // cluster-major re-evaluation: (refined query, cluster) pairs, clusters of <= one panel
    CNT_BPAIRS_B, // the same, larger clusters
    CNT_BITEMS,   // work items of the larger clusters
    CNT_BITEMS_S, // work items of the clusters of <= one panel
    CNT_BIGOK,    // 1 when the pairs fit the buffers
    CNT_NREF_FAST,// refined queries for the combination of the pass's pairs (0: the pass did not take all)
    CNT_RCH_SLOW, // re-evaluation chunks for the FP64 query kernel (0 when the pass took all)
    kCnt
};

// adds pred ? 1 : 0 per lane to a u32 counter; returns the lane's slot
__device__ inline uint32_t wave_count32(uint32_t *ctr, bool pred) {
    const uint64_t mb = __ballot(pred);
    if (!mb) return 0;
    const int leader = __ffsll((long long)mb) - 1;
    uint32_t base = 0;
    if ((threadIdx.x & 63) == leader) base = atomicAdd(ctr, uint32_t(__popcll(mb)));
    base = __shfl(base, leader, 64);
    return base + uint32_t(__popcll(mb & lanes_below()));
}

// a count bounded by n, read on the device when dn is given
__device__ __forceinline__ int64_t dev_count(int64_t n, const uint32_t *dn) {
    return dn ? (int64_t(*dn) < n ? int64_t(*dn) : n) : n;
}

// ---------------------------------------------------------------------------
// device status block (uint64 counters)
// ---------------------------------------------------------------------------
enum Stat : int {
    ST_SKIPPED_POINTS = 0,
    ST_NONPD,
    ST_NONFINITE_Q,
    ST_VALID_Q,
    ST_REFINE,       // number of refine records
    ST_HASH_FULL,
    ST_GLOBAL_FULL,
    ST_FUSED,
    ST_FUSE_SKIPPED,
    ST_GLOBAL_COUNT, // voxels in the global grid
    ST_CELLS,        // query cells of the last query call
    ST_CHUNKS,       // query chunks of the last query call
    ST_TESTPTS,      // unique test voxels of the last frame
    ST_GATED,
    ST_PAIRS,        // (query, cluster) pairs of the last evaluation pass
    ST_POINTS,       // kernel evaluations (sum of n over pairs)
    ST_TRI,          // variance multiply-adds (sum of n (n + 1) / 2 over pairs)
    ST_REF_D,        // last query: FP32 error estimates above the distance,
    ST_REF_G,        // gradient and variance thresholds
    ST_REF_V,
    ST_CAPACITY,     // a capacity was exceeded on the device (clusters, cluster
                     // size, factor storage, test voxels)
    ST_COUNT
};

// Per-wavefront statistics of the hot kernels are spread over kSpread rows
// of counters, one 128-byte line each, picked by the workgroup index: device
// atomics on one address serialise, and tens of thousands of wavefronts
// adding to a single line queue behind each other.  fold_stats adds the rows
// into the statistics array and clears them (a kernel, so that it can be
// captured in a graph).
// Work counters of persistent launches: a slot per launch kind (0 FP32 /
// FP64 evaluation, 1 FP64 re-evaluation, 2 large-cluster training), each
// with one counter per XCD on its own 128-byte line.
constexpr int kXcds = 8;
constexpr int kCtrStride = 32;                     // u32 per counter line
constexpr int kWorkSlot = kXcds * kCtrStride;
constexpr int kWorkSlots = 4;
constexpr int kBuckets = CNT_HUGE - CNT_TINY + 1;  // training size buckets (lists of C clusters each)
constexpr unsigned kGraphEvalGrid0 = 1024;  // captured grid of the graph's evaluation node, before any replay

constexpr int kSpread = 64;
constexpr int kSpreadStride = 16 * ((ST_COUNT + 15) / 16);
static_assert(ST_COUNT <= 64, "fold_stats takes one lane per counter");
__device__ __forceinline__ void spread_add(unsigned long long *sp, int st, unsigned long long v) {
    atomicAdd(&sp[size_t(blockIdx.x % kSpread) * kSpreadStride + st], v);
}
// adds the wavefront's count of pred to counter st of the spread rows; no
// value comes back, so no lane waits for the atomic
__device__ __forceinline__ void spread_count(unsigned long long *sp, int st, bool pred) {
    const uint64_t mb = __ballot(pred);
    if (mb && int(threadIdx.x & 63) == __ffsll((long long)mb) - 1) spread_add(sp, st, __popcll(mb));
}

// per-cluster FP32 factor layout: packed rows for n <= 32, 32-row panels
// (column-major inside the panel) above that
constexpr int kPanel = 32;
// tail pads of the FP32 point and factor arrays (zero at create): the FP32
// evaluation loads whole groups of rows or column pairs and reads up to
// kPanel points and kPanel^2 factor elements past the last cluster
constexpr int64_t kPtsPad = 2 * kPanel;
constexpr int64_t kW32Pad = 2 * kPanel * kPanel;
__host__ __device__ inline int64_t w32_size(int64_t n) {
    if (n <= kPanel) return n * (n + 1) / 2;
    int64_t nb = (n + kPanel - 1) / kPanel, s = 0;
    for (int64_t r = 0; r < nb; ++r) s += int64_t(kPanel) * ((r + 1) * kPanel < n ? (r + 1) * kPanel : n);
    return s;
}
__host__ __device__ inline int64_t w32_panel_offset(int64_t n, int64_t r) {
    int64_t s = 0;
    for (int64_t q = 0; q < r; ++q) s += int64_t(kPanel) * ((q + 1) * kPanel < n ? (q + 1) * kPanel : n);
    return s;
}

// query arithmetic knobs passed by value to the kernels
struct QueryConsts {
    float l, a;             // length scale and sqrt(3)/l (Matern) or 1/l (SE)
    float c;                // l / sqrt(3) (Matern) or l (SE)
    float lam;              // smooth-minimum lambda
    float omin, omax;
    float tau_d, tau_g, tau_v;  // FP32 error-estimate thresholds for FP64 refinement
    float tau_c;                // the same for the surface property (absolute)
    float err_c;            // error-bound constant on sum |alpha k|
    int kernel, combine, grad_mode, knn_q;
    int signed_, has_origin_pad;
    float ox, oy, oz;       // sensor origin (signed queries)
    const float *d_origin;  // when set, the origin is read here on the device (graph replays)
    double ld, sd, hv, hc;  // FP64 copies: l, s, voxel, cell
    double lamd, omind, omaxd;
    double ad, cd;          // FP64 copies of a and c
    float cap_hi[3], cap_lo[3];     // d, Lambda, gradient scale at occ_max and occ_min
    double cap_hid[3], cap_lod[3];  // the same in FP64
};

struct Model {
    int64_t nclusters = 0, npoints = 0, nonpd = 0, skipped = 0, max_n = 0;
    bool trained = false;
    bool bf16_ready = false;   // BF16 copies of [W; alpha] built for this model
    bool host_counts = false;  // counts below were read back (eager calls)
    bool lazy = false;         // clusters are factored when a query selects them
    bool props = false;        // trained with a surface property (beta valid)
    int64_t ntrained = 0;      // clusters factored (host count, eager calls)
};

}  // namespace gpdf

// launch shapes picked by the autotuner (defaults until it runs)
struct gpdf_tune {
    int train_threads = 1024;  // workgroup of the large-cluster trainer: 256, 512 or 1024
    int eval_persistent = 0;   // evaluation: 0 = one workgroup per chunk, else persistent waves per SIMD
    int mfma_min_n = 0;        // FP32 evaluation: clusters of at least this size (to 248) take the
                               // variance product on FP32 MFMA; 0 = VALU only
    int tuned = 0;
};

struct gpdf_ctx {
    gpdf_params p{};
    gpdf_tune tune;
    bool capturing = false;        // recording the frame graph: no read-backs, no stage events
    bool offs_ready = false;       // band offsets of the test voxels uploaded
    // per-frame graph (fuse_frame with every count on the device)
    hipStream_t gstream = nullptr; // capture stream
    // the captured frame's FP32 evaluation: its one-workgroup-per-chunk node,
    // whose grid is set before each replay (captured, largest, current), the
    // chunks that node took (device word, written by it, read by the
    // persistent instance after it), the chunk count of the last replay
    // (pinned host word and its device address)
    hipGraphNode_t geval_node = nullptr;
    hipKernelNodeParams geval_params{};
    bool geval_ok = false;
    unsigned geval_grid0 = 0, geval_gridmax = 0, geval_cur = 0;
    uint32_t *d_gfirst = nullptr;
    uint32_t *h_gchunks = nullptr, *d_gchunks = nullptr;
    hipStream_t side = nullptr;    // second stream: the large-cluster trainers beside the others
    hipStream_t side2 = nullptr;   // third stream: the blocked trainers with their tiles in LDS
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, join2_ev = nullptr;
    // an eager training leaves the large-cluster trainer running on `side`;
    // the first later operation that needs the model (or its buffers) makes
    // the caller's stream wait for join_ev (join_train)
    bool join_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    float *d_gin = nullptr;        // input points of the graph [max_points][3]
    float *d_gorigin = nullptr;    // sensor origin of the graph [4]
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    gpdf::Model model;

    // ---- training arenas --------------------------------------------------
    uint64_t *d_key = nullptr, *d_key2 = nullptr;  // sort keys  [max_points]
    uint32_t *d_val = nullptr, *d_val2 = nullptr;  // sort values
    uint32_t *d_flag = nullptr, *d_scan = nullptr; // [max_points + 1]
    uint32_t *d_hist = nullptr;                    // radix histograms
    uint32_t *d_part = nullptr;                    // scan partials
    uint64_t *d_red = nullptr;                     // small reductions
    uint32_t *d_work = nullptr;                    // work counters of persistent launches [kWorkSlots][kWorkSlot]
    uint32_t *d_cnt = nullptr;                     // device counts [kCnt]
    uint32_t *d_wsz = nullptr, *d_asz = nullptr;   // per-cluster factor / workspace sizes
    uint32_t *d_wo32 = nullptr, *d_ao32 = nullptr; // their exclusive scans
    float4 *d_pts = nullptr;                       // training points (x, y, z, alpha32)
    double *d_alpha64 = nullptr;                   // alpha in FP64
    double *d_cprop = nullptr;                     // property of each training point (FP64), properties = 1
    double *d_beta64 = nullptr;                    // (K + s^2 I)^{-1} c per point (Eq. (6))
    float *d_beta32 = nullptr;                     // its FP32 copy, with a zero tail pad of 64
    uint64_t *d_ckey = nullptr;                    // cluster keys [max_clusters]
    int32_t *d_coff = nullptr;                     // CSR offsets  [max_clusters + 1]
    uint8_t *d_pd = nullptr;                       // positive definite
    int64_t *d_woff = nullptr;                     // factor offsets, query layout
    int64_t *d_aoff = nullptr;                     // workspace offsets
    float *d_W32 = nullptr;                        // L^{-1} in FP32, query layout
    double *d_W64 = nullptr;                       // L^{-1} in FP64, query layout
    uint32_t *d_tile_cnt = nullptr, *d_tile_off = nullptr;  // table compaction
    void *d_bfM = nullptr;                         // BF16 [W; alpha] per cluster (precision BF16)
    int64_t *d_bfoff = nullptr;                    // their offsets (elements)
    int64_t cap_bfM = 0, cap_bfoff = 0;
    std::vector<int64_t> h_bfoff;
    double *d_A = nullptr;                         // FP64 workspace: packed A, L, then L^{-1} (n > 192)
    int64_t cap_w = 0, cap_a = 0;
    int32_t *d_blist = nullptr;
    uint8_t *d_need = nullptr, *d_trained = nullptr;  // lazy training: selected / factored clusters
    unsigned long long *d_chash = nullptr;         // cluster hash keys
    int32_t *d_chash_val = nullptr;
    uint32_t chash_mask = 0;

    // ---- query arenas ------------------------------------------------------
    unsigned long long *d_qhash = nullptr;         // cell table keys
    uint32_t *d_qhash_cnt = nullptr;               // queries per slot
    int32_t *d_qhash_cell = nullptr;               // slot -> cell id
    uint32_t qhash_mask = 0;
    int32_t *d_qslot = nullptr;                    // per query slot (-1 invalid)
    uint32_t *d_qrank = nullptr;                   // rank inside the cell
    uint32_t *d_order = nullptr;                   // queries in cell order
    uint64_t *d_cell_key = nullptr;                // per cell
    uint32_t *d_cell_cnt = nullptr, *d_cell_off = nullptr;
    uint32_t *d_cell_chunks = nullptr, *d_chunk_off = nullptr;
    int4 *d_cell_list = nullptr;                   // [cells][28]: count, cluster descriptors
    int64_t cap_cells = 0;                         // cells the lists hold
    int4 *scratch_lists = nullptr;                 // this device's fixed cell lists (noalloc query)
    uint2 *d_chunk = nullptr;                      // (cell, start)
    uint2 *d_refine = nullptr;                     // (cell, query) records to redo in FP64
    uint32_t *d_rcnt = nullptr, *d_roff = nullptr; // refine records per cell
    uint32_t *d_rchunks = nullptr, *d_rchunk_off = nullptr;
    uint32_t *d_rorder = nullptr, *d_rrank = nullptr;
    uint2 *d_rchunk = nullptr;
    // cluster-major re-evaluation: per cell (at its first chunk index) and
    // descriptor the cell's first slot in the cluster's run; per cluster the
    // pair count, run offset, the counts and offsets split by size class, and
    // the item counts and offsets of the larger clusters; the items, each
    // pair's query and result slot, and the reverted pairs (struct BigOut, 80 bytes)
    int64_t cap_bchunks = 0, cap_bpairs = 0;
    uint32_t *d_bbase = nullptr, *d_bcnt = nullptr, *d_boff = nullptr;
    uint32_t *d_bcs = nullptr, *d_boffs = nullptr, *d_bcb = nullptr, *d_boffb = nullptr;
    uint32_t *d_bnit = nullptr, *d_bioff = nullptr, *d_bnits = nullptr, *d_bioffs = nullptr;
    uint2 *d_bitem = nullptr, *d_bitems = nullptr;
    uint32_t *d_bq = nullptr;                     // per pair: query,
    uint32_t *d_bdst = nullptr;                   //   result slot s * cap_bref + (refine position)
    int64_t cap_bref = 0;                         // refined queries the result layout holds
    uint32_t *d_rcell = nullptr;                  // cell of each refined query (refine order)
    void *d_bres = nullptr;
    float *d_tmp_dist = nullptr, *d_tmp_var = nullptr, *d_tmp_grad = nullptr;
    uint8_t *d_tmp_valid = nullptr;

    // ---- fusion / global grid ---------------------------------------------
    unsigned long long *d_tset = nullptr;          // test-voxel set keys
    uint32_t tset_mask = 0;
    unsigned long long *d_vhash = nullptr;         // ray-cast test points: training voxel keys
    uint32_t vhash_mask = 0;
    uint64_t *d_tkeys = nullptr;                   // compacted test keys
    float *d_tpts = nullptr;                       // test points [3]
    gpdf::GSlot *d_gslot = nullptr;                // global grid slots (key, D, V)
    uint32_t *d_gstamp = nullptr;
    float2 *d_gprop = nullptr;                     // per slot: fused property C and its variance or weight W
                                                   // (NaN: none fused yet), properties = 1
    float *d_tprop = nullptr, *d_tpropv = nullptr; // property query of the test voxels
    uint32_t gmask = 0;
    uint32_t frame = 0;
    std::vector<int4> h_offs;                      // band offsets (host)
    int4 *d_offs = nullptr;
    int64_t offs_cap = 0;
    // zero crossings of the grid (G-GPDF input), grown on demand
    uint64_t *d_zkey = nullptr, *d_zkey2 = nullptr;
    uint32_t *d_zslot = nullptr, *d_zslot2 = nullptr, *d_zcnt = nullptr, *d_zoff = nullptr;
    uint32_t *d_zhist = nullptr, *d_zpart = nullptr, *d_ztile = nullptr, *d_ztoff = nullptr;
    int64_t zcap = 0, ztiles = 0;
    int64_t last_test = 0;

    // ---- MLP ----------------------------------------------------------------
    float *d_mlp_w = nullptr;       // FP32 master weights [8897]
    float *d_mlp_m = nullptr, *d_mlp_v = nullptr;  // Adam moments
    float *d_mlp_g = nullptr;       // reduced gradient [8897]
    float *d_mlp_rec = nullptr;     // per-wavefront gradient records
    void *d_mlp_pack = nullptr;     // BF16 copies of the weight matrices
    float *d_mlp_norm = nullptr;    // mean[7], std[7]
    float *d_mlp_loss = nullptr;    // per-wavefront losses + accumulator
    double *d_mlp_mom = nullptr;    // feature moments (standardisation)
    int64_t mlp_step = 0;           // Adam step counter
    bool mlp_ready = false;
    int64_t adam_t = 0;

    // ---- stage timers (GPDF_MS_*) -------------------------------------------
    hipEvent_t ev[16] = {};
    bool ev_ok[8] = {};

    // ---- counters ----------------------------------------------------------
    unsigned long long *d_stat = nullptr;          // [ST_COUNT]
    unsigned long long *d_spread = nullptr;        // [kSpread][kSpreadStride], zero between calls
    unsigned long long *h_stat = nullptr;          // pinned mirror
    unsigned long long *h_read = nullptr;          // pinned words of read_back()
    int64_t last_queries = 0;
};

namespace gpdf {
// stage timers: HIP events recorded on the context stream when p.timing is set
inline void stage_begin(gpdf_ctx *c, int k) {
    if (c->p.timing && !c->capturing) (void)hipEventRecord(c->ev[2 * k], c->stream);
}
inline void stage_end(gpdf_ctx *c, int k) {
    if (c->p.timing && !c->capturing) {
        if (c->join_pending) {
            // the stage ends when both streams have: record on `side` after
            // it has waited for the caller's stream (which does not wait)
            (void)hipEventRecord(c->fork_ev, c->stream);
            (void)hipStreamWaitEvent(c->side, c->fork_ev, 0);
            (void)hipEventRecord(c->ev[2 * k + 1], c->side);
        } else {
            (void)hipEventRecord(c->ev[2 * k + 1], c->stream);
        }
        c->ev_ok[k] = true;
    }
}
// makes the caller's stream wait for a pending large-cluster trainer
inline hipError_t join_train(gpdf_ctx *c) {
    if (!c->join_pending) return hipSuccess;
    c->join_pending = false;
    return hipStreamWaitEvent(c->stream, c->join_ev, 0);
}
// error helpers
gpdf_status fail(gpdf_ctx *c, gpdf_status s, const std::string &msg);
gpdf_status hip_fail(gpdf_ctx *c, hipError_t e, const char *what);

// scans and sorting (sort.hip)
// out[i] = sum_{j < i} in[j] for i <= n (out has n + 1 entries).  With dn,
// the count is min(n, *dn) read on the device (n is then a bound that sizes
// the grid); total_out, when given, receives the total.  partials needs
// ceil(n / 4096) + 1 entries.  by_count (with dn): one block whatever n, its
// work following *dn, for a count known to be small beside a loose bound n
// (a captured graph, which cannot read the count back to size the scan).
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                        hipStream_t s, const uint32_t *dn = nullptr, uint32_t *total_out = nullptr,
                        bool by_count = false);
// up to four exclusive scans of the same length n (and device count dn),
// each as exclusive_scan_u32: one launch when n is small, else one after
// the other (the partials are then shared in stream order)
struct ScanList {
    static constexpr int kMax = 4;
    const uint32_t *in[kMax] = {};
    uint32_t *out[kMax] = {};
    uint32_t *total[kMax] = {};
    int count = 0;
    void add(const uint32_t *i, uint32_t *o, uint32_t *t) {
        in[count] = i;
        out[count] = o;
        total[count] = t;
        ++count;
    }
};
void exclusive_scan_u32_multi(const ScanList &L, int64_t n, uint32_t *partials, hipStream_t s,
                              const uint32_t *dn = nullptr, bool by_count = false);
void radix_sort_pairs(uint64_t *&keys, uint64_t *&keys_alt, uint32_t *&vals, uint32_t *&vals_alt,
                      int64_t n, uint64_t varying_bits, uint32_t *hist, uint32_t *partials,
                      hipStream_t s);
// occupied slots (key != kNoKey) per tile of kCompactTile slots, scanned:
// tile_off[t] = first output index of tile t, tile_off[ntiles] = total
void count_occupied(const unsigned long long *keys, int64_t cap, uint32_t *tile_cnt,
                    uint32_t *tile_off, uint32_t *partials, hipStream_t s);
// keys per block of the radix sort (its histogram holds 256 counts per block)
constexpr int64_t kRsTileKeys = 1024;
void fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t s);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);

// several fills in one launch (counters and tables cleared together at the
// start of a call, where each separate launch would cost a host round trip)
struct FillOp {
    void *p;
    unsigned long long v;
    int64_t n;
    int bytes;  // 4 or 8
};
struct FillList {
    static constexpr int kMax = 12;
    FillOp op[kMax];
    int count = 0;
    bool overflow = false;  // an op past kMax was dropped (fill_multi then fails)
    void add(const FillOp &o) {
        if (count < kMax) op[count++] = o;
        else overflow = true;
    }
    void u64(unsigned long long *p, unsigned long long v, int64_t n) { add(FillOp{p, v, n, 8}); }
    void u32(uint32_t *p, uint32_t v, int64_t n) { add(FillOp{p, v, n, 4}); }
};
hipError_t fill_multi(const FillList &L, hipStream_t s);

// small read-backs: one kernel stores the listed device words into the
// context's pinned host words (as u64), then the stream is synchronised
struct ReadList {
    static constexpr int kMax = 32;
    const void *src[kMax];
    int bytes[kMax];
    int count = 0;
    bool overflow = false;  // a word past kMax was dropped (read_back then fails)
    void add(const void *p, int b) {
        if (count < kMax) { src[count] = p; bytes[count++] = b; }
        else overflow = true;
    }
    void u32(const uint32_t *p, int n = 1) {
        for (int k = 0; k < n; ++k) add(p + k, 4);
    }
    void u64(const unsigned long long *p) { add(p, 8); }
};
void fold_stats(unsigned long long *spread, unsigned long long *stat, hipStream_t s);
// the values land in c->h_read[0 .. L.count)
hipError_t read_back(gpdf_ctx *c, const ReadList &L, hipStream_t s);
void grid_clear(gpdf_ctx *c, hipStream_t s);

// stages (train.hip, query.hip, fuse.hip, mlp.hip)
// d_prop (may be NULL): a surface property per input point (Eq. (6))
gpdf_status train(gpdf_ctx *c, const float *d_xyz, int64_t n, const uint32_t *dn = nullptr,
                  const float *d_prop = nullptr);
// With dm (a device count of queries, at most m) and optionally d_origin, the
// call reads nothing back and can be captured in a graph.
gpdf_status scratch_setup(gpdf_ctx *c);
gpdf_status query(gpdf_ctx *c, const float *d_q, int64_t m, const float *origin, float *dist,
                  float *grad, float *var, uint8_t *valid, float *aux, int32_t correct,
                  const uint32_t *dm = nullptr, const float *d_origin = nullptr, bool noalloc = false,
                  float *prop = nullptr, float *prop_var = nullptr);
gpdf_status fuse(gpdf_ctx *c, const float *origin, const float *d_origin = nullptr, int64_t npts_bound = -1);
gpdf_status query_global_prop(gpdf_ctx *c, const float *d_q, int64_t m, float *prop, uint8_t *valid);
gpdf_status zero_crossings(gpdf_ctx *c, float *d_out, int64_t cap, int64_t *count);
// lazy training: factor the clusters marked in d_need that are not trained
// yet (one round; *ntrained receives their number)
gpdf_status lazy_train_round(gpdf_ctx *c, int64_t *ntrained);
gpdf_status ensure_offsets(gpdf_ctx *c);
gpdf_status query_global(gpdf_ctx *c, const float *d_q, int64_t m, float *dist, float *grad,
                         uint8_t *valid);
gpdf_status nearest_distance(gpdf_ctx *c, const float *pts, int64_t n, const float *q, int64_t m,
                             float *out);
gpdf_status mlp_apply(gpdf_ctx *c, const float *d_dist, const float *d_var, const float *d_grad,
                      const float *d_aux, const uint8_t *valid, int64_t m, float *dist_out);
QueryConsts make_consts(const gpdf_params &p, const float *origin, const float *d_origin = nullptr);
hipError_t ensure_cell_lists(gpdf_ctx *c, int64_t cap);
}  // namespace gpdf

// fuse.hip -- test points, probabilistic fusion into the global grid, and the
// global query (Sec. IV-B, IV-C, Eq. (7)-(8)).
//
// The global VDB is replaced by an open-addressing hash of voxel keys with
// structure-of-arrays payload (D, V, stamp).  Test voxels are unique per
// frame, so every voxel has at most one writer per fusion launch and the
// update needs no floating-point atomics.
#include "gpdf_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace gpdf {

namespace {

constexpr int kT = 256;

inline unsigned blocks_for(int64_t n, int t = kT) {
    int64_t g = (n + t - 1) / t;
    return unsigned(g < 1 ? 1 : g);
}

// candidate test voxels: the global-grid cell of every training point plus
// every integer offset inside the band ball
__global__ void k_test_insert(const float4 *__restrict__ pts, int64_t nb, const uint32_t *__restrict__ dn, double hf,
                              const int4 *__restrict__ offs, int noffs, HashView set,
                              unsigned long long *__restrict__ stat) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= dev_count(nb, dn) * noffs) return;
    const int64_t i = t / noffs;
    const int k = int(t - i * noffs);
    const float4 p = pts[i];
    int64_t c[3];
    if (!(cell_coord(p.x, hf, c[0]) && cell_coord(p.y, hf, c[1]) && cell_coord(p.z, hf, c[2]))) return;
    const int4 o = offs[k];
    const int64_t v[3] = {c[0] + o.x, c[1] + o.y, c[2] + o.z};
    for (int a = 0; a < 3; ++a)
        if (v[a] < -kBias || v[a] >= kBias) return;
    bool ins;
    // by mini-brick: the voxels of one ball share lines, and the compaction
    // (slot order) hands the fusion neighbouring voxels together
    if (brick_insert(set, pack_key(v[0], v[1], v[2]), &ins) < 0) atomicAdd(&stat[ST_HASH_FULL], 1ull);
}

__global__ __launch_bounds__(256) void k_test_compact(
    const unsigned long long *__restrict__ keys, int64_t cap, const uint32_t *__restrict__ tile_off,
    int64_t ntiles, uint64_t *__restrict__ out, int64_t out_cap, double hf, float *__restrict__ xyz,
    unsigned long long *__restrict__ stat, uint32_t *__restrict__ ntest) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t t = tile_off[ntiles];
        stat[ST_TESTPTS] = t;
        *ntest = uint32_t(min(int64_t(t), out_cap));
        if (int64_t(t) > out_cap) atomicAdd(&stat[ST_CAPACITY], 1ull);
    }
    for_occupied_in_tile(keys, cap, tile_off[blockIdx.x], [&](int64_t, unsigned long long k, uint32_t id) {
        if (int64_t(id) >= out_cap) return;
        out[id] = k;
        int64_t c[3];
        unpack_key(k, c);
        // voxel centre (c + 1/2) h formed in FP64, rounded once
        xyz[3 * int64_t(id)] = float((double(c[0]) + 0.5) * hf);
        xyz[3 * int64_t(id) + 1] = float((double(c[1]) + 0.5) * hf);
        xyz[3 * int64_t(id) + 2] = float((double(c[2]) + 0.5) * hf);
    });
}

// Slots of the global grid, by mini-brick (brick_slot): a group of 8 slots
// is one 128-byte line, and the 8 voxel centres around a point lie in 1 to 8
// lines (3.4 on average) instead of 8 scattered slots, each with its D and V
// beside it.
__device__ __forceinline__ uint64_t grid_start(uint64_t key, uint32_t gmask) { return brick_slot(key, gmask); }

// find-or-insert (claims an empty slot with compare-and-swap); -1 when full
__device__ inline int64_t grid_insert(GSlot *g, uint32_t gmask, uint64_t key, bool *inserted) {
    uint64_t s = grid_start(key, gmask);
    const uint32_t ngroups = (gmask >> 3) + 1;
    for (uint32_t p = 0; p < ngroups; ++p) {
        unsigned long long cur = __hip_atomic_load(&g[s].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == key) { *inserted = false; return int64_t(s); }
        if (cur == kNoKey) {
            cur = atomicCAS(&g[s].key, (unsigned long long)kNoKey, (unsigned long long)key);
            if (cur == kNoKey) { *inserted = true; return int64_t(s); }
            if (cur == key) { *inserted = false; return int64_t(s); }
        }
        s = (s + 8) & gmask;
    }
    *inserted = false;
    return -1;
}

// D of a voxel, continuing a probe at slot s whose record e is already read
__device__ inline bool grid_resolve(const GSlot *__restrict__ g, uint32_t gmask, uint64_t key, uint64_t s,
                                    GSlot e, float *D) {
    const uint32_t ngroups = (gmask >> 3) + 1;
    for (uint32_t p = 0; p < ngroups; ++p) {
        if (e.key == key) { *D = e.D; return true; }
        if (e.key == kNoKey) return false;
        s = (s + 8) & gmask;
        e = g[s];
    }
    return false;
}

// the slot of a voxel, or -1 when the grid does not hold it
__device__ inline int64_t grid_find(const GSlot *__restrict__ g, uint32_t gmask, uint64_t key) {
    uint64_t s = grid_start(key, gmask);
    const uint32_t ngroups = (gmask >> 3) + 1;
    for (uint32_t p = 0; p < ngroups; ++p) {
        const uint64_t k = g[s].key;
        if (k == key) return int64_t(s);
        if (k == kNoKey) return -1;
        s = (s + 8) & gmask;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// ray-cast test points (Sec. IV-B): for every training voxel, the global
// voxels on the ray from the sensor that the grid already holds (previously
// observed surface), the measured voxel itself, and the voxels along its
// surface normal up to the normal reach R (in global voxels).
// ---------------------------------------------------------------------------
// the training voxels (keys at the training voxel size), for the normals
__global__ void k_vox_insert(const float4 *__restrict__ pts, int64_t nb, const uint32_t *__restrict__ dn, double hv,
                             HashView vh, unsigned long long *__restrict__ stat) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= dev_count(nb, dn)) return;
    const float4 p = pts[i];
    int64_t c[3];
    if (!(cell_coord(p.x, hv, c[0]) && cell_coord(p.y, hv, c[1]) && cell_coord(p.z, hv, c[2]))) return;
    bool ins;
    if (hash_insert(vh, pack_key(c[0], c[1], c[2]), &ins) < 0) atomicAdd(&stat[ST_HASH_FULL], 1ull);
}

__device__ inline void test_add(HashView set, const int64_t v[3], unsigned long long *stat) {
    if (v[0] < -kBias || v[0] >= kBias || v[1] < -kBias || v[1] >= kBias || v[2] < -kBias || v[2] >= kBias) return;
    bool ins;
    if (brick_insert(set, pack_key(v[0], v[1], v[2]), &ins) < 0) atomicAdd(&stat[ST_HASH_FULL], 1ull);
}

__device__ inline int64_t igcd(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// The ray of every training voxel: an exact integer walk between the
// centres of the origin's voxel O and the measured voxel E that visits every
// voxel the segment passes through.  With A = |E - O| per axis the n-th
// boundary crossing on axis a lies at parameter (2n + 1) / (2 A_a); each
// step takes the axis of the smallest such parameter (cross-multiplied in
// integers), the lower axis at equal parameters.  The voxels the grid holds
// before this frame are test voxels (E itself is added by k_normal_tests).
// kRaySeg lanes share a ray: lane j walks the crossings with parameter in
// [j / kRaySeg, (j + 1) / kRaySeg), starting from the counts of the crossings
// before it (n with (2n + 1) kRaySeg < 2 j A_a), so the crossings of one
// parameter stay in one piece and the pieces visit exactly the voxels of the
// whole walk; piece 0 also probes O.
constexpr int kRaySeg = 16;

__device__ inline int64_t crossings_before(int64_t jj, int64_t A) {
    const int64_t num = 2 * jj * A - kRaySeg, den = 2 * kRaySeg;
    const int64_t c = num <= 0 ? 0 : (num + den - 1) / den;
    return c < A ? c : A;
}

__global__ __launch_bounds__(256) void k_ray_walk(const float4 *__restrict__ pts, int64_t nb,
                                                  const uint32_t *__restrict__ dn, double hf, float ox, float oy,
                                                  float oz, const float *__restrict__ d_origin,
                                                  const GSlot *__restrict__ g, uint32_t gmask, HashView set,
                                                  unsigned long long *__restrict__ stat) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = t / kRaySeg;
    const int j = int(t - i * kRaySeg);
    if (i >= dev_count(nb, dn)) return;
    if (d_origin) { ox = d_origin[0]; oy = d_origin[1]; oz = d_origin[2]; }
    int64_t O[3], E[3];
    if (!(cell_coord(ox, hf, O[0]) && cell_coord(oy, hf, O[1]) && cell_coord(oz, hf, O[2]))) return;
    const float4 p = pts[i];
    if (!(cell_coord(p.x, hf, E[0]) && cell_coord(p.y, hf, E[1]) && cell_coord(p.z, hf, E[2]))) return;
    int64_t A[3], st[3], n[3], cur[3], total = 0, k = 0, steps = 0;
    for (int a = 0; a < 3; ++a) {
        const int64_t d = E[a] - O[a];
        A[a] = d < 0 ? -d : d;
        st[a] = d < 0 ? -1 : 1;
        total += A[a];
        n[a] = crossings_before(j, A[a]);
        steps += crossings_before(j + 1, A[a]) - n[a];
        k += n[a];
        cur[a] = O[a] + st[a] * n[a];
    }
    if (total == 0) return;
    if (j == 0 && grid_find(g, gmask, pack_key(O[0], O[1], O[2])) >= 0) test_add(set, O, stat);
    // kRayBatch steps at a time: the walk does not depend on the probes, so
    // the first slot of every step's voxel is loaded together
    constexpr int kRayBatch = 8;
    for (int64_t s0i = 0; s0i < steps; s0i += kRayBatch) {
        uint64_t key[kRayBatch], sl[kRayBatch];
        GSlot e[kRayBatch];
        bool use[kRayBatch];
#pragma unroll
        for (int b = 0; b < kRayBatch; ++b) {
            use[b] = false;
            if (s0i + b < steps) {
                int ax = -1;
                for (int a = 0; a < 3; ++a) {
                    if (n[a] >= A[a]) continue;
                    if (ax < 0 || (2 * n[a] + 1) * A[ax] < (2 * n[ax] + 1) * A[a]) ax = a;
                }
                cur[ax] += st[ax];
                ++n[ax];
                ++k;
                use[b] = k < total;   // the last position is E
            }
            key[b] = pack_key(cur[0], cur[1], cur[2]);
            sl[b] = grid_start(key[b], gmask);
        }
#pragma unroll
        for (int b = 0; b < kRayBatch; ++b)
            if (use[b]) e[b] = g[sl[b]];
#pragma unroll
        for (int b = 0; b < kRayBatch; ++b) {
            float D;
            if (use[b] && grid_resolve(g, gmask, key[b], sl[b], e[b], &D)) {
                int64_t v[3];
                unpack_key(key[b], v);
                test_add(set, v, stat);
            }
        }
    }
}

// One lane per training voxel: the measured voxel E and the voxels along its
// normal.  The normal: among the integer directions d with components in
// [-2, 2] (primitive, first non-zero component positive, in lexicographic
// order), the first minimising d^T M d / |d|^2 with M = N S2 - s1 s1^T over
// the training voxels within +-2 voxels (N, s1 = sum of offsets, S2 = sum of
// their outer products), compared exactly; no normal with fewer than 3.
__global__ __launch_bounds__(256) void k_normal_tests(const float4 *__restrict__ pts, int64_t nb,
                                                      const uint32_t *__restrict__ dn, double hv, double hf, int R,
                                                      HashView vh, HashView set,
                                                      unsigned long long *__restrict__ stat) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= dev_count(nb, dn)) return;
    int64_t E[3], cv[3];
    const float4 p = pts[i];
    if (!(cell_coord(p.x, hf, E[0]) && cell_coord(p.y, hf, E[1]) && cell_coord(p.z, hf, E[2]) &&
          cell_coord(p.x, hv, cv[0]) && cell_coord(p.y, hv, cv[1]) && cell_coord(p.z, hv, cv[2])))
        return;
    // the measured voxel
    test_add(set, E, stat);
    // the normal
    // the 5 x 5 x 5 block, a 5 x 5 slice at a time: the first slots of its
    // 25 lookups are loaded together
    int64_t N = 0, s1[3] = {0, 0, 0}, S2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = -2; a <= 2; ++a) {
        uint64_t key[25], sl[25];
        unsigned long long f[25];
        bool in[25];
#pragma unroll
        for (int j = 0; j < 25; ++j) {
            const int64_t v[3] = {cv[0] + a, cv[1] + j / 5 - 2, cv[2] + j % 5 - 2};
            in[j] = !(v[0] < -kBias || v[0] >= kBias || v[1] < -kBias || v[1] >= kBias || v[2] < -kBias ||
                      v[2] >= kBias);
            key[j] = in[j] ? pack_key(v[0], v[1], v[2]) : 0ull;
            sl[j] = mix64(key[j]) & vh.mask;
        }
#pragma unroll
        for (int j = 0; j < 25; ++j) f[j] = in[j] ? vh.keys[sl[j]] : (unsigned long long)kNoKey;
#pragma unroll
        for (int j = 0; j < 25; ++j) {
            if (!in[j]) continue;
            // linear probing from the slot already read
            bool found = false;
            uint64_t sj = sl[j];
            unsigned long long kj = f[j];
            for (uint32_t p = 0; p <= vh.mask; ++p) {
                if (kj == key[j]) { found = true; break; }
                if (kj == kNoKey) break;
                sj = (sj + 1) & vh.mask;
                kj = vh.keys[sj];
            }
            if (!found) continue;
            const int64_t o[3] = {a, j / 5 - 2, j % 5 - 2};
            ++N;
            for (int r = 0; r < 3; ++r) {
                s1[r] += o[r];
                for (int q = 0; q < 3; ++q) S2[r][q] += o[r] * o[q];
            }
        }
    }
    if (N < 3) return;
    int64_t M[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) M[r][q] = N * S2[r][q] - s1[r] * s1[q];
    int64_t bn = 0, bd = 1, bdir[3] = {0, 0, 0};
    bool have = false;
    for (int x = -2; x <= 2; ++x)
        for (int y = -2; y <= 2; ++y)
            for (int z = -2; z <= 2; ++z) {
                const int f = x != 0 ? x : (y != 0 ? y : z);
                if (f <= 0 || igcd(igcd(x, y), z) != 1) continue;
                const int64_t d[3] = {x, y, z};
                int64_t num = 0, den = 0;
                for (int r = 0; r < 3; ++r) {
                    den += d[r] * d[r];
                    for (int q = 0; q < 3; ++q) num += d[r] * M[r][q] * d[q];
                }
                if (!have || num * bd < bn * den) {
                    have = true;
                    bn = num;
                    bd = den;
                    bdir[0] = x; bdir[1] = y; bdir[2] = z;
                }
            }
    for (int64_t k = -R; k <= R; ++k) {
        if (k == 0 || k * k * bd > int64_t(R) * R) continue;
        const int64_t v[3] = {E[0] + k * bdir[0], E[1] + k * bdir[1], E[2] + k * bdir[2]};
        test_add(set, v, stat);
    }
}


// Eq. (7)-(8): D <- (V d + v D) / (V + v), V <- V v / (V + v); an absent voxel
// takes (d, v) (the V = infinity limit).
// TSDF (Eq. (9)): weight w = 1 - v, D <- (w d + V D) / (V + w), V <- V + w; an
// absent voxel takes (d, w); w <= 0 carries no weight and is skipped.
//
// Surface property (gprop != NULL; Sec. IV-C): the same expressions with the
// property's variance w in place of v (TSDF: weight 1 - w).  It rides on the
// voxel's distance observation; an observation whose variance (weight) is not
// positive and finite, or a frame without a property (cp == NULL), leaves the
// voxel's property as it is, and a new voxel then holds none (NaN).  A voxel
// with no property takes the observation as is.
__global__ void k_fuse(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ nptr,
                       const float *__restrict__ d, const float *__restrict__ v,
                       const uint8_t *__restrict__ ok, GSlot *__restrict__ g, uint32_t gmask,
                       uint32_t *__restrict__ gstamp, uint32_t frame_h, const uint32_t *__restrict__ dframe,
                       unsigned long long *__restrict__ spread, int tsdf, const float *__restrict__ cp,
                       const float *__restrict__ cpv, float2 *__restrict__ gprop) {
    const int64_t n = int64_t(*nptr);
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (int64_t(blockIdx.x) * blockDim.x >= n) return;  // whole block past the end
    const bool in = i < n;
    const float di = in ? d[i] : 0.f, vi = in ? v[i] : 0.f;
    const float wi = 1.f - vi;
    const bool use = in && ok[i] && isfinite(di) && isfinite(vi) && (tsdf ? wi > 0.f : vi > 0.f);
    spread_count(spread, ST_FUSE_SKIPPED, in && !use);
    bool ins = false;
    int64_t s = -1;
    if (use) s = grid_insert(g, gmask, keys[i], &ins);
    spread_count(spread, ST_GLOBAL_FULL, use && s < 0);
    spread_count(spread, ST_GLOBAL_COUNT, s >= 0 && ins);
    spread_count(spread, ST_FUSED, s >= 0);
    if (s < 0) return;
    if (ins) {
        g[s].D = di;
        g[s].V = tsdf ? wi : vi;
    } else if (tsdf) {
        const float Vp = g[s].V, Dp = g[s].D;
        const float den = Vp + wi;
        g[s].D = (wi * di + Vp * Dp) / den;
        g[s].V = den;
    } else {
        const float Vp = g[s].V, Dp = g[s].D;
        const float den = Vp + vi;
        g[s].D = (Vp * di + vi * Dp) / den;
        g[s].V = (Vp * vi) / den;
    }
    gstamp[s] = dframe ? *dframe : frame_h;
    if (gprop) {
        const float ci = cp ? cp[i] : 0.f, wi2 = cp ? cpv[i] : 0.f;
        const float wt = tsdf ? 1.f - wi2 : wi2;
        const bool pok = cp && isfinite(ci) && isfinite(wi2) && wt > 0.f;
        if (ins || pok) {
            float2 P = ins ? make_float2(NAN, NAN) : gprop[s];
            if (pok) {
                if (isnan(P.x)) {
                    P = make_float2(ci, wt);
                } else if (tsdf) {
                    const float den = P.y + wt;
                    P = make_float2((wt * ci + P.y * P.x) / den, den);
                } else {
                    const float den = P.y + wt;
                    P = make_float2((P.y * ci + wt * P.x) / den, (P.y * wt) / den);
                }
            }
            gprop[s] = P;
        }
    }
}

// trilinear interpolation of the fused property C over the eight voxel
// centres around x; valid where all eight exist and hold a property
__global__ void k_global_query_prop(const float *__restrict__ q, int64_t m, double h,
                                    const GSlot *__restrict__ g, const float2 *__restrict__ gprop,
                                    uint32_t gmask, float *__restrict__ prop, uint8_t *__restrict__ valid) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double f[3];
    int64_t i0[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const float x = q[3 * j + a];
        if (!isfinite(x)) { ok = false; break; }
        const double u = double(x) / h - 0.5;
        const double fl = floor(u);
        if (fl < -double(kBias) || fl + 1.0 >= double(kBias)) { ok = false; break; }
        i0[a] = int64_t(fl);
        f[a] = u - fl;
    }
    double Cc[8];
    if (ok) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t key = pack_key(i0[0] + ((b >> 2) & 1), i0[1] + ((b >> 1) & 1), i0[2] + (b & 1));
            const int64_t sl = grid_find(g, gmask, key);
            const float cb = sl >= 0 ? gprop[sl].x : NAN;
            ok = ok && !isnan(cb);
            Cc[b] = double(cb);
        }
    }
    if (!ok) {
        prop[j] = 0.f;
        valid[j] = 0;
        return;
    }
    double C = 0.0;
    for (int b = 0; b < 8; ++b) {
        const int bx = (b >> 2) & 1, by = (b >> 1) & 1, bz = b & 1;
        const double wx = bx ? f[0] : 1.0 - f[0], wy = by ? f[1] : 1.0 - f[1],
                     wz = bz ? f[2] : 1.0 - f[2];
        C += wx * wy * wz * Cc[b];
    }
    prop[j] = float(C);
    valid[j] = 1;
}

// trilinear interpolation of D over the eight voxel centres around x
__global__ void k_global_query(const float *__restrict__ q, int64_t m, double h,
                               const GSlot *__restrict__ g, uint32_t gmask, float *__restrict__ dist,
                               float *__restrict__ grad, uint8_t *__restrict__ valid) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double f[3];
    int64_t i0[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        const float x = q[3 * j + a];
        if (!isfinite(x)) { ok = false; break; }
        const double u = double(x) / h - 0.5;
        const double fl = floor(u);
        if (fl < -double(kBias) || fl + 1.0 >= double(kBias)) { ok = false; break; }
        i0[a] = int64_t(fl);
        f[a] = u - fl;
    }
    double Dc[8];
    if (ok) {
        // the first slot of all 8 corners is read at once; a probe goes on
        // only past a slot held by another voxel
        uint64_t key[8], s0[8];
        GSlot e[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            key[b] = pack_key(i0[0] + ((b >> 2) & 1), i0[1] + ((b >> 1) & 1), i0[2] + (b & 1));
            s0[b] = grid_start(key[b], gmask);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) e[b] = g[s0[b]];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            float Db = 0.f;
            ok = grid_resolve(g, gmask, key[b], s0[b], e[b], &Db) && ok;
            Dc[b] = double(Db);
        }
    }
    if (!ok) {
        dist[j] = INFINITY;
        valid[j] = 0;
        if (grad) { grad[3 * j] = 0.f; grad[3 * j + 1] = 0.f; grad[3 * j + 2] = 0.f; }
        return;
    }
    double D = 0.0, G[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < 8; ++b) {
        const int bx = (b >> 2) & 1, by = (b >> 1) & 1, bz = b & 1;
        const double wx = bx ? f[0] : 1.0 - f[0], wy = by ? f[1] : 1.0 - f[1],
                     wz = bz ? f[2] : 1.0 - f[2];
        const double sx = bx ? 1.0 : -1.0, sy = by ? 1.0 : -1.0, sz = bz ? 1.0 : -1.0;
        D += wx * wy * wz * Dc[b];
        G[0] += sx * wy * wz * Dc[b];
        G[1] += wx * sy * wz * Dc[b];
        G[2] += wx * wy * sz * Dc[b];
    }
    dist[j] = float(D);
    valid[j] = 1;
    if (grad) {
        grad[3 * j] = float(G[0] / h);
        grad[3 * j + 1] = float(G[1] / h);
        grad[3 * j + 2] = float(G[2] / h);
    }
}

__global__ void k_global_load(const uint64_t *__restrict__ k, const float *__restrict__ D,
                              const float *__restrict__ V, const uint32_t *__restrict__ st, int64_t n,
                              GSlot *__restrict__ g, uint32_t gmask, uint32_t *__restrict__ gs,
                              unsigned long long *__restrict__ stat, const float2 *__restrict__ cw,
                              float2 *__restrict__ gprop) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    bool ins = false;
    int64_t s = -1;
    if (i < n) s = grid_insert(g, gmask, k[i], &ins);
    wave_count(&stat[ST_GLOBAL_FULL], i < n && s < 0);
    wave_count(&stat[ST_GLOBAL_COUNT], s >= 0 && ins);
    if (s < 0) return;
    g[s].D = D[i];
    g[s].V = V[i];
    gs[s] = st[i];
    if (gprop) gprop[s] = cw ? cw[i] : make_float2(NAN, NAN);
}

__global__ void k_grid_clear(GSlot *__restrict__ g, int64_t n, float2 *__restrict__ gprop) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        g[i] = GSlot{(unsigned long long)kNoKey, 0.f, 0.f};
        if (gprop) gprop[i] = make_float2(NAN, NAN);
    }
}

// brute-force nearest distance, FP32 differences, exact minimum
__global__ void k_nearest(const float *__restrict__ pts, int64_t n, const float *__restrict__ q,
                          int64_t m, float *__restrict__ out) {
    __shared__ float sp[3][kT];
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool act = j < m;
    const float qx = act ? q[3 * j] : 0.f, qy = act ? q[3 * j + 1] : 0.f, qz = act ? q[3 * j + 2] : 0.f;
    float best = INFINITY;
    for (int64_t b = 0; b < n; b += kT) {
        __syncthreads();
        const int64_t i = b + threadIdx.x;
        if (i < n) { sp[0][threadIdx.x] = pts[3 * i]; sp[1][threadIdx.x] = pts[3 * i + 1]; sp[2][threadIdx.x] = pts[3 * i + 2]; }
        __syncthreads();
        const int cnt = int(min<int64_t>(kT, n - b));
        for (int t = 0; t < cnt; ++t) {
            const float dx = qx - sp[0][t], dy = qy - sp[1][t], dz = qz - sp[2][t];
            best = fminf(best, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        }
    }
    if (act) out[j] = sqrtf(best);
}

}  // namespace

// band offsets of the test voxels (fixed by the parameters), uploaded once
gpdf_status ensure_offsets(gpdf_ctx *c) {
    if (c->offs_ready) return GPDF_OK;
    const double hf = c->p.fuse_voxel_size;
    const int R = int(std::floor(c->p.fuse_band / hf + 1e-9));
    std::vector<int4> &offs = c->h_offs;
    offs.clear();
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int d = -R; d <= R; ++d)
                if (a * a + b * b + d * d <= R * R) offs.push_back(make_int4(a, b, d, 0));
    if (int64_t(offs.size()) > c->offs_cap) return fail(c, GPDF_E_CAPACITY, "fuse: band too wide");
    hipError_t e;
    if ((e = hipMemcpyAsync(c->d_offs, offs.data(), sizeof(int4) * offs.size(), hipMemcpyHostToDevice,
                            c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "fuse: upload offsets");
    c->offs_ready = true;
    return GPDF_OK;
}

// Test voxels of the current training points, their signed query and the
// fusion.  With npts_bound >= 0 (graph capture) the counts stay on the
// device: training points at cnt[CNT_PTS] (at most npts_bound), test voxels
// at cnt[CNT_TEST], the frame stamp at cnt[CNT_FRAME] and the origin at
// d_origin; nothing is read back.
gpdf_status fuse(gpdf_ctx *c, const float *origin, const float *d_origin, int64_t npts_bound) {
    hipStream_t s = c->stream;
    const Model &M = c->model;
    const bool eager = npts_bound < 0;
    if (!M.trained) return fail(c, GPDF_E_NOT_TRAINED, "fuse before training");
    hipError_t e;
    uint32_t *cnt = c->d_cnt;
    FillList F;
    F.u64(c->d_stat + ST_TESTPTS, 0ull, 1);
    F.u64(c->d_stat + ST_FUSED, 0ull, 1);
    F.u64(c->d_stat + ST_FUSE_SKIPPED, 0ull, 1);
    F.u32(cnt + CNT_TEST, 0u, 1);
    const int64_t npts = eager ? M.npoints : npts_bound;
    if (eager && npts == 0) {
        (void)fill_multi(F, s);
        c->last_test = 0;
        c->frame++;
        return GPDF_OK;
    }
    const bool ray = c->p.test_points == GPDF_TEST_RAYCAST;
    gpdf_status st = ray ? GPDF_OK : ensure_offsets(c);
    if (st != GPDF_OK) {
        (void)fill_multi(F, s);
        return st;
    }
    const double hf = c->p.fuse_voxel_size;
    const int64_t tcap = int64_t(c->tset_mask) + 1;
    stage_begin(c, GPDF_MS_TESTPTS);
    F.u64(c->d_tset, (unsigned long long)kNoKey, tcap);
    if (ray) F.u64(c->d_vhash, (unsigned long long)kNoKey, int64_t(c->vhash_mask) + 1);
    if ((e = fill_multi(F, s)) != hipSuccess) return hip_fail(c, e, "fuse: clear");
    HashView set{c->d_tset, c->tset_mask};
    const uint32_t *dpts = eager ? nullptr : cnt + CNT_PTS;
    if (ray) {
        // Sec. IV-B: rays from the sensor to the training voxels against the
        // grid as it is before this frame, the measured voxels and their
        // normals
        const HashView vh{c->d_vhash, c->vhash_mask};
        const int R = int(std::floor(c->p.normal_reach / hf + 1e-9));
        hipLaunchKernelGGL(k_vox_insert, dim3(blocks_for(npts)), dim3(kT), 0, s, c->d_pts, npts, dpts,
                           c->p.voxel_size, vh, c->d_stat);
        hipLaunchKernelGGL(k_ray_walk, dim3(blocks_for(npts * kRaySeg)), dim3(kT), 0, s, c->d_pts, npts, dpts, hf,
                           origin ? origin[0] : 0.f, origin ? origin[1] : 0.f, origin ? origin[2] : 0.f, d_origin,
                           c->d_gslot, c->gmask, set, c->d_stat);
        hipLaunchKernelGGL(k_normal_tests, dim3(blocks_for(npts)), dim3(kT), 0, s, c->d_pts, npts, dpts,
                           c->p.voxel_size, hf, R, vh, set, c->d_stat);
    } else {
        const int noffs = int(c->h_offs.size());
        const int64_t work = npts * int64_t(noffs);
        hipLaunchKernelGGL(k_test_insert, dim3(blocks_for(work)), dim3(kT), 0, s, c->d_pts, npts, dpts, hf,
                           c->d_offs, noffs, set, c->d_stat);
    }
    count_occupied(c->d_tset, tcap, c->d_tile_cnt, c->d_tile_off, c->d_part, s);
    const int64_t ntiles = compact_tiles(tcap);
    hipLaunchKernelGGL(k_test_compact, dim3(unsigned(ntiles)), dim3(256), 0, s, c->d_tset, tcap,
                       c->d_tile_off, ntiles, c->d_tkeys, c->p.max_queries, hf, c->d_tpts, c->d_stat,
                       cnt + CNT_TEST);
    stage_end(c, GPDF_MS_TESTPTS);
    int64_t nt = c->p.max_queries;
    if (eager) {
        ReadList R;
        R.u64(c->d_stat + ST_TESTPTS);
        if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "fuse: read test count");
        const unsigned long long t = c->h_read[0];
        if (int64_t(t) > c->p.max_queries) return fail(c, GPDF_E_CAPACITY, "fuse: test points exceed max_queries");
        nt = int64_t(t);
        c->last_test = nt;
    }
    // a model trained with a property fuses it too (Sec. IV-C)
    const bool props = M.props && c->d_gprop;
    st = query(c, c->d_tpts, nt, origin, c->d_tmp_dist, nullptr, c->d_tmp_var, c->d_tmp_valid, nullptr, 0,
               eager ? nullptr : cnt + CNT_TEST, d_origin, false, props ? c->d_tprop : nullptr,
               props ? c->d_tpropv : nullptr);
    if (st != GPDF_OK) return st;
    stage_begin(c, GPDF_MS_FUSE);
    hipLaunchKernelGGL(k_fuse, dim3(blocks_for(nt)), dim3(kT), 0, s, c->d_tkeys, cnt + CNT_TEST, c->d_tmp_dist,
                       c->d_tmp_var, c->d_tmp_valid, c->d_gslot, c->gmask, c->d_gstamp, c->frame,
                       eager ? nullptr : cnt + CNT_FRAME, c->d_spread, c->p.fuse_rule == GPDF_FUSE_TSDF ? 1 : 0,
                       props ? c->d_tprop : nullptr, props ? c->d_tpropv : nullptr, c->d_gprop);
    fold_stats(c->d_spread, c->d_stat, s);
    stage_end(c, GPDF_MS_FUSE);
    if (eager) c->frame++;
    return (e = hipGetLastError()) == hipSuccess ? GPDF_OK : hip_fail(c, e, "fuse launch");
}

// ---------------------------------------------------------------------------
// zero crossings of the fused grid, the surface points of the G-GPDF
// (Sec. IV-D): the vertices marching cubes places on the grid edges whose two
// voxel centres carry distances of opposite sign, at the zero of the linear
// interpolant along the edge.  Listed in ascending key of the edge's lower
// voxel, then axis (x, y, z).
// ---------------------------------------------------------------------------
namespace {

// sign-changing edges from voxel e to its +x, +y, +z neighbours (bits 0..2)
__device__ inline uint32_t zc_edges(const GSlot *__restrict__ g, uint32_t gmask, const GSlot e, float *Dn) {
    if (e.key == kNoKey) return 0u;
    int64_t c[3];
    unpack_key(e.key, c);
    uint32_t m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int64_t nb[3] = {c[0], c[1], c[2]};
        nb[a] += 1;
        if (nb[a] >= kBias) continue;
        const uint64_t k = pack_key(nb[0], nb[1], nb[2]);
        const uint64_t s0 = grid_start(k, gmask);
        float Db = 0.f;
        if (grid_resolve(g, gmask, k, s0, g[s0], &Db) && ((e.D < 0.f) != (Db < 0.f))) {
            m |= 1u << a;
            if (Dn) Dn[a] = Db;
        }
    }
    return m;
}

// voxels with at least one crossing edge, per tile of kCompactTile slots
__global__ __launch_bounds__(256) void k_zc_count(const GSlot *__restrict__ g, uint32_t gmask, int64_t cap,
                                                  uint32_t *__restrict__ cnt) {
    __shared__ uint32_t wsum[4];
    const int64_t t0 = int64_t(blockIdx.x) * kCompactTile;
    uint32_t n = 0;
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t s = t0 + r * 256 + threadIdx.x;
        const uint32_t m = s < cap ? zc_edges(g, gmask, g[s], nullptr) : 0u;
        n += uint32_t(__popcll(__ballot(m != 0u)));
    }
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// (key, slot) of those voxels in slot order at the tile offsets
__global__ __launch_bounds__(256) void k_zc_emit(const GSlot *__restrict__ g, uint32_t gmask, int64_t cap,
                                                 const uint32_t *__restrict__ tile_off, uint64_t *__restrict__ ekey,
                                                 uint32_t *__restrict__ eslot) {
    __shared__ uint32_t wsum[4];
    const int w = threadIdx.x >> 6;
    const int64_t t0 = int64_t(blockIdx.x) * kCompactTile;
    uint32_t base = tile_off[blockIdx.x];
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t s = t0 + r * 256 + threadIdx.x;
        const GSlot e = s < cap ? g[s] : GSlot{(unsigned long long)kNoKey, 0.f, 0.f};
        const uint32_t m = zc_edges(g, gmask, e, nullptr);
        const uint64_t b = __ballot(m != 0u);
        if ((threadIdx.x & 63) == 0) wsum[w] = uint32_t(__popcll(b));
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int i = 0; i < 4; ++i) {
            before += i < w ? wsum[i] : 0u;
            tot += wsum[i];
        }
        if (m) {
            const uint32_t id = base + before + uint32_t(__popcll(b & lanes_below()));
            ekey[id] = e.key;
            eslot[id] = uint32_t(s);
        }
        __syncthreads();
        base += tot;
    }
}

// crossings per sorted voxel
__global__ void k_zc_points_count(const uint32_t *__restrict__ eslot, int64_t ne, const GSlot *__restrict__ g,
                                  uint32_t gmask, uint32_t *__restrict__ cnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    cnt[i] = uint32_t(__popc(zc_edges(g, gmask, g[eslot[i]], nullptr)));
}

// the points: on the edge's axis (c + 1/2 + t) h with t = D_a / (D_a - D_b),
// (c + 1/2) h on the others, in FP64 (no contraction) rounded once to FP32
__global__ void k_zc_points(const uint32_t *__restrict__ eslot, int64_t ne, const GSlot *__restrict__ g,
                            uint32_t gmask, const uint32_t *__restrict__ off, double h, float *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const GSlot e = g[eslot[i]];
    float Dn[3] = {0.f, 0.f, 0.f};
    const uint32_t m = zc_edges(g, gmask, e, Dn);
    int64_t c[3];
    unpack_key(e.key, c);
    uint32_t o = off[i];
    for (int a = 0; a < 3; ++a) {
        if (!((m >> a) & 1u)) continue;
        const double Da = double(e.D), Db = double(Dn[a]);
        const double t = __ddiv_rn(Da, __dsub_rn(Da, Db));
        for (int b = 0; b < 3; ++b) {
            double u = __dadd_rn(double(c[b]), 0.5);
            if (b == a) u = __dadd_rn(u, t);
            out[3 * int64_t(o) + b] = float(__dmul_rn(u, h));
        }
        ++o;
    }
}

hipError_t zc_reserve(gpdf_ctx *c, int64_t ne, int64_t ntiles) {
    hipError_t e;
    if (ntiles + 1 > c->ztiles) {
        if (c->d_ztile) (void)hipFree(c->d_ztile);
        if (c->d_ztoff) (void)hipFree(c->d_ztoff);
        c->d_ztile = c->d_ztoff = nullptr;
        c->ztiles = 0;
        if ((e = hipMalloc((void **)&c->d_ztile, sizeof(uint32_t) * size_t(ntiles + 1))) != hipSuccess ||
            (e = hipMalloc((void **)&c->d_ztoff, sizeof(uint32_t) * size_t(ntiles + 1))) != hipSuccess)
            return e;
        c->ztiles = ntiles + 1;
    }
    if (ne + 1 <= c->zcap) return hipSuccess;
    void *old[] = {c->d_zkey, c->d_zkey2, c->d_zslot, c->d_zslot2, c->d_zcnt, c->d_zoff, c->d_zhist, c->d_zpart};
    for (void *p : old)
        if (p) (void)hipFree(p);
    c->d_zkey = c->d_zkey2 = nullptr;
    c->d_zslot = c->d_zslot2 = c->d_zcnt = c->d_zoff = c->d_zhist = c->d_zpart = nullptr;
    c->zcap = 0;
    const int64_t cap = ne + ne / 4 + 1024;
    const int64_t nh = 256 * ((cap + kRsTileKeys - 1) / kRsTileKeys) + 1;
    const int64_t np = std::max<int64_t>(nh, cap) / 4096 + 64;
    if ((e = hipMalloc((void **)&c->d_zkey, sizeof(uint64_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zkey2, sizeof(uint64_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zslot, sizeof(uint32_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zslot2, sizeof(uint32_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zcnt, sizeof(uint32_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zoff, sizeof(uint32_t) * size_t(cap))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zhist, sizeof(uint32_t) * size_t(nh))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_zpart, sizeof(uint32_t) * size_t(np))) != hipSuccess)
        return e;
    c->zcap = cap;
    return hipSuccess;
}

}  // namespace

gpdf_status zero_crossings(gpdf_ctx *c, float *d_out, int64_t cap, int64_t *count) {
    hipStream_t s = c->stream;
    hipError_t e;
    const int64_t slots = int64_t(c->gmask) + 1;
    const int64_t ntiles = compact_tiles(slots);
    if ((e = zc_reserve(c, 0, ntiles)) != hipSuccess) return hip_fail(c, e, "zero crossings: alloc");
    hipLaunchKernelGGL(k_zc_count, dim3(unsigned(ntiles)), dim3(256), 0, s, c->d_gslot, c->gmask, slots, c->d_ztile);
    exclusive_scan_u32(c->d_ztile, c->d_ztoff, ntiles, c->d_part, s);
    ReadList R;
    R.u32(c->d_ztoff + ntiles);
    if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "zero crossings: count");
    const int64_t ne = int64_t(c->h_read[0]);
    if (ne == 0) {
        *count = 0;
        return GPDF_OK;
    }
    if ((e = zc_reserve(c, ne, ntiles)) != hipSuccess) return hip_fail(c, e, "zero crossings: alloc");
    hipLaunchKernelGGL(k_zc_emit, dim3(unsigned(ntiles)), dim3(256), 0, s, c->d_gslot, c->gmask, slots, c->d_ztoff,
                       c->d_zkey, c->d_zslot);
    // ascending voxel key (the radix sort is stable, keys are unique)
    uint64_t *k = c->d_zkey, *ka = c->d_zkey2;
    uint32_t *v = c->d_zslot, *va = c->d_zslot2;
    radix_sort_pairs(k, ka, v, va, ne, ~uint64_t(0), c->d_zhist, c->d_zpart, s);
    const unsigned gb = unsigned((ne + 255) / 256);
    hipLaunchKernelGGL(k_zc_points_count, dim3(gb), dim3(256), 0, s, v, ne, c->d_gslot, c->gmask, c->d_zcnt);
    exclusive_scan_u32(c->d_zcnt, c->d_zoff, ne, c->d_zpart, s);
    R = ReadList();
    R.u32(c->d_zoff + ne);
    if ((e = read_back(c, R, s)) != hipSuccess) return hip_fail(c, e, "zero crossings: points");
    const int64_t np = int64_t(c->h_read[0]);
    *count = np;
    if (d_out && cap >= np)
        hipLaunchKernelGGL(k_zc_points, dim3(gb), dim3(256), 0, s, v, ne, c->d_gslot, c->gmask, c->d_zoff,
                           c->p.fuse_voxel_size, d_out);
    return (e = hipGetLastError()) == hipSuccess ? GPDF_OK : hip_fail(c, e, "zero crossings: launch");
}

gpdf_status query_global(gpdf_ctx *c, const float *d_q, int64_t m, float *dist, float *grad,
                         uint8_t *valid) {
    if (m < 0) return fail(c, GPDF_E_INVALID_ARG, "query_global: m < 0");
    if (m == 0) return GPDF_OK;
    if (!d_q || !dist || !valid) return fail(c, GPDF_E_INVALID_ARG, "query_global: null buffer");
    hipLaunchKernelGGL(k_global_query, dim3(blocks_for(m)), dim3(kT), 0, c->stream, d_q, m,
                       c->p.fuse_voxel_size, c->d_gslot, c->gmask, dist, grad, valid);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "query_global launch");
}

gpdf_status query_global_prop(gpdf_ctx *c, const float *d_q, int64_t m, float *prop, uint8_t *valid) {
    if (!c->d_gprop) return fail(c, GPDF_E_INVALID_ARG, "query_global_prop: properties are off in the parameters");
    if (m < 0) return fail(c, GPDF_E_INVALID_ARG, "query_global_prop: m < 0");
    if (m == 0) return GPDF_OK;
    if (!d_q || !prop || !valid) return fail(c, GPDF_E_INVALID_ARG, "query_global_prop: null buffer");
    hipLaunchKernelGGL(k_global_query_prop, dim3(blocks_for(m)), dim3(kT), 0, c->stream, d_q, m,
                       c->p.fuse_voxel_size, c->d_gslot, c->d_gprop, c->gmask, prop, valid);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "query_global_prop launch");
}

void grid_clear(gpdf_ctx *c, hipStream_t s) {
    const int64_t n = int64_t(c->gmask) + 1;
    hipLaunchKernelGGL(k_grid_clear, dim3(unsigned(std::min<int64_t>((n + kT - 1) / kT, 65536))), dim3(kT), 0, s,
                       c->d_gslot, n, c->d_gprop);
}

gpdf_status nearest_distance(gpdf_ctx *c, const float *pts, int64_t n, const float *q, int64_t m,
                             float *out) {
    if (n <= 0 || m < 0 || !pts || !out || (m > 0 && !q))
        return fail(c, GPDF_E_INVALID_ARG, "nearest_distance: bad arguments");
    if (m == 0) return GPDF_OK;
    hipLaunchKernelGGL(k_nearest, dim3(blocks_for(m)), dim3(kT), 0, c->stream, pts, n, q, m, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPDF_OK : hip_fail(c, e, "nearest launch");
}

}  // namespace gpdf

using namespace gpdf;

namespace {
struct Rec {
    uint64_t k;
    float D, V;
    uint32_t st;
    float C, W;   // fused property (NaN: none, or properties off)
};

gpdf_status read_global(gpdf_ctx *c, std::vector<Rec> &out) {
    const int64_t cap = int64_t(c->gmask) + 1;
    std::vector<GSlot> g(cap);
    std::vector<uint32_t> st(cap);
    std::vector<float2> cw(c->d_gprop ? cap : 0);
    hipError_t e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess ||
        (e = hipMemcpy(g.data(), c->d_gslot, sizeof(GSlot) * cap, hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(st.data(), c->d_gstamp, 4 * cap, hipMemcpyDeviceToHost)) != hipSuccess ||
        (c->d_gprop &&
         (e = hipMemcpy(cw.data(), c->d_gprop, sizeof(float2) * cap, hipMemcpyDeviceToHost)) != hipSuccess))
        return hip_fail(c, e, "read global grid");
    out.clear();
    for (int64_t i = 0; i < cap; ++i)
        if (g[i].key != kNoKey)
            out.push_back(Rec{g[i].key, g[i].D, g[i].V, st[i], c->d_gprop ? cw[i].x : NAN, c->d_gprop ? cw[i].y : NAN});
    std::sort(out.begin(), out.end(), [](const Rec &a, const Rec &b) { return a.k < b.k; });
    return GPDF_OK;
}
}  // namespace

extern "C" gpdf_status gpdf_export_global(gpdf_ctx *c, uint64_t *h_key, float *h_D, float *h_V,
                                          uint32_t *h_stamp, int64_t cap, int64_t *count) {
    if (!c || !count) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    std::vector<Rec> r;
    gpdf_status s = read_global(c, r);
    if (s != GPDF_OK) return s;
    *count = int64_t(r.size());
    if (int64_t(r.size()) > cap) return GPDF_OK;
    for (size_t i = 0; i < r.size(); ++i) {
        if (h_key) h_key[i] = r[i].k;
        if (h_D) h_D[i] = r[i].D;
        if (h_V) h_V[i] = r[i].V;
        if (h_stamp) h_stamp[i] = r[i].st;
    }
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_export_global_prop(gpdf_ctx *c, uint64_t *h_key, float *h_C, float *h_W,
                                               int64_t cap, int64_t *count) {
    if (!c || !count) return GPDF_E_INVALID_ARG;
    if (!c->d_gprop) return fail(c, GPDF_E_INVALID_ARG, "export_global_prop: properties are off in the parameters");
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    std::vector<Rec> r;
    gpdf_status s = read_global(c, r);
    if (s != GPDF_OK) return s;
    *count = int64_t(r.size());
    if (int64_t(r.size()) > cap) return GPDF_OK;
    for (size_t i = 0; i < r.size(); ++i) {
        if (h_key) h_key[i] = r[i].k;
        if (h_C) h_C[i] = r[i].C;
        if (h_W) h_W[i] = r[i].W;
    }
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_query_global_prop(gpdf_ctx *c, const float *d_q, int64_t m, float *d_prop,
                                              uint8_t *d_valid) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    return query_global_prop(c, d_q, m, d_prop, d_valid);
}

extern "C" gpdf_status gpdf_zero_crossings(gpdf_ctx *c, float *d_out, int64_t cap, int64_t *count) {
    if (!c || !count) return GPDF_E_INVALID_ARG;
    if (cap < 0 || (cap > 0 && !d_out)) return fail(c, GPDF_E_INVALID_ARG, "zero crossings: bad output buffer");
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    try {
        return zero_crossings(c, d_out, cap, count);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "zero crossings: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_export_test_points(gpdf_ctx *c, uint64_t *h_key, int64_t cap,
                                               int64_t *count) {
    if (!c || !count) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    hipError_t e;
    const int64_t n = c->last_test;
    *count = n;
    if (n > cap || n == 0) return GPDF_OK;
    std::vector<uint64_t> k(n);
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess ||
        (e = hipMemcpy(k.data(), c->d_tkeys, 8 * n, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "export test points");
    std::sort(k.begin(), k.end());
    std::memcpy(h_key, k.data(), 8 * n);
    return GPDF_OK;
}

namespace {
constexpr uint64_t kMagic = 0x4650444742445631ull;  // "1VDBGDPF"
struct FileHeader {
    uint64_t magic;
    uint32_t version, frame;
    double voxel;
    int64_t count;
};
}  // namespace

extern "C" gpdf_status gpdf_save_global(gpdf_ctx *c, const char *path) {
    if (!c || !path) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    std::vector<Rec> r;
    gpdf_status s = read_global(c, r);
    if (s != GPDF_OK) return s;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(c, GPDF_E_INVALID_ARG, "save_global: cannot open file");
    // version 1: (key, D, V, stamp); version 2 adds the property (C, W)
    const uint32_t ver = c->d_gprop ? 2u : 1u;
    FileHeader h{kMagic, ver, c->frame, c->p.fuse_voxel_size, int64_t(r.size())};
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1;
    for (size_t i = 0; ok && i < r.size(); ++i) {
        ok = std::fwrite(&r[i].k, 8, 1, f) == 1 && std::fwrite(&r[i].D, 4, 1, f) == 1 &&
             std::fwrite(&r[i].V, 4, 1, f) == 1 && std::fwrite(&r[i].st, 4, 1, f) == 1;
        if (ok && ver == 2u) ok = std::fwrite(&r[i].C, 4, 1, f) == 1 && std::fwrite(&r[i].W, 4, 1, f) == 1;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GPDF_OK : fail(c, GPDF_E_INVALID_ARG, "save_global: write failed");
}

extern "C" gpdf_status gpdf_load_global(gpdf_ctx *c, const char *path) {
    if (!c || !path) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(c, GPDF_E_INVALID_ARG, "load_global: cannot open file");
    FileHeader h{};
    if (std::fread(&h, sizeof h, 1, f) != 1 || h.magic != kMagic || (h.version != 1u && h.version != 2u) ||
        h.count < 0 || h.voxel != c->p.fuse_voxel_size) {
        std::fclose(f);
        return fail(c, GPDF_E_INVALID_ARG, "load_global: bad header or voxel size");
    }
    if (h.version == 2u && !c->d_gprop) {
        std::fclose(f);
        return fail(c, GPDF_E_INVALID_ARG, "load_global: the file holds properties and properties are off");
    }
    if (h.count > c->p.global_capacity) {
        std::fclose(f);
        return fail(c, GPDF_E_CAPACITY, "load_global: file exceeds global_capacity");
    }
    std::vector<uint64_t> k(h.count);
    std::vector<float> D(h.count), V(h.count);
    std::vector<uint32_t> st(h.count);
    std::vector<float2> cw(h.version == 2u ? h.count : 0);
    bool ok = true;
    for (int64_t i = 0; ok && i < h.count; ++i) {
        ok = std::fread(&k[i], 8, 1, f) == 1 && std::fread(&D[i], 4, 1, f) == 1 &&
             std::fread(&V[i], 4, 1, f) == 1 && std::fread(&st[i], 4, 1, f) == 1;
        if (ok && h.version == 2u) ok = std::fread(&cw[i].x, 4, 1, f) == 1 && std::fread(&cw[i].y, 4, 1, f) == 1;
    }
    std::fclose(f);
    if (!ok) return fail(c, GPDF_E_INVALID_ARG, "load_global: truncated file");
    hipStream_t s = c->stream;
    hipError_t e;
    grid_clear(c, s);
    fill_u64(c->d_stat + ST_GLOBAL_COUNT, 0ull, 1, s);
    c->frame = h.frame;
    if (h.count == 0) return GPDF_OK;
    // stage the records through the test-point buffers (host to device)
    uint64_t *dk = nullptr;
    float *dD = nullptr, *dV = nullptr;
    uint32_t *ds = nullptr;
    float2 *dcw = nullptr;
    if ((e = hipMallocAsync((void **)&dk, 8 * h.count, s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&dD, 4 * h.count, s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&dV, 4 * h.count, s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&ds, 4 * h.count, s)) != hipSuccess ||
        (!cw.empty() && (e = hipMallocAsync((void **)&dcw, sizeof(float2) * h.count, s)) != hipSuccess))
        return hip_fail(c, e, "load_global: allocate staging");
    if ((e = hipMemcpyAsync(dk, k.data(), 8 * h.count, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dD, D.data(), 4 * h.count, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dV, V.data(), 4 * h.count, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(ds, st.data(), 4 * h.count, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (dcw && (e = hipMemcpyAsync(dcw, cw.data(), sizeof(float2) * h.count, hipMemcpyHostToDevice, s)) !=
                    hipSuccess))
        return hip_fail(c, e, "load_global: upload");
    hipLaunchKernelGGL(k_global_load, dim3(unsigned((h.count + kT - 1) / kT)), dim3(kT), 0, s, dk, dD,
                       dV, ds, h.count, c->d_gslot, c->gmask, c->d_gstamp, c->d_stat, dcw, c->d_gprop);
    if (dcw) (void)hipFreeAsync(dcw, s);
    (void)hipFreeAsync(dk, s);
    (void)hipFreeAsync(dD, s);
    (void)hipFreeAsync(dV, s);
    (void)hipFreeAsync(ds, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "load_global");
    return GPDF_OK;
}

// api.hip -- the C ABI of libvdbgpdf.so: parameters, context and arenas,
// argument checks, statistics and model export.  Every computational step
// runs in the kernels of sort.hip, train.hip, query.hip, fuse.hip, mlp.hip.
#include "gpdf_internal.hpp"

#include <cmath>
#include <cstring>
#include <new>

namespace gpdf {

gpdf_status fail(gpdf_ctx *c, gpdf_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

gpdf_status hip_fail(gpdf_ctx *c, hipError_t e, const char *what) {
    if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
    return GPDF_E_HIP;
}

}  // namespace gpdf

using namespace gpdf;

namespace {


void release(gpdf_ctx *c) {
    if (c->side) (void)hipStreamSynchronize(c->side);  // a trainer may still run there
    if (c->side2) (void)hipStreamSynchronize(c->side2);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->side2) (void)hipStreamDestroy(c->side2);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->join2_ev) (void)hipEventDestroy(c->join2_ev);
    c->side = c->side2 = nullptr;
    c->fork_ev = c->join_ev = c->join2_ev = nullptr;
    if (c->d_gin) (void)hipFree(c->d_gin);
    if (c->d_gorigin) (void)hipFree(c->d_gorigin);
    if (c->d_gfirst) (void)hipFree(c->d_gfirst);
    if (c->h_gchunks) (void)hipHostFree(c->h_gchunks);
    c->d_gfirst = c->h_gchunks = c->d_gchunks = nullptr;
    c->geval_node = nullptr;
    c->geval_ok = false;
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gstream = nullptr;
    void *ptrs[] = {c->d_key, c->d_key2, c->d_val, c->d_val2, c->d_flag, c->d_scan, c->d_hist,
                    c->d_part, c->d_red, c->d_pts, c->d_alpha64, c->d_ckey, c->d_coff, c->d_pd,
                    c->d_woff, c->d_aoff, c->d_W32, c->d_W64, c->d_A, c->d_chash,
                    c->d_chash_val, c->d_qhash, c->d_qhash_cnt, c->d_qhash_cell, c->d_qslot,
                    c->d_qrank, c->d_order, c->d_cell_key, c->d_cell_cnt, c->d_cell_off,
                    c->d_cell_chunks, c->d_chunk_off, c->d_cell_list, c->d_chunk, c->d_refine,
                    c->d_rcnt, c->d_roff, c->d_rchunks, c->d_rchunk_off, c->d_rorder, c->d_rrank,
                    c->d_rchunk, c->d_bbase, c->d_bcnt, c->d_boff, c->d_bcs, c->d_boffs, c->d_bcb,
                    c->d_boffb, c->d_bnit, c->d_bioff, c->d_bitem, c->d_bnits, c->d_bioffs, c->d_bitems, c->d_bq, c->d_bdst, c->d_rcell, c->d_bres,
                    c->d_tmp_dist, c->d_tmp_var, c->d_tmp_grad, c->d_tmp_valid, c->d_tset,
                    c->d_tkeys, c->d_tpts, c->d_gslot, c->d_gstamp, c->d_offs,
                    c->d_mlp_w, c->d_mlp_m, c->d_mlp_v, c->d_mlp_g, c->d_mlp_rec, c->d_mlp_pack,
                    c->d_mlp_norm, c->d_mlp_loss, c->d_mlp_mom, c->d_stat, c->d_spread, c->d_blist, c->d_tile_cnt, c->d_tile_off, c->d_bfM, c->d_bfoff, c->d_work, c->d_cnt, c->d_wsz, c->d_asz, c->d_wo32, c->d_ao32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    void *zptrs[] = {c->d_zkey, c->d_zkey2, c->d_zslot, c->d_zslot2, c->d_zcnt, c->d_zoff,
                     c->d_zhist, c->d_zpart, c->d_ztile, c->d_ztoff, c->d_need, c->d_trained,
                     c->d_cprop, c->d_beta64, c->d_beta32, c->d_gprop, c->d_tprop, c->d_tpropv, c->d_vhash};
    for (void *p : zptrs)
        if (p) (void)hipFree(p);
    if (c->h_stat) (void)hipHostFree(c->h_stat);
    if (c->h_read) (void)hipHostFree(c->h_read);
    for (hipEvent_t &e : c->ev)
        if (e) (void)hipEventDestroy(e);
}

template <typename T>
bool dalloc(T *&p, int64_t count, hipError_t &e) {
    if (count < 1) count = 1;
    e = hipMalloc((void **)&p, sizeof(T) * size_t(count));
    return e == hipSuccess;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" gpdf_status gpdf_params_default(gpdf_params *p) {
    if (!p) return GPDF_E_INVALID_ARG;
    std::memset(p, 0, sizeof *p);
    p->abi_version = GPDF_ABI_VERSION;
    p->kernel = GPDF_KERNEL_MATERN32;
    p->length_scale = 0.2;
    p->noise_sigma = 0.01;
    p->voxel_size = 0.0;
    p->cluster_size = 0.4;
    p->selection = GPDF_SEL_NEIGHBOR27;
    p->knn_q = 8;
    p->combine = GPDF_COMB_SMOOTHMIN;
    p->grad_mode = GPDF_GRAD_WEIGHTED;
    p->smooth_min_lambda = 100.0;
    p->occ_min = 1e-15;
    p->occ_max = 1.0 - 1e-5;
    p->precision = GPDF_PREC_FP32;
    p->timing = 0;
    p->fuse_voxel_size = 0.05;
    p->fuse_band = 0.2;
    p->mlp_gate = 0.05;
    p->max_points = int64_t(1) << 21;
    p->max_clusters = int64_t(1) << 18;
    p->max_cluster_points = 1024;
    p->max_factor_elems = int64_t(1) << 24;
    p->max_queries = int64_t(6) << 20;
    p->global_capacity = int64_t(1) << 24;
    p->fuse_rule = GPDF_FUSE_INVVAR;
    p->test_points = GPDF_TEST_BAND;
    p->normal_reach = 0.2;
    p->lazy_train = 0;
    p->properties = 0;
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_create(const gpdf_params *p, void *hip_stream, gpdf_ctx **out) {
    if (!p || !out) return GPDF_E_INVALID_ARG;
    *out = nullptr;
    if (p->abi_version != GPDF_ABI_VERSION) return GPDF_E_INVALID_ARG;
    if (!finite_pos(p->length_scale) || !(std::isfinite(p->noise_sigma) && p->noise_sigma >= 0.0) ||
        !(std::isfinite(p->voxel_size) && p->voxel_size >= 0.0) ||
        (p->voxel_size == 0.0 && !finite_pos(p->cluster_size)) ||
        !finite_pos(p->smooth_min_lambda) || !finite_pos(p->occ_min) ||
        !(p->occ_max > p->occ_min && p->occ_max < 1.0) || !finite_pos(p->fuse_voxel_size) ||
        !(std::isfinite(p->fuse_band) && p->fuse_band >= 0.0) ||
        (p->kernel != GPDF_KERNEL_MATERN32 && p->kernel != GPDF_KERNEL_SE) ||
        (p->selection != GPDF_SEL_NEIGHBOR27 && p->selection != GPDF_SEL_KNN) ||
        (p->selection == GPDF_SEL_KNN && (p->knn_q < 1 || p->knn_q > 16)) ||
        (p->combine != GPDF_COMB_SMOOTHMIN && p->combine != GPDF_COMB_HARDMIN) ||
        (p->grad_mode != GPDF_GRAD_WEIGHTED && p->grad_mode != GPDF_GRAD_PAPER_MEAN) ||
        (p->precision < GPDF_PREC_FP32 || p->precision > GPDF_PREC_FP32_MFMA) ||
        ((p->precision == GPDF_PREC_BF16 || p->precision == GPDF_PREC_FP32_MFMA) && p->selection == GPDF_SEL_KNN) ||
        (p->timing != 0 && p->timing != 1) || p->max_points < 1 ||
        p->max_points > (int64_t(1) << 30) || p->max_clusters < 1 || p->max_cluster_points < 1 ||
        p->max_cluster_points > 1024 || p->max_factor_elems < 1 ||
        p->max_factor_elems > (int64_t(1) << 31) - 1 || p->max_queries < 1 ||
        p->max_queries > (int64_t(1) << 30) || p->global_capacity < 1 ||
        p->global_capacity > (int64_t(1) << 30) ||
        (p->fuse_rule != GPDF_FUSE_INVVAR && p->fuse_rule != GPDF_FUSE_TSDF) ||
        (p->test_points != GPDF_TEST_BAND && p->test_points != GPDF_TEST_RAYCAST) ||
        !(std::isfinite(p->normal_reach) && p->normal_reach >= 0.0) ||
        (p->test_points == GPDF_TEST_RAYCAST && p->voxel_size <= 0.0) ||
        (p->lazy_train != 0 && p->lazy_train != 1) || (p->properties != 0 && p->properties != 1) ||
        (p->properties && (p->precision == GPDF_PREC_BF16 || p->precision == GPDF_PREC_FP32_MFMA ||
                           p->selection != GPDF_SEL_NEIGHBOR27 ||
                           p->lazy_train)))
        return GPDF_E_INVALID_ARG;
    gpdf_ctx *c = new (std::nothrow) gpdf_ctx();
    if (!c) return GPDF_E_OOM;
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&c->device);
    hipError_t e = hipSuccess;
    const int64_t P = p->max_points, C = p->max_clusters, M = p->max_queries;
    const int64_t nbP = (P + kRsTileKeys - 1) / kRsTileKeys;
    const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(P, M), 256 * nbP) + 1;
    c->cap_w = p->max_factor_elems;
    c->cap_a = p->max_factor_elems;
    c->cap_cells = std::min<int64_t>(M + 1, int64_t(1) << 16);  // grown on demand
    c->chash_mask = pow2_mask(2 * C);
    c->qhash_mask = pow2_mask(2 * M);
    c->tset_mask = pow2_mask(2 * M);
    c->gmask = pow2_mask(2 * p->global_capacity);
    c->offs_cap = 1 << 16;
    const int64_t chunks = M + M / 64 + 2;
    const int64_t ntile = compact_tiles(std::max<int64_t>(int64_t(c->qhash_mask), int64_t(c->tset_mask)) + 1);
    bool ok = dalloc(c->d_key, P + 1, e) && dalloc(c->d_key2, P + 1, e) && dalloc(c->d_val, P + 1, e) &&
              dalloc(c->d_val2, P + 1, e) && dalloc(c->d_flag, P + 1, e) &&
              dalloc(c->d_scan, scan_n, e) && dalloc(c->d_hist, 256 * nbP + 1, e) &&
              dalloc(c->d_part, scan_n / 4096 + 64, e) && dalloc(c->d_red, 8, e) && dalloc(c->d_work, int64_t(kWorkSlots) * kWorkSlot, e) && dalloc(c->d_cnt, kCnt, e) &&
              dalloc(c->d_wsz, C + 1, e) && dalloc(c->d_asz, C + 1, e) && dalloc(c->d_wo32, C + 1, e) &&
              dalloc(c->d_ao32, C + 1, e) &&
              dalloc(c->d_pts, P + kPtsPad, e) && dalloc(c->d_alpha64, P, e) && dalloc(c->d_ckey, C + 1, e) &&
              dalloc(c->d_coff, C + 1, e) && dalloc(c->d_pd, C + 1, e) && dalloc(c->d_woff, C, e) && dalloc(c->d_blist, int64_t(kBuckets) * C, e) &&
              dalloc(c->d_need, C + 8, e) && dalloc(c->d_trained, C + 8, e) &&
              dalloc(c->d_aoff, C, e) && dalloc(c->d_W32, c->cap_w + kW32Pad, e) &&
              dalloc(c->d_W64, c->cap_w, e) &&
              dalloc(c->d_A, c->cap_a, e) &&
              dalloc(c->d_tile_cnt, ntile + 1, e) && dalloc(c->d_tile_off, ntile + 1, e) &&
              dalloc(c->d_chash, int64_t(c->chash_mask) + 1, e) &&
              dalloc(c->d_chash_val, int64_t(c->chash_mask) + 1, e) &&
              dalloc(c->d_qhash, int64_t(c->qhash_mask) + 1, e) &&
              dalloc(c->d_qhash_cnt, int64_t(c->qhash_mask) + 1, e) &&
              dalloc(c->d_qhash_cell, int64_t(c->qhash_mask) + 1, e) && dalloc(c->d_qslot, M, e) &&
              dalloc(c->d_qrank, M, e) && dalloc(c->d_order, M, e) && dalloc(c->d_cell_key, M + 1, e) &&
              dalloc(c->d_cell_cnt, M + 1, e) && dalloc(c->d_cell_off, M + 1, e) &&
              dalloc(c->d_cell_chunks, M + 1, e) && dalloc(c->d_chunk_off, M + 1, e) &&
              dalloc(c->d_cell_list, c->cap_cells * kCellListStride, e) && dalloc(c->d_chunk, chunks, e) &&
              dalloc(c->d_refine, M, e) && dalloc(c->d_rcnt, M + 1, e) && dalloc(c->d_roff, M + 1, e) &&
              dalloc(c->d_rchunks, M + 1, e) && dalloc(c->d_rchunk_off, M + 1, e) &&
              dalloc(c->d_rorder, M, e) && dalloc(c->d_rrank, M, e) && dalloc(c->d_rchunk, chunks, e) && dalloc(c->d_tmp_dist, M, e) && dalloc(c->d_tmp_var, M, e) &&
              dalloc(c->d_tmp_grad, 3 * M, e) && dalloc(c->d_tmp_valid, M, e) &&
              dalloc(c->d_tset, int64_t(c->tset_mask) + 1, e) && dalloc(c->d_tkeys, M, e) &&
              dalloc(c->d_tpts, 3 * M, e) && dalloc(c->d_gslot, int64_t(c->gmask) + 1, e) &&
              dalloc(c->d_gstamp, int64_t(c->gmask) + 1, e) && dalloc(c->d_offs, c->offs_cap, e) &&
              dalloc(c->d_stat, ST_COUNT, e) && dalloc(c->d_spread, int64_t(kSpread) * kSpreadStride, e);
    if (ok) {
        // cluster-major re-evaluation: frames beyond these bounds fall back
        // to the chunk pass on the device
        c->cap_bchunks = std::min<int64_t>(std::max<int64_t>(M / 16, int64_t(1) << 14), int64_t(1) << 18);
        c->cap_bpairs = std::min<int64_t>(std::max<int64_t>(M, int64_t(1) << 16), int64_t(1) << 22);
        // results are laid out per cell-list slot: 27 slots per refined query
        c->cap_bref = c->cap_bpairs / (kCellListStride - 1);
        ok = dalloc(c->d_bbase, c->cap_bchunks * (kCellListStride - 1), e) && dalloc(c->d_bcnt, C + 1, e) &&
             dalloc(c->d_boff, C + 1, e) && dalloc(c->d_bcs, C + 1, e) && dalloc(c->d_boffs, C + 1, e) &&
             dalloc(c->d_bcb, C + 1, e) && dalloc(c->d_boffb, C + 1, e) && dalloc(c->d_bnit, C + 1, e) &&
             dalloc(c->d_bioff, C + 1, e) && dalloc(c->d_bitem, c->cap_bpairs, e) &&
             dalloc(c->d_bnits, C + 1, e) && dalloc(c->d_bioffs, C + 1, e) && dalloc(c->d_bitems, c->cap_bpairs, e) &&
             dalloc(c->d_bq, c->cap_bpairs, e) &&
             dalloc(c->d_bdst, c->cap_bpairs, e) && dalloc(c->d_rcell, M, e) &&
             (e = hipMalloc(&c->d_bres, size_t(80) * c->cap_bpairs)) == hipSuccess;
    }
    if (ok && p->test_points == GPDF_TEST_RAYCAST) {
        c->vhash_mask = pow2_mask(2 * P);
        ok = dalloc(c->d_vhash, int64_t(c->vhash_mask) + 1, e);
    }
    if (ok && p->properties)
        ok = dalloc(c->d_cprop, P, e) && dalloc(c->d_beta64, P, e) && dalloc(c->d_beta32, P + kPtsPad, e) &&
             dalloc(c->d_gprop, int64_t(c->gmask) + 1, e) && dalloc(c->d_tprop, M, e) && dalloc(c->d_tpropv, M, e);
    if (ok) {
        ok = (e = hipHostMalloc((void **)&c->h_stat, sizeof(unsigned long long) * ST_COUNT, 0)) == hipSuccess &&
             (e = hipHostMalloc((void **)&c->h_read, sizeof(unsigned long long) * ReadList::kMax, 0)) == hipSuccess;
    }
    for (int i = 0; ok && p->timing && i < 16; ++i) {
        e = hipEventCreate(&c->ev[i]);
        ok = e == hipSuccess;
    }
    if (ok) {
        // default priority, like the caller's stream
        ok = (e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking)) == hipSuccess &&
             (e = hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking)) == hipSuccess &&
             (e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming)) == hipSuccess &&
             (e = hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming)) == hipSuccess &&
             (e = hipEventCreateWithFlags(&c->join2_ev, hipEventDisableTiming)) == hipSuccess;
    }
    if (!ok) {
        release(c);
        delete c;
        return e == hipErrorOutOfMemory ? GPDF_E_OOM : GPDF_E_HIP;
    }
    // this device's fixed scratch of gpdf_query_distance_noalloc
    if (scratch_setup(c) != GPDF_OK) {
        release(c);
        delete c;
        return GPDF_E_HIP;
    }
    fill_u64(c->d_stat, 0ull, ST_COUNT, c->stream);
    fill_u64(c->d_spread, 0ull, int64_t(kSpread) * kSpreadStride, c->stream);
    // finite contents everywhere, pads included (masked FP32 rows read them)
    fill_u32(reinterpret_cast<uint32_t *>(c->d_pts), 0u, 4 * (P + kPtsPad), c->stream);
    fill_u32(reinterpret_cast<uint32_t *>(c->d_W32), 0u, c->cap_w + kW32Pad, c->stream);
    if (c->d_beta32) fill_u32(reinterpret_cast<uint32_t *>(c->d_beta32), 0u, P + kPtsPad, c->stream);
    grid_clear(c, c->stream);
    fill_u64(c->d_chash, (unsigned long long)kNoKey, int64_t(c->chash_mask) + 1, c->stream);
    fill_u32(reinterpret_cast<uint32_t *>(c->d_need), 0u, (C + 4) / 4, c->stream);
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) {
        release(c);
        delete c;
        return GPDF_E_HIP;
    }
    *out = c;
    return GPDF_OK;
}

extern "C" void gpdf_destroy(gpdf_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

extern "C" gpdf_status gpdf_train_local_gps(gpdf_ctx *c, const float *d_xyz, int64_t n) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (n < 0 || (n > 0 && !d_xyz)) return fail(c, GPDF_E_INVALID_ARG, "train: bad arguments");
    try {
        stage_begin(c, GPDF_MS_TRAIN);
        gpdf_status s = train(c, d_xyz, n);
        stage_end(c, GPDF_MS_TRAIN);
        return s;
    } catch (...) {
        return fail(c, GPDF_E_OOM, "train: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_train_local_gps_prop(gpdf_ctx *c, const float *d_xyz, const float *d_prop,
                                                 int64_t n) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!d_xyz || !d_prop))) return fail(c, GPDF_E_INVALID_ARG, "train_prop: bad arguments");
    try {
        stage_begin(c, GPDF_MS_TRAIN);
        gpdf_status s = train(c, d_xyz, n, nullptr, d_prop);
        stage_end(c, GPDF_MS_TRAIN);
        return s;
    } catch (...) {
        return fail(c, GPDF_E_OOM, "train_prop: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_query_distance_prop(gpdf_ctx *c, const float *d_q, int64_t m,
                                                const float *h_origin, float *d_dist, float *d_grad,
                                                float *d_var, uint8_t *d_valid, float *d_aux, float *d_prop,
                                                float *d_prop_var) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (m > 0 && !d_prop && !d_prop_var) return fail(c, GPDF_E_INVALID_ARG, "query_prop: no property output");
    try {
        return query(c, d_q, m, h_origin, d_dist, d_grad, d_var, d_valid, d_aux, 0, nullptr, nullptr, false, d_prop,
                     d_prop_var);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "query_prop: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_fuse_frame_prop(gpdf_ctx *c, const float *d_xyz, const float *d_prop, int64_t n,
                                            const float *h_origin) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (!d_xyz || (n > 0 && !d_prop)) return fail(c, GPDF_E_INVALID_ARG, "fuse_prop: bad arguments");
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (!h_origin || !(std::isfinite(h_origin[0]) && std::isfinite(h_origin[1]) &&
                       std::isfinite(h_origin[2])))
        return fail(c, GPDF_E_INVALID_ARG, "fuse_prop: origin required");
    try {
        stage_begin(c, GPDF_MS_TRAIN);
        gpdf_status s = train(c, d_xyz, n, nullptr, d_prop);
        stage_end(c, GPDF_MS_TRAIN);
        if (s != GPDF_OK) return s;
        return fuse(c, h_origin);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "fuse_prop: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_query_distance(gpdf_ctx *c, const float *d_q, int64_t m,
                                           const float *h_origin, float *d_dist, float *d_grad,
                                           float *d_var, uint8_t *d_valid, float *d_aux,
                                           int32_t correct) {
    if (!c) return GPDF_E_INVALID_ARG;
    try {
        return query(c, d_q, m, h_origin, d_dist, d_grad, d_var, d_valid, d_aux, correct);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "query: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_query_distance_noalloc(gpdf_ctx *c, const float *d_q, int64_t m,
                                                   const float *h_origin, float *d_dist, float *d_grad,
                                                   float *d_var, uint8_t *d_valid, float *d_aux,
                                                   int32_t correct) {
    if (!c) return GPDF_E_INVALID_ARG;
    try {
        return query(c, d_q, m, h_origin, d_dist, d_grad, d_var, d_valid, d_aux, correct, nullptr, nullptr, true);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "query_distance_noalloc: host exception");
    }
}

extern "C" gpdf_status gpdf_fuse_frame(gpdf_ctx *c, const float *d_xyz, int64_t n,
                                       const float *h_origin) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (!h_origin || !(std::isfinite(h_origin[0]) && std::isfinite(h_origin[1]) &&
                       std::isfinite(h_origin[2])))
        return fail(c, GPDF_E_INVALID_ARG, "fuse: origin required");
    try {
        if (d_xyz) {
            stage_begin(c, GPDF_MS_TRAIN);
            gpdf_status s = train(c, d_xyz, n);
            stage_end(c, GPDF_MS_TRAIN);
            if (s != GPDF_OK) return s;
        }
        return fuse(c, h_origin);
    } catch (...) {
        return fail(c, GPDF_E_OOM, "fuse: host allocation failed");
    }
}

namespace {

// inputs of one graph replay, passed by value as kernel arguments
__global__ void k_set_frame(uint32_t *cnt, uint32_t n, uint32_t frame, float ox, float oy, float oz,
                            float *origin) {
    if (threadIdx.x != 0) return;
    cnt[CNT_IN] = n;
    cnt[CNT_FRAME] = frame;
    origin[0] = ox;
    origin[1] = oy;
    origin[2] = oz;
}

gpdf_status capture_frame_graph(gpdf_ctx *c) {
    hipError_t e;
    const int64_t P = c->p.max_points;
    // buffers of an earlier capture that failed
    if (c->d_gin) (void)hipFree(c->d_gin);
    if (c->d_gorigin) (void)hipFree(c->d_gorigin);
    if (c->d_gfirst) (void)hipFree(c->d_gfirst);
    if (c->h_gchunks) (void)hipHostFree(c->h_gchunks);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    c->d_gin = c->d_gorigin = nullptr;
    c->d_gfirst = c->h_gchunks = c->d_gchunks = nullptr;
    c->gstream = nullptr;
    if ((e = hipMalloc((void **)&c->d_gin, sizeof(float) * 3 * size_t(P))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_gorigin, sizeof(float) * 4)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_gfirst, 256)) != hipSuccess ||
        (e = hipHostMalloc((void **)&c->h_gchunks, 256, hipHostMallocMapped)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void **)&c->d_gchunks, c->h_gchunks, 0)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(c, e, "graph: allocate");
    *c->h_gchunks = 0;
    c->geval_node = nullptr;
    c->geval_ok = false;
    gpdf_status st = ensure_offsets(c);
    if (st != GPDF_OK) return st;
    if ((e = ensure_cell_lists(c, c->p.max_queries + 1)) != hipSuccess) return hip_fail(c, e, "graph: cell lists");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "graph: sync");
    hipStream_t user = c->stream;
    c->stream = c->gstream;
    c->capturing = true;
    if ((e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        st = hip_fail(c, e, "graph: begin capture");
    } else {
        st = train(c, c->d_gin, P, c->d_cnt + CNT_IN);
        if (st == GPDF_OK) st = fuse(c, nullptr, c->d_gorigin, P);
        // every stream forked in the capture joins it before it ends
        if (hipError_t je = join_train(c); je != hipSuccess && st == GPDF_OK) st = hip_fail(c, je, "graph: join");
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->gstream, &g);
        if (st == GPDF_OK && e != hipSuccess) st = hip_fail(c, e, "graph: end capture");
        if (st == GPDF_OK) {
            c->graph = g;
            if ((e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0)) != hipSuccess) {
                c->gexec = nullptr;
                st = hip_fail(c, e, "graph: instantiate");
            } else if (c->geval_node) {
                // without the node's parameters every replay keeps the
                // captured grid (the persistent instance takes the rest)
                c->geval_ok = hipGraphKernelNodeGetParams(c->geval_node, &c->geval_params) == hipSuccess;
                c->geval_cur = c->geval_grid0;
            }
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
        if (st != GPDF_OK) {
            c->geval_node = nullptr;
            c->geval_ok = false;
        }
    }
    c->capturing = false;
    c->stream = user;
    return st;
}

}  // namespace

extern "C" gpdf_status gpdf_fuse_frame_graph(gpdf_ctx *c, const float *d_xyz, int64_t n, const float *h_origin) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (!h_origin || !(std::isfinite(h_origin[0]) && std::isfinite(h_origin[1]) && std::isfinite(h_origin[2])))
        return fail(c, GPDF_E_INVALID_ARG, "fuse_frame_graph: origin required");
    if (n < 0 || n > c->p.max_points) return fail(c, GPDF_E_CAPACITY, "fuse_frame_graph: n exceeds max_points");
    if (n > 0 && !d_xyz) return fail(c, GPDF_E_INVALID_ARG, "fuse_frame_graph: null points");
    if (c->p.selection != GPDF_SEL_NEIGHBOR27 || c->p.precision == GPDF_PREC_BF16 ||
        c->p.precision == GPDF_PREC_FP32_MFMA || c->p.lazy_train)
        return fail(c, GPDF_E_INVALID_ARG, "fuse_frame_graph: needs NEIGHBOR27 selection in FP32 or FP64");
    try {
        if (!c->gexec) {
            const gpdf_status st = capture_frame_graph(c);
            if (st != GPDF_OK) {
                if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
                if (c->graph) (void)hipGraphDestroy(c->graph);
                c->gexec = nullptr;
                c->graph = nullptr;
                return st;
            }
        }
        hipStream_t s = c->stream;
        hipError_t e;
        if (n > 0 && (e = hipMemcpyAsync(c->d_gin, d_xyz, sizeof(float) * 3 * size_t(n), hipMemcpyDeviceToDevice,
                                         s)) != hipSuccess)
            return hip_fail(c, e, "fuse_frame_graph: copy points");
        // the evaluation node's grid: from the chunk count of the last replay
        // that has finished (a replay still running gives an older count;
        // either way only the speed changes), reset to that count with a
        // quarter and 64 chunks to spare when the count outgrew the grid or
        // the grid is over twice the count, and left alone otherwise (setting
        // it while replays are queued can wait for them)
        if (c->geval_ok) {
            const uint32_t last = *static_cast<volatile uint32_t *>(c->h_gchunks);
            const unsigned want = std::min<unsigned>(c->geval_gridmax, ((last + last / 4 + 64) + 7u) & ~7u);
            if (last > 0 && (last > c->geval_cur || uint64_t(last) * 2 < c->geval_cur) && want != c->geval_cur) {
                hipKernelNodeParams kp = c->geval_params;
                kp.gridDim = dim3(want);
                if ((e = hipGraphExecKernelNodeSetParams(c->gexec, c->geval_node, &kp)) == hipSuccess) c->geval_cur = want;
                else c->geval_ok = false;  // keep the grid it has
            }
        }
        hipLaunchKernelGGL(k_set_frame, dim3(1), dim3(64), 0, s, c->d_cnt, uint32_t(n), uint32_t(c->frame),
                           h_origin[0], h_origin[1], h_origin[2], c->d_gorigin);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipGraphLaunch(c->gexec, s)) != hipSuccess)
            return hip_fail(c, e, "fuse_frame_graph: launch");
        c->frame++;
        c->model = gpdf::Model();
        c->model.trained = true;
        c->last_test = -1;
        return GPDF_OK;
    } catch (...) {
        return fail(c, GPDF_E_OOM, "fuse_frame_graph: host allocation failed");
    }
}

extern "C" gpdf_status gpdf_query_global(gpdf_ctx *c, const float *d_q, int64_t m, float *d_dist,
                                         float *d_grad, uint8_t *d_valid) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    stage_begin(c, GPDF_MS_GLOBAL);
    gpdf_status s = query_global(c, d_q, m, d_dist, d_grad, d_valid);
    stage_end(c, GPDF_MS_GLOBAL);
    return s;
}

extern "C" gpdf_status gpdf_get_stats(gpdf_ctx *c, gpdf_stats *out) {
    if (!c || !out) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    hipError_t e;
    if ((e = hipMemcpyAsync(c->h_stat, c->d_stat, sizeof(unsigned long long) * ST_COUNT,
                            hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "get_stats");
    const unsigned long long *h = c->h_stat;
    std::memset(out, 0, sizeof *out);
    out->clusters = c->model.nclusters;
    out->points = c->model.npoints;
    if (!c->model.host_counts) {
        // the last frame ran as a graph: its counts are on the device
        uint32_t dc[kCnt];
        if ((e = hipMemcpy(dc, c->d_cnt, sizeof dc, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(c, e, "get_stats");
        out->clusters = dc[CNT_CL];
        out->points = dc[CNT_PTS];
    }
    out->nonpd_clusters = int64_t(h[ST_NONPD]);
    out->skipped_points = int64_t(h[ST_SKIPPED_POINTS]);
    out->queries = c->last_queries;
    out->valid_queries = int64_t(h[ST_VALID_Q]);
    out->refined_queries = int64_t(h[ST_REFINE]);
    out->test_points = c->last_test >= 0 ? c->last_test : int64_t(h[ST_TESTPTS]);
    out->fused = int64_t(h[ST_FUSED]);
    out->fuse_skipped = int64_t(h[ST_FUSE_SKIPPED]);
    out->global_voxels = int64_t(h[ST_GLOBAL_COUNT]);
    out->gated = int64_t(h[ST_GATED]);
    out->eval_pairs = int64_t(h[ST_PAIRS]);
    out->eval_points = int64_t(h[ST_POINTS]);
    out->eval_tri = int64_t(h[ST_TRI]);
    out->refine_dist = int64_t(h[ST_REF_D]);
    out->refine_grad = int64_t(h[ST_REF_G]);
    out->refine_var = int64_t(h[ST_REF_V]);
    out->trained_clusters = c->model.ntrained;
    {
        uint32_t dc[kCnt];
        if ((e = hipMemcpy(dc, c->d_cnt, sizeof dc, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(c, e, "get_stats");
        if (dc[CNT_NREF_FAST] > 0) {
            out->refine_pairs_small = dc[CNT_BPAIRS_S];
            out->refine_pairs_large = dc[CNT_BPAIRS_B];
            out->refine_items_large = dc[CNT_BITEMS];
        }
    }
    uint32_t bits = 0;
    if (h[ST_HASH_FULL]) bits |= GPDF_STATUS_HASH_FULL;
    if (h[ST_GLOBAL_FULL]) bits |= GPDF_STATUS_GLOBAL_FULL;
    if (h[ST_SKIPPED_POINTS] || h[ST_NONFINITE_Q]) bits |= GPDF_STATUS_NONFINITE;
    if (h[ST_NONPD]) bits |= GPDF_STATUS_NONPD;
    if (h[ST_CAPACITY]) bits |= GPDF_STATUS_CAPACITY;
    out->status_bits = bits;
    for (int k = 0; k < 8; ++k) {
        float ms = -1.f;
        if (c->ev_ok[k] && hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) != hipSuccess)
            ms = -1.f;
        out->ms[k] = ms;
    }
    // the status bits and training counters are read once; per-call counters
    // are reset by the calls themselves
    FillList F;
    F.u64(c->d_stat + ST_HASH_FULL, 0ull, 1);
    F.u64(c->d_stat + ST_GLOBAL_FULL, 0ull, 1);
    if (hipError_t e = fill_multi(F, c->stream); e != hipSuccess) return hip_fail(c, e, "stats: reset");
    return GPDF_OK;
}

extern "C" const char *gpdf_last_error(const gpdf_ctx *c) {
    return c ? c->err.c_str() : "null context";
}

extern "C" gpdf_status gpdf_export_model(gpdf_ctx *c, uint64_t *h_ckey, int64_t *h_off,
                                         float *h_points, double *h_alpha, uint8_t *h_pd) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    if (!c->model.trained) return fail(c, GPDF_E_NOT_TRAINED, "export before training");
    const int64_t nc = c->model.nclusters, np = c->model.npoints;
    hipError_t e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "export");
    if (h_ckey && nc && (e = hipMemcpy(h_ckey, c->d_ckey, 8 * nc, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "export keys");
    if (h_off) {
        std::vector<int32_t> o(nc + 1, 0);
        if (nc && (e = hipMemcpy(o.data(), c->d_coff, 4 * (nc + 1), hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(c, e, "export offsets");
        for (int64_t i = 0; i <= nc; ++i) h_off[i] = o[i];
    }
    if (h_points && np) {
        std::vector<float4> p(np);
        if ((e = hipMemcpy(p.data(), c->d_pts, 16 * np, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(c, e, "export points");
        for (int64_t i = 0; i < np; ++i) {
            h_points[3 * i] = p[i].x; h_points[3 * i + 1] = p[i].y; h_points[3 * i + 2] = p[i].z;
        }
    }
    if (h_alpha && np && (e = hipMemcpy(h_alpha, c->d_alpha64, 8 * np, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "export alpha");
    if (h_pd && nc && (e = hipMemcpy(h_pd, c->d_pd, nc, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "export pd");
    return GPDF_OK;
}

extern "C" gpdf_status gpdf_nearest_distance(gpdf_ctx *c, const float *d_pts, int64_t n,
                                             const float *d_q, int64_t m, float *d_out) {
    if (!c) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    return nearest_distance(c, d_pts, n, d_q, m, d_out);
}

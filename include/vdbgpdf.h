/*
 * vdbgpdf.h -- C ABI of the MI355X L-GPDF library (libvdbgpdf.so).
 *
 * The library implements the data-parallel hot path of VDB-GPDF (Wu,
 * Le Gentil, Vidal-Calleja, "VDB-GPDF: Online Gaussian Process Distance
 * Field with VDB Structure", arXiv:2407.09649): local Gaussian-process
 * distance fields trained per leaf cluster of a voxelised point cloud
 * (L-GPDF, Sec. IV-A), queried for distance, gradient and variance
 * (Eq. (1)-(5), Eq. (10)), and fused by inverse-variance weighting into a
 * device-resident hashed voxel grid standing in for the global VDB
 * (Sec. IV-C, Eq. (7)-(8)).
 *
 * Conventions for every call:
 *  - Pointers named d_* are DEVICE pointers owned by the caller (for example
 *    torch tensor storage on the GPU).  Point arrays are row-major float[n][3]
 *    in the world frame.  Outputs are written in input order.
 *  - Pointers named h_* are HOST pointers owned by the caller.
 *  - All calls enqueue work on the context's HIP stream and may return before
 *    it finishes; the caller keeps device buffers alive until the stream is
 *    synchronised.  gpdf_train_local_gps and gpdf_fuse_frame synchronise the
 *    stream once internally to size their launches.
 *  - Training runs its clusters above 64 points on a second, internal stream
 *    of the same context.  After gpdf_train_local_gps returns that part may
 *    still run: the next call of this library that needs the model or its
 *    buffers (any call below except gpdf_params_default, gpdf_create,
 *    gpdf_last_error and the tuning getters/setters) first makes the
 *    context's stream wait for it, and gpdf_destroy waits for it.  Work that
 *    the caller enqueues on the stream directly does not wait for it.
 *  - The library owns its arenas.  They are sized at gpdf_create from the
 *    capacities in gpdf_params and never grow: a call that would exceed one
 *    returns GPDF_E_CAPACITY and leaves the previous state untouched.
 *  - Return codes report host-detectable errors (null or non-finite
 *    arguments, capacity, use before training, HIP failures).  Conditions
 *    found on the device (non-finite inputs, non-positive-definite clusters,
 *    refined queries, hash overflow) are counted and read with
 *    gpdf_get_stats.
 *  - An invalid query (no usable cluster around it, or a non-finite
 *    coordinate) returns dist = +inf, grad = 0, var = +inf, valid = 0.
 *  - No C++ exception crosses the ABI.  A context is used by one host thread
 *    at a time.
 */
#ifndef VDBGPDF_H
#define VDBGPDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPDF_ABI_VERSION 4u

typedef struct gpdf_ctx gpdf_ctx;

typedef enum {
    GPDF_OK = 0,
    GPDF_E_INVALID_ARG = 1,
    GPDF_E_OOM = 2,
    GPDF_E_HIP = 3,
    GPDF_E_CAPACITY = 4,
    GPDF_E_NOT_TRAINED = 5
} gpdf_status;

/* covariance function: Matern-3/2 k(r) = (1 + sqrt3 r/l) e^{-sqrt3 r/l}, or
 * the squared exponential k(r) = e^{-r^2 / 2l^2} of Sec. III-A (k(0) = 1) */
enum { GPDF_KERNEL_MATERN32 = 0, GPDF_KERNEL_SE = 1 };
/* which local GPs a query uses: the 27 cells around its own, or the Q whose
 * cell centres are nearest (the Q nearest nodes of Sec. IV-D) */
enum { GPDF_SEL_NEIGHBOR27 = 0, GPDF_SEL_KNN = 1 };
/* combination: smooth minimum of Eq. (10) read with exp(-lambda d), or the
 * closest node only (the node with the smallest distance, Sec. IV-B) */
enum { GPDF_COMB_SMOOTHMIN = 0, GPDF_COMB_HARDMIN = 1 };
/* gradient combination: smooth-min weights, or the plain mean of the node
 * gradients ("directly average", Sec. IV-D) */
enum { GPDF_GRAD_WEIGHTED = 0, GPDF_GRAD_PAPER_MEAN = 1 };
/* query arithmetic: FP32 with an FP64 re-evaluation of the queries whose FP32
 * error bound exceeds the tolerance; everything in FP64; the FP32 path with
 * the variance product W k on BF16 MFMA (FP32 accumulation), whose queries are
 * re-evaluated in FP64 for distance and gradient but not for the variance,
 * which keeps the BF16 error; or the FP32 path with W k on FP32 MFMA
 * (v_mfma_f32_16x16x4_f32, clusters up to 248 points), every output keeping
 * the FP32 path's tolerances.  The two MFMA modes need NEIGHBOR27 selection
 * and are not captured in the frame graph. */
enum { GPDF_PREC_FP32 = 0, GPDF_PREC_BF16 = 1, GPDF_PREC_FP64 = 2, GPDF_PREC_FP32_MFMA = 3 };
/* fusion rule: inverse-variance weighting of Eq. (7)-(8), or the TSDF-style
 * accumulated weights of Eq. (9) with the weight 1 - v of each observation
 * (non-positive weights are skipped) */
enum { GPDF_FUSE_INVVAR = 0, GPDF_FUSE_TSDF = 1 };
/* test points of a fused frame: every global voxel within fuse_band of a
 * training point, or the voxels that the rays from the sensor to the
 * training voxels cross and that the grid already holds, plus the voxels
 * along each training voxel's surface normal up to normal_reach
 * (Sec. IV-B) */
enum { GPDF_TEST_BAND = 0, GPDF_TEST_RAYCAST = 1 };

typedef struct {
    uint32_t abi_version;      /* must equal GPDF_ABI_VERSION */
    int32_t kernel;            /* GPDF_KERNEL_* */
    double length_scale;       /* l, metres */
    double noise_sigma;        /* s: K + s^2 I (Eq. (1)) */
    double voxel_size;         /* > 0: training points are the centres of the
                                  occupied voxels and a cluster is a leaf of
                                  8^3 voxels (Sec. III-B, IV-A);
                                  0: raw points in cells of cluster_size */
    double cluster_size;       /* raw-mode cluster edge, metres */
    int32_t selection;         /* GPDF_SEL_* */
    int32_t knn_q;             /* Q for GPDF_SEL_KNN, 1..16 */
    int32_t combine;           /* GPDF_COMB_* */
    int32_t grad_mode;         /* GPDF_GRAD_* */
    double smooth_min_lambda;  /* 100 in Sec. IV-D */
    double occ_min, occ_max;   /* caps on the latent occupancy (footnote 1) */
    int32_t precision;         /* GPDF_PREC_* */
    int32_t timing;            /* 1: time each stage with HIP events on the
                                  context stream (gpdf_stats.ms) */
    double fuse_voxel_size;    /* global grid edge */
    double fuse_band;          /* test-point band radius, metres */
    double mlp_gate;           /* correction applied where variance <= gate */
    int64_t max_points;        /* capacity: points per training call */
    int64_t max_clusters;      /* capacity: clusters per training call */
    int64_t max_cluster_points;/* capacity: points in one cluster (<= 1024) */
    int64_t max_factor_elems;  /* capacity: sum over clusters of n(n+1)/2 */
    int64_t max_queries;       /* capacity: queries per call (also test points) */
    int64_t global_capacity;   /* capacity: voxels of the global grid */
    int32_t fuse_rule;         /* GPDF_FUSE_* */
    int32_t test_points;       /* GPDF_TEST_* */
    double normal_reach;       /* GPDF_TEST_RAYCAST: metres along the normal */
    int32_t lazy_train;        /* 1: gpdf_train_local_gps builds the clusters
                                  but factors none; each query call trains
                                  the clusters its queries select that are
                                  not trained yet (the lazily trained nodes
                                  of the G-GPDF, Sec. IV-D).  Not with
                                  gpdf_fuse_frame_graph. */
    int32_t properties;        /* 1: the context also carries one surface
                                  property per point (intensity, a colour
                                  channel; Eq. (6), Sec. IV-C): its GP, its
                                  fusion and its global query (the *_prop
                                  calls).  Needs FP32 or FP64 precision,
                                  NEIGHBOR27 selection and lazy_train = 0. */
} gpdf_params;

typedef struct {
    int64_t clusters;          /* clusters of the last training */
    int64_t points;            /* training points of the last training */
    int64_t nonpd_clusters;    /* excluded: factor not positive definite */
    int64_t skipped_points;    /* non-finite or out-of-range inputs */
    int64_t queries;           /* queries of the last query call */
    int64_t valid_queries;
    int64_t refined_queries;   /* FP32 queries re-evaluated in FP64 */
    int64_t test_points;       /* test points of the last fused frame */
    int64_t fused;             /* observations fused in the last frame */
    int64_t fuse_skipped;      /* invalid or non-finite observations */
    int64_t global_voxels;     /* voxels in the global grid */
    int64_t gated;             /* queries corrected by the MLP */
    int64_t eval_pairs;        /* last query, FP32 27-cell pass: (query, cluster) pairs */
    int64_t eval_points;       /*   kernel evaluations, sum of n over the pairs */
    int64_t eval_tri;          /*   variance multiply-adds, sum of n (n + 1) / 2 */
    int64_t refine_dist;       /* last query: FP32 estimates above the distance, */
    int64_t refine_grad;       /*   gradient and variance thresholds (a query   */
    int64_t refine_var;        /*   can count in several)                       */
    uint32_t status_bits;      /* GPDF_STATUS_* set since the last read */
    uint32_t pad0;
    float ms[8];               /* with timing = 1: GPU time of the last run of
                                  each stage (GPDF_MS_*), milliseconds;
                                  -1 when the stage has not run */
    int64_t trained_clusters;  /* clusters factored since the last training
                                  (all of them unless lazy_train) */
    int64_t refine_pairs_small;/* last query, FP64 re-evaluation: (refined
                                  query, cluster) pairs of clusters of at most
                                  32 points, */
    int64_t refine_pairs_large;/*   of 33 to 256 points, */
    int64_t refine_items_large;/*   and the work items of the latter (up to
                                  16 queries of one cluster each); all 0
                                  when the pass did not run (KNN selection,
                                  a cluster above 256 points, or more pairs
                                  than its buffers hold) */
} gpdf_stats;

enum {
    GPDF_MS_TRAIN = 0,   /* gpdf_train_local_gps, all kernels */
    GPDF_MS_GROUP = 1,   /* query: grouping by cell and neighbour lists */
    GPDF_MS_EVAL = 2,    /* query: the main evaluation kernel */
    GPDF_MS_REFINE = 3,  /* query: regrouping and FP64 re-evaluation */
    GPDF_MS_TESTPTS = 4, /* fuse: test-voxel generation */
    GPDF_MS_FUSE = 5,    /* fuse: the update of the global grid */
    GPDF_MS_GLOBAL = 6,  /* gpdf_query_global */
    GPDF_MS_MLP = 7      /* learned correction (features, forward, gate) */
};

enum {
    GPDF_STATUS_HASH_FULL = 1u,       /* a probe sequence exhausted a table */
    GPDF_STATUS_GLOBAL_FULL = 2u,     /* the global grid is full */
    GPDF_STATUS_NONFINITE = 4u,       /* non-finite input points or queries */
    GPDF_STATUS_NONPD = 8u,           /* some cluster was not positive definite */
    GPDF_STATUS_CAPACITY = 16u        /* a capacity was exceeded inside a frame graph */
};

/* Fill *p with defaults: Matern-3/2, l = 0.2 m, s = 0.01, raw points in 0.4 m
 * cells, 27-cell selection, smooth minimum with lambda = 100 (Sec. IV-D),
 * occupancy caps [1e-15, 1 - 1e-5], FP32, global grid 0.05 m with a 0.2 m
 * band, gate 0.05 m^2, and capacities for a few million points and queries. */
gpdf_status gpdf_params_default(gpdf_params *p);

/* Create a context bound to one HIP stream (hipStream_t passed as void*; NULL
 * is the null stream) on the current device.  Allocates every arena.
 * Errors: GPDF_E_INVALID_ARG (bad parameters or ABI version), GPDF_E_OOM. */
gpdf_status gpdf_create(const gpdf_params *p, void *hip_stream, gpdf_ctx **out);

/* Release the context and its device memory (synchronises its stream). */
void gpdf_destroy(gpdf_ctx *ctx);

/* Replace the local GPs with ones trained on d_xyz [n][3] (the L-GPDF of the
 * current frame, re-modelled every frame, Sec. IV-A): voxelise (voxel mode),
 * group into leaf clusters, and for every cluster assemble K + s^2 I, factor
 * it in FP64 and solve for alpha = (K + s^2 I)^{-1} 1 (Eq. (1)).  Non-finite
 * points are skipped and counted.  n = 0 leaves an empty model.
 * Errors: GPDF_E_CAPACITY (n, cluster count, cluster size or factor storage
 * beyond the arenas), GPDF_E_INVALID_ARG. */
gpdf_status gpdf_train_local_gps(gpdf_ctx *ctx, const float *d_xyz, int64_t n);

/* gpdf_train_local_gps with a surface property per point, d_prop [n]
 * (device; Eq. (6)).  The property of a training point is that of its raw
 * points: in voxel mode their mean (summed in FP64 in input order), in raw
 * mode the point's own.  The property GP of a cluster has the distance GP's
 * kernel and noise s, so beta = (K + s^2 I)^{-1} c is solved on the same
 * factor: beta = W^T (W c).  Properties are expected of order one (an
 * intensity or colour channel in [0, 1]); the FP32 query refines them in
 * FP64 beyond an estimated error of 2e-5 in their own units.
 * Errors: GPDF_E_INVALID_ARG (properties = 0 in the parameters, or null
 * pointers), and those of gpdf_train_local_gps. */
gpdf_status gpdf_train_local_gps_prop(gpdf_ctx *ctx, const float *d_xyz, const float *d_prop, int64_t n);

/* Distance field at d_q [m][3] from the current local GPs: per selected
 * cluster the latent occupancy (Eq. (1)), its variance (Eq. (2), posterior
 * minus sign), reverting (Eq. (3)), distance variance (Eq. (4)) and gradient
 * (Eq. (5) with the chain rule), combined over clusters (Eq. (10)).  With
 * h_origin (host float[3]) the distance and gradient carry the sign of the
 * sensor side (Sec. IV); NULL gives the unsigned field.
 * Outputs (device, may be NULL except d_dist and d_valid): d_dist [m],
 * d_grad [m][3], d_var [m], d_valid [m] (uint8), d_aux [m][3] = latent
 * occupancy and latent variance of the closest cluster and the number of
 * training points used.  correct != 0 applies the learned correction where
 * the variance is at most mlp_gate (requires gpdf_mlp_* weights).
 * Precision: FP32 with an FP64 re-evaluation of the queries whose estimated
 * FP32 error exceeds the tolerance of a requested output (distance always,
 * gradient and variance when their buffers are given).
 * Errors: GPDF_E_NOT_TRAINED, GPDF_E_CAPACITY (m > max_queries). */
gpdf_status gpdf_query_distance(gpdf_ctx *ctx, const float *d_q, int64_t m,
                                const float *h_origin, float *d_dist,
                                float *d_grad, float *d_var, uint8_t *d_valid,
                                float *d_aux, int32_t correct);

/* gpdf_query_distance plus the surface property (Eq. (6)): per selected
 * cluster c_q = k . beta and its variance, the latent variance u of
 * Eq. (2) (the property GP's posterior variance); both combined over the
 * clusters like the distance variance (smooth-minimum weights of the
 * distances, or the closest node).  d_prop [m] and d_prop_var [m] (device;
 * either may be NULL, not both); invalid queries get 0 and infinity.
 * Errors: as gpdf_query_distance; GPDF_E_INVALID_ARG when the current
 * model was trained without a property. */
gpdf_status gpdf_query_distance_prop(gpdf_ctx *ctx, const float *d_q, int64_t m,
                                     const float *h_origin, float *d_dist, float *d_grad,
                                     float *d_var, uint8_t *d_valid, float *d_aux,
                                     float *d_prop, float *d_prop_var);

/* gpdf_query_distance for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation, arguments and results, and no hipMalloc,
 * hipFree or other allocating call.  gpdf_query_distance keeps its per-cell
 * cluster lists in a context buffer that it grows when a call meets more
 * cells than before; this variant uses a fixed array in device memory
 * instead, 28 MiB per GPU (one copy per GPU that the library runs on, held
 * until the process ends), holding the lists of at most 65,536 query cells
 * (cells of the cluster grid that hold at least one query).
 * Every call of this function on a GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other contexts, other streams) race and must
 * be serialised by the caller.  Each call rebuilds the lists it reads, so no
 * contents carry over between calls.
 * Errors: as gpdf_query_distance; GPDF_E_CAPACITY when the queries fall in
 * more than 65,536 cells (nothing is evaluated); GPDF_E_INVALID_ARG for a
 * context with BF16 precision (its factor copy is built on first use). */
gpdf_status gpdf_query_distance_noalloc(gpdf_ctx *ctx, const float *d_q, int64_t m,
                                        const float *h_origin, float *d_dist,
                                        float *d_grad, float *d_var, uint8_t *d_valid,
                                        float *d_aux, int32_t correct);

/* One frame of fusion (Sec. IV-B, IV-C): train on d_xyz [n][3] (or, with
 * d_xyz == NULL, reuse the current local GPs), generate the test voxels of
 * the global grid (GPDF_TEST_BAND: those within fuse_band of the training
 * points; GPDF_TEST_RAYCAST: for every training voxel the voxels on the ray
 * from h_origin that the grid already holds, the measured voxel, and the
 * voxels along its surface normal within normal_reach -- an exact integer
 * walk between voxel centres, and the least-spread integer direction of the
 * training voxels within +-2 voxels), query them signed from h_origin, and
 * fuse each valid result into the grid:
 * D <- (V d + v D) / (V + v), V <- V v / (V + v) (Eq. (7)-(8)); absent voxels
 * take (d, v).  Updated voxels are stamped with the frame counter.
 * Errors: GPDF_E_CAPACITY (test points > max_queries, grid full),
 * GPDF_E_NOT_TRAINED (d_xyz == NULL before any training). */
gpdf_status gpdf_fuse_frame(gpdf_ctx *ctx, const float *d_xyz, int64_t n,
                            const float *h_origin);

/* gpdf_fuse_frame with a surface property per point, d_prop [n] (device):
 * trains with it (gpdf_train_local_gps_prop) and fuses the property of each
 * test voxel beside its distance, with the same expressions and the
 * property's variance w in place of v (Eq. (7)-(8); with GPDF_FUSE_TSDF the
 * weight 1 - w): C <- (W c + w C) / (W + w), W <- W w / (W + w).  A voxel
 * with no property yet takes (c, w); an observation whose variance (weight)
 * is not positive and finite leaves the voxel's property unchanged.  Voxels
 * fused by calls without a property hold none (NaN).
 * Errors: as gpdf_fuse_frame and gpdf_train_local_gps_prop. */
gpdf_status gpdf_fuse_frame_prop(gpdf_ctx *ctx, const float *d_xyz, const float *d_prop, int64_t n,
                                 const float *h_origin);

/* gpdf_fuse_frame as one replay of a captured HIP graph (batching
 * extension).  The first call records training, test voxels, their query and
 * the fusion with every count kept on the device and every grid sized by the
 * capacities (max_points input points, max_queries test voxels); each call
 * then copies d_xyz [n][3] (n <= max_points), the frame stamp and h_origin
 * into context buffers and replays the graph on the context stream, with no
 * host round trip.  Results equal gpdf_fuse_frame.  Needs NEIGHBOR27
 * selection in FP32 or FP64.  The first call allocates cell lists for
 * max_queries cells (448 B each).  A capacity exceeded inside the graph
 * (max_clusters, max_cluster_points, max_factor_elems, max_queries) is not
 * returned: the affected clusters are left out and GPDF_STATUS_CAPACITY is
 * set in gpdf_stats.status_bits.  The graph fuses no surface property (voxels
 * it creates hold none).
 * Errors: GPDF_E_INVALID_ARG, GPDF_E_CAPACITY (n > max_points). */
gpdf_status gpdf_fuse_frame_graph(gpdf_ctx *ctx, const float *d_xyz, int64_t n,
                                  const float *h_origin);

/* Query the fused grid at d_q [m][3]: trilinear interpolation of D over the
 * eight voxel centres around each point and its analytic gradient; valid only
 * where all eight voxels exist (stand-in for the global field of Sec. IV-D).
 * Outputs: d_dist [m], d_grad [m][3] (may be NULL), d_valid [m]. */
gpdf_status gpdf_query_global(gpdf_ctx *ctx, const float *d_q, int64_t m,
                              float *d_dist, float *d_grad, uint8_t *d_valid);

/* The fused surface property at d_q [m][3]: trilinear interpolation of C
 * over the eight voxel centres around each point; valid only where all
 * eight exist and hold a property.  Outputs (device): d_prop [m] (0 where
 * invalid), d_valid [m].  Errors: GPDF_E_INVALID_ARG (properties = 0). */
gpdf_status gpdf_query_global_prop(gpdf_ctx *ctx, const float *d_q, int64_t m, float *d_prop,
                                   uint8_t *d_valid);

/* Counters of the last calls (synchronises the stream). */
gpdf_status gpdf_get_stats(gpdf_ctx *ctx, gpdf_stats *out);

/* Message of the last error on this context (owned by the context). */
const char *gpdf_last_error(const gpdf_ctx *ctx);

/* Copy the current local GPs to host memory (synchronises): cluster keys
 * (three 21-bit offset-binary cell coordinates), CSR offsets [clusters + 1],
 * training points [points][3], alpha in FP64 [points], positive-definite
 * flags [clusters].  Any pointer may be NULL.  Sizes come from gpdf_get_stats.
 * Errors: GPDF_E_NOT_TRAINED. */
gpdf_status gpdf_export_model(gpdf_ctx *ctx, uint64_t *h_ckey, int64_t *h_off,
                              float *h_points, double *h_alpha, uint8_t *h_pd);

/* Copy the global grid, sorted by key, to host memory (synchronises).  *count
 * receives the number of voxels; nothing is written if it exceeds cap. */
gpdf_status gpdf_export_global(gpdf_ctx *ctx, uint64_t *h_key, float *h_D,
                               float *h_V, uint32_t *h_stamp, int64_t cap,
                               int64_t *count);

/* The fused property of every voxel of the global grid, in the order of
 * gpdf_export_global (host arrays; C and W are NaN where none was fused).
 * Errors: GPDF_E_INVALID_ARG (properties = 0). */
gpdf_status gpdf_export_global_prop(gpdf_ctx *ctx, uint64_t *h_key, float *h_C, float *h_W,
                                    int64_t cap, int64_t *count);

/* Copy the sorted unique test-voxel keys of the last fused frame. */
gpdf_status gpdf_export_test_points(gpdf_ctx *ctx, uint64_t *h_key,
                                    int64_t cap, int64_t *count);

/* Zero crossings of the global grid: the surface points from which the
 * global GP distance field (G-GPDF, Sec. IV-D) is trained.  On every edge
 * between two neighbouring voxels of the grid whose distances D have opposite
 * signs (one negative, the other not), the point where the linear
 * interpolant of D along the edge is zero -- the vertices that marching cubes
 * places (Lorensen and Cline 1987).  The coordinate along the edge is
 * (c + 1/2 + t) h with t = D_a / (D_a - D_b) computed in FP64, the others
 * (c + 1/2) h; rounded once to FP32.  Points are listed by ascending key of
 * the edge's lower voxel, then by axis x, y, z.
 * *count receives the number of points; d_out (device, [cap][3]) is written
 * only when cap >= *count (call with d_out NULL and cap 0 to size it).
 * Synchronises the stream twice; allocates its work buffers on first use
 * (and when a larger grid needs more).  A G-GPDF is a second context with
 * voxel_size 0, cluster_size 8 fuse_voxel_size (a leaf of the grid) and
 * GPDF_SEL_KNN (the Q nearest nodes), trained on these points.
 * Errors: GPDF_E_INVALID_ARG (null count, cap > 0 with null d_out). */
gpdf_status gpdf_zero_crossings(gpdf_ctx *ctx, float *d_out, int64_t cap, int64_t *count);

/* Write / read the global grid: a header (magic, version, voxel size, count,
 * frame counter) and the key-sorted (key, D, V, stamp) records; version 2
 * (written with properties = 1) appends (C, W) to each record and loads only
 * into a context with properties = 1. */
gpdf_status gpdf_save_global(gpdf_ctx *ctx, const char *path);
gpdf_status gpdf_load_global(gpdf_ctx *ctx, const char *path);

/* Brute-force distance from every d_q [m][3] to the nearest of d_pts [n][3]
 * (FP32 differences, exact minimum) -- the truth used to generate training
 * pairs for the learned correction. */
gpdf_status gpdf_nearest_distance(gpdf_ctx *ctx, const float *d_pts, int64_t n,
                                  const float *d_q, int64_t m, float *d_out);

/* ---- batching: launch shapes picked by measurement (an extension) --------
 * train_threads: workgroup of the trainer of the clusters above 256 points
 * (256, 512 or 1024).  eval_persistent: 0 launches one wavefront per 64-query
 * chunk; 1, 2 or 4 keep that many persistent wavefronts per SIMD taking
 * chunks from a counter (NEIGHBOR27 selection; KNN ignores it).  mfma_min_n:
 * the size bucket boundary of the FP32 evaluation -- the clusters of
 * mfma_min_n (17, 33, 65 or 129) to 248 points take the variance product on
 * FP32 MFMA (as GPDF_PREC_FP32_MFMA), the others the VALU path; 0 keeps the
 * VALU path for every cluster (eager NEIGHBOR27 queries without a property;
 * with a non-zero boundary eval_persistent does not apply).
 * gpdf_autotune trains on d_xyz [n][3], then times the train_threads
 * candidates and, on queries d_q [m][3] (signed from h_origin, or unsigned
 * with NULL), the eval_persistent candidates and the mfma_min_n boundaries,
 * three timed runs after a warm-up each; it keeps the fastest and leaves the
 * context trained on d_xyz.  h_ms (float[11] or NULL) receives the median
 * times in ms: train 256/512/1024, query 0/1/2/4, MFMA from 17/33/65/129
 * points (-1 where not run).  The result is cached, process-wide, under the
 * shape of the workload (precision, selection, kernel, clustering mode, the
 * cluster-size histogram over 1-8, 9-16, ..., 129-256, >256 and the query
 * count, counts rounded to powers of two): a later call with a cached shape
 * takes the cached shapes without timing and sets *h_cached (may be NULL)
 * to 1.  gpdf_tuning_cache_save / _load write and read the cache as text
 * (a header line, then `shape|train_threads eval_persistent mfma_min_n`
 * lines); _clear empties it.
 * Errors: GPDF_E_INVALID_ARG (empty input, unknown shape, unreadable or
 * malformed cache file), GPDF_E_CAPACITY. */
gpdf_status gpdf_set_tuning(gpdf_ctx *ctx, int32_t train_threads,
                            int32_t eval_persistent, int32_t mfma_min_n);
gpdf_status gpdf_get_tuning(const gpdf_ctx *ctx, int32_t *train_threads,
                            int32_t *eval_persistent, int32_t *mfma_min_n);
gpdf_status gpdf_autotune(gpdf_ctx *ctx, const float *d_xyz, int64_t n,
                          const float *d_q, int64_t m, const float *h_origin,
                          float *h_ms, int32_t *h_cached);
gpdf_status gpdf_tuning_cache_save(const char *path);
gpdf_status gpdf_tuning_cache_load(const char *path);
gpdf_status gpdf_tuning_cache_clear(void);

/* ---- measured peaks (measurement support; not in the paper) -------------
 * gpdf_measure_peaks runs small probe kernels on the context's device and
 * writes what this device sustains into h_out[0..8]: a 1 GiB device copy in
 * GB/s (bytes read plus written), FP32 FMA chains in TFLOP/s (an FMA counts
 * two) in the VOP2 register form (v_fmac_f32), exp2 in Gop/s, BF16 16x16x32,
 * FP32 16x16x4 and FP64 16x16x4 MFMA in TFLOP/s, the copy size in GiB, and
 * FP32 FMA in the VOP3 form (v_fma_f32) and the VOP2 literal form
 * (v_fmamk_f32).  Each probe is timed with HIP events on
 * the context's stream after one warm-up launch.  It allocates 2 GiB of
 * device memory for the duration of the call, and frees it before it returns.
 * Errors: GPDF_E_INVALID_ARG (n_out < 9 or a NULL pointer), GPDF_E_HIP. */
gpdf_status gpdf_measure_peaks(gpdf_ctx *ctx, double *h_out, int32_t n_out);

/* ---- learned correction (an extension; not in the paper) ----------------
 * A 7-64-64-64-1 GELU network maps standardised features
 * [d, log v, o, grad d (3), log(1 + n_local)] to a residual r.  Parameters
 * are 8,897 FP32 master weights in the order W1[64x7], b1, W2[64x64], b2,
 * W3[64x64], b3, W4[1x64], b4 (row-major W[out][in]); forward and backward
 * run on BF16 MFMA with FP32 accumulation. */
#define GPDF_MLP_NPARAM 8897
gpdf_status gpdf_mlp_init(gpdf_ctx *ctx, uint64_t seed);
gpdf_status gpdf_mlp_set_weights(gpdf_ctx *ctx, const float *h_w, int64_t n);
gpdf_status gpdf_mlp_get_weights(gpdf_ctx *ctx, float *h_w, int64_t cap);
/* feature standardisation: z = (f - mean) / std, h_mean and h_std float[7] */
gpdf_status gpdf_mlp_set_norm(gpdf_ctx *ctx, const float *h_mean,
                              const float *h_std);
/* the standardisation in use (set by gpdf_mlp_set_norm or by training) */
gpdf_status gpdf_mlp_get_norm(gpdf_ctx *ctx, float *h_mean, float *h_std);
/* raw features [n][7] from query outputs (dist, var, aux, grad) */
gpdf_status gpdf_mlp_features(gpdf_ctx *ctx, const float *d_dist,
                              const float *d_var, const float *d_grad,
                              const float *d_aux, int64_t n, float *d_feat);
/* residual r [n] from raw features [n][7] */
gpdf_status gpdf_mlp_forward(gpdf_ctx *ctx, const float *d_feat, int64_t n,
                             float *d_r);
/* mean squared error of r against d_target [n] and its gradient [8897] */
gpdf_status gpdf_mlp_grad(gpdf_ctx *ctx, const float *d_feat,
                          const float *d_target, int64_t n, float *d_grad,
                          float *h_loss);
/* epochs of shuffled mini-batch Adam (beta 0.9/0.999, eps 1e-8) on
 * (feature, target) pairs; *h_loss receives the last epoch's mean loss */
gpdf_status gpdf_mlp_train(gpdf_ctx *ctx, const float *d_feat,
                           const float *d_target, int64_t n, int32_t epochs,
                           int32_t batch, float lr, uint64_t seed,
                           float *h_loss);

#ifdef __cplusplus
}
#endif
#endif /* VDBGPDF_H */

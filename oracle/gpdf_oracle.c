/*
 * gpdf_oracle.c -- plain, slow FP64 CPU oracle of the L-GPDF hot path of
 * VDB-GPDF (Wu, Le Gentil, Vidal-Calleja, "VDB-GPDF: Online Gaussian Process
 * Distance Field with VDB Structure", arXiv:2407.09649).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the HIP path against an independent
 * implementation.  It shares no code, header, table or constant generator
 * with the HIP sources.
 *
 * Everything is computed in IEEE double from the FP32 inputs, in the order
 * the paper describes, with no blocking or fusion:
 *   keys / voxel centres / leaf clusters ... Sec. IV (overview) and IV-A
 *   local GP training, K + s^2 I, Cholesky ... Eq. (1)
 *   latent occupancy, latent variance ....... Eq. (1), Eq. (2)
 *   reverting function and its derivative ... Eq. (3), Eq. (4)
 *   gradient ................................ Eq. (5)
 *   combination over Q nodes ................ Eq. (10)
 *   fusion of mean and variance ............. Eq. (7), Eq. (8)
 * Readings taken where the paper is silent, ambiguous or garbled are noted in
 * place (variance sign, smooth-min sign, cap values, sign rule, test points,
 * global interpolation).
 *
 * The sign of the distance follows the sensor side of the nearest training
 * point.  That point and the side are decided here in FP64 from the FP32
 * inputs (ties to the smaller cluster key, then the smaller member index).
 * A query whose decision an FP32 evaluation could take the other way (two
 * candidates on different sides whose squared distances lie within FP32
 * rounding of each other, or a side product within its FP32 rounding of
 * zero) is flagged as a sign near-tie, so that a comparison can tell such a
 * query from a wrong sign.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math, no
 * contraction: every double operation is a single rounded IEEE operation).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* parameters                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t kernel;      /* 0 Matern-3/2, 1 squared exponential (Sec. III-A) */
    int32_t selection;   /* 0 the 27 cells around the query, 1 Q nearest     */
    int32_t knn_q;       /* Q for selection 1                                */
    int32_t combine;     /* 0 smooth minimum Eq. (10), 1 closest node only   */
    int32_t grad_mode;   /* 0 smooth-min weights, 1 plain mean (Sec. IV-D)   */
    int32_t pad_;
    double l;            /* kernel length scale                              */
    double s;            /* noise sigma: the diagonal gets s^2 (Eq. (1))     */
    double voxel;        /* voxel edge for downsampling, 0 = raw points      */
    double cell;         /* cluster edge when voxel == 0                     */
    double lambda;       /* smooth-minimum sharpness (100 in Sec. IV-D)      */
    double occ_min;      /* lower cap of the latent occupancy (footnote 1)   */
    double occ_max;      /* upper cap                                        */
    double fuse_voxel;   /* global grid edge                                 */
    double fuse_band;    /* test-point band radius in metres                 */
    int32_t fuse_rule;   /* 0 inverse-variance Eq. (7)-(8), 1 TSDF-style (9) */
    int32_t tp_mode;     /* 0 band test points, 1 ray-cast + normals (IV-B)  */
    double normal_reach; /* metres along the normal (tp_mode 1)              */
} orc_params;

/* ------------------------------------------------------------------------ */
/* keys: floor(x / h) per axis in double, three 21-bit offset-binary fields  */
/* (voxelisation of Sec. IV overview; VDB's integer coordinates)             */
/* ------------------------------------------------------------------------ */
#define ORC_KEY_BIAS 1048576LL /* 2^20 */

static int orc_floor_coord(float x, double h, int64_t *c)
{
    double q, f;
    if (!isfinite(x)) return 0;
    q = (double)x / h;
    f = floor(q);
    if (f < -(double)ORC_KEY_BIAS || f >= (double)ORC_KEY_BIAS) return 0;
    *c = (int64_t)f;
    return 1;
}

static uint64_t orc_pack(int64_t cx, int64_t cy, int64_t cz)
{
    return ((uint64_t)(cx + ORC_KEY_BIAS) << 42) |
           ((uint64_t)(cy + ORC_KEY_BIAS) << 21) |
           (uint64_t)(cz + ORC_KEY_BIAS);
}

static void orc_unpack(uint64_t k, int64_t c[3])
{
    c[0] = (int64_t)((k >> 42) & 0x1FFFFF) - ORC_KEY_BIAS;
    c[1] = (int64_t)((k >> 21) & 0x1FFFFF) - ORC_KEY_BIAS;
    c[2] = (int64_t)(k & 0x1FFFFF) - ORC_KEY_BIAS;
}

/* integer floor division (leaf = 8 voxels per axis, Sec. III-B) */
static int64_t orc_floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

/* keys of n points at edge h; ok[i] = 0 for non-finite or out-of-range */
int64_t orc_keys(const float *xyz, int64_t n, double h, uint64_t *key,
                 uint8_t *ok)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        int good = orc_floor_coord(xyz[3 * i], h, &c[0]) &&
                   orc_floor_coord(xyz[3 * i + 1], h, &c[1]) &&
                   orc_floor_coord(xyz[3 * i + 2], h, &c[2]);
        ok[i] = (uint8_t)good;
        key[i] = good ? orc_pack(c[0], c[1], c[2]) : ~(uint64_t)0;
        bad += !good;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* kernels and the reverting function (Sec. III-A)                           */
/* ------------------------------------------------------------------------ */
static const double ORC_SQRT3 = 1.7320508075688772935;

/* k(r) with k(0) = 1 */
static double orc_kernel(const orc_params *p, double r)
{
    if (p->kernel == 0) {
        double a = ORC_SQRT3 * r / p->l;
        return (1.0 + a) * exp(-a);
    }
    return exp(-r * r / (2.0 * p->l * p->l));
}

/* grad_x k(|x - xi|) = coef * (x - xi) */
static double orc_kernel_grad_coef(const orc_params *p, double r)
{
    if (p->kernel == 0) {
        /* d/dr (1+ar)e^{-ar} = -a^2 r e^{-ar}; divided by r */
        double a = ORC_SQRT3 / p->l;
        return -a * a * exp(-a * r);
    }
    return -orc_kernel(p, r) / (p->l * p->l);
}

/* phi(t) = t - log(1 + t) >= 0, increasing for t > 0.  Below t = 0.1 the
 * subtraction would cancel, so the alternating series sum_{k>=2} (-t)^k / k
 * (|terms| fall by 10x per step) is summed instead. */
static double orc_phi(double t)
{
    if (t >= 0.1) return t - log1p(t);
    {
        double s = 0.0, pw = t * t;
        for (int k = 2; k <= 24; ++k) {
            s += ((k & 1) ? -pw : pw) / (double)k;
            pw *= t;
        }
        return s;
    }
}

/* Matern-3/2 reverting: the t >= 0 with (1 + t) e^{-t} = o, o in (0, 1].
 * Taking logs, t - log(1 + t) = -log(o); the left side rises strictly from 0,
 * so the root is unique.  -log(o) is formed as -log1p(o - 1) near o = 1
 * (o - 1 is exact there).  Safeguarded Newton: the bracket [lo, hi] always
 * holds the root and a step leaving it is replaced by bisection (Press et
 * al., rtsafe). */
double orc_matern_t(double o)
{
    double y, lo = 0.0, hi = 1.0, t;
    if (!(o < 1.0)) return 0.0;
    y = o > 0.5 ? -log1p(o - 1.0) : -log(o);
    while (orc_phi(hi) < y) hi *= 2.0;
    t = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double f = orc_phi(t) - y;           /* increasing in t */
        double fp = t / (1.0 + t);
        double tn;
        if (f < 0.0) lo = t; else hi = t;
        if (fp > 0.0) tn = t - f / fp; else tn = 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (fabs(tn - t) <= 1e-17 * t) { t = tn; break; }
        t = tn;
        if (hi - lo <= 1e-17 * t) break;
    }
    return t;
}

/* Eq. (3) and the derivative used in Eq. (4): d = r(o), Lambda = dr/do. */
void orc_revert(const orc_params *p, double o, double *d, double *lam)
{
    if (p->kernel == 0) {
        double t = orc_matern_t(o);
        double c = p->l / ORC_SQRT3;
        *d = c * t;
        /* dt/do = 1 / (d/dt (1+t)e^{-t}) = -e^{t} / t */
        *lam = -c * exp(t) / t;
    } else {
        double g = sqrt(-2.0 * log(o));
        *d = p->l * g;
        *lam = -p->l / (o * g);
    }
}

/* ------------------------------------------------------------------------ */
/* Cholesky of an n x n symmetric matrix (row-major, lower triangle used).   */
/* Returns 1 if every pivot exceeds 1e-10 times its diagonal entry.          */
/* ------------------------------------------------------------------------ */
int orc_cholesky(double *A, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 1e-10 * A[j * n + j])) return 0;
        double ljj = sqrt(d);
        A[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / ljj;
        }
        for (int64_t k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
    }
    return 1;
}

/* solve L y = b in place (forward substitution) */
static void orc_forward(const double *L, int64_t n, double *b)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* solve L^T x = b in place (back substitution) */
static void orc_backward(const double *L, int64_t n, double *b)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* the local GPs: one per leaf cluster (Sec. IV-A)                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_params p;
    int64_t nclusters, npoints, nonpd, skipped;
    uint64_t *ckey;   /* [nclusters] ascending */
    int64_t *off;     /* [nclusters + 1] */
    float *pts;       /* [npoints][3] training points, cluster after cluster */
    double *alpha;    /* [npoints]  (K + s^2 I)^{-1} 1 */
    int64_t *loff;    /* [nclusters] offset of the cluster's n*n factor */
    double *L;        /* dense row-major Cholesky factors */
    uint8_t *pd;      /* [nclusters] */
    double *cprop;    /* [npoints] surface property of each training point, or NULL */
    double *beta;     /* [npoints] (K + s^2 I)^{-1} c (Eq. (6)), or NULL */
} orc_model;

typedef struct { uint64_t key; uint64_t sub; int64_t src; } orc_item;

static int orc_item_cmp(const void *a, const void *b)
{
    const orc_item *x = (const orc_item *)a, *y = (const orc_item *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->sub != y->sub) return x->sub < y->sub ? -1 : 1;
    if (x->src != y->src) return x->src < y->src ? -1 : 1;
    return 0;
}

static int orc_u64_cmp(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

void orc_free(orc_model *m)
{
    if (!m) return;
    free(m->ckey); free(m->off); free(m->pts); free(m->alpha);
    free(m->loff); free(m->L); free(m->pd); free(m->cprop); free(m->beta); free(m);
}

/* cell coordinates of a point for cluster selection, consistent with the
 * cluster keys: raw mode floor(x / cell); voxel mode floor_div(voxel, 8) */
static int orc_cell_of(const orc_params *p, const float *x, int64_t c[3])
{
    for (int a = 0; a < 3; ++a) {
        if (p->voxel > 0.0) {
            int64_t v;
            if (!orc_floor_coord(x[a], p->voxel, &v)) return 0;
            c[a] = orc_floor_div(v, 8);
        } else {
            if (!orc_floor_coord(x[a], p->cell, &c[a])) return 0;
        }
    }
    return 1;
}

/* prop (may be NULL): a surface property per input point (intensity,
 * colour channel).  The property of a training point is that of its raw
 * points: in voxel mode their mean, summed in FP64 in input order; in raw
 * mode the point's own.  The property GP of each cluster shares the kernel
 * matrix and noise of the distance GP, so beta = (K + s^2 I)^{-1} c is a
 * second right-hand side on the same factor (Eq. (6)). */
orc_model *orc_train_prop(const orc_params *prm, const float *xyz, const float *prop,
                          int64_t n, int nthreads)
{
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    orc_item *it = (orc_item *)malloc(sizeof(orc_item) * (size_t)(n > 0 ? n : 1));
    int64_t cnt = 0;
    m->p = *prm;
    /* 1. keys (voxel mode: unique voxel centres are the training points) */
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        const float *x = xyz + 3 * i;
        if (prm->voxel > 0.0) {
            if (!(orc_floor_coord(x[0], prm->voxel, &c[0]) &&
                  orc_floor_coord(x[1], prm->voxel, &c[1]) &&
                  orc_floor_coord(x[2], prm->voxel, &c[2]))) { m->skipped++; continue; }
            it[cnt].key = orc_pack(orc_floor_div(c[0], 8), orc_floor_div(c[1], 8),
                                   orc_floor_div(c[2], 8));
            it[cnt].sub = orc_pack(c[0], c[1], c[2]);
        } else {
            if (!(orc_floor_coord(x[0], prm->cell, &c[0]) &&
                  orc_floor_coord(x[1], prm->cell, &c[1]) &&
                  orc_floor_coord(x[2], prm->cell, &c[2]))) { m->skipped++; continue; }
            it[cnt].key = orc_pack(c[0], c[1], c[2]);
            it[cnt].sub = (uint64_t)i;   /* members keep input order */
        }
        it[cnt].src = i;
        cnt++;
    }
    /* 2. order by (cluster key, member key, input index); voxel mode drops
     * duplicates, keeping the mean property of each voxel's raw points */
    qsort(it, (size_t)cnt, sizeof(orc_item), orc_item_cmp);
    if (prop) m->cprop = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    if (prm->voxel > 0.0 && cnt > 0) {
        int64_t w = 0;
        for (int64_t i = 0; i < cnt;) {
            int64_t e = i + 1;
            double sum = prop ? (double)prop[it[i].src] : 0.0;
            while (e < cnt && it[e].sub == it[i].sub) {
                if (prop) sum += (double)prop[it[e].src];
                e++;
            }
            if (prop) m->cprop[w] = sum / (double)(e - i);
            it[w++] = it[i];
            i = e;
        }
        cnt = w;
    } else if (prop) {
        for (int64_t i = 0; i < cnt; ++i) m->cprop[i] = (double)prop[it[i].src];
    }
    m->npoints = cnt;
    m->pts = (float *)malloc(sizeof(float) * 3 * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t i = 0; i < cnt; ++i) {
        if (prm->voxel > 0.0) {
            int64_t c[3];
            orc_unpack(it[i].sub, c);
            for (int a = 0; a < 3; ++a)
                m->pts[3 * i + a] = (float)(((double)c[a] + 0.5) * prm->voxel);
        } else {
            for (int a = 0; a < 3; ++a) m->pts[3 * i + a] = xyz[3 * it[i].src + a];
        }
    }
    /* 3. clusters = runs of equal cluster key */
    m->nclusters = 0;
    for (int64_t i = 0; i < cnt; ++i)
        if (i == 0 || it[i].key != it[i - 1].key) m->nclusters++;
    m->ckey = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m->nclusters + 1));
    m->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m->nclusters + 1));
    {
        int64_t c = 0;
        for (int64_t i = 0; i < cnt; ++i)
            if (i == 0 || it[i].key != it[i - 1].key) {
                m->ckey[c] = it[i].key;
                m->off[c] = i;
                c++;
            }
        m->off[m->nclusters] = cnt;
    }
    free(it);
    /* 4. train each cluster: A = K + s^2 I, L = chol(A), alpha = A^{-1} 1 */
    m->loff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m->nclusters + 1));
    {
        int64_t tot = 0;
        for (int64_t c = 0; c < m->nclusters; ++c) {
            int64_t nc = m->off[c + 1] - m->off[c];
            m->loff[c] = tot;
            tot += nc * nc;
        }
        m->L = (double *)malloc(sizeof(double) * (size_t)(tot > 0 ? tot : 1));
    }
    m->alpha = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    if (prop) m->beta = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    m->pd = (uint8_t *)malloc((size_t)(m->nclusters + 1));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < m->nclusters; ++c) {
        int64_t o = m->off[c], nc = m->off[c + 1] - o;
        double *A = m->L + m->loff[c];
        const float *P = m->pts + 3 * o;
        for (int64_t i = 0; i < nc; ++i)
            for (int64_t j = 0; j < nc; ++j) {
                double dx = (double)P[3 * i] - (double)P[3 * j];
                double dy = (double)P[3 * i + 1] - (double)P[3 * j + 1];
                double dz = (double)P[3 * i + 2] - (double)P[3 * j + 2];
                A[i * nc + j] = orc_kernel(&m->p, sqrt(dx * dx + dy * dy + dz * dz));
            }
        for (int64_t i = 0; i < nc; ++i) A[i * nc + i] += m->p.s * m->p.s;
        m->pd[c] = (uint8_t)orc_cholesky(A, nc);
        for (int64_t i = 0; i < nc; ++i) m->alpha[o + i] = 1.0;
        if (m->pd[c]) {
            orc_forward(A, nc, m->alpha + o);
            orc_backward(A, nc, m->alpha + o);
        } else {
            for (int64_t i = 0; i < nc; ++i) m->alpha[o + i] = 0.0;
        }
        if (m->beta) {
            /* Eq. (6): the property right-hand side on the same factor */
            for (int64_t i = 0; i < nc; ++i) m->beta[o + i] = m->pd[c] ? m->cprop[o + i] : 0.0;
            if (m->pd[c]) {
                orc_forward(A, nc, m->beta + o);
                orc_backward(A, nc, m->beta + o);
            }
        }
    }
    m->nonpd = 0;
    for (int64_t c = 0; c < m->nclusters; ++c) m->nonpd += !m->pd[c];
    return m;
}

orc_model *orc_train(const orc_params *prm, const float *xyz, int64_t n,
                     int nthreads)
{
    return orc_train_prop(prm, xyz, NULL, n, nthreads);
}

/* training-point properties and beta of a model trained with properties */
int orc_model_props(const orc_model *m, double *cprop, double *beta)
{
    if (!m->beta) return 0;
    memcpy(cprop, m->cprop, sizeof(double) * (size_t)m->npoints);
    memcpy(beta, m->beta, sizeof(double) * (size_t)m->npoints);
    return 1;
}

void orc_model_sizes(const orc_model *m, int64_t out[4])
{
    out[0] = m->nclusters; out[1] = m->npoints; out[2] = m->nonpd; out[3] = m->skipped;
}

void orc_model_export(const orc_model *m, uint64_t *ckey, int64_t *off,
                      float *pts, double *alpha, uint8_t *pd)
{
    memcpy(ckey, m->ckey, sizeof(uint64_t) * (size_t)m->nclusters);
    memcpy(off, m->off, sizeof(int64_t) * (size_t)(m->nclusters + 1));
    memcpy(pts, m->pts, sizeof(float) * 3 * (size_t)m->npoints);
    memcpy(alpha, m->alpha, sizeof(double) * (size_t)m->npoints);
    memcpy(pd, m->pd, (size_t)m->nclusters);
}

/* factor of one cluster (dense n x n lower, row-major) */
void orc_model_factor(const orc_model *m, int64_t c, double *out)
{
    int64_t nc = m->off[c + 1] - m->off[c];
    memcpy(out, m->L + m->loff[c], sizeof(double) * (size_t)(nc * nc));
}

static int64_t orc_find(const orc_model *m, uint64_t key)
{
    int64_t lo = 0, hi = m->nclusters - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (m->ckey[mid] == key) return mid;
        if (m->ckey[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* cluster selection for one query                                           */
/* ------------------------------------------------------------------------ */
#define ORC_MAXSEL 64

static int orc_select(const orc_model *m, const float *x, int64_t *sel)
{
    const orc_params *p = &m->p;
    int64_t c[3];
    int ns = 0;
    if (!orc_cell_of(p, x, c)) return 0;
    if (p->selection == 0) {
        /* the cell of the query and its 26 neighbours, ascending key; a
         * neighbour outside the key range holds no cluster (and has no key) */
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t n3[3] = {c[0] + dx, c[1] + dy, c[2] + dz}, k;
                    int inr = 1;
                    for (int a = 0; a < 3; ++a)
                        if (n3[a] < -ORC_KEY_BIAS || n3[a] >= ORC_KEY_BIAS) inr = 0;
                    if (!inr) continue;
                    k = orc_find(m, orc_pack(n3[0], n3[1], n3[2]));
                    if (k >= 0 && m->pd[k] && m->off[k + 1] > m->off[k]) sel[ns++] = k;
                }
        return ns;
    }
    /* Q nearest clusters by distance from the query to the cell centre,
     * ties to the smaller key; brute force over all clusters */
    {
        int q = p->knn_q < ORC_MAXSEL ? p->knn_q : ORC_MAXSEL;
        double bd[ORC_MAXSEL];
        double edge = p->voxel > 0.0 ? 8.0 * p->voxel : p->cell;
        for (int64_t k = 0; k < m->nclusters; ++k) {
            int64_t cc[3];
            double d2 = 0.0;
            if (!m->pd[k] || m->off[k + 1] == m->off[k]) continue;
            orc_unpack(m->ckey[k], cc);
            for (int a = 0; a < 3; ++a) {
                double ctr = ((double)cc[a] + 0.5) * edge;
                double dd = (double)x[a] - ctr;
                d2 += dd * dd;
            }
            /* insertion into the sorted list of the best q */
            if (ns < q || d2 < bd[ns - 1]) {
                int pos = ns < q ? ns : q - 1;
                if (ns < q) ns++;
                while (pos > 0 && d2 < bd[pos - 1]) {
                    bd[pos] = bd[pos - 1]; sel[pos] = sel[pos - 1]; pos--;
                }
                bd[pos] = d2; sel[pos] = k;
            }
        }
        /* evaluate in ascending key (= ascending cluster index) order */
        for (int i = 1; i < ns; ++i) {
            int64_t v = sel[i];
            int j = i;
            while (j > 0 && sel[j - 1] > v) { sel[j] = sel[j - 1]; j--; }
            sel[j] = v;
        }
        return ns;
    }
}

/* ------------------------------------------------------------------------ */
/* one (query, cluster) pair: Eq. (1), (2), (5), then (3), (4)               */
/* ------------------------------------------------------------------------ */
typedef struct { double o, u, d, g[3], v, c; } orc_pair;

static void orc_eval_pair(const orc_model *m, int64_t c, const double x[3],
                          double *kbuf, orc_pair *r)
{
    const orc_params *p = &m->p;
    int64_t o = m->off[c], nc = m->off[c + 1] - o;
    const float *P = m->pts + 3 * o;
    const double *L = m->L + m->loff[c];
    double occ = 0.0, go[3] = {0.0, 0.0, 0.0}, ss = 0.0, cp = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        double dx[3], rr;
        for (int a = 0; a < 3; ++a) dx[a] = x[a] - (double)P[3 * i + a];
        rr = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        kbuf[i] = orc_kernel(p, rr);
        occ += m->alpha[o + i] * kbuf[i];                 /* Eq. (1) */
        if (m->beta) cp += m->beta[o + i] * kbuf[i];      /* Eq. (6) */
        {
            double gc = m->alpha[o + i] * orc_kernel_grad_coef(p, rr);
            for (int a = 0; a < 3; ++a) go[a] += gc * dx[a];  /* Eq. (5) */
        }
    }
    /* Eq. (2) with the standard GP posterior sign (minus): the paper prints
     * a plus, which would make the posterior exceed the prior k(x,x) = 1. */
    orc_forward(L, nc, kbuf);
    for (int64_t i = 0; i < nc; ++i) ss += kbuf[i] * kbuf[i];
    r->u = 1.0 - ss;
    if (r->u < 0.0) r->u = 0.0;
    if (r->u > 1.0) r->u = 1.0;
    r->o = occ;
    r->c = cp;
    {
        /* footnote 1: the occupancy is capped before reverting */
        double oc = occ, d, lam;
        if (oc < p->occ_min) oc = p->occ_min;
        if (oc > p->occ_max) oc = p->occ_max;
        orc_revert(p, oc, &d, &lam);                   /* Eq. (3) */
        r->d = d;
        r->v = lam * lam * r->u;                       /* Eq. (4) */
        /* chain rule on the returned distance r(clamp(o)): below the lower
         * cap that distance is the constant r(occ_min), so its gradient is
         * zero; at the upper cap Lambda(occ_max) grad o keeps the direction
         * of the surface normal (the cap only guards the singularity of r
         * at o = 1) */
        for (int a = 0; a < 3; ++a) r->g[a] = occ < p->occ_min ? 0.0 : lam * go[a];
    }
}

/* ------------------------------------------------------------------------ */
/* sign of the distance: the sensor side of the nearest training point        */
/* (Sec. IV overview: the sign comes from the sensor origin and the points)   */
/* ------------------------------------------------------------------------ */
#define ORC_U32 5.9604644775390625e-08 /* 2^-24, unit roundoff of FP32 */

/* (x - p).(o - p) in FP64 and the sum of |products| that bounds its rounding */
static double orc_side(const float *x, const float *p, const float *o, double *mag)
{
    double dot = 0.0, m = 0.0;
    for (int a = 0; a < 3; ++a) {
        double t = ((double)x[a] - (double)p[a]) * ((double)o[a] - (double)p[a]);
        dot += t;
        m += fabs(t);
    }
    *mag = m;
    return dot;
}

static double orc_r2(const float *x, const float *p)
{
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = (double)x[a] - (double)p[a];
        r2 += d * d;
    }
    return r2;
}

/* Returns -1 if the query lies behind its nearest training point as seen
 * from the origin, +1 otherwise, 0 if no point is selected.  *tie is set when
 * FP32 arithmetic could decide differently.  Bounds: an FP32 coordinate
 * difference has relative error at most u = 2^-24, and a three-term sum of
 * products adds three roundings, so an FP32 squared distance or side product
 * is within 6u of the exact value (times r^2, or times the sum of |products|);
 * 8u is used. */
static int orc_sign(const orc_model *m, const int64_t *sel, int ns, const float *x,
                    const float *origin, uint8_t *tie)
{
    const float *best = NULL;
    double b2 = INFINITY, mag, dot, side;
    int t = 0;
    /* the exact nearest point; strict < keeps the first in ascending
     * cluster key and member order */
    for (int s = 0; s < ns; ++s)
        for (int64_t i = m->off[sel[s]]; i < m->off[sel[s] + 1]; ++i) {
            double r2 = orc_r2(x, m->pts + 3 * i);
            if (r2 < b2) { b2 = r2; best = m->pts + 3 * i; }
        }
    if (!best) { *tie = 0; return 0; }
    dot = orc_side(x, best, origin, &mag);
    side = dot >= 0.0 ? 1.0 : -1.0;
    if (fabs(dot) < 8.0 * ORC_U32 * mag) t = 1;
    /* any candidate FP32 could take for the nearest that lies on the other
     * side (or on an undecidable side) */
    for (int s = 0; s < ns && !t; ++s)
        for (int64_t i = m->off[sel[s]]; i < m->off[sel[s] + 1] && !t; ++i) {
            const float *p = m->pts + 3 * i;
            double r2, d2, m2;
            if (p == best) continue;
            r2 = orc_r2(x, p);
            if (r2 - b2 > 8.0 * ORC_U32 * (r2 + b2)) continue;
            d2 = orc_side(x, p, origin, &m2);
            if ((d2 >= 0.0 ? 1.0 : -1.0) != side || fabs(d2) < 8.0 * ORC_U32 * m2) t = 1;
        }
    *tie = (uint8_t)t;
    return side > 0.0 ? 1 : -1;
}

/* ------------------------------------------------------------------------ */
/* query: selection, per-pair inference, Eq. (10), sign                      */
/* ------------------------------------------------------------------------ */
/* The closest node (the pair of smallest distance) is an argmin that an FP32
 * evaluation can take differently when two pairs lie close.  alt (may be
 * NULL) reports, per query, whether the second-closest pair lies within
 * ORC_NODE_TIE of the closest (alt->tie), and the results the query would
 * have with that pair as the closest node (distance and gradient with the
 * query's sign, variance, property and its variance) -- the other valid
 * answer of the closest-node rule there. */
#define ORC_NODE_TIE 2e-4
typedef struct {
    uint8_t *tie;
    double *dist, *grad, *var, *prop, *prop_var;
} orc_alt;

/* prop, prop_var (may be NULL; need a model trained with properties): the
 * surface property (Eq. (6)) and its variance.  The property GP has the
 * distance GP's kernel and noise, so its posterior variance is the latent
 * variance u of Eq. (2).  Both are combined over the selected clusters like
 * the distance variance: with the smooth-minimum weights of the distances,
 * or from the closest node alone.  An invalid query gives prop 0 and
 * prop_var infinity. */
void orc_query_prop(const orc_model *m, const float *q, int64_t nq,
                    const float *origin, double *dist, double *grad, double *var,
                    uint8_t *valid, double *aux, uint8_t *tie, double *prop,
                    double *prop_var, const orc_alt *alt, int nthreads)
{
    const orc_params *p = &m->p;
    int64_t maxn = 1;
    for (int64_t c = 0; c < m->nclusters; ++c)
        if (m->off[c + 1] - m->off[c] > maxn) maxn = m->off[c + 1] - m->off[c];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *kbuf = (double *)malloc(sizeof(double) * (size_t)maxn);
        orc_pair *pr = (orc_pair *)malloc(sizeof(orc_pair) * ORC_MAXSEL);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
        for (int64_t j = 0; j < nq; ++j) {
            const float *xf = q + 3 * j;
            double x[3] = {(double)xf[0], (double)xf[1], (double)xf[2]};
            int64_t sel[ORC_MAXSEL];
            int ns = orc_select(m, xf, sel);
            int64_t ntot = 0;
            if (tie) tie[j] = 0;
            if (alt) alt->tie[j] = 0;
            if (ns == 0) {
                dist[j] = INFINITY; var[j] = INFINITY; valid[j] = 0;
                if (prop) prop[j] = 0.0;
                if (prop_var) prop_var[j] = INFINITY;
                for (int a = 0; a < 3; ++a) grad[3 * j + a] = 0.0;
                if (aux) { aux[3 * j] = 0.0; aux[3 * j + 1] = 0.0; aux[3 * j + 2] = 0.0; }
                continue;
            }
            for (int s = 0; s < ns; ++s) {
                orc_eval_pair(m, sel[s], x, kbuf, &pr[s]);
                ntot += m->off[sel[s] + 1] - m->off[sel[s]];
            }
            {
                /* Eq. (10) read as a smooth MINIMUM: the printed exponent
                 * exp(+lambda d) with large lambda selects the maximum; the
                 * text calls it a smooth minimum, so the weights are
                 * exp(-lambda (d_q - d_min)).  Subtracting d_min leaves the
                 * ratio unchanged. */
                int amin = 0;
                double dmin, W = 0.0, D = 0.0, V = 0.0, G[3] = {0, 0, 0}, Cp = 0.0, Cw = 0.0;
                for (int s = 1; s < ns; ++s) if (pr[s].d < pr[amin].d) amin = s;
                dmin = pr[amin].d;
                if (p->combine == 1) {
                    D = pr[amin].d; V = pr[amin].v;
                    Cp = pr[amin].c; Cw = pr[amin].u;
                    for (int a = 0; a < 3; ++a) G[a] = pr[amin].g[a];
                } else {
                    for (int s = 0; s < ns; ++s) {
                        double w = exp(-p->lambda * (pr[s].d - dmin));
                        W += w; D += w * pr[s].d; V += w * pr[s].v;
                        Cp += w * pr[s].c; Cw += w * pr[s].u;
                        for (int a = 0; a < 3; ++a) G[a] += w * pr[s].g[a];
                    }
                    D /= W; V /= W; Cp /= W; Cw /= W;
                    if (p->grad_mode == 1) {
                        /* "directly average" the Q gradients */
                        for (int a = 0; a < 3; ++a) {
                            G[a] = 0.0;
                            for (int s = 0; s < ns; ++s) G[a] += pr[s].g[a];
                            G[a] /= (double)ns;
                        }
                    } else {
                        for (int a = 0; a < 3; ++a) G[a] /= W;
                    }
                }
                {
                    double sg = 1.0;
                    int a2 = -1;
                    if (origin) {
                        uint8_t t = 0;
                        if (orc_sign(m, sel, ns, xf, origin, &t) < 0) {
                            sg = -1.0;
                            D = -D;
                            for (int a = 0; a < 3; ++a) G[a] = -G[a];
                        }
                        if (tie) tie[j] = t;
                    }
                    for (int s = 0; s < ns; ++s)
                        if (s != amin && (a2 < 0 || pr[s].d < pr[a2].d)) a2 = s;
                    if (alt && a2 >= 0 && pr[a2].d - pr[amin].d <= ORC_NODE_TIE) {
                        alt->tie[j] = 1;
                        alt->dist[j] = sg * pr[a2].d;
                        alt->var[j] = pr[a2].v;
                        for (int a = 0; a < 3; ++a) alt->grad[3 * j + a] = sg * pr[a2].g[a];
                        alt->prop[j] = pr[a2].c;
                        alt->prop_var[j] = pr[a2].u;
                    }
                }
                dist[j] = D; var[j] = V; valid[j] = 1;
                if (prop) prop[j] = Cp;
                if (prop_var) prop_var[j] = Cw;
                for (int a = 0; a < 3; ++a) grad[3 * j + a] = G[a];
                if (aux) {
                    aux[3 * j] = pr[amin].o;
                    aux[3 * j + 1] = pr[amin].u;
                    aux[3 * j + 2] = (double)ntot;
                }
            }
        }
        free(kbuf);
        free(pr);
    }
}

void orc_query(const orc_model *m, const float *q, int64_t nq,
               const float *origin, double *dist, double *grad, double *var,
               uint8_t *valid, double *aux, uint8_t *tie, int nthreads)
{
    orc_query_prop(m, q, nq, origin, dist, grad, var, valid, aux, tie, NULL, NULL, NULL, nthreads);
}

/* ------------------------------------------------------------------------ */
/* test points for fusion: global-grid voxels within a ball (in voxels) of   */
/* the cell of some training point.  Stand-in for the ray-cast test points   */
/* of Sec. IV-B: a band around the observed surface, one test per voxel.     */
/* ------------------------------------------------------------------------ */
static int64_t orc_band_radius(const orc_params *p)
{
    return (int64_t)floor(p->fuse_band / p->fuse_voxel + 1e-9);
}

int64_t orc_test_points(const orc_model *m, uint64_t *out, int64_t cap)
{
    const orc_params *p = &m->p;
    int64_t R = orc_band_radius(p), nofs = 0, n = 0;
    int64_t (*ofs)[3];
    uint64_t *all;
    for (int64_t a = -R; a <= R; ++a)
        for (int64_t b = -R; b <= R; ++b)
            for (int64_t c = -R; c <= R; ++c)
                if (a * a + b * b + c * c <= R * R) nofs++;
    ofs = malloc(sizeof(*ofs) * (size_t)nofs);
    nofs = 0;
    for (int64_t a = -R; a <= R; ++a)
        for (int64_t b = -R; b <= R; ++b)
            for (int64_t c = -R; c <= R; ++c)
                if (a * a + b * b + c * c <= R * R) {
                    ofs[nofs][0] = a; ofs[nofs][1] = b; ofs[nofs][2] = c; nofs++;
                }
    all = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m->npoints * nofs + 1));
    for (int64_t i = 0; i < m->npoints; ++i) {
        int64_t c[3];
        if (!(orc_floor_coord(m->pts[3 * i], p->fuse_voxel, &c[0]) &&
              orc_floor_coord(m->pts[3 * i + 1], p->fuse_voxel, &c[1]) &&
              orc_floor_coord(m->pts[3 * i + 2], p->fuse_voxel, &c[2]))) continue;
        for (int64_t k = 0; k < nofs; ++k) {
            int64_t v[3] = {c[0] + ofs[k][0], c[1] + ofs[k][1], c[2] + ofs[k][2]};
            int okv = 1;
            for (int a = 0; a < 3; ++a)
                if (v[a] < -ORC_KEY_BIAS || v[a] >= ORC_KEY_BIAS) okv = 0;
            if (okv) all[n++] = orc_pack(v[0], v[1], v[2]);
        }
    }
    qsort(all, (size_t)n, sizeof(uint64_t), orc_u64_cmp);
    {
        int64_t w = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || all[i] != all[i - 1]) {
                if (out && w < cap) out[w] = all[i];
                w++;
            }
        n = w;
    }
    free(all);
    free(ofs);
    return n;
}

/* centre of a global voxel, rounded once to FP32 */
void orc_voxel_centres(const uint64_t *keys, int64_t n, double h, float *xyz)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        orc_unpack(keys[i], c);
        for (int a = 0; a < 3; ++a) xyz[3 * i + a] = (float)(((double)c[a] + 0.5) * h);
    }
}

/* ------------------------------------------------------------------------ */
/* global grid: a sorted array of (key, D, V, stamp), Eq. (7)-(8)            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    uint64_t *key;
    double *D, *V;
    uint32_t *stamp;
    uint8_t *tie;     /* some fused observation had a sign near-tie */
    double *C, *W;    /* fused surface property and its variance (or weight);
                         NaN where no property has been fused; NULL until a
                         frame with properties is merged */
} orc_map;

orc_map *orc_map_new(void) { return (orc_map *)calloc(1, sizeof(orc_map)); }

void orc_map_free(orc_map *g)
{
    if (!g) return;
    free(g->key); free(g->D); free(g->V); free(g->stamp); free(g->tie);
    free(g->C); free(g->W); free(g);
}

int64_t orc_map_size(const orc_map *g) { return g->n; }

void orc_map_export(const orc_map *g, uint64_t *key, double *D, double *V,
                    uint32_t *stamp, uint8_t *tie)
{
    memcpy(key, g->key, sizeof(uint64_t) * (size_t)g->n);
    memcpy(D, g->D, sizeof(double) * (size_t)g->n);
    memcpy(V, g->V, sizeof(double) * (size_t)g->n);
    memcpy(stamp, g->stamp, sizeof(uint32_t) * (size_t)g->n);
    if (tie) memcpy(tie, g->tie, (size_t)g->n);
}

/* Merge one frame of observations (sorted unique keys) into the map.
 * An absent voxel takes the observation (the V_{i-1} = infinity limit of
 * Eq. (8)); a present one is updated by Eq. (7)-(8):
 *   D <- (V d + v D) / (V + v),  V <- (1/V + 1/v)^{-1} = V v / (V + v).
 * Observations with a non-finite or non-positive variance are skipped.
 *
 * rule 1 is the TSDF-style alternative of Eq. (9): the observation's weight
 * is w = 1 - v, V accumulates the weights, and
 *   D <- (w d + V D) / (V + w),  V <- V + w;
 * an absent voxel takes (d, w).  1 - v can be negative (v is a variance in
 * m^2); observations with w <= 0 carry no weight and are skipped.
 *
 * tie (may be NULL) marks observations whose sign was a near-tie; the mark
 * stays on the voxel. */
/* Surface properties (c, cv may be NULL): Sec. IV-C fuses them with the
 * same expressions, using their own variance cv in place of v.  A property
 * observation rides on its voxel's distance observation (a voxel skipped
 * for the distance skips its property too); one whose variance (rule 0) or
 * weight 1 - cv (rule 1) is not positive and finite leaves the voxel's
 * property unchanged.  A voxel with no property yet (NaN) takes the
 * observation: (c, cv), or (c, 1 - cv) under rule 1. */
int64_t orc_map_merge_prop(orc_map *g, const uint64_t *k, const double *d,
                           const double *v, const uint8_t *ok, const uint8_t *tie,
                           const double *c, const double *cv,
                           int64_t n, uint32_t frame, int rule)
{
    int64_t cap = g->n + n, i = 0, j = 0, w = 0, skipped = 0;
    const int props = c != NULL || g->C != NULL;
    double *nC = NULL, *nW = NULL;
    if (props) {
        nC = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
        nW = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    }
    uint64_t *nk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1));
    double *nD = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    double *nV = (double *)malloc(sizeof(double) * (size_t)(cap + 1));
    uint32_t *ns = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 1));
    uint8_t *nt = (uint8_t *)malloc((size_t)(cap + 1));
    while (i < g->n || j < n) {
        int use_obs;
        if (j < n && !(ok[j] && isfinite(v[j]) && isfinite(d[j]) &&
                       (rule == 1 ? 1.0 - v[j] > 0.0 : v[j] > 0.0))) {
            skipped += ok[j] ? 1 : 0;
            j++;
            continue;
        }
        if (j >= n) use_obs = 0;
        else if (i >= g->n) use_obs = 1;
        else use_obs = k[j] <= g->key[i];
        if (!use_obs) {
            nk[w] = g->key[i]; nD[w] = g->D[i]; nV[w] = g->V[i]; ns[w] = g->stamp[i];
            nt[w] = g->tie[i];
            if (props) {
                nC[w] = g->C ? g->C[i] : NAN;
                nW[w] = g->C ? g->W[i] : NAN;
            }
            i++; w++;
        } else if (i < g->n && k[j] == g->key[i]) {
            double Vp = g->V[i], Dp = g->D[i];
            nk[w] = k[j];
            if (props) {
                double Cp = g->C ? g->C[i] : NAN, Wp = g->C ? g->W[i] : NAN;
                nC[w] = Cp; nW[w] = Wp;
                if (c && isfinite(c[j]) && isfinite(cv[j]) &&
                    (rule == 1 ? 1.0 - cv[j] > 0.0 : cv[j] > 0.0)) {
                    double wt = rule == 1 ? 1.0 - cv[j] : cv[j];
                    if (isnan(Cp)) {
                        nC[w] = c[j]; nW[w] = wt;
                    } else if (rule == 1) {
                        nC[w] = (wt * c[j] + Wp * Cp) / (Wp + wt);
                        nW[w] = Wp + wt;
                    } else {
                        nC[w] = (Wp * c[j] + wt * Cp) / (Wp + wt);
                        nW[w] = (Wp * wt) / (Wp + wt);
                    }
                }
            }
            if (rule == 1) {
                double wt = 1.0 - v[j];
                nD[w] = (wt * d[j] + Vp * Dp) / (Vp + wt);
                nV[w] = Vp + wt;
            } else {
                nD[w] = (Vp * d[j] + v[j] * Dp) / (Vp + v[j]);
                nV[w] = (Vp * v[j]) / (Vp + v[j]);
            }
            ns[w] = frame;
            nt[w] = (uint8_t)(g->tie[i] | (tie ? tie[j] : 0));
            i++; j++; w++;
        } else {
            nk[w] = k[j]; nD[w] = d[j]; nV[w] = rule == 1 ? 1.0 - v[j] : v[j]; ns[w] = frame;
            nt[w] = tie ? tie[j] : 0;
            if (props) {
                nC[w] = NAN; nW[w] = NAN;
                if (c && isfinite(c[j]) && isfinite(cv[j]) &&
                    (rule == 1 ? 1.0 - cv[j] > 0.0 : cv[j] > 0.0)) {
                    nC[w] = c[j]; nW[w] = rule == 1 ? 1.0 - cv[j] : cv[j];
                }
            }
            j++; w++;
        }
    }
    free(g->key); free(g->D); free(g->V); free(g->stamp); free(g->tie);
    free(g->C); free(g->W);
    g->key = nk; g->D = nD; g->V = nV; g->stamp = ns; g->tie = nt; g->n = w;
    g->C = nC; g->W = nW;
    return skipped;
}

int64_t orc_map_merge(orc_map *g, const uint64_t *k, const double *d,
                      const double *v, const uint8_t *ok, const uint8_t *tie,
                      int64_t n, uint32_t frame, int rule)
{
    return orc_map_merge_prop(g, k, d, v, ok, tie, NULL, NULL, n, frame, rule);
}

/* fused properties in key order (NaN where none); 0 if the map has none */
int orc_map_export_prop(const orc_map *g, double *C, double *W)
{
    if (!g->C) return 0;
    memcpy(C, g->C, sizeof(double) * (size_t)g->n);
    memcpy(W, g->W, sizeof(double) * (size_t)g->n);
    return 1;
}

int64_t orc_test_points_ray(const orc_model *m, const orc_map *g, const float origin[3],
                            uint64_t *out, int64_t cap);

/* One frame of fusion against an already trained model: test points (the
 * band, or the ray-cast and normal voxels of Sec. IV-B against the map as it
 * is before this frame), signed query, merge.  Returns the number of test
 * points. */
int64_t orc_fuse(orc_map *g, const orc_model *m, const float origin[3],
                 uint32_t frame, int64_t *skipped, int nthreads)
{
    const int ray = m->p.tp_mode == 1;
    int64_t n = ray ? orc_test_points_ray(m, g, origin, NULL, 0) : orc_test_points(m, NULL, 0);
    uint64_t *k = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n + 1));
    float *x = (float *)malloc(sizeof(float) * 3 * (size_t)(n + 1));
    double *d = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *gr = (double *)malloc(sizeof(double) * 3 * (size_t)(n + 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    uint8_t *ok = (uint8_t *)malloc((size_t)(n + 1));
    uint8_t *tie = (uint8_t *)malloc((size_t)(n + 1));
    int64_t sk;
    if (ray) orc_test_points_ray(m, g, origin, k, n);
    else orc_test_points(m, k, n);
    orc_voxel_centres(k, n, m->p.fuse_voxel, x);
    {
        double *c = NULL, *cv = NULL;
        if (m->beta) {
            c = (double *)malloc(sizeof(double) * (size_t)(n + 1));
            cv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        }
        orc_query_prop(m, x, n, origin, d, gr, v, ok, NULL, tie, c, cv, NULL, nthreads);
        sk = orc_map_merge_prop(g, k, d, v, ok, tie, c, cv, n, frame, m->p.fuse_rule);
        free(c); free(cv);
    }
    if (skipped) *skipped = sk;
    free(k); free(x); free(d); free(gr); free(v); free(ok); free(tie);
    return n;
}

static int64_t orc_map_find(const orc_map *g, uint64_t key)
{
    int64_t lo = 0, hi = g->n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->key[mid] == key) return mid;
        if (g->key[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* ray-cast test points (Sec. IV-B): for every training voxel, the global    */
/* voxels on the ray from the sensor that the map already holds (previously  */
/* observed surface), the voxel of the measurement itself, and the voxels    */
/* along its surface normal up to normal_reach.                             */
/* ------------------------------------------------------------------------ */
/* The ray is walked in global-voxel units from the centre of the origin's
 * voxel O to the centre of the training point's voxel E, visiting every
 * voxel the segment passes through (a face-connected walk, the traversal of
 * Amanatides and Woo) in exact integer arithmetic: with A = |E - O| per
 * axis, the n-th boundary crossing on axis a lies at parameter
 * (2n + 1) / (2 A_a), so the next axis is the one with the smallest
 * (2 n_a + 1) / A_a, compared by cross-multiplication; equal parameters
 * (the segment through an edge or corner) step the lower axis first. */
static int orc_key_ok(const int64_t v[3])
{
    for (int a = 0; a < 3; ++a)
        if (v[a] < -ORC_KEY_BIAS || v[a] >= ORC_KEY_BIAS) return 0;
    return 1;
}

static int64_t orc_gcd(int64_t a, int64_t b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a;
}

/* candidate normal directions: the integer vectors with components in
 * [-2, 2], primitive (gcd 1) and canonical (first non-zero component
 * positive), in ascending lexicographic order of (x, y, z): 49 of them */
static int orc_normal_dirs(int64_t d[64][3])
{
    int n = 0;
    for (int64_t x = -2; x <= 2; ++x)
        for (int64_t y = -2; y <= 2; ++y)
            for (int64_t z = -2; z <= 2; ++z) {
                int64_t f = x != 0 ? x : (y != 0 ? y : z);
                if (f <= 0) continue;
                if (orc_gcd(orc_gcd(x, y), z) != 1) continue;
                d[n][0] = x; d[n][1] = y; d[n][2] = z; n++;
            }
    return n;
}

static int64_t orc_find_sorted(const uint64_t *a, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] == key) return mid;
        if (a[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* The surface normal of a training voxel is the direction of least spread
 * of the training voxels in the 5 x 5 x 5 block around it: among the
 * candidate directions d the one minimising d^T M d / |d|^2, with
 * M = N S2 - s1 s1^T (N^2 times the covariance of the integer offsets o:
 * N their count, s1 = sum o, S2 = sum o o^T), compared exactly in integers;
 * ties go to the first candidate.  Fewer than 3 neighbours: no normal. */
int64_t orc_test_points_ray(const orc_model *m, const orc_map *g, const float origin[3],
                            uint64_t *out, int64_t cap)
{
    const orc_params *p = &m->p;
    const int64_t R = (int64_t)floor(p->normal_reach / p->fuse_voxel + 1e-9);
    int64_t dirs[64][3];
    const int nd = orc_normal_dirs(dirs);
    int64_t O[3], n = 0, alloc = 1024;
    uint64_t *vk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m->npoints + 1));
    uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)alloc);
    int okO = orc_floor_coord(origin[0], p->fuse_voxel, &O[0]) &&
              orc_floor_coord(origin[1], p->fuse_voxel, &O[1]) &&
              orc_floor_coord(origin[2], p->fuse_voxel, &O[2]);
#define ORC_PUSH(key) do { if (n == alloc) { alloc *= 2; all = (uint64_t *)realloc(all, sizeof(uint64_t) * (size_t)alloc); } all[n++] = (key); } while (0)
    /* the training voxels (voxel mode: one training point per voxel) */
    for (int64_t i = 0; i < m->npoints; ++i) {
        int64_t c[3] = {0, 0, 0};
        orc_floor_coord(m->pts[3 * i], p->voxel, &c[0]);
        orc_floor_coord(m->pts[3 * i + 1], p->voxel, &c[1]);
        orc_floor_coord(m->pts[3 * i + 2], p->voxel, &c[2]);
        vk[i] = orc_pack(c[0], c[1], c[2]);
    }
    qsort(vk, (size_t)m->npoints, sizeof(uint64_t), orc_u64_cmp);
    for (int64_t i = 0; i < m->npoints && okO; ++i) {
        int64_t E[3], cv[3];
        const float *x = m->pts + 3 * i;
        if (!(orc_floor_coord(x[0], p->fuse_voxel, &E[0]) && orc_floor_coord(x[1], p->fuse_voxel, &E[1]) &&
              orc_floor_coord(x[2], p->fuse_voxel, &E[2]) && orc_floor_coord(x[0], p->voxel, &cv[0]) &&
              orc_floor_coord(x[1], p->voxel, &cv[1]) && orc_floor_coord(x[2], p->voxel, &cv[2]))) continue;
        /* the ray O -> E: previously observed voxels */
        {
            int64_t A[3], st[3], cnt[3] = {0, 0, 0}, cur[3] = {O[0], O[1], O[2]}, total = 0;
            for (int a = 0; a < 3; ++a) {
                int64_t dd = E[a] - O[a];
                A[a] = dd < 0 ? -dd : dd;
                st[a] = dd < 0 ? -1 : 1;
                total += A[a];
            }
            for (int64_t k = 0; k <= total; ++k) {
                if (k > 0) {
                    int best = -1;
                    for (int a = 0; a < 3; ++a) {
                        if (cnt[a] >= A[a]) continue;
                        if (best < 0 || (2 * cnt[a] + 1) * A[best] < (2 * cnt[best] + 1) * A[a]) best = a;
                    }
                    cur[best] += st[best];
                    cnt[best]++;
                }
                if (k < total && g && orc_map_find(g, orc_pack(cur[0], cur[1], cur[2])) >= 0)
                    ORC_PUSH(orc_pack(cur[0], cur[1], cur[2]));
            }
        }
        /* the measured voxel */
        ORC_PUSH(orc_pack(E[0], E[1], E[2]));
        /* the normal: least spread of the training voxels within +-2 */
        {
            int64_t N = 0, s1[3] = {0, 0, 0}, S2[3][3] = {{0}};
            for (int64_t a = -2; a <= 2; ++a)
                for (int64_t b = -2; b <= 2; ++b)
                    for (int64_t c = -2; c <= 2; ++c) {
                        int64_t v[3] = {cv[0] + a, cv[1] + b, cv[2] + c}, o[3] = {a, b, c};
                        if (!orc_key_ok(v) || orc_find_sorted(vk, m->npoints, orc_pack(v[0], v[1], v[2])) < 0)
                            continue;
                        N++;
                        for (int r = 0; r < 3; ++r) {
                            s1[r] += o[r];
                            for (int q = 0; q < 3; ++q) S2[r][q] += o[r] * o[q];
                        }
                    }
            if (N >= 3) {
                int64_t M[3][3], bn = 0, bd = 1;
                int best = -1;
                for (int r = 0; r < 3; ++r)
                    for (int q = 0; q < 3; ++q) M[r][q] = N * S2[r][q] - s1[r] * s1[q];
                for (int t = 0; t < nd; ++t) {
                    int64_t num = 0, den = 0;
                    for (int r = 0; r < 3; ++r) {
                        den += dirs[t][r] * dirs[t][r];
                        for (int q = 0; q < 3; ++q) num += dirs[t][r] * M[r][q] * dirs[t][q];
                    }
                    if (best < 0 || num * bd < bn * den) { best = t; bn = num; bd = den; }
                }
                for (int64_t k = -R; k <= R; ++k) {
                    int64_t v[3];
                    if (k == 0 || k * k * bd > R * R) continue;
                    for (int a = 0; a < 3; ++a) v[a] = E[a] + k * dirs[best][a];
                    if (orc_key_ok(v)) ORC_PUSH(orc_pack(v[0], v[1], v[2]));
                }
            }
        }
    }
#undef ORC_PUSH
    qsort(all, (size_t)n, sizeof(uint64_t), orc_u64_cmp);
    {
        int64_t w = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || all[i] != all[i - 1]) {
                if (out && w < cap) out[w] = all[i];
                w++;
            }
        n = w;
    }
    free(all);
    free(vk);
    return n;
}

/* Global query on the fused grid: trilinear interpolation of D over the
 * eight voxel centres around x and the analytic gradient of that
 * interpolant; valid only when all eight voxels exist.  (Stand-in for the
 * G-GPDF query of Sec. IV-D.) */
void orc_query_global(const orc_map *g, double h, const float *q, int64_t nq,
                      double *dist, double *grad, uint8_t *valid, uint8_t *tie)
{
    for (int64_t j = 0; j < nq; ++j) {
        double u[3], f[3], Dc[8];
        int64_t i0[3];
        int okq = 1;
        if (tie) tie[j] = 0;
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(q[3 * j + a])) { okq = 0; break; }
            u[a] = (double)q[3 * j + a] / h - 0.5;
            i0[a] = (int64_t)floor(u[a]);
            f[a] = u[a] - (double)i0[a];
            if (i0[a] < -ORC_KEY_BIAS || i0[a] + 1 >= ORC_KEY_BIAS) okq = 0;
        }
        for (int b = 0; b < 8 && okq; ++b) {
            int64_t k = orc_map_find(g, orc_pack(i0[0] + ((b >> 2) & 1),
                                                 i0[1] + ((b >> 1) & 1),
                                                 i0[2] + (b & 1)));
            if (k < 0) okq = 0;
            else {
                Dc[b] = g->D[k];
                if (tie && g->tie[k]) tie[j] = 1;
            }
        }
        if (!okq) {
            dist[j] = INFINITY; valid[j] = 0;
            grad[3 * j] = grad[3 * j + 1] = grad[3 * j + 2] = 0.0;
            continue;
        }
        {
            double D = 0.0, G[3] = {0.0, 0.0, 0.0};
            for (int b = 0; b < 8; ++b) {
                int bit[3] = {(b >> 2) & 1, (b >> 1) & 1, b & 1};
                double w[3], dw[3];
                for (int a = 0; a < 3; ++a) {
                    w[a] = bit[a] ? f[a] : 1.0 - f[a];
                    dw[a] = bit[a] ? 1.0 : -1.0;
                }
                D += w[0] * w[1] * w[2] * Dc[b];
                G[0] += dw[0] * w[1] * w[2] * Dc[b];
                G[1] += w[0] * dw[1] * w[2] * Dc[b];
                G[2] += w[0] * w[1] * dw[2] * Dc[b];
            }
            dist[j] = D; valid[j] = 1;
            for (int a = 0; a < 3; ++a) grad[3 * j + a] = G[a] / h;
        }
    }
}

/* Fused surface property at q: the same trilinear interpolation, of C;
 * valid only when all eight voxels exist and hold a property.  Invalid
 * queries give 0. */
void orc_query_global_prop(const orc_map *g, double h, const float *q, int64_t nq,
                           double *prop, uint8_t *valid)
{
    for (int64_t j = 0; j < nq; ++j) {
        double u[3], f[3], Cc[8];
        int64_t i0[3];
        int okq = g->C != NULL;
        for (int a = 0; a < 3 && okq; ++a) {
            if (!isfinite(q[3 * j + a])) { okq = 0; break; }
            u[a] = (double)q[3 * j + a] / h - 0.5;
            i0[a] = (int64_t)floor(u[a]);
            f[a] = u[a] - (double)i0[a];
            if (i0[a] < -ORC_KEY_BIAS || i0[a] + 1 >= ORC_KEY_BIAS) okq = 0;
        }
        for (int b = 0; b < 8 && okq; ++b) {
            int64_t k = orc_map_find(g, orc_pack(i0[0] + ((b >> 2) & 1),
                                                 i0[1] + ((b >> 1) & 1),
                                                 i0[2] + (b & 1)));
            if (k < 0 || isnan(g->C[k])) okq = 0;
            else Cc[b] = g->C[k];
        }
        if (!okq) { prop[j] = 0.0; valid[j] = 0; continue; }
        {
            double C = 0.0;
            for (int b = 0; b < 8; ++b) {
                double w0 = ((b >> 2) & 1) ? f[0] : 1.0 - f[0];
                double w1 = ((b >> 1) & 1) ? f[1] : 1.0 - f[1];
                double w2 = (b & 1) ? f[2] : 1.0 - f[2];
                C += w0 * w1 * w2 * Cc[b];
            }
            prop[j] = C; valid[j] = 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* zero crossings of the fused grid (Sec. IV-D): the surface points that the  */
/* marching cubes (Lorensen and Cline) place on the grid edges whose two      */
/* voxel centres carry distances of opposite sign, where the linear           */
/* interpolant of D along the edge is zero.  They train the global GPs        */
/* (G-GPDF, one GP per leaf of 8^3 voxels).                                   */
/* ------------------------------------------------------------------------ */
/* Edges from voxel a to its neighbour b = a + e_axis (axis x, y, z); a sign
 * change means (D_a < 0) != (D_b < 0).  The point lies at t = D_a / (D_a - D_b)
 * of the edge: coordinate (c_a + 1/2 + t) h on the edge's axis, (c + 1/2) h on
 * the others, each formed in FP64 and rounded once to FP32.  Order: ascending
 * key of a, then axis.  Returns the count; writes at most cap points. */
int64_t orc_zero_crossings(const orc_map *g, double h, float *out, int64_t cap)
{
    int64_t n = 0;
    for (int64_t i = 0; i < g->n; ++i) {
        int64_t c[3];
        orc_unpack(g->key[i], c);
        for (int a = 0; a < 3; ++a) {
            int64_t nb[3] = {c[0], c[1], c[2]}, j;
            double Da = g->D[i], Db, t;
            nb[a] += 1;
            if (nb[a] >= ORC_KEY_BIAS) continue;
            j = orc_map_find(g, orc_pack(nb[0], nb[1], nb[2]));
            if (j < 0) continue;
            Db = g->D[j];
            if ((Da < 0.0) == (Db < 0.0)) continue;
            t = Da / (Da - Db);
            if (out && n < cap)
                for (int b = 0; b < 3; ++b) {
                    double u = (double)c[b] + 0.5;
                    if (b == a) u = u + t;
                    out[3 * n + b] = (float)(u * h);
                }
            n++;
        }
    }
    return n;
}

/* brute-force distance from each query to the nearest of n points (FP64) */
void orc_nearest_distance(const float *pts, int64_t n, const float *q,
                          int64_t nq, double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t j = 0; j < nq; ++j) {
        double best = INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            double dx = (double)q[3 * j] - (double)pts[3 * i];
            double dy = (double)q[3 * j + 1] - (double)pts[3 * i + 1];
            double dz = (double)q[3 * j + 2] - (double)pts[3 * i + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < best) best = r2;
        }
        out[j] = sqrt(best);
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

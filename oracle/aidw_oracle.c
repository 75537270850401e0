/*
 * Plain FP64 CPU oracle for Adaptive Inverse Distance Weighting (AIDW),
 * Mei, Xu & Xu, "Accelerating Adaptive IDW Interpolation Algorithm on a
 * Single GPU" (arXiv 1511.02186).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU path is checked against.  Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the HIP library, and the HIP
 * library never calls it.
 *
 * What is computed, per interpolated (query) point q, over ALL m data points:
 *
 *   1. d_i = sqrt(dx*dx + dy*dy) in FP64 (no FMA contraction: built with
 *      -ffp-contract=off), for every data point i.
 *   2. The k nearest data points: the k smallest squared distances, found by
 *      a full sort of (d_i^2, i) pairs; equal distances keep the smaller
 *      index first.  sqrt is monotone, so ordering by d^2 is ordering by d.
 *      The paper's insertion procedure (Sec. 3.1.2, "Method for Finding the
 *      Nearest Data Points") selects the same multiset of distances.
 *   3. r_obs = (1/k) * sum of the k nearest distances            (Eq. 3)
 *      r_exp = 1 / (2 * sqrt(m / A))                             (Eq. 2)
 *      R     = r_obs / r_exp                                     (Eq. 4)
 *      In Eq. 2 the point count is the number of DATA points m (the paper's
 *      Sec. 2 calls the data count n; Sec. 3 renames it m).
 *   4. mu_R by the fuzzy membership function of Eq. 5, evaluated literally
 *      with the argument (pi / R_max) * (R - R_min); the first case whose
 *      condition holds is taken.
 *   5. alpha by the triangular membership function of Eq. 6, literally
 *      (first matching case), with the five levels alpha_1..alpha_5.
 *   6. Eq. 1 over all m data points:  Z = sum(w_i z_i) / sum(w_i),
 *      w_i = d_i^(-alpha) computed with libm pow, both sums Neumaier-
 *      compensated.  The paper does not define the case d_i = 0 (a query
 *      that coincides with data points).  Reading used here: when alpha > 0
 *      and some d_i == 0, Z is the mean of z_i over the points with d_i == 0
 *      (the limit of Eq. 1 as the query approaches them).  When alpha == 0,
 *      pow(d, -0) == 1 for every d, so Eq. 1 is the plain mean and needs no
 *      special case.
 *
 * Also provided: the standard (constant-power) IDW of Eq. 1 alone
 * (Sec. 2.1), used for the plain Shepard cross-check and the IDW mode.
 *
 * Range limit of the plain definition: the unscaled weights d^(-alpha)
 * overflow FP64 only when d < ~1e-308^(1/alpha); inputs rounded from FP32
 * have d >= 1.4e-45 or d == 0, which is always safe for alpha <= 6.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

/* ---- Eq. 2: expected nearest-neighbour distance of a random pattern ---- */
double aidw_oracle_r_exp(int64_t m, double area)
{
    return 1.0 / (2.0 * sqrt((double)m / area));
}

/* ---- Eq. 5: fuzzy normalisation of R into [0, 1] ---- */
double aidw_oracle_mu(double R, double R_min, double R_max)
{
    const double pi = 3.14159265358979323846;
    if (R <= R_min)
        return 0.0;
    if (R <= R_max)
        return 0.5 - 0.5 * cos((pi / R_max) * (R - R_min));
    return 1.0;
}

/* ---- Eq. 6: triangular membership mapping mu_R to a decay power ---- */
double aidw_oracle_alpha(double mu, const double lv[5])
{
    const double a1 = lv[0], a2 = lv[1], a3 = lv[2], a4 = lv[3], a5 = lv[4];
    if (mu <= 0.1)
        return a1;
    if (mu <= 0.3)
        return a1 * (1.0 - 5.0 * (mu - 0.1)) + 5.0 * a2 * (mu - 0.1);
    if (mu <= 0.5)
        return 5.0 * a3 * (mu - 0.3) + a2 * (1.0 - 5.0 * (mu - 0.3));
    if (mu <= 0.7)
        return a3 * (1.0 - 5.0 * (mu - 0.5)) + 5.0 * a4 * (mu - 0.5);
    if (mu <= 0.9)
        return 5.0 * a5 * (mu - 0.7) + a4 * (1.0 - 5.0 * (mu - 0.7));
    return a5;
}

/* Neumaier-compensated running sum. */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum* a) { return a->s + a->c; }

typedef struct {
    double d2;
    int64_t idx;
} keyed;

static int keyed_cmp(const void* pa, const void* pb)
{
    const keyed* a = (const keyed*)pa;
    const keyed* b = (const keyed*)pb;
    if (a->d2 < b->d2)
        return -1;
    if (a->d2 > b->d2)
        return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Squared distance, two products and one sum, never fused. */
static double sqdist(double qx, double qy, double px, double py)
{
    double ex = qx - px;
    double ey = qy - py;
    double xx = ex * ex;
    double yy = ey * ey;
    return xx + yy;
}

/* Eq. 1 with a given power over all m data points (both AIDW phase two and
 * standard IDW).  d2[i] holds the squared distance to data point i. */
static double weighted_average(const double* d2, const double* z, int64_t m, double alpha)
{
    if (alpha > 0.0) {
        nsum zs = {0.0, 0.0};
        int64_t cnt = 0;
        for (int64_t i = 0; i < m; ++i)
            if (d2[i] == 0.0) {
                nsum_add(&zs, z[i]);
                ++cnt;
            }
        if (cnt > 0)
            return nsum_value(&zs) / (double)cnt;
    }
    nsum num = {0.0, 0.0}, den = {0.0, 0.0};
    for (int64_t i = 0; i < m; ++i) {
        double d = sqrt(d2[i]);
        double w = pow(d, -alpha);
        nsum_add(&num, w * z[i]);
        nsum_add(&den, w);
    }
    return nsum_value(&num) / nsum_value(&den);
}

/* One query of AIDW: kNN, Eq. 2-6, then Eq. 1.  buf holds m keyed entries,
 * d2 holds m doubles; both are scratch owned by the caller. */
static void aidw_one(const double* x, const double* y, const double* z, int64_t m, double qx,
                     double qy, int k, const double lv[5], double R_min, double R_max,
                     double r_exp, keyed* buf, double* d2, double* out, double* r_obs_out,
                     double* alpha_out, int64_t* knn_out)
{
    for (int64_t i = 0; i < m; ++i) {
        d2[i] = sqdist(qx, qy, x[i], y[i]);
        buf[i].d2 = d2[i];
        buf[i].idx = i;
    }
    qsort(buf, (size_t)m, sizeof(keyed), keyed_cmp);

    nsum s = {0.0, 0.0};
    for (int j = 0; j < k; ++j)
        nsum_add(&s, sqrt(buf[j].d2));
    double r_obs = nsum_value(&s) / (double)k;
    double R = r_obs / r_exp;
    double mu = aidw_oracle_mu(R, R_min, R_max);
    double alpha = aidw_oracle_alpha(mu, lv);

    *out = weighted_average(d2, z, m, alpha);
    if (r_obs_out)
        *r_obs_out = r_obs;
    if (alpha_out)
        *alpha_out = alpha;
    if (knn_out)
        for (int j = 0; j < k; ++j)
            knn_out[j] = buf[j].idx;
}

typedef struct {
    const double *x, *y, *z, *qx, *qy;
    int64_t m, n;
    int k;
    const double* lv;
    double R_min, R_max, r_exp, idw_power;
    int idw_mode;
    double *out, *r_obs, *alpha;
    int64_t* knn;
    int64_t q_begin, q_end;
    int status;
} job;

static void* worker(void* arg)
{
    job* jb = (job*)arg;
    keyed* buf = NULL;
    double* d2 = (double*)malloc(sizeof(double) * (size_t)jb->m);
    if (!jb->idw_mode)
        buf = (keyed*)malloc(sizeof(keyed) * (size_t)jb->m);
    if (!d2 || (!jb->idw_mode && !buf)) {
        free(d2);
        free(buf);
        jb->status = ORACLE_ENOMEM;
        return NULL;
    }
    for (int64_t q = jb->q_begin; q < jb->q_end; ++q) {
        if (jb->idw_mode) {
            for (int64_t i = 0; i < jb->m; ++i)
                d2[i] = sqdist(jb->qx[q], jb->qy[q], jb->x[i], jb->y[i]);
            jb->out[q] = weighted_average(d2, jb->z, jb->m, jb->idw_power);
            continue;
        }
        aidw_one(jb->x, jb->y, jb->z, jb->m, jb->qx[q], jb->qy[q], jb->k, jb->lv, jb->R_min,
                 jb->R_max, jb->r_exp, buf, d2, &jb->out[q], jb->r_obs ? &jb->r_obs[q] : NULL,
                 jb->alpha ? &jb->alpha[q] : NULL, jb->knn ? &jb->knn[q * jb->k] : NULL);
    }
    free(d2);
    free(buf);
    jb->status = ORACLE_OK;
    return NULL;
}

static int run_threads(job* proto, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if ((int64_t)nthreads > proto->n)
        nthreads = (int)(proto->n > 0 ? proto->n : 1);
    job* jobs = (job*)calloc((size_t)nthreads, sizeof(job));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    char* joined = (char*)calloc((size_t)nthreads, 1);
    if (!jobs || !th || !joined) {
        free(jobs);
        free(th);
        free(joined);
        return ORACLE_ENOMEM;
    }
    int64_t per = (proto->n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].q_begin = (int64_t)t * per < proto->n ? (int64_t)t * per : proto->n;
        jobs[t].q_end = jobs[t].q_begin + per < proto->n ? jobs[t].q_begin + per : proto->n;
        jobs[t].status = ORACLE_OK;
        if (jobs[t].q_begin >= jobs[t].q_end)
            continue;
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) == 0)
            joined[t] = 1;
        else
            worker(&jobs[t]); /* run inline if a thread cannot be started */
    }
    int status = ORACLE_OK;
    for (int t = 0; t < nthreads; ++t) {
        if (joined[t])
            pthread_join(th[t], NULL);
        if (jobs[t].status != ORACLE_OK)
            status = jobs[t].status;
    }
    free(jobs);
    free(th);
    free(joined);
    return status;
}

static int finite_pos(double v) { return isfinite(v) && v > 0.0; }

/*
 * AIDW over n queries.  x, y, z: the m data points; qx, qy: the n queries.
 * Outputs: out[n]; optional r_obs[n], alpha[n], knn[n*k] (may be NULL).
 * Returns 0, or ORACLE_EINVAL for m < 1, k < 1, k > m, area <= 0,
 * R_max <= R_min, R_max <= 0, or a negative / non-finite level.
 */
int aidw_oracle_run(const double* x, const double* y, const double* z, int64_t m,
                    const double* qx, const double* qy, int64_t n, int k,
                    const double alpha_levels[5], double R_min, double R_max, double area,
                    double* out, double* r_obs, double* alpha, int64_t* knn, int nthreads)
{
    if (m < 1 || n < 0 || k < 1 || (int64_t)k > m || !finite_pos(area) || !isfinite(R_min) ||
        !isfinite(R_max) || R_max <= R_min || R_max <= 0.0)
        return ORACLE_EINVAL;
    for (int j = 0; j < 5; ++j)
        if (!isfinite(alpha_levels[j]) || alpha_levels[j] < 0.0)
            return ORACLE_EINVAL;
    if (n == 0)
        return ORACLE_OK;
    job proto;
    memset(&proto, 0, sizeof(proto));
    proto.x = x;
    proto.y = y;
    proto.z = z;
    proto.qx = qx;
    proto.qy = qy;
    proto.m = m;
    proto.n = n;
    proto.k = k;
    proto.lv = alpha_levels;
    proto.R_min = R_min;
    proto.R_max = R_max;
    proto.r_exp = aidw_oracle_r_exp(m, area);
    proto.out = out;
    proto.r_obs = r_obs;
    proto.alpha = alpha;
    proto.knn = knn;
    return run_threads(&proto, nthreads);
}

/* Standard IDW (Sec. 2.1, Eq. 1) with a constant power p >= 0. */
int aidw_oracle_idw(const double* x, const double* y, const double* z, int64_t m,
                    const double* qx, const double* qy, int64_t n, double power, double* out,
                    int nthreads)
{
    if (m < 1 || n < 0 || !isfinite(power) || power < 0.0)
        return ORACLE_EINVAL;
    if (n == 0)
        return ORACLE_OK;
    job proto;
    memset(&proto, 0, sizeof(proto));
    proto.x = x;
    proto.y = y;
    proto.z = z;
    proto.qx = qx;
    proto.qy = qy;
    proto.m = m;
    proto.n = n;
    proto.idw_mode = 1;
    proto.idw_power = power;
    proto.out = out;
    return run_threads(&proto, nthreads);
}

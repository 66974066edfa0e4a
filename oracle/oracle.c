/*
 * Plain CPU reference ("oracle") for the SpMV + Krylov hot path of
 * "Cascaded Prediction and Asynchronous Execution of Iterative Algorithms on
 * Heterogeneous Platforms" (Gao, Liu, Wang, Ji, Huang; arXiv 2411.10143).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it is used by the test-suite, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no code with the GPU path.
 *
 * Everything is IEEE double precision, compiled without FMA contraction and
 * without fast-math, so every result is reproducible.  The code favours
 * being checkable by eye over speed.  Built with OpenMP (the all-core CPU
 * baseline), only the rows of orc_spmv are shared out among threads; each
 * row is still summed alone in ascending order, so both builds give the same
 * bits.
 *
 * Contents and the passage each follows:
 *   orc_spmv            y = alpha*A*x + beta*y over CSR (the kernel the whole
 *                       paper optimises; Introduction).  Row sums in ascending
 *                       storage order.
 *   orc_features_int    integer accumulators of the 15 matrix features of the
 *                       feature table (Section III-B-1), plus a row-length
 *                       histogram, the main-diagonal count and a symmetry flag.
 *   orc_features_derive the floating-point features of the same table,
 *                       derived only from those integers.
 *   orc_ell_shape,      CSR -> ELL, COO, DIA and HYB conversion, the formats
 *   orc_csr_to_ell,     of the configuration space (Section III-B-2) and the
 *   orc_csr_to_coo_rows conversion step of the online phase (Section III-C-1).
 *   orc_dia_shape,
 *   orc_csr_to_dia,
 *   orc_hyb_width,
 *   orc_hyb_tail_rows
 *   orc_tree_eval,      decision-tree inference and the three-stage cascade
 *   orc_cascade         (Section III-C-1, the cascaded-prediction figure).
 *   orc_cg              conjugate gradient (Hestenes-Stiefel form; Saad,
 *                       Iterative Methods for Sparse Linear Systems, Alg. 6.18),
 *                       the first of the two solvers the Introduction names.
 *   orc_gmres,          restarted GMRES(m) with modified Gram-Schmidt Arnoldi
 *   orc_arnoldi         and Givens rotations (Saad, Alg. 6.9 / 6.10), the
 *                       solver of the evaluation (Section IV).
 *   orc_relres          true relative residual ||b - A x|| / ||b||.
 *
 * Status codes: 0 ok, -1 invalid, -4 not converged, -5 breakdown,
 *               -6 unsupported (ELL refused for fill).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_INVALID (-1)
#define ORC_NOT_CONVERGED (-4)
#define ORC_BREAKDOWN (-5)
#define ORC_UNSUPPORTED (-6)

/* ------------------------------------------------------------------------ */
/* SpMV                                                                      */
/* ------------------------------------------------------------------------ */

/* y_i = alpha * sum_{k=rp[i]}^{rp[i+1]-1} val[k]*x[col[k]] + beta*y_i.
 * The sum runs in ascending k.  With beta == 0, y is not read (so NaN in y
 * does not propagate). */
void orc_spmv(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
              double alpha, const double *x, double beta, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            s = s + val[k] * x[col[k]];
        if (beta == 0.0)
            y[i] = alpha * s;
        else
            y[i] = alpha * s + beta * y[i];
    }
}

/* Threads orc_spmv runs on (1 without OpenMP). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s = s + a[i] * b[i];
    return s;
}

static double nrm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

/* ||b - A x|| / ||b|| (0 when b == 0 and x == 0 gives a zero residual). */
double orc_relres(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                  const double *b, const double *x)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(r, b, sizeof(double) * (size_t)n);
    orc_spmv(n, rp, col, val, -1.0, x, 1.0, r);
    double nr = nrm2(n, r), nb = nrm2(n, b);
    free(r);
    if (nb == 0.0)
        return nr;
    return nr / nb;
}

/* ------------------------------------------------------------------------ */
/* Features (feature table, Section III-B-1)                                 */
/* ------------------------------------------------------------------------ */

/* Output layout of the integer accumulators (int64[28]):
 *  0 nrows  1 ncols  2 nnz  3 sum r_i  4 sum r_i^2  5 max r_i  6 min r_i
 *  7 sum (c_last - c_first)   8 sum cl_i (longest run of consecutive columns)
 *  9 ndiag (distinct col-row over stored entries)  10 stored main-diagonal
 *  11..26 histogram: bin 0 empty rows, bin b>=1 lengths in [2^(b-1), 2^b),
 *         bin 15 open-ended
 *  27 is_symmetric (square, and a_ij == a_ji for every stored entry, with the
 *     transposed entry stored too)
 * Returns ORC_INVALID when the CSR arrays are malformed. */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int orc_csr_validate(int64_t n, int64_t ncols, int64_t nnz, const int32_t *rp,
                     const int32_t *col)
{
    if (n < 0 || ncols < 0 || nnz < 0 || rp[0] != 0 || rp[n] != nnz)
        return ORC_INVALID;
    for (int64_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i])
            return ORC_INVALID;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= ncols)
                return ORC_INVALID;
            if (k > rp[i] && col[k] <= col[k - 1])
                return ORC_INVALID;
        }
    }
    return ORC_OK;
}

int orc_features_int(int64_t n, int64_t ncols, const int32_t *rp, const int32_t *col,
                     const double *val, int64_t *out)
{
    memset(out, 0, sizeof(int64_t) * 28);
    int64_t nnz = rp[n];
    if (orc_csr_validate(n, ncols, nnz, rp, col) != ORC_OK)
        return ORC_INVALID;
    out[0] = n;
    out[1] = ncols;
    out[2] = nnz;
    int64_t maxr = 0, minr = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = rp[i + 1] - rp[i];
        out[3] += r;
        out[4] += r * r;
        if (i == 0 || r > maxr)
            maxr = r;
        if (i == 0 || r < minr)
            minr = r;
        if (r > 0) {
            out[7] += (int64_t)col[rp[i + 1] - 1] - (int64_t)col[rp[i]];
            int64_t run = 1, best = 1;
            for (int64_t k = rp[i] + 1; k < rp[i + 1]; ++k) {
                if (col[k] == col[k - 1] + 1)
                    run = run + 1;
                else
                    run = 1;
                if (run > best)
                    best = run;
            }
            out[8] += best;
        }
        int bin = 0;
        if (r > 0) {
            bin = 1;
            while (bin < 15 && r >= ((int64_t)1 << bin))
                bin = bin + 1;
        }
        out[11 + bin] += 1;
    }
    out[5] = maxr;
    out[6] = minr;
    /* diagonals: d = col - row + (n - 1) in [0, n + ncols - 2] */
    int64_t nd = n + ncols - 1;
    unsigned char *seen = (unsigned char *)calloc((size_t)(nd > 0 ? nd : 1), 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            seen[(int64_t)col[k] - i + (n - 1)] = 1;
            if (col[k] == i)
                out[10] += 1;
        }
    for (int64_t d = 0; d < nd; ++d)
        out[9] += seen[d];
    free(seen);
    /* symmetry: every stored (i, j, v) has a stored (j, i, v) */
    int sym = (n == ncols);
    for (int64_t i = 0; i < n && sym; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1] && sym; ++k) {
            int32_t j = col[k];
            int32_t key = (int32_t)i;
            const int32_t *hit = (const int32_t *)bsearch(&key, col + rp[j],
                                                          (size_t)(rp[j + 1] - rp[j]),
                                                          sizeof(int32_t), cmp_i32);
            if (hit == NULL || val[hit - col] != val[k])
                sym = 0;
        }
    out[27] = sym;
    return ORC_OK;
}

/* Derived features, in this order (double[9]):
 *  0 density = nnz / (nrows*ncols)          1 mean = nnz / nrows
 *  2 sd = sqrt(nrows*sum r^2 - (sum r)^2) / nrows   (population sd; the
 *        radicand is formed exactly in 128-bit integers)
 *  3 cov = sd / mean (0 if mean == 0)       4 maxavg = max - mean
 *  5 distavg = sum (c_last - c_first) / nrows
 *  6 clusteravg = sum cl_i / nrows
 *  7 fill = nrows*max / nnz (0 if nnz == 0)
 *  8 diagfill = nrows*ndiag / nnz (0 if nnz == 0)
 * Every value is 0 when nrows == 0. */
void orc_features_derive(const int64_t *a, double *d)
{
    for (int t = 0; t < 9; ++t)
        d[t] = 0.0;
    int64_t n = a[0], ncols = a[1], nnz = a[2];
    if (n <= 0)
        return;
    double dn = (double)n;
    d[0] = (ncols > 0) ? (double)nnz / (dn * (double)ncols) : 0.0;
    d[1] = (double)nnz / dn;
    __int128 V = (__int128)n * (__int128)a[4] - (__int128)a[3] * (__int128)a[3];
    d[2] = sqrt((double)V) / dn;
    d[3] = (d[1] > 0.0) ? d[2] / d[1] : 0.0;
    d[4] = (double)a[5] - d[1];
    d[5] = (double)a[7] / dn;
    d[6] = (double)a[8] / dn;
    d[7] = (nnz > 0) ? (dn * (double)a[5]) / (double)nnz : 0.0;
    d[8] = (nnz > 0) ? (dn * (double)a[9]) / (double)nnz : 0.0;
}

/* The 15 model inputs of the feature table, in table order:
 * nrows ncols nnz density mean sd cov max min maxavg distavg clusteravg
 * fill ndiag diagfill */
void orc_feature_vector(const int64_t *a, const double *d, double *f)
{
    f[0] = (double)a[0];
    f[1] = (double)a[1];
    f[2] = (double)a[2];
    f[3] = d[0];
    f[4] = d[1];
    f[5] = d[2];
    f[6] = d[3];
    f[7] = (double)a[5];
    f[8] = (double)a[6];
    f[9] = d[4];
    f[10] = d[5];
    f[11] = d[6];
    f[12] = d[7];
    f[13] = (double)a[9];
    f[14] = d[8];
}

/* ------------------------------------------------------------------------ */
/* Format conversions                                                        */
/* ------------------------------------------------------------------------ */

/* ELL shape: K = max row length, pitch = n rounded up to a multiple of 64.
 * The conversion is refused (ORC_UNSUPPORTED) when K*pitch > 8*nnz: past
 * that fill ELL moves more than eight times the CSR bytes. */
int orc_ell_shape(int64_t n, const int32_t *rp, int64_t *K, int64_t *pitch)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > k)
            k = rp[i + 1] - rp[i];
    *K = k;
    *pitch = (n + 63) / 64 * 64;
    if (k * (*pitch) > 8 * (int64_t)rp[n])
        return ORC_UNSUPPORTED;
    return ORC_OK;
}

/* Column-major ELLPACK: slot s of row i lives at s*pitch + i.  Unused slots
 * (and rows n..pitch-1) hold column -1 and value +0.0. */
int orc_csr_to_ell(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                   int64_t K, int64_t pitch, int32_t *ell_col, double *ell_val)
{
    for (int64_t s = 0; s < K; ++s)
        for (int64_t i = 0; i < pitch; ++i) {
            int64_t at = s * pitch + i;
            if (i < n && s < rp[i + 1] - rp[i]) {
                ell_col[at] = col[rp[i] + s];
                ell_val[at] = val[rp[i] + s];
            } else {
                ell_col[at] = -1;
                ell_val[at] = 0.0;
            }
        }
    return ORC_OK;
}

/* COO row array in CSR (row-major) order: row[k] = i for rp[i] <= k < rp[i+1].
 * Column and value arrays are the CSR ones. */
void orc_csr_to_coo_rows(int64_t n, const int32_t *rp, int32_t *row)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            row[k] = (int32_t)i;
}

/* DIA shape (DIA is one of the formats of the configuration space, Section
 * III-B-2): the stored diagonals are the distinct values of col - row over
 * the stored entries, in ascending order; pitch = n rounded up to a multiple
 * of 64.  Refused (ORC_UNSUPPORTED) when ndiag*pitch > 8*nnz, the same fill
 * limit as ELL.  off may be NULL (shape only); otherwise it receives the
 * ndiag offsets. */
int orc_dia_shape(int64_t n, int64_t ncols, const int32_t *rp, const int32_t *col,
                  int64_t *ndiag, int64_t *pitch, int32_t *off)
{
    /* seen[d + n - 1] marks offset d, d in [-(n-1), ncols-1] */
    int64_t span = n + ncols - 1;
    unsigned char *seen = (unsigned char *)calloc(span > 0 ? (size_t)span : 1, 1);
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            seen[(int64_t)col[k] - i + n - 1] = 1;
    for (int64_t t = 0; t < span; ++t)
        if (seen[t]) {
            if (off)
                off[count] = (int32_t)(t - (n - 1));
            ++count;
        }
    free(seen);
    *ndiag = count;
    *pitch = ((n + 63) / 64) * 64;
    if (count * (*pitch) > 8 * (int64_t)rp[n])
        return ORC_UNSUPPORTED;
    return ORC_OK;
}

/* DIA values: diagonal d of row i lives at d*pitch + i and holds a(i, i +
 * off[d]) when that entry is stored; every other slot (absent entries,
 * columns outside [0, ncols), rows n..pitch-1) holds +0.0. */
int orc_csr_to_dia(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                   int64_t ndiag, int64_t pitch, const int32_t *off, double *dia_val)
{
    for (int64_t t = 0; t < ndiag * pitch; ++t)
        dia_val[t] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            int64_t d = 0;            /* find col - row among the offsets */
            while (off[d] != (int64_t)col[k] - i)
                ++d;
            dia_val[d * pitch + i] = val[k];
        }
    return ORC_OK;
}

/* HYB width (HYB, ELL plus a remainder, is one of the formats of the
 * configuration space, Section III-B-2; the width rule is Bell and
 * Garland's): K = the largest k >= 0 such that at least a third of the rows
 * have k or more entries, i.e. 3 * #{i : r_i >= k} >= n.  n = 0 gives 0. */
int64_t orc_hyb_width(int64_t n, const int32_t *rp)
{
    int64_t K = 0;
    for (int64_t k = 1;; ++k) {
        int64_t rows = 0;
        for (int64_t i = 0; i < n; ++i)
            if (rp[i + 1] - rp[i] >= k)
                ++rows;
        if (rows == 0 || 3 * rows < n)
            break;
        K = k;
    }
    return K;
}

/* HYB layout: the ELL part is the ELL layout of width K (each row's first
 * min(r_i, K) entries; orc_csr_to_ell with that K), and the remainder is
 * the list of rows longer than K in ascending order (their entries K..r_i-1
 * stay in the CSR arrays).  Returns the number of such rows; tail_rows may
 * be NULL to count only. */
int64_t orc_hyb_tail_rows(int64_t n, const int32_t *rp, int64_t K, int32_t *tail_rows)
{
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > K) {
            if (tail_rows)
                tail_rows[t] = (int32_t)i;
            ++t;
        }
    return t;
}

/* ------------------------------------------------------------------------ */
/* Decision trees and the cascade (Section III-C-1)                          */
/* ------------------------------------------------------------------------ */

/* Node t: internal if feature[t] >= 0, then go left iff
 * (double)(float)f[feature[t]] <= thr[t]; a leaf returns cls[t].  The float
 * cast matches a classifier trained on single-precision inputs. */
int32_t orc_tree_eval(const int32_t *feature, const double *thr, const int32_t *left,
                      const int32_t *right, const int32_t *cls, const double *f)
{
    int32_t t = 0;
    while (feature[t] >= 0) {
        double v = (double)(float)f[feature[t]];
        if (v <= thr[t])
            t = left[t];
        else
            t = right[t];
    }
    return cls[t];
}

/* Cascade over three trees given as (feature, thr, left, right, cls) blocks.
 * Stage 1 picks the format (0 CSR, 1 ELL, 2 COO, 3 DIA, 4 HYB); only for CSR
 * does stage 2 pick the CSR algorithm (0 scalar, 1 vector, 2 merge-path,
 * 3 column panels); only for vector does stage 3 pick log2 of the lanes per
 * row.
 * out[0..2] = the three decisions (-1 when a stage does not run). */
void orc_cascade(const int32_t *f1, const double *t1, const int32_t *l1, const int32_t *r1,
                 const int32_t *c1, const int32_t *f2, const double *t2, const int32_t *l2,
                 const int32_t *r2, const int32_t *c2, const int32_t *f3, const double *t3,
                 const int32_t *l3, const int32_t *r3, const int32_t *c3, const double *feat,
                 int32_t *out)
{
    out[0] = orc_tree_eval(f1, t1, l1, r1, c1, feat);
    out[1] = -1;
    out[2] = -1;
    if (out[0] == 0) {
        out[1] = orc_tree_eval(f2, t2, l2, r2, c2, feat);
        if (out[1] == 1)
            out[2] = orc_tree_eval(f3, t3, l3, r3, c3, feat);
    }
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient (Hestenes-Stiefel)                                     */
/* ------------------------------------------------------------------------ */

/* Solves A x = b for SPD A from the given x0 (in x).  Stops when
 * sqrt(r.r)/||b|| <= tol on the recurred residual, then recomputes
 * r = b - A x; if that true residual is above tol, CG restarts from the
 * current x with p = r (at most 3 restarts, then ORC_NOT_CONVERGED).
 * p.Ap <= 0 is a breakdown (A not SPD).  maxit bounds the SpMV count.
 * Optional records (NULL to skip): alpha_h/beta_h/res_h (hist_cap entries;
 * res_h[k] = recurred ||r_k||/||b|| with res_h[0] the start), and the first
 * nrec residual / direction vectors (column-major n x nrec). */
int orc_cg(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
           const double *b, double *x, double tol, int64_t maxit, int64_t *iters_out,
           double *relres_out, double *alpha_h, double *beta_h, double *res_h,
           int64_t hist_cap, double *R_rec, double *P_rec, int64_t nrec)
{
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(bytes), *p = (double *)malloc(bytes);
    double *q = (double *)malloc(bytes);
    double nb = nrm2(n, b);
    int64_t it = 0;
    int status = ORC_NOT_CONVERGED;
    *iters_out = 0;
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = 0.0;
        *relres_out = 0.0;
        free(r); free(p); free(q);
        return ORC_OK;
    }
    for (int restart = 0; restart <= 3; ++restart) {
        /* r = b - A x, p = r, rho = r.r */
        memcpy(r, b, bytes);
        orc_spmv(n, rp, col, val, -1.0, x, 1.0, r);
        memcpy(p, r, bytes);
        double rho = dot(n, r, r);
        if (res_h && it < hist_cap && restart == 0)
            res_h[0] = sqrt(rho) / nb;
        if (sqrt(rho) / nb <= tol) {
            status = ORC_OK;
            break;
        }
        int stopped = 0;
        while (it < maxit) {
            orc_spmv(n, rp, col, val, 1.0, p, 0.0, q);         /* q = A p      */
            double sigma = dot(n, p, q);                       /* sigma = p.q  */
            if (!(sigma > 0.0)) {
                status = ORC_BREAKDOWN;
                goto done;
            }
            double alpha = rho / sigma;
            if (R_rec && it < nrec) {
                memcpy(R_rec + it * n, r, bytes);
                memcpy(P_rec + it * n, p, bytes);
            }
            for (int64_t i = 0; i < n; ++i)
                x[i] = x[i] + alpha * p[i];                    /* x += alpha p */
            for (int64_t i = 0; i < n; ++i)
                r[i] = r[i] - alpha * q[i];                    /* r -= alpha q */
            double rho_new = dot(n, r, r);
            double beta = rho_new / rho;
            it = it + 1;
            if (alpha_h && it - 1 < hist_cap) {
                alpha_h[it - 1] = alpha;
                beta_h[it - 1] = beta;
            }
            if (res_h && it < hist_cap)
                res_h[it] = sqrt(rho_new) / nb;
            if (sqrt(rho_new) / nb <= tol) {
                stopped = 1;
                break;
            }
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * p[i];                     /* p = r + beta p */
            rho = rho_new;
        }
        double true_res = orc_relres(n, rp, col, val, b, x);
        if (true_res <= tol) {
            status = ORC_OK;
            break;
        }
        if (!stopped)
            break; /* iteration budget spent */
    }
done:
    *iters_out = it;
    *relres_out = orc_relres(n, rp, col, val, b, x);
    free(r); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Arnoldi (modified Gram-Schmidt) and restarted GMRES(m)                    */
/* ------------------------------------------------------------------------ */

/* One Arnoldi step j: w = A v_j, orthogonalise against v_0..v_j with modified
 * Gram-Schmidt, store h_{0..j+1, j} in column j of H (leading dim ldh) and,
 * unless h_{j+1,j} == 0, v_{j+1} = w / h_{j+1,j}.  V is column-major n x (m+1).
 * Returns 1 on a happy breakdown (h_{j+1,j} == 0), else 0. */
static int arnoldi_step(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                        double *V, double *H, int64_t ldh, int64_t j, double *w)
{
    orc_spmv(n, rp, col, val, 1.0, V + j * n, 0.0, w);
    for (int64_t i = 0; i <= j; ++i) {
        double h = dot(n, w, V + i * n);
        H[j * ldh + i] = h;
        for (int64_t t = 0; t < n; ++t)
            w[t] = w[t] - h * V[i * n + t];
    }
    double hn = nrm2(n, w);
    H[j * ldh + j + 1] = hn;
    if (hn == 0.0)
        return 1;
    for (int64_t t = 0; t < n; ++t)
        V[(j + 1) * n + t] = w[t] / hn;
    return 0;
}

/* m Arnoldi steps from v0 (normalised here).  V: n x (m+1), H: (m+1) x m,
 * both column-major and zero-filled on entry.  *steps = steps completed
 * (fewer than m after a happy breakdown). */
int orc_arnoldi(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
                const double *v0, int64_t m, double *V, double *H, int64_t *steps)
{
    double nv = nrm2(n, v0);
    *steps = 0;
    if (nv == 0.0)
        return ORC_INVALID;
    for (int64_t t = 0; t < n; ++t)
        V[t] = v0[t] / nv;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < m; ++j) {
        int brk = arnoldi_step(n, rp, col, val, V, H, m + 1, j, w);
        *steps = j + 1;
        if (brk)
            break;
    }
    free(w);
    return ORC_OK;
}

/* Restarted GMRES(m), x0 in x, no preconditioner.  Each cycle starts from the
 * true residual r = b - A x (so the stopping decision is always confirmed on
 * b - A x), runs up to m Arnoldi steps with Givens rotations, stops early when
 * the rotated residual |g_{j+1}| / ||b|| <= tol or on a happy breakdown, then
 * solves the triangular system and updates x.  maxit bounds the total number
 * of Arnoldi steps.  res_h (optional): res_h[k] = |g| / ||b|| after total
 * step k (res_h[0] = start); cycle starts overwrite with the true residual. */
int orc_gmres(int64_t n, const int32_t *rp, const int32_t *col, const double *val,
              const double *b, double *x, int64_t m, double tol, int64_t maxit,
              int64_t *iters_out, double *relres_out, double *res_h, int64_t hist_cap)
{
    size_t nb_bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *V = (double *)malloc(nb_bytes * (size_t)(m + 1));
    double *H = (double *)calloc((size_t)((m + 1) * m), sizeof(double));
    double *w = (double *)malloc(nb_bytes), *r = (double *)malloc(nb_bytes);
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    double nb = nrm2(n, b);
    int64_t it = 0;
    int status = ORC_NOT_CONVERGED;
    if (nb == 0.0) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = 0.0;
        *iters_out = 0;
        *relres_out = 0.0;
        status = ORC_OK;
        goto out;
    }
    for (;;) {
        memcpy(r, b, nb_bytes);
        orc_spmv(n, rp, col, val, -1.0, x, 1.0, r);             /* r = b - A x */
        double beta = nrm2(n, r);
        if (res_h && it < hist_cap)
            res_h[it] = beta / nb;
        if (beta / nb <= tol) {
            status = ORC_OK;
            break;
        }
        if (it >= maxit)
            break;
        for (int64_t t = 0; t < n; ++t)
            V[t] = r[t] / beta;
        memset(H, 0, sizeof(double) * (size_t)((m + 1) * m));
        for (int64_t t = 0; t <= m; ++t)
            g[t] = 0.0;
        g[0] = beta;
        int64_t k = 0; /* columns formed in this cycle */
        for (int64_t j = 0; j < m && it < maxit; ++j) {
            int brk = arnoldi_step(n, rp, col, val, V, H, m + 1, j, w);
            double *hj = H + j * (m + 1);
            for (int64_t i = 0; i < j; ++i) {                  /* old rotations */
                double a = hj[i], c = hj[i + 1];
                hj[i] = cs[i] * a + sn[i] * c;
                hj[i + 1] = -sn[i] * a + cs[i] * c;
            }
            double a = hj[j], c = hj[j + 1];
            double d = sqrt(a * a + c * c);
            if (d == 0.0) {
                status = ORC_BREAKDOWN;
                goto finish;
            }
            cs[j] = a / d;
            sn[j] = c / d;
            hj[j] = d;
            hj[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            it = it + 1;
            k = j + 1;
            if (res_h && it < hist_cap)
                res_h[it] = fabs(g[j + 1]) / nb;
            if (brk || fabs(g[j + 1]) / nb <= tol)
                break;
        }
        /* back substitution R y = g, then x += V y */
        for (int64_t i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int64_t t = i + 1; t < k; ++t)
                s = s - H[t * (m + 1) + i] * y[t];
            y[i] = s / H[i * (m + 1) + i];
        }
        for (int64_t i = 0; i < k; ++i)
            for (int64_t t = 0; t < n; ++t)
                x[t] = x[t] + y[i] * V[i * n + t];
    }
finish:
    *iters_out = it;
    *relres_out = orc_relres(n, rp, col, val, b, x);
out:
    free(V); free(H); free(w); free(r); free(cs); free(sn); free(g); free(y);
    return status;
}

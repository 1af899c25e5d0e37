/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU statement of what the wide/tall sparse
 * product path computes, written from Eckstein & Matyasfalvi, "Efficient
 * Distributed-Memory Parallel Matrix-Vector Multiplication with Wide or Tall
 * Unstructured Sparse Matrices" (arXiv:1812.00904).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library; the two only
 * meet on the seeded inputs produced by the `synth` package.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (no FMA
 * contraction: every product is rounded before it is added, round-to-nearest-
 * even, IEEE binary64 throughout).
 *
 * Contents and what each part follows:
 *   - orc_mv_csc / orc_vtm_csc / *_csr / *_batch: the products y = A x and
 *     u^T = v^T A as defined in Section I (problem statement), for a wide matrix
 *     stored column-major and, by swapping the roles of rows and columns
 *     (Section II, first paragraph), a tall matrix stored row-major.  Each also
 *     returns the per-component error denominator d = sum |a||x| used by the
 *     parity tolerances.
 *   - orc_round_bits: single round-to-nearest-even from binary64 to a shorter
 *     binary format (used for binary32 and bfloat16 value storage).
 *   - orc_offsets_paper / orc_offsets_fixed: the split of the Z nonzeros into
 *     contiguous groups (Section II: first Z mod P groups hold ceil(Z/P)).
 *   - orc_cover, orc_zones: the cover sets J_i through their first and last
 *     columns, and the overlap zones j_k with their processor sets S_k, from
 *     their definitions (Section II; Section IV-A, Table I).
 *   - orc_setup_vars: the one-time setup of Section IV-B (needLeft, needRight,
 *     leftGroupEnd, rightGroup, leftGroup, procsOnLeft, procsOnRight; Table II).
 *   - orc_nzp_mv / orc_nzp_vtm: a serial simulation of the nonzero-partitioned
 *     algorithms of Section III (local products, then y = sum of y_(i)) and
 *     Section IV-A (local products, then zone sums over S_k).
 *   - orc_cgls: a first-order solver that alternates the two products with
 *     vector updates and inner products, as Section VII describes such methods.
 *     The paper names conjugate gradients without fixing a variant; this is
 *     conjugate gradients on the least-squares problem min ||b - A x||_2
 *     (CGLS, Hestenes and Stiefel 1952, in the arrangement of Bjorck,
 *     "Numerical Methods for Least Squares Problems", 1996, Section 7.4),
 *     one A p and one A^T r per iteration, inner products summed in index order.
 *
 * Parity status: every function here is pinned by tests/test_oracle_pins.py
 * (dense brute force, exact integer arithmetic, closed forms, the worked
 * example of Figures 1-3 and Tables I-II).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Products (Section I).  Column-major (CSC) storage of a wide m x n matrix:  */
/* column j holds positions ptr[j] .. ptr[j+1]-1, row index idx[p], value     */
/* val[p].  Outputs are overwritten.                                          */
/* ------------------------------------------------------------------------ */

/* y = A x for CSC A.  d[i] = sum_j |a_ij| |x_j|. */
void orc_mv_csc(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx,
                const double *val, const double *x, double *y, double *d)
{
    for (int64_t i = 0; i < m; ++i) { y[i] = 0.0; if (d) d[i] = 0.0; }
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) {
            int64_t i = idx[p];
            double prod = val[p] * x[j];
            y[i] = y[i] + prod;
            if (d) d[i] = d[i] + fabs(val[p]) * fabs(x[j]);
        }
    }
}

/* u^T = v^T A for CSC A: u_j = sum_i v_i a_ij.  d[j] = sum_i |v_i| |a_ij|. */
void orc_vtm_csc(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx,
                 const double *val, const double *v, double *u, double *d)
{
    (void)m;
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0, a = 0.0;
        for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) {
            double prod = val[p] * v[idx[p]];
            s = s + prod;
            a = a + fabs(val[p]) * fabs(v[idx[p]]);
        }
        u[j] = s;
        if (d) d[j] = a;
    }
}

/* Row-major (CSR) storage of a tall m x n matrix: row i holds positions       */
/* ptr[i] .. ptr[i+1]-1 with column index idx[p].                              */

/* y = A x for CSR A: y_i = sum_j a_ij x_j, summed along the row. */
void orc_mv_csr(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx,
                const double *val, const double *x, double *y, double *d)
{
    (void)n;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0, a = 0.0;
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
            double prod = val[p] * x[idx[p]];
            s = s + prod;
            a = a + fabs(val[p]) * fabs(x[idx[p]]);
        }
        y[i] = s;
        if (d) d[i] = a;
    }
}

/* u^T = v^T A for CSR A: u_j accumulates v_i a_ij row by row. */
void orc_vtm_csr(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx,
                 const double *val, const double *v, double *u, double *d)
{
    for (int64_t j = 0; j < n; ++j) { u[j] = 0.0; if (d) d[j] = 0.0; }
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
            int64_t j = idx[p];
            double prod = val[p] * v[i];
            u[j] = u[j] + prod;
            if (d) d[j] = d[j] + fabs(val[p]) * fabs(v[i]);
        }
    }
}

/* Multi-right-hand-side forms.  X is n x k (CSC mv) with X[j*ldx + c];  Y is   */
/* m x k with Y[i*ldy + c]; D like Y (may be NULL).  Column c of the block is   */
/* exactly the single-vector product of column c, so these loop over c.         */
static void gather_col(const double *X, int64_t rows, int64_t ld, int64_t c, double *out)
{
    for (int64_t r = 0; r < rows; ++r) out[r] = X[r * ld + c];
}
static void scatter_col(double *Y, int64_t rows, int64_t ld, int64_t c, const double *in)
{
    for (int64_t r = 0; r < rows; ++r) Y[r * ld + c] = in[r];
}

typedef void (*orc_op_fn)(int64_t, int64_t, const int64_t *, const int32_t *,
                          const double *, const double *, double *, double *);

static int batch_apply(orc_op_fn fn, int64_t in_len, int64_t out_len, int64_t m, int64_t n,
                       const int64_t *ptr, const int32_t *idx, const double *val,
                       int64_t k, const double *X, int64_t ldx, double *Y, int64_t ldy,
                       double *D, int64_t ldd)
{
    double *xin = (double *)malloc(sizeof(double) * (size_t)(in_len > 0 ? in_len : 1));
    double *yout = (double *)malloc(sizeof(double) * (size_t)(out_len > 0 ? out_len : 1));
    double *dout = (double *)malloc(sizeof(double) * (size_t)(out_len > 0 ? out_len : 1));
    if (!xin || !yout || !dout) { free(xin); free(yout); free(dout); return -1; }
    for (int64_t c = 0; c < k; ++c) {
        gather_col(X, in_len, ldx, c, xin);
        fn(m, n, ptr, idx, val, xin, yout, dout);
        scatter_col(Y, out_len, ldy, c, yout);
        if (D) scatter_col(D, out_len, ldd, c, dout);
    }
    free(xin); free(yout); free(dout);
    return 0;
}

int orc_mv_csc_batch(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
                     int64_t k, const double *X, int64_t ldx, double *Y, int64_t ldy, double *D, int64_t ldd)
{ return batch_apply(orc_mv_csc, n, m, m, n, ptr, idx, val, k, X, ldx, Y, ldy, D, ldd); }

int orc_vtm_csc_batch(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
                      int64_t k, const double *V, int64_t ldv, double *U, int64_t ldu, double *D, int64_t ldd)
{ return batch_apply(orc_vtm_csc, m, n, m, n, ptr, idx, val, k, V, ldv, U, ldu, D, ldd); }

int orc_mv_csr_batch(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
                     int64_t k, const double *X, int64_t ldx, double *Y, int64_t ldy, double *D, int64_t ldd)
{ return batch_apply(orc_mv_csr, n, m, m, n, ptr, idx, val, k, X, ldx, Y, ldy, D, ldd); }

int orc_vtm_csr_batch(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
                      int64_t k, const double *V, int64_t ldv, double *U, int64_t ldu, double *D, int64_t ldd)
{ return batch_apply(orc_vtm_csr, m, n, m, n, ptr, idx, val, k, V, ldv, U, ldu, D, ldd); }

/* ------------------------------------------------------------------------ */
/* Value storage precision.  Round a binary64 value once, to nearest with    */
/* ties to even, into a binary format with `p` significand bits (implicit    */
/* bit included) and minimum normal exponent `emin`; the result is returned  */
/* as the binary64 number it represents.  Binary32: p = 24, emin = -126.     */
/* bfloat16: p = 8, emin = -126.  Values beyond the largest finite number of */
/* the format round to +-inf; inputs are assumed finite.                     */
/* ------------------------------------------------------------------------ */
double orc_round_bits(double x, int p, int emin, int emax)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(fabs(x), &e);          /* |x| = f * 2^e, f in [0.5, 1) => exponent e-1 */
    int ex = e - 1;
    if (ex < emin) ex = emin;    /* subnormal range: fixed quantum */
    double q = ldexp(1.0, ex - (p - 1)); /* spacing of the target format near x */
    double r = nearbyint(x / q) * q;     /* x/q is exact (power-of-two scaling); RNE */
    double maxf = ldexp(2.0 - ldexp(1.0, -(p - 1)), emax);
    if (fabs(r) > maxf) r = copysign(INFINITY, x);
    return r;
}

void orc_round_array(const double *in, double *out, int64_t len, int p, int emin, int emax)
{
    for (int64_t i = 0; i < len; ++i) out[i] = orc_round_bits(in[i], p, emin, emax);
}

/* ------------------------------------------------------------------------ */
/* Nonzero partitioning (Section II).                                        */
/* Groups are contiguous in storage order.  Paper rule: the first Z mod P    */
/* groups hold ceil(Z/P) nonzeros, the rest floor(Z/P).  off has P+1 entries. */
/* ------------------------------------------------------------------------ */
void orc_offsets_paper(int64_t Z, int64_t P, int64_t *off)
{
    int64_t big = Z % P, q = Z / P;
    off[0] = 0;
    for (int64_t i = 0; i < P; ++i) off[i + 1] = off[i] + (i < big ? q + 1 : q);
}

/* Fixed-size rule: group c holds positions [c*C, min((c+1)*C, Z)).  Returns the
 * number of groups G = ceil(Z/C) and fills off[0..G]. */
int64_t orc_offsets_fixed(int64_t Z, int64_t C, int64_t *off)
{
    int64_t G = (Z + C - 1) / C;
    for (int64_t c = 0; c <= G; ++c) off[c] = (c * C < Z) ? c * C : Z;
    return G;
}

/* Column of every stored position: colOf[p] = j for p in [ptr[j], ptr[j+1]). */
static int64_t *column_of_positions(int64_t n, const int64_t *ptr)
{
    int64_t Z = ptr[n];
    int64_t *col = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Z > 0 ? Z : 1));
    if (!col) return NULL;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t p = ptr[j]; p < ptr[j + 1]; ++p) col[p] = j;
    return col;
}

/* First and last column of each group's cover set J_i: the columns holding
 * the group's first and last nonzero.  Every group must be non-empty. */
int orc_cover(int64_t n, const int64_t *ptr, int64_t P, const int64_t *off, int64_t *jf, int64_t *jl)
{
    int64_t *col = column_of_positions(n, ptr);
    if (!col) return -1;
    for (int64_t i = 0; i < P; ++i) {
        if (off[i + 1] <= off[i]) { free(col); return -2; }
        jf[i] = col[off[i]];
        jl[i] = col[off[i + 1] - 1];
    }
    free(col);
    return 0;
}

/* Overlap zones from their definition: a column is a zone when two or more
 * groups hold a nonzero of it; S_k is the set of those groups, which is a run
 * of consecutive groups because groups are contiguous in storage order.
 * Writes zone columns zcol[k] and the first/last group sfirst[k], slast[k]
 * (arrays sized >= P); returns z.  Computed by walking every position. */
int64_t orc_zones(int64_t n, const int64_t *ptr, int64_t P, const int64_t *off,
                  int64_t *zcol, int64_t *sfirst, int64_t *slast)
{
    int64_t *col = column_of_positions(n, ptr);
    if (!col && ptr[n] > 0) return -1;
    /* For each column: the first and last group that touches it. */
    int64_t *gfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *glast = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!gfirst || !glast) { free(col); free(gfirst); free(glast); return -1; }
    for (int64_t j = 0; j < n; ++j) { gfirst[j] = -1; glast[j] = -1; }
    for (int64_t g = 0; g < P; ++g) {
        for (int64_t p = off[g]; p < off[g + 1]; ++p) {
            int64_t j = col[p];
            if (gfirst[j] < 0) gfirst[j] = g;
            glast[j] = g;
        }
    }
    int64_t z = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (gfirst[j] >= 0 && glast[j] > gfirst[j]) {
            zcol[z] = j; sfirst[z] = gfirst[j]; slast[z] = glast[j]; ++z;
        }
    }
    free(col); free(gfirst); free(glast);
    return z;
}

/* The segmented addition of Section IV-B on integer pairs:
 *   (s,k) o (t,l) = (s+t, l) if k == l, else (t, l). */
static void seg_op(int64_t s, int64_t k, int64_t t, int64_t l, int64_t *rs, int64_t *rk)
{
    if (k == l) { *rs = s + t; *rk = l; }
    else        { *rs = t;     *rk = l; }
}

/* One-time setup of Section IV-B, from jf/jl of the P groups.  Outputs are P
 * entries each.  needLeft/needRight compare first/last columns of neighbours;
 * leftGroupEnd = needLeft and (not needRight or jf != jl); rightGroup is the
 * inclusive additive forward scan of leftGroupEnd; leftGroup = rightGroup -
 * leftGroupEnd; procsOnLeft is the first component of the inclusive forward
 * o-scan of (needLeft, leftGroup); procsOnRight is the first component of the
 * backward o-scan of (needRight, rightGroup), folding from the right so that
 * result_i = result_{i+1} o x_i. */
void orc_setup_vars(int64_t P, const int64_t *jf, const int64_t *jl,
                    int64_t *needLeft, int64_t *needRight, int64_t *leftGroupEnd,
                    int64_t *rightGroup, int64_t *leftGroup,
                    int64_t *procsOnLeft, int64_t *procsOnRight)
{
    for (int64_t i = 0; i < P; ++i) {
        needLeft[i] = (i > 0 && jf[i] == jl[i - 1]) ? 1 : 0;
        needRight[i] = (i < P - 1 && jl[i] == jf[i + 1]) ? 1 : 0;
    }
    for (int64_t i = 0; i < P; ++i)
        leftGroupEnd[i] = (needLeft[i] == 1 && (needRight[i] == 0 || jf[i] != jl[i])) ? 1 : 0;
    int64_t acc = 0;
    for (int64_t i = 0; i < P; ++i) { acc += leftGroupEnd[i]; rightGroup[i] = acc; }
    for (int64_t i = 0; i < P; ++i) leftGroup[i] = rightGroup[i] - leftGroupEnd[i];
    /* forward o-scan */
    int64_t s = 0, k = 0;
    for (int64_t i = 0; i < P; ++i) {
        if (i == 0) { s = needLeft[0]; k = leftGroup[0]; }
        else seg_op(s, k, needLeft[i], leftGroup[i], &s, &k);
        procsOnLeft[i] = s;
    }
    /* backward o-scan */
    for (int64_t i = P - 1; i >= 0; --i) {
        if (i == P - 1) { s = needRight[i]; k = rightGroup[i]; }
        else seg_op(s, k, needRight[i], rightGroup[i], &s, &k);
        procsOnRight[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Serial simulation of the nonzero-partitioned algorithms.                   */
/* ------------------------------------------------------------------------ */

/* Section III: each group computes y_(i) = A_(i) x_(i) over its own positions
 * (missing entries of partial columns are zero), then y = sum_i y_(i) with the
 * groups added in ascending order.  CSC storage. */
int orc_nzp_mv(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
               int64_t P, const int64_t *off, const double *x, double *y)
{
    int64_t *col = column_of_positions(n, ptr);
    double *yi = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if ((!col && ptr[n] > 0) || !yi) { free(col); free(yi); return -1; }
    for (int64_t r = 0; r < m; ++r) y[r] = 0.0;
    for (int64_t g = 0; g < P; ++g) {
        for (int64_t r = 0; r < m; ++r) yi[r] = 0.0;
        for (int64_t p = off[g]; p < off[g + 1]; ++p) {
            double prod = val[p] * x[col[p]];
            yi[idx[p]] = yi[idx[p]] + prod;
        }
        for (int64_t r = 0; r < m; ++r) y[r] = y[r] + yi[r];
    }
    free(col); free(yi);
    return 0;
}

/* Section IV-A: each group computes its local u^p_j = v^T A^p_j for the columns
 * of its cover (storage order within the column); a column held by one group
 * takes that value, a zone column j_k takes the sum over S_k in ascending
 * group order.  Columns with no nonzero are zero.  CSC storage. */
int orc_nzp_vtm(int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
                int64_t P, const int64_t *off, const double *v, double *u)
{
    (void)m;
    int64_t *col = column_of_positions(n, ptr);
    if (!col && ptr[n] > 0) return -1;
    for (int64_t j = 0; j < n; ++j) u[j] = 0.0;
    for (int64_t g = 0; g < P; ++g) {
        int64_t p = off[g];
        while (p < off[g + 1]) {
            int64_t j = col[p];
            double part = 0.0;
            while (p < off[g + 1] && col[p] == j) {
                double prod = val[p] * v[idx[p]];
                part = part + prod;
                ++p;
            }
            /* the first group to touch column j stores its part; later groups
             * of the same zone add theirs, in ascending group order */
            if (g > 0 && off[g] > ptr[j]) u[j] = u[j] + part;
            else u[j] = part;
        }
    }
    free(col);
    return 0;
}

/* Column partitioning comparison statistic (Section VI): with the columns cut
 * into P contiguous spans of (almost) equal column count, the imbalance
 * Delta = P (max - min nonzeros per span) / Z.  Span i holds columns
 * [i*n/P, (i+1)*n/P) using the same first-n-mod-P-get-one-more rule. */
double orc_colp_imbalance(int64_t n, const int64_t *ptr, int64_t P)
{
    int64_t Z = ptr[n];
    if (Z == 0 || P <= 0) return 0.0;
    int64_t big = n % P, q = n / P, j0 = 0, mx = -1, mn = -1;
    for (int64_t i = 0; i < P; ++i) {
        int64_t j1 = j0 + (i < big ? q + 1 : q);
        int64_t cnt = ptr[j1] - ptr[j0];
        if (mx < 0 || cnt > mx) mx = cnt;
        if (mn < 0 || cnt < mn) mn = cnt;
        j0 = j1;
    }
    return (double)P * (double)(mx - mn) / (double)Z;
}

/* ------------------------------------------------------------------------ */
/* CGLS (Section VII's first-order use of the two products).  A is m x n, wide */
/* CSC (csr = 0) or tall CSR (csr = 1).  x holds x_0 on entry and x_iters on  */
/* exit.  hist_gamma[k] = ||A^T r_k||^2 and hist_rho[k] = ||r_k||^2 for        */
/* k = 0 .. iters (either may be NULL).  An exact zero in a denominator (the  */
/* iterate already solves the normal equations) makes that step size zero.    */
/* Returns 0, or -1 when out of memory.                                       */
/* ------------------------------------------------------------------------ */
static double dot_seq(const double *a, const double *b, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s = s + a[i] * b[i];
    return s;
}

int orc_cgls(int csr, int64_t m, int64_t n, const int64_t *ptr, const int32_t *idx, const double *val,
             const double *b, double *x, int64_t iters, double *hist_gamma, double *hist_rho)
{
    double *r = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double *q = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double *s = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *p = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!r || !q || !s || !p) { free(r); free(q); free(s); free(p); return -1; }
#define ORC_MV(in, out) (csr ? orc_mv_csr(m, n, ptr, idx, val, in, out, NULL) : orc_mv_csc(m, n, ptr, idx, val, in, out, NULL))
#define ORC_VTM(in, out) (csr ? orc_vtm_csr(m, n, ptr, idx, val, in, out, NULL) : orc_vtm_csc(m, n, ptr, idx, val, in, out, NULL))
    /* r_0 = b - A x_0,  s_0 = A^T r_0,  p_0 = s_0,  gamma_0 = ||s_0||^2 */
    ORC_MV(x, q);
    for (int64_t i = 0; i < m; ++i) r[i] = b[i] - q[i];
    ORC_VTM(r, s);
    for (int64_t j = 0; j < n; ++j) p[j] = s[j];
    double gamma = dot_seq(s, s, n);
    if (hist_gamma) hist_gamma[0] = gamma;
    if (hist_rho) hist_rho[0] = dot_seq(r, r, m);
    for (int64_t k = 0; k < iters; ++k) {
        ORC_MV(p, q);                                   /* q_k = A p_k */
        const double delta = dot_seq(q, q, m);
        const double alpha = (gamma > 0.0 && delta > 0.0) ? gamma / delta : 0.0;
        for (int64_t j = 0; j < n; ++j) x[j] = x[j] + alpha * p[j];
        for (int64_t i = 0; i < m; ++i) r[i] = r[i] - alpha * q[i];
        ORC_VTM(r, s);                                  /* s_{k+1} = A^T r_{k+1} */
        const double gamma_new = dot_seq(s, s, n);
        const double beta = gamma > 0.0 ? gamma_new / gamma : 0.0;
        for (int64_t j = 0; j < n; ++j) p[j] = s[j] + beta * p[j];
        gamma = gamma_new;
        if (hist_gamma) hist_gamma[k + 1] = gamma;
        if (hist_rho) hist_rho[k + 1] = dot_seq(r, r, m);
    }
#undef ORC_MV
#undef ORC_VTM
    free(r); free(q); free(s); free(p);
    return 0;
}

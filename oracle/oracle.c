/*
 * FP64 CPU oracle for the BiCGSafe family of Huynh & Suito,
 * "Communication-hiding pipelined BiCGSafe methods for solving large linear
 * systems" (arXiv 2108.10591).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header or constant with the GPU library.
 *
 * Conventions (kept deliberately simple so the code can be checked against
 * the paper by eye):
 *   - every vector statement is one plain loop over all n entries;
 *   - an inner product is the exact sum of the products rounded once (see
 *     dot() below), so its value does not depend on any summation order;
 *   - a sparse product y = A x is, per row, a sequential sum of the rounded
 *     products over the row's entries in storage order, carried with the
 *     same compensated summation (see spmv() below);
 *   - compiled with -ffp-contract=off, so no fused multiply-adds.
 *
 * Variants:
 *   0  ssBiCGSafe2            Algorithm 3 (Section 2)
 *   1  p-BiCGSafe             Algorithm 4 (Section 3)
 *   2  p-BiCGSafe-rr          Algorithm 5 (Section 4)
 *   3  p-BiCGStab             pipelined BiCGStab of Cools & Vanroose, cited in
 *                             the introduction and Table 1 but not printed;
 *                             derived here from BiCGStab (Algorithm 1) by the
 *                             auxiliary definitions given below
 *   4  BiCGStab               Algorithm 1 (Section 2), with omega written for
 *                             the coefficient the listing calls zeta
 *
 * Precision (argument `precision` of orc_setup, orc_run and orc_solve): the
 * mixed-precision forms keep every vector, inner product, coefficient and the
 * stop test in FP64 and change only the matrix values a product reads:
 *   0  the given FP64 values everywhere;
 *   1  every product reads the values rounded to the nearest FP32 number (ties
 *      to even) and widened back, so the system solved is that rounded matrix;
 *   2  the residual statements -- r_0 = b - A x_0 at set-up and the true
 *      residual r_{i+1} = b - A x_{i+1} of a replacement step (Algorithm 5,
 *      Section 4) -- read the FP64 values, every other product the rounded
 *      ones, so the replacement steps re-anchor the iteration to the FP64
 *      system (R23);
 *   3  as 2, and the search directions p_i, u_i and the auxiliary vector z_i
 *      of p-BiCGSafe(-rr) are held as FP32 numbers: each is rounded to the
 *      nearest FP32 number (ties to even) when it is formed and widened
 *      exactly when it is read, so all arithmetic stays FP64 (R24).
 *
 * Initial guess (argument `x0_mode` of orc_setup and orc_solve; with x0 given):
 *   0  x_0 as given;
 *   1  kept only if ||b - A x_0|| <= ||b||, else x_0 = 0 (a guess worse than
 *      zero costs nothing);
 *   2  first scaled by the factor c = (A x_0, b) / (A x_0, A x_0) that
 *      minimises ||b - c A x_0|| (x_0 = 0 when c cannot be formed), then the
 *      rule of 1.
 *   The products of these tests are residual statements (FP64 values under
 *   precision 2 and 3).
 *
 * Threads: every vector statement and every row of a sparse product is
 * computed independently of the others, and an inner product is an exact
 * integer sum, so the results do not depend on the number of OpenMP threads.
 *
 * Readings of points the paper leaves open (each is used below):
 *   R1  the shadow residual is r0* = r0, fixed for the whole solve.
 *   R2  Algorithms 4/5 use s_0 without computing it; s_0 = A r_0 by its
 *       definition s_i := A r_i (Section 3), one extra product at setup.
 *   R3  vectors with index -1 (and y_0, g_0) start at zero.
 *   R4  the i = 0 branch is special-cased as printed.
 *   R5  the stop test is taken before the coefficients are formed (the
 *       listings form them first); this changes nothing on iterations that
 *       continue and avoids 0/0 when r_i is exactly zero.
 *   R6  iters = the number of x updates made; hist[i] = sqrt(rho_i)/sqrt(rho_ref),
 *       rho_i = (r_i, r_i) of the recursively updated residual.
 *   R7  Algorithm 5 computes "A t_{i+1}" but assigns l_i = A t_i; t_{i+1}
 *       does not exist yet, so l_i = A t_i.
 *   R9  the replacement cut-off M defaults to maxit.
 *   R10 a zero or non-finite denominator in alpha, beta, zeta, eta (or
 *       omega's successor) stops the solve with status BREAKDOWN and x_i.
 *   R23 mixed precision (precision 1, 2) rounds only the matrix values; the
 *       paper's experiments are FP64 throughout (Section 5).
 *   R24 precision 3 also stores p, u and z in FP32 (the vectors whose
 *       rounding leaves the recurrences of Section 3 consistent with A).
 *
 * Status codes: 0 converged, 1 maxit, 2 breakdown, 3 non-finite inner product.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* vectors shorter than this are processed by one thread (thread start-up
   would cost more than the work) */
#define ORC_PAR_MIN 32768

/* vector slots in the caller-provided state array V[NV][n] */
enum {
  VX = 0, VR, VRS, VS, VY, VT, VP, VU, VZ, VW, VL, VG, VQ, VO, VAS, VAW, VV, VTMP,
  NV
};
/* scalar slots in the caller-provided array S[NS] */
enum {
  S_ALPHA = 0, S_BETA, S_ZETA, S_ETA, S_OMEGA, S_F, S_RHOREF, S_RHO,
  S_NSPMV, S_NDOT, S_NPHASE, S_PENDING_BREAKDOWN,
  S_GS, S_GW, S_GZ, /* p-BiCGStab: (r*, s), (r*, w), (r*, z) of the last phase */
  NS
};
enum { ST_CONVERGED = 0, ST_MAXIT = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3, ST_RUNNING = -1 };
enum { V_SSBICGSAFE2 = 0, V_PBICGSAFE = 1, V_PBICGSAFE_RR = 2, V_PBICGSTAB = 3, V_BICGSTAB = 4 };

typedef struct {
  int64_t n;
  const int64_t *rowptr;
  const int32_t *col;
  const double *val;
} csr_t;

/* ---------------------------------------------------------------- kernels */

/*
 * (s, c) += v: Knuth's two-sum splits s + v exactly into the rounded sum and its
 * error; the error is added to c.  s + c then carries a running sum to about
 * twice the working precision.
 */
static void two_sum_acc(double *s, double *c, double v) {
  const double t = *s + v;
  const double z = t - *s;
  const double e = (*s - (t - z)) + (v - z);
  *s = t;
  *c = *c + e;
}

/* y = A x (the "matrix-vector product" of every listing): for each row, the
   rounded products a_ij x_j in storage order, summed with two_sum_acc and
   rounded once, so that the row's value does not depend on the order in which
   its products are added */
static void spmv(const csr_t *A, const double *x, double *y, double *S) {
#pragma omp parallel for schedule(static) if (A->n >= ORC_PAR_MIN)
  for (int64_t i = 0; i < A->n; ++i) {
    double s = 0.0, c = 0.0;
    for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) two_sum_acc(&s, &c, A->val[k] * x[A->col[k]]);
    y[i] = s + c;
  }
  S[S_NSPMV] += 1.0;
}

/*
 * Exact summation of doubles in a long fixed-point accumulator, used for the
 * inner products.  Every finite double is an integer multiple of 2^-1074, so
 * a sum of doubles is an integer in units of 2^-1074.  The accumulator holds
 * that integer in base 2^32: digit i carries weight 2^(32 i) units, and each
 * digit is an int64_t, so a digit can take more than 2^30 additions of
 * magnitude below 2^32 before carries must be propagated.  Adding is exact
 * integer arithmetic; the only rounding is the final one, to the nearest
 * double with ties to even.
 */
#define XDIG 72          /* 72 * 32 bits > 2098 bit positions of the doubles + carries */
#define XNORM (1 << 29)  /* additions between carry propagations */
typedef struct {
  int64_t d[XDIG];
  int64_t adds;
} xsum_t;

/* carry every digit into the next: digits 0..XDIG-2 end in [0, 2^32) */
static void xsum_carry(xsum_t *X) {
  for (int i = 0; i < XDIG - 1; ++i) {
    const int64_t c = X->d[i] >> 32; /* floor division by 2^32 */
    X->d[i] -= c * ((int64_t)1 << 32);
    X->d[i + 1] += c;
  }
  X->adds = 0;
}

static void xsum_add(xsum_t *X, double x) {
  if (x == 0.0) return;
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  const int bexp = (int)((bits >> 52) & 0x7FF);
  uint64_t m = bits & (((uint64_t)1 << 52) - 1);
  int pos; /* x = +-m * 2^(pos - 1074) */
  if (bexp == 0) {
    pos = 0; /* subnormal: m * 2^-1074 */
  } else {
    m |= (uint64_t)1 << 52;
    pos = bexp - 1;
  }
  const int i = pos / 32, sh = pos % 32;
  const unsigned __int128 w = (unsigned __int128)m << sh; /* at most 85 bits */
  const int64_t w0 = (int64_t)(uint64_t)(w & 0xFFFFFFFFu);
  const int64_t w1 = (int64_t)(uint64_t)((w >> 32) & 0xFFFFFFFFu);
  const int64_t w2 = (int64_t)(uint64_t)(w >> 64);
  if (bits >> 63) {
    X->d[i] -= w0; X->d[i + 1] -= w1; X->d[i + 2] -= w2;
  } else {
    X->d[i] += w0; X->d[i + 1] += w1; X->d[i + 2] += w2;
  }
  if (++X->adds == XNORM) xsum_carry(X);
}

/* the double nearest to the accumulated integer (ties to even); +-inf beyond
   the double range */
static double xsum_round(xsum_t *X) {
  xsum_carry(X);
  int neg = X->d[XDIG - 1] < 0;
  if (neg) { /* work with the magnitude */
    for (int i = 0; i < XDIG; ++i) X->d[i] = -X->d[i];
    xsum_carry(X);
  }
  int t = XDIG - 1;
  while (t >= 0 && X->d[t] == 0) --t;
  if (t < 0) return 0.0;
  /* the top three digits as one integer, and whether anything lies below them */
  unsigned __int128 M = 0;
  for (int i = t; i >= t - 2; --i) M = (M << 32) | (uint64_t)(i >= 0 ? X->d[i] : 0);
  int sticky = 0;
  for (int i = t - 3; i >= 0; --i) sticky |= X->d[i] != 0;
  int scale = 32 * (t - 2) - 1074; /* the value is (M + below) * 2^scale */
  int len = 0;
  for (unsigned __int128 v = M; v != 0; v >>= 1) ++len;
  if (len > 53) {
    const int drop = len - 53;
    const unsigned __int128 rem = M & ((((unsigned __int128)1) << drop) - 1);
    const unsigned __int128 half = ((unsigned __int128)1) << (drop - 1);
    M >>= drop;
    scale += drop;
    if (rem > half || (rem == half && (sticky || (M & 1)))) {
      M += 1;
      if (M >> 53) { M >>= 1; scale += 1; }
    }
  } /* else: the integer has at most 53 bits and nothing below them -- exact */
  const double r = ldexp((double)(uint64_t)M, scale);
  return neg ? -r : r;
}

/*
 * (u, v): the inner product rounded once from its exact value (to nearest,
 * ties to even).  Each product u_k v_k is exactly p + ep (p rounded, ep its
 * error from one FMA), and all of these are summed exactly.  The value is
 * thus the plain definition of the inner product in floating point, and it
 * does not depend on any order of summation.  A non-finite product (or a sum
 * beyond the double range) makes the result NaN.  The split is exact while
 * the product's error is representable, i.e. for products above about
 * 2^-969; below that, far from any value a solve produces, ep is the error
 * rounded to the subnormal grid.
 */
static double dot(int64_t n, const double *u, const double *v, double *S) {
  xsum_t X;
  memset(&X, 0, sizeof X);
  int finite = 1;
#pragma omp parallel if (n >= ORC_PAR_MIN)
  {
    /* each thread sums its share exactly; the shares are added digit by digit,
       which is exact integer addition, so the thread count changes nothing */
    xsum_t T;
    memset(&T, 0, sizeof T);
    int fin = 1;
#pragma omp for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
      const double p = u[k] * v[k];
      if (!isfinite(p)) fin = 0;
      if (!fin) continue;
      xsum_add(&T, p);
      xsum_add(&T, fma(u[k], v[k], -p)); /* u_k v_k = p + ep exactly */
    }
    xsum_carry(&T);
#pragma omp critical(orc_dot_merge)
    {
      for (int i = 0; i < XDIG; ++i) X.d[i] += T.d[i];
      finite = finite && fin;
    }
  }
  S[S_NDOT] += 1.0;
  if (!finite) return NAN;
  const double r = xsum_round(&X);
  return isfinite(r) ? r : NAN;
}

static int bad(double d) { return d == 0.0 || !isfinite(d); }

/* ----------------------------------------------------------- entry points */

/* The matrices of a solve at `precision` (see the header): Ak for the Krylov
   products, Ar for the residual statements.  *rounded receives the rounded
   copy of the values (to be freed), or NULL. */
static int precision_pair(int precision, const csr_t *A, csr_t *Ak, csr_t *Ar, double **rounded) {
  *rounded = NULL;
  *Ak = *A;
  *Ar = *A;
  if (precision == 0) return 0;
  if (precision < 1 || precision > 3) return -1;
  const int64_t nnz = A->rowptr[A->n];
  double *v = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  if (!v) return -2;
  for (int64_t k = 0; k < nnz; ++k) v[k] = (double)(float)A->val[k];
  Ak->val = v;
  if (precision == 1) Ar->val = v;
  *rounded = v;
  return 0;
}

/* A vector entry as stored: FP64, or (f32 != 0: precision 3's p, u, z) the
   nearest FP32 number, widened exactly */
static double held(int f32, double v) { return f32 ? (double)(float)v : v; }

/*
 * Initialise the state for `variant` (the steps before each listing's loop).
 * V holds NV vectors of length n (zeroed here); S holds NS scalars.
 * x0 may be NULL (zero initial guess); x0_mode as in the header.  norm_ref
 * selects the stop-test scale: 0 = ||r_0|| (the paper's criterion, Section 5),
 * 1 = ||b||.
 */
int orc_setup(int variant, int precision, int64_t n, const int64_t *rowptr, const int32_t *col,
              const double *val, const double *b, const double *x0, int x0_mode, int norm_ref,
              double *V, double *S) {
  if (x0_mode < 0 || x0_mode > 2) return -1;
  if (precision == 3 && variant != V_PBICGSAFE && variant != V_PBICGSAFE_RR) return -1;
  const csr_t A64 = {n, rowptr, col, val};
  csr_t A, Ares;
  double *rounded;
  const int rc = precision_pair(precision, &A64, &A, &Ares, &rounded);
  if (rc) return rc;
  double *v[NV];
  for (int k = 0; k < NV; ++k) v[k] = V + (size_t)k * (size_t)n;
  memset(V, 0, sizeof(double) * (size_t)NV * (size_t)n);   /* R3: everything starts at zero */
  memset(S, 0, sizeof(double) * NS);
  double *x = v[VX], *r = v[VR], *rs = v[VRS], *tmp = v[VTMP];

  /* x_0 */
  for (int64_t k = 0; k < n; ++k) x[k] = x0 ? x0[k] : 0.0;
  if (x0 && x0_mode == 2) {
    /* the multiple c x_0 with the least residual: c = (A x_0, b) / (A x_0, A x_0) */
    spmv(&Ares, x, tmp, S);
    const double num = dot(n, tmp, b, S), den = dot(n, tmp, tmp, S);
    S[S_NDOT] -= 2.0; /* not inner products of the method */
    const double c = num / den;
    const int ok = den != 0.0 && isfinite(c);
    for (int64_t k = 0; k < n; ++k) x[k] = ok ? c * x[k] : 0.0;
  }
  /* r_0 = b - A x_0 */
  spmv(&Ares, x, tmp, S);
  for (int64_t k = 0; k < n; ++k) r[k] = b[k] - tmp[k];
  if (x0 && x0_mode >= 1) {
    /* a guess whose residual exceeds ||b|| (or is not finite) is replaced by 0 */
    const double rr = dot(n, r, r, S), bb = dot(n, b, b, S);
    S[S_NDOT] -= 2.0;
    if (!(rr <= bb)) {
      for (int64_t k = 0; k < n; ++k) x[k] = 0.0;
      for (int64_t k = 0; k < n; ++k) r[k] = b[k]; /* b - A 0 */
    }
  }
  /* R1: r0* = r0 */
  for (int64_t k = 0; k < n; ++k) rs[k] = r[k];

  if (variant == V_PBICGSAFE || variant == V_PBICGSAFE_RR) {
    spmv(&A, r, v[VS], S);                       /* R2: s_0 = A r_0 */
  }
  if (variant == V_PBICGSTAB) {
    /* w_0 = A r_0, t_0 = A w_0, alpha_0 = (r0*, r_0)/(r0*, w_0), rho_0 = (r_0, r_0) */
    spmv(&A, r, v[VW], S);
    spmv(&A, v[VW], v[VT], S);
    double f = dot(n, rs, r, S);
    double rsw = dot(n, rs, v[VW], S);
    double rho = dot(n, r, r, S);
    S[S_NPHASE] += 1.0;
    S[S_F] = f;
    S[S_RHO] = rho;
    S[S_GW] = rsw;
    if (bad(rsw) || !isfinite(f / rsw)) S[S_PENDING_BREAKDOWN] = 1.0;
    else S[S_ALPHA] = f / rsw;
    S[S_BETA] = 0.0;
    S[S_OMEGA] = 0.0;
  }
  if (variant == V_BICGSTAB) {
    S[S_BETA] = 0.0;
  }
  /* reference norm for the stop test */
  if (norm_ref == 1) S[S_RHOREF] = dot(n, b, b, S), S[S_NDOT] -= 1.0;
  else S[S_RHOREF] = dot(n, r, r, S), S[S_NDOT] -= 1.0;
  free(rounded);
  return 0;
}

/* hist[i] and the stop test shared by every variant: returns a status or ST_RUNNING */
static int stop_test(double rho, double *S, int64_t i, int64_t maxit, double tol, double *hist) {
  double ref = sqrt(S[S_RHOREF]);
  double nr = sqrt(rho);
  if (hist) hist[i] = ref > 0.0 ? nr / ref : 0.0;
  if (nr <= tol * ref) return ST_CONVERGED;                 /* R14: "<=" */
  if (i >= maxit) return ST_MAXIT;
  return ST_RUNNING;
}

/* coefficient record per iteration: alpha, beta, zeta, eta, omega, rho, f, spare */
#define NCOEF 8
static void record(double *coef, int64_t i, double al, double be, double ze, double et, double om,
                   double rho, double f) {
  if (!coef) return;
  double *c = coef + (size_t)i * NCOEF;
  c[0] = al; c[1] = be; c[2] = ze; c[3] = et; c[4] = om; c[5] = rho; c[6] = f; c[7] = 0.0;
}

/*
 * The nine inner products of the single reduction phase (Algorithms 3-5):
 *   a = (s,s), b = (y,y), c = (s,y), d = (s,r), e = (y,r),
 *   f = (r0*,r), g^ = (r0*,s), h = (r0*,t_{i-1}), rho = (r,r).
 * At i = 0 only a, d, f, g^ and rho are formed.
 * Then the stop test and the coefficients beta, alpha, zeta, eta.
 * Returns a status, or ST_RUNNING to continue with the updates.
 */
static int safe_phase(int64_t n, double **v, double *S, int64_t i, int64_t maxit, double tol,
                      double *hist, double *coef) {
  const double *s = v[VS], *y = v[VY], *r = v[VR], *rs = v[VRS], *t = v[VT];
  double a, bb = 0, c = 0, d, e = 0, f, gh, h = 0, rho;
  if (i == 0) {
    a = dot(n, s, s, S);
    d = dot(n, s, r, S);
    f = dot(n, rs, r, S);
    gh = dot(n, rs, s, S);
    rho = dot(n, r, r, S);
  } else {
    a = dot(n, s, s, S);
    bb = dot(n, y, y, S);
    c = dot(n, s, y, S);
    d = dot(n, s, r, S);
    e = dot(n, y, r, S);
    f = dot(n, rs, r, S);
    gh = dot(n, rs, s, S);
    h = dot(n, rs, t, S);
    rho = dot(n, r, r, S);
  }
  S[S_NPHASE] += 1.0;
  S[S_RHO] = rho;
  if (!(isfinite(a) && isfinite(bb) && isfinite(c) && isfinite(d) && isfinite(e) && isfinite(f) &&
        isfinite(gh) && isfinite(h) && isfinite(rho))) {
    if (hist) hist[i] = NAN;
    return ST_NONFINITE;
  }
  int st = stop_test(rho, S, i, maxit, tol, hist);
  if (st != ST_RUNNING) return st;

  double beta, alpha, zeta, eta;
  if (i == 0) {
    if (bad(gh) || bad(a)) return ST_BREAKDOWN;
    beta = 0.0;
    alpha = f / gh;
    zeta = d / a;
    eta = 0.0;
  } else {
    /* previous iteration's alpha, zeta, f are still in S */
    double den_beta = S[S_ZETA] * S[S_F];
    if (bad(den_beta)) return ST_BREAKDOWN;
    beta = (S[S_ALPHA] * f) / den_beta;
    double den_alpha = gh + beta * h;
    double den_ze = a * bb - c * c;
    if (bad(den_alpha) || bad(den_ze)) return ST_BREAKDOWN;
    alpha = f / den_alpha;
    zeta = (bb * d - c * e) / den_ze;
    eta = (a * e - c * d) / den_ze;
  }
  if (!isfinite(beta) || !isfinite(alpha) || !isfinite(zeta) || !isfinite(eta)) return ST_BREAKDOWN;
  S[S_ALPHA] = alpha;
  S[S_BETA] = beta;
  S[S_ZETA] = zeta;
  S[S_ETA] = eta;
  S[S_F] = f;
  record(coef, i, alpha, beta, zeta, eta, 0.0, rho, f);
  return ST_RUNNING;
}

/*
 * ssBiCGSafe2, Algorithm 3: one iteration i.  After the reduction phase the
 * updates fall into two row-local groups around the product A u_i:
 *   directions   p_i = r_i + beta (p_{i-1} - u_{i-1}),  u_i = zeta o_i + eta (y_i + beta u_{i-1}),
 *                with o_i = s_i + beta t_{i-1} (kept for t_i and r_{i+1});
 *   residuals    t_i = o_i - w_i,  z_i = zeta r_i + eta z_{i-1} - alpha u_i,
 *                y_{i+1} = zeta s_i + eta y_i - alpha w_i,  x_{i+1} = x_i + alpha p_i + z_i,
 *                r_{i+1} = r_i - alpha o_i - y_{i+1}   (w_i = A u_i).
 */
static int iter_ssbicgsafe2(const csr_t *A, double **v, double *S, int64_t i, int64_t maxit,
                            double tol, double *hist, double *coef) {
  int64_t n = A->n;
  double *x = v[VX], *r = v[VR], *s = v[VS], *y = v[VY], *t = v[VT], *p = v[VP], *u = v[VU];
  double *z = v[VZ], *w = v[VW], *o = v[VO];
  spmv(A, r, s, S);                                        /* s_i = A r_i */
  int st = safe_phase(n, v, S, i, maxit, tol, hist, coef);
  if (st != ST_RUNNING) return st;
  const double al = S[S_ALPHA], be = S[S_BETA], ze = S[S_ZETA], et = S[S_ETA];
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    o[k] = s[k] + be * t[k];
    p[k] = r[k] + be * (p[k] - u[k]);
    u[k] = ze * o[k] + et * (y[k] + be * u[k]);
  }
  spmv(A, u, w, S);                                        /* w_i = A u_i */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    t[k] = o[k] - w[k];
    z[k] = ze * r[k] + et * z[k] - al * u[k];
    y[k] = ze * s[k] + et * y[k] - al * w[k];
    x[k] = x[k] + al * p[k] + z[k];
    r[k] = r[k] - al * o[k] - y[k];
  }
  return ST_RUNNING;
}

/*
 * p-BiCGSafe, Algorithm 4, and p-BiCGSafe-rr, Algorithm 5: one iteration i.
 * The product A s_i does not depend on the reduction phase (Section 3), which
 * is what the pipelining overlaps.  The updates are the directions and
 * residuals of Algorithm 3, with the products A o_i and A u_i replaced by the
 * recurrences Eq. (q) q_i = As_i + beta l_{i-1} and Eq. (w)
 * w_i = zeta q_i + eta (g_i + beta w_{i-1}), and after A w_i the recurrences
 * Eq. (l) l_i = q_i - A w_i, Eq. (g) g_{i+1} = zeta As_i + eta g_i - alpha A w_i
 * and Eq. (sip1) s_{i+1} = s_i - alpha q_i - g_{i+1}.  A replacement step of
 * Algorithm 5 forms q_i, w_i, r_{i+1}, l_i, g_{i+1}, s_{i+1} as true products
 * instead.  f32v (precision 3): p, u, z are held as FP32 numbers.
 */
static int iter_pbicgsafe(const csr_t *A, const csr_t *Ares, const double *b, double **v,
                          double *S, int64_t i, int64_t maxit, double tol, int rr, int64_t m,
                          int64_t M, int f32v, double *hist, double *coef) {
  int64_t n = A->n;
  double *x = v[VX], *r = v[VR], *s = v[VS], *y = v[VY], *t = v[VT], *p = v[VP], *u = v[VU];
  double *z = v[VZ], *w = v[VW], *l = v[VL], *g = v[VG], *q = v[VQ], *o = v[VO];
  double *As = v[VAS], *Aw = v[VAW], *tmp = v[VTMP];
  spmv(A, s, As, S);                                       /* As_i (overlapped in the paper) */
  int st = safe_phase(n, v, S, i, maxit, tol, hist, coef);
  if (st != ST_RUNNING) return st;
  const double al = S[S_ALPHA], be = S[S_BETA], ze = S[S_ZETA], et = S[S_ETA];
  const int replace = rr && m > 0 && (i % m == 0) && i > 0 && i < M;

  /* directions, and unless replacing, q_i and w_i by Eqs. (q), (w) */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    o[k] = s[k] + be * t[k];
    p[k] = held(f32v, r[k] + be * (p[k] - u[k]));
    u[k] = held(f32v, ze * o[k] + et * (y[k] + be * u[k]));
    if (!replace) {
      q[k] = As[k] + be * l[k];
      w[k] = ze * q[k] + et * (g[k] + be * w[k]);
    }
  }
  if (replace) {
    spmv(A, o, q, S);                                      /* q_i = A o_i */
    spmv(A, u, w, S);                                      /* w_i = A u_i */
  }
  /* residuals and the iterate; r_{i+1} by its recurrence unless replacing */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    t[k] = o[k] - w[k];
    z[k] = held(f32v, ze * r[k] + et * z[k] - al * u[k]);
    y[k] = ze * s[k] + et * y[k] - al * w[k];
    x[k] = x[k] + al * p[k] + z[k];
    if (!replace) r[k] = r[k] - al * o[k] - y[k];
  }
  if (replace) {
    spmv(Ares, x, tmp, S);                                 /* A x_{i+1} (precision 2, 3: FP64) */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t k = 0; k < n; ++k) r[k] = b[k] - tmp[k];  /* r_{i+1} = b - A x_{i+1} */
    spmv(A, t, l, S);                                      /* R7: l_i = A t_i */
    spmv(A, y, g, S);                                      /* g_{i+1} = A y_{i+1} */
    spmv(A, r, s, S);                                      /* s_{i+1} = A r_{i+1} */
  } else {
    spmv(A, w, Aw, S);                                     /* Aw_i */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int64_t k = 0; k < n; ++k) {
      l[k] = q[k] - Aw[k];
      g[k] = ze * As[k] + et * g[k] - al * Aw[k];
      s[k] = s[k] - al * q[k] - g[k];
    }
  }
  return ST_RUNNING;
}

/*
 * p-BiCGStab: one iteration i.  Derived from BiCGStab (Algorithm 1, omega in
 * place of the listing's zeta) by carrying the products
 *     s_i = A p_i,  z_i = A s_i,  w_i = A r_i,  t_i = A w_i,  v_i = A z_i,
 *     q_i = r_i - alpha_i s_i,  y_i = A q_i = w_i - alpha_i z_i
 * as recurrences, so each iteration does two products (v_i = A z_i and
 * t_{i+1} = A w_{i+1}) and two reduction phases of 2 and 5 inner products,
 * each independent of the product next to it (Table 1: 2 products, 7 inner
 * products).  Substituting the definitions:
 *     p_i = r_i + beta_{i-1} (p_{i-1} - omega_{i-1} s_{i-1})
 *     s_i = w_i + beta_{i-1} (s_{i-1} - omega_{i-1} z_{i-1})
 *     z_i = t_i + beta_{i-1} (z_{i-1} - omega_{i-1} v_{i-1})
 *     omega_i = (q_i, y_i) / (y_i, y_i)
 *     x_{i+1} = x_i + alpha_i p_i + omega_i q_i,   r_{i+1} = q_i - omega_i y_i
 *     w_{i+1} = A r_{i+1} = y_i - omega_i (t_i - alpha_i v_i)
 *     beta_i = (alpha_i/omega_i) (r0*, r_{i+1}) / (r0*, r_i)
 *     alpha_{i+1} = (r0*, r_{i+1}) / ((r0*, w_{i+1}) + beta_i (r0*, s_i) - beta_i omega_i (r0*, z_i))
 * where the last denominator is (r0*, A p_{i+1}) expanded by the p recurrence.
 * (y_i, y_i) = 0 means y_i = 0, hence q_i = 0 for nonsingular A: then
 * omega_i = 0, x_{i+1} = x_i + alpha_i p_i and r_{i+1} = q_i; the next stop
 * test decides, and beta_i (which divides by omega_i) is flagged as a
 * breakdown only if the solve has to continue.
 */
static int iter_pbicgstab(const csr_t *A, double **v, double *S, int64_t i, int64_t maxit,
                          double tol, double *hist, double *coef) {
  int64_t n = A->n;
  double *x = v[VX], *r = v[VR], *rs = v[VRS], *s = v[VS], *y = v[VY], *t = v[VT], *p = v[VP];
  double *z = v[VZ], *w = v[VW], *q = v[VQ], *vv = v[VV];
  /* rho_i and the phase that formed alpha_i were computed by the previous iteration (or setup) */
  double rho = S[S_RHO];
  if (!isfinite(rho) || !isfinite(S[S_F]) || !isfinite(S[S_GW]) || !isfinite(S[S_GS]) ||
      !isfinite(S[S_GZ])) {
    if (hist) hist[i] = NAN;
    return ST_NONFINITE;
  }
  int st = stop_test(rho, S, i, maxit, tol, hist);
  if (st != ST_RUNNING) return st;
  if (S[S_PENDING_BREAKDOWN] != 0.0) return ST_BREAKDOWN;
  const double al = S[S_ALPHA], be = S[S_BETA], omp = S[S_OMEGA];

  /* p_i and the products s_i = A p_i, z_i = A s_i by their recurrences; q_i and
     y_i = A q_i */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    p[k] = r[k] + be * (p[k] - omp * s[k]);
    s[k] = w[k] + be * (s[k] - omp * z[k]);
    z[k] = t[k] + be * (z[k] - omp * vv[k]);
    q[k] = r[k] - al * s[k];
    y[k] = w[k] - al * z[k];
  }
  /* phase 1: (q, y), (y, y), overlapped with v_i = A z_i */
  double qy = dot(n, q, y, S);
  double yy = dot(n, y, y, S);
  S[S_NPHASE] += 1.0;
  spmv(A, z, vv, S);                                                       /* v_i = A z_i */
  if (!isfinite(qy) || !isfinite(yy)) return ST_NONFINITE;
  double om = (yy == 0.0) ? 0.0 : qy / yy;
  if (!isfinite(om)) return ST_BREAKDOWN;
  /* the iterate, the residual and w_{i+1} = A r_{i+1} by its recurrence */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    x[k] = x[k] + al * p[k] + om * q[k];
    r[k] = q[k] - om * y[k];
    w[k] = y[k] - om * (t[k] - al * vv[k]);
  }
  /* phase 2: (r0*, r), (r0*, w), (r0*, s), (r0*, z), (r, r), overlapped with t_{i+1} = A w_{i+1} */
  double f = dot(n, rs, r, S);
  double gw = dot(n, rs, w, S);
  double gs = dot(n, rs, s, S);
  double gz = dot(n, rs, z, S);
  double rho1 = dot(n, r, r, S);
  S[S_NPHASE] += 1.0;
  spmv(A, w, t, S);                                                        /* t_{i+1} = A w_{i+1} */
  double beta = 0.0, alpha = 0.0;
  int pend = 0;
  double den_beta = om * S[S_F];
  if (bad(den_beta)) pend = 1;
  else {
    beta = (al * f) / den_beta;
    double den_alpha = gw + beta * gs - beta * om * gz;
    if (bad(den_alpha)) pend = 1;
    else alpha = f / den_alpha;
    if (!isfinite(beta) || !isfinite(alpha)) pend = 1;
  }
  record(coef, i, al, be, 0.0, 0.0, om, rho, S[S_F]);
  S[S_ALPHA] = alpha;
  S[S_BETA] = beta;
  S[S_OMEGA] = om;
  S[S_F] = f;
  S[S_GW] = gw;
  S[S_GS] = gs;
  S[S_GZ] = gz;
  S[S_RHO] = rho1;
  S[S_PENDING_BREAKDOWN] = pend ? 1.0 : 0.0;
  return ST_RUNNING;
}

/* BiCGStab, Algorithm 1 (omega for the listing's zeta): one iteration i.
   Slots: p = VP, Ap = VS, t = VQ (the listing's t_i), At = VY. */
static int iter_bicgstab(const csr_t *A, double **v, double *S, int64_t i, int64_t maxit,
                         double tol, double *hist, double *coef) {
  int64_t n = A->n;
  double *x = v[VX], *r = v[VR], *rs = v[VRS], *p = v[VP], *Ap = v[VS], *t = v[VQ], *At = v[VY];
  double rho = dot(n, r, r, S);
  S[S_NDOT] -= 1.0; /* the norm is not one of the method's counted inner products */
  S[S_RHO] = rho;
  if (!isfinite(rho)) { if (hist) hist[i] = NAN; return ST_NONFINITE; }
  int st = stop_test(rho, S, i, maxit, tol, hist);
  if (st != ST_RUNNING) return st;
  const double be = S[S_BETA], omp = S[S_OMEGA];
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) p[k] = r[k] + be * (p[k] - omp * Ap[k]);  /* p_i */
  spmv(A, p, Ap, S);                                                        /* A p_i */
  double f = dot(n, rs, r, S);
  double rsap = dot(n, rs, Ap, S);
  S[S_NPHASE] += 1.0;
  if (!isfinite(f) || !isfinite(rsap)) return ST_NONFINITE;
  if (bad(rsap)) return ST_BREAKDOWN;
  double al = f / rsap;                                                      /* alpha_i */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) t[k] = r[k] - al * Ap[k];                  /* t_i */
  spmv(A, t, At, S);                                                        /* A t_i */
  double att = dot(n, At, t, S);
  double atat = dot(n, At, At, S);
  S[S_NPHASE] += 1.0;
  if (!isfinite(att) || !isfinite(atat)) return ST_NONFINITE;
  double om = (atat == 0.0) ? 0.0 : att / atat;                             /* omega_i */
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
  for (int64_t k = 0; k < n; ++k) {
    x[k] = x[k] + al * p[k] + om * t[k];                                     /* x_{i+1} */
    r[k] = t[k] - om * At[k];                                                /* r_{i+1} */
  }
  double f1 = dot(n, rs, r, S);
  S[S_NPHASE] += 1.0;
  record(coef, i, al, be, 0.0, 0.0, om, rho, f);
  double beta = 0.0;
  if (om != 0.0 && f != 0.0) beta = (al / om) * (f1 / f);                   /* beta_i */
  S[S_BETA] = beta;
  S[S_OMEGA] = om;
  S[S_ALPHA] = al;
  S[S_F] = f1;
  if ((om == 0.0 || f == 0.0 || !isfinite(beta))) S[S_PENDING_BREAKDOWN] = 1.0;
  return ST_RUNNING;
}

/*
 * Run iterations i = i_begin, i_begin+1, ... from the state (V, S) until a
 * stop.  hist (length >= maxit+1, indexed by i) and coef (NCOEF doubles per
 * iteration) may be NULL.  rr_m / rr_M are the replacement period and cut-off
 * of Algorithm 5 (ignored by the other variants).  On return *iters is the
 * index i at which the solve stopped (= the number of x updates from 0) and
 * V holds the state at the start of that iteration.
 */
int orc_run(int variant, int precision, int64_t n, const int64_t *rowptr, const int32_t *col,
            const double *val, const double *b, double *V, double *S, int64_t i_begin,
            int64_t maxit, double tol, int64_t rr_m, int64_t rr_M, int64_t *iters, double *hist,
            double *coef, int32_t *status) {
  if (precision == 3 && variant != V_PBICGSAFE && variant != V_PBICGSAFE_RR) return -1;
  const csr_t A64 = {n, rowptr, col, val};
  csr_t A, Ares;
  double *rounded;
  const int rc = precision_pair(precision, &A64, &A, &Ares, &rounded);
  if (rc) return rc;
  double *v[NV];
  for (int k = 0; k < NV; ++k) v[k] = V + (size_t)k * (size_t)n;
  int st = ST_RUNNING;
  int64_t i = i_begin;
  for (;; ++i) {
    if (variant == V_BICGSTAB && i > i_begin && S[S_PENDING_BREAKDOWN] != 0.0) {
      /* the previous beta was not finite: only a converged stop may follow */
      double rho = dot(n, v[VR], v[VR], S);
      S[S_NDOT] -= 1.0;
      st = stop_test(rho, S, i, maxit, tol, hist);
      if (st == ST_RUNNING) st = ST_BREAKDOWN;
      break;
    }
    switch (variant) {
      case V_SSBICGSAFE2: st = iter_ssbicgsafe2(&A, v, S, i, maxit, tol, hist, coef); break;
      case V_PBICGSAFE:
        st = iter_pbicgsafe(&A, &Ares, b, v, S, i, maxit, tol, 0, 0, 0, precision == 3, hist,
                            coef);
        break;
      case V_PBICGSAFE_RR:
        st = iter_pbicgsafe(&A, &Ares, b, v, S, i, maxit, tol, 1, rr_m, rr_M, precision == 3,
                            hist, coef);
        break;
      case V_PBICGSTAB: st = iter_pbicgstab(&A, v, S, i, maxit, tol, hist, coef); break;
      case V_BICGSTAB: st = iter_bicgstab(&A, v, S, i, maxit, tol, hist, coef); break;
      default: free(rounded); return -1;
    }
    if (st != ST_RUNNING) break;
  }
  *iters = i;
  *status = st;
  free(rounded);
  return 0;
}

/* setup + run from i = 0; x (length n) receives the final iterate. */
int orc_solve(int variant, int precision, int64_t n, const int64_t *rowptr, const int32_t *col,
              const double *val, const double *b, const double *x0, int x0_mode, double tol,
              int64_t maxit, int64_t rr_m, int64_t rr_M, int norm_ref, double *x, int64_t *iters,
              double *hist, double *coef, int32_t *status, double *counters) {
  if (n < 1 || variant < 0 || variant > 4 || precision < 0 || precision > 3) return -1;
  double *V = (double *)malloc(sizeof(double) * (size_t)NV * (size_t)n);
  double S[NS];
  if (!V) return -2;
  int rc = orc_setup(variant, precision, n, rowptr, col, val, b, x0, x0_mode, norm_ref, V, S);
  if (!rc)
    rc = orc_run(variant, precision, n, rowptr, col, val, b, V, S, 0, maxit, tol, rr_m, rr_M,
                 iters, hist, coef, status);
  if (rc) {
    free(V);
    return rc;
  }
  memcpy(x, V + (size_t)VX * (size_t)n, sizeof(double) * (size_t)n);
  if (counters) { counters[0] = S[S_NSPMV]; counters[1] = S[S_NDOT]; counters[2] = S[S_NPHASE]; }
  free(V);
  return 0;
}

/* y = A x, exposed for checks of the sparse product alone */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
              const double *x, double *y) {
  csr_t A = {n, rowptr, col, val};
  double S[NS];
  spmv(&A, x, y, S);
}

/* (u, v), exposed for checks of the inner product alone */
double orc_dot(int64_t n, const double *u, const double *v) {
  double S[NS];
  return dot(n, u, v, S);
}

/* OpenMP threads of later calls (n >= 1), and the number in use */
void orc_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}
int orc_threads(void) { return omp_get_max_threads(); }

int orc_nv(void) { return NV; }
int orc_ns(void) { return NS; }

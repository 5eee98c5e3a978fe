/*
 * ocd_oracle.c -- plain FP64 CPU oracle for OCD soft-output detection.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP detector.
 * Only the test-suite, the package's smoke check and the benchmark's CPU
 * baseline leg may load it.  The detector never calls it, and the two share
 * no code, header, table or constant.
 *
 * Paper: M. Wu, C. Dick, J. R. Cavallaro, C. Studer, "High-Throughput Data
 * Detection for Massive MU-MIMO-OFDM using Coordinate Descent" (arXiv
 * 1611.08779).  Every function below names the passage it follows.
 *
 * Written for reading, not speed: C99 `double complex`, one vector at a
 * time, no blocking or fusion; built with -O2 -ffp-contract=off.  The only
 * concession is an OpenMP loop over independent (subcarrier, symbol)
 * vectors, which does not change any vector's arithmetic.
 *
 * Layouts (interleaved complex, C order; see synth/__init__.py):
 *   H [W][U][B]   y [W][S][B]   z [W][S][U]   z_hist [W][S][K][U]
 *   llr, bits [W][S][U][Q]      dy [W][S][B]
 *
 * Readings of the paper that the oracle fixes (the paper is silent or uses
 * one symbol for two things):
 *   R1  Regulariser lambda_k per sweep k.  MMSE mode: lambda_k = N0/Es
 *       (Alg. 1 initialisation uses N0 with unit-energy symbols); BOX mode:
 *       lambda_k = 0; HYBRID mode (box AND lambda > 0): lambda_k given,
 *       default N0/Es.  An explicit lambda[] overrides the default in every
 *       mode.
 *   R2  Box half-width beta (the paper calls it alpha in Section II-D, the
 *       same letter as the regulariser): beta <= 0 selects the edge of the
 *       constellation, max Re{a} * sqrt(Es).
 *   R3  Soft output (Section III-C): mu = g/(g+lambda_K) = p_u and
 *       rho = mu/(1-mu) = g/lambda_K when lambda_K > 0.  When lambda_K = 0
 *       (BOX) the formula gives mu = 1 and an infinite rho; the oracle then
 *       uses mu = 1 and rho = g Es/N0, the value of g/lambda at the MMSE
 *       regulariser N0/Es.  (BOX-mode LLR magnitude: parity unpinned by the
 *       paper; only its sign is pinned.)
 *   R4  LLR sign as printed in equation eq:exactinversellr: L > 0 favours
 *       bit 1.  The LLR is evaluated at x = z/(mu sqrt(Es)) against the
 *       unit-energy constellation.
 *   R5  Gray square QAM: per axis M = 2^(Q/2) levels (2m-M+1)/sqrt(2(M^2-1)/3),
 *       label gray(m) = m ^ (m>>1), I bits then Q bits, MSB first.
 *   R6  A user with g_u + lambda_k = 0 gets dinv = 0 (never updated); a user
 *       with rho = 0 or mu = 0 gets LLR 0.
 *   R7  Ties: slicing and argmins take the first point in enumeration order.
 *   R8  Explicit MMSE (Section II-B) writes A = G + N0 I for unit-energy
 *       symbols; with symbol energy Es the regulariser is N0/Es, as in R1.
 *   R9  Section II-E forms the exact gain from "row i of A^-1" and "column i
 *       of G"; the oracle takes mu_i = sum_j [A^-1]_ij G_ji = [A^-1 G]_ii, the
 *       reading under which mu_i is real and rho_i = mu_i/(1-mu_i) is the
 *       post-equalisation SINR (pinned by the error-covariance test).
 *
 * Parity pins (tests/test_oracle_pins.py, all CPU):
 *   oracle_ocd   Alg. 1 form; equals oracle_cd (plain CD, eq:CDrule and
 *                eq:CDruleBOX) to 1e-12; MMSE limit = Cholesky solve of
 *                (G + lambda I) z = H^H y; BOX limit = brute-force box QP;
 *                U = 1 and orthogonal-column closed forms; monotone objective
 *                (via oracle_ocd_trace).
 *   oracle_llr   per-axis closed form of the max-log minima; LLR signs equal
 *                the slicer's bits; at high SNR the slicer returns the
 *                transmitted bits; for orthogonal columns the LLR equals the
 *                exact-MMSE LLR of Section II-E.  BOX magnitude: unpinned (R3).
 *   oracle_hard  textbook MRC BER for U = 1 QPSK; transmitted bits at high SNR.
 *   oracle_grad  FP64 central finite differences of the oracle's own forward
 *                pass, away from kinks (steps across which oracle_active_set
 *                is unchanged).
 *   oracle_mmse  normal equations (G + lambda I) z = H^H y by matrix products;
 *                a library linear solve; the K -> infinity limit of oracle_ocd;
 *                U = 1 and orthogonal-column closed forms (where the LLRs equal
 *                oracle_ocd's at K = 1); mu_i^2 Es / E|z_i - mu_i s_i|^2 =
 *                rho_i from the explicit error covariance; 0 < mu_i < 1.
 *   oracle_ocd_fixed  the reciprocal unit against the true reciprocal; exact
 *                recovery on exactly representable orthogonal channels; within
 *                4 LSB of oracle_ocd on the dequantised inputs; zero-mean
 *                rounding error; saturation and clipping in closed form; the
 *                36-bit range check.  The value of b (F3) only moves rounding by
 *                LSBs (its two shifts cancel): parity unpinned beyond the reading.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { MODE_MMSE = 0, MODE_BOX = 1, MODE_HYBRID = 2 };

/* ---------------------------------------------------------------------- */
/* Constellation (Section II-A; reading R5)                                */
/* ---------------------------------------------------------------------- */

/* Unit-energy Gray square QAM with Q bits: 2^Q points and their labels.
 * label bit (Q-1-b) is bit b of the symbol (bit 0 = MSB of the I label). */
static int qam_points(int Q, cplx *pts, unsigned *labels)
{
    if (Q != 2 && Q != 4 && Q != 6) return -1;
    int half = Q / 2, M = 1 << half;
    double scale = sqrt(2.0 * (double)(M * M - 1) / 3.0);
    int i = 0;
    for (int mi = 0; mi < M; ++mi)
        for (int mq = 0; mq < M; ++mq) {
            double ai = (2.0 * mi - M + 1) / scale;
            double aq = (2.0 * mq - M + 1) / scale;
            unsigned gi = (unsigned)(mi ^ (mi >> 1));
            unsigned gq = (unsigned)(mq ^ (mq >> 1));
            pts[i] = ai + I * aq;
            labels[i] = (gi << half) | gq;
            ++i;
        }
    return 1 << Q;
}

static int symbol_bit(unsigned label, int Q, int b) { return (int)((label >> (Q - 1 - b)) & 1u); }

/* Exported for tests: the 2^Q points (interleaved) and labels. */
int oracle_constellation(int Q, double *pts_out, unsigned *labels_out)
{
    cplx pts[64];
    unsigned lab[64];
    int n = qam_points(Q, pts, lab);
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i) {
        pts_out[2 * i] = creal(pts[i]);
        pts_out[2 * i + 1] = cimag(pts[i]);
        labels_out[i] = lab[i];
    }
    return n;
}

/* Section II-D: the tightest box around square QAM has half-width max Re{a}. */
static double box_edge(int Q)
{
    int M = 1 << (Q / 2);
    return (double)(M - 1) / sqrt(2.0 * (double)(M * M - 1) / 3.0);
}

/* ---------------------------------------------------------------------- */
/* Problem set-up (readings R1, R2)                                        */
/* ---------------------------------------------------------------------- */

typedef struct {
    int B, U, W, S, K, Q, mode;
    double N0, Es, beta;  /* beta resolved; unused in MMSE mode */
    int box;              /* projection onto the box is active */
    double *lambda;       /* [K] resolved regulariser per sweep */
} problem;

static int setup(problem *P, int B, int U, int W, int S, int K, int Q, int mode,
                 double N0, double Es, const double *lambda, double beta)
{
    if (B < 1 || U < 1 || U > B || W < 0 || S < 0 || K < 1 || Es <= 0.0) return -1;
    if (Q != 2 && Q != 4 && Q != 6) return -1;
    if (mode != MODE_MMSE && mode != MODE_BOX && mode != MODE_HYBRID) return -1;
    if (N0 <= 0.0) return -1;
    P->B = B; P->U = U; P->W = W; P->S = S; P->K = K; P->Q = Q; P->mode = mode;
    P->N0 = N0; P->Es = Es;
    P->box = (mode != MODE_MMSE);
    P->beta = (beta > 0.0) ? beta : box_edge(Q) * sqrt(Es);
    P->lambda = (double *)malloc(sizeof(double) * (size_t)K);
    if (!P->lambda) return -1;
    for (int k = 0; k < K; ++k) {
        if (lambda) P->lambda[k] = lambda[k];
        else P->lambda[k] = (mode == MODE_BOX) ? 0.0 : N0 / Es;
        if (P->lambda[k] < 0.0) { free(P->lambda); return -1; }
    }
    return 0;
}

/* Equation eq:projection: orthogonal projection onto the QAM box, i.e. clip
 * the real and the imaginary part independently to [-beta, beta]. */
static cplx project(const problem *P, cplx w)
{
    if (!P->box) return w;
    double re = creal(w), im = cimag(w);
    if (re > P->beta) re = P->beta;
    if (re < -P->beta) re = -P->beta;
    if (im > P->beta) im = P->beta;
    if (im < -P->beta) im = -P->beta;
    return re + I * im;
}

/* Squared column norms g_u = ||h_u||^2 (the Gram diagonal). */
static void column_norms(const problem *P, const cplx *Hw, double *g)
{
    for (int u = 0; u < P->U; ++u) {
        double acc = 0.0;
        for (int b = 0; b < P->B; ++b) {
            cplx h = Hw[(size_t)u * P->B + b];
            acc += creal(h) * creal(h) + cimag(h) * cimag(h);
        }
        g[u] = acc;
    }
}

/* Alg. 1 preprocessing: d_u^-1 = (||h_u||^2 + alpha)^-1 and p_u = d_u^-1 ||h_u||^2,
 * one pair per sweep since lambda may change per sweep (reading R1, R6). */
static void regularised_gains(const problem *P, const double *g, double *dinv, double *p)
{
    for (int k = 0; k < P->K; ++k)
        for (int u = 0; u < P->U; ++u) {
            double den = g[u] + P->lambda[k];
            double di = (den > 0.0) ? 1.0 / den : 0.0;
            dinv[k * P->U + u] = di;
            p[k * P->U + u] = di * g[u];
        }
}

/* ---------------------------------------------------------------------- */
/* Equalisation, form (ii): Algorithm 1 (OCD) as printed                   */
/* ---------------------------------------------------------------------- */

/* Which side of the box a pre-projection value lies on, per component: -1
 * below -beta, +1 above beta, 0 inside (|w| <= beta counts as inside, the
 * convention of the adjoint, reading C9); always 0 without the box. */
static void clip_state(const problem *P, cplx w, signed char *out)
{
    double c[2] = {creal(w), cimag(w)};
    for (int i = 0; i < 2; ++i)
        out[i] = (signed char)(!P->box ? 0 : c[i] > P->beta ? 1 : c[i] < -P->beta ? -1 : 0);
}

/* One vector.  r starts at y and z at 0 (initialisation); each sweep k and
 * user u computes z_u = proj(d_u^-1 h_u^H r + p_u z_u), the change Delta, and
 * the incremental residual update r <- r - h_u Delta (equation eq:residual).
 * clip (optional, [K][U][2]) receives the side of the box of every projection. */
static void ocd_one(const problem *P, const cplx *Hw, const cplx *yv,
                    const double *dinv, const double *p,
                    cplx *r, cplx *z, cplx *hist /* [K][U] or NULL */,
                    signed char *clip /* [K][U][2] or NULL */)
{
    int B = P->B, U = P->U;
    for (int b = 0; b < B; ++b) r[b] = yv[b];
    for (int u = 0; u < U; ++u) z[u] = 0.0;
    for (int k = 0; k < P->K; ++k) {
        for (int u = 0; u < U; ++u) {
            const cplx *h = Hw + (size_t)u * B;
            cplx ip = 0.0;
            for (int b = 0; b < B; ++b) ip += conj(h[b]) * r[b];
            cplx c = dinv[k * U + u] * ip + p[k * U + u] * z[u];
            if (clip) clip_state(P, c, clip + ((size_t)k * U + u) * 2);
            cplx znew = project(P, c);
            cplx delta = znew - z[u];
            for (int b = 0; b < B; ++b) r[b] -= h[b] * delta;
            z[u] = znew;
        }
        if (hist)
            for (int u = 0; u < U; ++u) hist[(size_t)k * U + u] = z[u];
    }
}

int oracle_ocd(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
               const double *lambda, double beta, const double *H, const double *y,
               double *z_out, double *z_hist, int threads)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    const cplx *Hc = (const cplx *)H;
    const cplx *yc = (const cplx *)y;
    long nvec = (long)W * S;
    int err = 0;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        double *g = malloc(sizeof(double) * U);
        double *dinv = malloc(sizeof(double) * (size_t)K * U);
        double *p = malloc(sizeof(double) * (size_t)K * U);
        cplx *r = malloc(sizeof(cplx) * B);
        cplx *z = malloc(sizeof(cplx) * U);
        if (!g || !dinv || !p || !r || !z) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (long v = 0; v < nvec; ++v) {
                long w = v / S;
                const cplx *Hw = Hc + (size_t)w * U * B;
                column_norms(&P, Hw, g);
                regularised_gains(&P, g, dinv, p);
                ocd_one(&P, Hw, yc + (size_t)v * B, dinv, p, r, z,
                        z_hist ? (cplx *)z_hist + (size_t)v * K * U : NULL, NULL);
                for (int u = 0; u < U; ++u) ((cplx *)z_out)[(size_t)v * U + u] = z[u];
            }
        }
        free(g); free(dinv); free(p); free(r); free(z);
    }
    free(P.lambda);
    return err ? -1 : 0;
}

/* Same as oracle_ocd for one vector, recording z after every single
 * coordinate update: trace [K][U][U] (update (k,u) -> the full z). */
int oracle_ocd_trace(int B, int U, int K, int Q, int mode, double N0, double Es,
                     const double *lambda, double beta, const double *H, const double *y,
                     double *trace)
{
    problem P;
    if (setup(&P, B, U, 1, 1, K, Q, mode, N0, Es, lambda, beta)) return -1;
    const cplx *Hw = (const cplx *)H;
    double *g = malloc(sizeof(double) * U);
    double *dinv = malloc(sizeof(double) * (size_t)K * U);
    double *p = malloc(sizeof(double) * (size_t)K * U);
    cplx *r = malloc(sizeof(cplx) * B);
    cplx *z = calloc((size_t)U, sizeof(cplx));
    column_norms(&P, Hw, g);
    regularised_gains(&P, g, dinv, p);
    for (int b = 0; b < B; ++b) r[b] = ((const cplx *)y)[b];
    cplx *tr = (cplx *)trace;
    for (int k = 0; k < K; ++k)
        for (int u = 0; u < U; ++u) {
            const cplx *h = Hw + (size_t)u * B;
            cplx ip = 0.0;
            for (int b = 0; b < B; ++b) ip += conj(h[b]) * r[b];
            cplx znew = project(&P, dinv[k * U + u] * ip + p[k * U + u] * z[u]);
            cplx delta = znew - z[u];
            for (int b = 0; b < B; ++b) r[b] -= h[b] * delta;
            z[u] = znew;
            for (int j = 0; j < U; ++j) tr[((size_t)k * U + u) * U + j] = z[j];
        }
    free(g); free(dinv); free(p); free(r); free(z); free(P.lambda);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Equalisation, form (i): plain coordinate descent (Section III-A)        */
/* ---------------------------------------------------------------------- */

/* eq:CDrule / eq:CDruleBOX with regulariser lambda_k:
 *   z_u = proj( (||h_u||^2 + lambda_k)^-1 h_u^H (y - sum_{j != u} h_j z_j) ),
 * the partial residual recomputed from scratch at every coordinate, the new
 * z_u re-used at once by the following users. */
int oracle_cd(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
              const double *lambda, double beta, const double *H, const double *y,
              double *z_out, int threads)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    const cplx *Hc = (const cplx *)H;
    const cplx *yc = (const cplx *)y;
    long nvec = (long)W * S;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        cplx *t = malloc(sizeof(cplx) * B);
        cplx *z = malloc(sizeof(cplx) * U);
#pragma omp for schedule(static)
        for (long v = 0; v < nvec; ++v) {
            const cplx *Hw = Hc + (size_t)(v / S) * U * B;
            const cplx *yv = yc + (size_t)v * B;
            for (int u = 0; u < U; ++u) z[u] = 0.0;
            for (int k = 0; k < K; ++k)
                for (int u = 0; u < U; ++u) {
                    for (int b = 0; b < B; ++b) {
                        cplx acc = yv[b];
                        for (int j = 0; j < U; ++j)
                            if (j != u) acc -= Hw[(size_t)j * B + b] * z[j];
                        t[b] = acc;
                    }
                    double gu = 0.0;
                    cplx ip = 0.0;
                    for (int b = 0; b < B; ++b) {
                        cplx h = Hw[(size_t)u * B + b];
                        gu += creal(h) * creal(h) + cimag(h) * cimag(h);
                        ip += conj(h) * t[b];
                    }
                    double den = gu + P.lambda[k];
                    z[u] = project(&P, den > 0.0 ? ip / den : 0.0);
                }
            for (int u = 0; u < U; ++u) ((cplx *)z_out)[(size_t)v * U + u] = z[u];
        }
        free(t); free(z);
    }
    free(P.lambda);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Soft output: equation eq:exactinversellr with Section III-C's mu, rho   */
/* ---------------------------------------------------------------------- */

/* Channel gain and SINR approximations (reading R3). */
static void gain_sinr(const problem *P, double g, double *mu, double *rho)
{
    double lamK = P->lambda[P->K - 1];
    if (lamK > 0.0) {
        *mu = g / (g + lamK);
        *rho = g / lamK;
    } else {
        *mu = 1.0;
        *rho = g * P->Es / P->N0;
    }
}

/* Max-log LLRs of one user by brute force over every constellation point:
 * L_b = rho * ( min_{a in O_b^0} |x - a|^2 - min_{a in O_b^1} |x - a|^2 ).
 * a0[b], a1[b] receive the indices of the two minimisers (first found). */
static void maxlog_one(int Q, const cplx *pts, const unsigned *labels, cplx x, double rho,
                       double *L, int *a0, int *a1)
{
    int n = 1 << Q;
    for (int b = 0; b < Q; ++b) {
        double d0 = INFINITY, d1 = INFINITY;
        int i0 = -1, i1 = -1;
        for (int i = 0; i < n; ++i) {
            cplx e = x - pts[i];
            double d = creal(e) * creal(e) + cimag(e) * cimag(e);
            if (symbol_bit(labels[i], Q, b) == 0) {
                if (d < d0) { d0 = d; i0 = i; }
            } else {
                if (d < d1) { d1 = d; i1 = i; }
            }
        }
        L[b] = rho * (d0 - d1);
        if (a0) a0[b] = i0;
        if (a1) a1[b] = i1;
    }
}

int oracle_llr(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
               const double *lambda, double beta, const double *H, const double *z,
               double *llr, int threads)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    cplx pts[64];
    unsigned labels[64];
    qam_points(Q, pts, labels);
    const cplx *Hc = (const cplx *)H;
    long nvec = (long)W * S;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        double *g = malloc(sizeof(double) * U);
#pragma omp for schedule(static)
        for (long v = 0; v < nvec; ++v) {
            column_norms(&P, Hc + (size_t)(v / S) * U * B, g);
            for (int u = 0; u < U; ++u) {
                double *Lout = llr + ((size_t)v * U + u) * Q;
                double mu, rho;
                gain_sinr(&P, g[u], &mu, &rho);
                if (!(rho > 0.0) || !(mu > 0.0)) {
                    for (int b = 0; b < Q; ++b) Lout[b] = 0.0;
                    continue;
                }
                cplx x = ((const cplx *)z)[(size_t)v * U + u] / (mu * sqrt(Es));
                maxlog_one(Q, pts, labels, x, rho, Lout, NULL, NULL);
            }
        }
        free(g);
    }
    free(P.lambda);
    return 0;
}

/* Hard output, equation eq:slicing applied to x = z/(mu sqrt(Es)): the bits
 * of the nearest constellation point (reading R7 for ties). */
int oracle_hard(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
                const double *lambda, double beta, const double *H, const double *z,
                unsigned char *bits)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    cplx pts[64];
    unsigned labels[64];
    int n = qam_points(Q, pts, labels);
    double *g = malloc(sizeof(double) * U);
    long nvec = (long)W * S;
    for (long v = 0; v < nvec; ++v) {
        column_norms(&P, (const cplx *)H + (size_t)(v / S) * U * B, g);
        for (int u = 0; u < U; ++u) {
            double mu, rho;
            gain_sinr(&P, g[u], &mu, &rho);
            if (!(mu > 0.0)) mu = 1.0;
            cplx x = ((const cplx *)z)[(size_t)v * U + u] / (mu * sqrt(Es));
            int best = 0;
            double bd = INFINITY;
            for (int i = 0; i < n; ++i) {
                cplx e = x - pts[i];
                double d = creal(e) * creal(e) + cimag(e) * cimag(e);
                if (d < bd) { bd = d; best = i; }
            }
            for (int b = 0; b < Q; ++b)
                bits[((size_t)v * U + u) * Q + b] = (unsigned char)symbol_bit(labels[best], Q, b);
        }
    }
    free(g); free(P.lambda);
    return 0;
}

/* The whole detection path of one slot: Alg. 1 then the soft output. */
int oracle_detect(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
                  const double *lambda, double beta, const double *H, const double *y,
                  double *z_out, double *llr, int threads)
{
    if (oracle_ocd(B, U, W, S, K, Q, mode, N0, Es, lambda, beta, H, y, z_out, NULL, threads))
        return -1;
    return oracle_llr(B, U, W, S, K, Q, mode, N0, Es, lambda, beta, H, z_out, llr, threads);
}

/* The active set of the whole path at these inputs: the pieces of the
 * piecewise-smooth map from (lambda, beta, y) to the LLRs that are in use.
 * The loss is differentiable wherever a small change of the inputs leaves
 * it unchanged, so central finite differences (the check of the reference
 * gradient) are taken only across steps that leave it unchanged.
 *   clip [W][S][K][U][2]: side of the box of every projection (clip_state);
 *   amin [W][S][U][Q][2]: the two max-log minimisers of every bit (maxlog_one),
 *                         -1 for a user whose LLRs are 0 (reading R6). */
int oracle_active_set(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
                      const double *lambda, double beta, const double *H, const double *y,
                      signed char *clip, signed char *amin)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    cplx pts[64];
    unsigned labels[64];
    qam_points(Q, pts, labels);
    const cplx *Hc = (const cplx *)H;
    const cplx *yc = (const cplx *)y;
    double *g = malloc(sizeof(double) * U);
    double *dinv = malloc(sizeof(double) * (size_t)K * U);
    double *p = malloc(sizeof(double) * (size_t)K * U);
    cplx *r = malloc(sizeof(cplx) * B);
    cplx *z = malloc(sizeof(cplx) * U);
    double Lv[6];
    int a0[6], a1[6];
    long nvec = (long)W * S;
    for (long v = 0; v < nvec; ++v) {
        const cplx *Hw = Hc + (size_t)(v / S) * U * B;
        column_norms(&P, Hw, g);
        regularised_gains(&P, g, dinv, p);
        ocd_one(&P, Hw, yc + (size_t)v * B, dinv, p, r, z, NULL, clip + (size_t)v * K * U * 2);
        for (int u = 0; u < U; ++u) {
            signed char *am = amin + ((size_t)v * U + u) * Q * 2;
            double mu, rho;
            gain_sinr(&P, g[u], &mu, &rho);
            if (!(rho > 0.0) || !(mu > 0.0)) {
                for (int b = 0; b < 2 * Q; ++b) am[b] = -1;
                continue;
            }
            maxlog_one(Q, pts, labels, z[u] / (mu * sqrt(Es)), rho, Lv, a0, a1);
            for (int b = 0; b < Q; ++b) {
                am[2 * b] = (signed char)a0[b];
                am[2 * b + 1] = (signed char)a1[b];
            }
        }
    }
    free(g); free(dinv); free(p); free(r); free(z); free(P.lambda);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Reference gradient: reverse mode through Alg. 1 and the soft output     */
/* ---------------------------------------------------------------------- */

/* Given dllr = dLoss/dL, returns dLoss/dlambda_k (K), dLoss/dbeta and
 * dLoss/dy.  Complex adjoints are dLoss/dRe + j dLoss/dIm.  The forward pass
 * is re-run storing the residual before every update and every pre-projection
 * value c; the reverse pass walks the updates backwards:
 *   Delta_bar = -h_u^H r_bar
 *   znew_bar  = z_u_bar + Delta_bar
 *   c_bar     = znew_bar on unclipped components, 0 on clipped ones
 *               (|c| <= beta counts as unclipped); clipped components add
 *               sign(c) * znew_bar to beta_bar
 *   z_u_bar   = -Delta_bar + p_u c_bar          (adjoint of the old z_u)
 *   r_bar    += h_u d_u^-1 c_bar                (adjoint of the old residual)
 *   lambda_bar_k += -dinv^2 Re(conj(h_u^H r) c_bar) - g dinv^2 Re(conj(z_u) c_bar)
 * and y_bar is the residual adjoint left after the first update.  The LLR
 * contributes z_bar = x_bar/(mu sqrt(Es)) with x_bar = sum_b Lbar_b rho 2(a1-a0),
 * and, when lambda_K > 0, terms through mu = g/(g+lambda_K), rho = g/lambda_K. */
int oracle_grad(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
                const double *lambda, double beta, const double *H, const double *y,
                const double *dllr, double *dlambda, double *dbeta, double *dy)
{
    problem P;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, lambda, beta)) return -1;
    cplx pts[64];
    unsigned labels[64];
    qam_points(Q, pts, labels);
    const cplx *Hc = (const cplx *)H;
    const cplx *yc = (const cplx *)y;
    double *g = malloc(sizeof(double) * U);
    double *dinv = malloc(sizeof(double) * (size_t)K * U);
    double *p = malloc(sizeof(double) * (size_t)K * U);
    cplx *r = malloc(sizeof(cplx) * B);
    cplx *rbar = malloc(sizeof(cplx) * B);
    cplx *z = malloc(sizeof(cplx) * U);
    cplx *zbar = malloc(sizeof(cplx) * U);
    cplx *rpre = malloc(sizeof(cplx) * (size_t)K * U * B);
    cplx *cval = malloc(sizeof(cplx) * (size_t)K * U);
    cplx *zold = malloc(sizeof(cplx) * (size_t)K * U);
    double Lv[6];
    int a0[6], a1[6];
    for (int k = 0; k < K; ++k) dlambda[k] = 0.0;
    *dbeta = 0.0;
    double lamK = P.lambda[K - 1];
    long nvec = (long)W * S;
    for (long v = 0; v < nvec; ++v) {
        const cplx *Hw = Hc + (size_t)(v / S) * U * B;
        const cplx *yv = yc + (size_t)v * B;
        column_norms(&P, Hw, g);
        regularised_gains(&P, g, dinv, p);
        /* forward, storing what the reverse pass needs */
        for (int b = 0; b < B; ++b) r[b] = yv[b];
        for (int u = 0; u < U; ++u) z[u] = 0.0;
        for (int k = 0; k < K; ++k)
            for (int u = 0; u < U; ++u) {
                const cplx *h = Hw + (size_t)u * B;
                size_t ku = (size_t)k * U + u;
                memcpy(rpre + ku * B, r, sizeof(cplx) * B);
                cplx ip = 0.0;
                for (int b = 0; b < B; ++b) ip += conj(h[b]) * r[b];
                cplx c = dinv[ku] * ip + p[ku] * z[u];
                cplx znew = project(&P, c);
                cplx delta = znew - z[u];
                for (int b = 0; b < B; ++b) r[b] -= h[b] * delta;
                cval[ku] = c;
                zold[ku] = z[u];
                z[u] = znew;
            }
        /* soft output adjoint */
        for (int u = 0; u < U; ++u) {
            const double *Lbar = dllr + ((size_t)v * U + u) * Q;
            double mu, rho;
            gain_sinr(&P, g[u], &mu, &rho);
            zbar[u] = 0.0;
            if (!(rho > 0.0) || !(mu > 0.0)) continue;
            double s = mu * sqrt(Es);
            cplx x = z[u] / s;
            maxlog_one(Q, pts, labels, x, rho, Lv, a0, a1);
            cplx xbar = 0.0;
            double dmu = 0.0, drho = 0.0;
            for (int b = 0; b < Q; ++b) {
                cplx grad_x = 2.0 * (pts[a1[b]] - pts[a0[b]]); /* dD_b/dx, D_b = d0 - d1 */
                xbar += Lbar[b] * rho * grad_x;
                drho += Lbar[b] * (Lv[b] / rho);
                /* x = z/(mu sqrt(Es)): dx/dmu = -x/mu */
                dmu += Lbar[b] * rho * creal(conj(grad_x) * (-x / mu));
            }
            zbar[u] = xbar / s;
            if (lamK > 0.0) {
                dlambda[K - 1] += drho * (-g[u] / (lamK * lamK));
                dlambda[K - 1] += dmu * (-g[u] / ((g[u] + lamK) * (g[u] + lamK)));
            }
        }
        /* reverse sweeps */
        for (int b = 0; b < B; ++b) rbar[b] = 0.0;
        for (int k = K - 1; k >= 0; --k)
            for (int u = U - 1; u >= 0; --u) {
                const cplx *h = Hw + (size_t)u * B;
                size_t ku = (size_t)k * U + u;
                cplx c = cval[ku];
                cplx hr = 0.0, ip = 0.0;
                for (int b = 0; b < B; ++b) {
                    hr += conj(h[b]) * rbar[b];
                    ip += conj(h[b]) * rpre[ku * B + b];
                }
                cplx dbar = -hr;
                cplx ztot = zbar[u] + dbar;
                double cre = 0.0, cim = 0.0;
                if (P.box && fabs(creal(c)) > P.beta) *dbeta += (creal(c) > 0 ? 1.0 : -1.0) * creal(ztot);
                else cre = creal(ztot);
                if (P.box && fabs(cimag(c)) > P.beta) *dbeta += (cimag(c) > 0 ? 1.0 : -1.0) * cimag(ztot);
                else cim = cimag(ztot);
                cplx cbar = cre + I * cim;
                double di = dinv[ku];
                dlambda[k] += -di * di * creal(conj(ip) * cbar)
                              - g[u] * di * di * creal(conj(zold[ku]) * cbar);
                zbar[u] = -dbar + p[ku] * cbar;
                for (int b = 0; b < B; ++b) rbar[b] += h[b] * (di * cbar);
            }
        for (int b = 0; b < B; ++b) ((cplx *)dy)[(size_t)v * B + b] = rbar[b];
    }
    if (!P.box) *dbeta = 0.0;
    free(g); free(dinv); free(p); free(r); free(rbar); free(z); free(zbar);
    free(rpre); free(cval); free(zold); free(P.lambda);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Explicit MMSE soft-output detection: Section II-B (the regularised Gram */
/* matrix and its inverse) with the exact gain and SINR of Section II-E    */
/* ---------------------------------------------------------------------- */

/* Cholesky factor of a Hermitian positive definite n x n matrix (row-major):
 * A = L L^H with L lower triangular and a real positive diagonal.  Returns -1
 * when a pivot is not positive. */
static int cholesky(int n, const cplx *A, cplx *Lf)
{
    for (int i = 0; i < n * n; ++i) Lf[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double d = creal(A[j * n + j]);
        for (int k = 0; k < j; ++k) {
            cplx l = Lf[j * n + k];
            d -= creal(l) * creal(l) + cimag(l) * cimag(l);
        }
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        Lf[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= Lf[i * n + k] * conj(Lf[j * n + k]);
            Lf[i * n + j] = s / ljj;
        }
    }
    return 0;
}

/* A^-1 column by column from the Cholesky factor: L w = e_j, then L^H x = w. */
static void cholesky_inverse(int n, const cplx *Lf, cplx *Ainv)
{
    cplx *w = malloc(sizeof(cplx) * n);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            cplx s = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= Lf[i * n + k] * w[k];
            w[i] = s / Lf[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            cplx s = w[i];
            for (int k = i + 1; k < n; ++k) s -= conj(Lf[k * n + i]) * Ainv[k * n + j];
            Ainv[i * n + j] = s / conj(Lf[i * n + i]);
        }
    }
    free(w);
}

/* Explicit MMSE detection of every vector (reading R8 for the regulariser and
 * R9 for the gain), then the max-log LLRs of eq:exactinversellr:
 *   G = H^H H, A = G + (N0/Es) I, z = A^-1 (H^H y)               (Section II-B)
 *   mu_i = row i of A^-1 times column i of G, rho_i = mu_i/(1-mu_i) (Section II-E)
 *   L_{i,b} at x = z_i/(mu_i sqrt(Es)) against the unit-energy points (R4, R5).
 * A user with mu_i <= 0 (an all-zero column) gets LLR 0 (R6).
 * z [W][S][U] and llr [W][S][U][Q] may each be NULL; mu [W][U] may be NULL. */
int oracle_mmse(int B, int U, int W, int S, int Q, double N0, double Es, const double *H,
                const double *y, double *z, double *llr, double *mu_out, int threads)
{
    if (B < 1 || U < 1 || U > B || W < 0 || S < 0 || !(N0 > 0.0) || !(Es > 0.0)) return -1;
    if (Q != 2 && Q != 4 && Q != 6) return -1;
    cplx pts[64];
    unsigned labels[64];
    qam_points(Q, pts, labels);
    const double lam = N0 / Es;
    const cplx *Hc = (const cplx *)H, *yc = (const cplx *)y;
    int failed = 0;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        cplx *G = malloc(sizeof(cplx) * U * U), *A = malloc(sizeof(cplx) * U * U);
        cplx *Lf = malloc(sizeof(cplx) * U * U), *Ainv = malloc(sizeof(cplx) * U * U);
        cplx *mf = malloc(sizeof(cplx) * U);
        double *mu = malloc(sizeof(double) * U), *rho = malloc(sizeof(double) * U);
#pragma omp for schedule(static)
        for (int w = 0; w < W; ++w) {
            const cplx *Hw = Hc + (size_t)w * U * B;   /* column u at Hw + u*B */
            for (int i = 0; i < U; ++i)
                for (int j = 0; j < U; ++j) {
                    cplx s = 0.0;
                    for (int b = 0; b < B; ++b) s += conj(Hw[i * B + b]) * Hw[j * B + b];
                    G[i * U + j] = s;
                    A[i * U + j] = s + ((i == j) ? lam : 0.0);
                }
            if (cholesky(U, A, Lf)) {
#pragma omp atomic write
                failed = 1;
                continue;
            }
            cholesky_inverse(U, Lf, Ainv);
            for (int i = 0; i < U; ++i) {
                cplx s = 0.0;
                for (int j = 0; j < U; ++j) s += Ainv[i * U + j] * G[j * U + i];
                mu[i] = creal(s);
                rho[i] = mu[i] / (1.0 - mu[i]);
                if (mu_out) mu_out[(size_t)w * U + i] = mu[i];
            }
            for (int s = 0; s < S; ++s) {
                const size_t v = (size_t)w * S + s;
                const cplx *yv = yc + v * B;
                for (int i = 0; i < U; ++i) {
                    cplx acc = 0.0;
                    for (int b = 0; b < B; ++b) acc += conj(Hw[i * B + b]) * yv[b];
                    mf[i] = acc;
                }
                for (int i = 0; i < U; ++i) {
                    cplx zi = 0.0;
                    for (int j = 0; j < U; ++j) zi += Ainv[i * U + j] * mf[j];
                    if (z) {
                        z[2 * (v * U + i)] = creal(zi);
                        z[2 * (v * U + i) + 1] = cimag(zi);
                    }
                    if (!llr) continue;
                    double *Lout = llr + (v * U + i) * Q;
                    if (!(mu[i] > 0.0) || !(rho[i] > 0.0)) {
                        for (int b = 0; b < Q; ++b) Lout[b] = 0.0;
                        continue;
                    }
                    maxlog_one(Q, pts, labels, zi / (mu[i] * sqrt(Es)), rho[i], Lout, NULL, NULL);
                }
            }
        }
        free(G); free(A); free(Lf); free(Ainv); free(mf); free(mu); free(rho);
    }
    return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* The fixed-point datapath of Section IV-C (readings F1-F8)               */
/* ---------------------------------------------------------------------- */
/*
 * F1  Words.  H, y, the residual r, z, beta, d^-1 and p are 16-bit two's
 *     complement with 11 fractional bits (Q5.11: value = integer / 2^11).
 *     Products of two such words are exact (Q.22); the inner products are
 *     exact sums of them (the paper's 36-bit adder tree; the oracle fails if a
 *     sum leaves the 36-bit range, so "exact" and "36-bit" agree).
 * F2  Scale.  The shifts below assume channel entries of unit average power
 *     (||h_u||^2 close to B); a caller with another channel scale multiplies H
 *     and y by one factor c and N0 by c^2, which leaves OCD's estimate unchanged.
 * F3  b = ceil(log2 B).  ||h_u||^2 + alpha and h_u^H r are shifted right by b
 *     (arithmetic shift: floor); the two shifts cancel in d^-1 h^H r.
 * F4  alpha = lambda (N0/Es in MMSE mode, 0 in BOX mode) enters as the Q.22
 *     integer round(lambda 2^22), an operand of the 36-bit adder beside
 *     ||h_u||^2: alpha >= 2^35 is not representable and is rejected.  beta is a
 *     Q5.11 word; c is narrowed (F6) before the clip, so a beta of 2^15 LSB or
 *     more clips nothing and is held at 2^15.
 * F5  Reciprocal of an integer x > 0 of bit length n (x / 2^n in [1/2, 1)):
 *     the index is the 11 bits after the leading one; the table holds the 18-bit
 *     normalised reciprocal round(2^18 / (1 + (i + 1/2) / 2048)) (1/x in Q1.17
 *     at the middle of the index's interval); denormalising to Q.11 multiplies by
 *     2^(16 - n) (x is in Q.22 units).  x = 0 gives 0.
 * F6  Every narrowing to 16 bits rounds half up (add half an LSB, shift) and
 *     saturates to [-2^15, 2^15 - 1].
 * F7  p_u = d_u^-1 (||h_u||^2 >> b), narrowed to Q.11 (F6).
 * F8  The FPGA design has no soft-output unit: LLRs are formed in floating
 *     point from the fixed-point z (mu = p / 2^11 in MMSE mode, 1 in BOX mode;
 *     rho = g / lambda, g = ||h_u||^2 / 2^22; BOX: g Es / N0), as in R3.
 */

#define FX_FRAC 11
#define FX_ACC_BITS 36

static int64_t fx_sat16(int64_t v)
{
    return v < -32768 ? -32768 : (v > 32767 ? 32767 : v);
}

/* v / 2^s rounded half up, s >= 1. */
static int64_t fx_round_shift(int64_t v, int s) { return (v + ((int64_t)1 << (s - 1))) >> s; }

static int fx_bitlen(uint64_t x)
{
    int n = 0;
    while (x) { ++n; x >>= 1; }
    return n;
}

/* F5 */
static int64_t fx_recip(int64_t x)
{
    if (x <= 0) return 0;
    int n = fx_bitlen((uint64_t)x);
    int64_t idx = n >= 12 ? (x >> (n - 12)) & 2047 : (x << (12 - n)) & 2047;
    int64_t lut = (int64_t)floor(262144.0 / (1.0 + ((double)idx + 0.5) / 2048.0) + 0.5);
    int64_t d = (16 - n >= 0) ? lut << (16 - n) : fx_round_shift(lut, n - 16);
    return fx_sat16(d);
}

/* Exported for tests: the reciprocal unit alone. */
int64_t oracle_fx_recip(int64_t x) { return fx_recip(x); }

static int fx_ceil_log2(int B)
{
    int b = 0;
    while ((1 << b) < B) ++b;
    return b;
}

static int fx_acc_ok(int64_t v)
{
    const int64_t lim = (int64_t)1 << (FX_ACC_BITS - 1);
    return v >= -lim && v < lim;
}

/* Algorithm 1 in the fixed-point datapath, one vector.  h: U columns of B
 * (re, im) int16 pairs; yv: B pairs; z: U pairs out; p_out: p_u of the sweeps
 * (F7).  Returns -1 if an inner product leaves the 36-bit range. */
static int ocd_fixed_one(int B, int U, int K, int box, int64_t lam_q, int64_t beta_fx,
                         const int16_t *h, const int16_t *yv, int16_t *zout, int64_t *G,
                         int64_t *dinv, int64_t *p)
{
    const int b = fx_ceil_log2(B);
    int64_t *r = malloc(sizeof(int64_t) * 2 * B), *z = malloc(sizeof(int64_t) * 2 * U);
    int ok = 1;
    for (int i = 0; i < 2 * B; ++i) r[i] = yv[i];
    for (int u = 0; u < 2 * U; ++u) z[u] = 0;
    /* preprocessing (Alg. 1, initialisation) */
    for (int u = 0; u < U; ++u) {
        const int16_t *hu = h + (size_t)2 * u * B;
        int64_t g = 0;
        for (int i = 0; i < B; ++i) g += (int64_t)hu[2 * i] * hu[2 * i] + (int64_t)hu[2 * i + 1] * hu[2 * i + 1];
        ok &= fx_acc_ok(g) && fx_acc_ok(g + lam_q);
        G[u] = g;
        dinv[u] = fx_recip((g + lam_q) >> b);
        p[u] = fx_sat16(fx_round_shift(dinv[u] * (g >> b), 22));
    }
    for (int k = 0; k < K; ++k)
        for (int u = 0; u < U; ++u) {
            const int16_t *hu = h + (size_t)2 * u * B;
            int64_t ire = 0, iim = 0;      /* h_u^H r, Q.22 */
            for (int i = 0; i < B; ++i) {
                const int64_t hr = hu[2 * i], hi = hu[2 * i + 1];
                ire += hr * r[2 * i] + hi * r[2 * i + 1];
                iim += hr * r[2 * i + 1] - hi * r[2 * i];
            }
            ok &= fx_acc_ok(ire) && fx_acc_ok(iim);
            ire >>= b;
            iim >>= b;
            /* c = d^-1 (h^H r) + p z, in Q.33, narrowed to Q.11 */
            int64_t cre = fx_sat16(fx_round_shift(dinv[u] * ire + (p[u] * z[2 * u] << 11), 22));
            int64_t cim = fx_sat16(fx_round_shift(dinv[u] * iim + (p[u] * z[2 * u + 1] << 11), 22));
            if (box) {
                if (cre > beta_fx) cre = beta_fx;
                if (cre < -beta_fx) cre = -beta_fx;
                if (cim > beta_fx) cim = beta_fx;
                if (cim < -beta_fx) cim = -beta_fx;
            }
            const int64_t dre = cre - z[2 * u], dim = cim - z[2 * u + 1];
            for (int i = 0; i < B; ++i) {
                const int64_t hr = hu[2 * i], hi = hu[2 * i + 1];
                r[2 * i] = fx_sat16(r[2 * i] - fx_round_shift(hr * dre - hi * dim, FX_FRAC));
                r[2 * i + 1] = fx_sat16(r[2 * i + 1] - fx_round_shift(hr * dim + hi * dre, FX_FRAC));
            }
            z[2 * u] = cre;
            z[2 * u + 1] = cim;
        }
    for (int u = 0; u < 2 * U; ++u) zout[u] = (int16_t)z[u];
    free(r); free(z);
    return ok ? 0 : -1;
}

/* Every vector through the fixed-point datapath, then the soft output (F8).
 * H [W][U][B] and y [W][S][B] int16 (re, im) pairs in Q5.11; z [W][S][U] pairs
 * (may be NULL); llr [W][S][U][Q] (may be NULL).  mode: MMSE or BOX. */
int oracle_ocd_fixed(int B, int U, int W, int S, int K, int Q, int mode, double N0, double Es,
                     double beta, const int16_t *H, const int16_t *y, int16_t *z, double *llr,
                     int threads)
{
    problem P;
    if (mode == MODE_HYBRID) return -1;
    if (setup(&P, B, U, W, S, K, Q, mode, N0, Es, NULL, beta)) return -1;
    const double lam = P.lambda[0];
    const double lam_s = floor(lam * 4194304.0 + 0.5);
    if (!(lam_s < 34359738368.0)) return -1;                  /* alpha < 2^35 (F4) */
    const int64_t lam_q = (int64_t)lam_s;
    const double beta_s = floor(P.beta * 2048.0 + 0.5);
    const int64_t beta_fx = beta_s < 32768.0 ? (int64_t)beta_s : 32768;   /* F4 */
    cplx pts[64];
    unsigned labels[64];
    qam_points(Q, pts, labels);
    int failed = 0;
    const long nvec = (long)W * S;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
    {
        int16_t *zv = malloc(sizeof(int16_t) * 2 * U);
        int64_t *G = malloc(sizeof(int64_t) * U), *dinv = malloc(sizeof(int64_t) * U);
        int64_t *p = malloc(sizeof(int64_t) * U);
#pragma omp for schedule(static)
        for (long v = 0; v < nvec; ++v) {
            const int16_t *h = H + (size_t)(v / S) * U * B * 2;
            if (ocd_fixed_one(B, U, K, P.box, lam_q, beta_fx, h, y + (size_t)v * B * 2, zv, G,
                              dinv, p)) {
#pragma omp atomic write
                failed = 1;
            }
            if (z) memcpy(z + (size_t)v * U * 2, zv, sizeof(int16_t) * 2 * U);
            if (!llr) continue;
            for (int u = 0; u < U; ++u) {
                double *Lout = llr + ((size_t)v * U + u) * Q;
                const double g = (double)G[u] / 4194304.0;
                double mu, rho;
                if (lam > 0.0) {
                    mu = (double)p[u] / 2048.0;
                    rho = g / lam;
                } else {
                    mu = 1.0;
                    rho = g * Es / N0;
                }
                if (!(mu > 0.0) || !(rho > 0.0)) {
                    for (int bq = 0; bq < Q; ++bq) Lout[bq] = 0.0;
                    continue;
                }
                const cplx zu = ((double)zv[2 * u] + I * (double)zv[2 * u + 1]) / 2048.0;
                maxlog_one(Q, pts, labels, zu / (mu * sqrt(Es)), rho, Lout, NULL, NULL);
            }
        }
        free(zv); free(G); free(dinv); free(p);
    }
    free(P.lambda);
    return failed ? -1 : 0;
}

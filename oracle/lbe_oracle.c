/*
 * Plain FP64 CPU oracle for the finite-difference lattice Boltzmann (FDLB) solver of the
 * simplified Enskog equation in vielbein (cylindrical / spherical) coordinates,
 * S. Busuioc, "Mesoscopic Lattice Boltzmann modeling of dense gas flows in curvilinear
 * geometries", arXiv:2403.15051.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never calls it and shares no code,
 * header, table or generator with it.
 *
 * Every routine follows the paper's definitions in the paper's order and notation, with
 * straight loops, fixed loop orders and no fusion:
 *   - quadratures: Sec. III ("Quadrature choice"), weights eq. for w^H and w^h;
 *     tables are generated in __float128 (Stieltjes on a discretised measure, roots by
 *     bisection with interlacing) and rounded to double once;
 *   - force-term matrices: Sec. III.B, eq. (force1)/(force2) and the printed K matrices;
 *   - equilibrium: Sec. III.C, eqs. (eq_gak_H), (eq_gak_hh);
 *   - moments: eqs. (macro_def), (mom_quad); two-pass (raw, then central) sums;
 *   - collision: eqs. (j0), (fmb), (j1), (enskog_approx); transport: eqs. (viscosity),
 *     (prandtl), (tau); Kn map: Sec. II (Kn = 1/(6 sqrt2 eta0 chi(eta0) C));
 *   - reduced equations: Sec. II.B (cylindrical), Sec. II.C (spherical);
 *   - schemes: Sec. III (TVD RK3, WENO-5, 4th-order central differences);
 *   - non-local density: eqs. (chi_ret), (fm) and Appendix A (volume intersections);
 *   - walls: Sec. IV (diffuse reflection at R_L + sigma/2 and R_R - sigma/2).
 *   - attractive mean field (beyond the paper, the step Sec. V names next): section 6b, an
 *     Enskog-Vlasov force from a Sutherland tail, evaluated by direct quadrature.
 * Readings of points the paper leaves open are marked "Reading:" where they are used.
 *
 * Parity status of each part is stated next to it; every public routine is pinned by a
 * CPU test against closed forms, invariants, brute force or the paper's Table 1.
 */
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 qreal;

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ENAN -5

#define QMAX 128 /* largest quadrature order the oracle accepts */
#define NMAX 16  /* largest equilibrium expansion order */

static const double PI = 3.14159265358979323846264338327950288;

/* ======================================================================================
 * 1. Extended-precision building blocks
 * ====================================================================================== */

/* Gauss-Legendre rule on [-1,1] in __float128: Newton iteration on P_n from the Chebyshev
 * initial guess.  Used only to discretise the half-range measure below. */
static void gl_rule_q(int n, qreal* x, qreal* w)
{
    for (int i = 0; i < (n + 1) / 2; i++) {
        qreal z = cosq(M_PIq * ((qreal)i + 0.75Q) / ((qreal)n + 0.5Q));
        qreal dp = 0;
        for (int it = 0; it < 200; it++) {
            qreal p0 = 1, p1 = z;
            for (int k = 2; k <= n; k++) {
                qreal p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            qreal dz = p1 / dp;
            z -= dz;
            if (fabsq(dz) < 1e-33Q) break;
        }
        {
            qreal p0 = 1, p1 = z;
            for (int k = 2; k <= n; k++) {
                qreal p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2 / ((1 - z * z) * dp * dp);
    }
}

/* Three-term recurrence of the polynomials orthonormal on [0, inf) with respect to
 * omega(x) = exp(-x^2/2)/sqrt(2 pi)  (Sec. III, weight function of the half-range
 * Hermite polynomials h_l):  x h_l = b[l+1] h_{l+1} + a[l] h_l + b[l] h_{l-1}, with
 * h_0 = 1/sqrt(mu_0) = sqrt(2).  b[0] holds mu_0 = 1/2.
 * Computed by the Stieltjes procedure: inner products are sums over a composite
 * Gauss-Legendre discretisation of the measure on [0, X]; the monic polynomials are
 * advanced by their own recurrence.  nrec coefficients a[0..nrec-1], b[0..nrec]. */
static void half_recurrence_q(int nrec, qreal* a, qreal* b)
{
    const int P = 24;                                  /* points per panel */
    const qreal X = sqrtq((qreal)(2 * nrec + 1)) + 16; /* exp(-X^2/2) x^(2n+1) negligible */
    const qreal h = 0.25Q;
    const int npan = (int)ceilq(X / h);
    const int M = npan * P;
    qreal gx[64], gw[64];
    gl_rule_q(P, gx, gw);
    qreal* y = malloc(sizeof(qreal) * M);
    qreal* lam = malloc(sizeof(qreal) * M);
    qreal* pk = malloc(sizeof(qreal) * M);
    qreal* pkm1 = malloc(sizeof(qreal) * M);
    const qreal c = 1 / sqrtq(2 * M_PIq);
    for (int p = 0; p < npan; p++)
        for (int j = 0; j < P; j++) {
            qreal t = p * h + h * (gx[j] + 1) / 2;
            y[p * P + j] = t;
            lam[p * P + j] = gw[j] * h / 2 * c * expq(-t * t / 2);
        }
    for (int m = 0; m < M; m++) {
        pk[m] = 1;
        pkm1[m] = 0;
    }
    qreal nprev = 1;
    for (int k = 0; k <= nrec; k++) {
        qreal nk = 0, xk = 0;
        for (int m = 0; m < M; m++) {
            nk += lam[m] * pk[m] * pk[m];
            xk += lam[m] * y[m] * pk[m] * pk[m];
        }
        qreal beta = (k == 0) ? nk : nk / nprev;
        b[k] = (k == 0) ? nk : sqrtq(beta);
        if (k == nrec) break;
        a[k] = xk / nk;
        for (int m = 0; m < M; m++) {
            qreal nxt = (y[m] - a[k]) * pk[m] - ((k == 0) ? 0 : beta) * pkm1[m];
            pkm1[m] = pk[m];
            pk[m] = nxt;
        }
        nprev = nk;
    }
    free(y);
    free(lam);
    free(pk);
    free(pkm1);
}

/* Values h_0(x) .. h_n(x) of the orthonormal half-range polynomials (recurrence above). */
static void half_values_q(int n, const qreal* a, const qreal* b, qreal x, qreal* hv)
{
    hv[0] = 1 / sqrtq(b[0]);
    if (n >= 1) hv[1] = (x - a[0]) * hv[0] / b[1];
    for (int l = 1; l < n; l++) hv[l + 1] = ((x - a[l]) * hv[l] - b[l] * hv[l - 1]) / b[l + 1];
}

/* Coefficients hc[l][s] of x^s in h_l (l, s = 0..n), i.e. the paper's h_{l,s}. */
static void half_coeffs_q(int n, const qreal* a, const qreal* b, qreal* hc /* (n+1)^2 */)
{
    memset(hc, 0, sizeof(qreal) * (n + 1) * (n + 1));
    hc[0] = 1 / sqrtq(b[0]);
    for (int l = 0; l < n; l++) {
        for (int s = 0; s <= l + 1; s++) {
            qreal v = 0;
            if (s >= 1) v += hc[l * (n + 1) + s - 1];
            v -= a[l] * hc[l * (n + 1) + s];
            if (l >= 1) v -= b[l] * hc[(l - 1) * (n + 1) + s];
            hc[(l + 1) * (n + 1) + s] = v / b[l + 1];
        }
    }
}

/* Probabilists' Hermite polynomials He_0(x) .. He_n(x)  (He_{l+1} = x He_l - l He_{l-1}). */
static void he_values_q(int n, qreal x, qreal* hv)
{
    hv[0] = 1;
    if (n >= 1) hv[1] = x;
    for (int l = 1; l < n; l++) hv[l + 1] = x * hv[l] - l * hv[l - 1];
}

/* Roots of the degree-Q member of a family given by a monic-value evaluator, found by
 * bisection inside the brackets given by the roots of the degree-(Q-1) member
 * (interlacing of the zeros of orthogonal polynomials).  lo/hi bound all zeros. */
typedef qreal (*poly_eval_fn)(int deg, qreal x, const void* ctx);

static void roots_by_interlacing(int Q, poly_eval_fn ev, const void* ctx, qreal lo, qreal hi,
                                 qreal* roots)
{
    qreal prev[QMAX + 1], cur[QMAX + 1];
    int nprev = 0;
    for (int d = 1; d <= Q; d++) {
        for (int r = 0; r < d; r++) {
            qreal L = (r == 0) ? lo : prev[r - 1];
            qreal R = (r == nprev) ? hi : prev[r];
            qreal fL = ev(d, L, ctx);
            for (int it = 0; it < 400; it++) {
                qreal M = (L + R) / 2;
                if (M <= L || M >= R) break;
                qreal fM = ev(d, M, ctx);
                if (fM == 0) {
                    L = R = M;
                    break;
                }
                if ((fM > 0) == (fL > 0)) {
                    L = M;
                    fL = fM;
                } else {
                    R = M;
                }
            }
            cur[r] = (L + R) / 2;
        }
        for (int r = 0; r < d; r++) prev[r] = cur[r];
        nprev = d;
    }
    for (int r = 0; r < Q; r++) roots[r] = prev[r];
}

typedef struct {
    const qreal* a;
    const qreal* b;
} half_ctx;

static qreal half_eval_cb(int deg, qreal x, const void* vctx)
{
    const half_ctx* c = (const half_ctx*)vctx;
    qreal hv[QMAX + 2];
    half_values_q(deg, c->a, c->b, x, hv);
    return hv[deg];
}

static qreal he_eval_cb(int deg, qreal x, const void* vctx)
{
    (void)vctx;
    qreal hv[QMAX + 2];
    he_values_q(deg, x, hv);
    return hv[deg];
}

/* ======================================================================================
 * 2. Quadratures (Sec. III, "Quadrature choice" and the weight formulas)
 * ====================================================================================== */

/* Half-range Gauss-Hermite rule of order Q: 2Q nodes, positive nodes first (ascending),
 * then their mirrors (Sec. III: indices 1..Q on the positive semi-axis, Q+1..2Q on the
 * negative one).  Weights by the paper's formula
 *   w_i = p_i a_{Q-1}^2 / ( h_{Q-1}(p_i)^2 [ p_i + h_Q(0)^2 / sqrt(2 pi) ] ),
 *   a_l = h_{l+1,l+1} / h_{l,l}.
 * Also returns, in extended precision, the recurrence (a,b) and the coefficient table
 * hc (Q+1)^2 when the pointers are non-null. */
static int half_rule_q(int Q, qreal* nodes, qreal* wts, qreal* ra, qreal* rb, qreal* hc)
{
    qreal a[QMAX + 2], b[QMAX + 3];
    half_recurrence_q(Q + 1, a, b);
    half_ctx ctx = {a, b};
    qreal hi = 0;
    for (int l = 0; l <= Q; l++) {
        qreal g = fabsq(a[l]) + b[l + 1] + (l >= 1 ? b[l] : 0);
        if (g > hi) hi = g;
    }
    qreal r[QMAX + 1];
    roots_by_interlacing(Q, half_eval_cb, &ctx, 0, hi * 1.01Q + 1, r);
    qreal* coef = malloc(sizeof(qreal) * (Q + 2) * (Q + 2));
    half_coeffs_q(Q + 1, a, b, coef);
    qreal hQ0 = coef[Q * (Q + 2) + 0];                             /* h_{Q,0} = h_Q(0) */
    qreal aQm1 = coef[Q * (Q + 2) + Q] / coef[(Q - 1) * (Q + 2) + Q - 1]; /* a_{Q-1} */
    for (int i = 0; i < Q; i++) {
        qreal hv[QMAX + 2];
        half_values_q(Q, a, b, r[i], hv);
        qreal w = r[i] * aQm1 * aQm1 / (hv[Q - 1] * hv[Q - 1] * (r[i] + hQ0 * hQ0 / sqrtq(2 * M_PIq)));
        nodes[i] = r[i];
        nodes[Q + i] = -r[i];
        wts[i] = w;
        wts[Q + i] = w;
    }
    if (ra)
        for (int l = 0; l <= Q; l++) ra[l] = a[l];
    if (rb)
        for (int l = 0; l <= Q + 1; l++) rb[l] = b[l];
    if (hc)
        for (int l = 0; l <= Q; l++)
            for (int s = 0; s <= Q; s++) hc[l * (Q + 1) + s] = coef[l * (Q + 2) + s];
    free(coef);
    return ORC_OK;
}

/* Full-range Gauss-Hermite rule of order Q: roots of the probabilists' He_Q (ascending);
 * weights w_i = Q! / He_{Q+1}(p_i)^2, normalised so that sum w = 1. */
static int full_rule_q(int Q, qreal* nodes, qreal* wts)
{
    qreal r[QMAX + 1];
    qreal hi = 2 * sqrtq((qreal)Q) + 2;
    roots_by_interlacing(Q, he_eval_cb, NULL, -hi, hi, r);
    qreal fact = 1;
    for (int k = 2; k <= Q; k++) fact *= k;
    for (int i = 0; i < Q; i++) {
        qreal hv[QMAX + 2];
        he_values_q(Q + 1, r[i], hv);
        nodes[i] = r[i];
        wts[i] = fact / (hv[Q + 1] * hv[Q + 1]);
    }
    return ORC_OK;
}

int orc_quad_half(int Q, double* nodes, double* weights)
{
    if (Q < 1 || Q > QMAX) return ORC_EINVAL;
    qreal n[2 * QMAX], w[2 * QMAX];
    half_rule_q(Q, n, w, NULL, NULL, NULL);
    for (int i = 0; i < 2 * Q; i++) {
        nodes[i] = (double)n[i];
        weights[i] = (double)w[i];
    }
    return ORC_OK;
}

int orc_quad_full(int Q, double* nodes, double* weights)
{
    if (Q < 1 || Q > QMAX) return ORC_EINVAL;
    qreal n[QMAX], w[QMAX];
    full_rule_q(Q, n, w);
    for (int i = 0; i < Q; i++) {
        nodes[i] = (double)n[i];
        weights[i] = (double)w[i];
    }
    return ORC_OK;
}

/* Recurrence coefficients (a[0..Q], b[0..Q+1]) and coefficient table h_{l,s}
 * (l, s = 0..Q) of the half-range polynomials, rounded to double (for pins). */
int orc_half_poly(int Q, double* a_out, double* b_out, double* hc_out)
{
    if (Q < 1 || Q > QMAX) return ORC_EINVAL;
    qreal n[2 * QMAX], w[2 * QMAX], a[QMAX + 2], b[QMAX + 3];
    qreal* hc = malloc(sizeof(qreal) * (Q + 1) * (Q + 1));
    half_rule_q(Q, n, w, a, b, hc);
    for (int l = 0; l <= Q; l++) a_out[l] = (double)a[l];
    for (int l = 0; l <= Q + 1; l++) b_out[l] = (double)b[l];
    for (int k = 0; k < (Q + 1) * (Q + 1); k++) hc_out[k] = (double)hc[k];
    free(hc);
    return ORC_OK;
}

/* ======================================================================================
 * 3. Force-term matrices (Sec. III.B, eqs. (force1), (force2))
 * ====================================================================================== */

/* Full-range K matrices, as printed:
 *   which = 1 (d f / d p):      K_{ii'} = -w_i sum_{l=0}^{Q-1} He_{l+1}(p_i) He_l(p_i') / l!
 *   which = 2 (d (f p) / d p):  K_{ii'} = -w_i sum_{l=0}^{Q-2} He_{l+1}(p_i)
 *                                          [He_{l+1}(p_i') + l He_{l-1}(p_i')] / l!      */
static void kmat_full_q(int Q, int which, const qreal* p, const qreal* w, double* K)
{
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++) {
            qreal hi[QMAX + 2], hj[QMAX + 2];
            he_values_q(Q + 1, p[i], hi);
            he_values_q(Q + 1, p[j], hj);
            qreal s = 0, fact = 1;
            if (which == 1) {
                for (int l = 0; l <= Q - 1; l++) {
                    if (l >= 2) fact *= l;
                    s += hi[l + 1] * hj[l] / fact;
                }
            } else {
                for (int l = 0; l <= Q - 2; l++) {
                    if (l >= 2) fact *= l;
                    qreal t = hj[l + 1] + (l >= 1 ? l * hj[l - 1] : 0);
                    s += hi[l + 1] * t / fact;
                }
            }
            K[i * Q + j] = (double)(-w[i] * s);
        }
}

/* Half-range K matrices (size 2Q x 2Q), as printed, with sigma_i = sign(p_i).
 * Reading (the printed formulas carry label typos): every polynomial argument is |p| of
 * the same axis, the index j' in the second matrix is i', and terms whose polynomial or
 * coefficient index is negative are absent.
 *   which = 1:  K_{ii'} = w_i s_i { (1+s_i s_i')/2 sum_{l=0}^{Q-2} h_l(|p_i'|)
 *                    [ h_{l,0}/sqrt(2pi) sum_{s=l+1}^{Q-1} h_{s,0} h_s(|p_i|)
 *                      - (h_{l,l}/h_{l+1,l+1}) h_{l+1}(|p_i|) ]
 *                  - Phi_0^Q(|p_i|) Phi_0^Q(|p_i'|) / (2 sqrt(2pi)) },
 *               Phi_s^n(x) = sum_{l=s}^n h_{l,s} h_l(x);
 *   which = 2:  K_{ii'} = -w_i (1+s_i s_i')/2 sum_{l=0}^{Q-1} h_l(|p_i|) [ l h_l(|p_i'|)
 *                    + (h_{l,0}^2 + h_{l-1,0}^2)/(a_{l-1} sqrt(2pi)) h_{l-1}(|p_i'|)
 *                    + h_{l-2}(|p_i'|)/(a_{l-1} a_{l-2}) ],   a_l = h_{l+1,l+1}/h_{l,l}.  */
static void kmat_half_q(int Q, int which, const qreal* p, const qreal* w, const qreal* ra,
                        const qreal* rb, const qreal* hc, double* K)
{
    const int n = 2 * Q;
    const qreal s2pi = sqrtq(2 * M_PIq);
#define HC(l, s) hc[(l) * (Q + 1) + (s)]
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            qreal si = p[i] > 0 ? 1 : -1, sj = p[j] > 0 ? 1 : -1;
            qreal hi[QMAX + 2], hj[QMAX + 2];
            half_values_q(Q, ra, rb, fabsq(p[i]), hi);
            half_values_q(Q, ra, rb, fabsq(p[j]), hj);
            qreal same = (1 + si * sj) / 2;
            qreal val;
            if (which == 1) {
                qreal acc = 0;
                for (int l = 0; l <= Q - 2; l++) {
                    qreal inner = 0;
                    for (int s = l + 1; s <= Q - 1; s++) inner += HC(s, 0) * hi[s];
                    acc += hj[l] * (HC(l, 0) / s2pi * inner - HC(l, l) / HC(l + 1, l + 1) * hi[l + 1]);
                }
                qreal phi_i = 0, phi_j = 0;
                for (int l = 0; l <= Q; l++) {
                    phi_i += HC(l, 0) * hi[l];
                    phi_j += HC(l, 0) * hj[l];
                }
                val = w[i] * si * (same * acc - phi_i * phi_j / (2 * s2pi));
            } else {
                qreal acc = 0;
                for (int l = 0; l <= Q - 1; l++) {
                    qreal t = l * hj[l];
                    if (l >= 1) {
                        qreal alm1 = HC(l, l) / HC(l - 1, l - 1);
                        t += (HC(l, 0) * HC(l, 0) + HC(l - 1, 0) * HC(l - 1, 0)) / (alm1 * s2pi) * hj[l - 1];
                        if (l >= 2) {
                            qreal alm2 = HC(l - 1, l - 1) / HC(l - 2, l - 2);
                            t += hj[l - 2] / (alm1 * alm2);
                        }
                    }
                    acc += hi[l] * t;
                }
                val = -w[i] * same * acc;
            }
            K[i * n + j] = (double)val;
        }
#undef HC
}

int orc_kmat_full(int Q, int which, double* K)
{
    if (Q < 1 || Q > QMAX || (which != 1 && which != 2)) return ORC_EINVAL;
    qreal p[QMAX], w[QMAX];
    full_rule_q(Q, p, w);
    kmat_full_q(Q, which, p, w, K);
    return ORC_OK;
}

int orc_kmat_half(int Q, int which, double* K)
{
    if (Q < 1 || Q > QMAX || (which != 1 && which != 2)) return ORC_EINVAL;
    qreal p[2 * QMAX], w[2 * QMAX], a[QMAX + 2], b[QMAX + 3];
    qreal* hc = malloc(sizeof(qreal) * (Q + 1) * (Q + 1));
    half_rule_q(Q, p, w, a, b, hc);
    kmat_half_q(Q, which, p, w, a, b, hc, K);
    free(hc);
    return ORC_OK;
}

/* ======================================================================================
 * 4. Discrete equilibrium (Sec. III.C)
 * ====================================================================================== */

/* Per-axis tables needed by the equilibrium, in double:
 *   full-range: He_l(p_k) for l = 0..N;
 *   half-range: Phi_s^N(|p_k|) = sum_{l=s}^N h_{l,s} h_l(|p_k|) for s = 0..N. */
typedef struct {
    int half;  /* 1 = half-range axis */
    int Q;     /* quadrature order */
    int nq;    /* number of nodes (2Q or Q) */
    int N;     /* expansion order */
    double* p; /* nodes */
    double* w; /* weights */
    qreal* tab; /* nq x (N+1): He_l(p_k) or Phi_s^N(|p_k|), kept in __float128 */
    qreal* wl;  /* weights in __float128 */
} axis_t;

static int axis_build(axis_t* ax, int half, int Q, int N)
{
    ax->half = half;
    ax->Q = Q;
    ax->nq = half ? 2 * Q : Q;
    ax->N = N;
    ax->p = malloc(sizeof(double) * ax->nq);
    ax->w = malloc(sizeof(double) * ax->nq);
    ax->tab = malloc(sizeof(qreal) * ax->nq * (N + 1));
    ax->wl = malloc(sizeof(qreal) * ax->nq);
    if (!ax->p || !ax->w || !ax->tab || !ax->wl) return ORC_ENOMEM;
    if (half) {
        qreal p[2 * QMAX], w[2 * QMAX], a[QMAX + 2], b[QMAX + 3];
        qreal* hc = malloc(sizeof(qreal) * (Q + 1) * (Q + 1));
        half_rule_q(Q, p, w, a, b, hc);
        for (int k = 0; k < ax->nq; k++) {
            ax->p[k] = (double)p[k];
            ax->w[k] = (double)w[k];
            ax->wl[k] = w[k];
            qreal hv[QMAX + 2];
            half_values_q(Q, a, b, fabsq(p[k]), hv);
            for (int s = 0; s <= N; s++) {
                qreal phi = 0;
                for (int l = s; l <= N; l++) phi += hc[l * (Q + 1) + s] * hv[l];
                ax->tab[k * (N + 1) + s] = phi;
            }
        }
        free(hc);
    } else {
        qreal p[QMAX], w[QMAX];
        full_rule_q(Q, p, w);
        for (int k = 0; k < Q; k++) {
            ax->p[k] = (double)p[k];
            ax->w[k] = (double)w[k];
            ax->wl[k] = w[k];
            qreal hv[QMAX + 2];
            he_values_q(N, p[k], hv);
            for (int l = 0; l <= N; l++) ax->tab[k * (N + 1) + l] = hv[l];
        }
    }
    return ORC_OK;
}

static void axis_free(axis_t* ax)
{
    free(ax->p);
    free(ax->w);
    free(ax->tab);
    free(ax->wl);
}

/* Polynomials of Sec. III.C: P_s^{+-}(x) = e^{-+x^2} d^s/dx^s e^{+-x^2} and
 * P_s^*(x) = sum_{j=0}^{s-1} binom(s,j) P_j^+(x) P_{s-j-1}^-(x), as coefficient arrays
 * (degree <= s).  Built from P_{s+1}^{+-} = (P_s^{+-})' +- 2x P_s^{+-}. */
static qreal PPLUS[NMAX + 1][NMAX + 2], PMINUS[NMAX + 1][NMAX + 2], PSTAR[NMAX + 1][NMAX + 2];
static int ptables_ready = 0;

static void build_ptables(void)
{
    if (ptables_ready) return;
    memset(PPLUS, 0, sizeof(PPLUS));
    memset(PMINUS, 0, sizeof(PMINUS));
    memset(PSTAR, 0, sizeof(PSTAR));
    PPLUS[0][0] = 1;
    PMINUS[0][0] = 1;
    for (int s = 0; s < NMAX; s++)
        for (int d = 0; d <= s + 1; d++) {
            qreal der_p = (d + 1 <= s) ? (d + 1) * PPLUS[s][d + 1] : 0;
            qreal der_m = (d + 1 <= s) ? (d + 1) * PMINUS[s][d + 1] : 0;
            qreal sh_p = (d >= 1) ? PPLUS[s][d - 1] : 0;
            qreal sh_m = (d >= 1) ? PMINUS[s][d - 1] : 0;
            PPLUS[s + 1][d] = der_p + 2 * sh_p;
            PMINUS[s + 1][d] = der_m - 2 * sh_m;
        }
    for (int s = 1; s <= NMAX; s++) {
        qreal binom = 1;
        for (int j = 0; j <= s - 1; j++) {
            if (j > 0) binom = binom * (s - j + 1) / j;
            for (int d1 = 0; d1 <= j; d1++)
                for (int d2 = 0; d2 <= s - j - 1; d2++)
                    PSTAR[s][d1 + d2] += binom * PPLUS[j][d1] * PMINUS[s - j - 1][d2];
        }
    }
    ptables_ready = 1;
}

static qreal poly_eval(const qreal* c, int deg, qreal x)
{
    qreal r = 0;
    for (int d = deg; d >= 0; d--) r = r * x + c[d];
    return r;
}

/* Full-range factor, eq. (eq_gak_H) with m = 1:
 *   g_k = w_k sum_{l=0}^{N} He_l(p_k) sum_{s=0}^{floor(l/2)} (T-1)^s u^{l-2s} / (2^s s! (l-2s)!)
 * The sums are accumulated in __float128 and rounded once: in the half-range case below the
 * printed monomial-basis sum cancels by up to ~1e6 (Hankel conditioning), so plain double or
 * long double evaluation would leave errors of 1e-13..1e-10 in g. */
static void geq_full(const axis_t* ax, double u_, double T_, double* g)
{
    const int N = ax->N;
    const qreal u = u_, T = T_;
    qreal coef[NMAX + 1];
    for (int l = 0; l <= N; l++) {
        qreal c = 0;
        for (int s = 0; 2 * s <= l; s++) {
            qreal den = powq(2, s);
            for (int k = 2; k <= s; k++) den *= k;
            for (int k = 2; k <= l - 2 * s; k++) den *= k;
            c += powq(T - 1, s) * powq(u, l - 2 * s) / den;
        }
        coef[l] = c;
    }
    for (int k = 0; k < ax->nq; k++) {
        qreal acc = 0;
        for (int l = 0; l <= N; l++) acc += ax->tab[k * (N + 1) + l] * coef[l];
        g[k] = (double)(ax->wl[k] * acc);
    }
}

/* Half-range factor, eq. (eq_gak_hh) with m = 1:
 *   g_k = (w_k/2) sum_{s=0}^{N} (T/2)^{s/2} Phi_s^N(|p_k|)
 *          [ (1 + erf z) P_s^+(z) + (2/sqrt(pi)) e^{-z^2} P_s^*(z) ],
 *   z = u sqrt(1/(2T)) for p_k > 0 and z = -u sqrt(1/(2T)) for p_k < 0.
 * Evaluated in qreal (the monomial-basis sum cancels strongly). */
static void geq_half(const axis_t* ax, double u_, double T_, double* g)
{
    build_ptables();
    const int N = ax->N;
    const qreal u = u_, T = T_;
    qreal bracket[2][NMAX + 1];
    for (int side = 0; side < 2; side++) {
        qreal z = (side == 0 ? u : -u) * sqrtq(1 / (2 * T));
        qreal e = erfq(z), ex = expq(-z * z);
        for (int s = 0; s <= N; s++) {
            qreal pp = poly_eval(PPLUS[s], s, z);
            qreal ps = (s >= 1) ? poly_eval(PSTAR[s], s - 1, z) : 0;
            bracket[side][s] = powq(T / 2, 0.5Q * s) * ((1 + e) * pp + 2 / sqrtq(M_PIq) * ex * ps);
        }
    }
    for (int k = 0; k < ax->nq; k++) {
        int side = ax->p[k] > 0 ? 0 : 1;
        qreal acc = 0;
        for (int s = 0; s <= N; s++) acc += ax->tab[k * (N + 1) + s] * bracket[side][s];
        g[k] = (double)(ax->wl[k] / 2 * acc);
    }
}

static void geq_axis(const axis_t* ax, double u, double T, double* g)
{
    if (ax->half)
        geq_half(ax, u, T, g);
    else
        geq_full(ax, u, T, g);
}

int orc_geq(int half, int Q, int N, double u, double T, double* g)
{
    if (Q < 1 || Q > QMAX || N < 0 || N > NMAX || N >= Q) return ORC_EINVAL;
    axis_t ax;
    if (axis_build(&ax, half, Q, N) != ORC_OK) return ORC_ENOMEM;
    geq_axis(&ax, u, T, g);
    axis_free(&ax);
    return ORC_OK;
}

/* ======================================================================================
 * 5. Closed forms of Sec. II: chi, transport coefficients, Kn map
 * ====================================================================================== */

/* Carnahan-Starling contact value, eq. (chi): chi = (2 - eta) / (2 (1 - eta)^3). */
double orc_chi(double eta) { return (2 - eta) / (2 * (1 - eta) * (1 - eta) * (1 - eta)); }

/* Kn = 1/(6 sqrt(2) eta0 chi(eta0) C)  =>  C = 1/(6 sqrt(2) eta0 chi(eta0) Kn). */
double orc_confinement(double eta0, double kn) { return 1 / (6 * sqrt(2.0) * eta0 * orc_chi(eta0) * kn); }
double orc_knudsen(double eta0, double C) { return 1 / (6 * sqrt(2.0) * eta0 * orc_chi(eta0) * C); }

/* Prandtl number, eq. (prandtl), as a function of x = b rho chi. */
double orc_prandtl(double x)
{
    double num = 1 + 0.8 * x + 4.0 / 25 * (1 + 12 / PI) * x * x;
    double den = 1 + 1.2 * x + 9.0 / 25 * (1 + 32 / (9 * PI)) * x * x;
    return 2.0 / 3 * num / den;
}

/* Relaxation time, eqs. (viscosity), (tau): tau = mu / P_i with P_i = n T and
 *   mu = mu_0 [1/chi + 4/5 b rho + 4/25 (1 + 12/pi) (b rho)^2 chi],
 *   mu_0 = 5/(16 sigma^2) sqrt(T/pi).
 * Reading (units): m = k_B = T_0 = 1, lengths in L = R_R - R_L, n normalised to mean 1 so
 * that b rho = 4 eta0 n; the mean physical density is n_0 = 6 eta0/(pi sigma^3) and
 * sigma = L / C.  Substituting gives
 *   tau = (5 sqrt(2 pi)/16) chi(eta0) Kn L [1/chi + 4/5 brho + 4/25(1+12/pi) brho^2 chi]/(n sqrt T). */
double orc_tau(double chi0, double kn, double L, double n, double T, double chi, double brho)
{
    double bracket = 1 / chi + 0.8 * brho + 4.0 / 25 * (1 + 12 / PI) * brho * brho * chi;
    return 5 * sqrt(2 * PI) / 16 * chi0 * kn * L * bracket / (n * sqrt(T));
}

/* ======================================================================================
 * 6. Volume intersections for the averaged density (eq. (fm), Appendix A)
 * ====================================================================================== */

/* Volume of the ball of radius s centred at distance b from the origin lying inside the
 * ball of radius R about the origin (Appendix A, two spheres):
 *   V = pi (r1 + r2 - d)^2 (d^2 + 2 d r2 - 3 r2^2 + 2 d r1 + 6 r1 r2 - 3 r1^2) / (12 d),
 * with the disjoint / nested cases handled explicitly. */
double orc_vol_sph(double s, double R, double b)
{
    const double ball = 4.0 / 3 * PI * s * s * s;
    if (R <= 0) return 0;
    if (b + s <= R) return ball;
    if (b >= R + s) return 0;
    if (b + R <= s) return 4.0 / 3 * PI * R * R * R;
    double r1 = s, r2 = R, d = b;
    return PI * (r1 + r2 - d) * (r1 + r2 - d) * (d * d + 2 * d * r2 - 3 * r2 * r2 + 2 * d * r1 + 6 * r1 * r2 - 3 * r1 * r1) /
           (12 * d);
}

/* Planar channel (the Cartesian model equation of Sec. II, the R_L -> infinity limit): volume of the
 * ball of radius s centred at x = b that lies at x < X, a spherical cap of height h = X - (b - s):
 * pi h^2 (3 s - h) / 3. */
double orc_vol_slab(double s, double X, double b)
{
    if (X <= b - s) return 0;
    if (X >= b + s) return 4.0 / 3 * PI * s * s * s;
    double h = X - (b - s);
    return PI * h * h * (3 * s - h) / 3;
}

/* alpha - sin(alpha) cos(alpha), the area of a circular segment of unit radius with half
 * angle alpha; a Taylor series for small alpha avoids the cancellation. */
static double seg_area(double a)
{
    if (a < 0.25) {
        double x = 2 * a, x2 = x * x, term = x * x2 / 6, sum = 0;
        for (int k = 1; k < 12; k++) {
            sum += term;
            term *= -x2 / ((2 * k + 2) * (2 * k + 3));
        }
        return sum / 2;
    }
    return a - sin(a) * cos(a);
}

/* Area of the intersection of a disk of radius rho centred at distance b from the origin
 * with the disk of radius R about the origin (plane geometry): the sum of the two circular
 * segments cut off by the common chord, whose half length is h = sqrt(k)/(2b) by Heron. */
static double disk_lens_area(double rho, double R, double b)
{
    if (rho <= 0) return 0;
    if (b + rho <= R) return PI * rho * rho;
    if (b >= R + rho) return 0;
    if (b + R <= rho) return PI * R * R;
    double k = (-b + rho + R) * (b + rho - R) * (b - rho + R) * (b + rho + R);
    if (k < 0) k = 0;
    double h = sqrt(k) / (2 * b);
    double a1 = atan2(h, ((b - R) * (b + R) + rho * rho) / (2 * b));
    double a2 = atan2(h, ((b - rho) * (b + rho) + R * R) / (2 * b));
    return rho * rho * seg_area(a1) + R * R * seg_area(a2);
}

/* 10-point Gauss-Legendre rule on [-1,1] (double), generated once. */
static double GL10X[10], GL10W[10];
static int gl10_ready = 0;
static void gl10_init(void)
{
    if (gl10_ready) return;
    qreal x[10], w[10];
    gl_rule_q(10, x, w);
    for (int i = 0; i < 10; i++) {
        GL10X[i] = (double)x[i];
        GL10W[i] = (double)w[i];
    }
    gl10_ready = 1;
}

typedef struct {
    double s, R, b, zs;
} lens_ctx;

/* Integrand of the slice integral over [0, z*] after z = z*(1 - t^2). */
static double lens_integrand(double t, const lens_ctx* c)
{
    double z = c->zs * (1 - t * t);
    double rho2 = c->s * c->s - z * z;
    double rho = rho2 > 0 ? sqrt(rho2) : 0;
    return disk_lens_area(rho, c->R, c->b) * 2 * c->zs * t;
}

static double gl10_on(double lo, double hi, const lens_ctx* c)
{
    double m = (lo + hi) / 2, h = (hi - lo) / 2, acc = 0;
    for (int i = 0; i < 10; i++) acc += GL10W[i] * lens_integrand(m + h * GL10X[i], c);
    return acc * h;
}

/* Adaptive bisection: accept an interval when the 10-point rule on it and on its two halves
 * agree to tol (an absolute tolerance, the same for every interval). */
static double adapt_gl(double lo, double hi, double whole, const lens_ctx* c, double tol, int depth)
{
    double m = (lo + hi) / 2;
    double left = gl10_on(lo, m, c), right = gl10_on(m, hi, c);
    double err = fabs(left + right - whole);
    if (depth >= 24 || err <= tol) return left + right;
    return adapt_gl(lo, m, left, c, tol, depth + 1) + adapt_gl(m, hi, right, c, tol, depth + 1);
}

/* Volume of the ball of radius s centred at distance b from the axis lying inside the
 * infinite cylinder of radius R (the quantity Appendix A evaluates with elliptic
 * integrals).  The oracle uses the plain definition instead: V = 2 int_0^s A(z) dz, where
 * A(z) is the area of the plane section, i.e. the intersection of the disk of radius
 * sqrt(s^2 - z^2) centred at distance b with the disk of radius R.  The section is a
 * partial lens for z < z* = sqrt(s^2 - (R-b)^2); beyond z* it is the whole disk (b < R) or
 * empty (b > R) and is integrated in closed form.  The lens part is integrated by adaptive
 * 10-point Gauss-Legendre after the substitution z = z*(1 - t^2), which removes the
 * (z* - z)^{3/2} behaviour at the tangency. */
double orc_vol_cyl(double s, double R, double b)
{
    gl10_init();
    const double ball = 4.0 / 3 * PI * s * s * s;
    if (R <= 0) return 0;
    double gap = fabs(R - b);
    if (b + s <= R) return ball;
    if (b >= R + s) return 0;
    if (b + R <= s) {
        /* cylinder section inside every slice of the ball near z = 0: handled by the
         * general integral below with z* = 0 (never reached for s < R) */
    }
    double zs = sqrt(s * s - gap * gap);
    lens_ctx c = {s, R, b, zs};
    double whole = gl10_on(0, 1, &c);
    double lens = adapt_gl(0, 1, whole, &c, 1e-17 * ball, 0);
    double tail = 0;
    if (b < R) tail = PI * (s * s * (s - zs) - (s * s * s - zs * zs * zs) / 3);
    return 2 * (lens + tail);
}

/* ======================================================================================
 * 6b. Attractive mean field (Enskog-Vlasov), beyond the paper: Sec. V names attractive forces
 *     between molecules as the next step towards multiphase flows.
 *
 * Reading: the attraction is a Sutherland tail phi(t) = -phi_a (sigma / t)^6 for t > sigma
 * (zero inside the core, whose effect stays with the Enskog collision terms), treated in the
 * mean-field (Vlasov) approximation: the potential energy of a molecule at x is
 *   Phi(x) = n0 int n(x') phi(|x - x'|) d^3x',   n0 sigma^3 = 6 eta0 / pi,
 * with n in units of n0 and n = 0 outside the computational domain (as for nbar), and the
 * force F = -dPhi/dr acts along the radial axis, adding F df/dp_r to the left-hand side of
 * the kinetic equation.  With n piecewise constant on cells, Phi_i = sum_j A_ij n_j with
 *   A_ij = n0 [U(r_i; ri_{j+1}) - U(r_i; ri_j)],
 * where U(r; s) is the integral of phi over the region of "radius" s (the ball |x'| < s, the
 * infinite cylinder R' < s, or the half space x' < s) seen from a point at radius r.
 *
 * The oracle evaluates U from its definition, about the point: t is the distance from the
 * point and M(t) the measure of the sphere of radius t about it inside the region,
 *   U = int_sigma^inf phi(t) M(t) dt,
 * (sphere: M is a spherical cap area, plane: the part of the sphere on one side of a plane).
 * For the cylinder the axial direction is integrated first, the line integral
 *   lam(d) = int phi(sqrt(d^2 + z^2)) dz  (d: distance from the point's axis-parallel line),
 * then U = int_0^{r+s} lam(d) d arc(d) dd with arc(d) the angle of the circle of radius d
 * about the point inside the disk of radius s.  Every one-dimensional integral is adaptive
 * 10-point Gauss-Legendre on the pieces between the points where the integrand has a kink
 * (t = sigma, t = |r - s|); pieces with square-root ends (the cylinder's arc and lam) are
 * taken in the variable theta of d = p + (q - p)(1 - cos theta) / 2, which makes them smooth.
 * ====================================================================================== */

typedef double (*mf_fn)(double x, const void* ctx);

static double mf_gl10(mf_fn f, const void* c, double lo, double hi)
{
    double m = (lo + hi) / 2, h = (hi - lo) / 2, acc = 0;
    for (int i = 0; i < 10; i++) acc += GL10W[i] * f(m + h * GL10X[i], c);
    return acc * h;
}

static double mf_adapt(mf_fn f, const void* c, double lo, double hi, double whole, double tol, int depth)
{
    double m = (lo + hi) / 2;
    double left = mf_gl10(f, c, lo, m), right = mf_gl10(f, c, m, hi);
    if (depth >= 30 || fabs(left + right - whole) <= tol) return left + right;
    return mf_adapt(f, c, lo, m, left, tol, depth + 1) + mf_adapt(f, c, m, hi, right, tol, depth + 1);
}

static double mf_integrate(mf_fn f, const void* c, double lo, double hi, double tol)
{
    if (!(hi > lo)) return 0;
    return mf_adapt(f, c, lo, hi, mf_gl10(f, c, lo, hi), tol, 0);
}

/* Line integral of t^-6 (t = sqrt(d^2 + z^2)) over the z with t > sigma, by z = d cot(beta):
 * 2 d^-5 int_0^beta0 sin^4(beta) dbeta with beta0 = atan(d / z0), z0 = sqrt(sigma^2 - d^2)
 * (beta0 = pi/2 for d >= sigma); four 10-point panels. */
static double mf_line(double d, double sigma)
{
    double z0 = d < sigma ? sqrt((sigma - d) * (sigma + d)) : 0;
    double b0 = atan2(d, z0), acc = 0;
    for (int p = 0; p < 4; p++) {
        double lo = b0 * p / 4, hi = b0 * (p + 1) / 4, m = (lo + hi) / 2, h = (hi - lo) / 2;
        for (int k = 0; k < 10; k++) {
            double sb = sin(m + h * GL10X[k]);
            acc += h * GL10W[k] * sb * sb * sb * sb;
        }
    }
    return 2 * acc / (d * d * d * d * d);
}

typedef struct {
    int geo;
    double sigma, r, s;
    double p, q;   /* piece of the cylinder integral (theta substitution) */
    double t1;     /* start of the plane's mapped tail */
} mf_ctx;

/* Measure of the sphere of radius t about the point inside the region (ball or half space). */
static double mf_measure(const mf_ctx* c, double t)
{
    if (c->geo == 1) { /* ball |x'| < s about the origin, point at distance r */
        if (t + c->r <= c->s) return 4 * PI * t * t;
        if (t >= c->r + c->s || t + c->s <= c->r) return 0;
        /* cap: directions w with |x + t w| < s, i.e. cos(angle to x) < (s^2 - r^2 - t^2)/(2 r t) */
        double mu = (c->s * c->s - c->r * c->r - t * t) / (2 * c->r * t);
        return 2 * PI * t * t * (1 + mu);
    }
    /* half space x' < s, point at x = r: signed distance h = s - x */
    double h = c->s - c->r;
    if (t <= -h) return 0;
    if (t <= h) return 4 * PI * t * t;
    return 2 * PI * t * (t + h);
}

static double mf_radial_integrand(double t, const void* vc)
{
    const mf_ctx* c = vc;
    double t2 = t * t;
    return mf_measure(c, t) / (t2 * t2 * t2);
}

/* plane tail t >= t1 in u = t1 / t */
static double mf_tail_integrand(double u, const void* vc)
{
    const mf_ctx* c = vc;
    if (u <= 0) return 0;
    double t = c->t1 / u;
    return mf_radial_integrand(t, c) * c->t1 / (u * u);
}

/* angle of the circle of radius d about the point (distance r from the axis) inside the disk
 * of radius s */
static double mf_arc(double d, double r, double s)
{
    if (r + d <= s) return 2 * PI;
    if (d >= r + s || d + s <= r) return 0;
    double cz = (r * r + d * d - s * s) / (2 * r * d);
    if (cz > 1) cz = 1;
    if (cz < -1) cz = -1;
    return 2 * acos(cz);
}

static double mf_cyl_integrand(double th, const void* vc)
{
    const mf_ctx* c = vc;
    double hw = (c->q - c->p) / 2;
    double d = c->p + hw * (1 - cos(th));
    if (d <= 0) return 0;
    return mf_line(d, c->sigma) * d * mf_arc(d, c->r, c->s) * hw * sin(th);
}

static int mf_cmp(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* U(r; s) (see above) for geometry 0 cylinder, 1 sphere, 2 plane; the point at radius (plane:
 * position) r, the region of radius (plane: x' <) s. */
double orc_mf_potential(int geometry, double sigma, double phi_a, double r, double s)
{
    gl10_init();
    mf_ctx c = {geometry, sigma, r, s, 0, 0, 0};
    const double s3 = sigma * sigma * sigma, amp = -phi_a * s3 * s3; /* phi(t) = amp t^-6 */
    const double tol = 4e-16 / s3; /* absolute, per interval: the integrals are of order 1 / sigma^3 */
    double acc = 0;
    if (geometry == 0) {
        double bp[4] = {0, sigma, fabs(r - s), r + s};
        qsort(bp, 4, sizeof(double), mf_cmp);
        for (int k = 0; k < 3; k++) {
            double lo = bp[k], hi = fmin(bp[k + 1], r + s);
            if (!(hi > lo)) continue;
            c.p = lo;
            c.q = hi;
            acc += mf_integrate(mf_cyl_integrand, &c, 0, PI, tol);
        }
        return amp * acc;
    }
    if (geometry == 1) {
        /* kinks at |r - s| and r + s (equal at the centre, r = 0) */
        double top = r + s, mid = fabs(r - s);
        if (mid > sigma) acc += mf_integrate(mf_radial_integrand, &c, sigma, fmin(mid, top), tol);
        acc += mf_integrate(mf_radial_integrand, &c, fmax(sigma, mid), top, tol);
        return amp * acc;
    }
    /* plane: kink at |h|, then the tail beyond t1 = 2 max(sigma, |h|) mapped to (0, 1] */
    double ah = fabs(s - r);
    c.t1 = 2 * fmax(sigma, ah);
    if (ah > sigma) {
        acc += mf_integrate(mf_radial_integrand, &c, sigma, ah, tol);
        acc += mf_integrate(mf_radial_integrand, &c, ah, c.t1, tol);
    } else {
        acc += mf_integrate(mf_radial_integrand, &c, sigma, c.t1, tol);
    }
    acc += mf_integrate(mf_tail_integrand, &c, 0, 1, tol);
    return amp * acc;
}

/* ======================================================================================
 * 7. The solver
 * ====================================================================================== */

typedef struct {
    int32_t geometry; /* 0 cylindrical (R, phi, z), 1 spherical (r, theta, phi) */
    double r_inner, r_outer;
    double u_wall_inner; /* tangential speed of the inner wall along the first transverse axis */
    double t_wall_inner, t_wall_outer;
    double eta0, kn;
    int32_t nr, q_radial, q_t1, q_t2;
    int32_t n_expand[3];
    double cfl;
    int32_t reduced; /* cylinder only: p_z integrated out (see "Reduced distributions" below) */
    double phi_a;    /* depth of the attractive tail in units of k_B T (section 6b); 0: none */
} orc_params;

typedef struct {
    orc_params prm;
    int nr, nv, n0, n1, n2; /* nodes per axis: n0 = 2 Q_R, n1, n2 */
    axis_t ax[3];
    double chi0, C, L, sigma, rcl, rcr, dr, dt;
    double* r;     /* node radii r_i */
    double* ri;    /* interface radii, nr + 1 */
    double* vol;   /* cell measures (r_i dr or (ri_{i+1}^3 - ri_i^3)/3) */
    double* W;     /* nr x nr averaged-density weights */
    double* Amf;   /* nr x nr mean-field weights A_ij (section 6b), NULL without attraction */
    double* K1;    /* (n0 x n0) d/dp along the radial axis (half-range) */
    double* K2a;   /* (n1 x n1) d(f p)/dp along transverse axis 1 */
    double* K2b;   /* (n2 x n2) d(f p)/dp along transverse axis 2 (spherical only) */
    double* gwl;   /* unit wall Maxwellians, nv each */
    double* gwr;
    double gin_l, gin_r; /* sum over incoming velocities of p_R * unit wall Maxwellian */
    double* f;     /* state nr x nv */
    double* fs1;   /* stage buffers */
    double* fs2;
    double* Lbuf;
    double* mom_prev; /* moments at the start of the last step: 5 x nr (n, u0, u1, u2, T) */
    double last_resid;
    int64_t steps;
    int nan_flag;
    int reduced;
} orc_solver;

/* Per-node macroscopic block computed from f, eqs. (macro_def) with quadrature sums
 * (mom_quad): raw sums first (n, j), then central sums with xi = p - u. */
typedef struct {
    double n, u[3], T, q[3], P[3][3];
    double nbar, chi, tau, Pr, brhochi;
    double phi, F; /* mean-field potential and radial force (zero without attraction) */
    double dlog_nnchiT, dlogT, du[3]; /* radial gradients used by J1 */
} node_t;

static inline void vel_of(const orc_solver* s, int v, double p[3])
{
    int i0 = v % s->n0;
    int rest = v / s->n0;
    int i1 = rest % s->n1;
    int i2 = rest / s->n1;
    p[0] = s->ax[0].p[i0];
    p[1] = s->ax[1].p[i1];
    p[2] = s->ax[2].p[i2];
}

/* Reduced distributions (cylinder, Sec. III "Quadrature choice": the trivial p_z dependence is
 * integrated out at the level of the model equation).  Reading: the state holds
 *   phi(R, p_R, p_phi) = int f dp_z   (velocity index i2 = 0) and
 *   chi(R, p_R, p_phi) = int p_z^2 f dp_z   (i2 = 1),
 * on the mixed (p_R, p_phi) quadrature, with u_z = q_z = 0 by the symmetry of the flow.  Both obey
 * the transport of f itself (radial advection and the (p_R, p_phi) force terms do not involve p_z).
 * Their collision terms are the p_z-integrals of eqs. (j0), (j1) over the Maxwellian factor in p_z
 * (mean 0, variance T): a polynomial linear in xi_z^2 integrates to its value at xi_z^2 = T
 * (weight 1) and, times p_z^2, to T times its value at xi_z^2 = 3T (since int p^4 G = 3T^2). */
static inline int is_chi(const orc_solver* s, int v) { return s->reduced && v / (s->n0 * s->n1) == 1; }

/* Factors of the third axis of the equilibrium: the discrete projection of Sec. III.C, or for the
 * reduced distributions the p_z-integrals int G dp_z = 1 and int p_z^2 G dp_z = T. */
static void zfactors(const orc_solver* s, double u2, double T, double* g2)
{
    if (s->reduced) {
        g2[0] = 1;
        g2[1] = T;
    } else {
        geq_axis(&s->ax[2], u2, T, g2);
    }
}


static void node_moments_reduced(const orc_solver* s, const double* fi, node_t* m)
{
    /* n, momentum from phi; the energy adds sum chi = int xi_z^2 f (u_z = 0). */
    double n = 0, j[2] = {0, 0};
    for (int v = 0; v < s->nv; v++) {
        if (is_chi(s, v)) continue;
        double p[3];
        vel_of(s, v, p);
        n += fi[v];
        j[0] += fi[v] * p[0];
        j[1] += fi[v] * p[1];
    }
    m->n = n;
    m->u[0] = j[0] / n;
    m->u[1] = j[1] / n;
    m->u[2] = 0;
    double e2 = 0, q[3] = {0, 0, 0}, P[3][3] = {{0}};
    for (int v = 0; v < s->nv; v++) {
        double p[3];
        vel_of(s, v, p);
        double xi[2] = {p[0] - m->u[0], p[1] - m->u[1]};
        if (is_chi(s, v)) {
            e2 += fi[v];
            for (int a = 0; a < 2; a++) q[a] += 0.5 * fi[v] * xi[a];
            P[2][2] += fi[v];
        } else {
            double x2 = xi[0] * xi[0] + xi[1] * xi[1];
            e2 += fi[v] * x2;
            for (int a = 0; a < 2; a++) {
                q[a] += 0.5 * fi[v] * x2 * xi[a];
                for (int b = 0; b < 2; b++) P[a][b] += fi[v] * xi[a] * xi[b];
            }
        }
    }
    m->T = e2 / (3 * n);
    for (int a = 0; a < 3; a++) {
        m->q[a] = q[a];
        for (int b = 0; b < 3; b++) m->P[a][b] = P[a][b];
    }
}

static void node_moments(const orc_solver* s, const double* fi, node_t* m)
{
    if (s->reduced) {
        node_moments_reduced(s, fi, m);
        return;
    }
    double n = 0, j[3] = {0, 0, 0};
    for (int v = 0; v < s->nv; v++) {
        double p[3];
        vel_of(s, v, p);
        n += fi[v];
        for (int a = 0; a < 3; a++) j[a] += fi[v] * p[a];
    }
    m->n = n;
    for (int a = 0; a < 3; a++) m->u[a] = j[a] / n;
    double e2 = 0, q[3] = {0, 0, 0}, P[3][3] = {{0}};
    for (int v = 0; v < s->nv; v++) {
        double p[3], xi[3];
        vel_of(s, v, p);
        for (int a = 0; a < 3; a++) xi[a] = p[a] - m->u[a];
        double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        e2 += fi[v] * x2;
        for (int a = 0; a < 3; a++) {
            q[a] += 0.5 * fi[v] * x2 * xi[a];
            for (int b = 0; b < 3; b++) P[a][b] += fi[v] * xi[a] * xi[b];
        }
    }
    m->T = e2 / (3 * n);
    for (int a = 0; a < 3; a++) {
        m->q[a] = q[a];
        for (int b = 0; b < 3; b++) m->P[a][b] = P[a][b];
    }
}

/* Fourth-order finite-difference derivative of phi at node i (Sec. III: 4th-order central
 * differences).  Reading: at the two nodes nearest each wall, the one-sided five-point
 * fourth-order stencils (Fornberg weights) are used, mirrored at the outer wall. */
static double fd4(const double* phi, int i, int nr, double dr)
{
    if (i == 0) return (-25 * phi[0] + 48 * phi[1] - 36 * phi[2] + 16 * phi[3] - 3 * phi[4]) / (12 * dr);
    if (i == 1) return (-3 * phi[0] - 10 * phi[1] + 18 * phi[2] - 6 * phi[3] + phi[4]) / (12 * dr);
    if (i == nr - 1)
        return (25 * phi[nr - 1] - 48 * phi[nr - 2] + 36 * phi[nr - 3] - 16 * phi[nr - 4] + 3 * phi[nr - 5]) / (12 * dr);
    if (i == nr - 2)
        return (3 * phi[nr - 1] + 10 * phi[nr - 2] - 18 * phi[nr - 3] + 6 * phi[nr - 4] - phi[nr - 5]) / (12 * dr);
    return (phi[i - 2] - 8 * phi[i - 1] + 8 * phi[i + 1] - phi[i + 2]) / (12 * dr);
}

double orc_fd4(const double* phi, int i, int nr, double dr) { return fd4(phi, i, nr, dr); }

/* WENO-5 (Jiang-Shu) reconstruction at the right face of cell c from the five values
 * (a, b, c, d, e) ordered along the upwind direction; epsilon = 1e-6, power 2. */
static double weno5(double a, double b, double c, double d, double e)
{
    const double eps = 1e-6;
    double q0 = (2 * a - 7 * b + 11 * c) / 6;
    double q1 = (-b + 5 * c + 2 * d) / 6;
    double q2 = (2 * c + 5 * d - e) / 6;
    double b0 = 13.0 / 12 * (a - 2 * b + c) * (a - 2 * b + c) + 0.25 * (a - 4 * b + 3 * c) * (a - 4 * b + 3 * c);
    double b1 = 13.0 / 12 * (b - 2 * c + d) * (b - 2 * c + d) + 0.25 * (b - d) * (b - d);
    double b2 = 13.0 / 12 * (c - 2 * d + e) * (c - 2 * d + e) + 0.25 * (3 * c - 4 * d + e) * (3 * c - 4 * d + e);
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

double orc_weno5(double a, double b, double c, double d, double e) { return weno5(a, b, c, d, e); }

void orc_free(orc_solver* s);

static int validate(const orc_params* p)
{
    if (!p) return ORC_EINVAL;
    if (p->geometry != 0 && p->geometry != 1 && p->geometry != 2) return ORC_EINVAL;
    if (!(p->r_inner > 0) || !(p->r_outer > p->r_inner)) return ORC_EINVAL;
    if (!(p->eta0 > 0 && p->eta0 < 0.5) || !(p->kn > 0)) return ORC_EINVAL;
    if (!(p->t_wall_inner > 0) || !(p->t_wall_outer > 0) || !(p->cfl > 0)) return ORC_EINVAL;
    if (p->nr < 8) return ORC_EINVAL;
    if (p->q_radial < 2 || p->q_t1 < 2 || p->q_t2 < 2) return ORC_EINVAL;
    if (p->q_radial > QMAX || p->q_t1 > QMAX || p->q_t2 > QMAX) return ORC_EINVAL;
    if (p->geometry == 1 && p->u_wall_inner != 0) return ORC_EINVAL;
    if (p->reduced && p->geometry == 1) return ORC_EINVAL;
    if (!isfinite(p->phi_a)) return ORC_EINVAL;
    double C = orc_confinement(p->eta0, p->kn);
    if (!(C > 1)) return ORC_EINVAL;
    int Q[3] = {p->q_radial, p->q_t1, p->q_t2};
    for (int a = 0; a < 3; a++) {
        int N = p->n_expand[a];
        if (N < 0 || N >= Q[a] || N > NMAX) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* Derived quantities and tables of one solve (Sec. IV set-up). */
orc_solver* orc_create(const orc_params* prm_in, int* status)
{
    build_ptables();
    gl10_init();
    orc_params prm = *prm_in;
    if (prm.reduced) { /* two planes (phi, chi) in place of the p_z axis */
        prm.q_t2 = 2;
        prm.n_expand[2] = 1;
    }
    int Q[3] = {prm.q_radial, prm.q_t1, prm.q_t2};
    /* Reading: expansion order N_a = min(7, Q_a - 1) when not given (the paper uses 7). */
    for (int a = 0; a < 3; a++)
        if (prm.n_expand[a] == 0) prm.n_expand[a] = (Q[a] - 1 < 7) ? Q[a] - 1 : 7;
    int st = validate(&prm);
    if (st != ORC_OK) {
        if (status) *status = st;
        return NULL;
    }
    orc_solver* s = calloc(1, sizeof(orc_solver));
    s->prm = prm;
    s->reduced = prm.reduced != 0;
    axis_build(&s->ax[0], 1, Q[0], prm.n_expand[0]);
    axis_build(&s->ax[1], 0, Q[1], prm.n_expand[1]);
    axis_build(&s->ax[2], 0, Q[2], prm.n_expand[2]);
    if (s->reduced) s->ax[2].p[0] = s->ax[2].p[1] = 0; /* no p_z node: the planes carry its moments */
    s->n0 = s->ax[0].nq;
    s->n1 = s->ax[1].nq;
    s->n2 = s->ax[2].nq;
    s->nv = s->n0 * s->n1 * s->n2;
    s->nr = prm.nr;
    const int nr = s->nr, nv = s->nv;

    /* Sec. II Kn map and Sec. IV geometry: sigma = L/C, computational walls at
     * R_L + sigma/2 and R_R - sigma/2.  Reading: uniform cell-centred grid. */
    s->chi0 = orc_chi(prm.eta0);
    s->C = orc_confinement(prm.eta0, prm.kn);
    s->L = prm.r_outer - prm.r_inner;
    s->sigma = s->L / s->C;
    s->rcl = prm.r_inner + s->sigma / 2;
    s->rcr = prm.r_outer - s->sigma / 2;
    s->dr = (s->rcr - s->rcl) / nr;
    s->r = malloc(sizeof(double) * nr);
    s->ri = malloc(sizeof(double) * (nr + 1));
    s->vol = malloc(sizeof(double) * nr);
    for (int i = 0; i <= nr; i++) s->ri[i] = s->rcl + i * s->dr;
    for (int i = 0; i < nr; i++) {
        s->r[i] = s->rcl + (i + 0.5) * s->dr;
        if (prm.geometry == 2)
            s->vol[i] = s->dr; /* planar: per unit wall area */
        else if (prm.geometry == 0)
            s->vol[i] = s->r[i] * s->dr;
        else
            s->vol[i] = (s->ri[i + 1] * s->ri[i + 1] * s->ri[i + 1] - s->ri[i] * s->ri[i] * s->ri[i]) / 3;
    }
    double pmax = 0;
    for (int k = 0; k < s->n0; k++)
        if (fabs(s->ax[0].p[k]) > pmax) pmax = fabs(s->ax[0].p[k]);
    s->dt = prm.cfl * s->dr / pmax;

    /* Force matrices (Sec. III.B): d f/dp along the radial (half-range) axis and
     * d(f p)/dp along the transverse (full-range) axes. */
    s->K1 = malloc(sizeof(double) * s->n0 * s->n0);
    s->K2a = malloc(sizeof(double) * s->n1 * s->n1);
    s->K2b = malloc(sizeof(double) * s->n2 * s->n2);
    orc_kmat_half(Q[0], 1, s->K1);
    orc_kmat_full(Q[1], 2, s->K2a);
    orc_kmat_full(Q[2], 2, s->K2b);

    /* Averaged-density weights, eq. (fm): nbar_i = sum_j W_ij n_j with
     * W_ij = [V(sigma; ri_{j+1}, r_i) - V(sigma; ri_j, r_i)] / (4 pi sigma^3 / 3).
     * Reading: n is piecewise constant on cells and vanishes outside the computational
     * domain (no particle centre can lie there). */
    s->W = malloc(sizeof(double) * nr * nr);
    {
        const double ball = 4.0 / 3 * PI * s->sigma * s->sigma * s->sigma;
        double* Vtab = malloc(sizeof(double) * nr * (nr + 1));
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < nr; i++)
            for (int j = 0; j <= nr; j++)
                Vtab[i * (nr + 1) + j] = (prm.geometry == 0)   ? orc_vol_cyl(s->sigma, s->ri[j], s->r[i])
                                         : (prm.geometry == 1) ? orc_vol_sph(s->sigma, s->ri[j], s->r[i])
                                                               : orc_vol_slab(s->sigma, s->ri[j], s->r[i]);
        for (int i = 0; i < nr; i++)
            for (int j = 0; j < nr; j++)
                s->W[i * nr + j] = (Vtab[i * (nr + 1) + j + 1] - Vtab[i * (nr + 1) + j]) / ball;
        free(Vtab);
    }

    /* Mean-field weights (section 6b): A_ij = n0 [U(r_i; ri_{j+1}) - U(r_i; ri_j)],
     * n0 = 6 eta0 / (pi sigma^3). */
    s->Amf = NULL;
    if (prm.phi_a != 0) {
        const double n0 = 6 * prm.eta0 / (PI * s->sigma * s->sigma * s->sigma);
        double* Utab = malloc(sizeof(double) * nr * (nr + 1));
#pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < nr; i++)
            for (int j = 0; j <= nr; j++)
                Utab[i * (nr + 1) + j] = orc_mf_potential(prm.geometry, s->sigma, prm.phi_a, s->r[i], s->ri[j]);
        s->Amf = malloc(sizeof(double) * nr * nr);
        for (int i = 0; i < nr; i++)
            for (int j = 0; j < nr; j++)
                s->Amf[i * nr + j] = n0 * (Utab[i * (nr + 1) + j + 1] - Utab[i * (nr + 1) + j]);
        free(Utab);
    }

    /* Unit wall Maxwellians (diffuse reflection, Sec. IV): g_R(0,T_w) g_1(u_w,T_w) g_2(0,T_w). */
    s->gwl = malloc(sizeof(double) * nv);
    s->gwr = malloc(sizeof(double) * nv);
    {
        double g0[2 * QMAX], g1[QMAX], g2[QMAX];
        for (int side = 0; side < 2; side++) {
            double Tw = side == 0 ? prm.t_wall_inner : prm.t_wall_outer;
            double uw = side == 0 ? prm.u_wall_inner : 0;
            geq_axis(&s->ax[0], 0, Tw, g0);
            geq_axis(&s->ax[1], uw, Tw, g1);
            zfactors(s, 0, Tw, g2);
            double* gw = side == 0 ? s->gwl : s->gwr;
            double gin = 0;
            for (int v = 0; v < nv; v++) {
                int i0 = v % s->n0, i1 = (v / s->n0) % s->n1, i2 = v / (s->n0 * s->n1);
                gw[v] = g0[i0] * g1[i1] * g2[i2];
                double pr = s->ax[0].p[i0];
                /* the mass flux of the reduced model is that of phi alone */
                if (is_chi(s, v)) continue;
                if ((side == 0 && pr > 0) || (side == 1 && pr < 0)) gin += pr * gw[v];
            }
            if (side == 0)
                s->gin_l = gin;
            else
                s->gin_r = gin;
        }
    }

    s->f = malloc(sizeof(double) * nr * nv);
    s->fs1 = malloc(sizeof(double) * nr * nv);
    s->fs2 = malloc(sizeof(double) * nr * nv);
    s->Lbuf = malloc(sizeof(double) * nr * nv);
    s->mom_prev = calloc(5 * nr, sizeof(double));

    /* Rest start: n = 1, u = 0, T = 1 everywhere (uniform Maxwellian). */
    {
        double g0[2 * QMAX], g1[QMAX], g2[QMAX];
        geq_axis(&s->ax[0], 0, 1, g0);
        geq_axis(&s->ax[1], 0, 1, g1);
        zfactors(s, 0, 1, g2);
        for (int i = 0; i < nr; i++)
            for (int v = 0; v < nv; v++) {
                int i0 = v % s->n0, i1 = (v / s->n0) % s->n1, i2 = v / (s->n0 * s->n1);
                s->f[(size_t)i * nv + v] = g0[i0] * g1[i1] * g2[i2];
            }
    }
    s->last_resid = -1;
    if (status) *status = ORC_OK;
    return s;
}

void orc_free(orc_solver* s)
{
    if (!s) return;
    for (int a = 0; a < 3; a++) axis_free(&s->ax[a]);
    free(s->r);
    free(s->ri);
    free(s->vol);
    free(s->W);
    free(s->Amf);
    free(s->K1);
    free(s->K2a);
    free(s->K2b);
    free(s->gwl);
    free(s->gwr);
    free(s->f);
    free(s->fs1);
    free(s->fs2);
    free(s->Lbuf);
    free(s->mom_prev);
    free(s);
}

/* Right-hand side L(f) of df/dt = L(f) for the reduced equations of Sec. II.B / II.C:
 *   L = - (advection) - (inertial force terms) + J_0 + J_1.
 * Also returns the node blocks (may be NULL). */
static void compute_rhs_terms(orc_solver* s, const double* f, double* Lout, node_t* nodes_out, double* tA, double* tI,
                              double* tJ0, double* tJ1)
{
    const int nr = s->nr, nv = s->nv, n0 = s->n0, n1 = s->n1, n2 = s->n2;
    const orc_params* P = &s->prm;
    const int sph = P->geometry == 1;
    const int planar = P->geometry == 2; /* Cartesian model equation: no vielbein force terms */
    node_t* nd = malloc(sizeof(node_t) * nr);

    /* (1) moments at every node. */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) node_moments(s, f + (size_t)i * nv, &nd[i]);

    /* (2) averaged density and contact value, eqs. (chi_ret), (fm), (chi).
     * Reading: chi at a node is chi_SET(eta0 * nbar) at that node. */
    for (int i = 0; i < nr; i++) {
        double acc = 0;
        for (int j = 0; j < nr; j++) acc += s->W[i * nr + j] * nd[j].n;
        nd[i].nbar = acc;
        nd[i].chi = orc_chi(P->eta0 * acc);
    }

    /* (2b) attractive mean field (section 6b): Phi_i = sum_j A_ij n_j, and the radial force
     * F_i = -dPhi/dr by the same fourth-order stencil as every other radial gradient. */
    {
        double* phi = malloc(sizeof(double) * nr);
        for (int i = 0; i < nr; i++) {
            double acc = 0;
            if (s->Amf)
                for (int j = 0; j < nr; j++) acc += s->Amf[i * nr + j] * nd[j].n;
            phi[i] = acc;
        }
        for (int i = 0; i < nr; i++) {
            nd[i].phi = phi[i];
            nd[i].F = s->Amf ? -fd4(phi, i, nr, s->dr) : 0;
        }
        free(phi);
    }

    /* (3) local coefficients.  Reading: b rho, tau and Pr use the local n with chi(nbar). */
    for (int i = 0; i < nr; i++) {
        double brho = 4 * P->eta0 * nd[i].n;
        nd[i].brhochi = brho * nd[i].chi;
        nd[i].tau = orc_tau(s->chi0, P->kn, s->L, nd[i].n, nd[i].T, nd[i].chi, brho);
        nd[i].Pr = orc_prandtl(nd[i].brhochi);
    }

    /* (4) radial gradients of ln(n^2 chi T), ln T and the velocity components. */
    double *g1 = malloc(sizeof(double) * nr), *g2 = malloc(sizeof(double) * nr);
    double *ua = malloc(sizeof(double) * nr * 3);
    for (int i = 0; i < nr; i++) {
        g1[i] = log(nd[i].n * nd[i].n * nd[i].chi * nd[i].T);
        g2[i] = log(nd[i].T);
        for (int a = 0; a < 3; a++) ua[a * nr + i] = nd[i].u[a];
    }
    double *dg1 = malloc(sizeof(double) * nr), *dg2 = malloc(sizeof(double) * nr), *du = malloc(sizeof(double) * nr * 3);
    for (int i = 0; i < nr; i++) {
        dg1[i] = fd4(g1, i, nr, s->dr);
        dg2[i] = fd4(g2, i, nr, s->dr);
        for (int a = 0; a < 3; a++) du[a * nr + i] = fd4(ua + a * nr, i, nr, s->dr);
        nd[i].dlog_nnchiT = dg1[i];
        nd[i].dlogT = dg2[i];
        for (int a = 0; a < 3; a++) nd[i].du[a] = du[a * nr + i];
    }

    /* (5) wall densities.  Reading (diffuse reflection): two ghost cells per side; for
     * velocities leaving the domain through a wall the ghosts are quadratic
     * extrapolations of the three nearest cells, for velocities entering they are
     * n_w times the unit wall Maxwellian; the wall flux of entering velocities is exactly
     * p_R n_w g_w, and n_w makes the net mass flux through the wall zero. */
    double nwl, nwr;
    {
        double outl = 0, outr = 0;
        for (int v = 0; v < nv; v++) {
            double pr = s->ax[0].p[v % n0];
            if (is_chi(s, v)) continue; /* zero net mass flux: phi alone carries mass */
            if (pr < 0) {
                double f0 = f[0 * (size_t)nv + v], f1 = f[1 * (size_t)nv + v], f2 = f[2 * (size_t)nv + v];
                double gm1 = 3 * f0 - 3 * f1 + f2, gm2 = 6 * f0 - 8 * f1 + 3 * f2;
                outl += pr * weno5(f2, f1, f0, gm1, gm2);
            } else {
                const double* fa = f + (size_t)(nr - 1) * nv;
                const double* fb = f + (size_t)(nr - 2) * nv;
                const double* fc = f + (size_t)(nr - 3) * nv;
                double gp1 = 3 * fa[v] - 3 * fb[v] + fc[v], gp2 = 6 * fa[v] - 8 * fb[v] + 3 * fc[v];
                outr += pr * weno5(fc[v], fb[v], fa[v], gp1, gp2);
            }
        }
        nwl = -outl / s->gin_l;
        nwr = -outr / s->gin_r;
    }

    /* (6) interface fluxes F[k][v] = p_R f_hat, k = 0..nr. */
    double* F = malloc(sizeof(double) * (size_t)(nr + 1) * nv);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; v++) {
        double pr = s->ax[0].p[v % n0];
        /* ghost-extended column e[c + 2], c = -2 .. nr+1 */
        double* e = malloc(sizeof(double) * (nr + 4));
        for (int c = 0; c < nr; c++) e[c + 2] = f[(size_t)c * nv + v];
        if (pr > 0) { /* entering at the inner wall, leaving at the outer wall */
            e[1] = e[0] = nwl * s->gwl[v];
            e[nr + 2] = 3 * e[nr + 1] - 3 * e[nr] + e[nr - 1];
            e[nr + 3] = 6 * e[nr + 1] - 8 * e[nr] + 3 * e[nr - 1];
        } else {
            e[1] = 3 * e[2] - 3 * e[3] + e[4];
            e[0] = 6 * e[2] - 8 * e[3] + 3 * e[4];
            e[nr + 2] = e[nr + 3] = nwr * s->gwr[v];
        }
        for (int k = 0; k <= nr; k++) {
            double fh;
            if (pr > 0) {
                if (k == 0) {
                    F[(size_t)k * nv + v] = pr * nwl * s->gwl[v];
                    continue;
                }
                /* right face of cell k-1, upwind from the left: cells k-3 .. k+1 */
                fh = weno5(e[k - 3 + 2], e[k - 2 + 2], e[k - 1 + 2], e[k + 2], e[k + 1 + 2]);
            } else {
                if (k == nr) {
                    F[(size_t)k * nv + v] = pr * nwr * s->gwr[v];
                    continue;
                }
                /* left face of cell k, upwind from the right: cells k+2 .. k-2 */
                fh = weno5(e[k + 2 + 2], e[k + 1 + 2], e[k + 2], e[k - 1 + 2], e[k - 2 + 2]);
            }
            F[(size_t)k * nv + v] = pr * fh;
        }
        free(e);
    }

    /* (7) assemble L at every node and velocity. */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        const node_t* m = &nd[i];
        const double* fi = f + (size_t)i * nv;
        double gR[2 * QMAX], gA[QMAX], gB[QMAX];
        geq_axis(&s->ax[0], m->u[0], m->T, gR);
        geq_axis(&s->ax[1], m->u[1], m->T, gA);
        zfactors(s, m->u[2], m->T, gB);
        double rl = s->ri[i], rr = s->ri[i + 1];
        /* Reading (flux form of d(fR)/dR^2 and d(fr^2)/dr^3): finite volume with exact
         * shell measures; geometric factor of the force terms 1/r_i (cylinder) and
         * G_i = 3 (rr^2 - rl^2) / (2 (rr^3 - rl^3)) (sphere). */
        double adv_fac, force_fac;
        if (planar) {
            adv_fac = 1 / s->dr;
            force_fac = 0;
        } else if (!sph) {
            adv_fac = 1 / (s->r[i] * s->dr);
            force_fac = 1 / s->r[i];
        } else {
            adv_fac = 3 / (rr * rr * rr - rl * rl * rl);
            force_fac = 3 * (rr * rr - rl * rl) / (2 * (rr * rr * rr - rl * rl * rl));
        }
        double shak = (1 - m->Pr) / (m->n * m->T * m->T);
        double divu, dur = du[0 * nr + i];
        if (planar)
            divu = dur;
        else if (!sph)
            divu = dur + m->u[0] / s->r[i];
        else
            divu = dur + 2 * m->u[0] / s->r[i];
        double s2T = sqrt(2 * m->T);
        for (int v = 0; v < nv; v++) {
            int i0 = v % n0, i1 = (v / n0) % n1, i2 = v / (n0 * n1);
            double p[3] = {s->ax[0].p[i0], s->ax[1].p[i1], s->ax[2].p[i2]};
            /* advection */
            double A;
            if (planar)
                A = (F[(size_t)(i + 1) * nv + v] - F[(size_t)i * nv + v]) * adv_fac;
            else if (!sph)
                A = (rr * F[(size_t)(i + 1) * nv + v] - rl * F[(size_t)i * nv + v]) * adv_fac;
            else
                A = (rr * rr * F[(size_t)(i + 1) * nv + v] - rl * rl * F[(size_t)i * nv + v]) * adv_fac;
            /* inertial terms: (1/R)[p_phi^2 (df/dp_R) - p_R d(f p_phi)/dp_phi] (cylinder),
             * G[(p_th^2 + p_ph^2) df/dp_r - p_r (d(f p_th)/dp_th + d(f p_ph)/dp_ph)] (sphere),
             * plus the mean-field force term F df/dp_r (section 6b) in every geometry. */
            double d0 = 0;
            for (int k = 0; k < n0; k++) d0 += s->K1[i0 * n0 + k] * fi[k + n0 * (i1 + n1 * i2)];
            double d1 = 0;
            for (int k = 0; k < n1; k++) d1 += s->K2a[i1 * n1 + k] * fi[i0 + n0 * (k + n1 * i2)];
            double I;
            if (planar) {
                I = 0;
                if (s->Amf) I = m->F * d0;
            } else if (!sph) {
                I = force_fac * (p[1] * p[1] * d0 - p[0] * d1);
            } else {
                double d2 = 0;
                for (int k = 0; k < n2; k++) d2 += s->K2b[i2 * n2 + k] * fi[i0 + n0 * (i1 + n1 * k)];
                I = force_fac * ((p[1] * p[1] + p[2] * p[2]) * d0 - p[0] * (d1 + d2));
            }
            if (s->Amf && !planar) I += m->F * d0;
            /* collision: Shakhov J0 (eq. (j0), sign as in eq. (enskog_approx)) and J1[f^MB]
             * (eq. (j1)) on the discrete equilibrium f^MB = n g_R g_1 g_2. */
            double fmb = m->n * gR[i0] * gA[i1] * gB[i2];
            double xi[3] = {p[0] - m->u[0], p[1] - m->u[1], p[2] - m->u[2]};
            double xi2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
            /* reduced distributions: the collision polynomials are linear in xi_z^2, which takes
             * the value T for phi and 3T for chi (whose factor T sits in fmb through gB) */
            if (s->reduced) {
                xi[2] = 0;
                xi2 = xi[0] * xi[0] + xi[1] * xi[1] + (i2 == 0 ? m->T : 3 * m->T);
            }
            double xq = xi[0] * m->q[0] + xi[1] * m->q[1] + xi[2] * m->q[2];
            double fS = fmb * (1 + shak * (xi2 / (5 * m->T) - 1) * xq);
            double zeta[3] = {xi[0] / s2T, xi[1] / s2T, xi[2] / s2T};
            double z2 = zeta[0] * zeta[0] + zeta[1] * zeta[1] + zeta[2] * zeta[2];
            if (s->reduced) z2 = xi2 / (2 * m->T); /* with xi_z^2 as above */
            /* Reading: zeta zeta : grad u in the covariant (orthonormal-frame) form. */
            double zzgu;
            if (planar)
                zzgu = zeta[0] * zeta[0] * dur + zeta[0] * zeta[1] * du[1 * nr + i] + zeta[0] * zeta[2] * du[2 * nr + i];
            else if (!sph)
                zzgu = zeta[0] * zeta[0] * dur + zeta[0] * zeta[1] * (du[1 * nr + i] - m->u[1] / s->r[i]) +
                       zeta[1] * zeta[1] * m->u[0] / s->r[i] + zeta[0] * zeta[2] * du[2 * nr + i];
            else
                zzgu = zeta[0] * zeta[0] * dur + (zeta[1] * zeta[1] + zeta[2] * zeta[2]) * m->u[0] / s->r[i];
            double S = xi[0] * (dg1[i] + 0.6 * (z2 - 2.5) * dg2[i]) + 0.4 * (2 * zzgu + (z2 - 2.5) * divu);
            double J1 = -m->brhochi * fmb * S;
            double J0 = -(fi[v] - fS) / m->tau;
            Lout[(size_t)i * nv + v] = -A - I + J0 + J1;
            if (tA) {
                tA[(size_t)i * nv + v] = A;
                tI[(size_t)i * nv + v] = I;
                tJ0[(size_t)i * nv + v] = J0;
                tJ1[(size_t)i * nv + v] = J1;
            }
        }
    }
    if (nodes_out) memcpy(nodes_out, nd, sizeof(node_t) * nr);
    free(F);
    free(g1);
    free(g2);
    free(ua);
    free(dg1);
    free(dg2);
    free(du);
    free(nd);
}

static void compute_rhs(orc_solver* s, const double* f, double* Lout, node_t* nodes_out)
{
    compute_rhs_terms(s, f, Lout, nodes_out, NULL, NULL, NULL, NULL);
}

static void snapshot_moments(orc_solver* s, const double* f, double* out5)
{
    const int nr = s->nr;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; i++) {
        node_t m;
        node_moments(s, f + (size_t)i * s->nv, &m);
        out5[0 * nr + i] = m.n;
        out5[1 * nr + i] = m.u[0];
        out5[2 * nr + i] = m.u[1];
        out5[3 * nr + i] = m.u[2];
        out5[4 * nr + i] = m.T;
    }
}

/* One TVD RK3 step (Shu-Osher form, Sec. III):
 *   f1 = f + dt L(f);  f2 = 3/4 f + 1/4 (f1 + dt L(f1));  f' = 1/3 f + 2/3 (f2 + dt L(f2)). */
static void rk3_step(orc_solver* s)
{
    const size_t tot = (size_t)s->nr * s->nv;
    const double dt = s->dt;
    compute_rhs(s, s->f, s->Lbuf, NULL);
    for (size_t k = 0; k < tot; k++) s->fs1[k] = s->f[k] + dt * s->Lbuf[k];
    compute_rhs(s, s->fs1, s->Lbuf, NULL);
    for (size_t k = 0; k < tot; k++) s->fs2[k] = 0.75 * s->f[k] + 0.25 * (s->fs1[k] + dt * s->Lbuf[k]);
    compute_rhs(s, s->fs2, s->Lbuf, NULL);
    for (size_t k = 0; k < tot; k++) s->f[k] = s->f[k] / 3 + 2.0 / 3 * (s->fs2[k] + dt * s->Lbuf[k]);
    s->steps++;
}

/* Steady-state residual (the paper does not define one).  Reading: the largest change over
 * one full step of n, u_R, u_1, u_2 and T at any node, divided by dt (a rate). */
static double residual_over_step(orc_solver* s)
{
    const int nr = s->nr;
    double* now = malloc(sizeof(double) * 5 * nr);
    snapshot_moments(s, s->f, now);
    double r = 0;
    for (int k = 0; k < 5 * nr; k++) {
        double d = fabs(now[k] - s->mom_prev[k]);
        if (d > r || d != d) r = d;
    }
    free(now);
    return r / s->dt;
}

static int check_finite(const orc_solver* s)
{
    const size_t tot = (size_t)s->nr * s->nv;
    for (size_t k = 0; k < tot; k++)
        if (!isfinite(s->f[k])) return 0;
    return 1;
}

int orc_step(orc_solver* s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; k++) {
        if (k == nsteps - 1) snapshot_moments(s, s->f, s->mom_prev);
        rk3_step(s);
    }
    if (nsteps > 0) s->last_resid = residual_over_step(s);
    if (!check_finite(s)) {
        s->nan_flag = 1;
        return ORC_ENAN;
    }
    return ORC_OK;
}

/* Run until the one-step residual, evaluated after every check_every-th step, is <= tol.
 * Returns 0 on convergence, 1 if max_steps was reached first. */
int orc_run_to_steady(orc_solver* s, double tol, int64_t max_steps, int32_t check_every, int64_t* steps_out,
                      double* resid_out)
{
    if (check_every < 1 || max_steps < 1) return ORC_EINVAL;
    int64_t done = 0;
    double r = -1;
    int conv = 0;
    while (done < max_steps) {
        int64_t chunk = check_every;
        if (chunk > max_steps - done) chunk = max_steps - done;
        for (int64_t k = 0; k < chunk; k++) {
            if (k == chunk - 1) snapshot_moments(s, s->f, s->mom_prev);
            rk3_step(s);
        }
        done += chunk;
        if (!check_finite(s)) {
            s->nan_flag = 1;
            if (steps_out) *steps_out = done;
            if (resid_out) *resid_out = NAN;
            return ORC_ENAN;
        }
        if (chunk == check_every) {
            r = residual_over_step(s);
            s->last_resid = r;
            if (r <= tol) {
                conv = 1;
                break;
            }
        }
    }
    if (steps_out) *steps_out = done;
    if (resid_out) *resid_out = r;
    return conv ? 0 : 1;
}

/* Output block [field][nr]: n, u_r, u_t1, u_t2, T, q_r, P_{r t1}, nbar, chi. */
int orc_moments(orc_solver* s, double* out)
{
    const int nr = s->nr;
    node_t* nd = malloc(sizeof(node_t) * nr);
    compute_rhs(s, s->f, s->Lbuf, nd);
    for (int i = 0; i < nr; i++) {
        out[0 * nr + i] = nd[i].n;
        out[1 * nr + i] = nd[i].u[0];
        out[2 * nr + i] = nd[i].u[1];
        out[3 * nr + i] = nd[i].u[2];
        out[4 * nr + i] = nd[i].T;
        out[5 * nr + i] = nd[i].q[0];
        out[6 * nr + i] = nd[i].P[0][1];
        out[7 * nr + i] = nd[i].nbar;
        out[8 * nr + i] = nd[i].chi;
    }
    free(nd);
    return ORC_OK;
}

/* Node coefficients [field][nr]: tau, Pr, b rho chi, q_1, q_2 (for pins). */
int orc_node_coeffs(orc_solver* s, double* out)
{
    const int nr = s->nr;
    node_t* nd = malloc(sizeof(node_t) * nr);
    compute_rhs(s, s->f, s->Lbuf, nd);
    for (int i = 0; i < nr; i++) {
        out[0 * nr + i] = nd[i].tau;
        out[1 * nr + i] = nd[i].Pr;
        out[2 * nr + i] = nd[i].brhochi;
        out[3 * nr + i] = nd[i].q[1];
        out[4 * nr + i] = nd[i].q[2];
    }
    free(nd);
    return ORC_OK;
}

/* Radial gradients [field][nr] entering J1 (for pins): d ln(n^2 chi T), d ln T, du_r, du_t1, du_t2. */
int orc_node_grads(orc_solver* s, double* out)
{
    const int nr = s->nr;
    node_t* nd = malloc(sizeof(node_t) * nr);
    compute_rhs(s, s->f, s->Lbuf, nd);
    for (int i = 0; i < nr; i++) {
        out[0 * nr + i] = nd[i].dlog_nnchiT;
        out[1 * nr + i] = nd[i].dlogT;
        for (int a = 0; a < 3; a++) out[(2 + a) * nr + i] = nd[i].du[a];
    }
    free(nd);
    return ORC_OK;
}

int orc_rhs(orc_solver* s, double* out)
{
    compute_rhs(s, s->f, out, NULL);
    return ORC_OK;
}

/* The four parts of L(f) = -A - I + J0 + J1 separately (advection, inertial force terms,
 * Shakhov relaxation, first-order Enskog correction), each nr x nv. */
int orc_rhs_terms(orc_solver* s, double* A, double* I, double* J0, double* J1)
{
    compute_rhs_terms(s, s->f, s->Lbuf, NULL, A, I, J0, J1);
    return ORC_OK;
}

int orc_get_f(orc_solver* s, double* out)
{
    memcpy(out, s->f, sizeof(double) * (size_t)s->nr * s->nv);
    return ORC_OK;
}

int orc_set_f(orc_solver* s, const double* in)
{
    memcpy(s->f, in, sizeof(double) * (size_t)s->nr * s->nv);
    s->nan_flag = 0;
    return ORC_OK;
}

int orc_get_W(orc_solver* s, double* out)
{
    memcpy(out, s->W, sizeof(double) * (size_t)s->nr * s->nr);
    return ORC_OK;
}

/* Mean-field weights A (nr x nr; zeros without attraction). */
int orc_get_attraction(orc_solver* s, double* out)
{
    if (s->Amf)
        memcpy(out, s->Amf, sizeof(double) * (size_t)s->nr * s->nr);
    else
        memset(out, 0, sizeof(double) * (size_t)s->nr * s->nr);
    return ORC_OK;
}

/* Mean-field potential Phi [nr] and radial force F [nr] of the current state. */
int orc_mean_field(orc_solver* s, double* phi, double* F)
{
    const int nr = s->nr;
    node_t* nd = malloc(sizeof(node_t) * nr);
    compute_rhs(s, s->f, s->Lbuf, nd);
    for (int i = 0; i < nr; i++) {
        phi[i] = nd[i].phi;
        F[i] = nd[i].F;
    }
    free(nd);
    return ORC_OK;
}

/* Scalars: [nr, nv, n0, n1, n2, chi0, C, L, sigma, rcl, rcr, dr, dt, steps, last_resid,
 *           N0, N1, N2] */
int orc_info(orc_solver* s, double* out)
{
    out[0] = s->nr;
    out[1] = s->nv;
    out[2] = s->n0;
    out[3] = s->n1;
    out[4] = s->n2;
    out[5] = s->chi0;
    out[6] = s->C;
    out[7] = s->L;
    out[8] = s->sigma;
    out[9] = s->rcl;
    out[10] = s->rcr;
    out[11] = s->dr;
    out[12] = s->dt;
    out[13] = (double)s->steps;
    out[14] = s->last_resid;
    out[15] = s->ax[0].N;
    out[16] = s->ax[1].N;
    out[17] = s->ax[2].N;
    return ORC_OK;
}

/* Per-axis nodes [n0 + n1 + n2], node radii [nr], interface radii [nr+1], cell measures [nr]. */
int orc_grid(orc_solver* s, double* pnodes, double* r, double* ri, double* vol)
{
    if (pnodes) {
        memcpy(pnodes, s->ax[0].p, sizeof(double) * s->n0);
        memcpy(pnodes + s->n0, s->ax[1].p, sizeof(double) * s->n1);
        memcpy(pnodes + s->n0 + s->n1, s->ax[2].p, sizeof(double) * s->n2);
    }
    if (r) memcpy(r, s->r, sizeof(double) * s->nr);
    if (ri) memcpy(ri, s->ri, sizeof(double) * (s->nr + 1));
    if (vol) memcpy(vol, s->vol, sizeof(double) * s->nr);
    return ORC_OK;
}

/* Total mass sum_i V_i n_i (per unit axial length / per unit solid angle). */
double orc_mass(orc_solver* s)
{
    double m = 0;
    for (int i = 0; i < s->nr; i++) {
        double n = 0;
        for (int v = 0; v < s->nv; v++)
            if (!is_chi(s, v)) n += s->f[(size_t)i * s->nv + v];
        m += s->vol[i] * n;
    }
    return m;
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

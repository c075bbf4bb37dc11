// Host precompute of liblbe: quadratures, force matrices, averaged-density weights, wall
// Maxwellians and the derived scalars of one instance (arXiv:2403.15051, Secs. II-IV,
// Appendix A).  Everything here runs once per lbe_init, in long double where accuracy
// matters, and is uploaded to the device.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "lbe_equilibrium.h"
#include "lbe_internal.h"

namespace lbe {

typedef long double ld;
static const ld kPi = 3.141592653589793238462643383279502884L;

// ------------------------------------------------------------------ closed forms (Sec. II)

// Carnahan-Starling contact value, eq. (chi).
double chi_cs(double eta) { return (2 - eta) / (2 * (1 - eta) * (1 - eta) * (1 - eta)); }

// ------------------------------------------------------------------ quadratures (Sec. III)

// Eigenvalues of the symmetric tridiagonal matrix with diagonal d[0..n-1] and off-diagonal e[1..n-1]
// (e[i] couples rows i-1 and i), in increasing order, by bisection on Sturm counts: the number of
// eigenvalues below x equals the number of negative pivots in the LDL^T factorisation of T - x I
// (Sylvester's law of inertia).  Each eigenvalue is bracketed to a few units in the last place of
// long double; the callers polish the zeros by Newton's method on the polynomial.
static int pivots_below(const std::vector<ld>& d, const std::vector<ld>& e, ld x)
{
    int neg = 0;
    ld piv = 1;
    for (size_t i = 0; i < d.size(); i++) {
        piv = (d[i] - x) - (i > 0 ? e[i] * e[i] / piv : 0);
        if (piv == 0) piv = -LDBL_EPSILON * (fabsl(d[i]) + fabsl(x) + (i > 0 ? fabsl(e[i]) : 0) + LDBL_MIN);
        if (piv < 0) neg++;
    }
    return neg;
}

static void tridiag_eigenvalues(const std::vector<ld>& d, const std::vector<ld>& e, std::vector<ld>& ev)
{
    const int n = (int)d.size();
    ld lo = 0, hi = 0;  // Gershgorin bounds
    for (int i = 0; i < n; i++) {
        const ld r = (i > 0 ? fabsl(e[i]) : 0) + (i + 1 < n ? fabsl(e[i + 1]) : 0);
        lo = i ? std::min(lo, d[i] - r) : d[i] - r;
        hi = i ? std::max(hi, d[i] + r) : d[i] + r;
    }
    ev.assign(n, 0);
    for (int k = 0; k < n; k++) {
        // the k-th eigenvalue lies where the count of eigenvalues below x steps from k to k + 1
        ld a = k > 0 ? ev[k - 1] : lo, b = hi;
        for (int it = 0; it < 256; it++) {
            const ld mid = a + (b - a) / 2;
            if (mid <= a || mid >= b) break;
            if (pivots_below(d, e, mid) > k)
                b = mid;
            else
                a = mid;
        }
        ev[k] = a + (b - a) / 2;
    }
}

// Gauss-Legendre rule on [-1, 1] in long double: the nodes are the eigenvalues of the Legendre
// Jacobi matrix (zero diagonal, off-diagonal l / sqrt(4 l^2 - 1)), polished by Newton's method
// on the orthonormal P_n; the weights are the Christoffel numbers 1 / sum_{l<n} p_l(x)^2 of the
// orthonormal Legendre polynomials p_l = sqrt(l + 1/2) P_l.
static void legendre_orthonormal(int n, ld x, ld* p, ld* dp)
{
    // p_{l+1} = (x p_l - beta_l p_{l-1}) / beta_{l+1}, beta_l = l / sqrt(4 l^2 - 1), p_0 = 1/sqrt 2
    p[0] = 1 / sqrtl(2.0L);
    dp[0] = 0;
    ld bprev = 0;
    for (int l = 0; l < n; l++) {
        const ld bnext = (l + 1) / sqrtl((ld)(4 * (l + 1) * (l + 1) - 1));
        const ld pm = l > 0 ? p[l - 1] : 0, dpm = l > 0 ? dp[l - 1] : 0;
        p[l + 1] = (x * p[l] - bprev * pm) / bnext;
        dp[l + 1] = (p[l] + x * dp[l] - bprev * dpm) / bnext;
        bprev = bnext;
    }
}

static void gauss_legendre(int n, std::vector<ld>& x, std::vector<ld>& w)
{
    std::vector<ld> d(n, 0), e(n, 0);
    for (int l = 1; l < n; l++) e[l] = l / sqrtl((ld)(4 * l * l - 1));
    tridiag_eigenvalues(d, e, x);
    std::vector<ld> p(n + 1), dp(n + 1);
    w.assign(n, 0);
    for (int i = 0; i < n; i++) {
        for (int it = 0; it < 2; it++) {
            legendre_orthonormal(n, x[i], p.data(), dp.data());
            x[i] -= p[n] / dp[n];
        }
        legendre_orthonormal(n, x[i], p.data(), dp.data());
        ld s = 0;
        for (int l = 0; l < n; l++) s += p[l] * p[l];
        w[i] = 1 / s;
    }
    for (int i = 0; i < n / 2; i++) {  // exact mirror symmetry
        const ld m = (x[n - 1 - i] - x[i]) / 2, wm = (w[i] + w[n - 1 - i]) / 2;
        x[i] = -m;
        x[n - 1 - i] = m;
        w[i] = w[n - 1 - i] = wm;
    }
    if (n % 2) x[n / 2] = 0;
}

// Recurrence x h_l = b_{l+1} h_{l+1} + a_l h_l + b_l h_{l-1} of the polynomials orthonormal on
// [0, inf) with weight exp(-x^2/2)/sqrt(2 pi) (the half-range Hermite polynomials of the
// paper), by the discretised Stieltjes procedure (Gautschi): the measure is replaced by a
// composite 20-point Gauss-Legendre rule on panels of width 1/2, and the polynomial values at its
// nodes are generated as vectors.  Each new vector is orthogonalised again, twice, against all
// earlier ones (in the discrete inner product): without that, rounding in the three-term step
// is amplified with the degree (nodes off by ~5e-12 at order 64 in long double).  Returns
// a[0..n-1], b[0..n] with b[0] = mu_0 = 1/2.
static void half_recurrence(int n, std::vector<ld>& a, std::vector<ld>& b)
{
    std::vector<ld> gx, gw;
    const int P = 20;
    gauss_legendre(P, gx, gw);
    const ld X = sqrtl((ld)(2 * n + 1)) + 15;
    const ld h = std::min(0.5L, 2 / sqrtl((ld)(2 * n + 1)));
    const int npan = (int)ceill(X / h);
    std::vector<ld> y, lam;
    for (int p = 0; p < npan; p++)
        for (int j = 0; j < P; j++) {
            ld t = p * h + h * (gx[j] + 1) / 2;
            y.push_back(t);
            lam.push_back(gw[j] * h / 2 * expl(-t * t / 2) / sqrtl(2 * kPi));
        }
    const size_t M = y.size();
    auto dot = [&](const ld* u, const ld* v) {
        ld s = 0;
        for (size_t m = 0; m < M; m++) s += lam[m] * u[m] * v[m];
        return s;
    };
    // basis[k] = h_k at the nodes
    std::vector<ld> basis((size_t)(n + 1) * M);
    ld mu0 = 0;
    for (size_t m = 0; m < M; m++) mu0 += lam[m];
    for (size_t m = 0; m < M; m++) basis[m] = 1 / sqrtl(mu0);
    a.assign(n, 0);
    b.assign(n + 1, 0);
    b[0] = mu0;
    std::vector<ld> nxt(M);
    for (int k = 0; k < n; k++) {
        const ld* cur = &basis[(size_t)k * M];
        const ld* prev = k > 0 ? &basis[(size_t)(k - 1) * M] : nullptr;
        std::vector<ld> ycur(M);
        for (size_t m = 0; m < M; m++) ycur[m] = y[m] * cur[m];
        const ld ak = dot(ycur.data(), cur);
        a[k] = ak;
        for (size_t m = 0; m < M; m++) nxt[m] = ycur[m] - ak * cur[m] - (k > 0 ? b[k] * prev[m] : 0);
        for (int pass = 0; pass < 2; pass++)
            for (int j = 0; j <= k; j++) {
                const ld* bj = &basis[(size_t)j * M];
                const ld c = dot(nxt.data(), bj);
                for (size_t m = 0; m < M; m++) nxt[m] -= c * bj[m];
            }
        const ld bk = sqrtl(dot(nxt.data(), nxt.data()));
        b[k + 1] = bk;
        ld* out = &basis[(size_t)(k + 1) * M];
        for (size_t m = 0; m < M; m++) out[m] = nxt[m] / bk;
    }
}

// Values of the orthonormal half-range polynomials h_0..h_n at x and their derivatives.
static void half_eval(int n, const std::vector<ld>& a, const std::vector<ld>& b, ld x, ld* h, ld* dh)
{
    h[0] = 1 / sqrtl(b[0]);
    if (dh) dh[0] = 0;
    if (n >= 1) {
        h[1] = (x - a[0]) * h[0] / b[1];
        if (dh) dh[1] = h[0] / b[1];
    }
    for (int l = 1; l < n; l++) {
        h[l + 1] = ((x - a[l]) * h[l] - b[l] * h[l - 1]) / b[l + 1];
        if (dh) dh[l + 1] = ((x - a[l]) * dh[l] + h[l] - b[l] * dh[l - 1]) / b[l + 1];
    }
}

// Half-range Gauss rule of order M for the weight exp(-x^2/2)/sqrt(2 pi) on [0, inf): the zeros of
// h_M (Jacobi-matrix eigenvalues, Newton-polished) and the Christoffel weights 1 / sum_{l<M} h_l^2.
// Built once and shared (the projection kernel's rule for the equilibrium at moderate u/sqrt(T)).
static void half_gauss_rule(int M, std::vector<double>& xo, std::vector<double>& wo)
{
    static std::mutex mu;
    static std::vector<double> cx, cw;
    static int cm = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (cm != M) {
        std::vector<ld> a, b;
        half_recurrence(M + 1, a, b);
        std::vector<ld> d(a.begin(), a.begin() + M), e(M, 0), roots;
        for (int k = 1; k < M; k++) e[k] = b[k];
        tridiag_eigenvalues(d, e, roots);
        std::vector<ld> h(M + 2), dh(M + 2);
        cx.assign(M, 0);
        cw.assign(M, 0);
        for (int i = 0; i < M; i++) {
            ld x = roots[i];
            for (int it = 0; it < 3; it++) {
                half_eval(M, a, b, x, h.data(), dh.data());
                x -= h[M] / dh[M];
            }
            half_eval(M, a, b, x, h.data(), nullptr);
            ld sum = 0;
            for (int l = 0; l < M; l++) sum += h[l] * h[l];
            cx[i] = (double)x;
            cw[i] = (double)(1 / sum);
        }
        cm = M;
    }
    xo = cx;
    wo = cw;
}

// Orthonormal probabilists' Hermite functions psi_l = He_l / sqrt(l!), l = 0..n.
static void herm_eval(int n, ld x, ld* psi)
{
    psi[0] = 1;
    if (n >= 1) psi[1] = x;
    for (int l = 1; l < n; l++) psi[l + 1] = (x * psi[l] - sqrtl((ld)l) * psi[l - 1]) / sqrtl((ld)(l + 1));
}

// Half-range rule of order Q (Golub-Welsch on the Jacobi matrix, Newton-polished zeros,
// Christoffel weights), with the derivative-projection force matrices of eq. (force1)/(force2).
static void build_half_axis(int Q, int N, double Y, double hwidth, AxisTables* ax, std::vector<double>* K1,
                            std::vector<double>* K2)
{
    std::vector<ld> a, b;
    half_recurrence(Q + 1, a, b);
    std::vector<ld> d(a.begin(), a.begin() + Q), e(Q, 0), roots;
    for (int k = 1; k < Q; k++) e[k] = b[k];
    tridiag_eigenvalues(d, e, roots);
    std::vector<ld> h(Q + 2), dh(Q + 2);
    for (int i = 0; i < Q; i++) {  // Newton polish on h_Q
        ld x = roots[i];
        for (int it = 0; it < 3; it++) {
            half_eval(Q, a, b, x, h.data(), dh.data());
            x -= h[Q] / dh[Q];
        }
        roots[i] = x;
    }
    ax->half = true;
    ax->Q = Q;
    ax->nq = 2 * Q;
    ax->N = N;
    ax->p.assign(2 * Q, 0);
    ax->w.assign(2 * Q, 0);
    std::vector<ld> pl(2 * Q), wl(2 * Q);
    for (int i = 0; i < Q; i++) {
        half_eval(Q, a, b, roots[i], h.data(), nullptr);
        ld s = 0;
        for (int l = 0; l < Q; l++) s += h[l] * h[l];
        pl[i] = roots[i];
        pl[Q + i] = -roots[i];
        wl[i] = wl[Q + i] = 1 / s;
    }
    for (int k = 0; k < 2 * Q; k++) {
        ax->p[k] = (double)pl[k];
        ax->w[k] = (double)wl[k];
    }
    ax->poly.assign(2 * Q * (N + 1), 0);
    for (int k = 0; k < 2 * Q; k++) {
        half_eval(Q, a, b, fabsl(pl[k]), h.data(), nullptr);
        for (int l = 0; l <= N; l++) ax->poly[k * (N + 1) + l] = (double)h[l];
    }
    // projection rule of the equilibrium: composite 16-point Gauss-Legendre on [0, Y], panels
    // of width hwidth, with h_l at its nodes
    {
        std::vector<ld> gx, gw;
        gauss_legendre(16, gx, gw);
        const ld hw = hwidth;
        ax->qpanel = hwidth;
        const int npan = (int)ceill(Y / hw);
        ax->qy.clear();
        ax->qlam.clear();
        ax->qh.clear();
        for (int pn = 0; pn < npan; pn++)
            for (int j = 0; j < 16; j++) {
                const ld t = pn * hw + hw * (gx[j] + 1) / 2;
                ax->qy.push_back((double)t);
                ax->qlam.push_back((double)(gw[j] * hw / 2));
                half_eval(std::max(N, 1), a, b, t, h.data(), nullptr);
                for (int l = 0; l <= N; l++) ax->qh.push_back((double)h[l]);
            }
    }
    // the same polynomials in monic form for the device: p_{l+1} = (x - a_l) p_l - b_l^2 p_{l-1},
    // p_0 = 1, h_l = p_l h_0 / (b_1 ... b_l); qrec = (a_l, b_l^2) for l < N, then the N + 1 norms
    ax->qrec.clear();
    for (int l = 0; l < N; l++) {
        ax->qrec.push_back((double)a[l]);
        ax->qrec.push_back((double)(b[l] * b[l]));
    }
    ld nrm = 1 / sqrtl(b[0]);
    for (int l = 0; l <= N; l++) {
        if (l > 0) nrm /= b[l];
        ax->qrec.push_back((double)nrm);
    }
    half_gauss_rule(kProjGauss, ax->gx, ax->gw);
    half_eval(Q, a, b, 0, h.data(), nullptr);
    std::vector<ld> hzero(h.begin(), h.begin() + Q);

    // Force matrices.  The projected derivative on each half-line, with the jump of f at
    // p = 0 shared equally by the two halves, gives
    //   K1_{ii'} = w_i s_i sum_{s<Q} h_s(|p_i|) [ -[s_i = s_i'] h_s'(|p_i'|)
    //              - h_s(0) Phi(|p_i'|) / (2 sqrt(2 pi)) ],  Phi(y) = sum_{l<Q} h_l(0) h_l(y);
    // d(f p)/dp has no jump, so K2_{ii'} = -w_i [s_i = s_i'] sum_{s<Q} h_s(|p_i|) |p_i'| h_s'(|p_i'|).
    // (These are the printed K^h matrices of eqs. (force1)/(force2) rewritten without the
    // monomial coefficients h_{l,s}.)
    const int n = 2 * Q;
    std::vector<ld> H(n * Q), DH(n * Q), PHI(n);
    for (int k = 0; k < n; k++) {
        half_eval(Q, a, b, fabsl(pl[k]), h.data(), dh.data());
        ld phi = 0;
        for (int l = 0; l < Q; l++) {
            H[k * Q + l] = h[l];
            DH[k * Q + l] = dh[l];
            phi += hzero[l] * h[l];
        }
        PHI[k] = phi;
    }
    const ld om0 = 1 / sqrtl(2 * kPi);
    K1->assign(n * n, 0);
    K2->assign(n * n, 0);
    for (int i = 0; i < n; i++) {
        ld si = pl[i] > 0 ? 1 : -1;
        for (int j = 0; j < n; j++) {
            bool same = (pl[i] > 0) == (pl[j] > 0);
            ld acc1 = 0, acc2 = 0;
            for (int s = 0; s < Q; s++) {
                ld t = -0.5L * om0 * hzero[s] * PHI[j];
                if (same) t -= DH[j * Q + s];
                acc1 += H[i * Q + s] * t;
                if (same) acc2 += H[i * Q + s] * fabsl(pl[j]) * DH[j * Q + s];
            }
            (*K1)[i * n + j] = (double)(wl[i] * si * acc1);
            (*K2)[i * n + j] = (double)(-wl[i] * acc2);
        }
    }
}

// Full-range rule of order Q (Golub-Welsch on the Hermite Jacobi matrix) and its force
// matrix for d(f p)/dp, eq. (force2): K1_{ii'} = -w_i sum_l sqrt(l+1) psi_{l+1}(p_i) psi_l(p_i')
// (the printed sum of He_{l+1}(p_i) He_l(p_i') / l!), and K2 = K1 diag(p) because the
// He_Q(p_i) = 0 truncation makes the printed two-term form identical to it.
static void build_full_axis(int Q, int N, AxisTables* ax, std::vector<double>* K2)
{
    std::vector<ld> d(Q, 0), e(Q, 0), roots;
    for (int k = 1; k < Q; k++) e[k] = sqrtl((ld)k);
    tridiag_eigenvalues(d, e, roots);
    std::vector<ld> psi(Q + 2);
    for (int i = 0; i < Q; i++) {
        ld x = roots[i];
        for (int it = 0; it < 3; it++) {
            // He_Q and its derivative Q He_{Q-1} via psi
            herm_eval(Q, x, psi.data());
            ld val = psi[Q], der = sqrtl((ld)Q) * psi[Q - 1];
            x -= val / der;
        }
        roots[i] = x;
    }
    // symmetric rule: enforce exact mirror symmetry of nodes
    for (int i = 0; i < Q / 2; i++) {
        ld m = (roots[Q - 1 - i] - roots[i]) / 2;
        roots[i] = -m;
        roots[Q - 1 - i] = m;
    }
    if (Q % 2) roots[Q / 2] = 0;
    ax->half = false;
    ax->Q = Q;
    ax->nq = Q;
    ax->N = N;
    ax->p.assign(Q, 0);
    ax->w.assign(Q, 0);
    std::vector<ld> wl(Q);
    for (int i = 0; i < Q; i++) {
        herm_eval(Q, roots[i], psi.data());
        ld s = 0;
        for (int l = 0; l < Q; l++) s += psi[l] * psi[l];
        wl[i] = 1 / s;
        ax->p[i] = (double)roots[i];
        ax->w[i] = (double)wl[i];
    }
    ax->poly.assign(Q * (N + 1), 0);
    for (int k = 0; k < Q; k++) {
        // He_l(p_k) = sqrt(l!) psi_l(p_k)
        herm_eval(std::max(N, 1), roots[k], psi.data());
        ld fact = 1;
        for (int l = 0; l <= N; l++) {
            if (l >= 2) fact *= l;
            ax->poly[k * (N + 1) + l] = (double)(sqrtl(fact) * psi[l]);
        }
    }
    K2->assign(Q * Q, 0);
    std::vector<ld> P(Q * (Q + 1));
    for (int k = 0; k < Q; k++) {
        herm_eval(Q, roots[k], psi.data());
        for (int l = 0; l <= Q; l++) P[k * (Q + 1) + l] = psi[l];
    }
    for (int i = 0; i < Q; i++)
        for (int j = 0; j < Q; j++) {
            ld acc = 0;
            for (int l = 0; l <= Q - 2; l++) acc += sqrtl((ld)(l + 1)) * P[i * (Q + 1) + l + 1] * P[j * (Q + 1) + l];
            (*K2)[i * Q + j] = (double)(-wl[i] * acc * roots[j]);
        }
}

// The p_z "axis" of the reduced distributions (cylinder, p_z integrated out): two planes, phi =
// int f dp_z (i2 = 0) and chi = int p_z^2 f dp_z (i2 = 1).  Written as a full-range axis so that the
// equilibrium machinery applies unchanged: nodes p = 0 (no p_z dependence is left), weights 1, and
// the expansion rows [1, 0, 0] and [1, 0, 2] with N = 2, so that with the full-range coefficients
// c_0 = 1, c_2 = (T - 1 + u^2) / 2 at u_z = 0 the factors are int G dp_z = 1 and int p_z^2 G dp_z =
// T.  No force term acts along it (K2 is zero; the cylinder has none along z anyway).
static void build_reduced_axis(AxisTables* ax, std::vector<double>* K2)
{
    ax->half = false;
    ax->Q = 2;
    ax->nq = 2;
    ax->N = 2;
    ax->p.assign(2, 0.0);
    ax->w.assign(2, 1.0);
    ax->poly = {1.0, 0.0, 0.0, 1.0, 0.0, 2.0};
    K2->assign(4, 0.0);
}

// ------------------------------------------------------------------ equilibrium (Sec. III.C)

void equilibrium_axis(const AxisTables& ax, double u, double T, double* g)
{
    const int N = ax.N;
    if (ax.half) {
        double Ip[kMaxN + 2], Im[kMaxN + 2];
        const int M = (int)ax.qy.size();
        half_projection_part(u, T, N, 0, M, ax.qy.data(), ax.qlam.data(), ax.qh.data(), Ip);
        half_projection_part(-u, T, N, 0, M, ax.qy.data(), ax.qlam.data(), ax.qh.data(), Im);
        for (int k = 0; k < ax.nq; k++) {
            const double* I = ax.p[k] > 0 ? Ip : Im;
            double acc = 0;
            for (int l = 0; l <= N; l++) acc += I[l] * ax.poly[k * (N + 1) + l];
            g[k] = ax.w[k] * acc;
        }
    } else {
        double c[kMaxN + 2];
        full_coeffs<kMaxN>(u, T, N, c);
        for (int k = 0; k < ax.nq; k++) {
            double acc = 0;
            for (int l = 0; l <= N; l++) acc += c[l] * ax.poly[k * (N + 1) + l];
            g[k] = ax.w[k] * acc;
        }
    }
}

// ------------------------------------------------------------------ volumes (Appendix A)

// Complete elliptic integrals by Gauss's arithmetic-geometric mean (DLMF 19.8.6-19.8.8), with
// k2 = k^2 and the characteristic alpha2 < 1 of the third kind
//   Pi(alpha2, k) = int_0^{pi/2} dt / ((1 - alpha2 sin^2 t) sqrt(1 - k2 sin^2 t)).
// With a_0 = 1, b_0 = sqrt(1 - k2), a_{n+1} = (a_n + b_n)/2, b_{n+1} = sqrt(a_n b_n), c_0 = k,
// c_{n+1} = (a_n - b_n)/2 and the common limit M:  K = pi/(2M),  E = K (1 - sum_n 2^(n-1) c_n^2);
// with g_0 = sqrt(1 - alpha2), z_0 = 1, g_{n+1} = (g_n^2 + a_n b_n)/(2 g_n) and
// z_{n+1} = z_n (g_n^2 - a_n b_n) / (2 (g_n^2 + a_n b_n)):  Pi = pi/(4M) (2 + alpha2/(1 - alpha2) sum_n z_n).
// The iteration converges quadratically; a few steps reach long double rounding.
struct CompleteElliptic {
    ld K, E, Pi;
};

static CompleteElliptic complete_elliptic(ld k2, ld alpha2)
{
    ld a = 1, b = sqrtl(1 - k2), g = sqrtl(1 - alpha2), z = 1;
    ld csum = k2 / 2, zsum = 1, pow2 = 1;  // pow2 = 2^(n-1) for the next c_n
    for (int it = 0; it < 64; it++) {
        const ld ab = a * b, g2 = g * g;
        const ld znext = z * (g2 - ab) / (2 * (g2 + ab));
        const ld gnext = (g2 + ab) / (2 * g);
        const ld c = (a - b) / 2;
        const ld an = (a + b) / 2, bn = sqrtl(ab);
        csum += pow2 * c * c;
        zsum += znext;
        pow2 *= 2;
        a = an;
        b = bn;
        g = gnext;
        z = znext;
        if (fabsl(c) <= 1e-21L * a && fabsl(z) <= 1e-21L) break;
    }
    CompleteElliptic out;
    out.K = kPi / (2 * a);
    out.E = out.K * (1 - csum);
    out.Pi = kPi / (4 * a) * (2 + alpha2 / (1 - alpha2) * zsum);
    return out;
}

// Volume of the ball of radius s centred at distance b from the axis inside the cylinder of
// radius R (Appendix A, the Lamarche-Leroy formula), valid as printed for s < R and
// |b - R| < s; the other cases are the whole ball or nothing.
double ball_in_cylinder(double s_, double R_, double b_)
{
    const ld s = s_, R = R_, b = b_;
    const ld ball = 4 * kPi * s * s * s / 3;
    if (R <= 0) return 0;
    if (b + s <= R) return (double)ball;
    if (b >= R + s) return 0;
    const ld A = std::max(s * s, (b + R) * (b + R));
    const ld B = std::min(s * s, (b + R) * (b + R));
    const ld C = (b - R) * (b - R);
    const ld k2 = (B - C) / (A - C);
    const ld m = (B - C) / C;  // the paper's -alpha^2
    const ld sg = (b + R) * (b - R);
    // K(k), E(k) and the third kind with alpha^2 = -m: int dz / ((1 + m z^2) sqrt((1 - z^2)(1 - k^2 z^2)))
    const CompleteElliptic ell = complete_elliptic(k2, -m);
    const ld Kk = ell.K, Ek = ell.E, Pk = ell.Pi;
    ld V = (R > b) ? ball : 0;
    V += 4 / (3 * sqrtl(A - C)) *
         (Pk * B * B * sg / C + Kk * (sg * (A - 2 * B) + (A - B) * (3 * B - C - 2 * A) / 3) +
          Ek * (A - C) * (-sg + (2 * A + 2 * C - 4 * B) / 3));
    return (double)V;
}

// Volume of the part x < X of the ball of radius s centred at x = b (plates: a spherical cap of
// height h = X - b + s, of volume pi h^2 (3 s - h) / 3).
double ball_below_plane(double s_, double X_, double b_)
{
    const ld s = s_, h = (ld)X_ - b_ + s;
    if (h <= 0) return 0;
    if (h >= 2 * s) return (double)(4 * kPi * s * s * s / 3);
    return (double)(kPi * h * h * (3 * s - h) / 3);
}

// Volume of the ball of radius s centred at distance b from the origin inside the ball of
// radius R about the origin (Appendix A, lens of two spheres).
double ball_in_sphere(double s_, double R_, double b_)
{
    const ld s = s_, R = R_, b = b_;
    if (R <= 0) return 0;
    if (b + s <= R) return (double)(4 * kPi * s * s * s / 3);
    if (b >= R + s) return 0;
    if (b + R <= s) return (double)(4 * kPi * R * R * R / 3);
    const ld t = s + R - b;
    return (double)(kPi * t * t * (b * b + 2 * b * (s + R) - 3 * (s - R) * (s - R)) / (12 * b));
}

// ------------------------------------------------------------------ attractive mean field
// Enskog-Vlasov mean field of a Sutherland tail phi(t) = -phi_a (sigma / t)^6, t > sigma (beyond
// the paper; its Sec. V names attractive forces as the next step).  mf_potential(r; s) is the
// integral of phi over the region of radius s (ball, infinite cylinder, or the half space x' < s)
// seen from a point at radius r:
//   plane:    over the transverse plane first, g(D) = -(pi/2) phi_a sigma^6 / max(D^2, sigma^2)^2,
//             then the integral of g over D > r - s in closed form;
//   sphere:   shells about the origin: by the shell theorem a shell of radius rho seen from r
//             contributes (2 pi rho / r) int_{|r-rho|}^{r+rho} t phi(t) dt = -(2 pi rho / r)
//             phi_a sigma^6 [h(|r - rho|) - h(r + rho)], h(t) = max(t, sigma)^-4 / 4; the rho
//             integral in closed form from the running integrals of h and t h;
//   cylinder: the axial direction first, lam(d) = int phi(sqrt(d^2 + z^2)) dz in closed form,
//             then int_0^{r+s} lam(d) d arc(d) dd over the disk about the point (arc: the angle
//             of the circle of radius d inside the disk of radius s).  On each piece [p, q]
//             between the kinks (sigma, |r - s|) d = p + (q - p)(1 - cos th)/2 makes the
//             square-root ends smooth; 16-point Gauss-Legendre panels in th, graded towards an
//             end where a singular point outside the piece comes close.

// int_0^t h, int_0^t tau h(tau) for h = max(tau, sigma)^-4 / 4
static ld mf_c0(ld t, ld sg)
{
    return t <= sg ? t / (4 * sg * sg * sg * sg) : 1 / (4 * sg * sg * sg) + (1 / (sg * sg * sg) - 1 / (t * t * t)) / 12;
}
static ld mf_c1(ld t, ld sg)
{
    return t <= sg ? t * t / (8 * sg * sg * sg * sg) : 1 / (8 * sg * sg) + (1 / (sg * sg) - 1 / (t * t)) / 8;
}

// int_0^beta sin^4: Taylor series (no cancellation) below 1/2, else 3b/8 - sin(2b)/4 + sin(4b)/32
static ld sin4_integral(ld b)
{
    if (b < 0.5L) {
        // sum_{k>=2} (-1)^k (16^k - 4^(k+1)) b^(2k+1) / (8 (2k+1)!)
        ld b2 = b * b, pw = b2 * b2 * b, fact = 120, p16 = 256, p4 = 64, sum = 0;
        for (int k = 2; k < 24; k++) {
            const ld term = (p16 - p4) * pw / (8 * fact);
            sum += (k % 2 ? -term : term);
            pw *= b2;
            fact *= (ld)(2 * k + 2) * (2 * k + 3);
            p16 *= 16;
            p4 *= 4;
        }
        return sum;
    }
    return 3 * b / 8 - sinl(2 * b) / 4 + sinl(4 * b) / 32;
}

// line integral of t^-6 over the z with t = sqrt(d^2 + z^2) > sigma: with z = d cot(beta),
// 2 d^-5 int_0^beta0 sin^4, beta0 = asin(d / sigma) (pi / 2 for d >= sigma)
static double mf_line(double d, double sg)
{
    const ld dd = d, d5 = dd * dd * dd * dd * dd;
    if (d >= sg) return (double)(3 * kPi / (8 * d5));
    return (double)(2 * sin4_integral(asinl(dd / sg)) / d5);
}

static double mf_arc(double d, double r, double s)
{
    if (r + d <= s) return 2 * M_PI;
    if (d >= r + s || d + s <= r) return 0.0;
    double c = (r * r + d * d - s * s) / (2 * r * d);
    c = std::min(1.0, std::max(-1.0, c));
    return 2 * std::acos(c);
}

static const std::vector<double>& gl16()
{
    static std::vector<double> xw;
    static std::once_flag once;
    std::call_once(once, [] {
        std::vector<ld> x, w;
        gauss_legendre(16, x, w);
        for (int i = 0; i < 16; i++) xw.push_back((double)x[i]);
        for (int i = 0; i < 16; i++) xw.push_back((double)w[i]);
    });
    return xw;
}

double mf_potential(int geometry, double sigma, double phi_a, double r, double s)
{
    const ld sg = sigma, sg3 = sg * sg * sg, amp = -(ld)phi_a * sg3 * sg3;
    if (geometry == LBE_PLANAR) {
        const ld t = (ld)r - s;  // U = int_t^inf g(D) dD
        ld k;
        if (t >= sg)
            k = 1 / (3 * t * t * t);
        else if (t >= -sg)
            k = (sg - t) / (sg3 * sg) + 1 / (3 * sg3);
        else
            k = 8 / (3 * sg3) + 1 / (3 * t * t * t);
        return (double)(amp * kPi / 2 * k);
    }
    if (geometry == LBE_SPH) {
        const ld R = r, S = s;
        if (R <= 0) return S > sg ? (double)(4 * kPi * amp * (1 / sg3 - 1 / (S * S * S)) / 3) : 0.0;
        const ld i1 = mf_c1(R + S, sg) - mf_c1(R, sg) - R * (mf_c0(R + S, sg) - mf_c0(R, sg));
        const ld m = std::min(R, S);
        ld i2 = R * (mf_c0(R, sg) - mf_c0(R - m, sg)) - (mf_c1(R, sg) - mf_c1(R - m, sg));
        if (S > R) i2 += R * mf_c0(S - R, sg) + mf_c1(S - R, sg);
        return (double)(2 * kPi * amp / R * (i2 - i1));
    }
    // singular points of lam(d) d arc(d) on the real d axis: 0 (pole), sigma (lam), |r - s| and
    // r + s (arc); each piece [p, q] lies between two of them.  A singular point at distance e
    // outside the piece sits at th = i acosh(1 + 2 e / (q - p)), so the panels are graded from each
    // end down to a quarter of that.
    const std::vector<double>& xw = gl16();
    double bp[4] = {0.0, sigma, std::fabs(r - s), r + s};
    std::sort(bp, bp + 4);
    ld acc = 0;
    std::vector<double> edges;
    for (int k = 0; k < 3; k++) {
        const double p = bp[k], q = std::min(bp[k + 1], r + s);
        if (!(q > p)) continue;
        const double hw = (q - p) / 2;
        double eL = HUGE_VAL, eR = HUGE_VAL;
        for (double x : bp) {
            if (x < p) eL = std::min(eL, p - x);
            if (x > q) eR = std::min(eR, x - q);
        }
        auto reach = [&](double e) { return e == HUGE_VAL ? M_PI : std::acosh(1 + 2 * e / (q - p)); };
        edges.assign(1, 0.0);
        for (double h = std::min(reach(eL), M_PI) / 4, x = 0; x + h < M_PI / 2; h = x) {
            x += h;
            edges.push_back(x);
        }
        std::vector<double> right;
        for (double h = std::min(reach(eR), M_PI) / 4, x = 0; x + h < M_PI / 2; h = x) {
            x += h;
            right.push_back(M_PI - x);
        }
        edges.push_back(M_PI / 2);
        for (auto it = right.rbegin(); it != right.rend(); ++it) edges.push_back(*it);
        edges.push_back(M_PI);
        for (size_t e = 0; e + 1 < edges.size(); e++) {
            const double c = (edges[e] + edges[e + 1]) / 2, h = (edges[e + 1] - edges[e]) / 2;
            ld part = 0;
            for (int g = 0; g < 16; g++) {
                const double th = c + h * xw[g];
                const double d = p + hw * (1 - std::cos(th));
                if (d <= 0) continue;
                part += (ld)xw[16 + g] * mf_line(d, sigma) * d * mf_arc(d, r, s) * hw * std::sin(th);
            }
            acc += part * h;
        }
    }
    return (double)(amp * acc);
}

// Mean-field weights: Phi_i = sum_j A_ij n_j, A_ij = n0 [U(r_i; ri_{j+1}) - U(r_i; ri_j)] with
// n0 = 6 eta0 / (pi sigma^3) (n in units of the mean density, zero outside the domain).
static void mf_weights(InstanceTables* t)
{
    const int nr = t->nr;
    const lbe_params& p = t->prm;
    const ld n0 = 6 * (ld)p.eta0 / (kPi * (ld)t->sigma * t->sigma * t->sigma);
    t->amf.assign((size_t)nr * nr, 0.0);
    // rows are independent: spread over host threads (each row's arithmetic is the same whatever the
    // thread, so the weights do not depend on the thread count)
    std::atomic<int> next{0};
    auto rows = [&]() {
        std::vector<double> U(nr + 1);
        for (int i = next++; i < nr; i = next++) {
            for (int j = 0; j <= nr; j++) U[j] = mf_potential(p.geometry, t->sigma, p.phi_a, t->r[i], t->ri[j]);
            for (int j = 0; j < nr; j++) t->amf[(size_t)i * nr + j] = (double)(n0 * ((ld)U[j + 1] - U[j]));
        }
    };
    const int nth = p.geometry == LBE_CYL ? std::max(1, std::min<int>(nr, (int)std::thread::hardware_concurrency())) : 1;
    std::vector<std::thread> pool;
    for (int k = 1; k < nth; k++) pool.emplace_back(rows);
    rows();
    for (std::thread& th : pool) th.join();
}

// ------------------------------------------------------------------ instance set-up

lbe_status validate_params(const lbe_params& in, lbe_params* out, std::string* err)
{
    lbe_params p = in;
    auto bad = [&](const char* m) {
        if (err) *err = m;
        return LBE_EINVAL;
    };
    if (p.geometry != LBE_CYL && p.geometry != LBE_SPH && p.geometry != LBE_PLANAR)
        return bad("geometry must be LBE_CYL, LBE_SPH or LBE_PLANAR");
    if (!(p.r_inner > 0) || !(p.r_outer > p.r_inner) || !std::isfinite(p.r_outer))
        return bad("need 0 < r_inner < r_outer");
    if (!(p.eta0 > 0 && p.eta0 < 0.5)) return bad("eta0 must lie in (0, 0.5)");
    if (!(p.kn > 0) || !std::isfinite(p.kn)) return bad("kn must be positive");
    if (!(p.t_wall_inner > 0) || !(p.t_wall_outer > 0)) return bad("wall temperatures must be positive");
    if (!(p.cfl > 0) || !std::isfinite(p.cfl)) return bad("cfl must be positive");
    if (!std::isfinite(p.u_wall_inner)) return bad("u_wall_inner must be finite");
    if (p.geometry == LBE_SPH && p.u_wall_inner != 0) return bad("a spherical instance cannot have a wall velocity");
    if (p.reduced != 0 && p.reduced != 1) return bad("reduced must be 0 or 1");
    if (p.reduced && p.geometry == LBE_SPH) return bad("the reduced distributions are for cylinders and plates");
    if (!std::isfinite(p.phi_a)) return bad("phi_a must be finite");
    if (p.reduced) {  // the (phi, chi) planes take the place of the p_z axis
        p.q_t2 = 2;
        p.n_expand[2] = 2;
    }
    if (p.nr < 8 || p.nr > 1024) return bad("nr must lie in [8, 1024]");
    if (p.precision != LBE_FP64 && p.precision != LBE_FP32_STORE) return bad("precision must be LBE_FP64 or LBE_FP32_STORE");
    const int Q[3] = {p.q_radial, p.q_t1, p.q_t2};
    for (int a = 0; a < 3; a++) {
        if (Q[a] < 2 || Q[a] > kMaxQ) return bad("quadrature orders must lie in [2, 100]");
        int N = p.n_expand[a];
        if (N == 0) N = std::min(7, Q[a] - 1);
        if (a == 2 && p.reduced) N = 2;  // the pseudo-axis of the reduced distributions (below)
        else if (N < 1 || N >= Q[a] || N > kMaxN) return bad("expansion orders need 1 <= N_a < Q_a and N_a <= 15");
        p.n_expand[a] = N;
    }
    const double C = 1 / (6 * std::sqrt(2.0) * p.eta0 * chi_cs(p.eta0) * p.kn);
    if (!(C > 1)) return bad("confinement ratio C = L/sigma must exceed 1 (sigma < L)");
    if (out) *out = p;
    return LBE_OK;
}

lbe_status build_instance(const lbe_params& pin, InstanceTables* t, std::string* err)
{
    lbe_params p;
    lbe_status st = validate_params(pin, &p, err);
    if (st != LBE_OK) return st;
    t->prm = p;
    // the equilibrium projection rule covers Gaussians up to 1.5 times the hottest wall
    const double Tmax = std::max(1.0, std::max(p.t_wall_inner, p.t_wall_outer));
    const double Y = 3 + 13 * std::sqrt(1.5 * Tmax) + std::fabs(p.u_wall_inner);
    // panel width of the projection rule: 16-point Gauss-Legendre integrates the Gaussian of
    // temperature T times h_l (l <= 7) to rounding (measured against 30-digit quadrature: 3e-16
    // at 3.35 sqrt(T), 2e-14 at 4.7 sqrt(T)); the width is sized for half the colder wall's
    // temperature and kept within [0.1875, 1.5]
    const double Tlow = 0.5 * std::min(p.t_wall_inner, p.t_wall_outer);
    const double hwidth = std::min(1.5, std::max(0.1875, 3.35 * std::sqrt(Tlow)));
    build_half_axis(p.q_radial, p.n_expand[0], Y, hwidth, &t->ax[0], &t->K1, &t->K2r);
    build_full_axis(p.q_t1, p.n_expand[1], &t->ax[1], &t->K2a);
    if (p.reduced)
        build_reduced_axis(&t->ax[2], &t->K2b);
    else
        build_full_axis(p.q_t2, p.n_expand[2], &t->ax[2], &t->K2b);
    t->n0 = t->ax[0].nq;
    t->n1 = t->ax[1].nq;
    t->n2 = t->ax[2].nq;
    t->nv = t->n0 * t->n1 * t->n2;
    t->nr = p.nr;

    // Kn map (Sec. II) and the computational domain (Sec. IV).
    t->chi0 = chi_cs(p.eta0);
    t->C = 1 / (6 * std::sqrt(2.0) * p.eta0 * t->chi0 * p.kn);
    t->L = p.r_outer - p.r_inner;
    t->sigma = t->L / t->C;
    t->rcl = p.r_inner + t->sigma / 2;
    t->rcr = p.r_outer - t->sigma / 2;
    t->dr = (t->rcr - t->rcl) / t->nr;
    const int nr = t->nr;
    t->r.resize(nr);
    t->ri.resize(nr + 1);
    for (int i = 0; i <= nr; i++) t->ri[i] = t->rcl + i * t->dr;
    for (int i = 0; i < nr; i++) t->r[i] = t->rcl + (i + 0.5) * t->dr;
    double pmax = 0;
    for (double v : t->ax[0].p) pmax = std::max(pmax, std::fabs(v));
    t->dt = p.cfl * t->dr / pmax;

    // Flux-form geometry: cell measure V_i (r_i dr, or (ri_{i+1}^3 - ri_i^3)/3), interface
    // weights ri/V_i (cylinder) or ri^2/V_i (sphere), force-term factor 1/r_i (cylinder) or
    // (ri_{i+1}^2 - ri_i^2)/(2 V_i) (sphere: balances the flux form exactly at rest).
    t->geo.resize(4 * nr);
    for (int i = 0; i < nr; i++) {
        const ld rl = t->ri[i], rr = t->ri[i + 1], rc = t->r[i];
        if (p.geometry == LBE_PLANAR) {  // Cartesian: no radius weights, no force terms
            t->geo[4 * i + 0] = t->geo[4 * i + 1] = (double)(1 / (ld)t->dr);
            t->geo[4 * i + 2] = 0.0;
            t->geo[4 * i + 3] = 0.0;
            continue;
        }
        if (p.geometry == LBE_CYL) {
            const ld V = rc * (ld)t->dr;
            t->geo[4 * i + 0] = (double)(rl / V);
            t->geo[4 * i + 1] = (double)(rr / V);
            t->geo[4 * i + 2] = (double)(1 / rc);
        } else {
            const ld V = (rr * rr * rr - rl * rl * rl) / 3;
            t->geo[4 * i + 0] = (double)(rl * rl / V);
            t->geo[4 * i + 1] = (double)(rr * rr / V);
            t->geo[4 * i + 2] = (double)((rr * rr - rl * rl) / (2 * V));
        }
        t->geo[4 * i + 3] = (double)(1 / rc);
    }

    // Averaged-density weights, eq. (fm) with n piecewise constant on cells and zero outside
    // the computational domain: W_ij = [V(sigma; ri_{j+1}, r_i) - V(sigma; ri_j, r_i)] / ball.
    {
        const double s = t->sigma;
        const ld ball = 4 * kPi * (ld)s * s * s / 3;
        t->wlo.assign(nr, 0);
        std::vector<int> whi(nr);
        int wb = 1;
        for (int i = 0; i < nr; i++) {
            int lo = (int)std::floor((t->r[i] - s - t->rcl) / t->dr) - 1;
            int hi = (int)std::floor((t->r[i] + s - t->rcl) / t->dr) + 1;
            lo = std::max(lo, 0);
            hi = std::min(hi, nr - 1);
            t->wlo[i] = lo;
            whi[i] = hi;
            wb = std::max(wb, hi - lo + 1);
        }
        t->wband = wb;
        t->wb.assign((size_t)nr * wb, 0);
        for (int i = 0; i < nr; i++) {
            const int lo = t->wlo[i], hi = whi[i];
            std::vector<double> V(hi - lo + 2);
            for (int j = lo; j <= hi + 1; j++)
                V[j - lo] = p.geometry == LBE_CYL   ? ball_in_cylinder(s, t->ri[j], t->r[i])
                            : p.geometry == LBE_SPH ? ball_in_sphere(s, t->ri[j], t->r[i])
                                                    : ball_below_plane(s, t->ri[j], t->r[i]);
            for (int j = lo; j <= hi; j++) t->wb[(size_t)i * wb + (j - lo)] = (double)(((ld)V[j + 1 - lo] - V[j - lo]) / ball);
        }
    }

    if (p.phi_a != 0) mf_weights(t);

    // Unit wall Maxwellians g_r(0, T_w) g_1(u_w, T_w) g_2(0, T_w) and the entering flux sums.
    t->gwl.resize(t->nv);
    t->gwr.resize(t->nv);
    {
        std::vector<double> g0(t->n0), g1(t->n1), g2(t->n2);
        for (int side = 0; side < 2; side++) {
            const double Tw = side == 0 ? p.t_wall_inner : p.t_wall_outer;
            const double uw = side == 0 ? p.u_wall_inner : 0.0;
            equilibrium_axis(t->ax[0], 0.0, Tw, g0.data());
            equilibrium_axis(t->ax[1], uw, Tw, g1.data());
            equilibrium_axis(t->ax[2], 0.0, Tw, g2.data());
            std::vector<double>& gw = side == 0 ? t->gwl : t->gwr;
            ld gin = 0;
            for (int v = 0; v < t->nv; v++) {
                const int i0 = v % t->n0, i1 = (v / t->n0) % t->n1, i2 = v / (t->n0 * t->n1);
                gw[v] = g0[i0] * g1[i1] * g2[i2];
                const double pr = t->ax[0].p[i0];
                if (p.reduced && i2 == 1) continue;  // the mass flux is carried by phi alone
                if ((side == 0 && pr > 0) || (side == 1 && pr < 0)) gin += (ld)pr * gw[v];
            }
            (side == 0 ? t->gin_l : t->gin_r) = (double)gin;
        }
    }
    return LBE_OK;
}

}  // namespace lbe

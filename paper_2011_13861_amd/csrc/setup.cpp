// Host setup of the KL operator in FP64 (runs once per problem, Sec. 3.5 and 4.1-4.3).
//
// Per direction k:
//   knots (open uniform, C^{p-1}, or an explicit open knot vector), B-spline evaluation
//   by the triangular Cox-de Boor
//   scheme restricted to the p+1 non-zero functions, Greville abscissae (knot averages),
//   Z_k = int B_i B_j (Gauss-Legendre, p+1 points per element; Remark massmatrix),
//   L_k = chol(Z_k) (eq. cholesky), Bt_k[i][j] = Bt_j(xhat_i) (eq. interpolation_matrix)
//   with partial-pivot LU, M_k = int Bt_i B_j (eq. univariate_mass_matrix2), and the
//   composed factor C_k = Bt_k^{-T} M_k L_k^{-T}.  By the mixed-product property of
//   Kronecker products (Sec. 2.2), stages 1-3 of Algorithm 1 equal one Kronecker
//   product C = C_d x ... x C_1, and stages 7-9 equal C^T.
// Over the Greville grid: X = F(xhat), J = sqrt(det DF(xhat)) (eq. integrand).
#include <cmath>
#include <cstring>
#include <sstream>
#include <string>

#include "kl_internal.h"

namespace kl {
namespace {

// Open knot vector on [0, 1] with ne uniform elements, each interior breakpoint repeated
// `mult` times (continuity C^{p-mult} there); n = p + 1 + (ne - 1) mult functions.
std::vector<double> uniform_knots(int p, int ne, int mult = 1) {
    std::vector<double> t;
    for (int i = 0; i <= p; ++i) t.push_back(0.0);
    for (int j = 1; j < ne; ++j)
        for (int m = 0; m < mult; ++m) t.push_back(double(j) / ne);
    for (int i = 0; i <= p; ++i) t.push_back(1.0);
    return t;
}

// Knot span s with t[s] <= x < t[s+1], p <= s <= n-1; the right end maps to n-1.
int find_span(const std::vector<double> &t, int p, int n, double x) {
    if (x >= t[n]) return n - 1;
    if (x <= t[p]) return p;
    int lo = p, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x < t[mid]) hi = mid; else lo = mid;
    }
    return lo;
}

// The span for the limit from one side: side >= 0 as find_span; side < 0 the span with
// t[s] < x <= t[s+1] (the non-empty span that ends at x when x is a knot).
int find_span_side(const std::vector<double> &t, int p, int n, double x, int side) {
    int s = find_span(t, p, n, x);
    if (side < 0)
        while (s > p && t[s] == x) --s;
    return s;
}

// The p+1 non-zero B-splines B_{s-p..s}(x) via the triangular recurrence.
void nonzero_basis(const std::vector<double> &t, int p, int s, double x, double *out) {
    double left[32], right[32];
    out[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double carry = 0.0;
        for (int r = 0; r < j; ++r) {
            double den = right[r + 1] + left[j - r];
            double tmp = den != 0.0 ? out[r] / den : 0.0;
            out[r] = carry + right[r + 1] * tmp;
            carry = left[j - r] * tmp;
        }
        out[j] = carry;
    }
}

// Values and first derivatives of the p+1 non-zero B-splines at x: the derivative of
// B_{i,p} is p B_{i,p-1} / (t_{i+p} - t_i) - p B_{i+1,p-1} / (t_{i+p+1} - t_{i+1}) (Sec. 2.3).
void nonzero_basis_ders(const std::vector<double> &t, int p, int s, double x, double *val, double *der) {
    double lower[32];
    nonzero_basis(t, p - 1, s, x, lower);      // B_{s-p+1..s, p-1}
    for (int a = 0; a <= p; ++a) {
        const int i = s - p + a;
        double d = 0.0;
        if (a >= 1) {
            const double den = t[i + p] - t[i];
            if (den > 0.0) d += p * lower[a - 1] / den;
        }
        if (a <= p - 1) {
            const double den = t[i + p + 1] - t[i + 1];
            if (den > 0.0) d -= p * lower[a] / den;
        }
        der[a] = d;
    }
    nonzero_basis(t, p, s, x, val);
}

// An explicit knot vector: finite, nondecreasing, open (first and last value repeated
// p + 1 times), from 0 to 1, interior values repeated at most max_mult times (p + 1 for
// the spline spaces: C^-1; p for maps: C^0).
bool valid_knots(const double *t, int len, int p, int max_mult, std::string &why) {
    if (!t || len < p + 2 + p) { why = "needs at least 2 p + 2 entries"; return false; }
    for (int i = 0; i < len; ++i)
        if (!std::isfinite(t[i]) || (i > 0 && t[i] < t[i - 1])) { why = "must be finite and nondecreasing"; return false; }
    if (t[0] != 0.0 || t[len - 1] != 1.0) { why = "must run from 0 to 1"; return false; }
    for (int i = 0; i <= p; ++i)
        if (t[i] != 0.0 || t[len - 1 - i] != 1.0) { why = "must be open (end values repeated p + 1 times)"; return false; }
    if (t[p + 1] == 0.0 || t[len - p - 2] == 1.0) { why = "must be open (end values repeated p + 1 times)"; return false; }
    for (int i = p + 1; i < len - p - 1;) {
        int j = i;
        while (j < len - p - 1 && t[j] == t[i]) ++j;
        if (j - i > max_mult) {
            why = max_mult > p ? "interior values may repeat at most p + 1 times (C^-1)"
                               : "interior values may repeat at most p times (C^0)";
            return false;
        }
        i = j;
    }
    return true;
}

// Greville abscissae (knot averages); the knot itself where the p knots coincide, so that
// the two abscissae at a knot repeated p + 1 times are equal.  side[i] = -1 where the
// abscissa is the right end of the support [t_i, t_{i+p+1}] of function i (the knots
// t_{i+1} .. t_{i+p+1} coincide: the left function at a C^-1 knot, and the last function at
// x = 1): there the basis is evaluated as the limit from the left; +1 elsewhere.
std::vector<double> greville(const std::vector<double> &t, int p, int n, std::vector<int> *side = nullptr) {
    std::vector<double> g(n);
    for (int i = 0; i < n; ++i) {
        if (t[i + 1] == t[i + p]) {
            g[i] = t[i + 1];
        } else {
            double s = 0.0;
            for (int j = 1; j <= p; ++j) s += t[i + j];
            g[i] = s / p;
        }
    }
    if (side) {
        side->assign(n, 1);
        for (int i = 0; i < n; ++i)
            if (t[i + 1] == t[i + p + 1]) (*side)[i] = -1;
    }
    return g;
}

// q-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_q.
void gauss_legendre(int q, std::vector<double> &x, std::vector<double> &w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < q; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_q(z), p0 = P_{q-1}(z)
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

std::vector<double> breakpoints(const std::vector<double> &t) {
    std::vector<double> b;
    for (double v : t)
        if (b.empty() || v > b.back()) b.push_back(v);
    return b;
}

// Composite rule with q points on each non-empty span of `br`.
void composite_rule(const std::vector<double> &br, int q, std::vector<double> &xs,
                    std::vector<double> &ws) {
    std::vector<double> gx, gw;
    gauss_legendre(q, gx, gw);
    xs.clear();
    ws.clear();
    for (size_t e = 0; e + 1 < br.size(); ++e) {
        double a = br[e], b = br[e + 1];
        for (int i = 0; i < q; ++i) {
            xs.push_back(0.5 * (b - a) * gx[i] + 0.5 * (a + b));
            ws.push_back(0.5 * (b - a) * gw[i]);
        }
    }
}

// Dense Cholesky, row-major n x n, lower factor in place.  false if not SPD.
bool cholesky(std::vector<double> &A, int n) {
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return false;
        double ljj = std::sqrt(s);
        A[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / ljj;
        }
        for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
    }
    return true;
}

// LU with partial pivoting, row-major n x n in place; piv[i] = row swapped with i.
bool lu_factor(std::vector<double> &A, int n, std::vector<int> &piv, double &max_abs) {
    piv.resize(n);
    max_abs = 0.0;
    for (double v : A) max_abs = std::fmax(max_abs, std::fabs(v));
    for (int k = 0; k < n; ++k) {
        int r = k;
        double best = std::fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > best) { best = std::fabs(A[i * n + k]); r = i; }
        piv[k] = r;
        if (!(best > 1e-13 * max_abs)) return false;
        if (r != k)
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[r * n + j]);
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            A[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
        }
    }
    return true;
}

// Solves A^T x = b with the LU factors of A (PA = LU  =>  A^T = U^T L^T P).
void lu_solve_transposed(const std::vector<double> &LU, const std::vector<int> &piv, int n,
                         double *b) {
    for (int i = 0; i < n; ++i) {           // U^T y = b (forward)
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= LU[k * n + i] * b[k];
        b[i] = s / LU[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {      // L^T z = y (backward, unit diagonal)
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= LU[k * n + i] * b[k];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i)        // x = P^T z
        if (piv[i] != i) std::swap(b[i], b[piv[i]]);
}

struct Dir {
    int p, pt, n, nt;
    std::vector<double> t, tt;
};

// C_k = Bt^{-T} M L^{-T} for one direction; also E_k = B(g) L^{-T}, the trial B-splines at
// the interpolation Greville abscissae g applied to standard-form coefficients (Sec. 3.4,
// 4.1), which evaluates eigenfunctions there.
kl_status build_direction(Dir &D, std::vector<double> &C, std::vector<double> &E, std::vector<double> &LT,
                          std::vector<double> &g, std::vector<int> &gside) {
    const int n = D.n, nt = D.nt;
    // Z_k by Gauss-Legendre with p+1 points per element
    std::vector<double> xs, ws;
    composite_rule(breakpoints(D.t), D.p + 1, xs, ws);
    std::vector<double> Z(size_t(n) * n, 0.0);
    double B[32], Bt[32];
    for (size_t q = 0; q < xs.size(); ++q) {
        int s = find_span(D.t, D.p, n, xs[q]);
        nonzero_basis(D.t, D.p, s, xs[q], B);
        for (int a = 0; a <= D.p; ++a)
            for (int b = 0; b <= D.p; ++b)
                Z[size_t(s - D.p + a) * n + (s - D.p + b)] += ws[q] * B[a] * B[b];
    }
    if (!cholesky(Z, n)) {
        set_error("univariate Gramian is not positive definite");
        return KL_ESINGULAR;
    }
    // M_k on the union of breakpoints, ceil((p + pt + 1) / 2) points per span
    std::vector<double> br = breakpoints(D.t), brt = breakpoints(D.tt), un;
    {
        size_t i = 0, j = 0;
        while (i < br.size() || j < brt.size()) {
            double v;
            if (j >= brt.size() || (i < br.size() && br[i] < brt[j])) v = br[i++];
            else if (i >= br.size() || brt[j] < br[i]) v = brt[j++];
            else { v = br[i]; ++i; ++j; }
            if (un.empty() || v > un.back()) un.push_back(v);
        }
    }
    composite_rule(un, (D.p + D.pt + 2) / 2, xs, ws);
    std::vector<double> M(size_t(nt) * n, 0.0);
    for (size_t q = 0; q < xs.size(); ++q) {
        int s = find_span(D.t, D.p, n, xs[q]);
        int st = find_span(D.tt, D.pt, nt, xs[q]);
        nonzero_basis(D.t, D.p, s, xs[q], B);
        nonzero_basis(D.tt, D.pt, st, xs[q], Bt);
        for (int a = 0; a <= D.pt; ++a)
            for (int b = 0; b <= D.p; ++b)
                M[size_t(st - D.pt + a) * n + (s - D.p + b)] += ws[q] * Bt[a] * B[b];
    }
    // collocation matrix at the Greville abscissae of the interpolation space, each
    // abscissa evaluated from the side of its own function
    g = greville(D.tt, D.pt, nt, &gside);
    std::vector<double> Bc(size_t(nt) * nt, 0.0);
    for (int i = 0; i < nt; ++i) {
        int st = find_span_side(D.tt, D.pt, nt, g[i], gside[i]);
        nonzero_basis(D.tt, D.pt, st, g[i], Bt);
        for (int a = 0; a <= D.pt; ++a) Bc[size_t(i) * nt + (st - D.pt + a)] = Bt[a];
    }
    std::vector<int> piv;
    double mx;
    if (!lu_factor(Bc, nt, piv, mx)) {
        set_error("collocation matrix is singular (coincident Greville points?)");
        return KL_ESINGULAR;
    }
    // W = M L^{-T}: each row w of W solves L w^T = m^T (forward substitution)
    std::vector<double> W(size_t(nt) * n);
    for (int r = 0; r < nt; ++r) {
        for (int i = 0; i < n; ++i) {
            double s = M[size_t(r) * n + i];
            for (int k = 0; k < i; ++k) s -= Z[size_t(i) * n + k] * W[size_t(r) * n + k];
            W[size_t(r) * n + i] = s / Z[size_t(i) * n + i];
        }
    }
    // E = B(g) L^{-T}: row r solves L e^T = b(g_r)^T (forward substitution)
    E.assign(size_t(nt) * n, 0.0);
    for (int r = 0; r < nt; ++r) {
        const int s0 = find_span_side(D.t, D.p, n, g[r], gside[r]);
        nonzero_basis(D.t, D.p, s0, g[r], B);
        double *e = &E[size_t(r) * n];
        for (int a = 0; a <= D.p; ++a) e[s0 - D.p + a] = B[a];
        for (int i = 0; i < n; ++i) {
            double s = e[i];
            for (int k = 0; k < i; ++k) s -= Z[size_t(i) * n + k] * e[k];
            e[i] = s / Z[size_t(i) * n + i];
        }
    }
    // L^{-T} (upper triangular): column j solves L^T x = e_j by back substitution
    LT.assign(size_t(n) * n, 0.0);
    for (int j = 0; j < n; ++j) {
        for (int i = j; i >= 0; --i) {
            double s = i == j ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) s -= Z[size_t(k) * n + i] * LT[size_t(k) * n + j];
            LT[size_t(i) * n + j] = s / Z[size_t(i) * n + i];
        }
    }
    // C = Bt^{-T} W, column by column
    C.assign(size_t(nt) * n, 0.0);
    std::vector<double> col(nt);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < nt; ++i) col[i] = W[size_t(i) * n + j];
        lu_solve_transposed(Bc, piv, nt, col.data());
        for (int i = 0; i < nt; ++i) C[size_t(i) * n + j] = col[i];
    }
    return KL_OK;
}

// Quarter-annulus arc: rational quadratic with weights (1, 1/sqrt 2, 1), unit radius.
void arc(double v, double &cx, double &cy, double &dx, double &dy) {
    const double w = std::sqrt(0.5);
    double b0 = (1 - v) * (1 - v), b1 = 2 * v * (1 - v), b2 = v * v;
    double d0 = -2 * (1 - v), d1 = 2 - 4 * v, d2 = 2 * v;
    double Px = b0 + w * b1, Py = w * b1 + b2, W = b0 + w * b1 + b2;
    double dPx = d0 + w * d1, dPy = w * d1 + d2, dW = d0 + w * d1 + d2;
    cx = Px / W;
    cy = Py / W;
    dx = (dPx * W - Px * dW) / (W * W);
    dy = (dPy * W - Py * dW) / (W * W);
}

// F(u) and det DF(u) for one parametric point; side[k] < 0 takes the derivative along u_k
// from the left (it differs from the right one only on a C^0 line of a NURBS map).
bool map_point(const kl_desc &desc, int d, const double *u, const int *side, double *x, double &det) {
    const double *mp = desc.map_params;
    switch (desc.map_kind) {
    case KL_MAP_IDENTITY:
        for (int k = 0; k < d; ++k) x[k] = u[k];
        det = 1.0;
        return true;
    case KL_MAP_BOX:
        det = 1.0;
        for (int k = 0; k < d; ++k) {
            double lo = mp[k], hi = mp[3 + k];
            x[k] = lo + (hi - lo) * u[k];
            det *= (hi - lo);
        }
        return true;
    case KL_MAP_ANNULUS_NURBS: {
        double r0 = mp[0], r1 = mp[1];
        double rho = r0 + (r1 - r0) * u[0];
        double cx, cy, dx, dy;
        arc(u[1], cx, cy, dx, dy);
        x[0] = rho * cx;
        x[1] = rho * cy;
        det = (r1 - r0) * rho * (cx * dy - cy * dx);
        return true;
    }
    case KL_MAP_ANNULUS_POLAR: {
        double r0 = mp[0], r1 = mp[1];
        double rho = r0 + (r1 - r0) * u[0], th = 0.5 * M_PI * u[1];
        x[0] = rho * std::cos(th);
        x[1] = rho * std::sin(th);
        det = (r1 - r0) * rho * 0.5 * M_PI;
        return true;
    }
    case KL_MAP_SINE_CUBE: {
        double eps = mp[0];
        const double *amp = mp + 1;
        double s = 1.0, sn[3], cs[3];
        for (int k = 0; k < d; ++k) {
            sn[k] = std::sin(M_PI * u[k]);
            cs[k] = std::cos(M_PI * u[k]);
            s *= sn[k];
        }
        double dots = 0.0;  // amp . grad s  (matrix determinant lemma: det(I + e a g^T) = 1 + e a.g)
        for (int k = 0; k < d; ++k) {
            double gk = M_PI * cs[k];
            for (int m = 0; m < d; ++m)
                if (m != k) gk *= sn[m];
            dots += amp[k] * gk;
        }
        for (int k = 0; k < d; ++k) x[k] = u[k] + eps * amp[k] * s;
        det = 1.0 + eps * dots;
        return true;
    }
    case KL_MAP_TENSOR_NURBS: {
        // F(u) = A(u) / W(u), A = sum_a w_a P_a N_a(u), W = sum_a w_a N_a(u) over the
        // (p_k + 1)^d non-zero tensor functions; dF/du_k = (dA/du_k - F dW/du_k) / W
        double val[3][32], der[3][32];
        int span[3], m[3];
        for (int k = 0; k < d; ++k) {
            const int pk = desc.map_degree[k];
            m[k] = desc.map_nknots[k] - pk - 1;
            const std::vector<double> t(desc.map_knots[k], desc.map_knots[k] + desc.map_nknots[k]);
            span[k] = find_span_side(t, pk, m[k], u[k], side[k]);
            nonzero_basis_ders(t, pk, span[k], u[k], val[k], der[k]);
        }
        double A[3] = {0, 0, 0}, dA[3][3] = {{0}}, W = 0.0, dW[3] = {0, 0, 0};
        const int q0 = desc.map_degree[0] + 1, q1 = d > 1 ? desc.map_degree[1] + 1 : 1,
                  q2 = d > 2 ? desc.map_degree[2] + 1 : 1;
        for (int c = 0; c < q2; ++c)
            for (int b = 0; b < q1; ++b)
                for (int a = 0; a < q0; ++a) {
                    const int ia[3] = {a, b, c};
                    int64_t idx = 0, stride = 1;
                    double Nv = 1.0, dN[3] = {1.0, 1.0, 1.0};
                    for (int k = 0; k < d; ++k) {
                        const int i = span[k] - desc.map_degree[k] + ia[k];
                        idx += stride * i;
                        stride *= m[k];
                        Nv *= val[k][ia[k]];
                        for (int j = 0; j < d; ++j) dN[j] *= (j == k ? der[k][ia[k]] : val[k][ia[k]]);
                    }
                    const double w = desc.map_weights ? desc.map_weights[idx] : 1.0;
                    const double *P = desc.map_ctrl + size_t(idx) * d;
                    W += w * Nv;
                    for (int j = 0; j < d; ++j) dW[j] += w * dN[j];
                    for (int i = 0; i < d; ++i) {
                        A[i] += w * Nv * P[i];
                        for (int j = 0; j < d; ++j) dA[i][j] += w * dN[j] * P[i];
                    }
                }
        double D[3][3];
        for (int i = 0; i < d; ++i) x[i] = A[i] / W;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) D[i][j] = (dA[i][j] - x[i] * dW[j]) / W;
        if (d == 1) det = D[0][0];
        else if (d == 2) det = D[0][0] * D[1][1] - D[0][1] * D[1][0];
        else
            det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                  D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                  D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
        return true;
    }
    default:
        return false;
    }
}

// Validates the TENSOR_NURBS fields of the description.
kl_status check_nurbs_map(const kl_desc &desc, int d) {
    int64_t npts = 1;
    for (int k = 0; k < d; ++k) {
        const int pk = desc.map_degree[k];
        std::string why;
        if (pk < 1 || pk > 20) { set_error("map_degree must be in 1..20"); return KL_EINVAL; }
        if (!valid_knots(desc.map_knots[k], desc.map_nknots[k], pk, pk, why)) {
            set_error("map knot vector " + std::to_string(k) + ": " + why);
            return KL_EINVAL;
        }
        npts *= desc.map_nknots[k] - pk - 1;
    }
    if (!desc.map_ctrl) { set_error("TENSOR_NURBS needs map_ctrl"); return KL_EINVAL; }
    for (int64_t i = 0; i < npts * d; ++i)
        if (!std::isfinite(desc.map_ctrl[i])) { set_error("map_ctrl must be finite"); return KL_EINVAL; }
    if (desc.map_weights)
        for (int64_t i = 0; i < npts; ++i)
            if (!(desc.map_weights[i] > 0.0) || !std::isfinite(desc.map_weights[i])) {
                set_error("map_weights must be positive");
                return KL_EINVAL;
            }
    return KL_OK;
}

}  // namespace

kl_status build_host_setup(const kl_desc &desc, HostSetup &hs) {
    const int d = desc.dim;
    if (d < 1 || d > 3) { set_error("dim must be 1, 2 or 3"); return KL_EINVAL; }
    if (desc.map_kind < KL_MAP_IDENTITY || desc.map_kind > KL_MAP_TENSOR_NURBS) {
        set_error("unknown map_kind"); return KL_EINVAL;
    }
    if (desc.map_kind == KL_MAP_TENSOR_NURBS) {
        kl_status st = check_nurbs_map(desc, d);
        if (st != KL_OK) return st;
    }
    if ((desc.map_kind == KL_MAP_ANNULUS_NURBS || desc.map_kind == KL_MAP_ANNULUS_POLAR) && d != 2) {
        set_error("annulus maps are two-dimensional"); return KL_EINVAL;
    }
    if ((desc.map_kind == KL_MAP_ANNULUS_NURBS || desc.map_kind == KL_MAP_ANNULUS_POLAR) &&
        !(desc.map_params[0] > 0 && desc.map_params[1] > desc.map_params[0])) {
        set_error("annulus needs 0 < r0 < r1"); return KL_EINVAL;
    }
    if (desc.cov_kind < KL_COV_EXP || desc.cov_kind > KL_COV_LIN) {
        set_error("unknown cov_kind"); return KL_EINVAL;
    }
    if (!(desc.sigma2 > 0) || !std::isfinite(desc.sigma2)) { set_error("sigma2 must be > 0"); return KL_EINVAL; }
    for (int k = 0; k < d; ++k)
        if (!(desc.corr_len[k] > 0) || !std::isfinite(desc.corr_len[k])) {
            set_error("corr_len must be > 0"); return KL_EINVAL;
        }
    hs = HostSetup();
    hs.d = d;
    Dir D[3];
    int64_t N = 1, Nt = 1;
    for (int k = 0; k < d; ++k) {
        Dir &r = D[k];
        r.p = desc.degree[k];
        r.pt = desc.interp_degree[k] > 0 ? desc.interp_degree[k] : r.p;
        if (r.p < 1 || r.p > 20 || r.pt < 1 || r.pt > 20) { set_error("degrees must be in 1..20"); return KL_EINVAL; }
        std::string why;
        if (desc.knots[k]) {
            if (!valid_knots(desc.knots[k], desc.nknots[k], r.p, r.p + 1, why)) {
                set_error("trial knot vector " + std::to_string(k) + ": " + why);
                return KL_EINVAL;
            }
            r.t.assign(desc.knots[k], desc.knots[k] + desc.nknots[k]);
        } else {
            if (desc.nelem[k] < 1 || desc.nelem[k] > 100000) { set_error("element counts must be >= 1"); return KL_EINVAL; }
            r.t = uniform_knots(r.p, desc.nelem[k]);
        }
        if (desc.interp_knots[k]) {
            if (!valid_knots(desc.interp_knots[k], desc.interp_nknots[k], r.pt, r.pt + 1, why)) {
                set_error("interpolation knot vector " + std::to_string(k) + ": " + why);
                return KL_EINVAL;
            }
            r.tt.assign(desc.interp_knots[k], desc.interp_knots[k] + desc.interp_nknots[k]);
        } else if (desc.knots[k] && r.pt == r.p && desc.interp_nelem[k] == 0 && desc.interp_mult[k] == 0) {
            r.tt = r.t;                      // the interpolation space is the trial space
        } else {
            const int net = desc.interp_nelem[k] > 0 ? desc.interp_nelem[k]
                            : desc.knots[k] ? int(breakpoints(r.t).size()) - 1 : desc.nelem[k];
            const int mult = desc.interp_mult[k] > 0 ? desc.interp_mult[k] : 1;
            if (net < 1 || net > 100000) { set_error("element counts must be >= 1"); return KL_EINVAL; }
            if (desc.interp_mult[k] < 0 || mult > r.pt + 1) {
                set_error("interp_mult must be in 1..interp degree + 1 (0 = 1)");
                return KL_EINVAL;
            }
            r.tt = uniform_knots(r.pt, net, mult);
        }
        r.n = int(r.t.size()) - r.p - 1;
        r.nt = int(r.tt.size()) - r.pt - 1;
        hs.p[k] = r.p; hs.pt[k] = r.pt;
        hs.ne[k] = int(breakpoints(r.t).size()) - 1;
        hs.net[k] = int(breakpoints(r.tt).size()) - 1;
        hs.n[k] = r.n; hs.nt[k] = r.nt;
        N *= r.n;
        Nt *= r.nt;
    }
    if (Nt > (int64_t(1) << 26) || N > (int64_t(1) << 26)) { set_error("problem too large"); return KL_EINVAL; }
    hs.N = N;
    hs.Nt = Nt;
    std::vector<double> g[3];
    std::vector<int> gside[3];
    for (int k = 0; k < d; ++k) {
        kl_status st = build_direction(D[k], hs.C[k], hs.E[k], hs.LT[k], g[k], gside[k]);
        if (st != KL_OK) return st;
    }
    hs.X.assign(size_t(Nt) * d, 0.0);
    hs.J.assign(size_t(Nt), 0.0);
    for (int64_t p = 0; p < Nt; ++p) {
        int64_t r = p;
        double u[3], x[3], det;
        int side[3] = {1, 1, 1};
        for (int k = 0; k < d; ++k) {
            u[k] = g[k][r % hs.nt[k]];
            side[k] = gside[k][r % hs.nt[k]];
            r /= hs.nt[k];
        }
        map_point(desc, d, u, side, x, det);
        if (!(det > 0.0) || !std::isfinite(det)) {
            std::ostringstream os;
            os << "det DF = " << det << " <= 0 at Greville point " << p;
            set_error(os.str());
            return KL_EDOMAIN;
        }
        for (int k = 0; k < d; ++k) hs.X[size_t(p) * d + k] = x[k];
        hs.J[size_t(p)] = std::sqrt(det);
    }
    return KL_OK;
}

}  // namespace kl

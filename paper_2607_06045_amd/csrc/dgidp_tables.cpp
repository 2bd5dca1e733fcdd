// Operator tables of the LGL-DGSEM (Sec. 2.1) and of the mortars (Sec. 2.2,
// App. A), built on the host in long double and uploaded once per degree N.
//
//  - LGL nodes: -1, 1 and the eigenvalues of the Jacobi matrix of the (1,1)
//    Jacobi weight (the roots of P_N'), polished by Newton; weights
//    2 / (N (N+1) P_N(x_i)^2).
//  - Derivative matrix of the LGL Lagrange basis in closed form.
//  - Sbar = 2 diag(w) D - Bbar, Bbar = diag(-1, 0, ..., 0, 1).
//  - Mortar interpolation by the barycentric Lagrange formula; L2 projection
//    from the two half faces by solving M P = B with the exact mass matrix M and
//    the exact mixed matrices B (Gauss-Legendre quadrature, Golub-Welsch nodes).
//  - Sparse mortar weights: overlap lengths of the LGL subcells of the large
//    face and of the two half faces (eq. local_weights, App. A).
#include <cmath>
#include <cstring>
#include <vector>

#include "dgidp_internal.h"

namespace dgidp {

namespace {

using ld = long double;

// eigenvalues of a small symmetric matrix by cyclic Jacobi rotations
std::vector<ld> sym_eig(std::vector<std::vector<ld>> A)
{
    const int m = (int)A.size();
    for (int sweep = 0; sweep < 100; ++sweep) {
        ld off = 0;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) off += A[i][j] * A[i][j];
        if (off < 1e-38L) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                if (std::fabs(A[p][q]) < 1e-40L) continue;
                const ld th = (A[q][q] - A[p][p]) / (2 * A[p][q]);
                const ld t = (th >= 0 ? 1 : -1) / (std::fabs(th) + std::sqrt(th * th + 1));
                const ld c = 1 / std::sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const ld akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const ld apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    std::vector<ld> ev(m);
    for (int i = 0; i < m; ++i) ev[i] = A[i][i];
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j)
            if (ev[j] < ev[i]) std::swap(ev[i], ev[j]);
    return ev;
}

// P_N(x) and P_N'(x)
void legendre(int N, ld x, ld& p, ld& dp)
{
    ld pm = 1, pc = x;
    if (N == 0) {
        p = 1;
        dp = 0;
        return;
    }
    for (int k = 1; k < N; ++k) {
        const ld pn = ((2 * k + 1) * x * pc - k * pm) / (k + 1);
        pm = pc;
        pc = pn;
    }
    p = pc;
    dp = N * (pm - x * pc) / (1 - x * x);  // valid for |x| < 1
}

void lgl(int N, std::vector<ld>& x, std::vector<ld>& w)
{
    const int n = N + 1;
    x.assign(n, 0);
    w.assign(n, 0);
    x[0] = -1;
    x[N] = 1;
    if (N >= 2) {
        // Jacobi matrix of the (1,1) weight: off-diagonal sqrt(k(k+2)/((2k+1)(2k+3)))
        const int m = N - 1;
        std::vector<std::vector<ld>> J(m, std::vector<ld>(m, 0));
        for (int k = 1; k < m; ++k) {
            const ld b = std::sqrt((ld)k * (k + 2) / ((ld)(2 * k + 1) * (2 * k + 3)));
            J[k - 1][k] = J[k][k - 1] = b;
        }
        std::vector<ld> ev = sym_eig(J);
        for (int i = 0; i < m; ++i) {
            ld s = ev[i];
            for (int it = 0; it < 20; ++it) {  // Newton on P_N'
                ld p, dp;
                legendre(N, s, p, dp);
                const ld d2 = (2 * s * dp - N * (N + 1) * p) / (1 - s * s);
                const ld ds = dp / d2;
                s -= ds;
                if (std::fabs(ds) < 1e-32L) break;
            }
            x[i + 1] = s;
        }
    }
    for (int i = 0; i < n; ++i) {
        ld p, dp;
        if (i == 0 || i == N) p = (i == 0 && (N % 2 == 1)) ? -1 : 1;
        else legendre(N, x[i], p, dp);
        w[i] = 2 / ((ld)N * (N + 1) * p * p);
    }
}

ld lagrange_bary(const std::vector<ld>& x, const std::vector<ld>& bw, int k, ld s)
{
    const int n = (int)x.size();
    for (int j = 0; j < n; ++j)
        if (s == x[j]) return j == k ? 1 : 0;
    ld num = 0, den = 0;
    for (int j = 0; j < n; ++j) {
        const ld t = bw[j] / (s - x[j]);
        den += t;
        if (j == k) num = t;
    }
    return num / den;
}

void gauss(int q, std::vector<ld>& x, std::vector<ld>& w)
{
    // Golub-Welsch for the Legendre weight: off-diagonal k / sqrt(4k^2 - 1);
    // weights 2 / ((1 - x^2) P_q'(x)^2)
    std::vector<std::vector<ld>> J(q, std::vector<ld>(q, 0));
    for (int k = 1; k < q; ++k) J[k - 1][k] = J[k][k - 1] = (ld)k / std::sqrt((ld)4 * k * k - 1);
    x = sym_eig(J);
    w.assign(q, 0);
    for (int i = 0; i < q; ++i) {
        ld s = x[i];
        for (int it = 0; it < 20; ++it) {
            ld p, dp;
            legendre(q, s, p, dp);
            const ld ds = p / dp;
            s -= ds;
            if (std::fabs(ds) < 1e-32L) break;
        }
        ld p, dp;
        legendre(q, s, p, dp);
        x[i] = s;
        w[i] = 2 / ((1 - s * s) * dp * dp);
    }
}

// solve A X = B (n x n, n x m) by Gaussian elimination with partial pivoting
void solve(std::vector<std::vector<ld>> A, std::vector<std::vector<ld>>& B)
{
    const int n = (int)A.size(), m = (int)B[0].size();
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
        std::swap(A[c], A[piv]);
        std::swap(B[c], B[piv]);
        for (int r = c + 1; r < n; ++r) {
            const ld f = A[r][c] / A[c][c];
            for (int k = c; k < n; ++k) A[r][k] -= f * A[c][k];
            for (int k = 0; k < m; ++k) B[r][k] -= f * B[c][k];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = 0; k < m; ++k) {
            ld s = B[c][k];
            for (int j = c + 1; j < n; ++j) s -= A[c][j] * B[j][k];
            B[c][k] = s / A[c][c];
        }
    }
}

template <int N>
void build(Tab<N>& t)
{
    constexpr int n = N + 1;
    std::memset(&t, 0, sizeof(t));
    std::vector<ld> x, w;
    lgl(N, x, w);
    // derivative matrix, closed form for LGL nodes
    std::vector<ld> PN(n);
    for (int i = 0; i < n; ++i) {
        ld p, dp;
        if (i == 0) p = (N % 2 == 1) ? -1 : 1;
        else if (i == N) p = 1;
        else legendre(N, x[i], p, dp);
        PN[i] = p;
    }
    ld D[n][n];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i != j) D[i][j] = PN[i] / (PN[j] * (x[i] - x[j]));
            else if (i == 0) D[i][j] = -(ld)N * (N + 1) / 4;
            else if (i == N) D[i][j] = (ld)N * (N + 1) / 4;
            else D[i][j] = 0;
        }
    for (int i = 0; i < n; ++i) {
        t.w[i] = (double)w[i];
        t.winv[i] = (double)(1 / w[i]);
        for (int j = 0; j < n; ++j) {
            ld s = 2 * w[i] * D[i][j];
            if (i == j && i == 0) s += 1;
            if (i == j && i == N) s -= 1;
            t.S[i][j] = (double)s;
        }
    }
    // barycentric weights
    std::vector<ld> bw(n);
    for (int j = 0; j < n; ++j) {
        ld p = 1;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= x[j] - x[k];
        bw[j] = 1 / p;
    }
    for (int h = 0; h < 2; ++h)
        for (int l = 0; l < n; ++l)
            for (int k = 0; k < n; ++k)
                t.I[h][l][k] = (double)lagrange_bary(x, bw, k, (x[l] + (h ? 1 : -1)) / 2);
    // L2 projection: M P^h = B^h
    std::vector<ld> gx, gw;
    gauss(n + 1, gx, gw);
    std::vector<std::vector<ld>> M(n, std::vector<ld>(n, 0));
    for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l)
            for (int q = 0; q < (int)gx.size(); ++q)
                M[k][l] += gw[q] * lagrange_bary(x, bw, k, gx[q]) * lagrange_bary(x, bw, l, gx[q]);
    for (int h = 0; h < 2; ++h) {
        std::vector<std::vector<ld>> B(n, std::vector<ld>(n, 0));
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < n; ++l)
                for (int q = 0; q < (int)gx.size(); ++q)
                    B[k][l] += 0.5L * gw[q] * lagrange_bary(x, bw, k, (gx[q] + (h ? 1 : -1)) / 2) *
                               lagrange_bary(x, bw, l, gx[q]);
        solve(M, B);
        for (int k = 0; k < n; ++k)
            for (int l = 0; l < n; ++l) t.P[h][k][l] = (double)B[k][l];
    }
    // sparse weights: overlap of the subcells [c_k, c_{k+1}] of the large face
    // with the half-face subcells [-1 + h + C_l / 2, -1 + h + C_{l+1} / 2]
    std::vector<ld> C(n + 1, 0);
    for (int k = 0; k < n; ++k) C[k + 1] = C[k] + w[k];
    for (int k = 0; k < n; ++k)
        for (int h = 0; h < 2; ++h)
            for (int l = 0; l < n; ++l) {
                const ld lo = std::max(-1 + C[k], -1 + h + C[l] / 2);
                const ld hi = std::min(-1 + C[k + 1], -1 + h + C[l + 1] / 2);
                t.Wt[k][h * n + l] = hi - lo > 1e-12L ? (double)(hi - lo) : 0.0;
            }
    for (int k = 0; k < n; ++k) {
        int c = 0;
        for (int j = 0; j < 2 * n; ++j) {
            t.lnz[k][j] = 0;
            if (t.Wt[k][j] != 0.0) t.lnz[k][c++] = j;
        }
        t.lnc[k] = c;
    }
    for (int h = 0; h < 2; ++h)
        for (int l = 0; l < n; ++l) {
            int c = 0;
            for (int k = 0; k < n; ++k) {
                t.snz[h][l][k] = 0;
                if (t.Wt[k][h * n + l] != 0.0) t.snz[h][l][c++] = k;
            }
            t.snc[h][l] = c;
        }
    // modal transform: V[a][i] = sqrt((2i+1)/2) P_i(x_a), Vinv = V^-1
    {
        std::vector<std::vector<ld>> V(n, std::vector<ld>(n, 0)), R(n, std::vector<ld>(n, 0));
        for (int a = 0; a < n; ++a) {
            ld pm = 1, pc = x[a];
            for (int i = 0; i < n; ++i) {
                const ld pi = i == 0 ? 1 : (i == 1 ? x[a] : pc);
                V[a][i] = std::sqrt((2 * i + 1) / 2.0L) * pi;
                if (i >= 1) {
                    const ld pn = ((2 * i + 1) * x[a] * pc - i * pm) / (i + 1);
                    pm = pc;
                    pc = pn;
                }
            }
            R[a][a] = 1;
        }
        solve(V, R);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < n; ++a) t.Vinv[i][a] = (double)R[i][a];
    }
    for (int i = 0; i < n; ++i) {
        t.wf[i] = (float)t.w[i];
        for (int j = 0; j < n; ++j) t.Sf[i][j] = (float)t.S[i][j];
    }
    for (int h = 0; h < 2; ++h)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                t.If[h][i][j] = (float)t.I[h][i][j];
                t.Pf[h][i][j] = (float)t.P[h][i][j];
            }
}

}  // namespace

int build_and_upload_tables(int N, std::vector<double>* nodes)
{
    if (N == 3) {
        Tab<3> t;
        build<3>(t);
        if (nodes) {
            std::vector<ld> x, w;
            lgl(3, x, w);
            nodes->assign(x.begin(), x.end());
        }
        return upload_tables(3, &t, sizeof(t));
    }
    if (N == 4) {
        Tab<4> t;
        build<4>(t);
        if (nodes) {
            std::vector<ld> x, w;
            lgl(4, x, w);
            nodes->assign(x.begin(), x.end());
        }
        return upload_tables(4, &t, sizeof(t));
    }
    return -1;
}

// host copy of the tables for tests of the table builder (flat doubles:
// w[n], S[n*n], I[2*n*n], P[2*n*n], Wt[n*2n], Vinv[n*n])
int host_tables(int N, double* out)
{
    auto dump = [&](auto& t, int n) {
        double* o = out;
        for (int i = 0; i < n; ++i) *o++ = t.w[i];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) *o++ = t.S[i][j];
        for (int h = 0; h < 2; ++h)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) *o++ = t.I[h][i][j];
        for (int h = 0; h < 2; ++h)
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) *o++ = t.P[h][i][j];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < 2 * n; ++j) *o++ = t.Wt[i][j];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) *o++ = t.Vinv[i][j];
    };
    if (N == 3) {
        Tab<3> t;
        build<3>(t);
        dump(t, 4);
        return 0;
    }
    if (N == 4) {
        Tab<4> t;
        build<4>(t);
        dump(t, 5);
        return 0;
    }
    return -1;
}

}  // namespace dgidp

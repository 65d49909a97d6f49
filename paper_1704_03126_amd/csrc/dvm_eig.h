// dvm_eig.h -- small dense eigenproblems on the host for deflated GMRES
// restarts (plain C++, no device code).
//
// A GMRES cycle of k Arnoldi steps leaves the (k+1) x k Hessenberg matrix
// Hb with A V_k = V_{k+1} Hb.  Deflated restarting (Morgan, SIAM J. Sci.
// Comput. 24 (2002) 20-37) keeps the harmonic Ritz vectors of the smallest
// harmonic Ritz values: the eigenvectors g of
//     M = H + h^2 f e_k^T,  H = Hb[0:k, 0:k],  h = Hb[k, k-1],  H^T f = e_k,
// together with the cycle's least-squares residual vector rho = c - Hb y.
// With P = orthonormal basis of [[G; 0], rho] the next cycle starts from
// V_{d+1} = V_{k+1} P and the (d+1) x d block P^T Hb P[0:k, 0:d]: for an
// invariant subspace of M the relation A V_d = V_{d+1} (P^T Hb P_d) holds
// exactly, because each harmonic residual Hb g - theta [g; 0] lies in the
// one-dimensional null space of Hb^T, which also holds rho.
//
// Steps: Householder reduction to Hessenberg form, Francis double-shift QR
// for the eigenvalues (Golub & Van Loan, Matrix Computations, Sec. 7.5),
// inverse iteration on the Hessenberg form in complex arithmetic for the
// selected eigenvectors, two passes of Gram-Schmidt for P.  Orders here are
// at most a few hundred.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace dvm_eig {

using cd = std::complex<double>;

// A (n x n, column-major) -> upper Hessenberg form Q^T A Q; with Q non-null
// the orthogonal Q (n x n, column-major) is accumulated.
inline void hessenberg(std::vector<double> &A, int n, std::vector<double> *Q = nullptr)
{
    std::vector<double> v(n);
    if (Q) {
        Q->assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            (*Q)[i + (size_t)i * n] = 1.0;
    }
    for (int k = 0; k + 2 < n; ++k) {
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i)
            alpha += A[i + (size_t)k * n] * A[i + (size_t)k * n];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0)
            continue;
        const double x0 = A[k + 1 + (size_t)k * n];
        const double s = x0 >= 0.0 ? -alpha : alpha;
        std::fill(v.begin(), v.end(), 0.0);
        v[k + 1] = x0 - s;
        for (int i = k + 2; i < n; ++i)
            v[i] = A[i + (size_t)k * n];
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i)
            vn += v[i] * v[i];
        if (vn == 0.0)
            continue;
        const double b = 2.0 / vn;
        for (int j = 0; j < n; ++j) {           // A <- (I - b v v^T) A
            double d = 0.0;
            for (int i = k + 1; i < n; ++i)
                d += v[i] * A[i + (size_t)j * n];
            d *= b;
            for (int i = k + 1; i < n; ++i)
                A[i + (size_t)j * n] -= d * v[i];
        }
        for (int i = 0; i < n; ++i) {           // A <- A (I - b v v^T)
            double d = 0.0;
            for (int j = k + 1; j < n; ++j)
                d += A[i + (size_t)j * n] * v[j];
            d *= b;
            for (int j = k + 1; j < n; ++j)
                A[i + (size_t)j * n] -= d * v[j];
        }
        if (Q)
            for (int i = 0; i < n; ++i) {       // Q <- Q (I - b v v^T)
                double d = 0.0;
                for (int j = k + 1; j < n; ++j)
                    d += (*Q)[i + (size_t)j * n] * v[j];
                d *= b;
                for (int j = k + 1; j < n; ++j)
                    (*Q)[i + (size_t)j * n] -= d * v[j];
            }
        for (int i = k + 2; i < n; ++i)
            A[i + (size_t)k * n] = 0.0;
    }
}

// Householder vector of (x, y[, z]): (I - beta v v^T) applied to it leaves
// only its first component.  n = 2 or 3.
inline void house(const double *x, int n, double *v, double &beta)
{
    double nrm = 0.0;
    for (int i = 0; i < n; ++i)
        nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i)
        v[i] = x[i];
    if (nrm == 0.0) {
        beta = 0.0;
        return;
    }
    v[0] += x[0] >= 0.0 ? nrm : -nrm;
    double vn = 0.0;
    for (int i = 0; i < n; ++i)
        vn += v[i] * v[i];
    beta = vn > 0.0 ? 2.0 / vn : 0.0;
}

// Eigenvalues of the upper Hessenberg H (n x n, column-major; destroyed).
// Returns false when the QR iteration does not converge.
inline bool hessenberg_eigenvalues(std::vector<double> &H, int n, std::vector<cd> &ev)
{
    ev.clear();
    auto h = [&](int i, int j) -> double & { return H[i + (size_t)j * n]; };
    double anorm = 0.0;
    for (double a : H)
        anorm = std::max(anorm, std::fabs(a));
    if (anorm == 0.0) {
        ev.assign(n, cd(0.0, 0.0));
        return true;
    }
    const double eps = 2.2204460492503131e-16;
    int hi = n - 1, its = 0, total = 0;
    while (hi >= 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
            if (s == 0.0)
                s = anorm;
            if (std::fabs(h(l, l - 1)) <= eps * s) {
                h(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            ev.push_back(cd(h(hi, hi), 0.0));
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {
            const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const double m = 0.5 * (a + d), disc = 0.25 * (a - d) * (a - d) + b * c;
            if (disc >= 0.0) {
                const double r = std::sqrt(disc);
                const double e1 = m + (m >= 0.0 ? r : -r);
                const double e2 = e1 != 0.0 ? (a * d - b * c) / e1 : m - (m >= 0.0 ? r : -r);
                ev.push_back(cd(e1, 0.0));
                ev.push_back(cd(e2, 0.0));
            } else {
                const double r = std::sqrt(-disc);
                ev.push_back(cd(m, r));
                ev.push_back(cd(m, -r));
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (++total > 100 * n)
            return false;
        ++its;
        // shifts: the eigenvalues of the trailing 2 x 2 block (sum s,
        // product t); an ad hoc pair now and then breaks a cycle
        double s, t;
        if (its % 10 == 0) {
            const double w = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        } else {
            s = h(hi - 1, hi - 1) + h(hi, hi);
            t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
        }
        // Francis double-shift step on rows and columns l..hi
        double x[3];
        x[0] = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
        x[1] = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
        x[2] = h(l + 1, l) * h(l + 2, l + 1);
        for (int k = l; k <= hi - 2; ++k) {
            double v[3], beta;
            house(x, 3, v, beta);
            const int q = std::max(l, k - 1);
            for (int j = q; j <= hi; ++j) {
                const double d = beta * (v[0] * h(k, j) + v[1] * h(k + 1, j) + v[2] * h(k + 2, j));
                h(k, j) -= d * v[0];
                h(k + 1, j) -= d * v[1];
                h(k + 2, j) -= d * v[2];
            }
            const int r = std::min(k + 3, hi);
            for (int i = l; i <= r; ++i) {
                const double d = beta * (h(i, k) * v[0] + h(i, k + 1) * v[1] + h(i, k + 2) * v[2]);
                h(i, k) -= d * v[0];
                h(i, k + 1) -= d * v[1];
                h(i, k + 2) -= d * v[2];
            }
            x[0] = h(k + 1, k);
            x[1] = h(k + 2, k);
            if (k < hi - 2)
                x[2] = h(k + 3, k);
        }
        {
            double v[2], beta;
            house(x, 2, v, beta);
            for (int j = std::max(l, hi - 2); j <= hi; ++j) {
                const double d = beta * (v[0] * h(hi - 1, j) + v[1] * h(hi, j));
                h(hi - 1, j) -= d * v[0];
                h(hi, j) -= d * v[1];
            }
            for (int i = l; i <= hi; ++i) {
                const double d = beta * (h(i, hi - 1) * v[0] + h(i, hi) * v[1]);
                h(i, hi - 1) -= d * v[0];
                h(i, hi) -= d * v[1];
            }
        }
    }
    return true;
}

// An eigenvector z of the upper Hessenberg H (n x n, column-major) for the
// eigenvalue estimate theta: three steps of inverse iteration, each a solve
// with H - theta I by Gaussian elimination with partial pivoting between
// neighbouring rows (O(n^2) for a Hessenberg matrix), in complex
// arithmetic.  Returns false on failure.
inline bool hess_eigenvector(const std::vector<double> &H, int n, cd theta, std::vector<cd> &z)
{
    double anorm = 0.0;
    for (double a : H)
        anorm = std::max(anorm, std::fabs(a));
    const double tiny = std::max(anorm, 1e-300) * 1e-14;
    std::vector<cd> B((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            B[i + (size_t)j * n] = cd(H[i + (size_t)j * n], 0.0) - (i == j ? theta : cd(0.0, 0.0));
    std::vector<cd> mult(n, cd(0.0, 0.0));
    std::vector<char> swp(n, 0);
    for (int k = 0; k + 1 < n; ++k) {           // B = L U, L bidiagonal with row swaps
        if (std::abs(B[k + 1 + (size_t)k * n]) > std::abs(B[k + (size_t)k * n])) {
            swp[k] = 1;
            for (int j = k; j < n; ++j)
                std::swap(B[k + (size_t)j * n], B[k + 1 + (size_t)j * n]);
        }
        if (std::abs(B[k + (size_t)k * n]) < tiny)
            B[k + (size_t)k * n] = tiny;
        const cd f = B[k + 1 + (size_t)k * n] / B[k + (size_t)k * n];
        mult[k] = f;
        B[k + 1 + (size_t)k * n] = 0.0;
        if (f != cd(0.0, 0.0))
            for (int j = k + 1; j < n; ++j)
                B[k + 1 + (size_t)j * n] -= f * B[k + (size_t)j * n];
    }
    if (std::abs(B[(n - 1) + (size_t)(n - 1) * n]) < tiny)
        B[(n - 1) + (size_t)(n - 1) * n] = tiny;
    z.assign(n, cd(1.0, 0.0));
    for (int i = 0; i < n; ++i)                 // deterministic start vector
        z[i] = cd(1.0 + 0.01 * (i % 7), 0.003 * (i % 5));
    for (int pass = 0; pass < 3; ++pass) {
        for (int k = 0; k + 1 < n; ++k) {
            if (swp[k])
                std::swap(z[k], z[k + 1]);
            z[k + 1] -= mult[k] * z[k];
        }
        for (int i = n - 1; i >= 0; --i) {
            cd a = z[i];
            for (int j = i + 1; j < n; ++j)
                a -= B[i + (size_t)j * n] * z[j];
            z[i] = a / B[i + (size_t)i * n];
        }
        double nrm = 0.0;
        for (const cd &a : z)
            nrm += std::norm(a);
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm))
            return false;
        for (cd &a : z)
            a /= nrm;
    }
    return true;
}

// Householder QR of the m x n (m >= n) column-major A: Q (m x m) and the
// upper triangular R (m x n, zero below the diagonal), A = Q R.
inline void qr_small(const std::vector<double> &A, int m, int n, std::vector<double> &Q, std::vector<double> &R)
{
    R = A;
    Q.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
        Q[i + (size_t)i * m] = 1.0;
    std::vector<double> v(m);
    for (int k = 0; k < n && k + 1 < m; ++k) {
        double alpha = 0.0;
        for (int i = k; i < m; ++i)
            alpha += R[i + (size_t)k * m] * R[i + (size_t)k * m];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0)
            continue;
        const double x0 = R[k + (size_t)k * m];
        const double s = x0 >= 0.0 ? -alpha : alpha;
        std::fill(v.begin(), v.end(), 0.0);
        v[k] = x0 - s;
        for (int i = k + 1; i < m; ++i)
            v[i] = R[i + (size_t)k * m];
        double vn = 0.0;
        for (int i = k; i < m; ++i)
            vn += v[i] * v[i];
        if (vn == 0.0)
            continue;
        const double b = 2.0 / vn;
        for (int j = 0; j < n; ++j) {
            double d = 0.0;
            for (int i = k; i < m; ++i)
                d += v[i] * R[i + (size_t)j * m];
            d *= b;
            for (int i = k; i < m; ++i)
                R[i + (size_t)j * m] -= d * v[i];
        }
        for (int i = 0; i < m; ++i) {
            double d = 0.0;
            for (int j = k; j < m; ++j)
                d += Q[i + (size_t)j * m] * v[j];
            d *= b;
            for (int j = k; j < m; ++j)
                Q[i + (size_t)j * m] -= d * v[j];
        }
        for (int i = k + 1; i < m; ++i)
            R[i + (size_t)k * m] = 0.0;
    }
}

// Deflated restart of one GMRES cycle.
//   Hb   (k+1) x k, column-major with leading dimension ld (>= k+1)
//   rho  the cycle's least-squares residual vector (k+1 entries)
//   want the number of harmonic Ritz vectors to keep (a complex pair is
//        kept whole, so the result may hold want + 1)
// On success returns d > 0 and fills P ((k+1) x (d+1), column-major, ld k+1:
// orthonormal columns, the first d with a zero last entry) and Hn ((d+1) x d,
// ld d+1) = P^T Hb P[0:k, 0:d].  Returns 0 when no deflation is possible.
inline int deflate(const std::vector<double> &Hb, int ld, int k, const std::vector<double> &rho, int want,
                   std::vector<double> &P, std::vector<double> &Hn)
{
    if (k < 2 || want < 1 || want >= k)
        return 0;
    const double hk = Hb[k + (size_t)(k - 1) * ld];
    // f = H^{-T} e_k by Gaussian elimination with partial pivoting on H^T
    std::vector<double> T((size_t)k * k), f(k, 0.0);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i)
            T[i + (size_t)j * k] = Hb[j + (size_t)i * ld];
    f[k - 1] = 1.0;
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int i = c + 1; i < k; ++i)
            if (std::fabs(T[i + (size_t)c * k]) > std::fabs(T[p + (size_t)c * k]))
                p = i;
        if (T[p + (size_t)c * k] == 0.0)
            return 0;
        if (p != c) {
            for (int j = 0; j < k; ++j)
                std::swap(T[c + (size_t)j * k], T[p + (size_t)j * k]);
            std::swap(f[c], f[p]);
        }
        for (int i = c + 1; i < k; ++i) {
            const double m = T[i + (size_t)c * k] / T[c + (size_t)c * k];
            if (m == 0.0)
                continue;
            for (int j = c; j < k; ++j)
                T[i + (size_t)j * k] -= m * T[c + (size_t)j * k];
            f[i] -= m * f[c];
        }
    }
    for (int i = k - 1; i >= 0; --i) {
        double a = f[i];
        for (int j = i + 1; j < k; ++j)
            a -= T[i + (size_t)j * k] * f[j];
        f[i] = a / T[i + (size_t)i * k];
    }
    std::vector<double> M((size_t)k * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i)
            M[i + (size_t)j * k] = Hb[i + (size_t)j * ld] + (j == k - 1 ? hk * hk * f[i] : 0.0);
    for (double a : M)
        if (!std::isfinite(a))
            return 0;
    std::vector<double> Hh = M, Qh;
    hessenberg(Hh, k, &Qh);
    std::vector<double> Hw = Hh;
    std::vector<cd> ev;
    if (!hessenberg_eigenvalues(Hw, k, ev) || (int)ev.size() != k)
        return 0;
    std::vector<int> order(k);
    for (int i = 0; i < k; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(ev[a]) < std::abs(ev[b]); });
    // columns of [G; 0]: real eigenvectors, real and imaginary parts of one
    // of each complex pair
    std::vector<std::vector<double>> cols;
    std::vector<char> used(k, 0);
    const double cplx_tol = 1e-10;
    for (int oi = 0; oi < k && (int)cols.size() < want; ++oi) {
        const int i = order[oi];
        if (used[i])
            continue;
        used[i] = 1;
        const cd th = ev[i];
        const bool cplx = std::fabs(th.imag()) > cplx_tol * std::max(std::abs(th), 1e-300);
        if (cplx) {
            int mate = -1;                      // its conjugate
            double best = INFINITY;
            for (int j = 0; j < k; ++j)
                if (!used[j] && std::abs(ev[j] - std::conj(th)) < best) {
                    best = std::abs(ev[j] - std::conj(th));
                    mate = j;
                }
            if (mate >= 0)
                used[mate] = 1;
            if ((int)cols.size() + 2 > k - 1)
                break;
        }
        std::vector<cd> z;
        if (!hess_eigenvector(Hh, k, th, z))
            return 0;
        std::vector<double> re(k + 1, 0.0), im(k + 1, 0.0);
        for (int r = 0; r < k; ++r) {           // g = Qh z
            cd a(0.0, 0.0);
            for (int j = 0; j < k; ++j)
                a += Qh[r + (size_t)j * k] * z[j];
            re[r] = a.real();
            im[r] = a.imag();
        }
        if (cplx) {
            cols.push_back(re);
            cols.push_back(im);
        } else {
            // a real eigenvalue's vector is real up to a complex phase
            double nr = 0.0, ni = 0.0;
            for (int r = 0; r < k; ++r) {
                nr += re[r] * re[r];
                ni += im[r] * im[r];
            }
            cols.push_back(nr >= ni ? re : im);
        }
    }
    // orthonormal columns: [G; 0] first, then rho; a column that adds less
    // than 1e-10 of its length is dropped (rho never is)
    std::vector<std::vector<double>> Q;
    auto orth = [&](std::vector<double> v) -> bool {
        double n0 = 0.0;
        for (double a : v)
            n0 += a * a;
        n0 = std::sqrt(n0);
        if (!(n0 > 0.0))
            return false;
        for (int pass = 0; pass < 2; ++pass)
            for (const auto &q : Q) {
                double d = 0.0;
                for (int r = 0; r <= k; ++r)
                    d += q[r] * v[r];
                for (int r = 0; r <= k; ++r)
                    v[r] -= d * q[r];
            }
        double n1 = 0.0;
        for (double a : v)
            n1 += a * a;
        n1 = std::sqrt(n1);
        if (!(n1 > 1e-10 * n0))
            return false;
        for (double &a : v)
            a /= n1;
        Q.push_back(v);
        return true;
    };
    for (auto &cl : cols)
        orth(cl);
    const int d = (int)Q.size();
    if (d < 1 || !orth(rho))
        return 0;
    P.assign((size_t)(k + 1) * (d + 1), 0.0);
    for (int c = 0; c <= d; ++c)
        for (int r = 0; r <= k; ++r)
            P[r + (size_t)c * (k + 1)] = Q[c][r];
    // Hn = P^T Hb P[0:k, 0:d] (Hb may hold a dense leading block left by a
    // previous deflation, so every row is summed)
    std::vector<double> HP((size_t)(k + 1) * d, 0.0);
    for (int c = 0; c < d; ++c)
        for (int j = 0; j < k; ++j) {
            const double pj = P[j + (size_t)c * (k + 1)];
            if (pj != 0.0)
                for (int r = 0; r <= k; ++r)
                    HP[r + (size_t)c * (k + 1)] += Hb[r + (size_t)j * ld] * pj;
        }
    Hn.assign((size_t)(d + 1) * d, 0.0);
    for (int c = 0; c < d; ++c)
        for (int r2 = 0; r2 <= d; ++r2) {
            double a = 0.0;
            for (int r = 0; r <= k; ++r)
                a += P[r + (size_t)r2 * (k + 1)] * HP[r + (size_t)c * (k + 1)];
            Hn[r2 + (size_t)c * (d + 1)] = a;
        }
    // the relation Hb P_d = P Hn holds to rounding only for an invariant
    // subspace; eigenvectors too ill-conditioned for it mean a plain restart
    double hmax = 0.0, err = 0.0;
    for (int j = 0; j < k; ++j)
        for (int r = 0; r <= k; ++r)
            hmax = std::max(hmax, std::fabs(Hb[r + (size_t)j * ld]));
    for (int c = 0; c < d; ++c)
        for (int r = 0; r <= k; ++r) {
            double a = HP[r + (size_t)c * (k + 1)];
            for (int r2 = 0; r2 <= d; ++r2)
                a -= P[r + (size_t)r2 * (k + 1)] * Hn[r2 + (size_t)c * (d + 1)];
            err = std::max(err, std::fabs(a));
        }
    if (!(err <= 1e-8 * hmax))
        return 0;
    return d;
}

}  // namespace dvm_eig

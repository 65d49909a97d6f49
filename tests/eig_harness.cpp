// C entry points over the host eigen-helpers of the deflated GMRES restart,
// for the CPU tests (compiled by the test with the host compiler).
#include "../paper_1704_03126_amd/csrc/dvm_eig.h"

extern "C" int eig_values(const double *A, int n, double *re, double *im)
{
    std::vector<double> H(A, A + (size_t)n * n);
    dvm_eig::hessenberg(H, n);
    std::vector<dvm_eig::cd> ev;
    if (!dvm_eig::hessenberg_eigenvalues(H, n, ev) || (int)ev.size() != n)
        return -1;
    for (int i = 0; i < n; ++i) {
        re[i] = ev[i].real();
        im[i] = ev[i].imag();
    }
    return 0;
}

extern "C" int eig_deflate(const double *Hb, int k, const double *rho, int want, double *P, double *Hn)
{
    std::vector<double> H(Hb, Hb + (size_t)(k + 1) * k), r(rho, rho + k + 1), Pv, Hv;
    const int d = dvm_eig::deflate(H, k + 1, k, r, want, Pv, Hv);
    for (size_t i = 0; i < Pv.size(); ++i)
        P[i] = Pv[i];
    for (size_t i = 0; i < Hv.size(); ++i)
        Hn[i] = Hv[i];
    return d;
}

extern "C" void eig_qr(const double *A, int m, int n, double *Q, double *R)
{
    std::vector<double> a(A, A + (size_t)m * n), q, r;
    dvm_eig::qr_small(a, m, n, q, r);
    for (size_t i = 0; i < q.size(); ++i)
        Q[i] = q[i];
    for (size_t i = 0; i < r.size(); ++i)
        R[i] = r[i];
}

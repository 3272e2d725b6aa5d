// The CPU oracle (oracle/vlct_ref.c, unchanged) compiled as C++ with a
// complex-step scalar in place of double: a state U + i h dU carried through
// the oracle's steps gives the directional derivative J dU = Im(out) / h to
// machine precision (no differencing), with every branch taken on the real
// part, i.e. at the unperturbed state.  Squire & Trapp's complex step: the
// functions the oracle uses continue analytically (sqrt on the principal
// branch), |x| is x times the sign of its real part, comparisons compare real
// parts.  OpenMP is not used here (the pragmas compile to nothing).
//
// Test infrastructure only.  Built by tests/complex_step/cs.py into a
// temporary directory, together with a copy of the oracle's header without
// its C-linkage block.
#include <complex>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

struct CS {
    std::complex<double> z;
    CS(double x = 0.0) : z(x, 0.0) {}
    CS(int x) : z((double)x, 0.0) {}
    CS(unsigned x) : z((double)x, 0.0) {}
    CS(long x) : z((double)x, 0.0) {}
    CS(long long x) : z((double)x, 0.0) {}
    CS(unsigned long x) : z((double)x, 0.0) {}
    explicit CS(std::complex<double> w) : z(w) {}
    CS &operator+=(const CS &b) { z += b.z; return *this; }
    CS &operator-=(const CS &b) { z -= b.z; return *this; }
    CS &operator*=(const CS &b) { z *= b.z; return *this; }
    CS &operator/=(const CS &b) { z /= b.z; return *this; }
};
inline CS operator+(const CS &a, const CS &b) { return CS(a.z + b.z); }
inline CS operator-(const CS &a, const CS &b) { return CS(a.z - b.z); }
inline CS operator*(const CS &a, const CS &b) { return CS(a.z * b.z); }
inline CS operator/(const CS &a, const CS &b) { return CS(a.z / b.z); }
inline CS operator-(const CS &a) { return CS(-a.z); }
inline CS operator+(const CS &a) { return a; }
inline bool operator<(const CS &a, const CS &b) { return a.z.real() < b.z.real(); }
inline bool operator>(const CS &a, const CS &b) { return a.z.real() > b.z.real(); }
inline bool operator<=(const CS &a, const CS &b) { return a.z.real() <= b.z.real(); }
inline bool operator>=(const CS &a, const CS &b) { return a.z.real() >= b.z.real(); }
inline bool operator==(const CS &a, const CS &b) { return a.z.real() == b.z.real(); }
inline bool operator!=(const CS &a, const CS &b) { return a.z.real() != b.z.real(); }
inline CS sqrt(const CS &a) { return CS(std::sqrt(a.z)); }
inline CS fabs(const CS &a) { return a.z.real() < 0.0 ? CS(-a.z) : a; }
inline bool isfinite(const CS &a) { return std::isfinite(a.z.real()) && std::isfinite(a.z.imag()); }
extern "C" void omp_set_num_threads(int) {}

#define double CS
#include "vlct_ref.c"
#undef double

extern "C" int cs_run(const int32_t n[3], const double dl[3], double gamma, double cfl,
                      int32_t recon, const int32_t bc[3], const double *const re[8],
                      const double *const im[8], const double *dts, int nsteps,
                      double *const out_re[8], double *const out_im[8], uint32_t *status)
{
    vref_grid g;
    g.nx = n[0]; g.ny = n[1]; g.nz = n[2];
    g.dx = CS(dl[0]); g.dy = CS(dl[1]); g.dz = CS(dl[2]);
    g.gamma = CS(gamma); g.cfl = CS(cfl); g.recon = recon;
    for (int d = 0; d < 3; ++d) g.bc[d] = bc[d];
    const size_t nx = n[0], ny = n[1], nz = n[2];
    const size_t len[8] = {nx * ny * nz, nx * ny * nz, nx * ny * nz, nx * ny * nz, nx * ny * nz,
                           (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)};
    CS *a[8], *b[8];
    for (int f = 0; f < 8; ++f) {
        a[f] = new CS[len[f]];
        b[f] = new CS[len[f]];
        for (size_t q = 0; q < len[f]; ++q) a[f][q] = CS(std::complex<double>(re[f][q], im[f][q]));
    }
    uint32_t st = 0;
    int rc = 0;
    for (int s = 0; s < nsteps && !rc; ++s) {
        CS next;
        uint32_t st1 = 0;
        rc = vref_step(&g, a, b, CS(dts[s]), &next, &st1, 0);
        st |= st1;
        for (int f = 0; f < 8; ++f) std::swap(a[f], b[f]);
    }
    for (int f = 0; f < 8; ++f) {
        for (size_t q = 0; q < len[f]; ++q) {
            out_re[f][q] = a[f][q].z.real();
            out_im[f][q] = a[f][q].z.imag();
        }
        delete[] a[f];
        delete[] b[f];
    }
    *status = st;
    return rc;
}

// Host build of the device physics header (mhd_physics.hpp) for unit checks of
// the GPU's HLLD solver: reads lines "rho u v w p by bz  rho u v w p by bz  bn
// gamma" from stdin and prints the 7 sweep-frame flux components and the CT
// upwind indicator of hlld(W_L, W_R, B_n).  Square roots are the library's
// (VLCT_HOST_COUNT), everything else is the header's own arithmetic.  Test
// infrastructure only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#define __host__
#define __device__
#define __forceinline__ inline
#define VLCT_HOST_COUNT
#include "mhd_physics.hpp"

int main()
{
    double a[16];
    while (true) {
        for (int q = 0; q < 16; ++q)
            if (scanf("%lf", &a[q]) != 1) return 0;
        const vlct::W7 L{a[0], a[1], a[2], a[3], a[4], a[5], a[6]};
        const vlct::W7 R{a[7], a[8], a[9], a[10], a[11], a[12], a[13]};
        double f[7], upw;
        vlct::hlld(L, R, a[14], a[15], 1.0 / (a[15] - 1.0), f, upw);
        for (int q = 0; q < 7; ++q) printf("%.17g ", f[q]);
        printf("%.17g\n", upw);
    }
}

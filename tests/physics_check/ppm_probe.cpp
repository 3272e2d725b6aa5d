// Host build of the device physics header (mhd_physics.hpp) for unit checks of
// the GPU's characteristic PPM reconstruction: reads lines of 37 numbers (the
// primitives rho u v w p by bz of cells i-2 .. i+2, then bn and gamma) from
// stdin and prints the 7 primitives of the face at i-1/2 followed by those of
// the face at i+1/2, as ppmc<true> (mode 1 on the command line selects
// ppmc<false>, the primitive-variable form) computes them.  Square roots are
// the library's (VLCT_HOST_COUNT), everything else is the header's own
// arithmetic.  Test infrastructure only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#define __host__
#define __device__
#define __forceinline__ inline
#define VLCT_HOST_COUNT
#include "mhd_physics.hpp"

int main(int argc, char **argv)
{
    const bool prim = argc > 1 && atoi(argv[1]) == 1;
    double a[37];
    while (true) {
        for (int q = 0; q < 37; ++q)
            if (scanf("%lf", &a[q]) != 1) return 0;
        vlct::W7 w[5];
        for (int s = 0; s < 5; ++s) {
            const double *c = a + 7 * s;
            w[s] = vlct::W7{c[0], c[1], c[2], c[3], c[4], c[5], c[6]};
        }
        vlct::W7 fm, fp;
        if (prim)
            vlct::ppmc<false>(w[0], w[1], w[2], w[3], w[4], a[35], a[36], fm, fp);
        else
            vlct::ppmc<true>(w[0], w[1], w[2], w[3], w[4], a[35], a[36], fm, fp);
        const double o[14] = {fm.d, fm.u, fm.v, fm.w, fm.p, fm.by, fm.bz,
                              fp.d, fp.u, fp.v, fp.w, fp.p, fp.by, fp.bz};
        for (int q = 0; q < 14; ++q) printf("%.17g%c", o[q], q == 13 ? '\n' : ' ');
    }
}

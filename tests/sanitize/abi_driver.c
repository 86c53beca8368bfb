/* Host-side entry points of libbs.so that need no device, over valid and
 * invalid parameters, for a host-only build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure only). */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "bs.h"

int main(void) {
    int bad = 0, n = 0;
    const double tols[] = {1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12, 1e-14, 0.0, -1.0, 0.7};
    const int grids[] = {16, 20, 32, 48, 64, 96, 128, 256, 512, 1024, 8, 18, 2048};
    for (unsigned it = 0; it < sizeof tols / sizeof *tols; it++)
        for (unsigned ig = 0; ig < sizeof grids / sizeof *grids; ig++)
            for (int prec = 0; prec < 3; prec++)
                for (int ns = -1; ns < 5; ns++)
                    for (int order = 2; order <= 6; order += 2) {
                        bs_params p, r;
                        memset(&p, 0, sizeof p);
                        p.L = 6.283185307179586;
                        p.a = 1e-6;
                        p.delta = 0.25;
                        p.tol = tols[it];
                        p.grid_n = grids[ig];
                        p.precision = prec;
                        p.ns_mode = ns;
                        p.spline_order = order;
                        p.fft_mode = (int)((it + ig) % 4);
                        p.Q = (int)(ig % 6);
                        p.local_frac = (ig % 3) * 0.05;
                        const int rc = bs_resolve_params(&p, &r);
                        n++;
                        if (rc == BS_OK && !(r.alpha > 0 && r.rcut > 0 && r.K > 0 && r.w >= 4))
                            bad++;
                        if (rc != BS_OK && !bs_last_error(NULL)[0]) bad++;
                    }
    double lo = 0, hi = 0;
    int nb = 0;
    bs_ns_error_bins(&lo, &hi, &nb);
    if (!(lo > 0 && hi > lo && nb > 0) || bs_mlp_nparams() != 9091) bad++;
    if (bs_resolve_params(NULL, NULL) == BS_OK) bad++;
    if (bs_destroy(NULL) != BS_OK) bad++;
    if (!bs_last_error(NULL)) bad++;
    printf("%d parameter sets, %d inconsistent\n", n, bad);
    return bad != 0;
}

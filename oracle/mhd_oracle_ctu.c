/* mhd_oracle_ctu.c -- CTU scheme of the FP64 oracle (test infrastructure only). */
#include "mhd_oracle.h"

int or_ctu_step_impl(int nx, int ny, int nz, double dx, double gam, int recon, int solver,
                     const double* U, const double* B, double dt, double* Uo, double* Bo,
                     int* nfallback) {
  (void)nx; (void)ny; (void)nz; (void)dx; (void)gam; (void)recon; (void)solver;
  (void)U; (void)B; (void)dt; (void)Uo; (void)Bo; (void)nfallback;
  return -1;
}

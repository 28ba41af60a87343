/* mhd_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure
 * only; see mhd_oracle.c).  Not included by, and shares nothing with, the
 * GPU library. */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#include <stddef.h>

enum { OR_VL = 0, OR_CTU = 1 };
enum { OR_PLM = 0, OR_PPM = 1, OR_FIRST_ORDER = 2, OR_PLM_UNLIMITED = 3, OR_PPM_UNLIMITED = 4 };
enum { OR_ROE = 0, OR_HLLE = 1, OR_HLLD = 2 };

int or_version(void);
void or_set_threads(int n);
int or_get_threads(void);
void or_prim_to_cons(int nx, int ny, int nz, double gam, const double* W5, const double* B, double* U);
void or_cons_to_prim(int nx, int ny, int nz, double gam, const double* U, const double* B, double* W8);
double or_cfl_dt(int nx, int ny, int nz, double dx, double gam, double courant, const double* U, const double* B);
void or_divb(int nx, int ny, int nz, double dx, const double* B, double* div);
void or_sums(int nx, int ny, int nz, double dx, const double* U, const double* B, double out[7]);
int or_step(int nx, int ny, int nz, double dx, double gam, int scheme, int recon, int solver,
            const double* U, const double* B, double dt, double* Uo, double* Bo, int* nfallback);
/* or_step that also returns the fluxes and edge EMFs of the full update (the
 * ones the paper's correction operation needs): Fout [3][5][N] (mass,
 * momentum x/y/z, energy through the lower d-face of each cell), Eout [3][N]
 * (Ex, Ey, Ez on the edge at the cell's lower corner); either may be NULL */
int or_step_ex(int nx, int ny, int nz, double dx, double gam, int scheme, int recon, int solver,
               const double* U, const double* B, double dt, double* Uo, double* Bo, int* nfallback,
               double* Fout, double* Eout);

void or_phys_flux(double gam, const double* w, double bn, double* f);
void or_w_to_u(double gam, const double* w, double bn, double* u);
void or_u_to_w(double gam, const double* u, double bn, double* w);
double or_fast_speed(double gam, const double* w, double bn);
int or_riemann(int solver, double gam, const double* wl, const double* wr, double bn, double* f);
void or_roe_eigen(double gam, const double* wl, const double* wr, double bn, double* lam, double* R);
void or_ppm_edges(const double* q, double* qL, double* qR);

/* shared between the oracle's own translation units */
void or__primitives(int nx, int ny, int nz, double dx, double gam, const double* U, const double* B, double* W);
int or__riemann(int solver, const double* wl, const double* wr, double bn, double gam, double* f);
void or__edge_emfs(int nx, int ny, int nz, double dx, const double* const F[3], const double* W, double* E);
void or__apply_update(int nx, int ny, int nz, double dx, const double* U, const double* B,
                      const double* const F[3], const double* E, double tau, double* Uo, double* Bo);
void or__copy_final(size_t N, const double* const F[3], const double* E, double* Fout, double* Eout);

#endif

// Host build of the single-thread small dense routines and the tolerance
// controller that the GPU kernels run; exported with C linkage so the CPU
// tests can compare them with NumPy and with the oracle.
#include "../../paper_2312_02891_amd/csrc/controller.h"
#include "../../paper_2312_02891_amd/csrc/small.h"

extern "C" {
int st_chol(const double* G, double* S, int n, double fl) { return lradi::chol_upper_reg(G, S, n, fl); }
void st_trinv(const double* S, double* X, int n) { lradi::tri_inv_upper(S, X, n); }
void st_jacobi(double* A, double* Q, int n) { lradi::jacobi_eig(A, Q, n); }
double st_lmax(const double* G, int n) { return lradi::lambda_max_sym(G, n); }
double st_lmax_ms16(const double* G, int n) { return lradi::lambda_max_sym_ms<16>(G, n); }
double st_lmax_ms64(const double* G, int n) { return lradi::lambda_max_sym_ms<64>(G, n); }
double st_lmax_prod(const double* A, const double* B, int n) { return lradi::lambda_max_prod(A, B, n); }
double st_lmax_prod_chol(const double* A, const double* B, int n) { return lradi::lambda_max_prod_chol(A, B, n); }
void st_house(double* M, double* Q, int n) { lradi::householder_2nxn(M, Q, n); }
void st_tol(int selection, int backlook, int paper_abs, int k, double nw, double nt, double u,
            double v, double eps, int kmax, double xi, double dmin, double dmax, double dfix,
            double rho, int balance, double* dA, double* dB) {
  lradi::CtlParams p;
  p.eps = eps; p.delta_min = dmin; p.delta_max = dmax; p.xi = xi; p.delta_fixed = dfix;
  p.rho = rho; p.kmax = kmax; p.selection = selection; p.backlook = backlook;
  p.paper_abs = paper_abs; p.balance = balance;
  lradi::ctl_tolerances(p, k, nw, nt, u, v, dA, dB);
}
void st_gap(double* u, double* v, double g, double nz, double ny, double rA, double rB) {
  lradi::ctl_update_gap(u, v, g, nz, ny, rA, rB);
}
}

// Launchers of the bilinear (Q1) and biquadratic (Q2) finite-element
// operators (kern_fe.hip).  Each applies to the handle's uniform square mesh
// (2D, kappa = 1); the finite-difference launchers call them when the handle
// was created with AAO_DISC_Q1 or AAO_DISC_Q2.
#pragma once

#include "aao_internal.h"

namespace aao {

// Chebyshev steps of the mass solve inside S-tilde (Sec. 5 uses 20)
constexpr int FE_CHEB_STEPS = 20;

// y = A x (or A^T x), the all-at-once operator of eq. (2.4) with M and K of the elements
template <class TX>
hipError_t fe_apply_A(const aao_problem* h, const TX* x, double* y, bool transpose, hipStream_t st);
// w = (I_s (x) M + tau A (x) K) z on B instances (strides sz, sw)
template <class T>
hipError_t fe_theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                          hipStream_t st);
// out = v - tau sum_{l < i} tab.L[i][l] K z_l on B instances
template <class T>
hipError_t fe_rana_rhs(const aao_problem* h, const Tab& tab, int i, const T* v, int64_t sv, const T* z, int64_t sz,
                       T* out, int64_t so, int B, hipStream_t st);
// t_v = r_v - Psi1 z_V (nt + 1 blocks)
template <class T>
hipError_t fe_schur_coupling(const aao_problem* h, const double* r, const T* zV, T* t, hipStream_t st);
// out_{b,i} = K zin_b, every stage i, B instances
template <class T>
hipError_t fe_schur_kz(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B,
                       hipStream_t st);
// t <- Chebyshev approximation of M^{-1} t on B blocks, in place (ya, yb: scratch, B N values each)
template <class T>
hipError_t fe_mass_solve(const aao_problem* h, T* t, T* ya, T* yb, int B, hipStream_t st);
// Level 0 of the multigrid for Q2 elements (M + a K, the shift a = tau L_ii
// scaled as the V-cycle asks): a weighted Jacobi sweep xin -> xout (from
// zero: omega D^{-1} b), and the residual r = b - (M + a K) x; B instances
template <class T>
hipError_t fe_q2_smooth(const aao_problem* h, double a, const T* xin, int64_t sxin, T* xout, int64_t sxout,
                        const T* b, int64_t sb, double omega, bool zero_init, int B, hipStream_t st);
template <class T>
hipError_t fe_q2_residual(const aao_problem* h, double a, const T* x, int64_t sx, const T* b, int64_t sb, T* r,
                          int64_t sr, int B, hipStream_t st);
// rhs = [M u0; 0; M f]
hipError_t fe_assemble_rhs(const aao_problem* h, const double* f, const double* u0, double* rhs, hipStream_t st);

}  // namespace aao

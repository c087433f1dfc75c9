// Batched Krylov building blocks: segmented multi-dot products, multi-AXPYs,
// the Givens least-squares update of GMRES, and the stage-level operators
// (Theta_hat, Rana coupling, S-tilde sweep pieces).
#pragma once

#include "aao_internal.h"

namespace aao {

// Per-instance scalar block of the batched inner GMRES (doubles).
struct InnerSlots {
  static constexpr int BETA = 0, ACTIVE = 1, M = 2, STRIDE = 512;
  static constexpr int G = 8;                    // g[KMAX+1]
  static constexpr int CS = G + 16;              // cs[KMAX]
  static constexpr int SN = CS + 16;             // sn[KMAX]
  static constexpr int H1 = SN + 16;             // h1[DOTS_PER_PASS]
  static constexpr int H2 = H1 + 16;             // h2[DOTS_PER_PASS]
  static constexpr int WW = H2 + 16;             // <w, w>
  static constexpr int INV = WW + 1;             // 1 / h_{j+1,j} (0 when inactive)
  static constexpr int Y = INV + 7;              // y[KMAX]
  static constexpr int R = Y + 16;               // R[(KMAX+1) * KMAX], column j at R + j*(KMAX+1)
};

// Number of workgroups per segment for the segmented reductions.
int seg_blocks(int64_t L, int B);

// partial[(inst*nblk + blk)*(DOTS_PER_PASS+1) + d] = block sums of
// <w_inst, V_d,inst> for d < nd, and of <w_inst, w_inst> in slot
// DOTS_PER_PASS when `self`.  V_d,inst = V + d*vstride + inst*sv.
template <class TW, class TV>
hipError_t seg_dots(const TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, bool self,
                    int64_t L, int B, double* partial, int nblk, hipStream_t st);

// out[inst*ostride + ooff + d] = sum over blocks (fixed order) for d < nd;
// the self product goes to out[inst*ostride + self_off] when self_off >= 0.
hipError_t seg_finish(const double* partial, int nblk, int nd, int self_off, int B, double* out,
                      int64_t ostride, int ooff, hipStream_t st);

// w_inst += scale * sum_{d<nd} coef[inst*cstride + coff + d] * V_d,inst
template <class TW, class TV>
hipError_t seg_axpy(TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, const double* coef,
                    int64_t cstride, int coff, double scale, int64_t L, int B, hipStream_t st);

// out_inst = sum_{d<nd} coef[...] * V_d,inst   (overwrite)
template <class TO, class TV>
hipError_t seg_combine(TO* out, int64_t so, const TV* V, int64_t vstride, int64_t sv, int nd,
                       const double* coef, int64_t cstride, int coff, int64_t L, int B, hipStream_t st);

// out_inst = in_inst * sc[inst*cstride + coff]
template <class TI, class TO>
hipError_t seg_scale(const TI* in, int64_t si, TO* out, int64_t so, const double* sc, int64_t cstride,
                     int coff, int64_t L, int B, hipStream_t st);

// Inner GMRES scalar updates (one thread per instance).
hipError_t inner_init(double* slots, int B, hipStream_t st);
hipError_t inner_givens(double* slots, int B, int j, hipStream_t st);
hipError_t inner_backsolve(double* slots, int B, int k, hipStream_t st);

// w = Theta_hat z for each instance (z, w: s*N per instance); tab gives A
// (tau A (x) K mixing).
template <class T>
hipError_t theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                       hipStream_t st);

// rhs = v_i - tau sum_{l<i} Lc[i][l] K z_l for each instance (stage i).
template <class T>
hipError_t rana_rhs(const aao_problem* h, const double* Lc, int i, const T* v, int64_t sv, const T* z,
                    int64_t sz, T* out, int64_t so, int B, hipStream_t st);

// S-tilde sweep pieces (see solver.hip).
template <class T>
hipError_t schur_coupling(const aao_problem* h, const double* r, T* z, hipStream_t st);
template <class T>
hipError_t schur_kz(const aao_problem* h, const T* zv, T* out, hipStream_t st);
template <class T>
hipError_t schur_update(const aao_problem* h, const T* tnext, const T* zcur, const T* y, T* znext,
                        hipStream_t st);

// Transposed-preconditioner pieces.
template <class T>
hipError_t schurT_bw(const aao_problem* h, const T* zv, T* out, hipStream_t st);
template <class T>
hipError_t schurT_update(const aao_problem* h, const double* rprev, const T* znext, const T* y, T* zcur,
                         hipStream_t st);
template <class T>
hipError_t thetaT_rhs(const aao_problem* h, const double* r, const T* z, T* out, hipStream_t st);

}  // namespace aao

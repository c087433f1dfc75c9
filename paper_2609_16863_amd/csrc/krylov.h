// Batched Krylov building blocks: a fused Gram-Schmidt pass (optional AXPY,
// multi-dot products finished by the last workgroup, GMRES scalar updates),
// basis updates and combinations, and the stage-level operators (Theta_hat,
// Rana coupling, S-tilde sweep pieces).
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

enum { GS_POST_NONE = 0, GS_POST_INIT = 1, GS_POST_GIVENS = 2 };

// One fused Gram-Schmidt pass over B instances of length L (see k_gs).
struct GSArgs {
  int64_t L;          // segment length
  int64_t sw;         // instance stride of w
  int64_t vstride;    // distance between consecutive basis vectors
  int64_t sv;         // instance stride of the basis
  int nd;             // basis vectors in this pass (<= DOTS_PER_PASS)
  int axpy, dots, self;
  double* slots;      // per-instance scalars
  int64_t sstride;
  int ca, od, os;     // coefficient / dot / self offsets in the slots
  double* partial;    // nblk * (DOTS_PER_PASS + 1) doubles per instance
  unsigned* counters; // one zero-initialised ticket per instance
  int nblk;
  int post, j;
};

// Number of workgroups per segment for the segmented reductions.
int seg_blocks(int64_t L, int B);

template <class TW, class TV>
hipError_t gs_pass(TW* w, const TV* V, const GSArgs& a, int B, hipStream_t st);

// out = (w - sum_{d<nd} slots[ca+d] V_d) * (cs >= 0 ? slots[cs] : alpha)
template <class TW, class TV, class TO>
hipError_t basis_update(const TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, TO* out,
                        int64_t so, const double* slots, int64_t sstride, int ca, int cs, double alpha, int64_t L,
                        int B, hipStream_t st);

// out (+)= sum_{d<nd} y_d Z_d, y from the GMRES least-squares solve (solve)
// or from slots[cy + d].
template <class TO, class TV>
hipError_t combine(TO* out, int64_t so, const TV* Z, int64_t vstride, int64_t sv, int nd, const double* slots,
                   int64_t sstride, int cy, bool solve, bool accumulate, int64_t L, int B, hipStream_t st);

// w = Theta_hat z for each instance (z, w: s*N per instance); tab gives A.
template <class T>
hipError_t theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                       hipStream_t st);

// rhs = v_i - tau sum_{l<i} Lc[i][l] K z_l for each instance (stage i).
template <class T>
hipError_t rana_rhs(const aao_problem* h, const double* Lc, int i, const T* v, int64_t sv, const T* z,
                    int64_t sz, T* out, int64_t so, int B, hipStream_t st);

// S-tilde sweep pieces.
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

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

enum { GS_POST_NONE = 0, GS_POST_INIT = 1, GS_POST_GIVENS = 2, GS_POST_MR = 3 };

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
  unsigned* counters; // [0]: inner GMRES iterations done, [1]: inner solves begun (or null)
  int nblk;
  int post, j;
  double rtol;        // GS_POST_GIVENS: stop an instance once |g_{j+1}| <= rtol * beta (0: never)
  int one_pass;       // GS_POST_GIVENS after a single classical pass: the column is this pass' dots
                      // alone (no first-pass h1 to add)
};

// Number of workgroups per segment for the segmented reductions.
int seg_blocks(int64_t L, int B);

template <class TW, class TV>
hipError_t gs_pass(TW* w, const TV* V, const GSArgs& a, int B, hipStream_t st);

// One instance (the outer solve): slots[od + d] = <w, V_d> and
// slots[od + nd + d] = <vlast, V_d> for d < nd (nd <= DOTS_PER_PASS / 2),
// slots[os] = <w, w> when a.self.
hipError_t gs_gram(const double* w, const double* V, const double* vlast, const GSArgs& a, hipStream_t st);

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

// S-tilde pieces (eq. (3.3)).  t = r_v - Psi1 z_V for every step (nt + 1
// blocks of N; zV: the nt stage blocks of s N).
template <class T>
hipError_t schur_coupling(const aao_problem* h, const double* r, const T* zV, T* t, hipStream_t st);

// Batched S-tilde steps: instance b reads base + b * stride of every operand
// (strides in elements, may be negative).
// out_b = (e (x) K) zin_b  (s blocks of N per instance)
template <class T>
hipError_t schur_kz(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B, hipStream_t st);
// out_b = t_b + zin_b - tab.tau sum_i b_i y_{b,i}
template <class T, class TT>
hipError_t phi_update(const aao_problem* h, const Tab& tab, const TT* t, int64_t stt, const T* zin, int64_t szin,
                      const T* y, int64_t sy, T* out, int64_t sout, int B, hipStream_t st);
// out_b = (b (x) I) zin_b
template <class T>
hipError_t schurT_bw(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B, hipStream_t st);
// out_b = t_b + zin_b - tau K sum_i y_{b,i}
template <class T, class TT>
hipError_t phiT_update(const aao_problem* h, double tau, const TT* t, int64_t stt, const T* zin, int64_t szin,
                       const T* y, int64_t sy, T* out, int64_t sout, int B, hipStream_t st);
// MGRIT coarse step at one C-point: znew = g + Phi_c(eprev) (eprev may be
// null: Phi_c(0) = 0), eout = znew - zC, zC = znew.
template <class T>
hipError_t mgrit_coarse(const aao_problem* h, const Tab& tabc, bool transpose, const T* g, const T* eprev,
                        const T* y, T* zC, T* eout, hipStream_t st);

// Transposed-preconditioner right-hand side of Theta-tilde^T.
template <class T>
hipError_t thetaT_rhs(const aao_problem* h, const double* r, const T* z, T* out, hipStream_t st);

}  // namespace aao

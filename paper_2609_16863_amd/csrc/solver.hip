// Host orchestration of the preconditioner P-tilde (eqs. (3.2)-(3.3)) and of
// the outer FP64 FGMRES (Algorithm 1 with P_L = I, restarted).
//
// P-tilde^{-1} r by block back-substitution:
//   z_V = Theta-tilde^{-1} r_V         one batched inner GMRES over all steps
//   t_v = r_v - Psi1 z_V              t_{v,n+1} = r_{v,n+1} + tau sum_i b_i z_{V,n,i}
//   z_v = S-tilde^{-1} t_v            forward sweep in time:
//        z_{v,n+1} = t_{v,n+1} + z_{v,n} - tau (b^T (x) I) Theta-tilde^{-1} (e (x) K) z_{v,n}
// Theta-tilde^{-1} is k right-preconditioned GMRES iterations from zero on the
// stage matrix Theta_hat = I_s (x) I + tau A (x) K, preconditioned by Rana's
// block-lower-triangular I_s (x) I + tau L (x) K (A_RK = L U, U unit upper)
// whose diagonal blocks I + tau L_ii K get `cycles` multigrid V-cycles.
//
// The transpose P-tilde^{-T} (used by the adjoint solve) is the same
// back-substitution on the transposed blocks: the S-tilde^T sweep runs
// backwards in time first, then Theta-tilde^{-T} (GMRES on Theta_hat^T with
// Rana's factor of A_RK^T).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "aao_internal.h"
#include "fe.h"
#include "krylov.h"
#include "mg.h"

namespace aao {

#define TRY(...)                         \
  do {                                   \
    hipError_t e_ = (__VA_ARGS__);       \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

namespace {

using S = InnerSlots;

template <class TI, class TM>
class Precond {
 public:
  // One S-tilde step size: the multigrid of Rana's diagonal blocks, the
  // tableau (transposed for P-tilde^T) with its step tau, and the Crout
  // factor the coupling uses.  `fine` steps tau; the MGRIT coarse stepper
  // steps mgrit_cf tau (its factor and shifts scaled by mgrit_cf).
  struct Stepper {
    Multigrid<TI, TM> mg;
    Tab tab;
    double Lc[SMAX * SMAX];
    int k;   // inner GMRES iterations of this step size
    Stepper(aao_problem* h, bool transpose, double scale, int cinv_set, int kin)
        : mg(h, h->stream, scaled(h, transpose, scale).data(), cinv_set), k(kin) {
      const std::vector<double> L = scaled(h, transpose, scale);
      for (int q = 0; q < SMAX * SMAX; ++q) Lc[q] = q < (int)L.size() ? L[q] : 0.0;
      tab = h->tab;
      tab.tau = h->tau * scale;
      if (transpose) {
        const int s = h->s;
        for (int i = 0; i < s; ++i)
          for (int j = 0; j < s; ++j) tab.A[i * s + j] = h->tab.A[j * s + i];
      }
    }
    static std::vector<double> scaled(const aao_problem* h, bool transpose, double scale) {
      const double* L = transpose ? h->LT : h->tab.L;
      std::vector<double> out(L, L + h->s * h->s);
      for (double& v : out) v *= scale;
      return out;
    }
  };

  Precond(aao_problem* h, bool transpose, int k, int cycles)
      : h_(h), st_(h->stream), transpose_(transpose), k_(k), cycles_(cycles),
        fine_(h, transpose, 1.0, transpose ? 1 : 0, k) {
    if (h->opts.schur == AAO_SCHUR_MGRIT)
      coarse_.reset(new Stepper(h, transpose, (double)h->opts.mgrit_cf, transpose ? 3 : 2,
                                h->opts.mgrit_coarse_k > 0 ? h->opts.mgrit_coarse_k : k));
    char* ws = h->ws;
    inV_ = reinterpret_cast<TI*>(ws + h->plan.inV);
    inZ_ = reinterpret_cast<TI*>(ws + h->plan.inZ);
    inW_ = reinterpret_cast<TI*>(ws + h->plan.inW);
    inX_ = reinterpret_cast<TI*>(ws + h->plan.inX);
    rana_ = reinterpret_cast<TI*>(ws + h->plan.rana);
    srhs_ = reinterpret_cast<TI*>(ws + h->plan.schurRhs);
    sy_ = reinterpret_cast<TI*>(ws + h->plan.schurY);
    mt_ = reinterpret_cast<TI*>(ws + h->plan.mgritT);
    mg_g_ = reinterpret_cast<TI*>(ws + h->plan.mgritG);
    mg_e_ = reinterpret_cast<TI*>(ws + h->plan.mgritE);
    fea_ = reinterpret_cast<TI*>(ws + h->plan.feA);
    feb_ = reinterpret_cast<TI*>(ws + h->plan.feB);
    partial_ = reinterpret_cast<double*>(ws + h->plan.partial);
    slots_ = reinterpret_cast<double*>(ws + h->plan.dscal);
    counters_ = reinterpret_cast<unsigned*>(ws + h->plan.counters);
  }

  GSArgs gs_args(int64_t L, int B) const {
    GSArgs a{};
    a.L = L;
    a.slots = slots_;
    a.sstride = S::STRIDE;
    a.partial = partial_;
    a.counters = counters_;
    a.nblk = seg_blocks(L, B);
    a.rtol = h_->opts.inner_tol;
    return a;
  }

  // out_b = Theta-tilde^{-1} rhs_b for B instances (rhs, out: s*N each),
  // with the step size of `sp`.
  template <class TR>
  hipError_t inner(Stepper& sp, const TR* rhs, int64_t srhs, TI* out, int64_t sout, int B, int kin = 0) {
    const int64_t N = h_->N, sN = (int64_t)h_->s * N, UV = h_->UV;
    // beta = ||rhs||, first basis vector rhs / beta
    GSArgs a0 = gs_args(sN, B);
    a0.sw = srhs;
    a0.self = 1;
    a0.os = S::WW;
    a0.post = GS_POST_INIT;
    TRY(gs_pass<TR, TI>(const_cast<TR*>(rhs), inV_, a0, B, st_));
    TRY(basis_update<TR, TI, TI>(rhs, srhs, inV_, UV, sN, 0, inV_, sN, slots_, S::STRIDE, 0, S::INV, 0.0, sN, B,
                                 st_));
    const int kk = kin > 0 ? kin : sp.k;
    if constexpr (std::is_same<TR, TI>::value) {
      if (kk == 1) return mr_inner(sp, rhs, srhs, out, sout, B);
    }
    for (int j = 0; j < kk; ++j) {
      TI* Vj = inV_ + (int64_t)j * UV;
      TI* Zj = inZ_ + (int64_t)j * UV;
      // Rana: forward substitution over the stages
      for (int i = 0; i < h_->s; ++i) {
        typename Multigrid<TI, TM>::Coupling cpl;
        cpl.z = Zj;
        cpl.sz = sN;
        cpl.zstride = N;
        cpl.nz = i;
        cpl.Lc = sp.Lc;
        cpl.out = rana_;
        cpl.so = N;
        TRY(sp.mg.solve(i, BVec<TI>{Zj + (int64_t)i * N, sN}, BVec<const TI>{Vj + (int64_t)i * N, sN}, B,
                        cycles_, i > 0 ? &cpl : nullptr));
      }
      TRY(theta_apply<TI>(h_, sp.tab, Zj, sN, inW_, sN, B, st_));
      // classical Gram-Schmidt, twice: h1 = V^T w; w -= V h1, h2 = V^T w,
      // <w,w> and the Givens update in the second pass' finishing workgroup
      const int nd = j + 1;
      GSArgs a1 = gs_args(sN, B);
      a1.sw = sN;
      a1.vstride = UV;
      a1.sv = sN;
      a1.nd = nd;
      a1.dots = 1;
      a1.od = S::H1;
      if (h_->opts.inner_orth == AAO_ORTH_CGS1) {
        // one classical pass: h = V^T w and <w,w> together, h_{j+1,j} from
        // their difference, then v_{j+1} = (w - V h) / h_{j+1,j}
        a1.od = S::H2;
        a1.self = 1;
        a1.os = S::WW;
        a1.post = GS_POST_GIVENS;
        a1.j = j;
        a1.one_pass = 1;
        TRY(gs_pass<TI, TI>(inW_, inV_, a1, B, st_));
        if (j + 1 < kk)
          TRY(basis_update<TI, TI, TI>(inW_, sN, inV_, UV, sN, nd, inV_ + (int64_t)(j + 1) * UV, sN, slots_,
                                       S::STRIDE, S::H2, S::INV, 0.0, sN, B, st_));
        continue;
      }
      TRY(gs_pass<TI, TI>(inW_, inV_, a1, B, st_));
      GSArgs a2 = a1;
      a2.axpy = 1;
      a2.ca = S::H1;
      a2.od = S::H2;
      a2.self = 1;
      a2.os = S::WW;
      a2.post = GS_POST_GIVENS;
      a2.j = j;
      TRY(gs_pass<TI, TI>(inW_, inV_, a2, B, st_));
      if (j + 1 < kk)
        TRY(basis_update<TI, TI, TI>(inW_, sN, inV_, UV, sN, nd, inV_ + (int64_t)(j + 1) * UV, sN, slots_,
                                     S::STRIDE, S::H2, S::INV, 0.0, sN, B, st_));
    }
    TRY(combine<TI, TI>(out, sout, inZ_, UV, sN, kk, slots_, S::STRIDE, 0, true, false, sN, B, st_));
    return hipSuccess;
  }

  // GMRES(1) from zero as the minimal-residual step it is: z = Rana(rhs),
  // w = Theta_hat z, out = (<w, rhs> / <w, w>) z -- the result of the
  // general loop above for one iteration, with one reduction instead of the
  // normalization, two Gram-Schmidt passes and the Givens update.
  hipError_t mr_inner(Stepper& sp, const TI* rhs, int64_t srhs, TI* out, int64_t sout, int B) {
    const int64_t N = h_->N, sN = (int64_t)h_->s * N, UV = h_->UV;
    TI* Z0 = inZ_;
    for (int i = 0; i < h_->s; ++i) {
      typename Multigrid<TI, TM>::Coupling cpl;
      cpl.z = Z0;
      cpl.sz = sN;
      cpl.zstride = N;
      cpl.nz = i;
      cpl.Lc = sp.Lc;
      cpl.out = rana_;
      cpl.so = N;
      TRY(sp.mg.solve(i, BVec<TI>{Z0 + (int64_t)i * N, sN}, BVec<const TI>{rhs + (int64_t)i * N, srhs}, B, cycles_,
                      i > 0 ? &cpl : nullptr));
    }
    TRY(theta_apply<TI>(h_, sp.tab, Z0, sN, inW_, sN, B, st_));
    GSArgs a = gs_args(sN, B);
    a.sw = sN;
    a.vstride = UV;
    a.sv = srhs;
    a.nd = 1;
    a.dots = 1;
    a.od = S::H1;
    a.self = 1;
    a.os = S::WW;
    a.post = GS_POST_MR;
    TRY(gs_pass<TI, TI>(inW_, rhs, a, B, st_));
    return combine<TI, TI>(out, sout, Z0, UV, sN, 1, slots_, S::STRIDE, S::Y, false, false, sN, B, st_);
  }

  // out_b = t_b + Phi(zin_b) for B instances, Phi the S-tilde step of `sp`:
  // forward  Phi(z) = z - tau (b^T (x) I) Theta-tilde^{-1} (e (x) K) z,
  // transposed Phi^T(z) = z - tau K sum_i [Theta-tilde^{-T} (b (x) z)]_i.
  // Strides (elements) may be negative; t is TI or FP64.
  template <class TT>
  hipError_t phi_step(Stepper& sp, const TT* t, int64_t stt, const TI* zin, int64_t szin, TI* out, int64_t sout,
                      int B) {
    const int64_t sN = (int64_t)h_->s * h_->N;
    const int ks = h_->opts.schur_k;   // S-tilde's own inner count (0: the stepper's)
    if (!transpose_) {
      TRY(schur_kz<TI>(h_, zin, szin, srhs_, sN, B, st_));
      TRY(inner<TI>(sp, srhs_, sN, sy_, sN, B, ks));
      return phi_update<TI, TT>(h_, sp.tab, t, stt, zin, szin, sy_, sN, out, sout, B, st_);
    }
    TRY(schurT_bw<TI>(h_, zin, szin, srhs_, sN, B, st_));
    TRY(inner<TI>(sp, srhs_, sN, sy_, sN, B, ks));
    return phiT_update<TI, TT>(h_, sp.tab.tau, t, stt, zin, szin, sy_, sN, out, sout, B, st_);
  }

  // z_m, m = 0..nt, of the recurrence z_0 = t_0, z_{m+1} = t_{m+1} + Phi(z_m)
  // with block m of z at z0 + m dz and of t at t0 + m dt (dz, dt = +-N):
  // forward substitution, or two-level MGRIT with C-points every c steps
  // (K = ceil(nt / c) intervals; initial guess t_0 at the first C-point and
  // 0 at the others).  One MGRIT iteration: F-relaxation of every interval
  // at once (step j of all intervals is one batched S-tilde step), FCF's
  // C-relaxation when asked, the fine propagation g_k into every C-point,
  // then the sequential coarse sweep z_kc <- g_k + Phi_c(e_{k-1}) with
  // e_k = (new - old) z_kc and Phi_c the step of size c tau.  A final
  // F-relaxation fills the F-points.
  template <class TT>
  hipError_t schur_solve(const TT* t0, int64_t dt, TI* z0, int64_t dz) {
    const int nt = h_->nt;
    const int64_t N = h_->N;
    const bool in_place = (const void*)t0 == (const void*)z0;   // t already sits in z
    if (!coarse_) {
      if (!in_place) TRY(launch_copy_cast<TI, TT>(z0, t0, N, st_));
      for (int m = 0; m < nt; ++m)
        TRY(phi_step<TT>(fine_, t0 + (m + 1) * dt, 0, z0 + m * dz, 0, z0 + (m + 1) * dz, 0, 1));
      return hipSuccess;
    }
    const int c = h_->opts.mgrit_cf;
    const int K = (nt + c - 1) / c;
    const int64_t cz = (int64_t)c * dz, ct = (int64_t)c * dt;
    // C-points: z_{kc}, k = 0..K-1, kept in place in z; initial guess t_0, 0, ...
    if (!in_place) TRY(launch_copy_cast<TI, TT>(z0, t0, N, st_));
    for (int k = 1; k < K; ++k) TRY(launch_fill<TI>(z0 + k * cz, TI(0), N, st_));
    // F-relaxation: step j of every interval k < Kj at once
    auto f_relax = [&](bool last) -> hipError_t {
      for (int j = 1; j < c && j <= nt; ++j) {
        const int Kj = std::min(K, (nt - j) / c + 1);   // intervals k with kc + j <= nt
        TRY(phi_step<TT>(fine_, t0 + j * dt, ct, z0 + (j - 1) * dz, cz, z0 + j * dz, cz, Kj));
      }
      // a last interval of full length ends at nt, one step past the others
      if (last && nt % c == 0) TRY(phi_step<TT>(fine_, t0 + nt * dt, 0, z0 + (nt - 1) * dz, 0, z0 + nt * dz, 0, 1));
      return hipSuccess;
    };
    for (int it = 0; it < h_->opts.mgrit_iters && K > 1; ++it) {
      TRY(f_relax(false));
      if (h_->opts.mgrit_fcf) {
        // C-relaxation: z_{kc} = t_{kc} + Phi(z_{kc-1}), k = 1..K-1, then F again
        TRY(phi_step<TT>(fine_, t0 + ct, ct, z0 + (c - 1) * dz, cz, z0 + cz, cz, K - 1));
        TRY(f_relax(false));
      }
      // g_k = t_{kc} + Phi(z_{kc-1}) for k = 1..K-1 (g block k at mg_g_ + k N)
      TRY(phi_step<TT>(fine_, t0 + ct, ct, z0 + (c - 1) * dz, cz, mg_g_ + N, N, K - 1));
      // coarse sweep: z_{kc} <- g_k + Phi_c(e_{k-1}), e_k = new - old
      const int64_t sN = (int64_t)h_->s * N;
      for (int k = 1; k < K; ++k) {
        const TI* eprev = nullptr;
        if (k >= 2) {
          eprev = mg_e_ + (k - 1) * N;
          if (!transpose_) TRY(schur_kz<TI>(h_, eprev, 0, srhs_, sN, 1, st_));
          else TRY(schurT_bw<TI>(h_, eprev, 0, srhs_, sN, 1, st_));
          TRY(inner<TI>(*coarse_, srhs_, sN, sy_, sN, 1));
        }
        TRY(mgrit_coarse<TI>(h_, coarse_->tab, transpose_, mg_g_ + k * N, eprev, sy_, z0 + k * cz, mg_e_ + k * N,
                             st_));
      }
    }
    return f_relax(true);
  }

  // z (TI, U values) = P-tilde^{-1} r (FP64) or its transpose, in two
  // phases.  Forward: phase 1 = Theta-tilde on every step and the coupling
  // t_v = r_v - Psi1 z_V, phase 2 = S-tilde^{-1} t_v.  Transposed: phase 1 =
  // the S-tilde^T solve backwards in time, phase 2 = Theta-tilde^T on every
  // step.
  hipError_t apply(const double* r, TI* z, int phase) {
    if (phase != 2) TRY(transpose_ ? schurT_phase(r, z) : theta_phase(r, z));
    if (phase != 1) TRY(transpose_ ? thetaT_phase(r, z) : schur_phase(r, z));
    return hipSuccess;
  }

  hipError_t theta_phase(const double* r, TI* z) {
    const int64_t N = h_->N, sN = (int64_t)h_->s * N;
    const int nt = h_->nt;
    TI* zV = z + (int64_t)(nt + 1) * N;
    const double* rV = r + (int64_t)(nt + 1) * N;
    TRY(inner<double>(fine_, rV, sN, zV, sN, nt));
    // t_v goes to z_v (substitution, which then works in place) or to the
    // separate t buffer (MGRIT)
    return schur_coupling<TI>(h_, r, zV, coarse_ ? mt_ : z, st_);
  }

  hipError_t schur_phase(const double* r, TI* z) {
    (void)r;
    TI* t = coarse_ ? mt_ : z;
    // finite elements: S-tilde = blockdiag(M) times the bidiagonal recurrence;
    // its block-diagonal mass solve first (Chebyshev, Sec. 5), in place
    if (h_->fe) TRY(fe_mass_solve<TI>(h_, t, fea_, feb_, h_->nt + 1, st_));
    return schur_solve<TI>(t, h_->N, z, h_->N);
  }

  // z_{v,nt} = r_{v,nt}, z_{v,n} = r_{v,n} + Phi^T(z_{v,n+1}): the forward
  // recurrence in the reversed time index m = nt - n.
  hipError_t schurT_phase(const double* r, TI* z) {
    const int64_t N = h_->N;
    const int nt = h_->nt;
    return schur_solve<double>(r + (int64_t)nt * N, -N, z + (int64_t)nt * N, -N);
  }

  hipError_t thetaT_phase(const double* r, TI* z) {
    const int64_t N = h_->N, sN = (int64_t)h_->s * N;
    const int nt = h_->nt;
    TI* zV = z + (int64_t)(nt + 1) * N;
    TRY(thetaT_rhs<TI>(h_, r, z, inX_, st_));
    return inner<TI>(fine_, inX_, sN, zV, sN, nt);
  }

 private:
  aao_problem* h_;
  hipStream_t st_;
  bool transpose_;
  int k_, cycles_;
  Stepper fine_;
  std::unique_ptr<Stepper> coarse_;
  TI *inV_, *inZ_, *inW_, *inX_, *rana_, *srhs_, *sy_, *mt_, *mg_g_, *mg_e_, *fea_, *feb_;
  double *partial_, *slots_;
  unsigned* counters_;
};

template <class TI, class TM>
hipError_t apply_P_typed(aao_problem* h, const double* r, TI* z, int k, int cycles, bool transpose, int phase) {
  Precond<TI, TM> P(h, transpose, k, cycles);
  return P.apply(r, z, phase);
}

// Dispatch on the handle's precision; z is TI-typed storage (double for FP64).
// phase: 1 or 2 for one phase of P-tilde, 0 for both.
hipError_t apply_P_any(aao_problem* h, const double* r, void* z, int k, int cycles, bool transpose, int phase) {
  switch (h->opts.precision) {
    case AAO_PREC_FP64: return apply_P_typed<double, double>(h, r, (double*)z, k, cycles, transpose, phase);
    case AAO_PREC_FP32: return apply_P_typed<float, float>(h, r, (float*)z, k, cycles, transpose, phase);
    case AAO_PREC_FP16: return apply_P_typed<float, __half>(h, r, (float*)z, k, cycles, transpose, phase);
    case AAO_PREC_FP16_ALL: return apply_P_typed<__half, __half>(h, r, (__half*)z, k, cycles, transpose, phase);
    default: return apply_P_typed<float, __hip_bfloat16>(h, r, (float*)z, k, cycles, transpose, phase);
  }
}

template <class TI, class TM>
hipError_t apply_mg_typed(aao_problem* h, bool transpose, int stage, int count, int cycles, const void* r, void* z) {
  Multigrid<TI, TM> mg(h, h->stream, transpose ? h->LT : h->tab.L);
  const int64_t N = h->N;
  return mg.solve(stage, BVec<TI>{static_cast<TI*>(z), N}, BVec<const TI>{static_cast<const TI*>(r), N}, count,
                  cycles);
}

// Apply P-tilde directly, or by replaying HIP graphs captured on the first
// call for this (transpose, k, cycles): one graph per phase, so that the
// phases can be timed apart.  The graphs read their input from and write
// their output to fixed workspace buffers; the copies in and out run on the
// handle's stream around the replays.
hipError_t precond_graph(aao_problem* h, int k, int cycles, bool transpose, int phase,
                         aao_problem::GraphEntry** out) {
  double* gin = reinterpret_cast<double*>(h->ws + h->plan.gIn);
  void* gout = h->ws + h->plan.gOut;
  aao_problem::GraphEntry* ent = nullptr;
  for (auto& g : h->graphs)
    if (g.transpose == transpose && g.k == k && g.cycles == cycles && g.phase == phase) ent = &g;
  if (!ent) {
    if (!h->capture_stream) TRY(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    hipStream_t saved = h->stream;
    h->stream = h->capture_stream;
    hipError_t e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      h->stream = saved;
      return e;
    }
    e = apply_P_any(h, gin, gout, k, cycles, transpose, phase);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(h->capture_stream, &graph);
    h->stream = saved;
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return e != hipSuccess ? e : e2;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return e;
    }
    h->graphs.push_back(aao_problem::GraphEntry{transpose, k, cycles, phase, graph, exec});
    ent = &h->graphs.back();
  }
  *out = ent;
  return hipSuccess;
}

// z = P-tilde^{-1} r.  With `timed`, the handle's phase events are recorded
// before phase 1, between the phases and after phase 2.
hipError_t precond_apply(aao_problem* h, const double* r, void* z, int k, int cycles, bool transpose, bool timed) {
  hipEvent_t* ev = h->phase_ev;
  if (!h->opts.use_graph || h->no_alloc) {
    if (timed) TRY(hipEventRecord(ev[0], h->stream));
    TRY(apply_P_any(h, r, z, k, cycles, transpose, 1));
    if (timed) TRY(hipEventRecord(ev[1], h->stream));
    TRY(apply_P_any(h, r, z, k, cycles, transpose, 2));
    if (timed) TRY(hipEventRecord(ev[2], h->stream));
    return hipSuccess;
  }
  const int64_t U = h->U;
  double* gin = reinterpret_cast<double*>(h->ws + h->plan.gIn);
  void* gout = h->ws + h->plan.gOut;
  // the entries live in a vector that capturing may grow: keep the handles
  aao_problem::GraphEntry* ent = nullptr;
  TRY(precond_graph(h, k, cycles, transpose, 1, &ent));
  const hipGraphExec_t x1 = ent->exec;
  TRY(precond_graph(h, k, cycles, transpose, 2, &ent));
  const hipGraphExec_t x2 = ent->exec;
  TRY(hipMemcpyAsync(gin, r, (size_t)U * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  if (timed) TRY(hipEventRecord(ev[0], h->stream));
  TRY(hipGraphLaunch(x1, h->stream));
  if (timed) TRY(hipEventRecord(ev[1], h->stream));
  TRY(hipGraphLaunch(x2, h->stream));
  if (timed) TRY(hipEventRecord(ev[2], h->stream));
  return hipMemcpyAsync(z, gout, (size_t)U * h->pi_bytes, hipMemcpyDeviceToDevice, h->stream);
}

// ---------------------------------------------------------------------------
// Outer FGMRES
// ---------------------------------------------------------------------------
template <class TI>
class Fgmres {
 public:
  Fgmres(aao_problem* h, bool transpose) : h_(h), st_(h->stream), transpose_(transpose) {
    char* ws = h->ws;
    V_ = reinterpret_cast<double*>(ws + h->plan.outV);
    Z_ = reinterpret_cast<TI*>(ws + h->plan.outZ);
    w_ = reinterpret_cast<double*>(ws + h->plan.outW);
    partial_ = reinterpret_cast<double*>(ws + h->plan.partial);
    oslots_ = reinterpret_cast<double*>(ws + h->plan.dscal) + (int64_t)(h->nt + 1) * S::STRIDE;
    counters_ = reinterpret_cast<unsigned*>(ws + h->plan.counters);
  }

  template <class TX>
  hipError_t op(const TX* x, double* y) {
    return transpose_ ? launch_apply_AT<TX>(h_, x, y, st_) : launch_apply_A<TX>(h_, x, y, st_);
  }

  GSArgs gs_args(int nd) const {
    GSArgs a{};
    a.L = h_->U;
    a.vstride = h_->U;
    a.nd = nd;
    a.slots = oslots_;
    a.partial = partial_;
    a.nblk = seg_blocks(h_->U, 1);
    return a;
  }

  // ||x||^2 of a U-vector, synchronous.
  hipError_t norm2(const double* x, double* out) {
    GSArgs a = gs_args(0);
    a.self = 1;
    a.os = 0;
    TRY(gs_pass<double, double>(const_cast<double*>(x), x, a, 1, st_));
    double* hp = h_->host_scalars();
    TRY(hipMemcpyAsync(hp, oslots_, sizeof(double), hipMemcpyDeviceToHost, st_));
    TRY(hipStreamSynchronize(st_));
    *out = hp[0];
    return hipSuccess;
  }

  // Classical Gram-Schmidt of w against V_0..V_{nd-1}, twice.  Leaves
  // w - V h1 in w, and on the host h1 + h2 (hcol), |h2|^2 and <w, w>.
  hipError_t orthogonalize(int nd, std::vector<double>& hcol, double& h2sq, double& ww) {
    if (h_->opts.outer_orth == AAO_ORTH_GRAM) return orthogonalize_gram(nd, hcol, h2sq, ww);
    const int64_t U = h_->U;
    const int H1 = 8, H2 = H1 + MMAX + 8, WW = H2 + MMAX + 8;
    for (int c0 = 0; c0 < nd; c0 += DOTS_PER_PASS) {
      GSArgs a = gs_args(std::min(DOTS_PER_PASS, nd - c0));
      a.dots = 1;
      a.od = H1 + c0;
      TRY(gs_pass<double, double>(w_, V_ + (int64_t)c0 * U, a, 1, st_));
    }
    if (nd <= DOTS_PER_PASS) {
      GSArgs a = gs_args(nd);
      a.axpy = 1;
      a.ca = H1;
      a.dots = 1;
      a.od = H2;
      a.self = 1;
      a.os = WW;
      TRY(gs_pass<double, double>(w_, V_, a, 1, st_));
    } else {
      for (int c0 = 0; c0 < nd; c0 += DOTS_PER_PASS) {
        GSArgs a = gs_args(std::min(DOTS_PER_PASS, nd - c0));
        a.axpy = 1;
        a.ca = H1 + c0;
        TRY(gs_pass<double, double>(w_, V_ + (int64_t)c0 * U, a, 1, st_));
      }
      for (int c0 = 0; c0 < nd; c0 += DOTS_PER_PASS) {
        const int cnt = std::min(DOTS_PER_PASS, nd - c0);
        GSArgs a = gs_args(cnt);
        a.dots = 1;
        a.od = H2 + c0;
        a.self = c0 + cnt >= nd;
        a.os = WW;
        TRY(gs_pass<double, double>(w_, V_ + (int64_t)c0 * U, a, 1, st_));
      }
    }
    double* hp = h_->host_scalars();
    TRY(hipMemcpyAsync(hp, oslots_ + H1, sizeof(double) * (size_t)(WW - H1 + 1), hipMemcpyDeviceToHost, st_));
    TRY(hipStreamSynchronize(st_));
    hcol.assign(nd, 0.0);
    h2sq = 0.0;
    for (int i = 0; i < nd; ++i) {
      const double a = hp[i], b = hp[(H2 - H1) + i];
      hcol[i] = a + b;
      h2sq += b * b;
    }
    ww = hp[WW - H1];
    return hipSuccess;
  }

  // Classical Gram-Schmidt twice, with the second pass taken from the Gram
  // matrix G = V^T V of the basis instead of a second sweep over it:
  // h1 = V^T w, h = h1 + V^T (w - V h1) = (2 I - G) h1 and
  // ||w - V h||^2 = <w,w> - 2 h^T h1 + h^T G h, in exact arithmetic the
  // two-pass result.  One sweep per iteration forms h1, <w,w> and the
  // newest basis vector's Gram column <V_d, v_{nd-1}> together; w itself is
  // left as it is, and h goes to the device slots (H2), where next_basis
  // and correct_and_norm take their coefficients from.  Returns h in hcol
  // and h2sq = <w,w> - ||w - V h||^2.
  hipError_t orthogonalize_gram(int nd, std::vector<double>& hcol, double& h2sq, double& ww) {
    const int64_t U = h_->U;
    const int H2 = 8 + MMAX + 8, WW = H2 + MMAX + 8, SCR = WW + 8;
    constexpr int CH = DOTS_PER_PASS / 2;
    const double* vlast = V_ + (int64_t)(nd - 1) * U;
    for (int c0 = 0; c0 < nd; c0 += CH) {
      const int cnt = std::min(CH, nd - c0);
      GSArgs a = gs_args(cnt);
      a.dots = 1;
      a.od = SCR + 2 * c0;
      a.self = c0 + cnt >= nd;
      a.os = WW;
      TRY(gs_gram(w_, V_ + (int64_t)c0 * U, vlast, a, st_));
    }
    double* hp = h_->host_scalars();
    TRY(hipMemcpyAsync(hp, oslots_ + WW, sizeof(double) * (size_t)(SCR - WW + 2 * nd), hipMemcpyDeviceToHost, st_));
    TRY(hipStreamSynchronize(st_));
    ww = hp[0];
    const double* sc = hp + (SCR - WW);
    const int ld = MMAX + 1;
    gram_.resize((size_t)ld * ld);
    std::vector<double> h1(nd);
    for (int c0 = 0; c0 < nd; c0 += CH) {
      const int cnt = std::min(CH, nd - c0);
      for (int d = 0; d < cnt; ++d) {
        h1[c0 + d] = sc[2 * c0 + d];
        const double gv = sc[2 * c0 + cnt + d];
        gram_[(size_t)(c0 + d) * ld + nd - 1] = gv;
        gram_[(size_t)(nd - 1) * ld + c0 + d] = gv;
      }
    }
    hcol.assign(nd, 0.0);
    for (int i = 0; i < nd; ++i) {
      double gh = 0.0;
      for (int k = 0; k < nd; ++k) gh += gram_[(size_t)i * ld + k] * h1[k];
      hcol[i] = 2.0 * h1[i] - gh;
    }
    double hh1 = 0.0, hgh = 0.0;
    for (int i = 0; i < nd; ++i) {
      hh1 += hcol[i] * h1[i];
      double gh = 0.0;
      for (int k = 0; k < nd; ++k) gh += gram_[(size_t)i * ld + k] * hcol[k];
      hgh += hcol[i] * gh;
    }
    h2sq = 2.0 * hh1 - hgh;
    hup_ = hcol;
    return hipMemcpyAsync(oslots_ + H2, hup_.data(), sizeof(double) * (size_t)nd, hipMemcpyHostToDevice, st_);
  }

  // The second Gram-Schmidt correction applied to w (w -= V h2), and
  // ||w||^2 computed directly: used when <w,w> - |h2|^2 cancels.
  hipError_t correct_and_norm(int nd, double& ww) {
    const int64_t U = h_->U;
    const int H2 = 8 + MMAX + 8, WW = H2 + MMAX + 8;
    for (int c0 = 0; c0 < nd; c0 += DOTS_PER_PASS) {
      const int cnt = std::min(DOTS_PER_PASS, nd - c0);
      GSArgs a = gs_args(cnt);
      a.axpy = 1;
      a.ca = H2 + c0;
      a.self = c0 + cnt >= nd;
      a.os = WW;
      TRY(gs_pass<double, double>(w_, V_ + (int64_t)c0 * U, a, 1, st_));
    }
    double* hp = h_->host_scalars();
    TRY(hipMemcpyAsync(hp, oslots_ + WW, sizeof(double), hipMemcpyDeviceToHost, st_));
    TRY(hipStreamSynchronize(st_));
    ww = hp[0];
    return hipSuccess;
  }

  // V_{nd} = (w - V h2) / hn, or w / hn when the correction was applied.
  hipError_t next_basis(int nd, double inv_hn, bool corrected) {
    const int64_t U = h_->U;
    const int H2 = 8 + MMAX + 8;
    if (corrected)
      return basis_update<double, double, double>(w_, 0, V_, U, 0, 0, V_ + (int64_t)nd * U, 0, oslots_, 0, 0, -1,
                                                  inv_hn, U, 1, st_);
    if (nd <= DOTS_PER_PASS)
      return basis_update<double, double, double>(w_, 0, V_, U, 0, nd, V_ + (int64_t)nd * U, 0, oslots_, 0, H2, -1,
                                                  inv_hn, U, 1, st_);
    for (int c0 = 0; c0 < nd; c0 += DOTS_PER_PASS) {
      GSArgs a = gs_args(std::min(DOTS_PER_PASS, nd - c0));
      a.axpy = 1;
      a.ca = H2 + c0;
      TRY(gs_pass<double, double>(w_, V_ + (int64_t)c0 * U, a, 1, st_));
    }
    return basis_update<double, double, double>(w_, 0, V_, U, 0, 0, V_ + (int64_t)nd * U, 0, oslots_, 0, 0, -1,
                                                inv_hn, U, 1, st_);
  }

  // P-tilde^{-1} of the FP64 vector r, into the TI vector z; phase times
  // are added once the stream has been synchronised (see phase_times).
  hipError_t precond(const double* r, TI* z) {
    if (pending_) {   // a previous application's times are still unread
      TRY(hipEventSynchronize(h_->phase_ev[2]));
      phase_times();
    }
    TRY(precond_apply(h_, r, z, h_->opts.inner_k, h_->opts.cycles, transpose_, timed_));
    pending_ = timed_;
    ++applications_;
    return hipSuccess;
  }

  void phase_times() {
    if (!pending_) return;
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, h_->phase_ev[0], h_->phase_ev[1]) == hipSuccess &&
        hipEventElapsedTime(&b, h_->phase_ev[1], h_->phase_ev[2]) == hipSuccess) {
      // forward: Theta-tilde first; transposed: the S-tilde^T sweep first
      theta_ms_ += transpose_ ? b : a;
      schur_ms_ += transpose_ ? a : b;
    }
    pending_ = false;
  }

  // Algorithm 1, restarted.  side RIGHT: z_j = P^{-1} v_j, w = A z_j, and
  // a cycle starts from r = rhs - A x; LEFT: w = P^{-1} (A v_j), r0 =
  // P^{-1} rhs - P^{-1} (A x); SPLIT: both.  P = P-tilde (or its transpose).
  int run(const double* rhs, double* x, aao_stats* stats) {
    const int64_t U = h_->U;
    const int m = h_->opts.restart;
    const int side = h_->opts.side;
    const bool left = side != AAO_SIDE_RIGHT, right = side != AAO_SIDE_LEFT;
    // approach A3: u = u_A = FP32, simulated by rounding every outer step's
    // result (a no-op in FP64)
    const bool chop = h_->opts.outer_precision == AAO_OUTER_FP32;
    auto rnd = [&](double* v) { return chop ? launch_round_f32(v, U, st_) : hipSuccess; };
    TI* tY = reinterpret_cast<TI*>(h_->ws + h_->plan.outY);     // P^{-1} of a product with A
    TI* pb = reinterpret_cast<TI*>(h_->ws + h_->plan.outPb);    // P^{-1} rhs
    double* tr = V_ + (int64_t)m * U;   // true residual, in the basis slot no cycle start uses
    auto t0 = std::chrono::steady_clock::now();
    timed_ = !h_->no_alloc;
    for (int i = 0; i < 3 && timed_; ++i)
      if (!h_->phase_ev[i] && hipEventCreate(&h_->phase_ev[i]) != hipSuccess) timed_ = false;
    aao_stats local{};
    aao_stats& stt = stats ? *stats : local;
    stt = aao_stats{};
    hipError_t e = launch_fill<unsigned>(counters_, 0u, 2, st_);
    if (e != hipSuccess) return status_from_hip(h_, e, "solve");
    double nb2 = 0.0;
    e = norm2(rhs, &nb2);
    if (e != hipSuccess) return status_from_hip(h_, e, "solve");
    const double nb = std::sqrt(nb2);
    if (!std::isfinite(nb)) {
      h_->err = "non-finite value in the right-hand side";
      return AAO_NONFINITE;
    }
    if (!(nb > 0.0)) {       // zero right-hand side: x = 0 is the solution
      e = launch_fill<double>(x, 0.0, U, st_);
      if (e == hipSuccess) e = hipStreamSynchronize(st_);
      stt.relres = 0.0;
      return e == hipSuccess ? AAO_OK : status_from_hip(h_, e, "solve");
    }
    if (left && (e = precond(rhs, pb)) != hipSuccess) return status_from_hip(h_, e, "solve");
    int its = 0;
    int status = AAO_NOT_CONVERGED;
    double beta0 = -1.0;   // the first cycle's residual norm (LEFT / SPLIT stopping reference)
    std::vector<double> R((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m), hcol;
    while (true) {
      // true residual rhs - A x, and the cycle's starting residual
      if ((e = op<double>(x, tr)) != hipSuccess) break;
      double ax2 = 0.0;
      if (left && (e = norm2(tr, &ax2)) != hipSuccess) break;
      if ((e = launch_sub_from(rhs, tr, U, st_)) != hipSuccess) break;
      double t2;
      if ((e = norm2(tr, &t2)) != hipSuccess) break;
      stt.relres = std::sqrt(t2) / nb;
      if (!std::isfinite(stt.relres)) { status = AAO_NONFINITE; break; }
      double beta;
      if (!left) {
        if (!chop) {
          if ((e = launch_copy_cast<double, double>(w_, tr, U, st_)) != hipSuccess) break;
          beta = std::sqrt(t2);
        } else {
          // r0 = fl(rhs - fl(A x)) with fl the rounding to FP32
          if ((e = op<double>(x, w_)) != hipSuccess || (e = rnd(w_)) != hipSuccess) break;
          if ((e = launch_sub_from(rhs, w_, U, st_)) != hipSuccess) break;
          if ((e = rnd(w_)) != hipSuccess) break;
          double b2;
          if ((e = norm2(w_, &b2)) != hipSuccess) break;
          beta = std::sqrt(b2);
          if (!std::isfinite(beta)) { status = AAO_NONFINITE; break; }
        }
      } else {
        // r0 = P^{-1} rhs - P^{-1} (A x); A x = rhs - tr (zero for x = 0)
        if (ax2 > 0.0) {
          if ((e = launch_diff<double, double>(w_, rhs, tr, U, st_)) != hipSuccess) break;
          if ((e = rnd(w_)) != hipSuccess) break;
          if ((e = precond(w_, tY)) != hipSuccess) break;
          if ((e = launch_diff<double, TI>(w_, pb, tY, U, st_)) != hipSuccess) break;
        } else {
          if ((e = launch_diff<double, TI>(w_, pb, nullptr, U, st_)) != hipSuccess) break;
        }
        if ((e = rnd(w_)) != hipSuccess) break;
        double b2;
        if ((e = norm2(w_, &b2)) != hipSuccess) break;
        beta = std::sqrt(b2);
        if (!std::isfinite(beta)) { status = AAO_NONFINITE; break; }
      }
      if (beta0 < 0.0) beta0 = left ? beta : nb;
      if (left ? beta <= h_->opts.tol * beta0 : stt.relres <= h_->opts.tol) { status = AAO_OK; break; }
      if (!(beta > 0.0)) { status = AAO_OK; break; }
      if (its >= h_->opts.maxit) { status = AAO_NOT_CONVERGED; break; }
      stt.restarts++;
      if ((e = launch_scale<double, double>(V_, w_, 1.0 / beta, U, st_)) != hipSuccess) break;
      if ((e = rnd(V_)) != hipSuccess) break;
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int mm = 0;
      bool stop = false, ls_met = false;
      double lsres = beta;   // least-squares residual after the previous iteration
      for (int j = 0; j < m && !stop; ++j) {
        its++;
        double* vj = V_ + (int64_t)j * U;
        if (right) {
          if ((e = precond(vj, Z_ + (int64_t)j * U)) != hipSuccess) break;
          if ((e = op<TI>(Z_ + (int64_t)j * U, w_)) != hipSuccess) break;
        } else {
          if ((e = op<double>(vj, w_)) != hipSuccess) break;
        }
        if ((e = rnd(w_)) != hipSuccess) break;
        if (h_->opts.relax_matvec && lsres > 0.0) {
          // the relative error this product may carry (Simoncini-Szyld)
          const double eta = h_->opts.tol * beta0 / lsres;
          if (eta >= 10.0 * 0x1p-8) {
            if ((e = launch_round_bf16(w_, U, st_)) != hipSuccess) break;
            stt.relaxed_bf16++;
          } else if (eta >= 10.0 * 0x1p-24) {
            if ((e = launch_round_f32(w_, U, st_)) != hipSuccess) break;
            stt.relaxed_fp32++;
          }
        }
        if (left) {
          if ((e = precond(w_, tY)) != hipSuccess) break;
          if ((e = launch_copy_cast<double, TI>(w_, tY, U, st_)) != hipSuccess) break;
        }
        double h2sq, ww;
        if ((e = orthogonalize(j + 1, hcol, h2sq, ww)) != hipSuccess) break;
        phase_times();
        // h_{j+1,j} = sqrt(<w,w> - |h2|^2) unless that cancels: then the
        // corrected w's norm is computed directly
        double nrm2 = ww - h2sq;
        bool corrected = false;
        if (!(nrm2 > 1e-8 * ww) && ww > 0.0 && std::isfinite(ww)) {
          if ((e = correct_and_norm(j + 1, nrm2)) != hipSuccess) break;
          corrected = true;
        }
        const double hn = nrm2 > 0.0 ? std::sqrt(nrm2) : 0.0;
        std::vector<double> col(hcol);
        col.push_back(hn);
        for (int i = 0; i < j; ++i) {
          const double a = col[i], b = col[i + 1];
          col[i] = cs[i] * a + sn[i] * b;
          col[i + 1] = -sn[i] * a + cs[i] * b;
        }
        const double rho = std::hypot(col[j], col[j + 1]);
        if (!std::isfinite(rho) || !std::isfinite(hn)) { status = AAO_NONFINITE; stop = true; break; }
        if (rho == 0.0) { stop = true; break; }
        cs[j] = col[j] / rho;
        sn[j] = col[j + 1] / rho;
        col[j] = rho;
        for (int i = 0; i <= j; ++i) R[(size_t)j * (m + 1) + i] = col[i];
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        mm = j + 1;
        lsres = std::fabs(g[j + 1]);
        const double est = lsres / beta0;
        if (stt.history_len < 128) stt.history[stt.history_len++] = est;
        if (est <= h_->opts.tol) ls_met = true;
        if (ls_met || hn == 0.0 || its >= h_->opts.maxit) stop = true;
        if (!stop && j + 1 < m) {
          if ((e = next_basis(j + 1, 1.0 / hn, corrected)) != hipSuccess) break;
          if ((e = rnd(V_ + (int64_t)(j + 1) * U)) != hipSuccess) break;
        }
      }
      if (e != hipSuccess || status == AAO_NONFINITE) break;
      // x += Z y (right, split) or V y (left)
      for (int i = mm - 1; i >= 0; --i) {
        double acc = g[i];
        for (int jj = i + 1; jj < mm; ++jj) acc -= R[(size_t)jj * (m + 1) + i] * y[jj];
        y[i] = acc / R[(size_t)i * (m + 1) + i];
      }
      const int YOFF = 4 * (MMAX + 8);
      double* ydev = oslots_ + YOFF;
      if (mm > 0) {
        double* hp = h_->host_scalars();
        for (int i = 0; i < mm; ++i) hp[i] = y[i];
        if ((e = hipMemcpyAsync(ydev, hp, sizeof(double) * mm, hipMemcpyHostToDevice, st_)) != hipSuccess)
          break;
        for (int c0 = 0; c0 < mm && e == hipSuccess; c0 += DOTS_PER_PASS) {
          const int cnt = std::min(DOTS_PER_PASS, mm - c0);
          if (right)
            e = combine<double, TI>(x, 0, Z_ + (int64_t)c0 * U, U, 0, cnt, oslots_, 0, YOFF + c0, false, true, U, 1,
                                    st_);
          else
            e = combine<double, double>(x, 0, V_ + (int64_t)c0 * U, U, 0, cnt, oslots_, 0, YOFF + c0, false, true,
                                        U, 1, st_);
        }
        if (e != hipSuccess || (e = rnd(x)) != hipSuccess) break;
        // the host buffer is reused by the next iteration: wait for the copy
        if ((e = hipStreamSynchronize(st_)) != hipSuccess) break;
      }
      if (left && ls_met) {
        // Algorithm 1 ends here: the least-squares residual of the
        // preconditioned system met the target; report the true residual
        if ((e = op<double>(x, tr)) != hipSuccess) break;
        if ((e = launch_sub_from(rhs, tr, U, st_)) != hipSuccess) break;
        double t2;
        if ((e = norm2(tr, &t2)) != hipSuccess) break;
        stt.relres = std::sqrt(t2) / nb;
        status = AAO_OK;
        break;
      }
    }
    if (e == hipSuccess) {
      phase_times();
      unsigned* hc = reinterpret_cast<unsigned*>(h_->host_scalars());
      e = hipMemcpyAsync(hc, counters_, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, st_);
      if (e == hipSuccess) e = hipStreamSynchronize(st_);
      if (e == hipSuccess) {
        stt.inner_iterations = hc[0];
        stt.inner_solves = (int)hc[1];
      }
    }
    stt.outer_iterations = its;
    stt.theta_ms = theta_ms_;
    stt.schur_ms = schur_ms_;
    stt.precond_ms = theta_ms_ + schur_ms_;
    stt.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) return status_from_hip(h_, e, transpose_ ? "solve_adjoint" : "solve");
    if (status == AAO_NONFINITE) h_->err = "non-finite value in the Krylov recurrence";
    if (status == AAO_NOT_CONVERGED) h_->err = "maximum number of iterations reached";
    return status;
  }

 private:
  aao_problem* h_;
  hipStream_t st_;
  bool transpose_;
  double *V_, *w_, *partial_, *oslots_;
  unsigned* counters_;
  TI* Z_;
  std::vector<double> gram_;   // Gram matrix of the outer basis (outer_orth GRAM), (MMAX + 1)^2
  std::vector<double> hup_;    // its projection coefficients, uploaded to the slots
  bool timed_ = false, pending_ = false;
  int applications_ = 0;
  double theta_ms_ = 0.0, schur_ms_ = 0.0;
};

}  // namespace

// ---------------------------------------------------------------------------
// Launch timing of the V-cycle and the tile autotuner
// ---------------------------------------------------------------------------
// The kernel nodes of a graph captured from one stream, in launch order
// (a chain: each node depends on the one before).
std::vector<hipGraphNode_t> chain_order(hipGraph_t g, hipError_t& e) {
  std::vector<hipGraphNode_t> out;
  size_t n = 0;
  e = hipGraphGetNodes(g, nullptr, &n);
  if (e != hipSuccess || n == 0) return out;
  std::vector<hipGraphNode_t> nodes(n);
  if ((e = hipGraphGetNodes(g, nodes.data(), &n)) != hipSuccess) return out;
  hipGraphNode_t cur = nullptr;
  for (auto nd : nodes) {
    size_t deps = 0;
    if ((e = hipGraphNodeGetDependencies(nd, nullptr, &deps)) != hipSuccess) return out;
    if (deps == 0) cur = nd;
  }
  while (cur && out.size() < n) {
    out.push_back(cur);
    size_t nd = 0;
    if ((e = hipGraphNodeGetDependentNodes(cur, nullptr, &nd)) != hipSuccess) return out;
    if (nd != 1) break;
    hipGraphNode_t next = nullptr;
    if ((e = hipGraphNodeGetDependentNodes(cur, &next, &nd)) != hipSuccess) return out;
    cur = next;
  }
  if (out.size() != n) e = hipErrorInvalidValue;   // not a chain
  return out;
}

// Mean microseconds per replay of an instantiated graph (events around
// `reps` back-to-back replays).
hipError_t time_graph(hipGraphExec_t x, hipStream_t st, int reps, double& us) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipGraphLaunch(x, st);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int k = 0; k < reps && e == hipSuccess; ++k) e = hipGraphLaunch(x, st);
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  us = 1e3 * ms / reps;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return e;
}

// Per-launch times of one V-cycle from zero on `count` blocks, two ways:
// in situ -- the cycle run `reps` times with an event recorded after every
// launch, so a launch's time is the interval since the previous event (the
// kernel with cold caches as in a solve, plus the dispatch gap after an
// event) -- and alone -- the cycle captured as a graph and each launch
// replayed by itself, `reps` copies back to back (every V-cycle kernel writes
// buffers it does not read, so repeating it alone is well defined).  The
// cycle time is the mean of `reps` replays of the cycle's graph.
template <class TI, class TM>
hipError_t profile_vcycle_typed(aao_problem* h, int stage, int count, int reps, std::vector<std::string>& labels,
                                std::vector<double>& us_situ, std::vector<double>& us_alone, double& total_us) {
  const int64_t N = h->N;
  TI* r = reinterpret_cast<TI*>(h->ws + h->plan.inV);
  TI* z = reinterpret_cast<TI*>(h->ws + h->plan.inZ);
  const BVec<TI> zv{z, N};
  const BVec<const TI> rv{r, N};
  TRY(launch_fill<TI>(r, TI(1), (int64_t)count * N, h->stream));
  TRY(hipStreamSynchronize(h->stream));
  // in situ
  {
    Multigrid<TI, TM> mg(h, h->stream, h->tab.L);
    TRY(mg.solve(stage, zv, rv, count, 1));   // warm-up
    constexpr int MAXM = 256;                 // launches per V-cycle, at most
    typename Multigrid<TI, TM>::Marks m;
    m.ev.assign((size_t)reps * MAXM, nullptr);
    m.label.assign(m.ev.size(), std::string());
    std::vector<hipEvent_t> start(reps, nullptr);
    hipError_t e = hipSuccess;
    for (auto& ev : m.ev)
      if (e == hipSuccess) e = hipEventCreate(&ev);
    for (auto& ev : start)
      if (e == hipSuccess) e = hipEventCreate(&ev);
    size_t per = 0;
    if (e == hipSuccess) {
      mg.set_marks(&m);
      for (int k = 0; k < reps && e == hipSuccess; ++k) {
        m.next = (size_t)k * MAXM;
        e = hipEventRecord(start[k], h->stream);
        if (e == hipSuccess) e = mg.solve(stage, zv, rv, count, 1);
        if (k == 0) per = m.next;
      }
      mg.set_marks(nullptr);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) {
      labels.assign(m.label.begin(), m.label.begin() + per);
      us_situ.assign(per, 0.0);
      for (int k = 0; k < reps; ++k) {
        hipEvent_t prev = start[k];
        for (size_t i = 0; i < per; ++i) {
          float ms = 0.f;
          hipEvent_t cur = m.ev[(size_t)k * MAXM + i];
          if (hipEventElapsedTime(&ms, prev, cur) == hipSuccess) us_situ[i] += 1e3 * ms / reps;
          prev = cur;
        }
      }
    }
    for (auto& ev : m.ev)
      if (ev) (void)hipEventDestroy(ev);
    for (auto& ev : start)
      if (ev) (void)hipEventDestroy(ev);
    TRY(e);
  }
  // alone, and the whole cycle, from a captured graph
  hipStream_t cap = nullptr;
  TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  Multigrid<TI, TM> mg(h, cap, h->tab.L);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t e1 = mg.solve(stage, zv, rv, count, 1);
    const hipError_t e2 = hipStreamEndCapture(cap, &g);
    e = e1 != hipSuccess ? e1 : e2;
  }
  hipGraphExec_t x = nullptr;
  std::vector<hipGraphNode_t> chain;
  if (e == hipSuccess) chain = chain_order(g, e);
  if (e == hipSuccess && chain.size() != labels.size()) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e == hipSuccess) e = time_graph(x, h->stream, reps, total_us);
  if (x) (void)hipGraphExecDestroy(x);
  us_alone.assign(chain.size(), 0.0);
  for (size_t i = 0; i < chain.size() && e == hipSuccess; ++i) {
    hipKernelNodeParams kp{};
    e = hipGraphKernelNodeGetParams(chain[i], &kp);
    hipGraph_t gi = nullptr;
    if (e == hipSuccess) e = hipGraphCreate(&gi, 0);
    hipGraphNode_t prev = nullptr;
    for (int k = 0; k < reps && e == hipSuccess; ++k) {
      hipGraphNode_t nd = nullptr;
      e = hipGraphAddKernelNode(&nd, gi, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
      prev = nd;
    }
    hipGraphExec_t xi = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&xi, gi, nullptr, nullptr, 0);
    double t = 0.0;
    if (e == hipSuccess) e = time_graph(xi, h->stream, 1, t);
    us_alone[i] = t / reps;
    if (xi) (void)hipGraphExecDestroy(xi);
    if (gi) (void)hipGraphDestroy(gi);
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  return e;
}

hipError_t profile_vcycle(aao_problem* h, int stage, int count, int reps, std::vector<std::string>& labels,
                          std::vector<double>& us_situ, std::vector<double>& us_alone, double& total_us) {
  switch (h->opts.precision) {
    case AAO_PREC_FP64:
      return profile_vcycle_typed<double, double>(h, stage, count, reps, labels, us_situ, us_alone, total_us);
    case AAO_PREC_FP32:
      return profile_vcycle_typed<float, float>(h, stage, count, reps, labels, us_situ, us_alone, total_us);
    case AAO_PREC_FP16:
      return profile_vcycle_typed<float, __half>(h, stage, count, reps, labels, us_situ, us_alone, total_us);
    case AAO_PREC_FP16_ALL:
      return profile_vcycle_typed<__half, __half>(h, stage, count, reps, labels, us_situ, us_alone, total_us);
    default:
      return profile_vcycle_typed<float, __hip_bfloat16>(h, stage, count, reps, labels, us_situ, us_alone, total_us);
  }
}

void release_graphs(aao_problem* h) {
  for (auto& g : h->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  h->graphs.clear();
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  h->capture_stream = nullptr;
}

int mg_tail_level(aao_problem* h) {
  switch (h->opts.precision) {
    case AAO_PREC_FP64: return Multigrid<double, double>(h, h->stream, h->tab.L).tail_level();
    case AAO_PREC_FP32: return Multigrid<float, float>(h, h->stream, h->tab.L).tail_level();
    case AAO_PREC_FP16: return Multigrid<float, __half>(h, h->stream, h->tab.L).tail_level();
    case AAO_PREC_FP16_ALL: return Multigrid<__half, __half>(h, h->stream, h->tab.L).tail_level();
    default: return Multigrid<float, __hip_bfloat16>(h, h->stream, h->tab.L).tail_level();
  }
}

hipError_t apply_mg(aao_problem* h, bool transpose, int stage, int count, int cycles, const void* r, void* z) {
  switch (h->opts.precision) {
    case AAO_PREC_FP64: return apply_mg_typed<double, double>(h, transpose, stage, count, cycles, r, z);
    case AAO_PREC_FP32: return apply_mg_typed<float, float>(h, transpose, stage, count, cycles, r, z);
    case AAO_PREC_FP16: return apply_mg_typed<float, __half>(h, transpose, stage, count, cycles, r, z);
    case AAO_PREC_FP16_ALL: return apply_mg_typed<__half, __half>(h, transpose, stage, count, cycles, r, z);
    default: return apply_mg_typed<float, __hip_bfloat16>(h, transpose, stage, count, cycles, r, z);
  }
}

hipError_t prepare_graph(aao_problem* h, bool transpose) {
  if (!h->opts.use_graph || h->no_alloc) return hipSuccess;
  aao_problem::GraphEntry* ent = nullptr;
  TRY(precond_graph(h, h->opts.inner_k, h->opts.cycles, transpose, 1, &ent));
  return precond_graph(h, h->opts.inner_k, h->opts.cycles, transpose, 2, &ent);
}

int apply_P(aao_problem* h, const double* r, double* z, int inner_k, int cycles, bool transpose) {
  hipError_t e;
  if (h->opts.precision == AAO_PREC_FP64) {
    e = precond_apply(h, r, z, inner_k, cycles, transpose, false);
  } else if (h->opts.precision == AAO_PREC_FP16_ALL) {
    __half* zp = reinterpret_cast<__half*>(h->ws + h->plan.outY);
    e = precond_apply(h, r, zp, inner_k, cycles, transpose, false);
    if (e == hipSuccess) e = launch_copy_cast<double, __half>(z, zp, h->U, h->stream);
  } else {
    float* zp = reinterpret_cast<float*>(h->ws + h->plan.outY);
    e = precond_apply(h, r, zp, inner_k, cycles, transpose, false);
    if (e == hipSuccess) e = launch_copy_cast<double, float>(z, zp, h->U, h->stream);
  }
  return status_from_hip(h, e, "apply_P");
}

int solve(aao_problem* h, const double* rhs, double* x, aao_stats* st, bool transpose) {
  if (transpose && h->fe) {
    h->err = "finite elements: the transposed solve is not available";
    return AAO_INVALID_ARG;
  }
  if (h->opts.precision == AAO_PREC_FP64) {
    Fgmres<double> F(h, transpose);
    return F.run(rhs, x, st);
  }
  if (h->opts.precision == AAO_PREC_FP16_ALL) {
    Fgmres<__half> F(h, transpose);
    return F.run(rhs, x, st);
  }
  Fgmres<float> F(h, transpose);
  return F.run(rhs, x, st);
}

}  // namespace aao

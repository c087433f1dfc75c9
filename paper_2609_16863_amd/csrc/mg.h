// Geometric multigrid V-cycles for the shifted blocks I + a K (a = tau L_ii),
// batched over many right-hand sides (one per time step) in one launch per
// level operation.
#pragma once

#include <string>
#include <vector>

#include "aao_internal.h"

namespace aao {

// TI: storage of the finest level (the inner-GMRES vectors); TM: storage of
// the coarse levels where the precision schedule puts them in the low
// format (opts.mg_low_from, opts.mg_coarse_fp32), TI elsewhere.  Arithmetic
// is in Acc<TI>::type.
template <class TI, class TM>
class Multigrid {
 public:
  using C = typename Acc<TI>::type;

  // L: lower Crout factor (s x s, row-major) whose diagonal gives the shifts
  // tau L_ii.  cinv_set: which precomputed coarsest-level inverses match
  // those shifts (0: P-tilde, 1: its transpose, 2 / 3: the same for the
  // MGRIT coarse step); -1 picks 0 or 1 from L.
  Multigrid(aao_problem* h, hipStream_t st, const double* L, int cinv_set = -1);

  // Rana's coupling for stage i = nz > 0: the block right-hand side is
  // rhs - tau sum_{l < i} Lc[i][l] K z_l (z_l at z + l * zstride, instance
  // stride sz; Lc the s x s lower factor), formed inside the first level-0
  // kernel where the tiled path runs (else by a separate kernel) and written
  // to `out` (stride so).
  struct Coupling {
    const TI* z = nullptr;
    int64_t sz = 0, zstride = 0;
    int nz = 0;
    const double* Lc = nullptr;
    TI* out = nullptr;
    int64_t so = 0;
  };

  // x_b <- (`cycles` V-cycles from zero) ~ (I + tau L_ii K)^{-1} rhs_b for
  // b = 0..B-1.  x and rhs are level-0 vectors with their own instance
  // strides; B <= nt.  With `cpl`, the right-hand side is rhs minus the
  // coupling terms (see Coupling).
  hipError_t solve(int stage, BVec<TI> x, BVec<const TI> rhs, int B, int cycles, const Coupling* cpl = nullptr);

  // First level solved by the one-workgroup LDS tail (= levels when none).
  int tail_level() const { return l0_; }

  // Launch labels ("kernel name@level") of vcycle(), in launch order, while
  // set; with events in `ev`, one is also recorded after every launch.
  struct Marks {
    std::vector<hipEvent_t> ev;
    std::vector<std::string> label;
    size_t next = 0;
  };
  void set_marks(Marks* m) { marks_ = m; }

 private:
  struct Vec {
    void* ptr;
    int64_t stride;
  };
  hipError_t vcycle(int l, int stage, Vec x, Vec b, bool zero_init, bool pre, int B, Vec* result,
                    const Coupling* cpl = nullptr);
  hipError_t smooth(int l, int stage, Vec xin, Vec xout, Vec b, bool zero_init, int B);
  hipError_t resid_restrict(int l, int stage, Vec x, Vec b, Vec bc, Vec xc, bool zero_next, int B);
  hipError_t prolong(int l, Vec xin, Vec ec, Vec xout, int B);
  hipError_t prolong_smooth0(int stage, Vec xin, Vec ec, Vec b, Vec xout, int B);
  hipError_t tail(int stage, Vec x, Vec b, bool zero_init, int B);
  hipError_t down2d(int l, int stage, Vec b, const void* x0, int64_t sx0, Vec xout, Vec bc, int B,
                    const Coupling* cpl = nullptr);
  hipError_t up2d(int l, int stage, Vec xin, Vec ec, Vec b, Vec xout, int B);
  // 3D level 0 as z-marches (constant kappa, two sweeps each way, zero
  // start, from tall_min_b blocks per launch on): sweeps, residual and full
  // weighting into bc (and the coarse first sweep into xc); prolongation and
  // sweeps into xout (!= x2)
  bool march3d_ok(int l, bool zero_init, bool pre, int B) const;
  hipError_t march3d_down(int stage, Vec b, Vec x2, Vec bc, Vec xc, bool zero_next, int B);
  hipError_t march3d_up(int stage, Vec x2, Vec ec, Vec b, Vec xout, int B);
  const C* coarse_inv(int stage) const;

  hipError_t mark(const char* kernel, int l);

  // Storage precision of every level (see the class comment).
  void set_level_storage();
  bool low(int l) const { return l > 0 && l < levels_ && low_[l] != 0; }
  // the residual of level l is formed once per node, then restricted (3D;
  // level 0 of Q2 elements, whose 25-point operator the fused kernel would
  // apply at all nine fine nodes around each coarse node)
  bool split_restrict(int l) const { return h_->dim == 3 || (l == 0 && h_->fe_order == 2); }
  // f(T{}) with the storage type T of level l; f(TF{}, TC{}) with those of
  // levels l and l + 1.
  template <class F>
  hipError_t typed1(int l, F&& f) const;
  template <class F>
  hipError_t typed2(int l, F&& f) const;

  aao_problem* h_;
  hipStream_t st_;
  Marks* marks_ = nullptr;
  double a_[SMAX];
  int levels_;
  int l0_;          // first level solved by the one-workgroup LDS tail
  size_t tail_bytes_;
  int fast_nls_;    // > 0: the tail runs k_tail_fast with this many smoothing levels
  int fast_npt_;    // its nodes per thread on the first tail level (1 or 4)
  size_t fast_bytes_;
  int cinv_set_;    // coarsest-level inverse set (see the constructor)
  std::vector<char> low_;   // low_[l]: level l stored in TM (else TI)
};

}  // namespace aao

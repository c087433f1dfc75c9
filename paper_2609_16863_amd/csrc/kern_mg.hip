// Geometric multigrid for the shifted blocks I + a K of Rana's stage
// preconditioner: weighted Jacobi smoothing, full-weighting restriction,
// linear prolongation, Galerkin coarse operators.  Every kernel is batched:
// blockIdx.y selects the right-hand side (one per time step).
//
// Level 0 applies I + a K matrix-free (5/7-point, constant or face
// diffusivities).  For constant diffusivity the Galerkin operator of level
// l >= 1 is  M(x)M + a (T(x)M + M(x)T)  (3D: three-fold products) with 1D
// tridiagonal factors M_l, T_l, so its 9/27 coefficients are formed in
// registers from six short arrays instead of being streamed from HBM.
#include "aao_internal.h"
#include "mg.h"
#include "stencil.h"

namespace aao {

namespace {

constexpr int TPB = 256;
enum { KIND_FINE = 0, KIND_FINE_VK = 1, KIND_TENSOR = 2 };

template <class C>
struct Tri3 {
  C m[3];  // M(i, i-1), M(i, i), M(i, i+1)
  C t[3];  // T(i, i-1), T(i, i), T(i, i+1)
};

template <class C>
__device__ __forceinline__ Tri3<C> tri_row(const C* __restrict__ tri, int n, int i) {
  Tri3<C> r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    r.m[q] = tri[q * n + i];
    r.t[q] = tri[(3 + q) * n + i];
  }
  return r;
}

template <int DIM, int KIND, class C>
__device__ __forceinline__ C level_diag(const LevelOp<C>& op, int p, int i, int j, int k) {
  if (KIND == KIND_FINE) return C(1) + op.a * op.ih2 * C(2 * DIM);
  if (KIND == KIND_FINE_VK) return C(1) + op.a * op.ih2 * stencil_K_diag<DIM, true, C>(p, op.faces);
  const Tri3<C> ri = tri_row(op.tri, op.n, i), rj = tri_row(op.tri, op.n, j);
  if (DIM == 2) return ri.m[1] * rj.m[1] + op.a * (ri.t[1] * rj.m[1] + ri.m[1] * rj.t[1]);
  const Tri3<C> rk = tri_row(op.tri, op.n, k);
  return ri.m[1] * rj.m[1] * rk.m[1] +
         op.a * (ri.t[1] * rj.m[1] * rk.m[1] + ri.m[1] * rj.t[1] * rk.m[1] + ri.m[1] * rj.m[1] * rk.t[1]);
}

// (A x)_p and the diagonal A_pp of the level operator.
template <int DIM, int KIND, class T, class C>
__device__ __forceinline__ void level_apply(const T* __restrict__ x, const LevelOp<C>& op, int p, int i,
                                            int j, int k, C& Ax, C& diag) {
  const int n = op.n;
  if (KIND == KIND_FINE || KIND == KIND_FINE_VK) {
    const C kx = stencil_K<DIM, KIND == KIND_FINE_VK, T, C>(x, p, i, j, k, n, (int)op.N, op.faces);
    Ax = ld<T, C>(x + p) + op.a * op.ih2 * kx;
    diag = level_diag<DIM, KIND, C>(op, p, i, j, k);
    return;
  }
  const Tri3<C> ri = tri_row(op.tri, n, i), rj = tri_row(op.tri, n, j);
  C mi_at[3], ti_at[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mi_at[q] = ri.m[q] + op.a * ri.t[q];   // (M + a T) along x
    ti_at[q] = ri.m[q];                    // M along x
  }
  auto row_sums = [&](int base, C& pv, C& qv) {  // base = index of (i, j', k')
    pv = C(0);
    qv = C(0);
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= n) continue;
      const C xv = ld<T, C>(x + base + di);
      pv += mi_at[di + 1] * xv;
      qv += ti_at[di + 1] * xv;
    }
  };
  C acc = C(0);
  if (DIM == 2) {
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= n) continue;
      C pv, qv;
      row_sums(p + dj * n, pv, qv);
      acc += rj.m[dj + 1] * pv + op.a * rj.t[dj + 1] * qv;
    }
    Ax = acc;
    diag = ri.m[1] * rj.m[1] + op.a * (ri.t[1] * rj.m[1] + ri.m[1] * rj.t[1]);
    return;
  }
  const Tri3<C> rk = tri_row(op.tri, n, k);
  const int nn = n * n;
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk) {
    const int kk = k + dk;
    if (kk < 0 || kk >= n) continue;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= n) continue;
      C pv, qv;
      row_sums(p + dk * nn + dj * n, pv, qv);
      const C mm = rj.m[dj + 1] * rk.m[dk + 1];
      const C tm = rj.t[dj + 1] * rk.m[dk + 1] + rj.m[dj + 1] * rk.t[dk + 1];
      acc += mm * pv + op.a * tm * qv;
    }
  }
  Ax = acc;
  diag = ri.m[1] * rj.m[1] * rk.m[1] +
         op.a * (ri.t[1] * rj.m[1] * rk.m[1] + ri.m[1] * rj.t[1] * rk.m[1] + ri.m[1] * rj.m[1] * rk.t[1]);
}

// x_out = x_in + omega D^{-1} (b - A x_in);  zero_init: x_out = omega D^{-1} b.
template <int DIM, int KIND, class T, class C>
__global__ __launch_bounds__(TPB) void k_smooth(const T* __restrict__ xin, int64_t sxin, T* xout,
                                                int64_t sxout, const T* __restrict__ b, int64_t sb,
                                                LevelOp<C> op, C omega, int zero_init) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= op.N) return;
  const int64_t inst = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, op.n, i, j, k);
  const C bp = ld<T, C>(b + inst * sb + p);
  C out;
  if (zero_init) {
    out = omega * bp / level_diag<DIM, KIND, C>(op, p, i, j, k);
  } else {
    const T* x = xin + inst * sxin;
    C Ax, d;
    level_apply<DIM, KIND, T, C>(x, op, p, i, j, k, Ax, d);
    out = ld<T, C>(x + p) + omega * (bp - Ax) / d;
  }
  st<T, C>(xout + inst * sxout + p, out);
}

// r = b - A x
template <int DIM, int KIND, class T, class C>
__global__ __launch_bounds__(TPB) void k_residual(const T* __restrict__ x, int64_t sx,
                                                  const T* __restrict__ b, int64_t sb,
                                                  T* __restrict__ r, int64_t sr, LevelOp<C> op) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= op.N) return;
  const int64_t inst = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, op.n, i, j, k);
  C Ax, d;
  level_apply<DIM, KIND, T, C>(x + inst * sx, op, p, i, j, k, Ax, d);
  st<T, C>(r + inst * sr + p, ld<T, C>(b + inst * sb + p) - Ax);
}

// Full weighting: b_c(I..) = 2^{-d} sum_{|d_a| <= 1} prod_a w(d_a) r(2I+1+d_i, ...),
// w(0) = 1, w(+-1) = 1/2, fine indices past the last node are boundary (zero).
template <int DIM, class TF, class TC, class C>
__global__ __launch_bounds__(TPB) void k_restrict(const TF* __restrict__ r, int64_t sr, int nf,
                                                  TC* __restrict__ bc, int64_t sbc, int nc, int Nc) {
  const int pc = blockIdx.x * TPB + threadIdx.x;
  if (pc >= Nc) return;
  const int64_t inst = blockIdx.y;
  int I, J, K;
  node_coords<DIM>(pc, nc, I, J, K);
  const TF* rr = r + inst * sr;
  const C w[3] = {C(0.5), C(1), C(0.5)};
  C acc = C(0);
  const int fi = 2 * I + 1, fj = 2 * J + 1, fk = 2 * K + 1;
  if (DIM == 2) {
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = fj + dj;
      if (jj >= nf) continue;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int ii = fi + di;
        if (ii >= nf) continue;
        acc += w[di + 1] * w[dj + 1] * ld<TF, C>(rr + jj * nf + ii);
      }
    }
    acc *= C(0.25);
  } else {
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      const int kk = fk + dk;
      if (kk >= nf) continue;
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const int jj = fj + dj;
        if (jj >= nf) continue;
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          const int ii = fi + di;
          if (ii >= nf) continue;
          acc += w[di + 1] * w[dj + 1] * w[dk + 1] * ld<TF, C>(rr + ((int64_t)kk * nf + jj) * nf + ii);
        }
      }
    }
    acc *= C(0.125);
  }
  st<TC, C>(bc + inst * sbc + pc, acc);
}

// x_out = x_in + P e_c (linear interpolation; coarse node I sits at fine 2I+1).
template <int DIM, class TX, class TE, class C>
__global__ __launch_bounds__(TPB) void k_prolong(const TX* xin, int64_t sxin, const TE* __restrict__ ec,
                                                 int64_t sec, TX* xout, int64_t sxout, int nf, int Nf,
                                                 int nc) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= Nf) return;
  const int64_t inst = blockIdx.y;
  int c[3];
  node_coords<DIM>(p, nf, c[0], c[1], c[2]);
  int idx[3][2];
  C wt[3][2];
  int cnt[3];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (c[a] & 1) {
      idx[a][0] = (c[a] - 1) >> 1;
      wt[a][0] = C(1);
      cnt[a] = 1;
    } else {
      cnt[a] = 0;
      const int lo = (c[a] >> 1) - 1, hi = c[a] >> 1;
      if (lo >= 0) { idx[a][cnt[a]] = lo; wt[a][cnt[a]] = C(0.5); ++cnt[a]; }
      if (hi < nc) { idx[a][cnt[a]] = hi; wt[a][cnt[a]] = C(0.5); ++cnt[a]; }
    }
  }
  const TE* e = ec + inst * sec;
  C acc = C(0);
  if (DIM == 2) {
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a) acc += wt[0][a] * wt[1][b] * ld<TE, C>(e + idx[1][b] * nc + idx[0][a]);
  } else {
    for (int q = 0; q < cnt[2]; ++q)
      for (int b = 0; b < cnt[1]; ++b)
        for (int a = 0; a < cnt[0]; ++a)
          acc += wt[0][a] * wt[1][b] * wt[2][q] *
                 ld<TE, C>(e + ((int64_t)idx[2][q] * nc + idx[1][b]) * nc + idx[0][a]);
  }
  st<TX, C>(xout + inst * sxout + p, ld<TX, C>(xin + inst * sxin + p) + acc);
}

// Exact solve on a one-node level: x = b / A_00.
template <int DIM, int KIND, class T, class C>
__global__ void k_coarsest(const T* __restrict__ b, int64_t sb, T* __restrict__ x, int64_t sx, LevelOp<C> op,
                           int B) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B) return;
  for (int p = 0; p < (int)op.N; ++p) {
    int i, j, k;
    node_coords<DIM>(p, op.n, i, j, k);
    st<T, C>(x + (int64_t)inst * sx + p,
             ld<T, C>(b + (int64_t)inst * sb + p) / level_diag<DIM, KIND, C>(op, p, i, j, k));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
template <class TI, class TM>
Multigrid<TI, TM>::Multigrid(aao_problem* h, hipStream_t st, const double* L)
    : h_(h), st_(st), levels_((int)h->lev_n.size()) {
  for (int i = 0; i < h->s; ++i) a_[i] = h->tau * L[i * h->s + i];
}

namespace {

template <class C>
LevelOp<C> make_op(const aao_problem* h, int l, double a) {
  LevelOp<C> op{};
  op.n = h->lev_n[l];
  op.N = h->lev_N[l];
  op.a = (C)a;
  op.ih2 = (C)h->ih2;
  const bool dbl = sizeof(C) == 8;
  const char* tri = h->ws + (dbl ? h->plan.tri_d : h->plan.tri_f);
  op.tri = reinterpret_cast<const C*>(tri) + h->tri_off[l];
  if (h->vark && l == 0) {
    const C* base = reinterpret_cast<const C*>(h->ws + (dbl ? h->plan.faces_d : h->plan.faces_f));
    for (int d = 0; d < h->dim; ++d) {
      op.faces.m[d] = base + (2 * d) * h->N;
      op.faces.p[d] = base + (2 * d + 1) * h->N;
    }
  }
  return op;
}

inline dim3 grid2(int64_t N, int B) { return dim3((unsigned)((N + TPB - 1) / TPB), (unsigned)B); }

}  // namespace

#define MG_KIND_DISPATCH(l, M)                                            \
  do {                                                                    \
    if ((l) > 0) {                                                        \
      if (h_->dim == 2) M(2, KIND_TENSOR); else M(3, KIND_TENSOR);        \
    } else if (h_->vark) {                                                \
      if (h_->dim == 2) M(2, KIND_FINE_VK); else M(3, KIND_FINE_VK);      \
    } else {                                                              \
      if (h_->dim == 2) M(2, KIND_FINE); else M(3, KIND_FINE);            \
    }                                                                     \
  } while (0)

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::smooth(int l, int stage, Vec xin, Vec xout, Vec b, bool zero_init, int B) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const C omega = (C)h_->omega;
  const dim3 g = grid2(op.N, B);
  if (l == 0) {
#define MG_SMOOTH0(D, K)                                                                              \
  hipLaunchKernelGGL((k_smooth<D, K, TI, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, \
                     (TI*)xout.ptr, xout.stride, (const TI*)b.ptr, b.stride, op, omega, (int)zero_init)
    MG_KIND_DISPATCH(l, MG_SMOOTH0);
#undef MG_SMOOTH0
  } else {
#define MG_SMOOTH1(D, K)                                                                              \
  hipLaunchKernelGGL((k_smooth<D, K, TM, C>), g, dim3(TPB), 0, st_, (const TM*)xin.ptr, xin.stride, \
                     (TM*)xout.ptr, xout.stride, (const TM*)b.ptr, b.stride, op, omega, (int)zero_init)
    MG_KIND_DISPATCH(l, MG_SMOOTH1);
#undef MG_SMOOTH1
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::residual(int l, int stage, Vec x, Vec b, Vec r, int B) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const dim3 g = grid2(op.N, B);
  if (l == 0) {
#define MG_RES0(D, K)                                                                                   \
  hipLaunchKernelGGL((k_residual<D, K, TI, C>), g, dim3(TPB), 0, st_, (const TI*)x.ptr, x.stride,     \
                     (const TI*)b.ptr, b.stride, (TI*)r.ptr, r.stride, op)
    MG_KIND_DISPATCH(l, MG_RES0);
#undef MG_RES0
  } else {
#define MG_RES1(D, K)                                                                                   \
  hipLaunchKernelGGL((k_residual<D, K, TM, C>), g, dim3(TPB), 0, st_, (const TM*)x.ptr, x.stride,     \
                     (const TM*)b.ptr, b.stride, (TM*)r.ptr, r.stride, op)
    MG_KIND_DISPATCH(l, MG_RES1);
#undef MG_RES1
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::restrict_to(int l, Vec r, Vec bc, int B) {
  const int nf = h_->lev_n[l], nc = h_->lev_n[l + 1];
  const int Nc = (int)h_->lev_N[l + 1];
  const dim3 g = grid2(Nc, B);
  if (l == 0) {
    if (h_->dim == 2)
      hipLaunchKernelGGL((k_restrict<2, TI, TM, C>), g, dim3(TPB), 0, st_, (const TI*)r.ptr, r.stride, nf,
                         (TM*)bc.ptr, bc.stride, nc, Nc);
    else
      hipLaunchKernelGGL((k_restrict<3, TI, TM, C>), g, dim3(TPB), 0, st_, (const TI*)r.ptr, r.stride, nf,
                         (TM*)bc.ptr, bc.stride, nc, Nc);
  } else {
    if (h_->dim == 2)
      hipLaunchKernelGGL((k_restrict<2, TM, TM, C>), g, dim3(TPB), 0, st_, (const TM*)r.ptr, r.stride, nf,
                         (TM*)bc.ptr, bc.stride, nc, Nc);
    else
      hipLaunchKernelGGL((k_restrict<3, TM, TM, C>), g, dim3(TPB), 0, st_, (const TM*)r.ptr, r.stride, nf,
                         (TM*)bc.ptr, bc.stride, nc, Nc);
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::prolong(int l, Vec xin, Vec ec, Vec xout, int B) {
  const int nf = h_->lev_n[l], nc = h_->lev_n[l + 1];
  const int Nf = (int)h_->lev_N[l];
  const dim3 g = grid2(Nf, B);
  if (l == 0) {
    if (h_->dim == 2)
      hipLaunchKernelGGL((k_prolong<2, TI, TM, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride,
                         (const TM*)ec.ptr, ec.stride, (TI*)xout.ptr, xout.stride, nf, Nf, nc);
    else
      hipLaunchKernelGGL((k_prolong<3, TI, TM, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride,
                         (const TM*)ec.ptr, ec.stride, (TI*)xout.ptr, xout.stride, nf, Nf, nc);
  } else {
    if (h_->dim == 2)
      hipLaunchKernelGGL((k_prolong<2, TM, TM, C>), g, dim3(TPB), 0, st_, (const TM*)xin.ptr, xin.stride,
                         (const TM*)ec.ptr, ec.stride, (TM*)xout.ptr, xout.stride, nf, Nf, nc);
    else
      hipLaunchKernelGGL((k_prolong<3, TM, TM, C>), g, dim3(TPB), 0, st_, (const TM*)xin.ptr, xin.stride,
                         (const TM*)ec.ptr, ec.stride, (TM*)xout.ptr, xout.stride, nf, Nf, nc);
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::coarsest(int l, int stage, Vec b, Vec x, int B) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const dim3 g((unsigned)((B + 63) / 64)), blk(64);
  if (l == 0) {
#define MG_CO0(D, K) \
  hipLaunchKernelGGL((k_coarsest<D, K, TI, C>), g, blk, 0, st_, (const TI*)b.ptr, b.stride, (TI*)x.ptr, x.stride, op, B)
    MG_KIND_DISPATCH(l, MG_CO0);
#undef MG_CO0
  } else {
#define MG_CO1(D, K) \
  hipLaunchKernelGGL((k_coarsest<D, K, TM, C>), g, blk, 0, st_, (const TM*)b.ptr, b.stride, (TM*)x.ptr, x.stride, op, B)
    MG_KIND_DISPATCH(l, MG_CO1);
#undef MG_CO1
  }
  return hipGetLastError();
}

#define MG_TRY(...)                           \
  do {                                        \
    hipError_t e_ = (__VA_ARGS__);            \
    if (e_ != hipSuccess) return e_;          \
  } while (0)

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::vcycle(int l, int stage, Vec x, Vec b, bool zero_init, int B, Vec* result) {
  auto& P = h_->plan;
  if (l == levels_ - 1) {
    MG_TRY(coarsest(l, stage, b, x, B));
    *result = x;
    return hipSuccess;
  }
  const int64_t Nl = h_->lev_N[l];
  Vec tmp{h_->ws + P.mgT[l], Nl};
  auto partner = [&](const Vec& v) { return v.ptr == x.ptr ? tmp : x; };
  Vec cur = x;
  int rem = h_->opts.nu1;
  if (zero_init) {
    MG_TRY(smooth(l, stage, cur, cur, b, true, B));
    --rem;
  }
  for (; rem > 0; --rem) {
    Vec nxt = partner(cur);
    MG_TRY(smooth(l, stage, cur, nxt, b, false, B));
    cur = nxt;
  }
  Vec r{h_->ws + P.mgR[l], Nl};
  MG_TRY(residual(l, stage, cur, b, r, B));
  const int64_t Nc = h_->lev_N[l + 1];
  Vec bc{h_->ws + P.mgB[l + 1], Nc};
  Vec xc{h_->ws + P.mgX[l + 1], Nc};
  MG_TRY(restrict_to(l, r, bc, B));
  Vec ec{};
  MG_TRY(vcycle(l + 1, stage, xc, bc, true, B, &ec));
  const int nu2 = h_->opts.nu2;
  Vec tgt = (nu2 % 2 == 0) ? x : tmp;
  MG_TRY(prolong(l, cur, ec, tgt, B));
  cur = tgt;
  for (int it = 0; it < nu2; ++it) {
    Vec nxt = partner(cur);
    MG_TRY(smooth(l, stage, cur, nxt, b, false, B));
    cur = nxt;
  }
  *result = cur;
  return hipSuccess;
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::solve(int stage, BVec<TI> x, BVec<const TI> rhs, int B, int cycles) {
  Vec xv{x.ptr, x.stride};
  Vec bv{const_cast<TI*>(rhs.ptr), rhs.stride};
  for (int c = 0; c < cycles; ++c) {
    Vec res{};
    MG_TRY(vcycle(0, stage, xv, bv, c == 0, B, &res));
    if (res.ptr != xv.ptr) return hipErrorUnknown;   // the driver always ends in x
  }
  return hipSuccess;
}

template class Multigrid<double, double>;
template class Multigrid<float, float>;
template class Multigrid<float, __half>;
template class Multigrid<float, __hip_bfloat16>;

}  // namespace aao

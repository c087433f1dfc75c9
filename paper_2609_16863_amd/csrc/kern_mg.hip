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
#include <type_traits>

#include "aao_internal.h"
#include "fe.h"
#include "krylov.h"
#include "mg.h"
#include "stencil.h"

namespace aao {

namespace {

constexpr int TPB = 256;
// KIND_TENSOR: Galerkin level; its K part comes from the 1D factors, or from
// the stored 9-point stencil op.st9 when that is set (2D, variable kappa).
// KIND_STENCIL9: the same level in the LDS-tiled kernels, which keep the
// stencil coefficients of their nodes in registers.
// (Level 0 of biquadratic elements has its own kernels, fe_q2_smooth and
// fe_q2_residual in kern_fe.hip.)
enum { KIND_FINE = 0, KIND_FINE_VK = 1, KIND_TENSOR = 2, KIND_STENCIL9 = 3 };

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
  if (DIM == 2 && op.st9) return ri.m[1] * rj.m[1] + op.a * op.st9[4 * op.N + p];
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
  if (DIM == 2 && op.st9) {
    // M(x)M from the factors plus a times the stored stencil of K
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = j + dj;
      if (jj < 0 || jj >= n) continue;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= n) continue;
        const C coef = rj.m[dj + 1] * ri.m[di + 1] + op.a * op.st9[((dj + 1) * 3 + di + 1) * op.N + p];
        acc += coef * ld<T, C>(x + p + dj * n + di);
      }
    }
    Ax = acc;
    diag = ri.m[1] * rj.m[1] + op.a * op.st9[4 * op.N + p];
    return;
  }
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

// (A x) and the diagonal at nodes (i, j, k) and (i, j, k + 1) of a 3D
// Galerkin level (has1: the second node exists).  The two share the row
// sums of planes k and k + 1, so a thread forms 12 of them instead of 18;
// each node adds its terms in level_apply's order, so both results are
// bitwise level_apply's.
template <class T, class C>
__device__ __forceinline__ void tensor3_apply2(const T* __restrict__ x, const LevelOp<C>& op, int p, int i, int j,
                                               int k, bool has1, C (&Ax)[2], C (&diag)[2]) {
  const int n = op.n, nn = n * n;
  const Tri3<C> ri = tri_row(op.tri, n, i), rj = tri_row(op.tri, n, j);
  C mi_at[3], ti_at[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mi_at[q] = ri.m[q] + op.a * ri.t[q];
    ti_at[q] = ri.m[q];
  }
  // row sums of planes k - 1 .. k + 2, rows j - 1 .. j + 1
  C pv[4][3], qv[4][3];
#pragma unroll
  for (int pk = 0; pk < 4; ++pk) {
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      pv[pk][dj + 1] = C(0);
      qv[pk][dj + 1] = C(0);
      const int kk = k - 1 + pk, jj = j + dj;
      if (kk < 0 || kk >= n || jj < 0 || jj >= n) continue;
      const int base = p + (pk - 1) * nn + dj * n;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int ii = i + di;
        if (ii < 0 || ii >= n) continue;
        const C xv = ld<T, C>(x + base + di);
        pv[pk][dj + 1] += mi_at[di + 1] * xv;
        qv[pk][dj + 1] += ti_at[di + 1] * xv;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    if (u == 1 && !has1) break;
    const int ku = k + u;
    const Tri3<C> rk = tri_row(op.tri, n, ku);
    C acc = C(0);
#pragma unroll
    for (int dk = -1; dk <= 1; ++dk) {
      const int kk = ku + dk;
      if (kk < 0 || kk >= n) continue;
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const int jj = j + dj;
        if (jj < 0 || jj >= n) continue;
        const C mm = rj.m[dj + 1] * rk.m[dk + 1];
        const C tm = rj.t[dj + 1] * rk.m[dk + 1] + rj.m[dj + 1] * rk.t[dk + 1];
        acc += mm * pv[u + dk + 1][dj + 1] + op.a * tm * qv[u + dk + 1][dj + 1];
      }
    }
    Ax[u] = acc;
    diag[u] = ri.m[1] * rj.m[1] * rk.m[1] +
              op.a * (ri.t[1] * rj.m[1] * rk.m[1] + ri.m[1] * rj.t[1] * rk.m[1] + ri.m[1] * rj.m[1] * rk.t[1]);
  }
}

// Thread t of a 3D Galerkin level owns nodes (i, j, 2 kp) and (i, j, 2 kp + 1).
__device__ __forceinline__ bool pair_coords(int t, int n, int& i, int& j, int& k, bool& has1) {
  const int nn = n * n, kp = t / nn, r = t - kp * nn;
  j = r / n;
  i = r - j * n;
  k = 2 * kp;
  has1 = k + 1 < n;
  return k < n;
}

// k_smooth on a 3D Galerkin level, two nodes (consecutive in z) per thread.
template <class T, class C>
__global__ __launch_bounds__(TPB) void k_smooth3t(const T* __restrict__ xin, int64_t sxin, T* xout, int64_t sxout,
                                                  const T* __restrict__ b, int64_t sb, LevelOp<C> op, C omega,
                                                  int zero_init) {
  int i, j, k;
  bool has1;
  if (!pair_coords(blockIdx.x * TPB + threadIdx.x, op.n, i, j, k, has1)) return;
  const int64_t inst = blockIdx.y;
  const int p = (k * op.n + j) * op.n + i, nn = op.n * op.n;
  const T* x = xin + inst * sxin;
  const T* bb = b + inst * sb;
  T* xo = xout + inst * sxout;
  if (zero_init) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (u == 0 || has1)
        st<T, C>(xo + p + u * nn, omega * ld<T, C>(bb + p + u * nn) / level_diag<3, KIND_TENSOR, C>(op, p + u * nn, i, j, k + u));
    return;
  }
  C Ax[2], d[2];
  tensor3_apply2<T, C>(x, op, p, i, j, k, has1, Ax, d);
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (u == 0 || has1)
      st<T, C>(xo + p + u * nn, ld<T, C>(x + p + u * nn) + omega * (ld<T, C>(bb + p + u * nn) - Ax[u]) / d[u]);
}

// k_residual on a 3D Galerkin level, two nodes (consecutive in z) per thread.
template <class T, class C>
__global__ __launch_bounds__(TPB) void k_residual3t(const T* __restrict__ x, int64_t sx, const T* __restrict__ b,
                                                    int64_t sb, T* __restrict__ r, int64_t sr, LevelOp<C> op) {
  int i, j, k;
  bool has1;
  if (!pair_coords(blockIdx.x * TPB + threadIdx.x, op.n, i, j, k, has1)) return;
  const int64_t inst = blockIdx.y;
  const int p = (k * op.n + j) * op.n + i, nn = op.n * op.n;
  C Ax[2], d[2];
  tensor3_apply2<T, C>(x + inst * sx, op, p, i, j, k, has1, Ax, d);
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (u == 0 || has1) st<T, C>(r + inst * sr + p + u * nn, ld<T, C>(b + inst * sb + p + u * nn) - Ax[u]);
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
  if constexpr (KIND == KIND_FINE) {
    // constant diagonal: the weighted inverse omega / d multiplies (the
    // form the 3D z-marches hoist out of their plane loop)
    const C wd = omega / level_diag<DIM, KIND, C>(op, p, i, j, k);
    if (zero_init) {
      out = wd * bp;
    } else {
      const T* x = xin + inst * sxin;
      C Ax, d;
      level_apply<DIM, KIND, T, C>(x, op, p, i, j, k, Ax, d);
      out = ld<T, C>(x + p) + wd * (bp - Ax);
    }
  } else if (zero_init) {
    out = omega * bp / level_diag<DIM, KIND, C>(op, p, i, j, k);
  } else {
    const T* x = xin + inst * sxin;
    C Ax, d;
    level_apply<DIM, KIND, T, C>(x, op, p, i, j, k, Ax, d);
    out = ld<T, C>(x + p) + omega * (bp - Ax) / d;
  }
  st<T, C>(xout + inst * sxout + p, out);
}

// x_out = x_in + P e_c (linear interpolation; coarse node I sits at fine 2I+1).
template <int DIM, class TX, class TE, class C>
__global__ __launch_bounds__(TPB) void k_prolong(const TX* xin, int64_t sxin, const TE* __restrict__ ec,
                                                 int64_t sec, TX* xout, int64_t sxout, int nf, int Nf,
                                                 int nc, C escale) {
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
  st<TX, C>(xout + inst * sxout + p, ld<TX, C>(xin + inst * sxin + p) + escale * acc);
}

// (P e)(i, j[, k]): linear interpolation of the coarse correction at a fine
// node (coarse node I sits at fine 2I+1; values past the grid are zero).
template <int DIM, class TE, class C>
__device__ __forceinline__ C prolong_at(const TE* __restrict__ e, int nc, int i, int j, int k) {
  int idx[3][2];
  C wt[3][2];
  int cnt[3];
  const int c[3] = {i, j, k};
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
  C acc = C(0);
  if (DIM == 2) {
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a) acc += wt[0][a] * wt[1][b] * ld<TE, C>(e + idx[1][b] * nc + idx[0][a]);
  } else {
    for (int q = 0; q < cnt[2]; ++q)
      for (int b = 0; b < cnt[1]; ++b)
        for (int a = 0; a < cnt[0]; ++a)
          acc += wt[0][a] * wt[1][b] * wt[2][q] * ld<TE, C>(e + ((int64_t)idx[2][q] * nc + idx[1][b]) * nc + idx[0][a]);
  }
  return acc;
}

// Residual at the 3^d fine nodes around each coarse node, full weighting:
// b_c = 2^{-d} sum w(d) (b - A x)(2I+1+d).  With `zero_next`, the coarse
// level's first Jacobi sweep from zero (pointwise) is fused: x_c = omega b_c / D_c.
template <int DIM, int KIND, class TF, class TC, class C>
__global__ __launch_bounds__(TPB) void k_resid_restrict(const TF* __restrict__ x, int64_t sx,
                                                        const TF* __restrict__ b, int64_t sb,
                                                        TC* __restrict__ bc, int64_t sbc, TC* __restrict__ xc,
                                                        int64_t sxc, LevelOp<C> opf, LevelOp<C> opc, C omega,
                                                        int zero_next, C bscale) {
  const int pc = blockIdx.x * TPB + threadIdx.x;
  if (pc >= opc.N) return;
  const int64_t inst = blockIdx.y;
  const int nf = opf.n, nc = opc.n;
  int I, J, K;
  node_coords<DIM>(pc, nc, I, J, K);
  const TF* xi = x + inst * sx;
  const TF* bi = b + inst * sb;
  const C w[3] = {C(0.5), C(1), C(0.5)};
  C acc = C(0);
  const int fi = 2 * I + 1, fj = 2 * J + 1, fk = 2 * K + 1;
  const int dk0 = DIM == 3 ? -1 : 0, dk1 = DIM == 3 ? 1 : 0;
  for (int dk = dk0; dk <= dk1; ++dk) {
    const int kk = fk + dk;
    if (DIM == 3 && kk >= nf) continue;
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = fj + dj;
      if (jj >= nf) continue;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int ii = fi + di;
        if (ii >= nf) continue;
        const int pf = DIM == 3 ? (kk * nf + jj) * nf + ii : jj * nf + ii;
        C Ax, d;
        level_apply<DIM, KIND, TF, C>(xi, opf, pf, ii, jj, DIM == 3 ? kk : 0, Ax, d);
        const C wt = DIM == 3 ? w[di + 1] * w[dj + 1] * w[dk + 1] : w[di + 1] * w[dj + 1];
        acc += wt * (ld<TF, C>(bi + pf) - Ax);
      }
    }
  }
  acc *= (DIM == 3 ? C(0.125) : C(0.25)) * bscale;
  st<TC, C>(bc + inst * sbc + pc, acc);
  if (zero_next) st<TC, C>(xc + inst * sxc + pc, omega * acc / level_diag<DIM, KIND_TENSOR, C>(opc, pc, I, J, K));
}

// r = b - A x at every node of a level (3D: the residual is formed once per
// node, then restricted by k_restrict; forming it at the 27 fine nodes
// around each coarse node would apply the 27-point operator 27 times).
template <int DIM, int KIND, class TF, class C>
__global__ __launch_bounds__(TPB) void k_residual(const TF* __restrict__ x, int64_t sx, const TF* __restrict__ b,
                                                  int64_t sb, TF* __restrict__ r, int64_t sr, LevelOp<C> op) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= op.N) return;
  const int64_t inst = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, op.n, i, j, k);
  C Ax, d;
  level_apply<DIM, KIND, TF, C>(x + inst * sx, op, p, i, j, k, Ax, d);
  st<TF, C>(r + inst * sr + p, ld<TF, C>(b + inst * sb + p) - Ax);
}

// Full weighting of a residual: b_c = 2^{-d} sum w(d) r(2I+1+d), scaled by
// bscale; with `zero_next` also the coarse level's first Jacobi sweep from
// zero, x_c = omega b_c / D_c.
template <int DIM, class TF, class TC, class C>
__global__ __launch_bounds__(TPB) void k_restrict(const TF* __restrict__ r, int64_t sr, TC* __restrict__ bc,
                                                  int64_t sbc, TC* __restrict__ xc, int64_t sxc, int nf,
                                                  LevelOp<C> opc, C omega, int zero_next, C bscale) {
  const int pc = blockIdx.x * TPB + threadIdx.x;
  if (pc >= opc.N) return;
  const int64_t inst = blockIdx.y;
  int I, J, K;
  node_coords<DIM>(pc, opc.n, I, J, K);
  const TF* ri = r + inst * sr;
  const C w[3] = {C(0.5), C(1), C(0.5)};
  const int fi = 2 * I + 1, fj = 2 * J + 1, fk = 2 * K + 1;
  const int dk0 = DIM == 3 ? -1 : 0, dk1 = DIM == 3 ? 1 : 0;
  C acc = C(0);
  for (int dk = dk0; dk <= dk1; ++dk) {
    const int kk = fk + dk;
    if (DIM == 3 && kk >= nf) continue;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int jj = fj + dj;
      if (jj >= nf) continue;
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int ii = fi + di;
        if (ii >= nf) continue;
        const int pf = DIM == 3 ? (kk * nf + jj) * nf + ii : jj * nf + ii;
        const C wt = DIM == 3 ? w[di + 1] * w[dj + 1] * w[dk + 1] : w[di + 1] * w[dj + 1];
        acc += wt * ld<TF, C>(ri + pf);
      }
    }
  }
  acc *= (DIM == 3 ? C(0.125) : C(0.25)) * bscale;
  st<TC, C>(bc + inst * sbc + pc, acc);
  if (zero_next) st<TC, C>(xc + inst * sxc + pc, omega * acc / level_diag<DIM, KIND_TENSOR, C>(opc, pc, I, J, K));
}

// Fine level: x_out = y + omega D^{-1} (b - A y) with y = x_in + P e_c formed
// on the fly at the node and its stencil neighbours (prolongation fused into
// the first post-smoothing sweep).
template <int DIM, bool VK, class TX, class TE, class C>
__global__ __launch_bounds__(TPB) void k_prolong_smooth(const TX* __restrict__ xin, int64_t sxin,
                                                        const TE* __restrict__ ec, int64_t sec,
                                                        const TX* __restrict__ b, int64_t sb, TX* __restrict__ xout,
                                                        int64_t sxout, LevelOp<C> op, int nc, C omega, C escale) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= op.N) return;
  const int64_t inst = blockIdx.y;
  const int n = op.n;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const TX* xi = xin + inst * sxin;
  const TE* e = ec + inst * sec;
  auto y = [&](int q, int qi, int qj, int qk) {
    return ld<TX, C>(xi + q) + escale * prolong_at<DIM, TE, C>(e, nc, qi, qj, qk);
  };
  const C yp = y(p, i, j, k);
  const C xm = i > 0 ? y(p - 1, i - 1, j, k) : C(0);
  const C xp = i + 1 < n ? y(p + 1, i + 1, j, k) : C(0);
  const C ym = j > 0 ? y(p - n, i, j - 1, k) : C(0);
  const C yq = j + 1 < n ? y(p + n, i, j + 1, k) : C(0);
  C zm = C(0), zp = C(0);
  if (DIM == 3) {
    const int nn = n * n;
    zm = k > 0 ? y(p - nn, i, j, k - 1) : C(0);
    zp = k + 1 < n ? y(p + nn, i, j, k + 1) : C(0);
  }
  C kx;
  if (!VK) {
    kx = C(2 * DIM) * yp - xm - xp - ym - yq;
    if (DIM == 3) kx -= zm + zp;
  } else {
    const Faces<C>& fc = op.faces;
    kx = fc.m[0][p] * (yp - xm) + fc.p[0][p] * (yp - xp) + fc.m[1][p] * (yp - ym) + fc.p[1][p] * (yp - yq);
    if (DIM == 3) kx += fc.m[2][p] * (yp - zm) + fc.p[2][p] * (yp - zp);
  }
  const C Ay = yp + op.a * op.ih2 * kx;
  const C d = level_diag<DIM, VK ? KIND_FINE_VK : KIND_FINE, C>(op, p, i, j, k);
  st<TX, C>(xout + inst * sxout + p, yp + omega * (ld<TX, C>(b + inst * sb + p) - Ay) / d);
}

// ---------------------------------------------------------------------------
// 2D LDS-tiled level kernels.  One "down" kernel per level does the first
// sweep from zero (pointwise), the remaining pre-smoothing sweeps, the
// residual and the full-weighting restriction; one "up" kernel does the
// prolongation and all post-smoothing sweeps.  Each workgroup loads its tile
// with a halo wide enough that every sweep can be recomputed locally (the
// halo work is redundant, the results are those of the separate sweeps).
// ---------------------------------------------------------------------------
constexpr int TCX = 16, TCY = 8;   // coarse nodes per down tile; fine tile is 2x
// Batched launches with FP32 arithmetic use TY0 coarse rows per tile: less
// halo and padding work per owned node (1.5x instead of 2x) in the HBM-bound
// batched sweeps; the LDS of an FP64 tile that tall would exceed 64 KiB.
constexpr int TY0 = 16;

// Shared memory of one tile with halo R: right-hand side, two iterates, and
// the operator staged for the sweeps (omega / diagonal per node; face
// coefficients times a/h^2 for variable kappa; the 1D Galerkin factor rows of
// the tile's columns and rows for tensor levels).  Every global load of a
// tile is issued up front, so a workgroup waits for memory once.
//
// Node t of the W x H tile (t = tx + W ty) lives at index G + t of each
// per-node array, which is padded to a whole number of 256-node rows (NP)
// plus a guard of G = W + 1 entries on both sides: every thread's nodes and
// their stencil neighbours are in bounds, so the sweeps run without
// branches, computing every node and selecting zero where a node is not
// updated (the tile border, nodes outside the domain, the padding).
template <int KIND, int R, class C, int TY>
struct Tile {
  static constexpr int W = 2 * TCX + 1 + 2 * R, H = 2 * TY + 1 + 2 * R, NE = W * H;
  static constexpr int IT = (NE + 255) / 256, NP = IT * 256, G = W + 1, NS = NP + 2 * G;
  static constexpr bool VK = KIND == KIND_FINE_VK, TEN = KIND == KIND_TENSOR, S9 = KIND == KIND_STENCIL9;
  C b[NS], x0[NS], x1[NS];
  C idg[KIND == KIND_FINE ? 1 : NS];
  C f[VK ? 4 * NS : 1];
  C cx[TEN ? 6 * W : (S9 ? 3 * W : 1)];  // per column: (M + a T)(i, i+d), M(i, i+d), d = -1, 0, 1 (S9: M only)
  C cy[TEN ? 6 * H : (S9 ? 3 * H : 1)];  // per row:    M(j, j+d), a T(j, j+d) (S9: M only)
};

// The nodes of a tile one thread handles: element it is node
// t = threadIdx.x + 256 it, at tile coordinates (tx, ty) (clamped into the
// tile for padding nodes); bit it of `dom` is set for a node of the tile
// inside the domain, of `inner` for one that is also off the tile border.
template <int IT>
struct Elems {
  int tx[IT], ty[IT];
  unsigned dom, inner;
};

template <int KIND, int R, class C, int TY>
__device__ __forceinline__ Elems<Tile<KIND, R, C, TY>::IT> tile_elems(int ox, int oy, int n) {
  using T = Tile<KIND, R, C, TY>;
  Elems<T::IT> e;
  e.dom = 0;
  e.inner = 0;
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = threadIdx.x + it * 256;
    const bool valid = t < T::NE;
    const int tx = t % T::W, ty = valid ? t / T::W : T::H - 1;
    e.tx[it] = tx;
    e.ty[it] = ty;
    const int gi = ox + tx, gj = oy + ty;
    const bool d = valid && gi >= 0 && gi < n && gj >= 0 && gj < n;
    const bool in = d && tx > 0 && tx < T::W - 1 && ty > 0 && ty < T::H - 1;
    e.dom |= (unsigned)d << it;
    e.inner |= (unsigned)in << it;
  }
  return e;
}

// The 9 operator coefficients of the nodes a thread sweeps, for the Galerkin
// kinds (KIND_TENSOR, KIND_STENCIL9): entry (dj+1)*3 + (di+1) multiplies x
// at (di, dj).  Loaded (stencil part, before the tile barrier) and completed
// from the staged factor rows (after it), then reused by every sweep.
template <int KIND, int IT, class C>
struct Coef9 {
  C v[IT][(KIND == KIND_STENCIL9 || KIND == KIND_TENSOR) ? 9 : 1];
};

template <int KIND, int R, class C, int TY>
__device__ __forceinline__ void tile_load_coef(Coef9<KIND, Tile<KIND, R, C, TY>::IT, C>& k9, const LevelOp<C>& op, int ox,
                                               int oy, const Elems<Tile<KIND, R, C, TY>::IT>& el) {
  using T = Tile<KIND, R, C, TY>;
  if constexpr (T::S9) {
    const int n = op.n;
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const bool in = (el.dom >> it) & 1u;
      const int64_t g = in ? (int64_t)(oy + el.ty[it]) * n + ox + el.tx[it] : 0;
#pragma unroll
      for (int d = 0; d < 9; ++d) k9.v[it][d] = in ? op.a * op.st9[d * op.N + g] : C(0);
    }
  }
}

// Stage the operator of the tile whose origin is (ox, oy) into LDS.  Loads
// only; the caller synchronizes.
template <int KIND, int R, class C, int TY>
__device__ __forceinline__ void tile_stage_op(Tile<KIND, R, C, TY>& sm, const LevelOp<C>& op, int ox, int oy,
                                              const Elems<Tile<KIND, R, C, TY>::IT>& el) {
  using T = Tile<KIND, R, C, TY>;
  constexpr int W = T::W, H = T::H;
  const int tid = threadIdx.x, n = op.n;
  if constexpr (T::VK) {
    const C s = op.a * op.ih2;
    C fv[4][T::IT];
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const bool in = (el.dom >> it) & 1u;
      const int64_t g = in ? (int64_t)(oy + el.ty[it]) * n + ox + el.tx[it] : 0;
      fv[0][it] = in ? op.faces.m[0][g] : C(0);
      fv[1][it] = in ? op.faces.p[0][g] : C(0);
      fv[2][it] = in ? op.faces.m[1][g] : C(0);
      fv[3][it] = in ? op.faces.p[1][g] : C(0);
    }
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const int t = tid + it * 256;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.f[q * T::NS + T::G + t] = s * fv[q][it];
    }
  }
  if constexpr (T::S9) {
    for (int t = tid; t < 3 * W + 3 * H; t += 256) {
      if (t < 3 * W) {
        const int d = t / W, c = t % W, gi = ox + c;
        sm.cx[d * W + c] = (gi >= 0 && gi < n) ? op.tri[d * n + gi] : C(0);
      } else {
        const int u = t - 3 * W, d = u / H, r = u % H, gj = oy + r;
        sm.cy[d * H + r] = (gj >= 0 && gj < n) ? op.tri[d * n + gj] : C(0);
      }
    }
  }
  if constexpr (T::TEN) {
    // columns: 6 W values, rows: 6 H values (W, H < 256 for R <= 4)
    for (int t = tid; t < 3 * W + 3 * H; t += 256) {
      if (t < 3 * W) {
        const int d = t / W, c = t % W, gi = ox + c;
        const bool in = gi >= 0 && gi < n;
        const C m = in ? op.tri[d * n + gi] : C(0), tt = in ? op.tri[(3 + d) * n + gi] : C(0);
        sm.cx[d * W + c] = m + op.a * tt;
        sm.cx[(3 + d) * W + c] = m;
      } else {
        const int u = t - 3 * W, d = u / H, r = u % H, gj = oy + r;
        const bool in = gj >= 0 && gj < n;
        sm.cy[d * H + r] = in ? op.tri[d * n + gj] : C(0);
        sm.cy[(3 + d) * H + r] = in ? op.a * op.tri[(3 + d) * n + gj] : C(0);
      }
    }
  }
}

template <int KIND, int R, class C, int TY>
__device__ __forceinline__ void tile_finish_coef(Coef9<KIND, Tile<KIND, R, C, TY>::IT, C>& k9,
                                                 const Tile<KIND, R, C, TY>& sm,
                                                 const Elems<Tile<KIND, R, C, TY>::IT>& el) {
  using T = Tile<KIND, R, C, TY>;
  if constexpr (T::S9 || T::TEN) {
    constexpr int W = T::W, H = T::H;
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const int tx = el.tx[it], ty = el.ty[it];
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          C& k = k9.v[it][(dj + 1) * 3 + di + 1];
          if constexpr (T::TEN)   // M_j (M + aT)_i + a T_j M_i
            k = sm.cy[(dj + 1) * H + ty] * sm.cx[(di + 1) * W + tx] + sm.cy[(4 + dj) * H + ty] * sm.cx[(4 + di) * W + tx];
          else                    // M_j M_i + a K (loaded)
            k += sm.cy[(dj + 1) * H + ty] * sm.cx[(di + 1) * W + tx];
        }
    }
  }
}

// Diagonal of the level operator at tile node t (per-node arrays offset by G).
template <int KIND, int R, class C, int TY>
__device__ __forceinline__ C tile_diag(const Tile<KIND, R, C, TY>& sm, const LevelOp<C>& op, int t, const C* kc) {
  using T = Tile<KIND, R, C, TY>;
  if constexpr (KIND == KIND_FINE) return C(1) + op.a * op.ih2 * C(4);
  else if constexpr (T::S9 || T::TEN)
    return kc[4];
  else if constexpr (T::VK) {
    const C* f = sm.f + T::G + t;
    return C(1) + f[0] + f[T::NS] + f[2 * T::NS] + f[3 * T::NS];
  } else
    return C(0);
}

// (A x)_t for tile node t; x points at node 0 of a per-node array.  Every
// neighbour index is inside the padded array; the value is only used for
// nodes whose 8 neighbours are tile nodes.
template <int KIND, int R, class C, int TY>
__device__ __forceinline__ C tile_Ax(const Tile<KIND, R, C, TY>& sm, const C* __restrict__ x, const LevelOp<C>& op, int t,
                                     const C* kc) {
  using T = Tile<KIND, R, C, TY>;
  constexpr int W = T::W;
  const C c = x[t];
  if constexpr (T::S9 || T::TEN) {
    C acc = C(0);
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) acc += kc[(dj + 1) * 3 + di + 1] * x[t + dj * W + di];
    return acc;
  } else if constexpr (KIND == KIND_FINE) {
    return c + op.a * op.ih2 * (C(4) * c - x[t - 1] - x[t + 1] - x[t - W] - x[t + W]);
  } else {
    const C* f = sm.f + T::G + t;
    return c + f[0] * (c - x[t - 1]) + f[T::NS] * (c - x[t + 1]) + f[2 * T::NS] * (c - x[t - W]) +
           f[3 * T::NS] * (c - x[t + W]);
  }
}

// One weighted Jacobi sweep cur -> nxt over the tile (cur, nxt at node 0;
// border, out-of-domain and padding nodes become zero).
template <int KIND, int R, class C, int TY>
__device__ __forceinline__ void tile_sweep(Tile<KIND, R, C, TY>& sm, const C* cur, C* nxt, const LevelOp<C>& op, C omega,
                                           const Coef9<KIND, Tile<KIND, R, C, TY>::IT, C>& k9,
                                           const Elems<Tile<KIND, R, C, TY>::IT>& el) {
  using T = Tile<KIND, R, C, TY>;
  const C idc = omega / (C(1) + op.a * op.ih2 * C(4));
  const C* b = sm.b + T::G;
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = threadIdx.x + it * 256;
    const C id = KIND == KIND_FINE ? idc : sm.idg[KIND == KIND_FINE ? 0 : T::G + t];
    const C v = cur[t] + id * (b[t] - tile_Ax<KIND, R, C, TY>(sm, cur, op, t, k9.v[it]));
    nxt[t] = ((el.inner >> it) & 1u) ? v : C(0);
  }
}

// omega / diagonal for every tile node (zero outside the domain); after the
// operator is staged.
template <int KIND, int R, class C, int TY>
__device__ __forceinline__ void tile_inv_diag(Tile<KIND, R, C, TY>& sm, const LevelOp<C>& op, C omega,
                                              const Coef9<KIND, Tile<KIND, R, C, TY>::IT, C>& k9,
                                              const Elems<Tile<KIND, R, C, TY>::IT>& el) {
  using T = Tile<KIND, R, C, TY>;
  if constexpr (KIND != KIND_FINE) {
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const int t = threadIdx.x + it * 256;
      const C v = omega / tile_diag<KIND, R, C, TY>(sm, op, t, k9.v[it]);
      sm.idg[T::G + t] = ((el.dom >> it) & 1u) ? v : C(0);
    }
  }
}

// Rana's coupling terms of a stage solve, formed on the fly in the level-0
// down kernel: the right-hand side is b - sum_{l < NZ} c_l K z_l.
template <class TF, class C>
struct CplArgs {
  const TF* z;        // z_0 of instance 0
  int64_t sz, zs;     // instance stride, stride between z_l
  C c[SMAX - 1];      // tau L_il
  TF* out;            // the formed right-hand side (owned nodes written)
  int64_t so;
};

// Down: x_NU (from zero, or from x0 when given) -> xout, and
// b_c = R (b - A x_NU) -> bc, on the fine nodes of coarse tile (I0.., J0..).
// NZ > 0 (level 0 only): b is first replaced by b - sum_l c_l K z_l, staged
// with one more halo ring of each z_l, and written to cpl.out.
template <int KIND, int NU, class TF, class TC, class C, int NZ, int TY>
__global__ __launch_bounds__(256) void k_down2d(const TF* __restrict__ b, int64_t sb, const TF* __restrict__ x0,
                                                int64_t sx0, TF* __restrict__ xout, int64_t sxo, TC* __restrict__ bc,
                                                int64_t sbc, LevelOp<C> op, int nc, C omega, int gx, int gy,
                                                CplArgs<TF, C> cpl, C bscale) {
  constexpr int R = NU + 1;
  using T = Tile<KIND, R, C, TY>;
  constexpr int W = T::W, G = T::G;
  constexpr int ZW = W + 2, ZH = T::H + 2, ZNE = NZ > 0 ? ZW * ZH : 1, ZIT = (ZNE + 255) / 256;
  static_assert(NZ == 0 || KIND == KIND_FINE || KIND == KIND_FINE_VK, "coupling terms live on level 0");
  __shared__ T sm;
  __shared__ C szt[NZ > 0 ? NZ : 1][ZNE];
  const int tid = threadIdx.x;
  const int nf = op.n;
  const int L = xcd_tile((int)blockIdx.x, (int)gridDim.x);  // grid: gx * gy tiles per block
  const int I0 = (L % gx) * TCX, J0 = ((L / gx) % gy) * TY;
  const int64_t inst = L / (gx * gy);
  const int ox = 2 * I0 - R, oy = 2 * J0 - R;
  const TF* bi = b + inst * sb;
  const TF* xi = x0 ? x0 + inst * sx0 : nullptr;
  const Elems<T::IT> el = tile_elems<KIND, R, C, TY>(ox, oy, nf);
  Coef9<KIND, T::IT, C> k9;
  tile_load_coef<KIND, R, C, TY>(k9, op, ox, oy, el);
  C bv[T::IT], xv[T::IT];
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const bool in = (el.dom >> it) & 1u;
    const int64_t g = in ? (int64_t)(oy + el.ty[it]) * nf + ox + el.tx[it] : 0;
    bv[it] = in ? ld<TF, C>(bi + g) : C(0);
    xv[it] = (in && xi) ? ld<TF, C>(xi + g) : C(0);
  }
  if constexpr (NZ > 0) {
    C zv[NZ][ZIT];
#pragma unroll
    for (int l = 0; l < NZ; ++l)
#pragma unroll
      for (int it = 0; it < ZIT; ++it) {
        const int t = tid + it * 256, gi = ox - 1 + t % ZW, gj = oy - 1 + t / ZW;
        const bool in = t < ZNE && gi >= 0 && gi < nf && gj >= 0 && gj < nf;
        zv[l][it] = in ? ld<TF, C>(cpl.z + inst * cpl.sz + l * cpl.zs + (int64_t)gj * nf + gi) : C(0);
      }
#pragma unroll
    for (int l = 0; l < NZ; ++l)
#pragma unroll
      for (int it = 0; it < ZIT; ++it) {
        const int t = tid + it * 256;
        if (t < ZNE) szt[l][t] = zv[l][it];
      }
  }
  tile_stage_op<KIND, R, C, TY>(sm, op, ox, oy, el);
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    sm.b[G + t] = bv[it];
    sm.x0[G + t] = xv[it];
  }
  __syncthreads();
  const int hx = (I0 + TCX >= nc) ? nf : 2 * (I0 + TCX), hy = (J0 + TY >= nc) ? nf : 2 * (J0 + TY);
  if constexpr (NZ > 0) {
    // b <- b - sum_l c_l K z_l at every in-domain tile node (each thread
    // updates only the nodes it reads later); owned nodes go to cpl.out
    const C inv_a = C(1) / op.a;
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      if ((el.dom >> it) & 1u) {
        const int t = tid + it * 256, tx = el.tx[it], ty = el.ty[it], gi = ox + tx, gj = oy + ty;
        const int zt = (ty + 1) * ZW + tx + 1;
        C acc = sm.b[G + t];
#pragma unroll
        for (int l = 0; l < NZ; ++l) {
          const C* z = szt[l];
          const C c0 = z[zt];
          C kz;
          if constexpr (KIND == KIND_FINE) {
            kz = op.ih2 * (C(4) * c0 - z[zt - 1] - z[zt + 1] - z[zt - ZW] - z[zt + ZW]);
          } else {   // staged face coefficients carry a / h^2
            const C* f = sm.f + G + t;
            kz = inv_a * (f[0] * (c0 - z[zt - 1]) + f[T::NS] * (c0 - z[zt + 1]) + f[2 * T::NS] * (c0 - z[zt - ZW]) +
                          f[3 * T::NS] * (c0 - z[zt + ZW]));
          }
          acc -= cpl.c[l] * kz;
        }
        sm.b[G + t] = acc;
        if (gi >= 2 * I0 && gi < hx && gj >= 2 * J0 && gj < hy)
          st<TF, C>(cpl.out + inst * cpl.so + (int64_t)gj * nf + gi, acc);
      }
    }
  }
  tile_finish_coef<KIND, R, C, TY>(k9, sm, el);
  tile_inv_diag<KIND, R, C, TY>(sm, op, omega, k9, el);
  C* cur = sm.x0 + G;
  C* nxt = sm.x1 + G;
  const C* bt = sm.b + G;
  int k = 0;
  if (!x0) {
    // first sweep from zero is pointwise: x = omega D^{-1} b
    __syncthreads();
    const C idc = omega / (C(1) + op.a * op.ih2 * C(4));
#pragma unroll
    for (int it = 0; it < T::IT; ++it) {
      const int t = tid + it * 256;
      const C id = KIND == KIND_FINE ? idc : sm.idg[KIND == KIND_FINE ? 0 : G + t];
      cur[t] = ((el.dom >> it) & 1u) ? id * bt[t] : C(0);
    }
    k = 1;
  }
  __syncthreads();
  for (; k < NU; ++k) {
    tile_sweep<KIND, R, C, TY>(sm, cur, nxt, op, omega, k9, el);
    __syncthreads();
    C* tmp = cur; cur = nxt; nxt = tmp;
  }
  // residual on the interior of the tile (zero elsewhere)
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    const C v = bt[t] - tile_Ax<KIND, R, C, TY>(sm, cur, op, t, k9.v[it]);
    nxt[t] = ((el.inner >> it) & 1u) ? v : C(0);
  }
  __syncthreads();
  for (int c = tid; c < TCX * TY; c += 256) {
    const int cx = c % TCX, cy = c / TCX, I = I0 + cx, J = J0 + cy;
    if (I >= nc || J >= nc) continue;
    const int tc = (2 * cy + 1 + R) * W + (2 * cx + 1 + R);
    const C acc = C(0.25) * bscale *
                  (nxt[tc] + C(0.5) * (nxt[tc - 1] + nxt[tc + 1] + nxt[tc - W] + nxt[tc + W]) +
                   C(0.25) * (nxt[tc - W - 1] + nxt[tc - W + 1] + nxt[tc + W - 1] + nxt[tc + W + 1]));
    st<TC, C>(bc + inst * sbc + J * nc + I, acc);
  }
  // owned fine nodes: [2 I0, 2 (I0 + TCX)) per axis, the last tile to the end
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    const int gi = ox + el.tx[it], gj = oy + el.ty[it];
    if (((el.dom >> it) & 1u) && gi >= 2 * I0 && gi < hx && gj >= 2 * J0 && gj < hy)
      st<TF, C>(xout + inst * sxo + (int64_t)gj * nf + gi, cur[t]);
  }
}

// floor(v / 2) for any sign
__device__ __forceinline__ int floor_half(int v) { return v >= 0 ? v / 2 : -((1 - v) / 2); }

// Up: y = x_in + P e on the tile (with halo NU), NU smoothing sweeps, the
// owned fine nodes written to xout.  The coarse correction of the tile is
// staged in LDS; fine node g takes lo = floor((g - 1) / 2) with weight 1
// (odd g) or lo and lo + 1 with weights 1/2 (even g) along each axis.
template <int KIND, int NU, class TF, class TE, class C, int TY>
__global__ __launch_bounds__(256) void k_up2d(const TF* __restrict__ xin, int64_t sxi, const TE* __restrict__ e,
                                              int64_t se, const TF* __restrict__ b, int64_t sb, TF* __restrict__ xout,
                                              int64_t sxo, LevelOp<C> op, int nc, C omega, int gx, int gy,
                                              C escale) {
  constexpr int R = NU;
  using T = Tile<KIND, R, C, TY>;
  constexpr int G = T::G;
  constexpr int CW = TCX + R + 3, CH = TY + R + 3, CNE = CW * CH, CIT = (CNE + 255) / 256;
  __shared__ T sm;
  __shared__ C sec[CNE];
  const int tid = threadIdx.x;
  const int nf = op.n;
  const int L = xcd_tile((int)blockIdx.x, (int)gridDim.x);  // grid: gx * gy tiles per block
  const int I0 = (L % gx) * TCX, J0 = ((L / gx) % gy) * TY;
  const int64_t inst = L / (gx * gy);
  const int ox = 2 * I0 - R, oy = 2 * J0 - R;
  const int cx0 = floor_half(ox - 1), cy0 = floor_half(oy - 1);
  const Elems<T::IT> el = tile_elems<KIND, R, C, TY>(ox, oy, nf);
  Coef9<KIND, T::IT, C> k9;
  tile_load_coef<KIND, R, C, TY>(k9, op, ox, oy, el);
  C bv[T::IT], xv[T::IT], ev[CIT];
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const bool in = (el.dom >> it) & 1u;
    const int64_t g = in ? (int64_t)(oy + el.ty[it]) * nf + ox + el.tx[it] : 0;
    bv[it] = in ? ld<TF, C>(b + inst * sb + g) : C(0);
    xv[it] = in ? ld<TF, C>(xin + inst * sxi + g) : C(0);
  }
#pragma unroll
  for (int it = 0; it < CIT; ++it) {
    const int t = tid + it * 256, I = cx0 + t % CW, J = cy0 + t / CW;
    const bool in = t < CNE && I >= 0 && I < nc && J >= 0 && J < nc;
    ev[it] = in ? escale * ld<TE, C>(e + inst * se + (int64_t)J * nc + I) : C(0);
  }
  tile_stage_op<KIND, R, C, TY>(sm, op, ox, oy, el);
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    sm.b[G + t] = bv[it];
    sm.x1[G + t] = xv[it];
  }
#pragma unroll
  for (int it = 0; it < CIT; ++it) {
    const int t = tid + it * 256;
    if (t < CNE) sec[t] = ev[it];
  }
  __syncthreads();
  tile_finish_coef<KIND, R, C, TY>(k9, sm, el);
  tile_inv_diag<KIND, R, C, TY>(sm, op, omega, k9, el);
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    const int gi = ox + el.tx[it], gj = oy + el.ty[it];
    const int li = floor_half(gi - 1), lj = floor_half(gj - 1);
    const C wi0 = (gi & 1) ? C(1) : C(0.5), wi1 = (gi & 1) ? C(0) : C(0.5);
    const C wj0 = (gj & 1) ? C(1) : C(0.5), wj1 = (gj & 1) ? C(0) : C(0.5);
    const int c = (lj - cy0) * CW + (li - cx0);
    const C pe = wj0 * (wi0 * sec[c] + wi1 * sec[c + 1]) + wj1 * (wi0 * sec[c + CW] + wi1 * sec[c + CW + 1]);
    sm.x0[G + t] = ((el.dom >> it) & 1u) ? sm.x1[G + t] + pe : C(0);
  }
  __syncthreads();
  C* cur = sm.x0 + G;
  C* nxt = sm.x1 + G;
  for (int k = 0; k < NU; ++k) {
    tile_sweep<KIND, R, C, TY>(sm, cur, nxt, op, omega, k9, el);
    __syncthreads();
    C* tmp = cur; cur = nxt; nxt = tmp;
  }
  const int hx = (I0 + TCX >= nc) ? nf : 2 * (I0 + TCX), hy = (J0 + TY >= nc) ? nf : 2 * (J0 + TY);
#pragma unroll
  for (int it = 0; it < T::IT; ++it) {
    const int t = tid + it * 256;
    const int gi = ox + el.tx[it], gj = oy + el.ty[it];
    if (((el.dom >> it) & 1u) && gi >= 2 * I0 && gi < hx && gj >= 2 * J0 && gj < hy)
      st<TF, C>(xout + inst * sxo + (int64_t)gj * nf + gi, cur[t]);
  }
}

// Up on level 0 of the constant-coefficient finite-difference operator,
// row-marching.  One wave owns OW = 64 - 2 NU adjacent columns (lane =
// column) and SEG rows of one instance, and computes NU more columns on
// each side and NU more rows below and above: the halo its sweeps consume
// (values there are wrong by the missing outer neighbours, which reach no
// owned node within NU sweeps).  The wave walks up the rows: row j takes
// x_in + P e, sweep k updates row j - k from a window of three rows of
// sweep k - 1 kept in registers, x neighbours come from the adjacent lanes,
// and the loads of rows j + 1 .. j + MPD are in flight meanwhile.  Each
// node takes the same arithmetic as in k_up2d, with no LDS staging and no
// barrier.  Coarse rows of the bilinear prolongation: fine rows 2m - 1 and
// 2m use coarse rows m - 1 (weight 1, resp. 1/2) and m (0, resp. 1/2).
constexpr int MPD = 4;    // rows fetched ahead

// x neighbours of the march: the value of lane - 1 (wave_shr:1) and of lane
// + 1 (wave_shl:1) as DPP moves, with no LDS traffic; the lane without a
// source keeps its own value.  An inactive source lane also leaves the
// lane's own value, so these run with every lane of the wave active (never
// under a lane-dependent condition).
__device__ __forceinline__ int dpp_left(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_right(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_left((int)(b & 0xffffffffll)), hi = dpp_left((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_right((int)(b & 0xffffffffll)), hi = dpp_right((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The operator of a row-marching kernel at one lane's column g, with the
// arithmetic of the tiles.  KIND_FINE: I + a K, K the 5-point Laplacian
// over h^2.  KIND_TENSOR: the Galerkin level with coefficient
// M_y(j, dj) (M + a T)_x(g, di) + a T_y(j, dj) M_x(g, di) on x(j + dj, g + di),
// the 1D factors staged per column (this lane) and per row (a Row, fetched
// with the row's other loads).  Ax takes the window of rows j - 1, j, j + 1.
template <int KIND, class C>
struct MarchOp;

template <class C>
struct MarchOp<KIND_FINE, C> {
  struct Row {};
  C s, idc;
  __device__ MarchOp(const LevelOp<C>& op, C omega, int, bool)
      : s(op.a * op.ih2), idc(omega / (C(1) + op.a * op.ih2 * C(4))) {}
  __device__ Row row(const LevelOp<C>&, int) const { return {}; }
  __device__ C Ax(const C* w, const Row&) const {
    const C c = w[1];
    const C xl = from_left(c), xr = from_right(c);
    return c + s * (C(4) * c - xl - xr - w[0] - w[2]);
  }
  __device__ C inv_diag(const Row&) const { return idc; }
};

template <class C>
struct MarchOp<KIND_TENSOR, C> {
  struct Row { C m[3], t[3]; };   // M_y(j, j + d - 1), a T_y(j, j + d - 1)
  C xa[3], xm[3];                 // (M + a T)_x(g, g + d - 1), M_x(g, g + d - 1)
  C omega;
  __device__ MarchOp(const LevelOp<C>& op, C om, int g, bool colin) : omega(om) {
    const int gc = colin ? g : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const C m = op.tri[d * op.n + gc], tt = op.tri[(3 + d) * op.n + gc];
      xa[d] = colin ? m + op.a * tt : C(0);
      xm[d] = colin ? m : C(0);
    }
  }
  __device__ Row row(const LevelOp<C>& op, int j) const {
    Row r;
    const bool in = j >= 0 && j < op.n;
    const int jc = in ? j : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const C m = op.tri[d * op.n + jc], tt = op.tri[(3 + d) * op.n + jc];
      r.m[d] = in ? m : C(0);
      r.t[d] = in ? op.a * tt : C(0);
    }
    return r;
  }
  __device__ C Ax(const C* w, const Row& r) const {
    C x[3][3];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj) {
      x[dj][0] = from_left(w[dj]);
      x[dj][1] = w[dj];
      x[dj][2] = from_right(w[dj]);
    }
    C acc = C(0);
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
      for (int di = 0; di < 3; ++di) acc += (r.m[dj] * xa[di] + r.t[dj] * xm[di]) * x[dj][di];
    return acc;
  }
  __device__ C inv_diag(const Row& r) const { return omega / (r.m[1] * xa[1] + r.t[1] * xm[1]); }
};

template <int KIND, int NU, class TF, class TE, class C, int SEG>
__global__ __launch_bounds__(256) void k_up2d_march(const TF* __restrict__ xin, int64_t sxi, const TE* __restrict__ e,
                                                    int64_t se, const TF* __restrict__ b, int64_t sb,
                                                    TF* __restrict__ xout, int64_t sxo, LevelOp<C> op, int nc,
                                                    C omega, int nstrips, int nsegs, int64_t units, C escale) {
  constexpr int OW = 64 - 2 * NU;
  const int64_t u = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 4 + (threadIdx.x >> 6);
  if (u >= units) return;   // whole wave
  const int lane = threadIdx.x & 63;
  const int strip = (int)(u % nstrips);
  const int64_t rest = u / nstrips;
  const int seg = (int)(rest % nsegs);
  const int64_t inst = rest / nsegs;
  const int n = op.n;
  const int g = strip * OW - NU + lane;
  const bool colin = g >= 0 && g < n;
  const bool own = colin && lane >= NU && lane < 64 - NU;
  const int j0 = seg * SEG, j1 = j0 + SEG < n ? j0 + SEG : n;
  const int jlo = j0 - NU, jlast = j1 - 1 + NU;
  const int li = floor_half(g - 1);
  const bool cin0 = colin && li >= 0 && li < nc, cin1 = colin && li + 1 >= 0 && li + 1 < nc;
  const C wi0 = (g & 1) ? C(1) : C(0.5), wi1 = (g & 1) ? C(0) : C(0.5);
  const TF* xi = xin + inst * sxi;
  const TF* bi = b + inst * sb;
  const TE* ei = e + inst * se;
  TF* xo = xout + inst * sxo;
  const MarchOp<KIND, C> mop(op, omega, g, colin);
  using Row = typename MarchOp<KIND, C>::Row;
  // Loads are unconditional from a clamped in-bounds address and masked
  // afterwards, so that no branch (and no wait) separates a fetch from the
  // rows computed meanwhile.  Coarse values stay unscaled until used.
  const int lic0 = cin0 ? li : 0, lic1 = cin1 ? li + 1 : 0;
  auto hrow = [&](int J) -> C {
    const bool jin = J >= 0 && J < nc;
    const int64_t o = jin ? (int64_t)J * nc : 0;
    const C e0 = ld<TE, C>(ei + o + lic0), e1 = ld<TE, C>(ei + o + lic1);
    return wi0 * ((jin && cin0) ? escale * e0 : C(0)) + wi1 * ((jin && cin1) ? escale * e1 : C(0));
  };
  C qx[MPD], qb[MPD], qe0[MPD], qe1[MPD];
  bool qin[MPD], qjin[MPD];
  auto fetch = [&](int r, int q) {
    const bool rin = colin && r >= 0 && r < n && r <= jlast;
    const int64_t o = rin ? (int64_t)r * n + g : 0;
    qx[q] = ld<TF, C>(xi + o);
    qb[q] = ld<TF, C>(bi + o);
    qin[q] = rin;
    const int J = floor_half(r - 1) + 1;
    const bool jin = r <= jlast && J >= 0 && J < nc;
    const int64_t oc = jin ? (int64_t)J * nc : 0;
    qe0[q] = ld<TE, C>(ei + oc + lic0);
    qe1[q] = ld<TE, C>(ei + oc + lic1);
    qjin[q] = jin;
  };
#pragma unroll
  for (int q = 0; q < MPD; ++q) fetch(jlo + q, q);
  C hlo = hrow(floor_half(jlo - 1)), hhi = hlo;
  C X[NU > 1 ? NU : 1][3];   // X[k]: sweep k at rows j - k - 2, j - k - 1, j - k
  C Bw[NU + 1];              // b at rows j, j - 1, .., j - NU
  Row Rw[NU + 1];            // operator rows j, j - 1, .., j - NU
  Row rnext = mop.row(op, jlo);   // operator rows are shared by every strip: one row ahead is enough
#pragma unroll
  for (int k = 0; k < NU; ++k) X[k][0] = X[k][1] = X[k][2] = C(0);
#pragma unroll
  for (int k = 0; k <= NU; ++k) Bw[k] = C(0);
  // the march is unrolled completely (a fixed SEG + 2 NU rows; those past
  // jlast load nothing and store nothing), so the fetch queue needs no
  // register moves between rows
  constexpr int ROWS = SEG + 2 * NU;
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    const int q = t % MPD;
    const int j = jlo + t;
    // prolongation and x_in on row j
    const C e0 = (qjin[q] && cin0) ? escale * qe0[q] : C(0), e1 = (qjin[q] && cin1) ? escale * qe1[q] : C(0);
    const C hnew = wi0 * e0 + wi1 * e1;
    const bool odd = j & 1;
    hlo = odd ? hhi : hlo;
    hhi = hnew;
    const C wj0 = odd ? C(1) : C(0.5), wj1 = odd ? C(0) : C(0.5);
    const C pe = wj0 * hlo + wj1 * hhi;
    const bool rin0 = colin && j >= 0 && j < n;
    const C x0 = rin0 ? qx[q] + pe : C(0);
#pragma unroll
    for (int k = NU; k > 0; --k) {
      Bw[k] = Bw[k - 1];
      Rw[k] = Rw[k - 1];
    }
    Bw[0] = qin[q] ? qb[q] : C(0);
    Rw[0] = rnext;
    if (t + 1 < ROWS) rnext = mop.row(op, j + 1);
    if (t + MPD < ROWS) fetch(j + MPD, q);
    X[0][0] = X[0][1];
    X[0][1] = X[0][2];
    X[0][2] = x0;
    // sweeps: sweep k on row j - k from the window of sweep k - 1
#pragma unroll
    for (int k = 1; k <= NU; ++k) {
      const C* w = X[k - 1];
      const C c = w[1];
      const C v = c + mop.inv_diag(Rw[k]) * (Bw[k] - mop.Ax(w, Rw[k]));
      const int jr = j - k;
      const bool rin = colin && jr >= 0 && jr < n;
      const C vk = rin ? v : C(0);
      if (k < NU) {
        X[k][0] = X[k][1];
        X[k][1] = X[k][2];
        X[k][2] = vk;
      } else if (own && jr >= j0 && jr < j1) {
        st<TF, C>(xo + (int64_t)jr * n + g, vk);
      }
    }
  }
}

// Down on level 0 of the constant-coefficient finite-difference operator
// from a zero initial guess, row-marching (the counterpart of
// k_up2d_march).  Row r of the march forms b - sum_l c_l K z_l (z rows
// r - 1 .. r + 1 in registers), the pointwise first sweep on row r, sweep k
// on row r - k, the residual on row r - NU and, when that row is even, the
// full-weighting restriction onto the coarse row centred one row below.  The
// residual must be exact one node beyond the owned columns and rows on the
// upper side (the stencil of the last coarse node) and on the owned nodes
// themselves, so a wave owns OW = 62 - 2 HC columns starting at lane HC =
// NU (+ 1 with coupling terms, whose K z needs one more lane) and marches
// NU rows below and NU + 1 above its SEG rows.  OW and SEG are even: strips
// and segments start at even fine indices, so every coarse node 2I + 1 has
// its whole stencil in the strip and segment that own it.
template <int KIND, int NU, class TF, class TC, class C, int NZ, int SEG>
__global__ __launch_bounds__(256) void k_down2d_march(const TF* __restrict__ b, int64_t sb, TF* __restrict__ xout,
                                                      int64_t sxo, TC* __restrict__ bc, int64_t sbc, LevelOp<C> op,
                                                      int nc, C omega, int nstrips, int nsegs, int64_t units,
                                                      CplArgs<TF, C> cpl, C bscale) {
  static_assert(NZ == 0 || KIND == KIND_FINE, "coupling terms are formed on the finite-difference level 0");
  constexpr int S = NU - 1;   // window sweeps after the pointwise one
  constexpr int HC = NU + (NZ > 0 ? 1 : 0), OW = 62 - 2 * HC;
  constexpr int ROWS = SEG + 2 * NU + 1;
  // rows fetched ahead: twice as many with one load per row (no coupling
  // terms, 5-point operator)
  constexpr int PD = (NZ == 0 && KIND == KIND_FINE) ? 2 * MPD : MPD;
  const int64_t u = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 4 + (threadIdx.x >> 6);
  if (u >= units) return;   // whole wave
  const int lane = threadIdx.x & 63;
  const int strip = (int)(u % nstrips);
  const int64_t rest = u / nstrips;
  const int seg = (int)(rest % nsegs);
  const int64_t inst = rest / nsegs;
  const int n = op.n;
  const int g = strip * OW - HC + lane;
  const bool colin = g >= 0 && g < n;
  const bool own = colin && lane >= HC && lane < HC + OW;
  const bool cown = own && (g & 1) && (g - 1) / 2 < nc;   // owns coarse column (g - 1) / 2
  const int j0 = seg * SEG, j1 = j0 + SEG < n ? j0 + SEG : n;
  const int jlo = j0 - NU, jlast = j1 + NU;
  const TF* bi = b + inst * sb;
  TF* xo = xout + inst * sxo;
  TC* bco = bc + inst * sbc + (cown ? (g - 1) / 2 : 0);
  const MarchOp<KIND, C> mop(op, omega, g, colin);
  using Row = typename MarchOp<KIND, C>::Row;
  const TF* zi[NZ > 0 ? NZ : 1];
#pragma unroll
  for (int l = 0; l < NZ; ++l) zi[l] = cpl.z + inst * cpl.sz + l * cpl.zs;
  // unconditional loads from clamped addresses, masked afterwards
  auto off = [&](int r) -> int64_t { return (colin && r >= 0 && r < n) ? (int64_t)r * n + g : 0; };
  auto inr = [&](int r) -> bool { return colin && r >= 0 && r < n; };
  C qb[PD], qz[NZ > 0 ? NZ : 1][PD];
  auto fetch = [&](int r, int q) {
    qb[q] = ld<TF, C>(bi + off(r));
#pragma unroll
    for (int l = 0; l < NZ; ++l) qz[l][q] = ld<TF, C>(zi[l] + off(r + 1));
  };
#pragma unroll
  for (int q = 0; q < PD; ++q) fetch(jlo + q, q);
  C Zw[NZ > 0 ? NZ : 1][3];   // z_l at rows r - 1, r, r + 1
#pragma unroll
  for (int l = 0; l < NZ; ++l) {
    Zw[l][0] = C(0);
    Zw[l][1] = inr(jlo - 1) ? ld<TF, C>(zi[l] + off(jlo - 1)) : C(0);
    Zw[l][2] = inr(jlo) ? ld<TF, C>(zi[l] + off(jlo)) : C(0);
  }
  C X[S + 1][3];   // X[k]: sweep k (0: the pointwise one) at rows r - k - 2 .. r - k
  C Bw[S + 2];     // right-hand side at rows r, r - 1, .., r - S - 1
  Row Ow[S + 2];   // operator rows r, r - 1, .., r - S - 1
  Row rnext = mop.row(op, jlo);
  C Rw[3];         // residual at rows r - NU - 2 .. r - NU
#pragma unroll
  for (int k = 0; k <= S; ++k) X[k][0] = X[k][1] = X[k][2] = C(0);
#pragma unroll
  for (int k = 0; k <= S + 1; ++k) Bw[k] = C(0);
  Rw[0] = Rw[1] = Rw[2] = C(0);
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    const int q = t % PD;
    const int r = jlo + t;
    const bool own_r = own && r >= j0 && r < j1;
    // right-hand side of row r, with Rana's coupling terms
    C acc = qb[q];
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      Zw[l][0] = Zw[l][1];
      Zw[l][1] = Zw[l][2];
      Zw[l][2] = inr(r + 1) ? qz[l][q] : C(0);
      const C c0 = Zw[l][1];
      const C zl = from_left(c0), zr = from_right(c0);
      const C kz = op.ih2 * (C(4) * c0 - zl - zr - Zw[l][0] - Zw[l][2]);
      acc -= cpl.c[l] * kz;
    }
    const bool din = inr(r);
    const C bb = din ? acc : C(0);
    const Row orow = rnext;   // operator rows are shared by every strip: one row ahead is enough
    if (t + 1 < ROWS) rnext = mop.row(op, r + 1);
    if (t + PD < ROWS) fetch(r + PD, q);
    if constexpr (NZ > 0)
      if (own_r) st<TF, C>(cpl.out + inst * cpl.so + (int64_t)r * n + g, bb);
#pragma unroll
    for (int k = S + 1; k > 0; --k) {
      Bw[k] = Bw[k - 1];
      Ow[k] = Ow[k - 1];
    }
    Bw[0] = bb;
    Ow[0] = orow;
    X[0][0] = X[0][1];
    X[0][1] = X[0][2];
    X[0][2] = din ? mop.inv_diag(Ow[0]) * bb : C(0);
    // sweep k on row r - k from the window of sweep k - 1
#pragma unroll
    for (int k = 1; k <= S; ++k) {
      const C* w = X[k - 1];
      const C c = w[1];
      const C v = c + mop.inv_diag(Ow[k]) * (Bw[k] - mop.Ax(w, Ow[k]));
      X[k][0] = X[k][1];
      X[k][1] = X[k][2];
      X[k][2] = inr(r - k) ? v : C(0);
    }
    // the smoothed iterate of row r - S
    if (own && r - S >= j0 && r - S < j1) st<TF, C>(xo + (int64_t)(r - S) * n + g, X[S][2]);
    // residual on row r - NU
    // (Ax outside the select: its DPP moves need every lane active)
    const C ax = mop.Ax(X[S], Ow[S + 1]);
    Rw[0] = Rw[1];
    Rw[1] = Rw[2];
    Rw[2] = inr(r - NU) ? Bw[S + 1] - ax : C(0);
    // restriction onto coarse row J = (r - NU) / 2 - 1 (fine row 2J + 1)
    const int rr = r - NU;
    if (rr >= 2 && !(rr & 1)) {   // wave-uniform
      const int J = rr / 2 - 1;
      const C rl = from_left(Rw[1]), rrt = from_right(Rw[1]);
      const C dl = from_left(Rw[0]), dr = from_right(Rw[0]);
      const C ul = from_left(Rw[2]), ur = from_right(Rw[2]);
      const C v = C(0.25) * bscale * (Rw[1] + C(0.5) * (rl + rrt + Rw[0] + Rw[2]) + C(0.25) * (dl + dr + ul + ur));
      if (cown && J < nc && 2 * J + 1 >= j0 && 2 * J + 1 < j1) st<TC, C>(bco + (int64_t)J * nc, v);
    }
  }
}

// Exact solve on the coarsest level (at most COARSE_MAX nodes) with its
// precomputed dense inverse, stored transposed: x_r = sum_c invT[c Nc + r] b_c.
template <class T, class C>
__global__ __launch_bounds__(1024) void k_coarse_solve(const T* __restrict__ b, int64_t sb, T* __restrict__ x,
                                                       int64_t sx, const C* __restrict__ invT, int Nc) {
  const int64_t inst = blockIdx.x;
  const T* bi = b + inst * sb;
  __shared__ C bs[COARSE_MAX];
  __shared__ C part_sum[4][COARSE_MAX];
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int c = tid; c < Nc; c += nth) bs[c] = ld<T, C>(bi + c);
  __syncthreads();
  const int parts = nth / Nc >= 4 ? 4 : (nth / Nc >= 2 ? 2 : 1);
  const int cols = (Nc + parts - 1) / parts;
  for (int t = tid; t < Nc * parts; t += nth) {
    const int r = t % Nc, part = t / Nc;
    const int c0 = part * cols, c1 = c0 + cols < Nc ? c0 + cols : Nc;
    C acc = C(0);
#pragma unroll 8
    for (int c = c0; c < c1; ++c) acc += invT[(int64_t)c * Nc + r] * bs[c];
    part_sum[part][r] = acc;
  }
  __syncthreads();
  for (int r = tid; r < Nc; r += nth) {
    C v = C(0);
    for (int q = 0; q < parts; ++q) v += part_sum[q][r];
    st<T, C>(x + inst * sx + r, v);
  }
}

// ---------------------------------------------------------------------------
// Coarse tail (2D): every level from `l0` down to one node in one workgroup
// per right-hand side.  Vectors and the 1D Galerkin factors live in LDS and
// are addressed by element offsets (so every access is an LDS instruction);
// barriers replace kernel launches.
// ---------------------------------------------------------------------------
constexpr int TAIL_MAXL = 12;
constexpr int TAIL_THREADS = 1024;

template <class C>
struct TailArgs {
  int nl;               // levels in the tail
  int first_fine;       // tail level 0 is the fine level (I + a K, matrix-free)
  int zero_init;        // start from x = 0 (else x is loaded)
  int nu1, nu2;
  C omega;
  int off[TAIL_MAXL];   // LDS offsets: X at off, Y at off + N, B at off + 2N
  int toff[TAIL_MAXL];  // LDS offset of the level's 6*n factor copy
  const C* cinv;        // dense inverse of the last level, transposed
  const C* fd;          // or its fast diagonalization (V, n^2 values, then lam, n values; null if absent)
  int fdoff;            // LDS offset of the staged fast-diagonalization data
  int scratch;          // LDS offset of 2 * N_last values for the coarse solve
  LevelOp<C> op[TAIL_MAXL];
};

// node p -> (i, j) on an n x n level; exact for p < 2^20, n <= 2^10:
// (p + 1/2) / n is never within 1/(2n) of an integer.
__device__ __forceinline__ void tail_ij(int p, int n, float inv_n, int& i, int& j) {
  j = (int)(((float)p + 0.5f) * inv_n);
  i = p - j * n;
}

// (A x)_p and A_pp for the 2D tensor Galerkin level with factors in LDS.
template <class C>
__device__ __forceinline__ void tail_tensor(const C* __restrict__ x, const C* __restrict__ tri, int n, C a, int p,
                                            int i, int j, C& Ax, C& d) {
  C mi[3], ti[3], mj[3], tj[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mi[q] = tri[q * n + i];
    ti[q] = tri[(3 + q) * n + i];
    mj[q] = tri[q * n + j];
    tj[q] = tri[(3 + q) * n + j];
  }
  C acc = C(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj) {
    const int jj = j + dj;
    if (jj < 0 || jj >= n) continue;
    C pv = C(0), qv = C(0);
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= n) continue;
      const C xv = x[p + dj * n + di];
      pv += (mi[di + 1] + a * ti[di + 1]) * xv;
      qv += mi[di + 1] * xv;
    }
    acc += mj[dj + 1] * pv + a * tj[dj + 1] * qv;
  }
  Ax = acc;
  d = mi[1] * mj[1] + a * (ti[1] * mj[1] + mi[1] * tj[1]);
}

// (A x)_p and A_pp for a 2D Galerkin level with a stored stencil of K: the
// M(x)M part from the LDS factor copy, the stencil from global memory.
template <class C>
__device__ __forceinline__ void tail_stencil9(const C* __restrict__ x, const C* __restrict__ tri, const LevelOp<C>& op,
                                              int p, int i, int j, C& Ax, C& d) {
  const int n = op.n;
  C acc = C(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj) {
    const int jj = j + dj;
    if (jj < 0 || jj >= n) continue;
    const C mj = tri[(dj + 1) * n + j];
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di;
      if (ii < 0 || ii >= n) continue;
      const C coef = mj * tri[(di + 1) * n + i] + op.a * op.st9[((dj + 1) * 3 + di + 1) * op.N + p];
      acc += coef * x[p + dj * n + di];
    }
  }
  Ax = acc;
  d = tri[n + i] * tri[n + j] + op.a * op.st9[4 * op.N + p];
}

// Level t of the tail: tensor Galerkin, or the fine operator when the tail
// starts at level 0.
template <bool VK, class C>
__device__ __forceinline__ void tail_op(const TailArgs<C>& ta, const C* sm, int t, const C* x, int p, int i, int j,
                                        C& Ax, C& d) {
  if (t == 0 && ta.first_fine) {
    if (VK) level_apply<2, KIND_FINE_VK, C, C>(x, ta.op[0], p, i, j, 0, Ax, d);
    else level_apply<2, KIND_FINE, C, C>(x, ta.op[0], p, i, j, 0, Ax, d);
  } else if (ta.op[t].st9) {
    tail_stencil9<C>(x, sm + ta.toff[t], ta.op[t], p, i, j, Ax, d);
  } else {
    tail_tensor<C>(x, sm + ta.toff[t], ta.op[t].n, ta.op[t].a, p, i, j, Ax, d);
  }
}

// Diagonal of level t of the tail at node p = (i, j).
template <bool VK, class C>
__device__ __forceinline__ C tail_diag(const TailArgs<C>& ta, const C* sm, int t, int p, int i, int j) {
  const LevelOp<C>& op = ta.op[t];
  if (t == 0 && ta.first_fine) return level_diag<2, VK ? KIND_FINE_VK : KIND_FINE, C>(op, p, i, j, 0);
  const C* tri = sm + ta.toff[t];
  const int n = op.n;
  if (op.st9) return tri[n + i] * tri[n + j] + op.a * op.st9[4 * op.N + p];
  return tri[n + i] * tri[n + j] + op.a * (tri[4 * n + i] * tri[n + j] + tri[n + i] * tri[4 * n + j]);
}

template <bool VK, class TX, class TB, class C>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(TX* __restrict__ xg, int64_t sx, const TB* __restrict__ bg,
                                                       int64_t sb, TailArgs<C> ta) {
  extern __shared__ unsigned char tail_smem[];
  C* sm = reinterpret_cast<C*>(tail_smem);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int64_t inst = blockIdx.x;
  const int last = ta.nl - 1;
  // stage the factors of the tensor levels and the right-hand side
  for (int t = (ta.first_fine ? 1 : 0); t <= last; ++t) {
    const int n6 = 6 * ta.op[t].n;
    for (int q = tid; q < n6; q += nth) sm[ta.toff[t] + q] = ta.op[t].tri[q];
  }
  if (ta.fd) {
    const int nl = ta.op[last].n, nfd = nl * nl + nl;
    for (int q = tid; q < nfd; q += nth) sm[ta.fdoff + q] = ta.fd[q];
  }
  const int N0 = (int)ta.op[0].N;
  for (int p = tid; p < N0; p += nth) {
    sm[ta.off[0] + 2 * N0 + p] = ld<TB, C>(bg + inst * sb + p);
    if (!ta.zero_init) sm[ta.off[0] + p] = ld<TX, C>(xg + inst * sx + p);
  }
  __syncthreads();
  unsigned cur_y = 0;   // bit t set: the level-t iterate is in Y (else X)
  for (int t = 0; t < last; ++t) {
    const int Nt = (int)ta.op[t].N, n = ta.op[t].n;
    const float inv_n = 1.0f / (float)n;
    const int X = ta.off[t], Y = X + Nt, Bt = X + 2 * Nt;
    int rem = ta.nu1;
    if (t > 0 || ta.zero_init) {
      for (int p = tid; p < Nt; p += nth) {
        int i, j;
        tail_ij(p, n, inv_n, i, j);
        sm[X + p] = ta.omega * sm[Bt + p] / tail_diag<VK, C>(ta, sm, t, p, i, j);
      }
      --rem;
      __syncthreads();
    }
    int c = X, o = Y;
    for (; rem > 0; --rem) {
      for (int p = tid; p < Nt; p += nth) {
        int i, j;
        tail_ij(p, n, inv_n, i, j);
        C Ax, d;
        tail_op<VK, C>(ta, sm, t, sm + c, p, i, j, Ax, d);
        sm[o + p] = sm[c + p] + ta.omega * (sm[Bt + p] - Ax) / d;
      }
      __syncthreads();
      const int tmp = c; c = o; o = tmp;
    }
    for (int p = tid; p < Nt; p += nth) {            // residual into the free buffer
      int i, j;
      tail_ij(p, n, inv_n, i, j);
      C Ax, d;
      tail_op<VK, C>(ta, sm, t, sm + c, p, i, j, Ax, d);
      sm[o + p] = sm[Bt + p] - Ax;
    }
    __syncthreads();
    const int Nc = (int)ta.op[t + 1].N, nc = ta.op[t + 1].n;
    const float inv_nc = 1.0f / (float)nc;
    const int Bc = ta.off[t + 1] + 2 * Nc;
    for (int pc = tid; pc < Nc; pc += nth) {          // full weighting
      int I, J;
      tail_ij(pc, nc, inv_nc, I, J);
      const int fi = 2 * I + 1, fj = 2 * J + 1;
      C acc = C(0);
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const int jj = fj + dj;
        if (jj >= n) continue;
        const C wj = dj == 0 ? C(1) : C(0.5);
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
          const int ii = fi + di;
          if (ii >= n) continue;
          acc += (di == 0 ? wj : C(0.5) * wj) * sm[o + jj * n + ii];
        }
      }
      sm[Bc + pc] = C(0.25) * acc;
    }
    if (c != X) cur_y |= 1u << t;
    __syncthreads();
  }
  if (ta.fd) {                                        // coarsest level: exact, fast diagonalization
    // A = M(x)M + a (T(x)M + M(x)T) on an n x n grid; with T V = M V diag(lam),
    // V^T M V = I:  X = V ((V^T B V) ./ (1 + a (lam_l + lam_k))) V^T, where
    // B[j][i] = b_{j n + i}.  Four n x n products through the free Y buffer.
    const int n = ta.op[last].n, Nt = n * n;
    const int X = ta.off[last], Y = X + Nt, Bl = X + 2 * Nt;
    const C* V = sm + ta.fdoff;
    const C* lam = V + Nt;
    const C a = ta.op[last].a;
    for (int q = tid; q < Nt; q += nth) {            // Y = B V
      const int j = q / n, k = q - j * n;
      C acc = C(0);
      for (int i = 0; i < n; ++i) acc += sm[Bl + j * n + i] * V[i * n + k];
      sm[Y + q] = acc;
    }
    __syncthreads();
    for (int q = tid; q < Nt; q += nth) {            // X = (V^T Y) ./ D
      const int l = q / n, k = q - l * n;
      C acc = C(0);
      for (int j = 0; j < n; ++j) acc += V[j * n + l] * sm[Y + j * n + k];
      sm[X + q] = acc / (C(1) + a * (lam[l] + lam[k]));
    }
    __syncthreads();
    for (int q = tid; q < Nt; q += nth) {            // Y = X V^T
      const int l = q / n, i = q - l * n;
      C acc = C(0);
      for (int k = 0; k < n; ++k) acc += sm[X + l * n + k] * V[i * n + k];
      sm[Y + q] = acc;
    }
    __syncthreads();
    for (int q = tid; q < Nt; q += nth) {            // X = V Y
      const int j = q / n, i = q - j * n;
      C acc = C(0);
      for (int l = 0; l < n; ++l) acc += V[j * n + l] * sm[Y + l * n + i];
      sm[X + q] = acc;
    }
    __syncthreads();
  } else {                                            // coarsest level: exact
    // x = A^{-1} b with the dense inverse: `parts` threads per row, each
    // summing a contiguous slice of columns; partial sums meet in the free
    // Y buffer of this level (Nt * parts <= 3 Nt values fit in X, Y, B? no:
    // they go to Y and beyond only when parts == 1), combined below.
    const int X = ta.off[last], Nt = (int)ta.op[last].N;
    const int Bl = X + 2 * Nt;
    const int parts = nth / Nt >= 4 ? 4 : (nth / Nt >= 2 ? 2 : 1);
    if (parts == 1) {
      C accs[4];
      int cnt = 0;
      for (int r = tid; r < Nt; r += nth) {        // at most 4 rows per thread (Nt <= 256 <= 4 nth)
        C acc = C(0);
#pragma unroll 8
        for (int c = 0; c < Nt; ++c) acc += ta.cinv[(int64_t)c * Nt + r] * sm[Bl + c];
        accs[cnt++ & 3] = acc;
      }
      __syncthreads();
      cnt = 0;
      for (int r = tid; r < Nt; r += nth) sm[X + r] = accs[cnt++ & 3];
    } else {
      const int cols = (Nt + parts - 1) / parts;
      C acc = C(0);
      int r = 0, part = 0;
      if (tid < Nt * parts) {
        r = tid % Nt;
        part = tid / Nt;
        const int c0 = part * cols, c1 = c0 + cols < Nt ? c0 + cols : Nt;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) acc += ta.cinv[(int64_t)c * Nt + r] * sm[Bl + c];
      }
      __syncthreads();
      // partial sums: part 0 -> X, part 1 -> Y (free), parts 2, 3 -> the
      // scratch reserved past the factor copies
      if (tid < Nt * parts) sm[(part == 0 ? X : (part == 1 ? X + Nt : ta.scratch + (part - 2) * Nt)) + r] = acc;
      __syncthreads();
      for (int q = tid; q < Nt; q += nth) {
        C v = sm[X + q] + sm[X + Nt + q];
        if (parts > 2) v += sm[ta.scratch + q] + sm[ta.scratch + Nt + q];
        sm[X + q] = v;
      }
    }
    __syncthreads();
  }
  for (int t = last - 1; t >= 0; --t) {
    const int Nt = (int)ta.op[t].N, n = ta.op[t].n;
    const float inv_n = 1.0f / (float)n;
    const int nc = ta.op[t + 1].n;
    const int X = ta.off[t], Y = X + Nt, Bt = X + 2 * Nt;
    int c = (cur_y >> t) & 1u ? Y : X;
    int o = c == X ? Y : X;
    const int Nc1 = (int)ta.op[t + 1].N;
    const int e = ((cur_y >> (t + 1)) & 1u) ? ta.off[t + 1] + Nc1 : ta.off[t + 1];
    for (int p = tid; p < Nt; p += nth) {
      int i, j;
      tail_ij(p, n, inv_n, i, j);
      sm[c + p] += prolong_at<2, C, C>(sm + e, nc, i, j, 0);
    }
    __syncthreads();
    for (int it = 0; it < ta.nu2; ++it) {
      for (int p = tid; p < Nt; p += nth) {
        int i, j;
        tail_ij(p, n, inv_n, i, j);
        C Ax, d;
        tail_op<VK, C>(ta, sm, t, sm + c, p, i, j, Ax, d);
        sm[o + p] = sm[c + p] + ta.omega * (sm[Bt + p] - Ax) / d;
      }
      __syncthreads();
      const int tmp = c; c = o; o = tmp;
    }
    if (c != X) cur_y |= 1u << t;
    else cur_y &= ~(1u << t);
  }
  const int res = (cur_y & 1u) ? ta.off[0] + N0 : ta.off[0];
  for (int p = tid; p < N0; p += nth) st<TX, C>(xg + inst * sx + p, sm[res + p]);
}

// ---------------------------------------------------------------------------
// Coarse tail for the common case: NLS (1 or 2) Galerkin smoothing levels,
// the first of at most NPT * TAIL_THREADS nodes (n <= 64, NPT-node vertical
// strips per thread), the second of at most TAIL_THREADS, then the exact coarsest level (fast diagonalization or
// the dense inverse, at most 16 x 16), entered from x = 0.  Each thread owns
// fixed nodes of every level and keeps their nine coefficients, omega /
// diagonal and right-hand side in registers for the whole cycle, so a sweep
// reads only the neighbours from LDS.  Iterates live in LDS with a zero ring
// (row pitch n + 2), so stencils, restriction and prolongation need no
// boundary tests.  The restricted right-hand side of a coarse node is formed
// by the thread that owns it, in a register.  Every global load is issued at
// entry.  Same arithmetic as k_tail, up to summation order.
// ---------------------------------------------------------------------------
constexpr int TF_NMAX = 64;                      // largest smoothing level: 64 x 64
constexpr int TF_NC = 16, TF_NCN = TF_NC * TF_NC;   // largest coarsest level: 16 x 16

template <class C>
struct TailFastArgs {
  int n[3];            // level sizes (n x n); level NLS is the exact one
  C a, omega;
  int nu1, nu2;
  const C* tri[2];     // 1D Galerkin factors of the smoothing levels (6 n each)
  const C* st9[2];     // variable kappa: 9 N stencil of K per smoothing level
  const C* fd;         // coarsest: V (n^2) then lam (n), or null
  const C* cinv;       // coarsest: dense inverse, transposed (when fd is null)
  int ov[2][2];        // LDS offsets (elements) of the two padded iterate buffers per smoothing level
  int ocb, ocy, ocx, ocw;   // coarsest: rhs, work, padded solution, V / partial sums
};

// One smoothing level as seen by one thread: NP owned nodes.  With NP > 1
// they are a vertical strip, nodes (i, NP q + m), so a sweep reads one
// (NP + 2) x 3 window of the iterate for all of them.
template <int KIND, int NP, class C>
struct TfLev {
  int n, P, o0, o1;              // size, padded pitch, buffer offsets
  int pi[NP], ci[NP], cj[NP];
  int woff[NP + 2];              // padded offsets of the window rows (column i - 1)
  unsigned own;                  // bit m: node m exists
  C k[NP][9], id[NP], b[NP];
  C fi[6], fj[NP][6];            // factor columns at i and at each j (loaded at entry)
  int cur;                       // buffer (0: o0, 1: o1) holding the smoothed iterate
  __device__ int off(int c) const { return c ? o1 : o0; }
};

template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_geom(TfLev<KIND, NP, C>& L, int n, int o0, int o1) {
  L.n = n;
  L.P = n + 2;
  L.o0 = o0;
  L.o1 = o1;
  L.own = 0;
  const int strips = (n + NP - 1) / NP;
  const bool act = (int)threadIdx.x < n * strips;
  const int q = act ? (int)threadIdx.x / n : 0;
  const int i = act ? (int)threadIdx.x - q * n : 0;
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int j = NP * q + m;
    const bool own = act && j < n;
    L.own |= (unsigned)own << m;
    L.ci[m] = own ? i : 0;
    L.cj[m] = own ? j : 0;
    L.pi[m] = (L.cj[m] + 1) * L.P + L.ci[m] + 1;
  }
#pragma unroll
  for (int r = 0; r < NP + 2; ++r) {
    const int row = NP * q + r < L.P - 1 ? NP * q + r : L.P - 1;
    L.woff[r] = row * L.P + i;
  }
}

// Issue the coefficient loads of a level (factor columns; stencil of K).
template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_load(TfLev<KIND, NP, C>& L, const C* __restrict__ tri, const C* __restrict__ st9) {
  const bool any = L.own != 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) L.fi[q] = any ? tri[q * L.n + L.ci[0]] : C(0);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const bool own = (L.own >> m) & 1u;
#pragma unroll
    for (int q = 0; q < 6; ++q) L.fj[m][q] = own ? tri[q * L.n + L.cj[m]] : C(0);
    if constexpr (KIND == KIND_STENCIL9) {
      const int p = L.cj[m] * L.n + L.ci[m];
#pragma unroll
      for (int d = 0; d < 9; ++d) L.k[m][d] = own ? st9[d * L.n * L.n + p] : C(0);
    }
  }
}

// Coefficients (M + aT)_i M_j + a M_i T_j (variable kappa: M_i M_j + a K) and
// omega / diagonal.
template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_coef(TfLev<KIND, NP, C>& L, C a, C omega) {
#pragma unroll
  for (int m = 0; m < NP; ++m) {
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        C& k = L.k[m][dj * 3 + di];
        if constexpr (KIND == KIND_TENSOR)
          k = L.fj[m][dj] * (L.fi[di] + a * L.fi[3 + di]) + a * L.fj[m][3 + dj] * L.fi[di];
        else
          k = L.fj[m][dj] * L.fi[di] + a * k;
      }
    L.id[m] = ((L.own >> m) & 1u) ? omega / L.k[m][4] : C(0);
  }
}

// Zero the ring of a padded n x n array at LDS offset o.
template <class C>
__device__ __forceinline__ void tf_ring(C* sm, int o, int P) {
  for (int e = threadIdx.x; e < 4 * (P - 1); e += TAIL_THREADS) {
    const int side = e / (P - 1), r = e - side * (P - 1);
    const int idx = side == 0 ? r : (side == 1 ? r * P + P - 1 : (side == 2 ? P * P - 1 - r : (P - 1 - r) * P));
    sm[o + idx] = C(0);
  }
}

// (A x) at every node of the thread, from the (NP + 2) x 3 window of x.
template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_apply(const TfLev<KIND, NP, C>& L, const C* __restrict__ x, C (&ax)[NP]) {
  C w[NP + 2][3];
#pragma unroll
  for (int r = 0; r < NP + 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) w[r][c] = x[L.woff[r] + c];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    C acc = C(0);
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
      for (int di = 0; di < 3; ++di) acc += L.k[m][dj * 3 + di] * w[m + dj][di];
    ax[m] = acc;
  }
}

// Pre-smoothing from zero (the first sweep pointwise), then the residual
// into the other buffer.
template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_down(TfLev<KIND, NP, C>& L, C* sm, int nu1) {
  C x[NP], ax[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    x[m] = L.id[m] * L.b[m];
    if ((L.own >> m) & 1u) sm[L.o0 + L.pi[m]] = x[m];
  }
  __syncthreads();
  int c = 0;
  for (int r = 1; r < nu1; ++r) {
    C* xo = sm + L.off(c ^ 1);
    tf_apply(L, sm + L.off(c), ax);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      x[m] += L.id[m] * (L.b[m] - ax[m]);
      if ((L.own >> m) & 1u) xo[L.pi[m]] = x[m];
    }
    __syncthreads();
    c ^= 1;
  }
  C* ro = sm + L.off(c ^ 1);
  tf_apply(L, sm + L.off(c), ax);
#pragma unroll
  for (int m = 0; m < NP; ++m)
    if ((L.own >> m) & 1u) ro[L.pi[m]] = L.b[m] - ax[m];
  __syncthreads();
  L.cur = c;
}

// Full weighting of the fine residual into the coarse owners' right-hand
// sides: coarse (I, J) sits at fine (2I + 1, 2J + 1).
template <int KIND, int NPC, int NPF, class C>
__device__ __forceinline__ void tf_restrict(TfLev<KIND, NPC, C>& Lc, const TfLev<KIND, NPF, C>& Lf, const C* sm) {
  const C* r = sm + Lf.off(Lf.cur ^ 1);
  const int Pf = Lf.P;
#pragma unroll
  for (int m = 0; m < NPC; ++m) {
    const int f = (2 * Lc.cj[m] + 2) * Pf + 2 * Lc.ci[m] + 2;
    const C v = C(0.25) * (r[f] + C(0.5) * (r[f - 1] + r[f + 1] + r[f - Pf] + r[f + Pf]) +
                           C(0.25) * (r[f - Pf - 1] + r[f - Pf + 1] + r[f + Pf - 1] + r[f + Pf + 1]));
    Lc.b[m] = ((Lc.own >> m) & 1u) ? v : C(0);
  }
}

// x = x_smoothed + P e (e: padded coarse array at LDS offset oe, pitch Pc),
// then nu2 sweeps.  Fine g takes coarse lo = floor((g - 1) / 2) and lo + 1
// with weights (1, 0) for odd g, (1/2, 1/2) for even g.
template <int KIND, int NP, class C>
__device__ __forceinline__ void tf_up(TfLev<KIND, NP, C>& L, C* sm, int oe, int Pc, int nu2, C (&x)[NP]) {
  const C* e = sm + oe;
  const C* xs = sm + L.off(L.cur);
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const int gi = L.ci[m], gj = L.cj[m];
    const int q = (((gj - 1) >> 1) + 1) * Pc + ((gi - 1) >> 1) + 1;
    const C wi0 = (gi & 1) ? C(1) : C(0.5), wi1 = (gi & 1) ? C(0) : C(0.5);
    const C wj0 = (gj & 1) ? C(1) : C(0.5), wj1 = (gj & 1) ? C(0) : C(0.5);
    x[m] = xs[L.pi[m]] + wj0 * (wi0 * e[q] + wi1 * e[q + 1]) + wj1 * (wi0 * e[q + Pc] + wi1 * e[q + Pc + 1]);
  }
  int c = L.cur ^ 1;
  for (int r = 0; r < nu2; ++r) {
    C* xo = sm + L.off(c);
#pragma unroll
    for (int m = 0; m < NP; ++m)
      if ((L.own >> m) & 1u) xo[L.pi[m]] = x[m];
    __syncthreads();
    C ax[NP];
    tf_apply(L, xo, ax);
#pragma unroll
    for (int m = 0; m < NP; ++m) x[m] += L.id[m] * (L.b[m] - ax[m]);
    c ^= 1;
  }
  L.cur = c;   // the buffer the final x would go to
}

template <int KIND, int NLS, int NPT, bool FD, class T, class C>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_fast(T* __restrict__ xg, int64_t sx, const T* __restrict__ bg,
                                                            int64_t sb, TailFastArgs<C> ta) {
  static_assert(KIND == KIND_TENSOR || KIND == KIND_STENCIL9, "Galerkin levels only");
  static_assert(NLS == 1 || NLS == 2, "one or two smoothing levels");
  extern __shared__ unsigned char tail_smem[];
  C* sm = reinterpret_cast<C*>(tail_smem);
  const int tid = threadIdx.x;
  const int64_t inst = blockIdx.x;
  TfLev<KIND, NPT, C> L0;
  TfLev<KIND, 1, C> L1;
  tf_geom(L0, ta.n[0], ta.ov[0][0], ta.ov[0][1]);
  if constexpr (NLS == 2) tf_geom(L1, ta.n[1], ta.ov[1][0], ta.ov[1][1]);
  const int nc = ta.n[NLS], Nc = nc * nc, Pc = nc + 2;
  const bool ownc = tid < Nc;
  const int cjc = ownc ? tid / nc : 0, cic = ownc ? tid - cjc * nc : 0;
  // --- every global load up front
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int p = L0.cj[m] * L0.n + L0.ci[m];
    L0.b[m] = ((L0.own >> m) & 1u) ? ld<T, C>(bg + inst * sb + p) : C(0);
  }
  tf_load(L0, ta.tri[0], ta.st9[0]);
  if constexpr (NLS == 2) tf_load(L1, ta.tri[1], ta.st9[1]);
  const int nfd = FD ? Nc + nc : 0;
  const C fdv = (FD && tid < nfd) ? ta.fd[tid] : C(0);
  // --- zero rings, staged fast-diagonalization data, coefficients
  tf_ring(sm, L0.o0, L0.P);
  tf_ring(sm, L0.o1, L0.P);
  if constexpr (NLS == 2) {
    tf_ring(sm, L1.o0, L1.P);
    tf_ring(sm, L1.o1, L1.P);
  }
  tf_ring(sm, ta.ocx, Pc);
  if (FD && tid < nfd) sm[ta.ocw + tid] = fdv;
  tf_coef(L0, ta.a, ta.omega);
  if constexpr (NLS == 2) tf_coef(L1, ta.a, ta.omega);
  // --- down
  tf_down(L0, sm, ta.nu1);
  C bc;
  if constexpr (NLS == 2) {
    tf_restrict(L1, L0, sm);
    tf_down(L1, sm, ta.nu1);
    TfLev<KIND, 1, C> Lc;   // coarse owner geometry for the restriction
    Lc.P = Pc;
    Lc.own = ownc;
    Lc.ci[0] = cic;
    Lc.cj[0] = cjc;
    tf_restrict(Lc, L1, sm);
    bc = Lc.b[0];
  } else {
    TfLev<KIND, 1, C> Lc;
    Lc.P = Pc;
    Lc.own = ownc;
    Lc.ci[0] = cic;
    Lc.cj[0] = cjc;
    tf_restrict(Lc, L0, sm);
    bc = Lc.b[0];
  }
  // --- coarsest level, exact
  C* cb = sm + ta.ocb;
  C* cy = sm + ta.ocy;
  C* cx = sm + ta.ocx;
  C* cw = sm + ta.ocw;
  const int pic = (cjc + 1) * Pc + cic + 1;
  if (ownc) cb[tid] = bc;
  __syncthreads();
  if constexpr (FD) {
    // A = M(x)M + a (T(x)M + M(x)T); with T V = M V diag(lam), V^T M V = I:
    // X = V ((V^T B V) ./ (1 + a (lam_l + lam_k))) V^T, B[j][i] = b_{j n + i}
    const C* V = cw;
    const C* lam = V + Nc;
    const int j = cjc, k = cic;
    if (ownc) {                                       // Y = B V
      C acc = C(0);
      for (int i = 0; i < nc; ++i) acc += cb[j * nc + i] * V[i * nc + k];
      cy[tid] = acc;
    }
    __syncthreads();
    if (ownc) {                                       // B <- (V^T Y) ./ D
      C acc = C(0);
      for (int jj = 0; jj < nc; ++jj) acc += V[jj * nc + j] * cy[jj * nc + k];
      cb[tid] = acc / (C(1) + ta.a * (lam[j] + lam[k]));
    }
    __syncthreads();
    if (ownc) {                                       // Y = B V^T
      C acc = C(0);
      for (int kk = 0; kk < nc; ++kk) acc += cb[j * nc + kk] * V[k * nc + kk];
      cy[tid] = acc;
    }
    __syncthreads();
    if (ownc) {                                       // X = V Y
      C acc = C(0);
      for (int l = 0; l < nc; ++l) acc += V[j * nc + l] * cy[l * nc + k];
      cx[pic] = acc;
    }
    __syncthreads();
  } else {
    // x = A^{-1} b: four threads per row, each over a quarter of the columns
    const int r = tid % Nc, part = tid / Nc, cols = (Nc + 3) / 4;
    if (part < 4) {
      const int c0 = part * cols, c1 = c0 + cols < Nc ? c0 + cols : Nc;
      C acc = C(0);
      for (int c = c0; c < c1; ++c) acc += ta.cinv[(int64_t)c * Nc + r] * cb[c];
      cw[part * TF_NCN + r] = acc;
    }
    __syncthreads();
    if (ownc) cx[pic] = cw[tid] + cw[TF_NCN + tid] + cw[2 * TF_NCN + tid] + cw[3 * TF_NCN + tid];
    __syncthreads();
  }
  // --- up; the finest tail level goes to global memory
  int oe = ta.ocx, Pe = Pc;
  if constexpr (NLS == 2) {
    C x1[1];
    tf_up(L1, sm, oe, Pe, ta.nu2, x1);
    if (L1.own & 1u) sm[L1.off(L1.cur) + L1.pi[0]] = x1[0];
    __syncthreads();
    oe = L1.off(L1.cur);
    Pe = L1.P;
  }
  C x0[NPT];
  tf_up(L0, sm, oe, Pe, ta.nu2, x0);
#pragma unroll
  for (int m = 0; m < NPT; ++m)
    if ((L0.own >> m) & 1u) st<T, C>(xg + inst * sx + L0.cj[m] * L0.n + L0.ci[m], x0[m]);
}

// LDS layout of k_tail_fast for levels n[0..nls] (elements of C); returns the total.
template <class C>
int tail_fast_layout(TailFastArgs<C>& ta, int nls) {
  int off = 0;
  for (int t = 0; t < nls; ++t) {
    const int q = (ta.n[t] + 2) * (ta.n[t] + 2);
    ta.ov[t][0] = off;
    ta.ov[t][1] = off + q;
    off += 2 * q;
  }
  const int nc = ta.n[nls];
  ta.ocb = off;
  ta.ocy = off + nc * nc;
  ta.ocx = off + 2 * nc * nc;
  ta.ocw = ta.ocx + (nc + 2) * (nc + 2);
  return ta.ocw + 4 * TF_NCN;
}

// ---------------------------------------------------------------------------
// 3D level 0 (constant kappa) as z-marches.  A workgroup owns a 32 x 32
// thread tile of (x, y) columns -- a core plus a halo of three (down) or two
// (up) nodes -- and walks a chunk of z-planes.  Each plane step runs
// pipelined stages, each on the plane one behind the stage before; a
// stage's z-neighbours stay in the thread's registers, its (x, y)-neighbours
// come from the previous step's plane in LDS (two slots per stage, one
// barrier per step).  Every stencil application shrinks the valid region by
// one node, so the halo rings compute values only the core consumes.  The
// arithmetic is that of k_smooth / k_residual / k_restrict / k_prolong,
// node by node.
// ---------------------------------------------------------------------------
constexpr int M3_T = 32;          // threads per tile side

struct March3Geo {
  int n, ntx, nz, zlen;   // grid side, tiles per side, z-chunks, planes per chunk
};

// Tile, chunk and thread coordinates of this workgroup for a halo of H
// nodes (core width 32 - 2H).  Logical tiles are spread so each XCD walks a
// contiguous range (xcd_tile).
template <int H>
struct March3Pos {
  static constexpr int CW = M3_T - 2 * H;
  int i, j, z0, z1;
  bool inside, core;
  int tx, ty;
  __device__ March3Pos(const March3Geo& g) {
    const int G = g.ntx * g.ntx * g.nz;
    const int t = xcd_tile((int)blockIdx.x, G);
    const int zc = t / (g.ntx * g.ntx);
    const int r = t - zc * g.ntx * g.ntx;
    const int by = r / g.ntx, bx = r - by * g.ntx;
    tx = (int)threadIdx.x & (M3_T - 1);
    ty = (int)threadIdx.x / M3_T;
    i = bx * CW - H + tx;
    j = by * CW - H + ty;
    z0 = zc * g.zlen;
    z1 = z0 + g.zlen < g.n ? z0 + g.zlen : g.n;
    inside = i >= 0 && i < g.n && j >= 0 && j < g.n;
    core = inside && tx >= H && tx < M3_T - H && ty >= H && ty < M3_T - H;
  }
};

// Barrier for the marches' plane steps: the stages exchange data only
// through LDS, so a wave waits for its own LDS operations and then for the
// workgroup.  (__syncthreads also waits for every global load in flight,
// which would stall each step on the loads issued for planes ahead.)  The
// memory clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void m3_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// h^2 K at the thread's node: (x, y)-neighbours from the LDS plane pl
// (the tile's edge threads read themselves: their results are
// never used), z-neighbours zm, zp from registers.  Same expression as
// stencil_K (values past the grid are the zeros the neighbours stored).
template <class C>
__device__ __forceinline__ C m3_k(const C* pl, int tx, int ty, C c0, C zm, C zp) {
  const int xm = tx > 0 ? tx - 1 : tx, xp = tx < M3_T - 1 ? tx + 1 : tx;
  const int ym = ty > 0 ? ty - 1 : ty, yp = ty < M3_T - 1 ? ty + 1 : ty;
  C acc = C(6) * c0 - pl[ty * M3_T + xm] - pl[ty * M3_T + xp] - pl[ym * M3_T + tx] - pl[yp * M3_T + tx];
  acc -= zm + zp;
  return acc;
}

// Planes are loaded PF steps before their first stage uses them (a ring of
// registers), so each step's global loads overlap the steps before it.
constexpr int M3_PF_DOWN = 4;
constexpr int M3_PF_UP = 2;

// Zero-start pre-smoothing (two weighted Jacobi sweeps, the first
// pointwise), the residual and its full weighting: x2 -> xout; b_c (and,
// with zero_next, the coarse level's first sweep x_c = omega b_c / D_c) for
// the coarse nodes centred in the tile's core.  A halo of three nodes leaves
// the residual valid one node past the core, where the 3 x 3 neighbourhoods
// of the core's coarse centres reach.  Stage 4 adds plane q - 3 of the
// residual to its coarse planes term by term in k_restrict's order, so b_c
// is bitwise k_restrict's.
template <class T, class TC, class C>
__global__ __launch_bounds__(M3_T * M3_T) void k_down3d_march(const T* __restrict__ b, int64_t sb,
                                                             T* __restrict__ xout, int64_t sx,
                                                             TC* __restrict__ bc, int64_t sbc,
                                                             TC* __restrict__ xc, int64_t sxc, March3Geo g,
                                                             LevelOp<C> op, LevelOp<C> opc, C omega, int zero_next,
                                                             C bscale) {
  constexpr int PF = M3_PF_DOWN;
  __shared__ C s1[2][M3_T * M3_T];   // x1 planes
  __shared__ C s2[2][M3_T * M3_T];   // x2 planes
  __shared__ C s3[2][M3_T * M3_T];   // residual planes
  const March3Pos<3> m(g);
  const int64_t inst = blockIdx.y;
  const int n = g.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t col = (int64_t)(m.inside ? m.j : 0) * n + (m.inside ? m.i : 0);
  const T* bi = b + inst * sb + col;
  T* xo = xout + inst * sx + col;
  const C wd = omega / level_diag<3, KIND_FINE, C>(op, 0, 0, 0, 0);
  const int me = m.ty * M3_T + m.tx;
  // coarse owner: a core node at odd (i, j) is the centre of coarse (I, J)
  const bool owner = m.core && (m.i & 1) && (m.j & 1);
  const int I = (m.i - 1) >> 1, J = (m.j - 1) >> 1, nc = opc.n;
  const int zc1 = m.z1 < n ? m.z1 : n;   // coarse planes K with z0 <= 2K + 1 < zc1 are this chunk's
  const C w3[3] = {C(0.5), C(1), C(0.5)};
  C acc = C(0);
  // the last plane the restriction reads is z1 (the + 1 neighbour of the
  // chunk's last centre plane); stage 4 trails stage 1 by three planes
  const int qlast = m.z1 + 3;
  // every thread loads, at a clamped plane, so the loads are unconditional
  // and the compiler's wait counts let them stay in flight; each stage reads
  // its plane's value only where that plane and node are real
  auto load_b = [&](int q) { return ld<T, C>(bi + (int64_t)min(max(q, 0), n - 1) * nn); };
  // ring of planes in flight: slot u holds plane q0 + u of the current block
  // of PF steps; each step consumes its slot and refills it PF planes ahead
  // (the loop is unrolled by PF, so the ring rotates by renaming)
  C pb[PF];
#pragma unroll
  for (int u = 0; u < PF; ++u) pb[u] = load_b(m.z0 - 2 + u);
  // register windows: b at q-1, q-2; x1 at q-2, q-1, q; x2 at q-3, q-2, q-1
  C b1 = C(0), b2 = C(0), x1a = C(0), x1b = C(0), x2a = C(0), x2b = C(0);
  // whole blocks of PF steps: steps past qlast write nothing
  for (int q0 = m.z0 - 2; q0 <= qlast; q0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int q = q0 + u;
      const int sl = q & 1;
      const C bq = pb[u];
      pb[u] = load_b(q + PF);
      // stage 1, plane q: x1 = (omega / d) b
      const bool in1 = m.inside && q >= 0 && q < n;
      const C x1q = in1 ? wd * bq : C(0);
      s1[sl][me] = x1q;
      // stage 2, plane q - 1: x2 = x1 + (omega / d) (b - A x1)
      const int p2 = q - 1;
      C x2q = C(0);
      if (m.inside && p2 >= 0 && p2 < n && p2 >= m.z0 - 1) {
        const C kx = m3_k(s1[sl ^ 1], m.tx, m.ty, x1b, x1a, x1q);
        const C Ax = x1b + op.a * op.ih2 * kx;
        x2q = x1b + wd * (b1 - Ax);
        if (m.core && p2 >= m.z0 && p2 < m.z1) st<T, C>(xo + (int64_t)p2 * nn, x2q);
      }
      s2[sl ^ 1][me] = x2q;
      // stage 3, plane q - 2: r = b - A x2 (zero off the grid)
      const int p3 = q - 2;
      C r = C(0);
      if (m.inside && p3 >= 0 && p3 < n && p3 >= m.z0) {
        const C kx = m3_k(s2[sl], m.tx, m.ty, x2b, x2a, x2q);
        const C Ax = x2b + op.a * op.ih2 * kx;
        r = b2 - Ax;
      }
      s3[sl][me] = r;
      // stage 4, plane p = q - 3 (written last step): coarse plane K takes
      // fine planes 2K, 2K + 1, 2K + 2 with weights w3[dk + 1]
      const int p4 = q - 3;
      if (owner && p4 >= m.z0 && p4 <= m.z1) {
        const C* rp = s3[sl ^ 1];
        auto add = [&](int dk) {
#pragma unroll
          for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
            for (int di = -1; di <= 1; ++di)
              acc += w3[di + 1] * w3[dj + 1] * w3[dk + 1] * rp[(m.ty + dj) * M3_T + m.tx + di];
        };
        if (p4 & 1) {
          add(0);                                   // centre plane of K = (p - 1) / 2
        } else {
          const int K = (p4 >> 1) - 1;              // plane 2K + 2 completes K
          if (2 * K + 1 >= m.z0 && 2 * K + 1 < zc1) {
            add(1);
            const C v = acc * (C(0.125) * bscale);
            const int64_t pc = ((int64_t)K * nc + J) * nc + I;
            st<TC, C>(bc + inst * sbc + pc, v);
            if (zero_next) st<TC, C>(xc + inst * sxc + pc, omega * v / level_diag<3, KIND_TENSOR, C>(opc, (int)pc, I, J, K));
          }
          acc = C(0);
          if (p4 + 1 < zc1) add(-1);                // first plane of K + 1
        }
      }
      m3_sync();
      b2 = b1;
      b1 = bq;
      x1a = x1b;
      x1b = x1q;
      x2a = x2b;
      x2b = x2q;
    }
  }
}

// Interpolation slots of fine coordinate c from a coarse axis of nc nodes
// (coarse node I at fine 2I + 1): two indices and weights, the unused slot
// with weight zero at a valid index.  Slot order matches prolong_at's term
// order, and a zero-weight term adds an exact zero, so sums agree with it.
template <class C>
__device__ __forceinline__ void m3_slots(int c, int nc, int (&ix)[2], C (&w)[2]) {
  if (c & 1) {
    ix[0] = ix[1] = (c - 1) >> 1;
    w[0] = C(1);
    w[1] = C(0);
  } else {
    const int lo = (c >> 1) - 1, hi = c >> 1;
    ix[0] = lo >= 0 ? lo : 0;
    ix[1] = hi < nc ? hi : nc - 1;
    w[0] = lo >= 0 ? C(0.5) : C(0);
    w[1] = hi < nc ? C(0.5) : C(0);
  }
}

// Coarse patch of a tile: the coarse nodes any of its 32 fine columns
// interpolates from lie in 18 consecutive indices from (o >> 1) - 1, o the
// fine index of the tile's first thread.
constexpr int M3_P = 18;

// Prolongation and two post-smoothing sweeps: y = xin + es P e, then
// y1 = y + (omega / d) (b - A y) and y2 likewise -> xout (xout != xin).
// Each coarse plane is staged once per tile as an 18 x 18 patch in LDS
// (two slots: fine plane q reads coarse planes ceil(q/2) - 1 and floor(q/2));
// plane m + 1 is written on step 2m + 1, its loads issued four steps before.
template <class T, class TE, class C>
__global__ __launch_bounds__(M3_T * M3_T) __attribute__((amdgpu_waves_per_eu(sizeof(C) == 4 ? 8 : 4)))
void k_up3d_march(const T* __restrict__ xin, int64_t sxi,
                                                           const TE* __restrict__ e, int64_t se,
                                                           const T* __restrict__ b, int64_t sb,
                                                           T* __restrict__ xout, int64_t sxo, March3Geo g, int nc,
                                                           LevelOp<C> op, C omega, C es) {
  constexpr int PF = sizeof(C) == 8 ? 2 : M3_PF_UP;
  static_assert(PF % 2 == 0, "blocks of PF steps start on even planes");
  __shared__ C s1[2][M3_T * M3_T];   // y planes
  __shared__ C s2[2][M3_T * M3_T];   // y1 planes
  __shared__ C sc[2][M3_P * M3_P];   // coarse patches
  const March3Pos<2> m(g);
  const int64_t inst = blockIdx.y;
  const int n = g.n;
  const int64_t nn = (int64_t)n * n;
  const int64_t col = (int64_t)(m.inside ? m.j : 0) * n + (m.inside ? m.i : 0);
  const T* xi = xin + inst * sxi + col;
  const T* bi = b + inst * sb + col;
  T* xo = xout + inst * sxo + col;
  const C wd = omega / level_diag<3, KIND_FINE, C>(op, 0, 0, 0, 0);
  const int me = m.ty * M3_T + m.tx;
  const int qlast = m.z1 + 1;
  // this thread's interpolation slots in x and y, as patch offsets
  const int cx0 = ((m.i - m.tx) >> 1) - 1, cy0 = ((m.j - m.ty) >> 1) - 1;
  int ixx[2], ixy[2];
  C wx[2], wy[2];
  m3_slots<C>(m.inside ? m.i : 0, nc, ixx, wx);
  m3_slots<C>(m.inside ? m.j : 0, nc, ixy, wy);
  int px[2], py[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    px[u] = min(max(ixx[u] - cx0, 0), M3_P - 1);
    py[u] = min(max(ixy[u] - cy0, 0), M3_P - 1);
  }
  // the patch entry this thread loads (threads past the patch load nothing)
  const int tid = (int)threadIdx.x;
  const bool loader = tid < M3_P * M3_P;
  const int lj = loader ? tid / M3_P : 0, li = loader ? tid - lj * M3_P : 0;
  const int gI = cx0 + li, gJ = cy0 + lj;
  const bool lin = loader && gI >= 0 && gI < nc && gJ >= 0 && gJ < nc;
  const TE* ep = e + inst * se + (lin ? (int64_t)gJ * nc + gI : 0);
  const int64_t ncc = (int64_t)nc * nc;
  // unconditional (clamped) like load_b: patch entries off the coarse grid,
  // and planes off it, are read only with zero interpolation weight
  auto load_c = [&](int K) { return ld<TE, C>(ep + (int64_t)min(max(K, 0), nc - 1) * ncc); };
  // fine planes start even (z0 is 0 or a multiple of 16): the first step
  // q0 = 2 m0 reads coarse planes m0 - 1 and m0
  const int m0 = (m.z0 - 2) >> 1;
  if (loader) {
    sc[(m0 - 1) & 1][tid] = load_c(m0 - 1);
    sc[m0 & 1][tid] = load_c(m0);
  }
  // coarse planes in flight: step 2k + 1 writes plane k + 1, and the odd
  // steps of a block of PF (even) steps take slots 0 .. PF/2 - 1 in turn
  C pc_[PF / 2];
#pragma unroll
  for (int u = 0; u < PF / 2; ++u) pc_[u] = load_c(m0 + 1 + u);
  auto load_xb = [&](int q, C& x, C& bb) {   // unconditional, as load_b of the down kernel
    const int64_t o = (int64_t)min(max(q, 0), n - 1) * nn;
    x = ld<T, C>(xi + o);
    bb = ld<T, C>(bi + o);
  };
  C px_[PF], pb_[PF];   // x and b, as the ring of the down kernel
#pragma unroll
  for (int u = 0; u < PF; ++u) load_xb(m.z0 - 2 + u, px_[u], pb_[u]);
  m3_sync();
  // windows: b at q-1, q-2; y at q-2, q-1, q; y1 at q-3, q-2, q-1
  C b1 = C(0), b2 = C(0), ya = C(0), yb = C(0), y1a = C(0), y1b = C(0);
  // whole blocks of PF steps: steps past qlast write nothing (their planes
  // lie beyond the chunk's last output)
  for (int q0 = m.z0 - 2; q0 <= qlast; q0 += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int q = q0 + u;
      const int sl = q & 1;
      const C xq = px_[u], bq = pb_[u];
      load_xb(q + PF, px_[u], pb_[u]);
      // stage 1, plane q: y = x + es P e (same terms and order as prolong_at)
      const bool in1 = m.inside && q >= 0 && q < n;
      C yq = C(0);
      if (in1) {
        int iz[2];
        C wz[2];
        m3_slots<C>(q, nc, iz, wz);
        C acc = C(0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const C* pc = sc[iz[c] & 1];
#pragma unroll
          for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) acc += wx[a] * wy[bb] * wz[c] * pc[py[bb] * M3_P + px[a]];
        }
        yq = xq + es * acc;
      }
      s1[sl][me] = yq;
      // stage 2, plane q - 1: first sweep
      const int p2 = q - 1;
      C y1q = C(0);
      if (m.inside && p2 >= 0 && p2 < n && p2 >= m.z0 - 1) {
        const C kx = m3_k(s1[sl ^ 1], m.tx, m.ty, yb, ya, yq);
        const C Ax = yb + op.a * op.ih2 * kx;
        y1q = yb + wd * (b1 - Ax);
      }
      s2[sl ^ 1][me] = y1q;
      // stage 3, plane q - 2: second sweep, stored
      const int p3 = q - 2;
      if (m.core && p3 >= m.z0 && p3 < m.z1) {
        const C kx = m3_k(s2[sl], m.tx, m.ty, y1b, y1a, y1q);
        const C Ax = y1b + op.a * op.ih2 * kx;
        st<T, C>(xo + (int64_t)p3 * nn, y1b + wd * (b2 - Ax));
      }
      // odd step 2k + 1 (q0 is even): coarse plane k + 1 into its slot (plane
      // k - 1's, last read on step 2k), then the slot's next plane
      if (u & 1) {
        const int K = (q >> 1) + 1;
        if (loader) sc[K & 1][tid] = pc_[u >> 1];
        pc_[u >> 1] = load_c(K + PF / 2);
      }
      m3_sync();
      b2 = b1;
      b1 = bq;
      ya = yb;
      yb = yq;
      y1a = y1b;
      y1b = y1q;
    }
  }
}

// Launch geometry of a 3D march with a halo of h nodes: chunks of 32
// planes when that gives at least two workgroups per compute unit over the
// launch, else 16.
inline March3Geo march3_geo(int n, int B, int h) {
  const int cw = M3_T - 2 * h;
  March3Geo g{};
  g.n = n;
  g.ntx = (n + cw - 1) / cw;
  g.zlen = n < 32 ? n : 32;
  g.nz = (n + g.zlen - 1) / g.zlen;
  if ((int64_t)g.ntx * g.ntx * g.nz * B < 512 && n > 16) {
    g.zlen = 16;
    g.nz = (n + 15) / 16;
  }
  return g;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
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
  op.st9 = nullptr;
  if (h->vark && l > 0) {
    const char* st9 = h->ws + (dbl ? h->plan.st9_d : h->plan.st9_f);
    op.st9 = reinterpret_cast<const C*>(st9) + h->st9_off[l];
  }
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
// threads of the two-nodes-per-thread 3D Galerkin kernels: n^2 ceil(n / 2)
inline int64_t pair_threads(int n) { return (int64_t)n * n * ((n + 1) / 2); }
// Two nodes per thread pay with FP32 arithmetic on launches of about a
// million nodes and more (measured on MI355X at 128^3: 64^3 level with 7 to
// 32 blocks, 32^3 with 32); smaller launches need the threads of one node
// each, and FP64 the registers.
template <class C>
inline bool pairs3(int64_t N, int B) { return sizeof(C) == 4 && N * B >= (int64_t)1 << 20; }

}  // namespace

// First level handled by the one-workgroup tail (2D): the largest set of
// coarse levels whose three LDS vectors and factor copies fit the device's
// LDS per workgroup (at most 128 KiB).
template <class TI, class TM>
Multigrid<TI, TM>::Multigrid(aao_problem* h, hipStream_t st, const double* L, int cinv_set)
    : h_(h), st_(st), levels_((int)h->lev_n.size()) {
  for (int i = 0; i < h->s; ++i) a_[i] = h->tau * L[i * h->s + i];
  cinv_set_ = cinv_set >= 0 ? cinv_set : ((L == h->LT) ? 1 : 0);
  if (h->dim == 3) {
    // The 3D instantiation of the LDS tail faulted on gfx950 (aperture
    // violation) for reasons not yet established; 3D runs every level with
    // grid kernels and a pointwise exact solve on the one-node level.
    l0_ = levels_;
    tail_bytes_ = 0;
    set_level_storage();
    return;
  }
  const size_t budget = h->lds_budget;
  auto cost = [&](int l) { return sizeof(C) * (3 * (size_t)h->lev_N[l] + 6 * (size_t)h->lev_n[l]); };
  l0_ = levels_ - 1;
  size_t bytes = cost(levels_ - 1) + sizeof(C) * 2 * (size_t)h->lev_N[levels_ - 1] +
                 sizeof(C) * (size_t)(h->fd_n * h->fd_n + h->fd_n);
  // measured on MI355X (512^2, s=3): one workgroup is faster than grid
  // kernels up to a 32 x 32 level, slower above it
  const int64_t tail_max = h->opts.mg_tail_max > 0 ? h->opts.mg_tail_max : 1024;
  // Q2: level 0 (five-diagonal factors) runs in the grid kernels only
  const int l0_min = h->fe_order == 2 ? 1 : 0;
  while (l0_ > l0_min && levels_ - l0_ < TAIL_MAXL) {
    const size_t more = bytes + cost(l0_ - 1);
    if (more > budget) break;
    if (tail_max > 0 && h->lev_N[l0_ - 1] > tail_max) break;
    bytes = more;
    --l0_;
  }
  tail_bytes_ = bytes;
  // The register-resident tail (k_tail_fast): one or two Galerkin smoothing
  // levels above an exact coarsest level of at most 16 x 16, the first at
  // most 64 x 64.  Unless the caller bounds the tail, it takes a 64 x 64
  // level too (measured on MI355X at 512^2, s = 3: faster than the tiled
  // kernels for it).
  fast_nls_ = 0;
  fast_npt_ = 0;
  fast_bytes_ = 0;
  const int nlast = h->lev_n[levels_ - 1];
  const bool fd = h->fd_n > 0 && h->fd_n == nlast;
  auto fast_ok = [&](int l) {
    const int nls = levels_ - 1 - l;
    if (l < 1 || nls < 1 || nls > 2 || nlast > TF_NC || (fd && h->vark)) return false;
    if (nls == 2 && sizeof(C) != 4) return false;   // FP64 coefficients of 4 nodes per thread do not fit registers
    if (h->lev_n[l] > (nls == 1 ? 32 : TF_NMAX)) return false;
    TailFastArgs<C> ta{};
    for (int t = 0; t <= nls; ++t) ta.n[t] = h->lev_n[l + t];
    return (size_t)tail_fast_layout<C>(ta, nls) * sizeof(C) <= budget;
  };
  if (h->opts.mg_tail_max <= 0 && h->tune.tail_extend && l0_ > 1 && levels_ - l0_ == 2 && fast_ok(l0_ - 1)) --l0_;
  if (fast_ok(l0_)) {
    fast_nls_ = levels_ - 1 - l0_;
    fast_npt_ = fast_nls_ == 2 ? 4 : 1;
    TailFastArgs<C> ta{};
    for (int t = 0; t <= fast_nls_; ++t) ta.n[t] = h->lev_n[l0_ + t];
    fast_bytes_ = (size_t)tail_fast_layout<C>(ta, fast_nls_) * sizeof(C);
  }
  set_level_storage();
}

// The precision schedule of the V-cycle (Sec. 4 cites per-level decreasing
// precision and a coarse-solve precision apart from the smoother's): levels
// from opts.mg_low_from on (default 1) are stored in TM, the ones above in
// TI; with opts.mg_coarse_fp32 the coarse solve -- the one-workgroup tail
// and its exact coarsest solve in 2D, the exactly solved coarsest level in
// 3D -- keeps TI as well.  Level 0 is always TI.
template <class TI, class TM>
void Multigrid<TI, TM>::set_level_storage() {
  low_.assign(levels_ + 1, 0);
  if (std::is_same<TI, TM>::value) return;
  const int from = h_->opts.mg_low_from > 0 ? h_->opts.mg_low_from : 1;
  for (int l = 1; l < levels_; ++l) {
    const bool coarse_solve = h_->dim == 2 ? l >= l0_ : l == levels_ - 1;
    low_[l] = l >= from && !(h_->opts.mg_coarse_fp32 && coarse_solve);
  }
}

template <class TI, class TM>
template <class F>
hipError_t Multigrid<TI, TM>::typed1(int l, F&& f) const {
  if constexpr (std::is_same<TI, TM>::value) {
    return f(TI{});
  } else {
    if (low(l)) return f(TM{});
    return f(TI{});
  }
}

template <class TI, class TM>
template <class F>
hipError_t Multigrid<TI, TM>::typed2(int l, F&& f) const {
  if constexpr (std::is_same<TI, TM>::value) {
    return f(TI{}, TI{});
  } else {
    if (low(l)) return low(l + 1) ? f(TM{}, TM{}) : f(TM{}, TI{});
    return low(l + 1) ? f(TI{}, TM{}) : f(TI{}, TI{});
  }
}

#define MG_TRY(...)                           \
  do {                                        \
    hipError_t e_ = (__VA_ARGS__);            \
    if (e_ != hipSuccess) return e_;          \
  } while (0)

template <class TI, class TM>
const typename Multigrid<TI, TM>::C* Multigrid<TI, TM>::coarse_inv(int stage) const {
  const bool dbl = sizeof(C) == 8;
  const C* base = reinterpret_cast<const C*>(h_->ws + (dbl ? h_->plan.cinv_d : h_->plan.cinv_f));
  return base + ((int64_t)cinv_set_ * h_->s + stage) * h_->cinv_N * h_->cinv_N;
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::smooth(int l, int stage, Vec xin, Vec xout, Vec b, bool zero_init, int B) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const C omega = (C)h_->omega;
  const dim3 g = grid2(op.N, B);
  const int d3 = h_->dim == 3;
  if (l == 0) {
    if (h_->fe_order == 2) {
      return fe_q2_smooth<TI>(h_, a_[stage], (const TI*)xin.ptr, xin.stride, (TI*)xout.ptr, xout.stride,
                              (const TI*)b.ptr, b.stride, h_->omega, zero_init, B, st_);
    } else if (h_->vark) {
      if (d3) hipLaunchKernelGGL((k_smooth<3, KIND_FINE_VK, TI, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, (TI*)xout.ptr, xout.stride, (const TI*)b.ptr, b.stride, op, omega, (int)zero_init);
      else hipLaunchKernelGGL((k_smooth<2, KIND_FINE_VK, TI, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, (TI*)xout.ptr, xout.stride, (const TI*)b.ptr, b.stride, op, omega, (int)zero_init);
    } else {
      if (d3) hipLaunchKernelGGL((k_smooth<3, KIND_FINE, TI, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, (TI*)xout.ptr, xout.stride, (const TI*)b.ptr, b.stride, op, omega, (int)zero_init);
      else hipLaunchKernelGGL((k_smooth<2, KIND_FINE, TI, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, (TI*)xout.ptr, xout.stride, (const TI*)b.ptr, b.stride, op, omega, (int)zero_init);
    }
  } else {
    return typed1(l, [&](auto t) {
      using TL = decltype(t);
      if (d3 && pairs3<C>(op.N, B)) hipLaunchKernelGGL((k_smooth3t<TL, C>), grid2(pair_threads(op.n), B), dim3(TPB), 0, st_, (const TL*)xin.ptr, xin.stride, (TL*)xout.ptr, xout.stride, (const TL*)b.ptr, b.stride, op, omega, (int)zero_init);
      else if (d3) hipLaunchKernelGGL((k_smooth<3, KIND_TENSOR, TL, C>), g, dim3(TPB), 0, st_, (const TL*)xin.ptr, xin.stride, (TL*)xout.ptr, xout.stride, (const TL*)b.ptr, b.stride, op, omega, (int)zero_init);
      else hipLaunchKernelGGL((k_smooth<2, KIND_TENSOR, TL, C>), g, dim3(TPB), 0, st_, (const TL*)xin.ptr, xin.stride, (TL*)xout.ptr, xout.stride, (const TL*)b.ptr, b.stride, op, omega, (int)zero_init);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::resid_restrict(int l, int stage, Vec x, Vec b, Vec bc, Vec xc, bool zero_next, int B) {
  const LevelOp<C> opf = make_op<C>(h_, l, a_[stage]);
  const LevelOp<C> opc = make_op<C>(h_, l + 1, a_[stage]);
  const C omega = (C)h_->omega;
  const dim3 g = grid2(opc.N, B);
  const int d3 = h_->dim == 3, z = (int)zero_next;
  if (split_restrict(l)) {
    // residual once per fine node into the level's residual buffer, then
    // the full weighting (3D has constant kappa: tensor or fine operator;
    // Q2 level 0: its 25-point operator)
    Vec r{h_->ws + h_->plan.mgR[l], (int64_t)opf.N};
    const C bs = l == 0 ? (C)h_->mg_scale : C(1);
    const dim3 gf = grid2(opf.N, B);
    return typed2(l, [&](auto tf, auto tc) {
      using TF = decltype(tf);
      using TC = decltype(tc);
#define RES(D, K) hipLaunchKernelGGL((k_residual<D, K, TF, C>), gf, dim3(TPB), 0, st_, (const TF*)x.ptr, x.stride, (const TF*)b.ptr, b.stride, (TF*)r.ptr, r.stride, opf)
      if (!d3) {
        // level 0 of Q2 elements, always stored as TI
        if constexpr (std::is_same<TF, TI>::value)
          MG_TRY(fe_q2_residual<TI>(h_, a_[stage], (const TI*)x.ptr, x.stride, (const TI*)b.ptr, b.stride,
                                    (TI*)r.ptr, r.stride, B, st_));
        else
          return hipErrorInvalidValue;
      } else if (l == 0) {
        RES(3, KIND_FINE);
      } else if (pairs3<C>(opf.N, B)) {
        hipLaunchKernelGGL((k_residual3t<TF, C>), grid2(pair_threads(opf.n), B), dim3(TPB), 0, st_, (const TF*)x.ptr,
                           x.stride, (const TF*)b.ptr, b.stride, (TF*)r.ptr, r.stride, opf);
      } else {
        RES(3, KIND_TENSOR);
      }
#undef RES
      MG_TRY(hipGetLastError());
      MG_TRY(mark("k_residual", l));
      if (d3)
        hipLaunchKernelGGL((k_restrict<3, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)r.ptr, r.stride, (TC*)bc.ptr,
                           bc.stride, (TC*)xc.ptr, xc.stride, opf.n, opc, omega, z, bs);
      else
        hipLaunchKernelGGL((k_restrict<2, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)r.ptr, r.stride, (TC*)bc.ptr,
                           bc.stride, (TC*)xc.ptr, xc.stride, opf.n, opc, omega, z, bs);
      return hipGetLastError();
    });
  }
  if (l == 0) {
    const C bs = (C)h_->mg_scale;
    return typed1(1, [&](auto tc) {
      using TC = decltype(tc);
#define RR0(D, K) hipLaunchKernelGGL((k_resid_restrict<D, K, TI, TC, C>), g, dim3(TPB), 0, st_, (const TI*)x.ptr, x.stride, (const TI*)b.ptr, b.stride, (TC*)bc.ptr, bc.stride, (TC*)xc.ptr, xc.stride, opf, opc, omega, z, bs)
      if (h_->vark) { if (d3) RR0(3, KIND_FINE_VK); else RR0(2, KIND_FINE_VK); }
      else { if (d3) RR0(3, KIND_FINE); else RR0(2, KIND_FINE); }
#undef RR0
      return hipGetLastError();
    });
  }
  return typed2(l, [&](auto tf, auto tc) {
    using TF = decltype(tf);
    using TC = decltype(tc);
    if (d3) hipLaunchKernelGGL((k_resid_restrict<3, KIND_TENSOR, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)x.ptr, x.stride, (const TF*)b.ptr, b.stride, (TC*)bc.ptr, bc.stride, (TC*)xc.ptr, xc.stride, opf, opc, omega, z, C(1));
    else hipLaunchKernelGGL((k_resid_restrict<2, KIND_TENSOR, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)x.ptr, x.stride, (const TF*)b.ptr, b.stride, (TC*)bc.ptr, bc.stride, (TC*)xc.ptr, xc.stride, opf, opc, omega, z, C(1));
    return hipGetLastError();
  });
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::prolong(int l, Vec xin, Vec ec, Vec xout, int B) {
  const int nf = h_->lev_n[l], nc = h_->lev_n[l + 1];
  const int Nf = (int)h_->lev_N[l];
  const dim3 g = grid2(Nf, B);
  // the coarse grid levels, and level 0 in 3D (2D fuses it into the first
  // post-smoothing sweep); at level 0 the FP16 levels' scale is removed
  const C es = l == 0 ? (C)(1.0 / h_->mg_scale) : C(1);
  return typed2(l, [&](auto tf, auto tc) {
    using TF = decltype(tf);
    using TC = decltype(tc);
    if (h_->dim == 2)
      hipLaunchKernelGGL((k_prolong<2, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)xin.ptr, xin.stride,
                         (const TC*)ec.ptr, ec.stride, (TF*)xout.ptr, xout.stride, nf, Nf, nc, es);
    else
      hipLaunchKernelGGL((k_prolong<3, TF, TC, C>), g, dim3(TPB), 0, st_, (const TF*)xin.ptr, xin.stride,
                         (const TC*)ec.ptr, ec.stride, (TF*)xout.ptr, xout.stride, nf, Nf, nc, es);
    return hipGetLastError();
  });
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::prolong_smooth0(int stage, Vec xin, Vec ec, Vec b, Vec xout, int B) {
  const LevelOp<C> op = make_op<C>(h_, 0, a_[stage]);
  const int nc = h_->lev_n[1];
  const C omega = (C)h_->omega;
  const dim3 g = grid2(op.N, B);
  const C es = (C)(1.0 / h_->mg_scale);
  return typed1(1, [&](auto tc) {
    using TC = decltype(tc);
#define PS0(D, V) hipLaunchKernelGGL((k_prolong_smooth<D, V, TI, TC, C>), g, dim3(TPB), 0, st_, (const TI*)xin.ptr, xin.stride, (const TC*)ec.ptr, ec.stride, (const TI*)b.ptr, b.stride, (TI*)xout.ptr, xout.stride, op, nc, omega, es)
    if (h_->dim == 3) { if (h_->vark) PS0(3, true); else PS0(3, false); }
    else { if (h_->vark) PS0(2, true); else PS0(2, false); }
#undef PS0
    return hipGetLastError();
  });
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::tail(int stage, Vec x, Vec b, bool zero_init, int B) {
  if (h_->dim != 2) return hipErrorUnknown;   // the tail is 2D only
  if (fast_nls_ > 0 && zero_init) {
    const int nls = fast_nls_;
    TailFastArgs<C> tf{};
    for (int t = 0; t <= nls; ++t) tf.n[t] = h_->lev_n[l0_ + t];
    tf.a = (C)a_[stage];
    tf.omega = (C)h_->omega;
    tf.nu1 = h_->opts.nu1;
    tf.nu2 = h_->opts.nu2;
    for (int t = 0; t < nls; ++t) {
      const LevelOp<C> op = make_op<C>(h_, l0_ + t, a_[stage]);
      tf.tri[t] = op.tri;
      tf.st9[t] = op.st9;
    }
    const bool dbl = sizeof(C) == 8;
    const bool use_fd = h_->fd_n > 0 && h_->fd_n == h_->lev_n[levels_ - 1];
    tf.fd = use_fd ? reinterpret_cast<const C*>(h_->ws + (dbl ? h_->plan.fd_d : h_->plan.fd_f)) : nullptr;
    tf.cinv = use_fd ? nullptr : coarse_inv(stage);
    tail_fast_layout<C>(tf, nls);
    const dim3 g((unsigned)B), blk((unsigned)TAIL_THREADS);
    return typed1(l0_, [&](auto t) {
      using TS = decltype(t);
      TS* xp = (TS*)x.ptr;
      const TS* bp = (const TS*)b.ptr;
#define TF_GO(K, NL, NP, F) \
  hipLaunchKernelGGL((k_tail_fast<K, NL, NP, F, TS, C>), g, blk, fast_bytes_, st_, xp, x.stride, bp, b.stride, tf)
#define TF_KIND(NL, NP)                                 \
  do {                                                  \
    if (h_->vark) TF_GO(KIND_STENCIL9, NL, NP, false);  \
    else if (use_fd) TF_GO(KIND_TENSOR, NL, NP, true);  \
    else TF_GO(KIND_TENSOR, NL, NP, false);             \
  } while (0)
      if (nls == 1) TF_KIND(1, 1);
      else if constexpr (sizeof(C) == 4) TF_KIND(2, 4);
#undef TF_KIND
#undef TF_GO
      return hipGetLastError();
    });
  }
  if (l0_ > 0 && !zero_init) return hipErrorInvalidValue;   // coarse tails always start from zero
  if (tail_bytes_ > h_->lds_budget) return hipErrorInvalidValue;
  TailArgs<C> ta{};
  ta.nl = levels_ - l0_;
  ta.first_fine = l0_ == 0 && !h_->fe;   // Q1: level 0 is a tensor level too (Q2 keeps it out of the tail)
  ta.zero_init = zero_init;
  ta.nu1 = h_->opts.nu1;
  ta.nu2 = h_->opts.nu2;
  ta.omega = (C)h_->omega;
  int off = 0;
  for (int t = 0; t < ta.nl; ++t) {
    ta.op[t] = make_op<C>(h_, l0_ + t, a_[stage]);
    ta.off[t] = off;
    off += 3 * (int)ta.op[t].N;
  }
  for (int t = 0; t < ta.nl; ++t) {
    ta.toff[t] = off;
    off += 6 * ta.op[t].n;
  }
  ta.fd = nullptr;
  ta.fdoff = off;
  if (h_->fd_n > 0 && h_->fd_n == ta.op[ta.nl - 1].n) {
    const bool dbl = sizeof(C) == 8;
    ta.fd = reinterpret_cast<const C*>(h_->ws + (dbl ? h_->plan.fd_d : h_->plan.fd_f));
    off += h_->fd_n * h_->fd_n + h_->fd_n;
  }
  ta.scratch = off;
  off += 2 * (int)ta.op[ta.nl - 1].N;
  ta.cinv = coarse_inv(stage);
  const size_t shm = (size_t)off * sizeof(C);
  const int nth = ta.op[0].N >= TAIL_THREADS ? TAIL_THREADS : (ta.op[0].N >= 256 ? 256 : 64);
  const dim3 g((unsigned)B), blk((unsigned)nth);
  if (l0_ == 0) {
    if (h_->vark)
      hipLaunchKernelGGL((k_tail<true, TI, TI, C>), g, blk, shm, st_, (TI*)x.ptr, x.stride, (const TI*)b.ptr, b.stride, ta);
    else
      hipLaunchKernelGGL((k_tail<false, TI, TI, C>), g, blk, shm, st_, (TI*)x.ptr, x.stride, (const TI*)b.ptr, b.stride, ta);
  } else {
    return typed1(l0_, [&](auto t) {
      using TS = decltype(t);
      hipLaunchKernelGGL((k_tail<false, TS, TS, C>), g, blk, shm, st_, (TS*)x.ptr, x.stride, (const TS*)b.ptr, b.stride, ta);
      return hipGetLastError();
    });
  }
  return hipGetLastError();
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::down2d(int l, int stage, Vec b, const void* x0, int64_t sx0, Vec xout, Vec bc, int B,
                                     const Coupling* cpl) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const int nc = h_->lev_n[l + 1];
  const C omega = (C)h_->omega;
  // tall tiles for batched launches (HBM-bound); latency-bound single blocks
  // keep the short ones (more workgroups, shorter critical path)
  const bool tall = sizeof(C) == 4 && B >= h_->tune.tall_min_b;
  constexpr int TY0L = sizeof(C) == 4 ? TY0 : TCY;
  const int ty = tall ? TY0 : TCY;
  const int gx = (nc + TCX - 1) / TCX, gy = (nc + ty - 1) / ty;
  const dim3 g((unsigned)(gx * gy * B));
  const int nu = h_->opts.nu1;
  const int nz = (l == 0 && cpl) ? cpl->nz : 0;
  CplArgs<TI, C> ca{};
  if (nz > 0) {
    ca.z = cpl->z;
    ca.sz = cpl->sz;
    ca.zs = cpl->zstride;
    for (int q = 0; q < nz; ++q) ca.c[q] = (C)(h_->tau * cpl->Lc[cpl->nz * h_->s + q]);
    ca.out = cpl->out;
    ca.so = cpl->so;
  }
  const C bs = l == 0 ? (C)h_->mg_scale : C(1);
  // TF / TC: storage of this level and of the next (the precision schedule)
#define DN_T(K, NU, TF, NZ, CA, TYV) hipLaunchKernelGGL((k_down2d<K, NU, TF, TC, C, NZ, TYV>), g, dim3(256), 0, st_, (const TF*)b.ptr, b.stride, (const TF*)x0, sx0, (TF*)xout.ptr, xout.stride, (TC*)bc.ptr, bc.stride, op, nc, omega, gx, gy, CA, bs)
#define DN(K, NU, TF, NZ, CA) do { if (tall) DN_T(K, NU, TF, NZ, CA, TY0L); else DN_T(K, NU, TF, NZ, CA, TCY); } while (0)
#define DN_NU(K, TF, NZ, CA) do { if (nu == 1) DN(K, 1, TF, NZ, CA); else if (nu == 2) DN(K, 2, TF, NZ, CA); else DN(K, 3, TF, NZ, CA); } while (0)
#define DN_Z(K) do { if (nz == 0) DN_NU(K, TI, 0, ca); else if (nz == 1) DN_NU(K, TI, 1, ca); else DN_NU(K, TI, 2, ca); } while (0)
  // batched cycles from zero: the row march on level 0 of the
  // constant-coefficient operator (with Rana's coupling terms) and on the
  // tensor levels (Q1 level 0, Galerkin levels of constant kappa) when
  // they give the chip 4 waves per SIMD at least (a tensor wave's chain of
  // rows is long: fewer waves leave it latency-bound, where the tiles are
  // faster); 16-row segments while one round of waves does not fill the
  // chip (8 per SIMD), 32-row ones (less halo) beyond
  const bool fine_const = l == 0 && !h_->fe && !h_->vark;
  const bool tensor = (l == 0 && h_->fe) || (l > 0 && !h_->vark);
  const int nf = h_->lev_n[l];
  const int nzm = fine_const ? nz : 0;
  const int ow = 62 - 2 * (nu + (nzm > 0 ? 1 : 0));
  const int nstrips = (nf + ow - 1) / ow;
  const int64_t waves16 = (int64_t)nstrips * ((nf + 15) / 16) * B;
  if (!x0 && B >= h_->tune.tall_min_b && (fine_const || (tensor && waves16 >= 4 * 4 * 256))) {
    const bool seg32 = waves16 > 8 * 4 * 256;
    const int seg = seg32 ? 32 : 16;
    const int nsegs = (nf + seg - 1) / seg;
    const int64_t units = (int64_t)nstrips * nsegs * B;
    const dim3 gm((unsigned)((units + 3) / 4));
#define DNM(K, NU, TF, NZ, CA, SEG) hipLaunchKernelGGL((k_down2d_march<K, NU, TF, TC, C, NZ, SEG>), gm, dim3(256), 0, st_, (const TF*)b.ptr, b.stride, (TF*)xout.ptr, xout.stride, (TC*)bc.ptr, bc.stride, op, nc, omega, nstrips, nsegs, units, CA, bs)
#define DNM_S(K, NU, TF, NZ, CA) do { if (seg32) DNM(K, NU, TF, NZ, CA, 32); else DNM(K, NU, TF, NZ, CA, 16); } while (0)
#define DNM_NU(K, TF, NZ, CA) do { if (nu == 1) DNM_S(K, 1, TF, NZ, CA); else if (nu == 2) DNM_S(K, 2, TF, NZ, CA); else DNM_S(K, 3, TF, NZ, CA); } while (0)
    if (fine_const)
      return typed1(1, [&](auto tc) {
        using TC = decltype(tc);
        if (nz == 0) DNM_NU(KIND_FINE, TI, 0, ca); else if (nz == 1) DNM_NU(KIND_FINE, TI, 1, ca); else DNM_NU(KIND_FINE, TI, 2, ca);
        return hipGetLastError();
      });
    if (l == 0)
      return typed1(1, [&](auto tc) {
        using TC = decltype(tc);
        DNM_NU(KIND_TENSOR, TI, 0, ca);
        return hipGetLastError();
      });
    return typed2(l, [&](auto tf, auto tc) {
      using TF = decltype(tf);
      using TC = decltype(tc);
      CplArgs<TF, C> cm{};
      DNM_NU(KIND_TENSOR, TF, 0, cm);
      return hipGetLastError();
    });
#undef DNM_NU
#undef DNM_S
#undef DNM
  }
  if (l == 0)
    return typed1(1, [&](auto tc) {
      using TC = decltype(tc);
      // Q1 elements: level 0 is the tensor form M1(x)M1 + a (T(x)M1 + M1(x)T)
      // of the 1D element matrices (Rana's coupling formed separately)
      if (h_->fe) DN_NU(KIND_TENSOR, TI, 0, ca);
      else if (h_->vark) DN_Z(KIND_FINE_VK);
      else DN_Z(KIND_FINE);
      return hipGetLastError();
    });
  return typed2(l, [&](auto tf, auto tc) {
    using TF = decltype(tf);
    using TC = decltype(tc);
    CplArgs<TF, C> cm{};
    if (h_->vark) DN_NU(KIND_STENCIL9, TF, 0, cm); else DN_NU(KIND_TENSOR, TF, 0, cm);
    return hipGetLastError();
  });
#undef DN_Z
#undef DN_NU
#undef DN
#undef DN_T
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::up2d(int l, int stage, Vec xin, Vec ec, Vec b, Vec xout, int B) {
  const LevelOp<C> op = make_op<C>(h_, l, a_[stage]);
  const int nc = h_->lev_n[l + 1];
  const C omega = (C)h_->omega;
  const bool tall = sizeof(C) == 4 && B >= h_->tune.tall_min_b;
  constexpr int TY0L = sizeof(C) == 4 ? TY0 : TCY;
  const int ty = tall ? TY0 : TCY;
  const int gx = (nc + TCX - 1) / TCX, gy = (nc + ty - 1) / ty;
  const dim3 g((unsigned)(gx * gy * B));
  const int nu = h_->opts.nu2;
  const C es = l == 0 ? (C)(1.0 / h_->mg_scale) : C(1);
#define UP_T(K, NU, TF, TYV) hipLaunchKernelGGL((k_up2d<K, NU, TF, TC, C, TYV>), g, dim3(256), 0, st_, (const TF*)xin.ptr, xin.stride, (const TC*)ec.ptr, ec.stride, (const TF*)b.ptr, b.stride, (TF*)xout.ptr, xout.stride, op, nc, omega, gx, gy, es)
#define UP(K, NU, TF) do { if (tall) UP_T(K, NU, TF, TY0L); else UP_T(K, NU, TF, TCY); } while (0)
#define UP_NU(K, TF) do { if (nu == 1) UP(K, 1, TF); else if (nu == 2) UP(K, 2, TF); else UP(K, 3, TF); } while (0)
  // batched: the row march on level 0 of the constant-coefficient operator
  // and on the tensor levels (the choice and segment height as in down2d)
  const bool fine_const = l == 0 && !h_->fe && !h_->vark;
  const bool tensor = (l == 0 && h_->fe) || (l > 0 && !h_->vark);
  const int nf = h_->lev_n[l];
  const int ow = 64 - 2 * nu;
  const int nstrips = (nf + ow - 1) / ow;
  const int64_t waves16 = (int64_t)nstrips * ((nf + 15) / 16) * B;
  if (B >= h_->tune.tall_min_b && (fine_const || (tensor && waves16 >= 4 * 4 * 256))) {
    const bool seg32 = waves16 > 8 * 4 * 256;
    const int nsegs = (nf + (seg32 ? 32 : 16) - 1) / (seg32 ? 32 : 16);
    const int64_t units = (int64_t)nstrips * nsegs * B;
    const dim3 gm((unsigned)((units + 3) / 4));
#define UPM(K, NU, TF, SEG) hipLaunchKernelGGL((k_up2d_march<K, NU, TF, TC, C, SEG>), gm, dim3(256), 0, st_, (const TF*)xin.ptr, xin.stride, (const TC*)ec.ptr, ec.stride, (const TF*)b.ptr, b.stride, (TF*)xout.ptr, xout.stride, op, nc, omega, nstrips, nsegs, units, es)
#define UPM_S(K, NU, TF) do { if (seg32) UPM(K, NU, TF, 32); else UPM(K, NU, TF, 16); } while (0)
#define UPM_NU(K, TF) do { if (nu == 1) UPM_S(K, 1, TF); else if (nu == 2) UPM_S(K, 2, TF); else UPM_S(K, 3, TF); } while (0)
    if (l == 0)
      return typed1(1, [&](auto tc) {
        using TC = decltype(tc);
        if (fine_const) UPM_NU(KIND_FINE, TI); else UPM_NU(KIND_TENSOR, TI);
        return hipGetLastError();
      });
    return typed2(l, [&](auto tf, auto tc) {
      using TF = decltype(tf);
      using TC = decltype(tc);
      UPM_NU(KIND_TENSOR, TF);
      return hipGetLastError();
    });
#undef UPM_NU
#undef UPM_S
#undef UPM
  }
  if (l == 0)
    return typed1(1, [&](auto tc) {
      using TC = decltype(tc);
      if (h_->fe) UP_NU(KIND_TENSOR, TI);
      else if (h_->vark) UP_NU(KIND_FINE_VK, TI);
      else UP_NU(KIND_FINE, TI);
      return hipGetLastError();
    });
  return typed2(l, [&](auto tf, auto tc) {
    using TF = decltype(tf);
    using TC = decltype(tc);
    if (h_->vark) UP_NU(KIND_STENCIL9, TF); else UP_NU(KIND_TENSOR, TF);
    return hipGetLastError();
  });
#undef UP_NU
#undef UP
#undef UP_T
}

template <class TI, class TM>
bool Multigrid<TI, TM>::march3d_ok(int l, bool zero_init, bool pre, int B) const {
  return h_->dim == 3 && l == 0 && zero_init && !pre && !h_->vark && !h_->fe && levels_ > 1 &&
         h_->opts.nu1 == 2 && h_->opts.nu2 == 2 && std::is_same<TI, C>::value && B >= h_->tune.tall_min_b;
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::march3d_down(int stage, Vec b, Vec x2, Vec bc, Vec xc, bool zero_next, int B) {
  const LevelOp<C> opf = make_op<C>(h_, 0, a_[stage]);
  const LevelOp<C> opc = make_op<C>(h_, 1, a_[stage]);
  const C omega = (C)h_->omega;
  const C bs = (C)h_->mg_scale;
  const March3Geo g = march3_geo(h_->lev_n[0], B, 3);
  const dim3 grid((unsigned)(g.ntx * g.ntx * g.nz), (unsigned)B);
  MG_TRY(typed1(1, [&](auto tc) {
    using TC = decltype(tc);
    hipLaunchKernelGGL((k_down3d_march<TI, TC, C>), grid, dim3(M3_T * M3_T), 0, st_, (const TI*)b.ptr, b.stride,
                       (TI*)x2.ptr, x2.stride, (TC*)bc.ptr, bc.stride, (TC*)xc.ptr, xc.stride, g, opf, opc, omega,
                       (int)zero_next, bs);
    return hipGetLastError();
  }));
  return mark("k_down3d_march", 0);
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::march3d_up(int stage, Vec x2, Vec ec, Vec b, Vec xout, int B) {
  const LevelOp<C> op = make_op<C>(h_, 0, a_[stage]);
  const C omega = (C)h_->omega;
  const C es = (C)(1.0 / h_->mg_scale);
  const March3Geo g = march3_geo(h_->lev_n[0], B, 2);
  const dim3 grid((unsigned)(g.ntx * g.ntx * g.nz), (unsigned)B);
  const int nc = h_->lev_n[1];
  MG_TRY(typed1(1, [&](auto tc) {
    using TC = decltype(tc);
    hipLaunchKernelGGL((k_up3d_march<TI, TC, C>), grid, dim3(M3_T * M3_T), 0, st_, (const TI*)x2.ptr, x2.stride,
                       (const TC*)ec.ptr, ec.stride, (const TI*)b.ptr, b.stride, (TI*)xout.ptr, xout.stride, g, nc,
                       op, omega, es);
    return hipGetLastError();
  }));
  return mark("k_up3d_march", 0);
}

// One V-cycle on level l.  `pre` = the first (pointwise) sweep from zero was
// already written into x by the restriction of the level above.
template <class TI, class TM>
hipError_t Multigrid<TI, TM>::mark(const char* kernel, int l) {
  if (!marks_) return hipSuccess;
  const std::string label = std::string(kernel) + "@" + std::to_string(l);
  if (marks_->ev.empty()) {   // labels only (a captured cycle)
    marks_->label.push_back(label);
    return hipSuccess;
  }
  if (marks_->next >= marks_->ev.size()) return hipSuccess;
  marks_->label[marks_->next] = label;
  return hipEventRecord(marks_->ev[marks_->next++], st_);
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::vcycle(int l, int stage, Vec x, Vec b, bool zero_init, bool pre, int B, Vec* result,
                                     const Coupling* cpl) {
  auto& P = h_->plan;
  if (l >= l0_) {
    MG_TRY(tail(stage, x, b, zero_init, B));
    MG_TRY(mark(fast_nls_ > 0 && zero_init ? "k_tail_fast" : "k_tail", l));
    *result = x;
    return hipSuccess;
  }
  if (l == levels_ - 1) {      // no tail (3D): exact solve on the coarsest level
    const int Nc = (int)h_->lev_N[l];
    const dim3 g((unsigned)B), blk(Nc * 4 <= 1024 ? (unsigned)((Nc * 4 + 63) / 64 * 64) : 1024u);
    if (l == 0)
      hipLaunchKernelGGL((k_coarse_solve<TI, C>), g, blk, 0, st_, (const TI*)b.ptr, b.stride, (TI*)x.ptr, x.stride,
                         coarse_inv(stage), Nc);
    else
      MG_TRY(typed1(l, [&](auto t) {
        using TS = decltype(t);
        hipLaunchKernelGGL((k_coarse_solve<TS, C>), g, blk, 0, st_, (const TS*)b.ptr, b.stride, (TS*)x.ptr, x.stride,
                           coarse_inv(stage), Nc);
        return hipGetLastError();
      }));
    MG_TRY(hipGetLastError());
    MG_TRY(mark("k_coarse_solve", l));
    *result = x;
    return hipSuccess;
  }
  const int nu1 = h_->opts.nu1, nu2 = h_->opts.nu2;
  const int64_t Nl = h_->lev_N[l];
  Vec tmp{h_->ws + P.mgT[l], Nl};
  if (h_->dim == 2 && nu1 <= 3 && nu2 <= 3 && !pre && !(l == 0 && h_->fe_order == 2)) {
    // tiled: down (sweeps, residual, restriction) -> coarse cycle -> up
    const int64_t Nc = h_->lev_N[l + 1];
    Vec bc{h_->ws + P.mgB[l + 1], Nc};
    Vec xc{h_->ws + P.mgX[l + 1], Nc};
    MG_TRY(down2d(l, stage, b, zero_init ? nullptr : x.ptr, x.stride, tmp, bc, B, cpl));
    MG_TRY(mark("k_down2d", l));
    if (cpl && cpl->nz > 0) b = Vec{cpl->out, cpl->so};   // the formed right-hand side
    Vec ec{};
    MG_TRY(vcycle(l + 1, stage, xc, bc, true, false, B, &ec));
    MG_TRY(up2d(l, stage, tmp, ec, b, x, B));
    MG_TRY(mark("k_up2d", l));
    *result = x;
    return hipSuccess;
  }
  if (march3d_ok(l, zero_init, pre, B)) {
    // z-marches: sweeps, residual and full weighting -> coarse cycle ->
    // prolongation and sweeps
    const int64_t Nc = h_->lev_N[1];
    Vec bc{h_->ws + P.mgB[1], Nc};
    Vec xc{h_->ws + P.mgX[1], Nc};
    const bool next_grid = 1 < l0_;
    MG_TRY(march3d_down(stage, b, tmp, bc, xc, next_grid, B));
    Vec ec{};
    MG_TRY(vcycle(1, stage, xc, bc, true, next_grid, B, &ec));
    MG_TRY(march3d_up(stage, tmp, ec, b, x, B));
    *result = x;
    return hipSuccess;
  }
  auto partner = [&](const Vec& v) { return v.ptr == x.ptr ? tmp : x; };
  // writes after the first sweep alternate buffers; at level 0 the result
  // must end in x, so the first sweep's target is chosen by parity
  const bool fused_post = (l == 0) && h_->dim == 2 && h_->fe_order != 2;
  Vec cur = x;
  int rem = nu1;
  if (zero_init) {
    if (!pre) {
      const int alternations = (nu1 - 1) + nu2;
      Vec first = (l == 0 && (alternations % 2 == 1)) ? tmp : x;
      MG_TRY(smooth(l, stage, first, first, b, true, B));
      MG_TRY(mark("k_smooth", l));
      cur = first;
    }
    --rem;
  }
  for (; rem > 0; --rem) {
    Vec nxt = partner(cur);
    MG_TRY(smooth(l, stage, cur, nxt, b, false, B));
    MG_TRY(mark("k_smooth", l));
    cur = nxt;
  }
  const int64_t Nc = h_->lev_N[l + 1];
  Vec bc{h_->ws + P.mgB[l + 1], Nc};
  Vec xc{h_->ws + P.mgX[l + 1], Nc};
  // the coarse level's first sweep fused into the restriction, unless that
  // level runs the tiled kernels (2D, nu1, nu2 <= 3: reached here only from
  // level 0 of Q2 elements), which start from zero themselves
  const bool next_tiled = h_->dim == 2 && nu1 <= 3 && nu2 <= 3;
  const bool next_grid = (l + 1) < l0_ && !next_tiled;
  MG_TRY(resid_restrict(l, stage, cur, b, bc, xc, next_grid, B));
  MG_TRY(mark(split_restrict(l) ? "k_restrict" : "k_resid_restrict", l));
  Vec ec{};
  MG_TRY(vcycle(l + 1, stage, xc, bc, true, next_grid, B, &ec));
  int post = nu2;
  if (fused_post) {
    Vec nxt = partner(cur);
    MG_TRY(prolong_smooth0(stage, cur, ec, b, nxt, B));
    MG_TRY(mark("k_prolong_smooth", l));
    cur = nxt;
    --post;
  } else {
    // pointwise prolongation: pick its target so the sweeps end in x
    Vec tgt = (post % 2 == 0) ? x : tmp;
    MG_TRY(prolong(l, cur, ec, tgt, B));
    MG_TRY(mark("k_prolong", l));
    cur = tgt;
  }
  for (; post > 0; --post) {
    Vec nxt = partner(cur);
    MG_TRY(smooth(l, stage, cur, nxt, b, false, B));
    MG_TRY(mark("k_smooth", l));
    cur = nxt;
  }
  if (l == 0 && cur.ptr != x.ptr) {   // odd sweep counts from a nonzero start: copy back
    MG_TRY(basis_update<TI, TI, TI>((const TI*)cur.ptr, cur.stride, (const TI*)cur.ptr, 0, 0, 0, (TI*)x.ptr,
                                    x.stride, nullptr, 0, 0, -1, 1.0, Nl, B, st_));
    MG_TRY(mark("k_basis", l));
    cur = x;
  }
  *result = cur;
  return hipSuccess;
}

template <class TI, class TM>
hipError_t Multigrid<TI, TM>::solve(int stage, BVec<TI> x, BVec<const TI> rhs, int B, int cycles,
                                    const Coupling* cpl) {
  Vec xv{x.ptr, x.stride};
  Vec bv{const_cast<TI*>(rhs.ptr), rhs.stride};
  const bool fused = cpl && cpl->nz > 0 && h_->dim == 2 && h_->opts.nu1 <= 3 && h_->opts.nu2 <= 3 && l0_ > 0 &&
                     !h_->fe;
  if (cpl && cpl->nz > 0 && !fused) {
    // the level-0 kernel that would form the coupling does not run: form it first
    MG_TRY(rana_rhs<TI>(h_, cpl->Lc, cpl->nz, rhs.ptr, rhs.stride, cpl->z, cpl->sz, cpl->out, cpl->so, B, st_));
    bv = Vec{cpl->out, cpl->so};
  }
  for (int c = 0; c < cycles; ++c) {
    Vec res{};
    MG_TRY(vcycle(0, stage, xv, bv, c == 0, false, B, &res, (fused && c == 0) ? cpl : nullptr));
    if (res.ptr != xv.ptr) return hipErrorUnknown;   // the driver always ends in x
    if (fused && c == 0) bv = Vec{cpl->out, cpl->so};
  }
  return hipSuccess;
}

// Largest dynamic LDS allocation the tail may use on the current device
// (opt-in above 64 KiB where the device allows it), capped at 128 KiB.
size_t mg_configure_lds() {
  int dev = 0, optin = 0, base = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&base, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) base = 65536;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = base;
  size_t want = (size_t)(optin > base ? optin : base);
  if (want > 131072) want = 131072;
  if (want <= 65536) return want < 65536 ? want : 65536;
  const void* kernels[] = {
      (const void*)k_tail<false, double, double, double>, (const void*)k_tail<true, double, double, double>,
      (const void*)k_tail<false, float, float, float>, (const void*)k_tail<true, float, float, float>,
      (const void*)k_tail<false, __half, __half, float>, (const void*)k_tail<true, __half, __half, float>,
      (const void*)k_tail<false, __hip_bfloat16, __hip_bfloat16, float>};
  for (const void* k : kernels)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) != hipSuccess) {
      (void)hipGetLastError();
      return 65536;
    }
#define TF_PTR1(T, C)                                                                                     \
  (const void*)k_tail_fast<KIND_STENCIL9, 1, 1, false, T, C>, (const void*)k_tail_fast<KIND_TENSOR, 1, 1, true, T, C>, \
      (const void*)k_tail_fast<KIND_TENSOR, 1, 1, false, T, C>
#define TF_PTR2(T, C)                                                                                     \
  (const void*)k_tail_fast<KIND_STENCIL9, 2, 4, false, T, C>, (const void*)k_tail_fast<KIND_TENSOR, 2, 4, true, T, C>, \
      (const void*)k_tail_fast<KIND_TENSOR, 2, 4, false, T, C>
  const void* fast[] = {TF_PTR1(double, double), TF_PTR1(float, float), TF_PTR1(__half, float),
                        TF_PTR1(__hip_bfloat16, float), TF_PTR2(float, float), TF_PTR2(__half, float),
                        TF_PTR2(__hip_bfloat16, float)};
#undef TF_PTR1
#undef TF_PTR2
  for (const void* k : fast)
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)want) != hipSuccess) {
      (void)hipGetLastError();
      return 65536;
    }
  return want;
}

template class Multigrid<double, double>;
template class Multigrid<float, float>;
template class Multigrid<float, __half>;
template class Multigrid<float, __hip_bfloat16>;
template class Multigrid<__half, __half>;

}  // namespace aao

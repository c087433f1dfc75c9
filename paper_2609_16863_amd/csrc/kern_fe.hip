// Bilinear (Q1) and biquadratic (Q2) finite elements on a uniform square
// mesh: the operators of the all-at-once system with a mass matrix (Sec. 2,
// eq. (2.4): Phi with M blocks, Psi1 = -(tau b^T (x) M), Theta_hat =
// I_s (x) M + tau A (x) K) and the pieces of P-tilde that meet M or K
// outside the multigrid: the stage operator, Rana's coupling, the Psi1
// coupling of S-tilde, the right-hand sides e (x) K z of its steps, and its
// block-diagonal mass solve by Chebyshev semi-iteration (Sec. 5: 20 steps
// with the Jacobi splitting).
//
// On the interior nodes of a uniform mesh (Dirichlet boundary eliminated)
// both element families give tensor products of 1D matrices:
//   M = M1 (x) M1,  K = T1 (x) M1 + M1 (x) T1,
// with, at node spacing h,
//   Q1: M1 = h (1/6, 2/3, 1/6),  T1 = (-1, 2, -1) / h        (every row);
//   Q2 (element side H = 2h): rows at element vertices (odd 0-based index)
//       M1 = H/30 (-1, 2, 8, 2, -1),  T1 = (1, -8, 14, -8, 1) / (3H),
//       rows at edge midpoints (even index)
//       M1 = H/30 (2, 16, 2),          T1 = (-8, 16, -8) / (3H).
// A node's rows follow from the parity of its index along each axis, so a
// kernel forms (M u)_p and (K u)_p from the (2R+1)^2 neighbourhood (R = 1
// for Q1, 2 for Q2) one mesh row at a time: with r_M = sum_di M1_x u and
// r_T = sum_di T1_x u on row dj, M u = sum_dj M1_y r_M and
// K u = sum_dj (M1_y r_T + T1_y r_M).  One thread per node and block (these
// kernels serve the finite-element path, not the benchmark's
// finite-difference one).
//
// Every kernel stages its fields in LDS tiles of 16 x 16 nodes with a halo of
// R (combining several fields into one tile where the operator is linear in
// them), then forms M and K at each node from the tile.
#include <type_traits>

#include "aao_internal.h"
#include "fe.h"
#include "krylov.h"
#include "stencil.h"

namespace aao {
namespace {

constexpr int TPB = 256;

// 1D element-matrix rows by index parity: m[p][d + 2] = M1(i, i + d),
// t[p][d + 2] = T1(i, i + d) for i with i % 2 == p, d = -2..2.
struct FeRows {
  double m[2][5];
  double t[2][5];
  double dinv[2][2];   // 1 / M_pp for a node of parities (px, py): [py][px]
};

FeRows fe_rows(const aao_problem* h) {
  FeRows r{};
  if (h->fe_order == 2) {
    const double H = 2.0 * h->h;
    static const double mv[5] = {-1, 2, 8, 2, -1}, tv[5] = {1, -8, 14, -8, 1};
    static const double mm[5] = {0, 2, 16, 2, 0}, tm[5] = {0, -8, 16, -8, 0};
    for (int d = 0; d < 5; ++d) {
      r.m[0][d] = H / 30.0 * mm[d];
      r.t[0][d] = tm[d] / (3.0 * H);
      r.m[1][d] = H / 30.0 * mv[d];
      r.t[1][d] = tv[d] / (3.0 * H);
    }
  } else {
    const double hh = h->h;
    const double m1[5] = {0, hh / 6.0, 2.0 * hh / 3.0, hh / 6.0, 0}, t1[5] = {0, -1.0 / hh, 2.0 / hh, -1.0 / hh, 0};
    for (int p = 0; p < 2; ++p)
      for (int d = 0; d < 5; ++d) {
        r.m[p][d] = m1[d];
        r.t[p][d] = t1[d];
      }
  }
  for (int py = 0; py < 2; ++py)
    for (int px = 0; px < 2; ++px) r.dinv[py][px] = 1.0 / (r.m[px][2] * r.m[py][2]);
  return r;
}

// The 1D rows of node (i, j) in the arithmetic type C.
template <int R, class C>
struct NodeRows {
  C mx[2 * R + 1], tx[2 * R + 1], my[2 * R + 1], ty[2 * R + 1];
  __device__ __forceinline__ NodeRows(const FeRows& rows, int i, int j) {
#pragma unroll
    for (int d = -R; d <= R; ++d) {
      mx[d + R] = (C)rows.m[i & 1][d + 2];
      tx[d + R] = (C)rows.t[i & 1][d + 2];
      my[d + R] = (C)rows.m[j & 1][d + 2];
      ty[d + R] = (C)rows.t[j & 1][d + 2];
    }
  }
};

// Tiles of TS x TS owned nodes (one per thread of a 256-thread workgroup),
// staged in LDS with a halo of R nodes: tile (tx, ty) of the mesh owns
// nodes [16 tx, 16 tx + 16) x [16 ty, 16 ty + 16).  Values outside the mesh
// are staged as zero, so the tensor products need no bounds checks.
constexpr int TS = 16;

template <int R>
struct FeTile {
  static constexpr int W = TS + 2 * R, NE = W * W;
};

struct TileIdx {
  int i, j;     // the thread's node
  int lx, ly;   // its position in the tile
  int ox, oy;   // mesh coordinates of the staged tile's first entry
  bool own;     // the node lies in the mesh
};

// Tile of workgroup blockIdx.x (XCD-aware order: neighbouring tiles share
// halo lines in one L2).
template <int R>
__device__ __forceinline__ TileIdx tile_idx(int n) {
  const int tiles = (n + TS - 1) / TS;
  const int L = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  TileIdx t;
  t.lx = (int)threadIdx.x % TS;
  t.ly = (int)threadIdx.x / TS;
  const int x0 = (L % tiles) * TS, y0 = (L / tiles) * TS;
  t.i = x0 + t.lx;
  t.j = y0 + t.ly;
  t.ox = x0 - R;
  t.oy = y0 - R;
  t.own = t.i < n && t.j < n;
  return t;
}

// s[0, NE) = val(g) at the staged nodes (g = jj n + ii), zero off the mesh.
// Every thread of the workgroup takes part; the caller synchronizes.
template <int R, class C, class F>
__device__ __forceinline__ void stage_tile(C* s, const TileIdx& t, int n, F&& val) {
  constexpr int W = FeTile<R>::W, NE = FeTile<R>::NE;
  for (int e = threadIdx.x; e < NE; e += TPB) {
    const int ii = t.ox + e % W, jj = t.oy + e / W;
    s[e] = (ii >= 0 && ii < n && jj >= 0 && jj < n) ? val((int64_t)jj * n + ii) : C(0);
  }
}

// (M f) and (K f) at the thread's node from the staged tile of f.
template <int R, class C>
__device__ __forceinline__ void tile_ms(const C* s, const TileIdx& t, const NodeRows<R, C>& q, C& Mf, C& Kf) {
  constexpr int W = FeTile<R>::W;
  Mf = C(0);
  Kf = C(0);
  const C* c = s + (t.ly + R) * W + t.lx + R;
#pragma unroll
  for (int dj = -R; dj <= R; ++dj) {
    C rm = C(0), rt = C(0);
#pragma unroll
    for (int di = -R; di <= R; ++di) {
      const C v = c[dj * W + di];
      rm += q.mx[di + R] * v;
      rt += q.tx[di + R] * v;
    }
    Mf += q.my[dj + R] * rm;
    Kf += q.my[dj + R] * rt + q.ty[dj + R] * rm;
  }
}

template <int R, class C>
__device__ __forceinline__ C tile_m(const C* s, const TileIdx& t, const NodeRows<R, C>& q) {
  constexpr int W = FeTile<R>::W;
  C Mf = C(0);
  const C* c = s + (t.ly + R) * W + t.lx + R;
#pragma unroll
  for (int dj = -R; dj <= R; ++dj) {
    C rm = C(0);
#pragma unroll
    for (int di = -R; di <= R; ++di) rm += q.mx[di + R] * c[dj * W + di];
    Mf += q.my[dj + R] * rm;
  }
  return Mf;
}

template <int R, class C>
__device__ __forceinline__ C tile_k(const C* s, const TileIdx& t, const NodeRows<R, C>& q) {
  C Mf, Kf;
  tile_ms<R, C>(s, t, q, Mf, Kf);
  return Kf;
}

// y = A x, one block row per blockIdx.y: rows 0..nt are v-rows, then the
// stage rows (m, i) in the layout of eq. (2.4).  M and K are linear, so the
// fields of a row are combined while they are staged:
//   v-row m > 0:  M u,  u = v_m - v_{m-1} - tau sum_q b_q V_{m-1,q};  row 0: M v_0;
//   stage row (m, st):  M V_{m,st} + K w,  w = v_m + tau sum_q a_{st,q} V_{m,q}.
template <int S, int R, class TX>
__global__ __launch_bounds__(TPB) void k_fe_apply_A(const TX* __restrict__ x, double* __restrict__ y, int n,
                                                    int nt, FeRows rows, Tab tab) {
  __shared__ double sa[FeTile<R>::NE], sb[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t NN = (int64_t)n * n;
  const int row = blockIdx.y;
  const TX* V = x + (int64_t)(nt + 1) * NN;
  if (row <= nt) {
    const TX* v0 = x + (int64_t)row * NN;
    const TX* v1 = x + (int64_t)(row - 1) * NN;
    const TX* Vp = V + (int64_t)(row - 1) * S * NN;
    stage_tile<R, double>(sa, t, n, [&](int64_t g) {
      double u = (double)v0[g];
      if (row > 0) {
        u -= (double)v1[g];
        for (int q = 0; q < S; ++q) u -= tab.tau * tab.b[q] * (double)Vp[q * NN + g];
      }
      return u;
    });
    __syncthreads();
    if (!t.own) return;
    const NodeRows<R, double> q(rows, t.i, t.j);
    y[(int64_t)row * NN + (int64_t)t.j * n + t.i] = tile_m<R, double>(sa, t, q);
    return;
  }
  const int r = row - (nt + 1), m = r / S, st = r - m * S;
  const TX* vm = x + (int64_t)m * NN;
  const TX* Vm = V + (int64_t)m * S * NN;
  stage_tile<R, double>(sa, t, n, [&](int64_t g) { return (double)Vm[st * NN + g]; });
  stage_tile<R, double>(sb, t, n, [&](int64_t g) {
    double w = (double)vm[g];
    for (int q = 0; q < S; ++q) w += tab.tau * tab.A[st * S + q] * (double)Vm[q * NN + g];
    return w;
  });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, double> q(rows, t.i, t.j);
  y[(int64_t)(nt + 1) * NN + (int64_t)r * NN + (int64_t)t.j * n + t.i] =
      tile_m<R, double>(sa, t, q) + tile_k<R, double>(sb, t, q);
}

// y = A^T x (M and K symmetric):
//   y_{v,m} = M (x_{v,m} - x_{v,m+1}) + K sum_i x_{V,m,i}  (m < nt),  y_{v,nt} = M x_{v,nt};
//   y_{V,m,st} = M (x_{V,m,st} - tau b_st x_{v,m+1}) + K tau sum_i a_{i,st} x_{V,m,i}.
template <int S, int R, class TX>
__global__ __launch_bounds__(TPB) void k_fe_apply_AT(const TX* __restrict__ x, double* __restrict__ y, int n,
                                                     int nt, FeRows rows, Tab tab) {
  __shared__ double sa[FeTile<R>::NE], sb[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t NN = (int64_t)n * n;
  const int row = blockIdx.y;
  const TX* V = x + (int64_t)(nt + 1) * NN;
  if (row <= nt) {
    const TX* v0 = x + (int64_t)row * NN;
    const TX* v1 = x + (int64_t)(row + 1) * NN;
    const TX* Vr = V + (int64_t)row * S * NN;
    const bool last = row == nt;
    stage_tile<R, double>(sa, t, n, [&](int64_t g) { return last ? (double)v0[g] : (double)v0[g] - (double)v1[g]; });
    stage_tile<R, double>(sb, t, n, [&](int64_t g) {
      double w = 0.0;
      if (!last)
        for (int q = 0; q < S; ++q) w += (double)Vr[q * NN + g];
      return w;
    });
    __syncthreads();
    if (!t.own) return;
    const NodeRows<R, double> q(rows, t.i, t.j);
    y[(int64_t)row * NN + (int64_t)t.j * n + t.i] = tile_m<R, double>(sa, t, q) + tile_k<R, double>(sb, t, q);
    return;
  }
  const int r = row - (nt + 1), m = r / S, st = r - m * S;
  const TX* vn = x + (int64_t)(m + 1) * NN;
  const TX* Vm = V + (int64_t)m * S * NN;
  stage_tile<R, double>(sa, t, n, [&](int64_t g) { return (double)Vm[st * NN + g] - tab.tau * tab.b[st] * (double)vn[g]; });
  stage_tile<R, double>(sb, t, n, [&](int64_t g) {
    double w = 0.0;
    for (int q = 0; q < S; ++q) w += tab.tau * tab.A[q * S + st] * (double)Vm[q * NN + g];
    return w;
  });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, double> q(rows, t.i, t.j);
  y[(int64_t)(nt + 1) * NN + (int64_t)r * NN + (int64_t)t.j * n + t.i] =
      tile_m<R, double>(sa, t, q) + tile_k<R, double>(sb, t, q);
}

// w_r = M z_r + tau sum_q A[r][q] K z_q   (Theta_hat), B instances
template <int S, int R, class T>
__global__ __launch_bounds__(TPB) void k_fe_theta(const T* __restrict__ z, int64_t sz, T* __restrict__ w,
                                                  int64_t sw, int n, FeRows rows, Tab tab) {
  using C = typename Acc<T>::type;
  __shared__ C sz_[S][FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const int64_t inst = blockIdx.y;
  const T* zi = z + inst * sz;
#pragma unroll
  for (int q = 0; q < S; ++q) stage_tile<R, C>(sz_[q], t, n, [&](int64_t g) { return ld<T, C>(zi + q * N + g); });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, C> nq(rows, t.i, t.j);
  C Mz[S], Kz[S];
#pragma unroll
  for (int q = 0; q < S; ++q) tile_ms<R, C>(sz_[q], t, nq, Mz[q], Kz[q]);
  const int64_t p = (int64_t)t.j * n + t.i;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    C mix = C(0);
#pragma unroll
    for (int q = 0; q < S; ++q) mix += (C)tab.A[r * S + q] * Kz[q];
    st<T, C>(w + inst * sw + (int64_t)r * N + p, Mz[r] + (C)tab.tau * mix);
  }
}

// out = v - K (tau sum_{l < stage} Lc[stage][l] z_l)   (Rana's coupling)
template <int R, class T>
__global__ __launch_bounds__(TPB) void k_fe_rana_rhs(const T* __restrict__ v, int64_t sv, const T* __restrict__ z,
                                                     int64_t sz, T* __restrict__ out, int64_t so, int n, int stage,
                                                     int ns, FeRows rows, Tab tab) {
  using C = typename Acc<T>::type;
  __shared__ C su[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const int64_t inst = blockIdx.y;
  const T* zi = z + inst * sz;
  stage_tile<R, C>(su, t, n, [&](int64_t g) {
    C u = C(0);
    for (int l = 0; l < stage; ++l) u += (C)(tab.tau * tab.L[stage * ns + l]) * ld<T, C>(zi + l * N + g);
    return u;
  });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, C> q(rows, t.i, t.j);
  const int64_t p = (int64_t)t.j * n + t.i;
  st<T, C>(out + inst * so + p, ld<T, C>(v + inst * sv + p) - tile_k<R, C>(su, t, q));
}

// t_0 = r_0;  t_{m+1} = r_{m+1} + tau M sum_i b_i z_{V,m,i}   (r_v - Psi1 z_V)
template <int R, class T>
__global__ __launch_bounds__(TPB) void k_fe_schur_coupling(const double* __restrict__ r, const T* __restrict__ zV,
                                                           T* __restrict__ t_out, int n, int ns, FeRows rows,
                                                           Tab tab) {
  using C = typename Acc<T>::type;
  __shared__ double su[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t NN = (int64_t)n * n;
  const int step = blockIdx.y;
  if (step > 0) {
    const T* zp = zV + (int64_t)(step - 1) * ns * NN;
    stage_tile<R, double>(su, t, n, [&](int64_t g) {
      double u = 0.0;
      for (int q = 0; q < ns; ++q) u += tab.b[q] * (double)ld<T, C>(zp + q * NN + g);
      return u;
    });
    __syncthreads();
  }
  if (!t.own) return;
  const int64_t p = (int64_t)t.j * n + t.i;
  double acc = r[(int64_t)step * NN + p];
  if (step > 0) {
    const NodeRows<R, double> q(rows, t.i, t.j);
    acc += tab.tau * tile_m<R, double>(su, t, q);
  }
  st<T, C>(t_out + (int64_t)step * NN + p, (C)acc);
}

// out_{b,i} = K zin_b for every stage i
template <int R, class T>
__global__ __launch_bounds__(TPB) void k_fe_schur_kz(const T* __restrict__ zin, int64_t szin, T* __restrict__ out,
                                                     int64_t sout, int n, int ns, FeRows rows) {
  using C = typename Acc<T>::type;
  __shared__ C su[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const int64_t b = blockIdx.y;
  stage_tile<R, C>(su, t, n, [&](int64_t g) { return ld<T, C>(zin + b * szin + g); });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, C> q(rows, t.i, t.j);
  const C kz = tile_k<R, C>(su, t, q);
  const int64_t p = (int64_t)t.j * n + t.i;
  for (int qq = 0; qq < ns; ++qq) st<T, C>(out + b * sout + (int64_t)qq * N + p, kz);
}

// One step of the Chebyshev semi-iteration for M y = t on B blocks:
// out = w (y - yprev + D^{-1} (t - M y) / theta) + yprev, or, on the first
// step, out = D^{-1} t / theta; yprev may be null (a zero y_{k-1}).  out may
// alias t or yprev (each element reads only its own entry of those); it
// never aliases y, whose neighbours other workgroups read.
template <int R, class T>
__global__ __launch_bounds__(TPB) void k_fe_cheb(const T* t_in, const T* __restrict__ y, const T* yprev, T* out,
                                                 int n, FeRows rows, typename Acc<T>::type ith,
                                                 typename Acc<T>::type w, int first) {
  using C = typename Acc<T>::type;
  __shared__ C sy[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const T* yb = y + (int64_t)blockIdx.y * N;
  if (!first) {
    stage_tile<R, C>(sy, t, n, [&](int64_t g) { return ld<T, C>(yb + g); });
    __syncthreads();
  }
  if (!t.own) return;
  const int64_t off = (int64_t)blockIdx.y * N + (int64_t)t.j * n + t.i;
  const C tv = ld<T, C>(t_in + off);
  const C dth = (C)rows.dinv[t.j & 1][t.i & 1] * ith;
  if (first) {
    st<T, C>(out + off, dth * tv);
    return;
  }
  const NodeRows<R, C> q(rows, t.i, t.j);
  constexpr int W = FeTile<R>::W;
  const C yc = sy[(t.ly + R) * W + t.lx + R];
  const C yp = yprev ? ld<T, C>(yprev + off) : C(0);
  st<T, C>(out + off, w * (yc - yp + dth * (tv - tile_m<R, C>(sy, t, q))) + yp);
}

// out_b = M in_b, B blocks (FP64)
template <int R>
__global__ __launch_bounds__(TPB) void k_fe_mass(const double* __restrict__ in, double* __restrict__ out, int n,
                                                 FeRows rows) {
  __shared__ double su[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const double* ib = in + (int64_t)blockIdx.y * N;
  stage_tile<R, double>(su, t, n, [&](int64_t g) { return ib[g]; });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, double> q(rows, t.i, t.j);
  out[(int64_t)blockIdx.y * N + (int64_t)t.j * n + t.i] = tile_m<R, double>(su, t, q);
}

// Level 0 of the multigrid for Q2 elements: the operator M + a K of the
// shifted block, its diagonal D = M1_ii M1_jj + a (T1_ii M1_jj + M1_ii T1_jj).
// Weighted Jacobi sweep xout = xin + omega D^{-1} (b - A xin), or from zero
// xout = omega D^{-1} b (pointwise); xout never aliases xin.
template <class T>
__global__ __launch_bounds__(TPB) void k_q2_smooth(const T* __restrict__ xin, int64_t sxin, T* __restrict__ xout,
                                                   int64_t sxout, const T* __restrict__ b, int64_t sb, int n,
                                                   FeRows rows, typename Acc<T>::type a,
                                                   typename Acc<T>::type omega, int zero_init) {
  using C = typename Acc<T>::type;
  constexpr int R = 2;
  __shared__ C sx[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t N = (int64_t)n * n;
  const int64_t inst = blockIdx.y;
  if (!zero_init) {
    const T* xi = xin + inst * sxin;
    stage_tile<R, C>(sx, t, n, [&](int64_t g) { return ld<T, C>(xi + g); });
    __syncthreads();
  }
  if (!t.own) return;
  const NodeRows<R, C> q(rows, t.i, t.j);
  const C d = q.mx[R] * q.my[R] + a * (q.tx[R] * q.my[R] + q.mx[R] * q.ty[R]);
  const int64_t p = (int64_t)t.j * n + t.i;
  const C bp = ld<T, C>(b + inst * sb + p);
  C out;
  if (zero_init) {
    out = omega * bp / d;
  } else {
    C Mx, Kx;
    tile_ms<R, C>(sx, t, q, Mx, Kx);
    constexpr int W = FeTile<R>::W;
    out = sx[(t.ly + R) * W + t.lx + R] + omega * (bp - (Mx + a * Kx)) / d;
  }
  st<T, C>(xout + inst * sxout + p, out);
}

// r = b - (M + a K) x at level 0 of Q2 elements
template <class T>
__global__ __launch_bounds__(TPB) void k_q2_residual(const T* __restrict__ x, int64_t sx, const T* __restrict__ b,
                                                     int64_t sb, T* __restrict__ r, int64_t sr, int n, FeRows rows,
                                                     typename Acc<T>::type a) {
  using C = typename Acc<T>::type;
  constexpr int R = 2;
  __shared__ C su[FeTile<R>::NE];
  const TileIdx t = tile_idx<R>(n);
  const int64_t inst = blockIdx.y;
  const T* xi = x + inst * sx;
  stage_tile<R, C>(su, t, n, [&](int64_t g) { return ld<T, C>(xi + g); });
  __syncthreads();
  if (!t.own) return;
  const NodeRows<R, C> q(rows, t.i, t.j);
  C Mx, Kx;
  tile_ms<R, C>(su, t, q, Mx, Kx);
  const int64_t p = (int64_t)t.j * n + t.i;
  st<T, C>(r + inst * sr + p, ld<T, C>(b + inst * sb + p) - (Mx + a * Kx));
}

// One workgroup per TS x TS tile of the mesh, blockIdx.y the instance.
inline dim3 fe_grid(const aao_problem* h, int64_t B) {
  const int64_t tiles = (h->n + TS - 1) / TS;
  return dim3((unsigned)(tiles * tiles), (unsigned)B);
}

// Calls f(std::integral_constant<int, R>) with the neighbourhood radius of the
// handle's elements (1: Q1, 2: Q2).
template <class F>
hipError_t by_radius(const aao_problem* h, F&& f) {
  if (h->fe_order == 2) f(std::integral_constant<int, 2>{});
  else f(std::integral_constant<int, 1>{});
  return hipGetLastError();
}

// Calls f(std::integral_constant<int, S>{}, std::integral_constant<int, R>{}).
template <class F>
hipError_t by_stages_radius(const aao_problem* h, F&& f) {
  return by_radius(h, [&](auto r) {
    if (h->s == 1) f(std::integral_constant<int, 1>{}, r);
    else if (h->s == 2) f(std::integral_constant<int, 2>{}, r);
    else f(std::integral_constant<int, 3>{}, r);
  });
}

}  // namespace

template <class TX>
hipError_t fe_apply_A(const aao_problem* h, const TX* x, double* y, bool transpose, hipStream_t st) {
  const dim3 g = fe_grid(h, (int64_t)(h->nt + 1) + (int64_t)h->nt * h->s);
  const FeRows rows = fe_rows(h);
  return by_stages_radius(h, [&](auto s_, auto r_) {
    constexpr int S = decltype(s_)::value, R = decltype(r_)::value;
    if (transpose)
      hipLaunchKernelGGL((k_fe_apply_AT<S, R, TX>), g, dim3(TPB), 0, st, x, y, h->n, h->nt, rows, h->tab);
    else
      hipLaunchKernelGGL((k_fe_apply_A<S, R, TX>), g, dim3(TPB), 0, st, x, y, h->n, h->nt, rows, h->tab);
  });
}

template <class T>
hipError_t fe_theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                          hipStream_t st) {
  const dim3 g = fe_grid(h, B);
  const FeRows rows = fe_rows(h);
  return by_stages_radius(h, [&](auto s_, auto r_) {
    constexpr int S = decltype(s_)::value, R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_theta<S, R, T>), g, dim3(TPB), 0, st, z, sz, w, sw, h->n, rows, tab);
  });
}

template <class T>
hipError_t fe_rana_rhs(const aao_problem* h, const Tab& tab, int i, const T* v, int64_t sv, const T* z, int64_t sz,
                       T* out, int64_t so, int B, hipStream_t st) {
  const FeRows rows = fe_rows(h);
  return by_radius(h, [&](auto r_) {
    constexpr int R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_rana_rhs<R, T>), fe_grid(h, B), dim3(TPB), 0, st, v, sv, z, sz, out, so, h->n, i,
                       h->s, rows, tab);
  });
}

template <class T>
hipError_t fe_schur_coupling(const aao_problem* h, const double* r, const T* zV, T* t, hipStream_t st) {
  const FeRows rows = fe_rows(h);
  return by_radius(h, [&](auto r_) {
    constexpr int R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_schur_coupling<R, T>), fe_grid(h, h->nt + 1), dim3(TPB), 0, st, r, zV, t, h->n,
                       h->s, rows, h->tab);
  });
}

template <class T>
hipError_t fe_schur_kz(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B,
                       hipStream_t st) {
  const FeRows rows = fe_rows(h);
  return by_radius(h, [&](auto r_) {
    constexpr int R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_schur_kz<R, T>), fe_grid(h, B), dim3(TPB), 0, st, zin, szin, out, sout, h->n, h->s,
                       rows);
  });
}

// t <- (CHEB_STEPS steps of Chebyshev semi-iteration with the Jacobi
// splitting) M^{-1} t on B consecutive blocks of N values, in place; ya, yb:
// two scratch vectors of B N values.  The spectrum of D^{-1} M lies in
// [1/4, 9/4] for Q1 squares and in [1/4, 25/16] for Q2 squares (the extreme
// eigenvalues of one element's D_e^{-1} M_e); theta is the interval's
// centre, rho = (beta - alpha) / (beta + alpha) the radius of the Jacobi
// iteration matrix I - D^{-1} M / theta.
template <class T>
hipError_t fe_mass_solve(const aao_problem* h, T* t, T* ya, T* yb, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  const double alpha = 0.25, beta = h->fe_order == 2 ? 1.5625 : 2.25;
  const double theta = 0.5 * (alpha + beta), rho = (beta - alpha) / (beta + alpha);
  const FeRows rows = fe_rows(h);
  const C ith = (C)(1.0 / theta);
  const dim3 g = fe_grid(h, B);
  const int n = h->n;
  auto step = [&](const T* tt, const T* y, const T* yp, T* out, C w, int first) {
    return by_radius(h, [&](auto r_) {
      constexpr int R = decltype(r_)::value;
      hipLaunchKernelGGL((k_fe_cheb<R, T>), g, dim3(TPB), 0, st, tt, y, yp, out, n, rows, ith, w, first);
    });
  };
  // y_1 -> ya; then y_{k+1} overwrites y_{k-1}; the last step writes into t
  hipError_t e = step((const T*)t, nullptr, nullptr, ya, C(1), 1);
  if (e != hipSuccess) return e;
  T* cur = ya;
  T* prev = yb;
  double w = 1.0;
  for (int k = 1; k < FE_CHEB_STEPS; ++k) {
    w = k == 1 ? 1.0 / (1.0 - rho * rho / 2.0) : 1.0 / (1.0 - rho * rho * w / 4.0);
    const bool last = k + 1 == FE_CHEB_STEPS;
    T* out = last ? t : prev;
    e = step((const T*)t, (const T*)cur, k == 1 ? (const T*)nullptr : (const T*)prev, out, (C)w, 0);
    if (e != hipSuccess) return e;
    prev = cur;
    cur = out;
  }
  return hipSuccess;
}

hipError_t fe_assemble_rhs(const aao_problem* h, const double* f, const double* u0, double* rhs, hipStream_t st) {
  const int64_t N = h->N;
  const FeRows rows = fe_rows(h);
  hipError_t e = by_radius(h, [&](auto r_) {
    constexpr int R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_mass<R>), fe_grid(h, 1), dim3(TPB), 0, st, u0, rhs, h->n, rows);
  });
  if (e != hipSuccess) return e;
  e = launch_fill<double>(rhs + N, 0.0, (int64_t)h->nt * N, st);
  if (e != hipSuccess) return e;
  return by_radius(h, [&](auto r_) {
    constexpr int R = decltype(r_)::value;
    hipLaunchKernelGGL((k_fe_mass<R>), fe_grid(h, (int64_t)h->nt * h->s), dim3(TPB), 0, st, f,
                       rhs + (int64_t)(h->nt + 1) * N, h->n, rows);
  });
}

template <class T>
hipError_t fe_q2_smooth(const aao_problem* h, double a, const T* xin, int64_t sxin, T* xout, int64_t sxout,
                        const T* b, int64_t sb, double omega, bool zero_init, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  hipLaunchKernelGGL((k_q2_smooth<T>), fe_grid(h, B), dim3(TPB), 0, st, xin, sxin, xout, sxout, b, sb, h->n,
                     fe_rows(h), (C)a, (C)omega, (int)zero_init);
  return hipGetLastError();
}

template <class T>
hipError_t fe_q2_residual(const aao_problem* h, double a, const T* x, int64_t sx, const T* b, int64_t sb, T* r,
                          int64_t sr, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  hipLaunchKernelGGL((k_q2_residual<T>), fe_grid(h, B), dim3(TPB), 0, st, x, sx, b, sb, r, sr, h->n, fe_rows(h),
                     (C)a);
  return hipGetLastError();
}

#define AAO_FE_INST(T)                                                                                          \
  template hipError_t fe_theta_apply<T>(const aao_problem*, const Tab&, const T*, int64_t, T*, int64_t, int,     \
                                        hipStream_t);                                                           \
  template hipError_t fe_rana_rhs<T>(const aao_problem*, const Tab&, int, const T*, int64_t, const T*, int64_t, \
                                     T*, int64_t, int, hipStream_t);                                            \
  template hipError_t fe_schur_coupling<T>(const aao_problem*, const double*, const T*, T*, hipStream_t);       \
  template hipError_t fe_schur_kz<T>(const aao_problem*, const T*, int64_t, T*, int64_t, int, hipStream_t);     \
  template hipError_t fe_mass_solve<T>(const aao_problem*, T*, T*, T*, int, hipStream_t);                       \
  template hipError_t fe_apply_A<T>(const aao_problem*, const T*, double*, bool, hipStream_t);                   \
  template hipError_t fe_q2_smooth<T>(const aao_problem*, double, const T*, int64_t, T*, int64_t, const T*,      \
                                      int64_t, double, bool, int, hipStream_t);                                  \
  template hipError_t fe_q2_residual<T>(const aao_problem*, double, const T*, int64_t, const T*, int64_t, T*,    \
                                        int64_t, int, hipStream_t);
AAO_FE_INST(double)
AAO_FE_INST(float)
AAO_FE_INST(__half)
#undef AAO_FE_INST

}  // namespace aao

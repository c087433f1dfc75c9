// All-at-once operator of eq. (2.4) and its transpose, matrix-free in FP64.
//
// One thread owns one grid node p of one time step n and produces every
// output row touching (n, p): the s stage rows of step n and the update row
// of v_{n+1}.  The s x s Runge--Kutta mixing is done in registers on K applied
// to each input block (K is linear, so K w_i = K v_n + tau sum_j a_ij K V_j).
// Stencil neighbours come through the L1/L2 caches: consecutive lanes own
// consecutive x, and a workgroup covers whole rows, so each value is fetched
// from HBM about once per launch.
#include "aao_internal.h"
#include "fe.h"
#include "stencil.h"

namespace aao {

namespace {

constexpr int TPB = 256;

template <int DIM, int S, bool VK, class TX>
__global__ __launch_bounds__(TPB) void k_apply_A(const TX* __restrict__ x, double* __restrict__ y,
                                                 int n, int N, int nt, double ih2, Tab tab,
                                                 Faces<double> fc) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int step = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const int64_t NN = N;
  const TX* v = x + (int64_t)step * NN;
  const TX* V = x + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
  const double Kv = ih2 * stencil_K<DIM, VK, TX, double>(v, p, i, j, k, n, N, fc);
  double KV[S], Vp[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    KV[q] = ih2 * stencil_K<DIM, VK, TX, double>(V + q * NN, p, i, j, k, n, N, fc);
    Vp[q] = ld<TX, double>(V + q * NN + p);
  }
  double* yV = y + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
  double upd = 0.0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    double mix = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q) mix += tab.A[r * S + q] * KV[q];
    yV[r * NN + p] = Vp[r] + Kv + tab.tau * mix;
    upd += tab.b[r] * Vp[r];
  }
  const double vp = ld<TX, double>(v + p);
  y[(int64_t)(step + 1) * NN + p] = ld<TX, double>(v + NN + p) - vp - tab.tau * upd;
  if (step == 0) y[p] = vp;
}

// 2D variant: each thread owns W adjacent x positions of one step and
// marches along y over ROWS rows with a register window of rows j-1 .. j+2 of
// every input field (row j+2 is fetched while row j is computed), so each
// value is read from HBM once per launch.  W = 2 uses 16-byte loads and
// stores (n even).  The x neighbours are taken from the adjacent lanes of the
// wave; only lanes 0 and 63 load the value beyond their wave.
constexpr int ROWS = 64;

template <int W, class TX>
__device__ __forceinline__ void ldw(const TX* p, double* out) {
  if constexpr (W == 1) {
    out[0] = ld<TX, double>(p);
  } else if constexpr (std::is_same<TX, double>::value) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    out[0] = t.x;
    out[1] = t.y;
  } else if constexpr (std::is_same<TX, float>::value) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    out[0] = t.x;
    out[1] = t.y;
  } else {
    out[0] = ld<TX, double>(p);
    out[1] = ld<TX, double>(p + 1);
  }
}

template <int W>
__device__ __forceinline__ void stw(double* p, const double* v) {
  if constexpr (W == 1) {
    p[0] = v[0];
  } else {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  }
}

template <int W>
struct March2D {
  int n, i, lane, j0, j1, eoff;
  bool live, edge;
  __device__ explicit March2D(int n_) : n(n_) {
    i = (blockIdx.x * TPB + threadIdx.x) * W;
    lane = threadIdx.x & 63;
    live = i < n;  // W = 2 only for even n: both columns live or neither
    eoff = lane == 0 ? -1 : W;
    edge = live && ((lane == 0 && i > 0) || (lane == 63 && i + W < n));
    j0 = blockIdx.y * ROWS;
    j1 = j0 + ROWS < n ? j0 + ROWS : n;
  }
  // whole wave beyond the last column: nothing to do (wave-uniform)
  __device__ bool idle() const { return (int)((blockIdx.x * TPB + (threadIdx.x & ~63)) * W) >= n; }
  // row jr of field f at this thread's columns (zero outside the grid and past jmax)
  template <class TX>
  __device__ void row(const TX* f, int jr, int jmax, double* out) const {
    if (live && jr >= 0 && jr <= jmax && jr < n) {
      ldw<W>(f + (int64_t)jr * n + i, out);
    } else {
#pragma unroll
      for (int c = 0; c < W; ++c) out[c] = 0.0;
    }
  }
  template <class TX>
  __device__ double row1(const TX* f, int jr, int jmax) const {
    return (live && jr <= jmax) ? ld<TX, double>(f + (int64_t)jr * n + i) : 0.0;
  }
  // edge lanes: the neighbour outside the wave on row jr
  template <class TX>
  __device__ double edge_val(const TX* f, int jr, int jmax) const {
    return (edge && jr <= jmax) ? ld<TX, double>(f + (int64_t)jr * n + i + eoff) : 0.0;
  }
  // x neighbours of column c given this thread's row values r and edge value e
  __device__ double left(const double* r, double e, int c) const {
    if (c > 0) return r[c - 1];
    const double s = __shfl_up(r[W - 1], 1);
    return lane == 0 ? e : s;
  }
  __device__ double right(const double* r, double e, int c) const {
    if (c < W - 1) return r[c + 1];
    const double s = __shfl_down(r[0], 1);
    return lane == 63 ? e : s;
  }
};

template <bool VK>
__device__ __forceinline__ double k5(double c, double xm, double xp, double ym, double yp, double ih2,
                                     const Faces<double>& fc, int64_t p) {
  if (!VK) return ih2 * (4.0 * c - xm - xp - ym - yp);
  return ih2 * (fc.m[0][p] * (c - xm) + fc.p[0][p] * (c - xp) + fc.m[1][p] * (c - ym) + fc.p[1][p] * (c - yp));
}

template <int S, bool VK, int W, class TX>
__global__ __launch_bounds__(TPB) void k_apply_A_2d(const TX* __restrict__ x, double* __restrict__ y, int n, int nt,
                                                    double ih2, Tab tab, Faces<double> fc) {
  const March2D<W> m(n);
  if (m.idle()) return;
  const int step = blockIdx.z;
  const int64_t N = (int64_t)n * n;
  constexpr int F = S + 1;  // v_n and the S stage fields
  const TX* fld[F];
  fld[0] = x + (int64_t)step * N;
#pragma unroll
  for (int q = 0; q < S; ++q) fld[q + 1] = x + ((int64_t)(nt + 1) + (int64_t)step * S + q) * N;
  const TX* vn = x + (int64_t)(step + 1) * N;
  double* yV = y + ((int64_t)(nt + 1) + (int64_t)step * S) * N;
  double* yv = y + (int64_t)(step + 1) * N;
  const int jl = m.j1;  // last row any window needs
  double r0[F][W], r1[F][W], r2[F][W], r3[F][W], e0[F], e1[F], w0[W], w1[W];
#pragma unroll
  for (int q = 0; q < F; ++q) {
    m.row(fld[q], m.j0 - 1, jl, r0[q]);
    m.row(fld[q], m.j0, jl, r1[q]);
    m.row(fld[q], m.j0 + 1, jl, r2[q]);
    e0[q] = m.edge_val(fld[q], m.j0, jl);
  }
  m.row(vn, m.j0, jl, w0);
  for (int j = m.j0; j < m.j1; ++j) {
#pragma unroll
    for (int q = 0; q < F; ++q) {
      m.row(fld[q], j + 2, jl, r3[q]);
      e1[q] = m.edge_val(fld[q], j + 1, m.j1 - 1);
    }
    m.row(vn, j + 1, m.j1 - 1, w1);
    const int64_t p = (int64_t)j * n + m.i;
    double KF[F][W];
#pragma unroll
    for (int q = 0; q < F; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c)
        KF[q][c] = k5<VK>(r1[q][c], m.left(r1[q], e0[q], c), m.right(r1[q], e0[q], c), r0[q][c], r2[q][c], ih2, fc,
                          m.live ? p + c : 0);
    if (m.live) {
      double yvv[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double upd = 0.0;
#pragma unroll
        for (int r = 0; r < S; ++r) upd += tab.b[r] * r1[r + 1][c];
        yvv[c] = w0[c] - r1[0][c] - tab.tau * upd;
      }
#pragma unroll
      for (int r = 0; r < S; ++r) {
        double out[W];
#pragma unroll
        for (int c = 0; c < W; ++c) {
          double mix = 0.0;
#pragma unroll
          for (int q = 0; q < S; ++q) mix += tab.A[r * S + q] * KF[q + 1][c];
          out[c] = r1[r + 1][c] + KF[0][c] + tab.tau * mix;
        }
        stw<W>(yV + (int64_t)r * N + p, out);
      }
      stw<W>(yv + p, yvv);
      if (step == 0) stw<W>(y + p, r1[0]);
    }
#pragma unroll
    for (int q = 0; q < F; ++q) {
#pragma unroll
      for (int c = 0; c < W; ++c) {
        r0[q][c] = r1[q][c];
        r1[q][c] = r2[q][c];
        r2[q][c] = r3[q][c];
      }
      e0[q] = e1[q];
    }
#pragma unroll
    for (int c = 0; c < W; ++c) w0[c] = w1[c];
  }
}

// 3D variant (constant kappa): the 64 lanes of a wave own W * 64 adjacent x
// positions of one row (j, plane k) of one step, the four waves of a
// workgroup four consecutive rows j, and each thread marches along z over
// ZR planes with a register window of planes k-1 .. k+2 of every input
// field (plane k+2 is fetched while plane k is computed).  x neighbours
// come from the adjacent lanes; the y neighbours (rows j +- 1 of plane k)
// are loaded directly: the sibling waves fetch those rows for themselves at
// the same time, so they come from L2.  Per value and field: one streamed
// load and two cached ones, against seven for one thread per node.
constexpr int ZR = 32;
constexpr int TPB3 = 512;
constexpr int RWG = TPB3 / 64;   // rows (waves) per workgroup

// Workgroup b of the 1D grid takes logical tile xcd_tile(b, B), ordered x
// block fastest, then row group, z chunk and step: each XCD walks a
// contiguous range, so the rows j +- 1 a workgroup reads from its
// neighbours' row groups sit in the same L2.
template <int W>
struct March3D {
  int n, i, j, lane, step, k0, k1, eoff, xb;
  bool live, edge;
  __device__ March3D(int n_, int xblocks, int jgroups, int zchunks) : n(n_) {
    int t = xcd_tile(blockIdx.x, gridDim.x);
    xb = t % xblocks;
    t /= xblocks;
    const int jg = t % jgroups;
    t /= jgroups;
    const int zc = t % zchunks;
    step = t / zchunks;
    lane = threadIdx.x & 63;
    i = (xb * 64 + lane) * W;
    j = jg * RWG + (threadIdx.x >> 6);
    k0 = zc * ZR;
    k1 = k0 + ZR < n ? k0 + ZR : n;
    live = i < n && j < n;
    eoff = lane == 0 ? -1 : W;
    edge = live && ((lane == 0 && i > 0) || (lane == 63 && i + W < n));
  }
  // the whole wave has no node (wave-uniform: j and the x range per wave)
  __device__ bool idle() const { return j >= n || xb * 64 * W >= n; }
  // row (jr, plane kr) of field f at this thread's columns; zero outside
  // the grid and for planes past kmax
  template <class TX>
  __device__ void row(const TX* f, int jr, int kr, int kmax, double* out) const {
    if (live && jr >= 0 && jr < n && kr >= 0 && kr <= kmax && kr < n) {
      ldw<W>(f + ((int64_t)kr * n + jr) * n + i, out);
    } else {
#pragma unroll
      for (int c = 0; c < W; ++c) out[c] = 0.0;
    }
  }
  template <class TX>
  __device__ double edge_val(const TX* f, int kr, int kmax) const {
    return (edge && kr <= kmax) ? ld<TX, double>(f + ((int64_t)kr * n + j) * n + i + eoff) : 0.0;
  }
  __device__ double left(const double* r, double e, int c) const {
    if (c > 0) return r[c - 1];
    const double s = __shfl_up(r[W - 1], 1);
    return lane == 0 ? e : s;
  }
  __device__ double right(const double* r, double e, int c) const {
    if (c < W - 1) return r[c + 1];
    const double s = __shfl_down(r[0], 1);
    return lane == 63 ? e : s;
  }
};

template <int S, int W, class TX>
__global__ __launch_bounds__(TPB3) void k_apply_A_3d(const TX* __restrict__ x, double* __restrict__ y, int n, int nt,
                                                     int xblocks, int jgroups, int zchunks, double ih2, Tab tab) {
  const March3D<W> m(n, xblocks, jgroups, zchunks);
  if (m.idle()) return;
  const int step = m.step;
  const int64_t N = (int64_t)n * n * n;
  constexpr int F = S + 1;  // v_n and the S stage fields
  const TX* fld[F];
  fld[0] = x + (int64_t)step * N;
#pragma unroll
  for (int q = 0; q < S; ++q) fld[q + 1] = x + ((int64_t)(nt + 1) + (int64_t)step * S + q) * N;
  const TX* vn = x + (int64_t)(step + 1) * N;
  double* yV = y + ((int64_t)(nt + 1) + (int64_t)step * S) * N;
  double* yv = y + (int64_t)(step + 1) * N;
  const int kl = m.k1;  // last plane any window needs
  double r0[F][W], r1[F][W], r2[F][W], r3[F][W], e0[F], e1[F], w0[W], w1[W];
#pragma unroll
  for (int q = 0; q < F; ++q) {
    m.row(fld[q], m.j, m.k0 - 1, kl, r0[q]);
    m.row(fld[q], m.j, m.k0, kl, r1[q]);
    m.row(fld[q], m.j, m.k0 + 1, kl, r2[q]);
    e0[q] = m.edge_val(fld[q], m.k0, kl);
  }
  m.row(vn, m.j, m.k0, kl, w0);
  for (int kp = m.k0; kp < m.k1; ++kp) {
    double ym[F][W], yp[F][W];
#pragma unroll
    for (int q = 0; q < F; ++q) {
      m.row(fld[q], m.j, kp + 2, kl, r3[q]);
      e1[q] = m.edge_val(fld[q], kp + 1, m.k1 - 1);
      m.row(fld[q], m.j - 1, kp, kl, ym[q]);
      m.row(fld[q], m.j + 1, kp, kl, yp[q]);
    }
    m.row(vn, m.j, kp + 1, m.k1 - 1, w1);
    const int64_t p = ((int64_t)kp * n + m.j) * n + m.i;
    double KF[F][W];
#pragma unroll
    for (int q = 0; q < F; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c)
        KF[q][c] = ih2 * (6.0 * r1[q][c] - m.left(r1[q], e0[q], c) - m.right(r1[q], e0[q], c) - ym[q][c] -
                          yp[q][c] - r0[q][c] - r2[q][c]);
    if (m.live) {
      double yvv[W];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double upd = 0.0;
#pragma unroll
        for (int r = 0; r < S; ++r) upd += tab.b[r] * r1[r + 1][c];
        yvv[c] = w0[c] - r1[0][c] - tab.tau * upd;
      }
#pragma unroll
      for (int r = 0; r < S; ++r) {
        double out[W];
#pragma unroll
        for (int c = 0; c < W; ++c) {
          double mix = 0.0;
#pragma unroll
          for (int q = 0; q < S; ++q) mix += tab.A[r * S + q] * KF[q + 1][c];
          out[c] = r1[r + 1][c] + KF[0][c] + tab.tau * mix;
        }
        stw<W>(yV + (int64_t)r * N + p, out);
      }
      stw<W>(yv + p, yvv);
      if (step == 0) stw<W>(y + p, r1[0]);
    }
#pragma unroll
    for (int q = 0; q < F; ++q) {
#pragma unroll
      for (int c = 0; c < W; ++c) {
        r0[q][c] = r1[q][c];
        r1[q][c] = r2[q][c];
        r2[q][c] = r3[q][c];
      }
      e0[q] = e1[q];
    }
#pragma unroll
    for (int c = 0; c < W; ++c) w0[c] = w1[c];
  }
}

// Transposed, 2D marching form (see k_apply_A_2d).
template <int S, bool VK, int W, class TX>
__global__ __launch_bounds__(TPB) void k_apply_AT_2d(const TX* __restrict__ x, double* __restrict__ y, int n, int nt,
                                                     double ih2, Tab tab, Faces<double> fc) {
  const March2D<W> m(n);
  if (m.idle()) return;
  const int step = blockIdx.z;
  const int64_t N = (int64_t)n * n;
  const TX* fld[S];
#pragma unroll
  for (int q = 0; q < S; ++q) fld[q] = x + ((int64_t)(nt + 1) + (int64_t)step * S + q) * N;
  const TX* xv = x + (int64_t)step * N;
  const TX* xvn = x + (int64_t)(step + 1) * N;
  double* yV = y + ((int64_t)(nt + 1) + (int64_t)step * S) * N;
  double* yv = y + (int64_t)step * N;
  const int jl = m.j1;
  double r0[S][W], r1[S][W], r2[S][W], r3[S][W], e0[S], e1[S], a0[W], b0[W], a1[W], b1[W];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    m.row(fld[q], m.j0 - 1, jl, r0[q]);
    m.row(fld[q], m.j0, jl, r1[q]);
    m.row(fld[q], m.j0 + 1, jl, r2[q]);
    e0[q] = m.edge_val(fld[q], m.j0, jl);
  }
  m.row(xv, m.j0, jl, a0);
  m.row(xvn, m.j0, jl, b0);
  for (int j = m.j0; j < m.j1; ++j) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      m.row(fld[q], j + 2, jl, r3[q]);
      e1[q] = m.edge_val(fld[q], j + 1, m.j1 - 1);
    }
    m.row(xv, j + 1, m.j1 - 1, a1);
    m.row(xvn, j + 1, m.j1 - 1, b1);
    const int64_t p = (int64_t)j * n + m.i;
    double KX[S][W], sumK[W];
#pragma unroll
    for (int c = 0; c < W; ++c) sumK[c] = 0.0;
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int c = 0; c < W; ++c) {
        KX[q][c] = k5<VK>(r1[q][c], m.left(r1[q], e0[q], c), m.right(r1[q], e0[q], c), r0[q][c], r2[q][c], ih2, fc,
                          m.live ? p + c : 0);
        sumK[c] += KX[q][c];
      }
    if (m.live) {
      double out[W];
#pragma unroll
      for (int c = 0; c < W; ++c) out[c] = a0[c] - b0[c] + sumK[c];
      stw<W>(yv + p, out);
#pragma unroll
      for (int cs = 0; cs < S; ++cs) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
          double mix = 0.0;
#pragma unroll
          for (int r = 0; r < S; ++r) mix += tab.A[r * S + cs] * KX[r][c];
          out[c] = r1[cs][c] + tab.tau * mix - tab.tau * tab.b[cs] * b0[c];
        }
        stw<W>(yV + (int64_t)cs * N + p, out);
      }
      if (step == nt - 1) stw<W>(y + (int64_t)nt * N + p, b0);
    }
#pragma unroll
    for (int q = 0; q < S; ++q) {
#pragma unroll
      for (int c = 0; c < W; ++c) {
        r0[q][c] = r1[q][c];
        r1[q][c] = r2[q][c];
        r2[q][c] = r3[q][c];
      }
      e0[q] = e1[q];
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
      a0[c] = a1[c];
      b0[c] = b1[c];
    }
  }
}

// Transposed rows:  y_{v,n} = x_{v,n} - x_{v,n+1} + K sum_i x_{V,n,i}  (n < nt)
//                   y_{v,nt} = x_{v,nt}
//                   y_{V,n,j} = x_{V,n,j} + tau K sum_i a_ij x_{V,n,i} - tau b_j x_{v,n+1}
template <int DIM, int S, bool VK, class TX>
__global__ __launch_bounds__(TPB) void k_apply_AT(const TX* __restrict__ x, double* __restrict__ y,
                                                  int n, int N, int nt, double ih2, Tab tab,
                                                  Faces<double> fc) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int step = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const int64_t NN = N;
  const TX* V = x + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
  double KX[S];
  double sumK = 0.0;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    KX[q] = ih2 * stencil_K<DIM, VK, TX, double>(V + q * NN, p, i, j, k, n, N, fc);
    sumK += KX[q];
  }
  const double xv = ld<TX, double>(x + (int64_t)step * NN + p);
  const double xvn = ld<TX, double>(x + (int64_t)(step + 1) * NN + p);
  y[(int64_t)step * NN + p] = xv - xvn + sumK;
  double* yV = y + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
#pragma unroll
  for (int c = 0; c < S; ++c) {
    double mix = 0.0;
#pragma unroll
    for (int r = 0; r < S; ++r) mix += tab.A[r * S + c] * KX[r];
    yV[c * NN + p] = ld<TX, double>(V + c * NN + p) + tab.tau * mix - tab.tau * tab.b[c] * xvn;
  }
  if (step == nt - 1) y[(int64_t)nt * NN + p] = xvn;
}

// g_p = - sum_{n,i} sum_{faces f of p} dkappa_f/dtheta_p (lam_p - lam_q)(w_p - w_q) / h^2,
// w_{n,i} = v_n + tau sum_j a_ij V_{n,j}; lam_q = w_q = 0 across boundary faces.
template <int DIM, int S>
__global__ __launch_bounds__(TPB) void k_grad_logkappa(const double* __restrict__ x,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ kappa,
                                                       double* __restrict__ g, int n, int N, int nt,
                                                       double ih2, Tab tab) {
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  int c[3];
  node_coords<DIM>(p, n, c[0], c[1], c[2]);
  const int64_t NN = N;
  const int strides[3] = {1, n, n * n};
  const double kp = kappa ? kappa[p] : 1.0;
  double dk[2 * DIM];          // dkappa_f / dtheta_p per face (minus, plus per axis)
  int nb[2 * DIM];             // neighbour index or -1
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const bool inside = sd == 0 ? c[a] > 0 : c[a] + 1 < n;
      const int q = sd == 0 ? p - strides[a] : p + strides[a];
      nb[2 * a + sd] = inside ? q : -1;
      if (inside) {
        const double kq = kappa ? kappa[q] : 1.0;
        dk[2 * a + sd] = kp * 2.0 * kq * kq / ((kp + kq) * (kp + kq));
      } else {
        dk[2 * a + sd] = kp;
      }
    }
  }
  double acc = 0.0;
  for (int step = 0; step < nt; ++step) {
    const double* v = x + (int64_t)step * NN;
    const double* V = x + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
    const double* L = lam + ((int64_t)(nt + 1) + (int64_t)step * S) * NN;
#pragma unroll
    for (int r = 0; r < S; ++r) {
      auto wat = [&](int q) {
        double m = 0.0;
#pragma unroll
        for (int jj = 0; jj < S; ++jj) m += tab.A[r * S + jj] * V[jj * NN + q];
        return v[q] + tab.tau * m;
      };
      const double wp = wat(p);
      const double lp = L[r * NN + p];
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f) {
        const int q = nb[f];
        const double wq = q >= 0 ? wat(q) : 0.0;
        const double lq = q >= 0 ? L[r * NN + q] : 0.0;
        acc += dk[f] * (lp - lq) * (wp - wq);
      }
    }
  }
  g[p] = -acc * ih2;
}

template <class TD, class TS>
__global__ void k_copy_cast(TD* __restrict__ d, const TS* __restrict__ s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    st<TD, typename Acc<TD>::type>(d + i, (typename Acc<TD>::type)ld<TS, double>(s + i));
}

// y = a - y
__global__ void k_sub_from(const double* __restrict__ a, double* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a[i] - y[i];
}

// y = alpha x
template <class TY, class TX>
__global__ void k_scale(TY* __restrict__ y, const TX* __restrict__ x, double alpha, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    st<TY, typename Acc<TY>::type>(y + i, (typename Acc<TY>::type)(alpha * ld<TX, double>(x + i)));
}

template <class T>
__global__ void k_fill(T* __restrict__ d, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = v;
}

inline unsigned grid1d(int64_t n) {
  int64_t b = (n + TPB - 1) / TPB;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

Faces<double> face_ptrs(const aao_problem* h) {
  Faces<double> f{};
  if (h->vark) {
    const double* base = reinterpret_cast<const double*>(h->ws + h->plan.faces_d);
    for (int a = 0; a < h->dim; ++a) {
      f.m[a] = base + (2 * a) * h->N;
      f.p[a] = base + (2 * a + 1) * h->N;
    }
  }
  return f;
}

}  // namespace

// The two-column 2D kernels need even n and 16-byte aligned x and y rows.
template <class TX>
static bool two_columns(int n, const TX* x, const double* y) {
  return n % 2 == 0 && reinterpret_cast<uintptr_t>(x) % (2 * sizeof(TX)) == 0 &&
         reinterpret_cast<uintptr_t>(y) % 16 == 0;
}

#define DISPATCH_SV(s_, vk_, M)                                          \
  do {                                                                   \
    if (vk_) { if ((s_) == 1) M(1, true); else if ((s_) == 2) M(2, true); else M(3, true); }       \
    else { if ((s_) == 1) M(1, false); else if ((s_) == 2) M(2, false); else M(3, false); }        \
  } while (0)

template <class TX>
hipError_t launch_apply_A(const aao_problem* h, const TX* x, double* y, hipStream_t st) {
  if (h->fe) return fe_apply_A<TX>(h, x, y, false, st);
  const int n = h->n, N = (int)h->N, nt = h->nt;
  Faces<double> fc = face_ptrs(h);
  if (h->dim == 2) {
    const int W = two_columns(n, x, y) ? 2 : 1;
    const dim3 g2((unsigned)((n + TPB * W - 1) / (TPB * W)), (unsigned)((n + ROWS - 1) / ROWS), (unsigned)nt);
#define AAO_A2(S, V)                                                                                          \
  do {                                                                                                     \
    if (W == 2) hipLaunchKernelGGL((k_apply_A_2d<S, V, 2, TX>), g2, dim3(TPB), 0, st, x, y, n, nt, h->ih2, h->tab, fc); \
    else hipLaunchKernelGGL((k_apply_A_2d<S, V, 1, TX>), g2, dim3(TPB), 0, st, x, y, n, nt, h->ih2, h->tab, fc);        \
  } while (0)
    DISPATCH_SV(h->s, h->vark, AAO_A2);
#undef AAO_A2
    return hipGetLastError();
  }
  if (h->dim == 3 && !h->vark) {
    const int W = two_columns(n, x, y) ? 2 : 1;
    const int xblocks = (n + 64 * W - 1) / (64 * W), jgroups = (n + RWG - 1) / RWG, zchunks = (n + ZR - 1) / ZR;
    const dim3 g3((unsigned)((int64_t)xblocks * jgroups * zchunks * nt));
#define AAO_A3(S, V)                                                                                          \
  do {                                                                                                       \
    if (W == 2)                                                                                              \
      hipLaunchKernelGGL((k_apply_A_3d<S, 2, TX>), g3, dim3(TPB3), 0, st, x, y, n, nt, xblocks, jgroups, zchunks, \
                         h->ih2, h->tab);                                                                    \
    else                                                                                                     \
      hipLaunchKernelGGL((k_apply_A_3d<S, 1, TX>), g3, dim3(TPB3), 0, st, x, y, n, nt, xblocks, jgroups, zchunks, \
                         h->ih2, h->tab);                                                                    \
  } while (0)
    DISPATCH_SV(h->s, false, AAO_A3);
#undef AAO_A3
    return hipGetLastError();
  }
  dim3 grid((unsigned)((h->N + TPB - 1) / TPB), (unsigned)h->nt);
#define AAO_LAUNCH_A(D, S, V) \
  hipLaunchKernelGGL((k_apply_A<D, S, V, TX>), grid, dim3(TPB), 0, st, x, y, n, N, nt, h->ih2, h->tab, fc)
  DISPATCH_DSV(h->dim, h->s, h->vark, AAO_LAUNCH_A);
#undef AAO_LAUNCH_A
  return hipGetLastError();
}

template <class TX>
hipError_t launch_apply_AT(const aao_problem* h, const TX* x, double* y, hipStream_t st) {
  if (h->fe) return fe_apply_A<TX>(h, x, y, true, st);
  const int n = h->n, N = (int)h->N, nt = h->nt;
  Faces<double> fc = face_ptrs(h);
  if (h->dim == 2) {
    const int W = two_columns(n, x, y) ? 2 : 1;
    const dim3 g2((unsigned)((n + TPB * W - 1) / (TPB * W)), (unsigned)((n + ROWS - 1) / ROWS), (unsigned)nt);
#define AAO_AT2(S, V)                                                                                          \
  do {                                                                                                     \
    if (W == 2) hipLaunchKernelGGL((k_apply_AT_2d<S, V, 2, TX>), g2, dim3(TPB), 0, st, x, y, n, nt, h->ih2, h->tab, fc); \
    else hipLaunchKernelGGL((k_apply_AT_2d<S, V, 1, TX>), g2, dim3(TPB), 0, st, x, y, n, nt, h->ih2, h->tab, fc);        \
  } while (0)
    DISPATCH_SV(h->s, h->vark, AAO_AT2);
#undef AAO_AT2
    return hipGetLastError();
  }
  dim3 grid((unsigned)((h->N + TPB - 1) / TPB), (unsigned)h->nt);
#define AAO_LAUNCH_AT(D, S, V) \
  hipLaunchKernelGGL((k_apply_AT<D, S, V, TX>), grid, dim3(TPB), 0, st, x, y, n, N, nt, h->ih2, h->tab, fc)
  DISPATCH_DSV(h->dim, h->s, h->vark, AAO_LAUNCH_AT);
#undef AAO_LAUNCH_AT
  return hipGetLastError();
}

hipError_t launch_grad_logkappa(const aao_problem* h, const double* x, const double* lam, double* g,
                                hipStream_t st) {
  dim3 grid((unsigned)((h->N + TPB - 1) / TPB));
  const int n = h->n, N = (int)h->N, nt = h->nt;
  const double* kap = h->vark ? reinterpret_cast<const double*>(h->ws + h->plan.faces_d) +
                                    (int64_t)2 * h->dim * h->N
                              : nullptr;
#define AAO_LAUNCH_G(D, S, V) \
  hipLaunchKernelGGL((k_grad_logkappa<D, S>), grid, dim3(TPB), 0, st, x, lam, kap, g, n, N, nt, h->ih2, h->tab)
  DISPATCH_DSV(h->dim, h->s, false, AAO_LAUNCH_G);
#undef AAO_LAUNCH_G
  return hipGetLastError();
}

hipError_t launch_assemble_rhs(const aao_problem* h, const double* f, const double* u0, double* rhs,
                               hipStream_t st) {
  if (h->fe) return fe_assemble_rhs(h, f, u0, rhs, st);
  const int64_t N = h->N;
  hipError_t e = hipMemcpyAsync(rhs, u0, N * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = launch_fill<double>(rhs + N, 0.0, (int64_t)h->nt * N, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(rhs + (int64_t)(h->nt + 1) * N, f, (size_t)h->UV * sizeof(double),
                        hipMemcpyDeviceToDevice, st);
}

// out = a - b (b may be null: out = a), converted to TO
template <class TO, class TA>
__global__ void k_diff(TO* __restrict__ out, const TA* __restrict__ a, const TA* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double v = ld<TA, double>(a + i) - (b ? ld<TA, double>(b + i) : 0.0);
    out[i] = (TO)v;
  }
}

template <class TO, class TA>
hipError_t launch_diff(TO* out, const TA* a, const TA* b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_diff<TO, TA>), dim3(grid1d(n)), dim3(TPB), 0, st, out, a, b, n);
  return hipGetLastError();
}
template hipError_t launch_diff<double, double>(double*, const double*, const double*, int64_t, hipStream_t);
template hipError_t launch_diff<double, float>(double*, const float*, const float*, int64_t, hipStream_t);

template <class TD, class TS>
hipError_t launch_copy_cast(TD* dst, const TS* src, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_cast<TD, TS>), dim3(grid1d(n)), dim3(TPB), 0, st, dst, src, n);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fill(T* dst, T v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid1d(n)), dim3(TPB), 0, st, dst, v, n);
  return hipGetLastError();
}

__global__ void k_round_f32(double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
    x[i] = (double)(float)x[i];
}

hipError_t launch_round_f32(double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_round_f32, dim3(grid1d(n)), dim3(TPB), 0, st, x, n);
  return hipGetLastError();
}

__global__ void k_round_bf16(double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
    x[i] = (double)__bfloat162float(__float2bfloat16((float)x[i]));
}

hipError_t launch_round_bf16(double* x, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_round_bf16, dim3(grid1d(n)), dim3(TPB), 0, st, x, n);
  return hipGetLastError();
}

hipError_t launch_sub_from(const double* a, double* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_from, dim3(grid1d(n)), dim3(TPB), 0, st, a, y, n);
  return hipGetLastError();
}

template <class TY, class TX>
hipError_t launch_scale(TY* y, const TX* x, double alpha, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_scale<TY, TX>), dim3(grid1d(n)), dim3(TPB), 0, st, y, x, alpha, n);
  return hipGetLastError();
}

template hipError_t launch_scale<double, double>(double*, const double*, double, int64_t, hipStream_t);
template hipError_t launch_scale<float, float>(float*, const float*, double, int64_t, hipStream_t);
template hipError_t launch_scale<float, double>(float*, const double*, double, int64_t, hipStream_t);
template hipError_t launch_apply_AT<double>(const aao_problem*, const double*, double*, hipStream_t);
template hipError_t launch_apply_AT<float>(const aao_problem*, const float*, double*, hipStream_t);
template hipError_t launch_apply_A<double>(const aao_problem*, const double*, double*, hipStream_t);
template hipError_t launch_apply_A<float>(const aao_problem*, const float*, double*, hipStream_t);
template hipError_t launch_apply_A<__half>(const aao_problem*, const __half*, double*, hipStream_t);
template hipError_t launch_apply_AT<__half>(const aao_problem*, const __half*, double*, hipStream_t);
template hipError_t launch_copy_cast<double, __half>(double*, const __half*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<__half, double>(__half*, const double*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<__half, __half>(__half*, const __half*, int64_t, hipStream_t);
template hipError_t launch_scale<__half, __half>(__half*, const __half*, double, int64_t, hipStream_t);
template hipError_t launch_scale<__half, double>(__half*, const double*, double, int64_t, hipStream_t);
template hipError_t launch_fill<__half>(__half*, __half, int64_t, hipStream_t);
template hipError_t launch_diff<double, __half>(double*, const __half*, const __half*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<double, float>(double*, const float*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<float, double>(float*, const double*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<double, double>(double*, const double*, int64_t, hipStream_t);
template hipError_t launch_copy_cast<float, float>(float*, const float*, int64_t, hipStream_t);
template hipError_t launch_fill<double>(double*, double, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float*, float, int64_t, hipStream_t);
template hipError_t launch_fill<unsigned>(unsigned*, unsigned, int64_t, hipStream_t);

}  // namespace aao

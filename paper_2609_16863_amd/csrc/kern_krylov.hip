// Batched Krylov kernels: segmented dot products (wave64 shuffles, LDS, and a
// fixed-order second pass, so results are bitwise reproducible), multi-AXPYs,
// the Givens update of GMRES on device, and the stage-level operators used by
// the preconditioner (Theta_hat, Rana coupling, S-tilde sweep pieces).
#include "aao_internal.h"
#include "fe.h"
#include "krylov.h"
#include "stencil.h"

namespace aao {

namespace {

constexpr int TPB = RED_THREADS;
constexpr int NSLOT = DOTS_PER_PASS + 1;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// GMRES scalar recurrences (run by one thread of the finishing workgroup)
// ---------------------------------------------------------------------------
using S = InnerSlots;

// Start: beta = ||r||, g = beta e1, 1/beta for the first basis vector.
__device__ void gmres_start(double* q, double ww, unsigned* counters) {
  const bool ok = ww > 0.0 && isfinite(ww);
  if (counters) atomicAdd(&counters[1], 1u);
  const double nb = ok ? sqrt(ww) : 0.0;
  q[S::BETA] = nb;
  q[S::ACTIVE] = ok ? 1.0 : 0.0;
  q[S::M] = 0.0;
  for (int i = 0; i <= KMAX; ++i) q[S::G + i] = 0.0;
  q[S::G] = nb;
  q[S::INV] = ok ? 1.0 / nb : 0.0;
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes:
// h = h1 + h2, h_{j+1,j} = sqrt(<w,w> - |h2|^2); apply the previous
// rotations, form the new one, update g, and the scale of the next basis
// vector (0 once the instance has stopped).  qs: a copy of the slots below
// InnerSlots::Y (in LDS) for the reads; results go to q.  An instance stops
// when the new direction is lost: h_{j+1,j} = 0, or <w,w> - |h2|^2 within
// 1e-12 <w,w> of cancelling (then fewer than ~6 digits of h_{j+1,j} would
// be left, and the next basis vector would be scaled by a wrong 1/h_{j+1,j}),
// or its residual estimate |g_{j+1}| has reached rtol * beta.
__device__ void gmres_givens(double* q, const double* qs, int j, const double* h2, double ww, double rtol,
                             unsigned* counters, bool one_pass) {
  if (qs[S::ACTIVE] == 0.0) {
    q[S::INV] = 0.0;
    return;
  }
  if (counters) atomicAdd(&counters[0], 1u);
  double col[KMAX + 1];
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) {
    q[S::H2 + i] = h2[i];
    col[i] = (one_pass ? 0.0 : qs[S::H1 + i]) + h2[i];
    h2sq += h2[i] * h2[i];
  }
  const double nrm2 = ww - h2sq;
  const double hn = nrm2 > 1e-12 * ww ? sqrt(nrm2) : 0.0;
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = qs[S::CS + i], s = qs[S::SN + i];
    const double a = col[i], b = col[i + 1];
    col[i] = c * a + s * b;
    col[i + 1] = -s * a + c * b;
  }
  const double rho = sqrt(col[j] * col[j] + col[j + 1] * col[j + 1]);
  if (!(rho > 0.0) || !isfinite(rho)) {   // no new direction: stop with m = j
    q[S::ACTIVE] = 0.0;
    q[S::INV] = 0.0;
    return;
  }
  const double c = col[j] / rho, s = col[j + 1] / rho;
  q[S::CS + j] = c;
  q[S::SN + j] = s;
  col[j] = rho;
  for (int i = 0; i <= j; ++i) q[S::R + j * (KMAX + 1) + i] = col[i];
  const double gj = qs[S::G + j];
  q[S::G + j] = c * gj;
  q[S::G + j + 1] = -s * gj;
  q[S::M] = (double)(j + 1);
  if (!(hn > 0.0) || fabs(s * gj) <= rtol * qs[S::BETA]) {   // breakdown, or converged
    q[S::ACTIVE] = 0.0;
    q[S::INV] = 0.0;
  } else {
    q[S::INV] = 1.0 / hn;
  }
}

// One inner GMRES iteration from zero is a minimal-residual step: with
// z = P_R^{-1} r and w = Theta_hat z, x = alpha z, alpha = <w, r> / <w, w>
// (the least-squares solution of GMRES(1), without forming the normalized
// basis vector).  alpha goes to slots[Y].
__device__ void mr_step(double* q, double wr, double ww, unsigned* counters) {
  const bool ok = ww > 0.0 && isfinite(ww);
  if (counters) {
    atomicAdd(&counters[1], 1u);
    if (ok) atomicAdd(&counters[0], 1u);
  }
  q[S::Y] = ok ? wr / ww : 0.0;
}

// One pass of Gram-Schmidt on every instance; block partials of the dot
// products go to `partial` and k_gs_finish completes them.  Optionally:
//   axpy:  w <- w - sum_{d<nd} slots[ca+d] V_d   (stored back to w)
//   dots:  slots[od+d] = <w, V_d>,  self: slots[os] = <w, w>
//   post:  GS_POST_INIT   -> GMRES start  (beta, g, 1/beta) from slots[os]
//          GS_POST_GIVENS -> Givens update of column j (slots hold h1 at H1,
//                            h2 at H2, <w,w> at WW)
//          GS_POST_MR     -> minimal-residual step: slots[Y] = <w,V_0> / <w,w>
// The block partials are summed in a fixed order, so results are bitwise
// reproducible run to run.
template <class TW, class TV, int ND>
__global__ __launch_bounds__(TPB) void k_gs(TW* __restrict__ w, const TV* __restrict__ V, GSArgs a) {
  // ND (a power of two >= nd) bounds the unrolled dot loops at compile time;
  // slot d of the block partials keeps its place, <w,w> stays at DOTS_PER_PASS.
  using C = typename Acc<TW>::type;
  const int inst = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  TW* wi = w + (int64_t)inst * a.sw;
  const TV* Vi = V + (int64_t)inst * a.sv;
  double* q = a.slots + (int64_t)inst * a.sstride;
  C cf[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) cf[d] = (a.axpy && d < a.nd) ? (C)q[a.ca + d] : C(0);
  double acc[ND + 1];
#pragma unroll
  for (int d = 0; d <= ND; ++d) acc[d] = 0.0;
  for (int64_t idx = (int64_t)blk * TPB + tid; idx < a.L; idx += (int64_t)a.nblk * TPB) {
    C wv = ld<TW, C>(wi + idx);
    C vv[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d)
      vv[d] = (d < a.nd) ? ld<TV, C>(Vi + d * a.vstride + idx) : C(0);
    if (a.axpy) {
#pragma unroll
      for (int d = 0; d < ND; ++d) wv -= cf[d] * vv[d];
      st<TW, C>(wi + idx, wv);
    }
    const double wd = (double)wv;
    if (a.dots) {
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[d] += (double)vv[d] * wd;
    }
    acc[ND] += wd * wd;
  }
  if (!a.dots && !a.self) return;
  __shared__ double red[TPB / 64][ND + 1];
  const int lane = tid & 63, wave = tid >> 6;
  const int nslots_used = a.dots ? a.nd : 0;
#pragma unroll
  for (int d = 0; d <= ND; ++d) {
    if (d < nslots_used || (d == ND && a.self)) {
      const double v = wave_sum(acc[d]);
      if (lane == 0) red[wave][d] = v;
    }
  }
  __syncthreads();
  double* part = a.partial + ((int64_t)inst * a.nblk) * NSLOT;
  if (tid <= ND) {
    const int d = tid;
    if (d < nslots_used || (d == ND && a.self)) {
      double sum = 0.0;
      for (int r = 0; r < TPB / 64; ++r) sum += red[r][d];
      part[(int64_t)blk * NSLOT + (d == ND ? DOTS_PER_PASS : d)] = sum;
    }
  }
}

// One pass over a chunk of the basis for the Gram-matrix form of classical
// Gram-Schmidt: block partials of <w, V_d> (slot d), <vlast, V_d> (slot
// nd + d, the newest basis vector's Gram column) and <w, w>; k_gs_finish with
// 2 nd dots completes them into slots[od ..].  nd <= DOTS_PER_PASS / 2.
template <class TW, class TV, int ND>
__global__ __launch_bounds__(TPB) void k_gs_gram(const TW* __restrict__ w, const TV* __restrict__ V,
                                                 const TV* __restrict__ vlast, GSArgs a) {
  const int blk = blockIdx.x, tid = threadIdx.x;
  double acc[ND], accg[ND], self = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = accg[d] = 0.0;
  for (int64_t idx = (int64_t)blk * TPB + tid; idx < a.L; idx += (int64_t)a.nblk * TPB) {
    const double wv = (double)w[idx], lv = (double)vlast[idx];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double vv = d < a.nd ? (double)V[d * a.vstride + idx] : 0.0;
      acc[d] += vv * wv;
      accg[d] += vv * lv;
    }
    self += wv * wv;
  }
  __shared__ double red[TPB / 64][2 * ND + 1];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    if (d < a.nd) {
      const double v1 = wave_sum(acc[d]), v2 = wave_sum(accg[d]);
      if (lane == 0) {
        red[wave][d] = v1;
        red[wave][ND + d] = v2;
      }
    }
  }
  const double vs = wave_sum(self);
  if (lane == 0) red[wave][2 * ND] = vs;
  __syncthreads();
  double* part = a.partial + (int64_t)blk * NSLOT;
  if (tid < 2 * ND + 1) {
    const int e = tid;
    const bool used = e == 2 * ND ? a.self != 0 : (e % ND) < a.nd;
    if (used) {
      double sum = 0.0;
      for (int r = 0; r < TPB / 64; ++r) sum += red[r][e];
      const int slot = e == 2 * ND ? DOTS_PER_PASS : (e < ND ? e : a.nd + (e - ND));
      part[slot] = sum;
    }
  }
}

// Second pass of a Gram-Schmidt reduction: one workgroup per instance sums
// the block partials in a fixed order (thread t takes blocks t, t+TPB, ...,
// then a tree), stores the results and runs the GMRES scalar update.  All
// partial loads of a thread are independent (slots unrolled inside the block
// loop), and the slots the update reads are staged in LDS meanwhile.
template <int ND>
__global__ __launch_bounds__(TPB) void k_gs_finish(GSArgs a) {
  const int inst = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  double* q = a.slots + (int64_t)inst * a.sstride;
  const double* part = a.partial + ((int64_t)inst * a.nblk) * NSLOT;
  const int nsd = a.dots ? a.nd : 0;
  __shared__ double red[TPB / 64][ND + 1];
  __shared__ double fin[NSLOT];
  __shared__ double qs[S::Y];
  if (a.post == GS_POST_GIVENS)
    for (int i = tid; i < S::Y; i += TPB) qs[i] = q[i];
  double acc[ND + 1];
#pragma unroll
  for (int d = 0; d <= ND; ++d) acc[d] = 0.0;
  for (int b = tid; b < a.nblk; b += TPB) {
    const double* pb = part + (int64_t)b * NSLOT;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nsd) acc[d] += pb[d];
    if (a.self) acc[ND] += pb[DOTS_PER_PASS];
  }
#pragma unroll
  for (int d = 0; d <= ND; ++d) {
    if (d < nsd || (d == ND && a.self)) {
      const double v = wave_sum(acc[d]);
      if (lane == 0) red[wave][d] = v;
    }
  }
  __syncthreads();
  if (tid <= ND) {
    const int d = tid;
    if (d < nsd || (d == ND && a.self)) {
      double sum = 0.0;
      for (int r = 0; r < TPB / 64; ++r) sum += red[r][d];
      if (d < nsd) {
        fin[d] = sum;
        q[a.od + d] = sum;
      } else {
        fin[DOTS_PER_PASS] = sum;
        q[a.os] = sum;
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (a.post == GS_POST_INIT) gmres_start(q, fin[DOTS_PER_PASS], a.counters);
    else if (a.post == GS_POST_GIVENS)
      gmres_givens(q, qs, a.j, fin, fin[DOTS_PER_PASS], a.rtol, a.counters, a.one_pass != 0);
    else if (a.post == GS_POST_MR) mr_step(q, fin[0], fin[DOTS_PER_PASS], a.counters);
  }
}

// out = (w - sum_{d<nd} slots[ca+d] V_d) * scale, scale = slots[cs] (cs >= 0) or `alpha`.
template <class TW, class TV, class TO, int ND>
__global__ __launch_bounds__(TPB) void k_basis(const TW* __restrict__ w, int64_t sw, const TV* __restrict__ V,
                                               int64_t vstride, int64_t sv, int nd, TO* __restrict__ out,
                                               int64_t so, const double* __restrict__ slots, int64_t sstride,
                                               int ca, int cs, double alpha, int64_t L, int nblk) {
  using C = typename Acc<TO>::type;
  const int inst = blockIdx.y;
  const double* q = slots + (int64_t)inst * sstride;
  C cf[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) cf[d] = d < nd ? (C)q[ca + d] : C(0);
  const C sc = (C)(cs >= 0 ? q[cs] : alpha);
  const TW* wi = w + (int64_t)inst * sw;
  const TV* Vi = V + (int64_t)inst * sv;
  TO* oi = out + (int64_t)inst * so;
  for (int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x; idx < L; idx += (int64_t)nblk * TPB) {
    C acc = ld<TW, C>(wi + idx);
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nd) acc -= cf[d] * ld<TV, C>(Vi + d * vstride + idx);
    st<TO, C>(oi + idx, acc * sc);
  }
}

// out (+)= sum_{d<nd} y_d Z_d.  With `solve`, y is the GMRES least-squares
// solution R y = g of the instance, recomputed by every workgroup from its
// slots (at most KMAX unknowns); otherwise y = slots[cy + d].
template <class TO, class TV, int ND>
__global__ __launch_bounds__(TPB) void k_combine(TO* __restrict__ out, int64_t so, const TV* __restrict__ Z,
                                                 int64_t vstride, int64_t sv, int nd,
                                                 const double* __restrict__ slots, int64_t sstride, int cy,
                                                 int solve, int accumulate, int64_t L, int nblk) {
  using C = typename Acc<TO>::type;
  const int inst = blockIdx.y;
  const double* q = slots + (int64_t)inst * sstride;
  __shared__ double ys[DOTS_PER_PASS];
  if (threadIdx.x == 0) {
    if (solve) {
      const int m = (int)q[InnerSlots::M];
      for (int i = 0; i < DOTS_PER_PASS; ++i) ys[i] = 0.0;
      for (int i = m - 1; i >= 0; --i) {
        double acc = q[InnerSlots::G + i];
        for (int jj = i + 1; jj < m; ++jj) acc -= q[InnerSlots::R + jj * (KMAX + 1) + i] * ys[jj];
        ys[i] = acc / q[InnerSlots::R + i * (KMAX + 1) + i];
      }
    } else {
      for (int i = 0; i < DOTS_PER_PASS; ++i) ys[i] = i < nd ? q[cy + i] : 0.0;
    }
  }
  __syncthreads();
  C cf[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) cf[d] = (C)ys[d];
  TO* oi = out + (int64_t)inst * so;
  const TV* Zi = Z + (int64_t)inst * sv;
  for (int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x; idx < L; idx += (int64_t)nblk * TPB) {
    C acc = accumulate ? ld<TO, C>(oi + idx) : C(0);
#pragma unroll
    for (int d = 0; d < ND; ++d)
      if (d < nd) acc += cf[d] * ld<TV, C>(Zi + d * vstride + idx);
    st<TO, C>(oi + idx, acc);
  }
}

// ---------------------------------------------------------------------------
// Stage operators
// ---------------------------------------------------------------------------
// w_r = z_r + tau sum_q A[r][q] K z_q   (Theta_hat = I_s (x) I + tau A (x) K)
template <int DIM, int NS, bool VK, class T>
__global__ __launch_bounds__(TPB) void k_theta_apply(const T* __restrict__ z, int64_t sz, T* __restrict__ w,
                                                     int64_t sw, int n, int N, typename Acc<T>::type ih2,
                                                     Tab tab, Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t inst = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const T* zi = z + inst * sz;
  T* wi = w + inst * sw;
  C KZ[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) KZ[q] = ih2 * stencil_K<DIM, VK, T, C>(zi + (int64_t)q * N, p, i, j, k, n, N, fc);
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    C mix = C(0);
#pragma unroll
    for (int q = 0; q < NS; ++q) mix += (C)tab.A[r * NS + q] * KZ[q];
    st<T, C>(wi + (int64_t)r * N + p, ld<T, C>(zi + (int64_t)r * N + p) + (C)tab.tau * mix);
  }
}

// out = v_i - tau sum_{l<i} Lc[i][l] K z_l
template <int DIM, bool VK, class T>
__global__ __launch_bounds__(TPB) void k_rana_rhs(const T* __restrict__ v, int64_t sv, const T* __restrict__ z,
                                                  int64_t sz, T* __restrict__ out, int64_t so, int n, int N,
                                                  typename Acc<T>::type ih2, int stage, int ns, Tab tab,
                                                  Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t inst = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const T* zi = z + inst * sz;
  C acc = ld<T, C>(v + inst * sv + p);
  for (int l = 0; l < stage; ++l)
    acc -= (C)(tab.tau * tab.L[stage * ns + l]) * ih2 *
           stencil_K<DIM, VK, T, C>(zi + (int64_t)l * N, p, i, j, k, n, N, fc);
  st<T, C>(out + inst * so + p, acc);
}

// t_{v,0} = r_{v,0};  t_{v,n+1} = r_{v,n+1} + tau sum_i b_i z_{V,n,i}
template <class T>
__global__ __launch_bounds__(TPB) void k_schur_coupling(const double* __restrict__ r, const T* __restrict__ zV,
                                                        T* __restrict__ t, int N, int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int step = blockIdx.y;   // 0..nt
  const int64_t NN = N;
  double acc = r[(int64_t)step * NN + p];
  if (step > 0) {
    const T* zs = zV + (int64_t)(step - 1) * ns * NN;
    for (int q = 0; q < ns; ++q) acc += tab.tau * tab.b[q] * ld<T, double>(zs + q * NN + p);
  }
  st<T, C>(t + (int64_t)step * NN + p, (C)acc);
}

// S-tilde steps on B instances b (blockIdx.y) at once.  Instance b reads
// its block at base + b * stride for every operand; strides may be negative
// (the transposed sweep walks backwards in time).

// out_{b,i} = K zin_b for every stage i (right-hand side (e (x) K) z of X-tilde)
template <int DIM, bool VK, class T>
__global__ __launch_bounds__(TPB) void k_schur_kz(const T* __restrict__ zin, int64_t szin, T* __restrict__ out,
                                                  int64_t sout, int n, int N, int ns, typename Acc<T>::type ih2,
                                                  Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t b = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const C kz = ih2 * stencil_K<DIM, VK, T, C>(zin + b * szin, p, i, j, k, n, N, fc);
  T* o = out + b * sout;
  for (int q = 0; q < ns; ++q) st<T, C>(o + (int64_t)q * N + p, kz);
}

// out_b = t_b + Phi(zin_b) = t_b + zin_b - tau sum_i b_i y_{b,i}   (y = Theta-tilde^{-1} rhs)
// out may alias t or zin (element-wise).
template <class T, class TT>
__global__ __launch_bounds__(TPB) void k_phi_update(const TT* t, int64_t stt, const T* zin, int64_t szin,
                                                    const T* __restrict__ y, int64_t sy, T* out, int64_t sout, int N,
                                                    int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t b = blockIdx.y;
  const T* yb = y + b * sy;
  C acc = ld<TT, C>(t + b * stt + p) + ld<T, C>(zin + b * szin + p);
  for (int q = 0; q < ns; ++q) acc -= (C)(tab.tau * tab.b[q]) * ld<T, C>(yb + (int64_t)q * N + p);
  st<T, C>(out + b * sout + p, acc);
}

// out_{b,i} = b_i zin_b   (right-hand side (b (x) I) z of the transposed X-tilde)
template <class T>
__global__ __launch_bounds__(TPB) void k_schurT_bw(const T* __restrict__ zin, int64_t szin, T* __restrict__ out,
                                                   int64_t sout, int N, int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t b = blockIdx.y;
  const C v = ld<T, C>(zin + b * szin + p);
  T* o = out + b * sout;
  for (int q = 0; q < ns; ++q) st<T, C>(o + (int64_t)q * N + p, (C)tab.b[q] * v);
}

// out_b = t_b + Phi^T(zin_b) = t_b + zin_b - tau K sum_i y_{b,i}
template <int DIM, bool VK, class T, class TT>
__global__ __launch_bounds__(TPB) void k_phiT_update(const TT* t, int64_t stt, const T* zin, int64_t szin,
                                                     const T* __restrict__ y, int64_t sy, T* out, int64_t sout, int n,
                                                     int N, int ns, typename Acc<T>::type ih2, double tau,
                                                     Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t b = blockIdx.y;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const T* yb = y + b * sy;
  C ky = C(0);
  for (int q = 0; q < ns; ++q) ky += stencil_K<DIM, VK, T, C>(yb + (int64_t)q * N, p, i, j, k, n, N, fc);
  st<T, C>(out + b * sout + p, ld<TT, C>(t + b * stt + p) + ld<T, C>(zin + b * szin + p) - (C)tau * ih2 * ky);
}

// MGRIT coarse-grid step at one C-point: znew = g + Phi_c(e_prev) (Phi_c = 0
// when e_prev is null), e_out = znew - zC, zC = znew.  Phi_c is the step with
// tau_c (forward: e - tau_c b^T y; transposed: e - tau_c K sum_i y_i).
template <int DIM, bool VK, bool TR, class T>
__global__ __launch_bounds__(TPB) void k_mgrit_coarse(const T* __restrict__ g, const T* __restrict__ eprev,
                                                      const T* __restrict__ y, T* __restrict__ zC,
                                                      T* __restrict__ eout, int n, int N, int ns,
                                                      typename Acc<T>::type ih2, Tab tabc,
                                                      Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  C znew = ld<T, C>(g + p);
  if (eprev) {
    C ph = ld<T, C>(eprev + p);
    if (TR) {
      int i, j, k;
      node_coords<DIM>(p, n, i, j, k);
      C ky = C(0);
      for (int q = 0; q < ns; ++q) ky += stencil_K<DIM, VK, T, C>(y + (int64_t)q * N, p, i, j, k, n, N, fc);
      ph -= (C)tabc.tau * ih2 * ky;
    } else {
      for (int q = 0; q < ns; ++q) ph -= (C)(tabc.tau * tabc.b[q]) * ld<T, C>(y + (int64_t)q * N + p);
    }
    znew += ph;
  }
  const C zold = ld<T, C>(zC + p);
  st<T, C>(eout + p, znew - zold);
  st<T, C>(zC + p, znew);
}

// out_{n,i} = r_{V,n,i} + tau b_i z_{v,n+1}
template <class T>
__global__ __launch_bounds__(TPB) void k_thetaT_rhs(const double* __restrict__ r, const T* __restrict__ z,
                                                    T* __restrict__ out, int N, int nt, int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int step = blockIdx.y;
  const int64_t NN = N;
  const double zn = ld<T, double>(z + (int64_t)(step + 1) * NN + p);
  const double* rV = r + ((int64_t)(nt + 1) + (int64_t)step * ns) * NN;
  T* o = out + (int64_t)step * ns * NN;
  for (int q = 0; q < ns; ++q) st<T, C>(o + q * NN + p, (C)(rV[q * NN + p] + tab.tau * tab.b[q] * zn));
}

// Dot-loop bound of a Krylov pass: the smallest of 1, 2, 4, 8, 16 that
// covers nd basis vectors.
#define DISPATCH_ND(nd, M)         \
  do {                             \
    if ((nd) <= 1) M(1);           \
    else if ((nd) <= 2) M(2);      \
    else if ((nd) <= 4) M(4);      \
    else if ((nd) <= 8) M(8);      \
    else M(DOTS_PER_PASS);         \
  } while (0)

inline dim3 seg_grid(int nblk, int B) { return dim3((unsigned)nblk, (unsigned)B); }
inline dim3 pts_grid(int64_t N, int B) { return dim3((unsigned)((N + TPB - 1) / TPB), (unsigned)B); }

template <class C>
Faces<C> faces_of(const aao_problem* h) {
  Faces<C> f{};
  if (h->vark) {
    const bool dbl = sizeof(C) == 8;
    const C* base = reinterpret_cast<const C*>(h->ws + (dbl ? h->plan.faces_d : h->plan.faces_f));
    for (int a = 0; a < h->dim; ++a) {
      f.m[a] = base + (2 * a) * h->N;
      f.p[a] = base + (2 * a + 1) * h->N;
    }
  }
  return f;
}

}  // namespace

int seg_blocks(int64_t L, int B) {
  int64_t want = (L + TPB * 4 - 1) / (TPB * 4);
  int64_t cap = B >= 2048 ? 1 : 2048 / B;
  if (want > cap) want = cap;
  return (int)(want < 1 ? 1 : want);
}

template <class TW, class TV>
hipError_t gs_pass(TW* w, const TV* V, const GSArgs& a, int B, hipStream_t st) {
#define AAO_GS(ND) hipLaunchKernelGGL((k_gs<TW, TV, ND>), seg_grid(a.nblk, B), dim3(TPB), 0, st, w, V, a)
  DISPATCH_ND(a.nd, AAO_GS);
#undef AAO_GS
  if (a.dots || a.self) {
#define AAO_GSF(ND) hipLaunchKernelGGL((k_gs_finish<ND>), dim3((unsigned)B), dim3(TPB), 0, st, a)
    DISPATCH_ND(a.dots ? a.nd : 0, AAO_GSF);
#undef AAO_GSF
  }
  return hipGetLastError();
}

hipError_t gs_gram(const double* w, const double* V, const double* vlast, const GSArgs& a, hipStream_t st) {
  if (a.nd < 1 || 2 * a.nd > DOTS_PER_PASS) return hipErrorInvalidValue;
#define AAO_GG(ND) hipLaunchKernelGGL((k_gs_gram<double, double, ND>), seg_grid(a.nblk, 1), dim3(TPB), 0, st, w, V, vlast, a)
  if (a.nd <= 1) AAO_GG(1);
  else if (a.nd <= 2) AAO_GG(2);
  else if (a.nd <= 4) AAO_GG(4);
  else AAO_GG(8);
#undef AAO_GG
  GSArgs f = a;
  f.dots = 1;
  f.nd = 2 * a.nd;
#define AAO_GSF(ND) hipLaunchKernelGGL((k_gs_finish<ND>), dim3(1u), dim3(TPB), 0, st, f)
  DISPATCH_ND(f.nd, AAO_GSF);
#undef AAO_GSF
  return hipGetLastError();
}

template <class TW, class TV, class TO>
hipError_t basis_update(const TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, TO* out,
                        int64_t so, const double* slots, int64_t sstride, int ca, int cs, double alpha, int64_t L,
                        int B, hipStream_t st) {
  const int nblk = seg_blocks(L, B);
#define AAO_BASIS(ND)                                                                                     \
  hipLaunchKernelGGL((k_basis<TW, TV, TO, ND>), seg_grid(nblk, B), dim3(TPB), 0, st, w, sw, V, vstride, sv, nd, \
                     out, so, slots, sstride, ca, cs, alpha, L, nblk)
  DISPATCH_ND(nd, AAO_BASIS);
#undef AAO_BASIS
  return hipGetLastError();
}

template <class TO, class TV>
hipError_t combine(TO* out, int64_t so, const TV* Z, int64_t vstride, int64_t sv, int nd, const double* slots,
                   int64_t sstride, int cy, bool solve, bool accumulate, int64_t L, int B, hipStream_t st) {
  const int nblk = seg_blocks(L, B);
#define AAO_COMB(ND)                                                                                         \
  hipLaunchKernelGGL((k_combine<TO, TV, ND>), seg_grid(nblk, B), dim3(TPB), 0, st, out, so, Z, vstride, sv, nd, \
                     slots, sstride, cy, (int)solve, (int)accumulate, L, nblk)
  DISPATCH_ND(nd, AAO_COMB);
#undef AAO_COMB
  return hipGetLastError();
}

template <class T>
hipError_t theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                       hipStream_t st) {
  if (h->fe) return fe_theta_apply<T>(h, tab, z, sz, w, sw, B, st);
  using C = typename Acc<T>::type;
  const dim3 g = pts_grid(h->N, B);
  const Faces<C> fc = faces_of<C>(h);
  const int n = h->n, N = (int)h->N;
  const C ih2 = (C)h->ih2;
#define AAO_TH(D, S_, V) \
  hipLaunchKernelGGL((k_theta_apply<D, S_, V, T>), g, dim3(TPB), 0, st, z, sz, w, sw, n, N, ih2, tab, fc)
  DISPATCH_DSV(h->dim, h->s, h->vark, AAO_TH);
#undef AAO_TH
  return hipGetLastError();
}

template <class T>
hipError_t rana_rhs(const aao_problem* h, const double* Lc, int i, const T* v, int64_t sv, const T* z, int64_t sz,
                    T* out, int64_t so, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  Tab tab = h->tab;
  for (int q = 0; q < h->s * h->s; ++q) tab.L[q] = Lc[q];
  if (h->fe) return fe_rana_rhs<T>(h, tab, i, v, sv, z, sz, out, so, B, st);
  const dim3 g = pts_grid(h->N, B);
  const Faces<C> fc = faces_of<C>(h);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
  if (h->dim == 2) {
    if (h->vark) hipLaunchKernelGGL((k_rana_rhs<2, true, T>), g, dim3(TPB), 0, st, v, sv, z, sz, out, so, n, N, ih2, i, ns, tab, fc);
    else hipLaunchKernelGGL((k_rana_rhs<2, false, T>), g, dim3(TPB), 0, st, v, sv, z, sz, out, so, n, N, ih2, i, ns, tab, fc);
  } else {
    if (h->vark) hipLaunchKernelGGL((k_rana_rhs<3, true, T>), g, dim3(TPB), 0, st, v, sv, z, sz, out, so, n, N, ih2, i, ns, tab, fc);
    else hipLaunchKernelGGL((k_rana_rhs<3, false, T>), g, dim3(TPB), 0, st, v, sv, z, sz, out, so, n, N, ih2, i, ns, tab, fc);
  }
  return hipGetLastError();
}

template <class T>
hipError_t schur_coupling(const aao_problem* h, const double* r, const T* zV, T* t, hipStream_t st) {
  if (h->fe) return fe_schur_coupling<T>(h, r, zV, t, st);
  hipLaunchKernelGGL((k_schur_coupling<T>), pts_grid(h->N, h->nt + 1), dim3(TPB), 0, st, r, zV, t, (int)h->N, h->s,
                     h->tab);
  return hipGetLastError();
}

template <class T>
hipError_t schur_kz(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B, hipStream_t st) {
  if (h->fe) return fe_schur_kz<T>(h, zin, szin, out, sout, B, st);
  using C = typename Acc<T>::type;
  const Faces<C> fc = faces_of<C>(h);
  const dim3 g = pts_grid(h->N, B);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
#define AAO_KZ(D, V) \
  hipLaunchKernelGGL((k_schur_kz<D, V, T>), g, dim3(TPB), 0, st, zin, szin, out, sout, n, N, ns, ih2, fc)
  if (h->dim == 2) { if (h->vark) AAO_KZ(2, true); else AAO_KZ(2, false); }
  else { if (h->vark) AAO_KZ(3, true); else AAO_KZ(3, false); }
#undef AAO_KZ
  return hipGetLastError();
}

template <class T, class TT>
hipError_t phi_update(const aao_problem* h, const Tab& tab, const TT* t, int64_t stt, const T* zin, int64_t szin,
                      const T* y, int64_t sy, T* out, int64_t sout, int B, hipStream_t st) {
  hipLaunchKernelGGL((k_phi_update<T, TT>), pts_grid(h->N, B), dim3(TPB), 0, st, t, stt, zin, szin, y, sy, out, sout,
                     (int)h->N, h->s, tab);
  return hipGetLastError();
}

template <class T>
hipError_t schurT_bw(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B, hipStream_t st) {
  hipLaunchKernelGGL((k_schurT_bw<T>), pts_grid(h->N, B), dim3(TPB), 0, st, zin, szin, out, sout, (int)h->N, h->s,
                     h->tab);
  return hipGetLastError();
}

template <class T, class TT>
hipError_t phiT_update(const aao_problem* h, double tau, const TT* t, int64_t stt, const T* zin, int64_t szin,
                       const T* y, int64_t sy, T* out, int64_t sout, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  const Faces<C> fc = faces_of<C>(h);
  const dim3 g = pts_grid(h->N, B);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
#define AAO_PT(D, V)                                                                                           \
  hipLaunchKernelGGL((k_phiT_update<D, V, T, TT>), g, dim3(TPB), 0, st, t, stt, zin, szin, y, sy, out, sout, n, N, \
                     ns, ih2, tau, fc)
  if (h->dim == 2) { if (h->vark) AAO_PT(2, true); else AAO_PT(2, false); }
  else { if (h->vark) AAO_PT(3, true); else AAO_PT(3, false); }
#undef AAO_PT
  return hipGetLastError();
}

template <class T>
hipError_t mgrit_coarse(const aao_problem* h, const Tab& tabc, bool transpose, const T* g, const T* eprev,
                        const T* y, T* zC, T* eout, hipStream_t st) {
  using C = typename Acc<T>::type;
  const Faces<C> fc = faces_of<C>(h);
  const dim3 gr = pts_grid(h->N, 1);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
#define AAO_MC(D, V, TR) \
  hipLaunchKernelGGL((k_mgrit_coarse<D, V, TR, T>), gr, dim3(TPB), 0, st, g, eprev, y, zC, eout, n, N, ns, ih2, tabc, fc)
#define AAO_MC_T(D, V) do { if (transpose) AAO_MC(D, V, true); else AAO_MC(D, V, false); } while (0)
  if (h->dim == 2) { if (h->vark) AAO_MC_T(2, true); else AAO_MC_T(2, false); }
  else { if (h->vark) AAO_MC_T(3, true); else AAO_MC_T(3, false); }
#undef AAO_MC_T
#undef AAO_MC
  return hipGetLastError();
}

template <class T>
hipError_t thetaT_rhs(const aao_problem* h, const double* r, const T* z, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_thetaT_rhs<T>), pts_grid(h->N, h->nt), dim3(TPB), 0, st, r, z, out, (int)h->N, h->nt, h->s,
                     h->tab);
  return hipGetLastError();
}

// explicit instantiations
#define AAO_INST_T(T)                                                                                             \
  template hipError_t gs_pass<T, T>(T*, const T*, const GSArgs&, int, hipStream_t);                                \
  template hipError_t basis_update<T, T, T>(const T*, int64_t, const T*, int64_t, int64_t, int, T*, int64_t,       \
                                            const double*, int64_t, int, int, double, int64_t, int, hipStream_t);  \
  template hipError_t combine<T, T>(T*, int64_t, const T*, int64_t, int64_t, int, const double*, int64_t, int,     \
                                    bool, bool, int64_t, int, hipStream_t);                                        \
  template hipError_t theta_apply<T>(const aao_problem*, const Tab&, const T*, int64_t, T*, int64_t, int,          \
                                     hipStream_t);                                                                 \
  template hipError_t rana_rhs<T>(const aao_problem*, const double*, int, const T*, int64_t, const T*, int64_t, T*, \
                                  int64_t, int, hipStream_t);                                                      \
  template hipError_t schur_coupling<T>(const aao_problem*, const double*, const T*, T*, hipStream_t);             \
  template hipError_t schur_kz<T>(const aao_problem*, const T*, int64_t, T*, int64_t, int, hipStream_t);           \
  template hipError_t phi_update<T, T>(const aao_problem*, const Tab&, const T*, int64_t, const T*, int64_t,       \
                                       const T*, int64_t, T*, int64_t, int, hipStream_t);                         \
  template hipError_t schurT_bw<T>(const aao_problem*, const T*, int64_t, T*, int64_t, int, hipStream_t);          \
  template hipError_t phiT_update<T, T>(const aao_problem*, double, const T*, int64_t, const T*, int64_t,          \
                                        const T*, int64_t, T*, int64_t, int, hipStream_t);                        \
  template hipError_t mgrit_coarse<T>(const aao_problem*, const Tab&, bool, const T*, const T*, const T*, T*, T*,  \
                                      hipStream_t);                                                               \
  template hipError_t thetaT_rhs<T>(const aao_problem*, const double*, const T*, T*, hipStream_t);

AAO_INST_T(double)
AAO_INST_T(float)
AAO_INST_T(__half)
template hipError_t phi_update<__half, double>(const aao_problem*, const Tab&, const double*, int64_t, const __half*,
                                               int64_t, const __half*, int64_t, __half*, int64_t, int, hipStream_t);
template hipError_t phiT_update<__half, double>(const aao_problem*, double, const double*, int64_t, const __half*,
                                                int64_t, const __half*, int64_t, __half*, int64_t, int, hipStream_t);
template hipError_t gs_pass<double, __half>(double*, const __half*, const GSArgs&, int, hipStream_t);
template hipError_t basis_update<double, __half, __half>(const double*, int64_t, const __half*, int64_t, int64_t,
                                                         int, __half*, int64_t, const double*, int64_t, int, int,
                                                         double, int64_t, int, hipStream_t);
template hipError_t combine<double, __half>(double*, int64_t, const __half*, int64_t, int64_t, int, const double*,
                                            int64_t, int, bool, bool, int64_t, int, hipStream_t);
template hipError_t phi_update<float, double>(const aao_problem*, const Tab&, const double*, int64_t, const float*,
                                              int64_t, const float*, int64_t, float*, int64_t, int, hipStream_t);
template hipError_t phiT_update<float, double>(const aao_problem*, double, const double*, int64_t, const float*,
                                               int64_t, const float*, int64_t, float*, int64_t, int, hipStream_t);
template hipError_t gs_pass<double, float>(double*, const float*, const GSArgs&, int, hipStream_t);
template hipError_t basis_update<double, float, float>(const double*, int64_t, const float*, int64_t, int64_t, int,
                                                       float*, int64_t, const double*, int64_t, int, int, double,
                                                       int64_t, int, hipStream_t);
template hipError_t combine<double, float>(double*, int64_t, const float*, int64_t, int64_t, int, const double*,
                                           int64_t, int, bool, bool, int64_t, int, hipStream_t);

}  // namespace aao

// Batched Krylov kernels: segmented dot products (wave64 shuffles, LDS, and a
// fixed-order second pass, so results are bitwise reproducible), multi-AXPYs,
// the Givens update of GMRES on device, and the stage-level operators used by
// the preconditioner (Theta_hat, Rana coupling, S-tilde sweep pieces).
#include "aao_internal.h"
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

template <class TW, class TV>
__global__ __launch_bounds__(TPB) void k_seg_dots(const TW* __restrict__ w, int64_t sw,
                                                  const TV* __restrict__ V, int64_t vstride, int64_t sv,
                                                  int nd, int self, int64_t L, double* __restrict__ partial,
                                                  int nblk) {
  const int inst = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const TW* wi = w + (int64_t)inst * sw;
  const TV* Vi = V + (int64_t)inst * sv;
  double acc[NSLOT];
#pragma unroll
  for (int d = 0; d < NSLOT; ++d) acc[d] = 0.0;
  for (int64_t idx = (int64_t)blk * TPB + tid; idx < L; idx += (int64_t)nblk * TPB) {
    const double wv = ld<TW, double>(wi + idx);
#pragma unroll
    for (int d = 0; d < DOTS_PER_PASS; ++d)
      if (d < nd) acc[d] += ld<TV, double>(Vi + d * vstride + idx) * wv;
    acc[DOTS_PER_PASS] += wv * wv;
  }
  __shared__ double red[TPB / 64][NSLOT];
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int d = 0; d < NSLOT; ++d) {
    if (d < nd || (d == DOTS_PER_PASS && self)) {
      const double v = wave_sum(acc[d]);
      if (lane == 0) red[wave][d] = v;
    }
  }
  __syncthreads();
  if (tid < NSLOT) {
    const int d = tid;
    if (d < nd || (d == DOTS_PER_PASS && self)) {
      double s = 0.0;
      for (int q = 0; q < TPB / 64; ++q) s += red[q][d];
      partial[((int64_t)inst * nblk + blk) * NSLOT + d] = s;
    }
  }
}

__global__ void k_seg_finish(const double* __restrict__ partial, int nblk, int nd, int self_off, int B,
                             double* __restrict__ out, int64_t ostride, int ooff) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = nd + (self_off >= 0 ? 1 : 0);
  if (t >= B * per) return;
  const int inst = t / per, d = t - inst * per;
  const int slot = d < nd ? d : DOTS_PER_PASS;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((int64_t)inst * nblk + b) * NSLOT + slot];
  if (d < nd) out[(int64_t)inst * ostride + ooff + d] = s;
  else out[(int64_t)inst * ostride + self_off] = s;
}

template <class TW, class TV>
__global__ __launch_bounds__(TPB) void k_seg_axpy(TW* __restrict__ w, int64_t sw, const TV* __restrict__ V,
                                                  int64_t vstride, int64_t sv, int nd,
                                                  const double* __restrict__ coef, int64_t cstride, int coff,
                                                  double scale, int64_t L, int nblk) {
  using C = typename Acc<TW>::type;
  const int inst = blockIdx.y;
  C cf[DOTS_PER_PASS];
#pragma unroll
  for (int d = 0; d < DOTS_PER_PASS; ++d)
    cf[d] = d < nd ? (C)(scale * coef[(int64_t)inst * cstride + coff + d]) : C(0);
  TW* wi = w + (int64_t)inst * sw;
  const TV* Vi = V + (int64_t)inst * sv;
  for (int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x; idx < L; idx += (int64_t)nblk * TPB) {
    C acc = ld<TW, C>(wi + idx);
#pragma unroll
    for (int d = 0; d < DOTS_PER_PASS; ++d)
      if (d < nd) acc += cf[d] * ld<TV, C>(Vi + d * vstride + idx);
    st<TW, C>(wi + idx, acc);
  }
}

template <class TO, class TV>
__global__ __launch_bounds__(TPB) void k_seg_combine(TO* __restrict__ out, int64_t so, const TV* __restrict__ V,
                                                     int64_t vstride, int64_t sv, int nd,
                                                     const double* __restrict__ coef, int64_t cstride, int coff,
                                                     int64_t L, int nblk) {
  using C = typename Acc<TO>::type;
  const int inst = blockIdx.y;
  C cf[KMAX];
#pragma unroll
  for (int d = 0; d < KMAX; ++d) cf[d] = d < nd ? (C)coef[(int64_t)inst * cstride + coff + d] : C(0);
  TO* oi = out + (int64_t)inst * so;
  const TV* Vi = V + (int64_t)inst * sv;
  for (int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x; idx < L; idx += (int64_t)nblk * TPB) {
    C acc = C(0);
#pragma unroll
    for (int d = 0; d < KMAX; ++d)
      if (d < nd) acc += cf[d] * ld<TV, C>(Vi + d * vstride + idx);
    st<TO, C>(oi + idx, acc);
  }
}

template <class TI, class TO>
__global__ __launch_bounds__(TPB) void k_seg_scale(const TI* __restrict__ in, int64_t si, TO* __restrict__ out,
                                                   int64_t so, const double* __restrict__ sc, int64_t cstride,
                                                   int coff, int64_t L, int nblk) {
  using C = typename Acc<TO>::type;
  const int inst = blockIdx.y;
  const double f = sc[(int64_t)inst * cstride + coff];
  const TI* ii = in + (int64_t)inst * si;
  TO* oi = out + (int64_t)inst * so;
  for (int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x; idx < L; idx += (int64_t)nblk * TPB)
    st<TO, C>(oi + idx, (C)(ld<TI, double>(ii + idx) * f));
}

// ---------------------------------------------------------------------------
// Inner GMRES scalars (one thread per instance)
// ---------------------------------------------------------------------------
using S = InnerSlots;

__global__ void k_inner_init(double* slots, int B) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B) return;
  double* q = slots + (int64_t)inst * S::STRIDE;
  const double beta = q[S::WW];
  const bool ok = beta > 0.0 && isfinite(beta);
  const double nb = ok ? sqrt(beta) : 0.0;
  q[S::BETA] = nb;
  q[S::ACTIVE] = ok ? 1.0 : 0.0;
  q[S::M] = 0.0;
  for (int i = 0; i <= KMAX; ++i) q[S::G + i] = 0.0;
  q[S::G] = nb;
  q[S::INV] = ok ? 1.0 / nb : 0.0;
}

__global__ void k_inner_givens(double* slots, int B, int j) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B) return;
  double* q = slots + (int64_t)inst * S::STRIDE;
  if (q[S::ACTIVE] == 0.0) {
    q[S::INV] = 0.0;
    return;
  }
  double col[KMAX + 1];
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) {
    col[i] = q[S::H1 + i] + q[S::H2 + i];
    h2sq += q[S::H2 + i] * q[S::H2 + i];
  }
  const double nrm2 = q[S::WW] - h2sq;
  const double hn = nrm2 > 0.0 ? sqrt(nrm2) : 0.0;
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = q[S::CS + i], s = q[S::SN + i];
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
  const double gj = q[S::G + j];
  q[S::G + j] = c * gj;
  q[S::G + j + 1] = -s * gj;
  q[S::M] = (double)(j + 1);
  if (!(hn > 0.0)) {                       // exact breakdown: solution in the space
    q[S::ACTIVE] = 0.0;
    q[S::INV] = 0.0;
  } else {
    q[S::INV] = 1.0 / hn;
  }
}

__global__ void k_inner_backsolve(double* slots, int B, int k) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= B) return;
  double* q = slots + (int64_t)inst * S::STRIDE;
  const int m = (int)q[S::M];
  for (int i = 0; i < KMAX; ++i) q[S::Y + i] = 0.0;
  for (int i = m - 1; i >= 0; --i) {
    double acc = q[S::G + i];
    for (int jj = i + 1; jj < m; ++jj) acc -= q[S::R + jj * (KMAX + 1) + i] * q[S::Y + jj];
    q[S::Y + i] = acc / q[S::R + i * (KMAX + 1) + i];
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

// z_{v,0} = r_{v,0};  z_{v,n+1} = r_{v,n+1} + tau sum_i b_i z_{V,n,i}
template <class T>
__global__ __launch_bounds__(TPB) void k_schur_coupling(const double* __restrict__ r, T* __restrict__ z, int N,
                                                        int nt, int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int step = blockIdx.y;   // 0..nt
  const int64_t NN = N;
  double acc = r[(int64_t)step * NN + p];
  if (step > 0) {
    const T* zV = z + ((int64_t)(nt + 1) + (int64_t)(step - 1) * ns) * NN;
    for (int q = 0; q < ns; ++q) acc += tab.tau * tab.b[q] * ld<T, double>(zV + q * NN + p);
  }
  st<T, C>(z + (int64_t)step * NN + p, (C)acc);
}

// out_i = K zv for every stage i (right-hand side e (x) K z of X-tilde)
template <int DIM, bool VK, class T>
__global__ __launch_bounds__(TPB) void k_schur_kz(const T* __restrict__ zv, T* __restrict__ out, int n, int N,
                                                  int ns, typename Acc<T>::type ih2,
                                                  Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  const C kz = ih2 * stencil_K<DIM, VK, T, C>(zv, p, i, j, k, n, N, fc);
  for (int q = 0; q < ns; ++q) st<T, C>(out + (int64_t)q * N + p, kz);
}

// znext = tnext + zcur - tau sum_i b_i y_i
template <class T>
__global__ __launch_bounds__(TPB) void k_schur_update(const T* tnext, const T* __restrict__ zcur,
                                                      const T* __restrict__ y, T* znext, int N, int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  C acc = ld<T, C>(tnext + p) + ld<T, C>(zcur + p);
  for (int q = 0; q < ns; ++q) acc -= (C)(tab.tau * tab.b[q]) * ld<T, C>(y + (int64_t)q * N + p);
  st<T, C>(znext + p, acc);
}

// out_i = b_i w   (right-hand side (b (x) I) w of the transposed X-tilde)
template <class T>
__global__ __launch_bounds__(TPB) void k_schurT_bw(const T* __restrict__ w, T* __restrict__ out, int N, int ns,
                                                   Tab tab) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const C v = ld<T, C>(w + p);
  for (int q = 0; q < ns; ++q) st<T, C>(out + (int64_t)q * N + p, (C)tab.b[q] * v);
}

// zcur = rprev + znext - tau K sum_i y_i
template <int DIM, bool VK, class T>
__global__ __launch_bounds__(TPB) void k_schurT_update(const double* __restrict__ rprev, const T* __restrict__ znext,
                                                       const T* __restrict__ y, T* __restrict__ zcur, int n, int N,
                                                       int ns, typename Acc<T>::type ih2, double tau,
                                                       Faces<typename Acc<T>::type> fc) {
  using C = typename Acc<T>::type;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  int i, j, k;
  node_coords<DIM>(p, n, i, j, k);
  C ky = C(0);
  for (int q = 0; q < ns; ++q) ky += stencil_K<DIM, VK, T, C>(y + (int64_t)q * N, p, i, j, k, n, N, fc);
  st<T, C>(zcur + p, (C)rprev[p] + ld<T, C>(znext + p) - (C)tau * ih2 * ky);
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
hipError_t seg_dots(const TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, bool self,
                    int64_t L, int B, double* partial, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_seg_dots<TW, TV>), seg_grid(nblk, B), dim3(TPB), 0, st, w, sw, V, vstride, sv, nd,
                     (int)self, L, partial, nblk);
  return hipGetLastError();
}

hipError_t seg_finish(const double* partial, int nblk, int nd, int self_off, int B, double* out, int64_t ostride,
                      int ooff, hipStream_t st) {
  const int total = B * (nd + (self_off >= 0 ? 1 : 0));
  hipLaunchKernelGGL(k_seg_finish, dim3((unsigned)((total + 63) / 64)), dim3(64), 0, st, partial, nblk, nd,
                     self_off, B, out, ostride, ooff);
  return hipGetLastError();
}

template <class TW, class TV>
hipError_t seg_axpy(TW* w, int64_t sw, const TV* V, int64_t vstride, int64_t sv, int nd, const double* coef,
                    int64_t cstride, int coff, double scale, int64_t L, int B, hipStream_t st) {
  const int nblk = seg_blocks(L, B);
  hipLaunchKernelGGL((k_seg_axpy<TW, TV>), seg_grid(nblk, B), dim3(TPB), 0, st, w, sw, V, vstride, sv, nd, coef,
                     cstride, coff, scale, L, nblk);
  return hipGetLastError();
}

template <class TO, class TV>
hipError_t seg_combine(TO* out, int64_t so, const TV* V, int64_t vstride, int64_t sv, int nd, const double* coef,
                       int64_t cstride, int coff, int64_t L, int B, hipStream_t st) {
  const int nblk = seg_blocks(L, B);
  hipLaunchKernelGGL((k_seg_combine<TO, TV>), seg_grid(nblk, B), dim3(TPB), 0, st, out, so, V, vstride, sv, nd,
                     coef, cstride, coff, L, nblk);
  return hipGetLastError();
}

template <class TI, class TO>
hipError_t seg_scale(const TI* in, int64_t si, TO* out, int64_t so, const double* sc, int64_t cstride, int coff,
                     int64_t L, int B, hipStream_t st) {
  const int nblk = seg_blocks(L, B);
  hipLaunchKernelGGL((k_seg_scale<TI, TO>), seg_grid(nblk, B), dim3(TPB), 0, st, in, si, out, so, sc, cstride,
                     coff, L, nblk);
  return hipGetLastError();
}

hipError_t inner_init(double* slots, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_init, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, slots, B);
  return hipGetLastError();
}
hipError_t inner_givens(double* slots, int B, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_givens, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, slots, B, j);
  return hipGetLastError();
}
hipError_t inner_backsolve(double* slots, int B, int k, hipStream_t st) {
  hipLaunchKernelGGL(k_inner_backsolve, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, slots, B, k);
  return hipGetLastError();
}

template <class T>
hipError_t theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                       hipStream_t st) {
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
hipError_t schur_coupling(const aao_problem* h, const double* r, T* z, hipStream_t st) {
  hipLaunchKernelGGL((k_schur_coupling<T>), pts_grid(h->N, h->nt + 1), dim3(TPB), 0, st, r, z, (int)h->N, h->nt,
                     h->s, h->tab);
  return hipGetLastError();
}

template <class T>
hipError_t schur_kz(const aao_problem* h, const T* zv, T* out, hipStream_t st) {
  using C = typename Acc<T>::type;
  const Faces<C> fc = faces_of<C>(h);
  const dim3 g = pts_grid(h->N, 1);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
  if (h->dim == 2) {
    if (h->vark) hipLaunchKernelGGL((k_schur_kz<2, true, T>), g, dim3(TPB), 0, st, zv, out, n, N, ns, ih2, fc);
    else hipLaunchKernelGGL((k_schur_kz<2, false, T>), g, dim3(TPB), 0, st, zv, out, n, N, ns, ih2, fc);
  } else {
    if (h->vark) hipLaunchKernelGGL((k_schur_kz<3, true, T>), g, dim3(TPB), 0, st, zv, out, n, N, ns, ih2, fc);
    else hipLaunchKernelGGL((k_schur_kz<3, false, T>), g, dim3(TPB), 0, st, zv, out, n, N, ns, ih2, fc);
  }
  return hipGetLastError();
}

template <class T>
hipError_t schur_update(const aao_problem* h, const T* tnext, const T* zcur, const T* y, T* znext, hipStream_t st) {
  hipLaunchKernelGGL((k_schur_update<T>), pts_grid(h->N, 1), dim3(TPB), 0, st, tnext, zcur, y, znext, (int)h->N,
                     h->s, h->tab);
  return hipGetLastError();
}

template <class T>
hipError_t schurT_bw(const aao_problem* h, const T* zv, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_schurT_bw<T>), pts_grid(h->N, 1), dim3(TPB), 0, st, zv, out, (int)h->N, h->s, h->tab);
  return hipGetLastError();
}

template <class T>
hipError_t schurT_update(const aao_problem* h, const double* rprev, const T* znext, const T* y, T* zcur,
                         hipStream_t st) {
  using C = typename Acc<T>::type;
  const Faces<C> fc = faces_of<C>(h);
  const dim3 g = pts_grid(h->N, 1);
  const int n = h->n, N = (int)h->N, ns = h->s;
  const C ih2 = (C)h->ih2;
  if (h->dim == 2) {
    if (h->vark) hipLaunchKernelGGL((k_schurT_update<2, true, T>), g, dim3(TPB), 0, st, rprev, znext, y, zcur, n, N, ns, ih2, h->tau, fc);
    else hipLaunchKernelGGL((k_schurT_update<2, false, T>), g, dim3(TPB), 0, st, rprev, znext, y, zcur, n, N, ns, ih2, h->tau, fc);
  } else {
    if (h->vark) hipLaunchKernelGGL((k_schurT_update<3, true, T>), g, dim3(TPB), 0, st, rprev, znext, y, zcur, n, N, ns, ih2, h->tau, fc);
    else hipLaunchKernelGGL((k_schurT_update<3, false, T>), g, dim3(TPB), 0, st, rprev, znext, y, zcur, n, N, ns, ih2, h->tau, fc);
  }
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
  template hipError_t seg_dots<T, T>(const T*, int64_t, const T*, int64_t, int64_t, int, bool, int64_t, int,       \
                                     double*, int, hipStream_t);                                                   \
  template hipError_t seg_axpy<T, T>(T*, int64_t, const T*, int64_t, int64_t, int, const double*, int64_t, int,   \
                                     double, int64_t, int, hipStream_t);                                           \
  template hipError_t seg_combine<T, T>(T*, int64_t, const T*, int64_t, int64_t, int, const double*, int64_t, int, \
                                        int64_t, int, hipStream_t);                                                \
  template hipError_t seg_scale<T, T>(const T*, int64_t, T*, int64_t, const double*, int64_t, int, int64_t, int,   \
                                      hipStream_t);                                                                \
  template hipError_t theta_apply<T>(const aao_problem*, const Tab&, const T*, int64_t, T*, int64_t, int,          \
                                     hipStream_t);                                                                 \
  template hipError_t rana_rhs<T>(const aao_problem*, const double*, int, const T*, int64_t, const T*, int64_t, T*, \
                                  int64_t, int, hipStream_t);                                                      \
  template hipError_t schur_coupling<T>(const aao_problem*, const double*, T*, hipStream_t);                       \
  template hipError_t schur_kz<T>(const aao_problem*, const T*, T*, hipStream_t);                                  \
  template hipError_t schur_update<T>(const aao_problem*, const T*, const T*, const T*, T*, hipStream_t);          \
  template hipError_t schurT_bw<T>(const aao_problem*, const T*, T*, hipStream_t);                                 \
  template hipError_t schurT_update<T>(const aao_problem*, const double*, const T*, const T*, T*, hipStream_t);    \
  template hipError_t thetaT_rhs<T>(const aao_problem*, const double*, const T*, T*, hipStream_t);

AAO_INST_T(double)
AAO_INST_T(float)
#define AAO_INST_MIX(T) \
  template hipError_t seg_scale<double, T>(const double*, int64_t, T*, int64_t, const double*, int64_t, int,       \
                                           int64_t, int, hipStream_t);                                             \
  template hipError_t seg_dots<double, T>(const double*, int64_t, const T*, int64_t, int64_t, int, bool, int64_t,  \
                                          int, double*, int, hipStream_t);                                         \
  template hipError_t seg_axpy<double, T>(double*, int64_t, const T*, int64_t, int64_t, int, const double*,        \
                                          int64_t, int, double, int64_t, int, hipStream_t);
AAO_INST_MIX(float)
template hipError_t seg_combine<double, float>(double*, int64_t, const float*, int64_t, int64_t, int,
                                               const double*, int64_t, int, int64_t, int, hipStream_t);
template hipError_t seg_scale<float, double>(const float*, int64_t, double*, int64_t, const double*, int64_t, int,
                                             int64_t, int, hipStream_t);

}  // namespace aao

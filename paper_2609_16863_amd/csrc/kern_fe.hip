// Bilinear (Q1) finite elements on a uniform square grid: the operators of
// the all-at-once system with a mass matrix (Sec. 2, eq. (2.4): Phi with M
// blocks, Psi1 = -(tau b^T (x) M), Theta_hat = I_s (x) M + tau A (x) K) and
// the pieces of P-tilde that meet M or K outside the multigrid: the stage
// operator, Rana's coupling, the Psi1 coupling of S-tilde, the right-hand
// sides e (x) K z of its steps, and its block-diagonal mass solve by
// Chebyshev semi-iteration (Sec. 5: 20 steps with the Jacobi splitting).
//
// On the interior nodes of a uniform grid of spacing h (Dirichlet boundary
// eliminated) the Q1 matrices are tensor products of the 1D ones:
//   M = M1 (x) M1,  K = T (x) M1 + M1 (x) T,
//   M1 = h tridiag(1/6, 2/3, 1/6),  T = tridiag(-1, 2, -1) / h,
// so at a node with neighbours e (edges) and c (corners)
//   (M u)_p = h^2/36 (16 u_p + 4 sum_e u_e + sum_c u_c),
//   (K u)_p = (8 u_p - sum_e u_e - sum_c u_c) / 3        (no h in 2D).
// One thread per node and block; the 3 x 3 neighbourhood is read through
// the caches (these kernels serve the finite-element path, not the
// benchmark's finite-difference one).
#include "aao_internal.h"
#include "fe.h"
#include "krylov.h"

namespace aao {
namespace {

constexpr int TPB = 256;

// Values of the field f on the 3 x 3 neighbourhood of (i, j), zero outside
// the interior grid; v[dj + 1][di + 1].
template <class T, class C>
__device__ __forceinline__ void gather9(const T* __restrict__ f, int i, int j, int n, C v[3][3]) {
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = i + di, jj = j + dj;
      v[dj + 1][di + 1] = (ii >= 0 && ii < n && jj >= 0 && jj < n) ? ld<T, C>(f + ii + (int64_t)jj * n) : C(0);
    }
}

template <class C>
__device__ __forceinline__ C mass9(const C v[3][3], C mh) {
  const C edges = v[0][1] + v[1][0] + v[1][2] + v[2][1];
  const C corners = v[0][0] + v[0][2] + v[2][0] + v[2][2];
  return mh * (C(16) * v[1][1] + C(4) * edges + corners);
}

template <class C>
__device__ __forceinline__ C stiff9(const C v[3][3]) {
  const C ring = v[0][0] + v[0][1] + v[0][2] + v[1][0] + v[1][2] + v[2][0] + v[2][1] + v[2][2];
  return (C(8) * v[1][1] - ring) / C(3);
}

// v += a * w (3 x 3)
template <class C>
__device__ __forceinline__ void axpy9(C v[3][3], C a, const C w[3][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) v[r][q] += a * w[r][q];
}

// y = A x, one block row per blockIdx.y: rows 0..nt are v-rows, then the
// stage rows (m, i) in the layout of eq. (2.4).
template <int S, class TX>
__global__ __launch_bounds__(TPB) void k_fe_apply_A(const TX* __restrict__ x, double* __restrict__ y, int n,
                                                    int nt, double mh, Tab tab) {
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int64_t NN = N;
  const int row = blockIdx.y;
  const TX* V = x + (int64_t)(nt + 1) * NN;
  double acc[3][3], w[3][3];
  if (row <= nt) {
    // M (v_m - v_{m-1} - tau sum_i b_i V_{m-1,i}), or M v_0
    gather9<TX, double>(x + (int64_t)row * NN, i, j, n, acc);
    if (row > 0) {
      gather9<TX, double>(x + (int64_t)(row - 1) * NN, i, j, n, w);
      axpy9<double>(acc, -1.0, w);
      for (int q = 0; q < S; ++q) {
        gather9<TX, double>(V + ((int64_t)(row - 1) * S + q) * NN, i, j, n, w);
        axpy9<double>(acc, -tab.tau * tab.b[q], w);
      }
    }
    y[(int64_t)row * NN + p] = mass9<double>(acc, mh);
    return;
  }
  const int r = row - (nt + 1), m = r / S, st = r - m * S;
  // M V_{m,st} + K (v_m + tau sum_q a_{st,q} V_{m,q})
  double mv[3][3];
  gather9<TX, double>(V + (int64_t)r * NN, i, j, n, mv);
  gather9<TX, double>(x + (int64_t)m * NN, i, j, n, acc);
  for (int q = 0; q < S; ++q) {
    gather9<TX, double>(V + ((int64_t)m * S + q) * NN, i, j, n, w);
    axpy9<double>(acc, tab.tau * tab.A[st * S + q], w);
  }
  y[(int64_t)(nt + 1) * NN + (int64_t)r * NN + p] = mass9<double>(mv, mh) + stiff9<double>(acc);
}

// y = A^T x (M and K symmetric):
//   y_{v,m} = M (x_{v,m} - x_{v,m+1}) + K sum_i x_{V,m,i}  (m < nt),  y_{v,nt} = M x_{v,nt};
//   y_{V,m,st} = M x_{V,m,st} + tau K sum_i a_{i,st} x_{V,m,i} - tau b_st M x_{v,m+1}.
template <int S, class TX>
__global__ __launch_bounds__(TPB) void k_fe_apply_AT(const TX* __restrict__ x, double* __restrict__ y, int n,
                                                     int nt, double mh, Tab tab) {
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int64_t NN = N;
  const int row = blockIdx.y;
  const TX* V = x + (int64_t)(nt + 1) * NN;
  double mv[3][3], kv[3][3], w[3][3];
  if (row <= nt) {
    gather9<TX, double>(x + (int64_t)row * NN, i, j, n, mv);
    double out;
    if (row < nt) {
      gather9<TX, double>(x + (int64_t)(row + 1) * NN, i, j, n, w);
      axpy9<double>(mv, -1.0, w);
      gather9<TX, double>(V + (int64_t)row * S * NN, i, j, n, kv);
      for (int q = 1; q < S; ++q) {
        gather9<TX, double>(V + ((int64_t)row * S + q) * NN, i, j, n, w);
        axpy9<double>(kv, 1.0, w);
      }
      out = mass9<double>(mv, mh) + stiff9<double>(kv);
    } else {
      out = mass9<double>(mv, mh);
    }
    y[(int64_t)row * NN + p] = out;
    return;
  }
  const int r = row - (nt + 1), m = r / S, st = r - m * S;
  gather9<TX, double>(V + (int64_t)r * NN, i, j, n, mv);
  gather9<TX, double>(x + (int64_t)(m + 1) * NN, i, j, n, w);
  axpy9<double>(mv, -tab.tau * tab.b[st], w);
  for (int rr = 0; rr < 3; ++rr)
    for (int qq = 0; qq < 3; ++qq) kv[rr][qq] = 0.0;
  for (int q = 0; q < S; ++q) {
    gather9<TX, double>(V + ((int64_t)m * S + q) * NN, i, j, n, w);
    axpy9<double>(kv, tab.tau * tab.A[q * S + st], w);
  }
  y[(int64_t)(nt + 1) * NN + (int64_t)r * NN + p] = mass9<double>(mv, mh) + stiff9<double>(kv);
}

// w_r = M z_r + tau sum_q A[r][q] K z_q   (Theta_hat), B instances
template <int S, class T>
__global__ __launch_bounds__(TPB) void k_fe_theta(const T* __restrict__ z, int64_t sz, T* __restrict__ w,
                                                  int64_t sw, int n, typename Acc<T>::type mh, Tab tab) {
  using C = typename Acc<T>::type;
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int64_t inst = blockIdx.y;
  const T* zi = z + inst * sz;
  C Mz[S], Kz[S];
#pragma unroll
  for (int q = 0; q < S; ++q) {
    C v[3][3];
    gather9<T, C>(zi + (int64_t)q * N, i, j, n, v);
    Mz[q] = mass9<C>(v, mh);
    Kz[q] = stiff9<C>(v);
  }
#pragma unroll
  for (int r = 0; r < S; ++r) {
    C mix = C(0);
#pragma unroll
    for (int q = 0; q < S; ++q) mix += (C)tab.A[r * S + q] * Kz[q];
    st<T, C>(w + inst * sw + (int64_t)r * N + p, Mz[r] + (C)tab.tau * mix);
  }
}

// out = v - tau sum_{l < stage} Lc[stage][l] K z_l   (Rana's coupling)
template <class T>
__global__ __launch_bounds__(TPB) void k_fe_rana_rhs(const T* __restrict__ v, int64_t sv, const T* __restrict__ z,
                                                     int64_t sz, T* __restrict__ out, int64_t so, int n, int stage,
                                                     int ns, Tab tab) {
  using C = typename Acc<T>::type;
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int64_t inst = blockIdx.y;
  C acc = ld<T, C>(v + inst * sv + p);
  for (int l = 0; l < stage; ++l) {
    C w[3][3];
    gather9<T, C>(z + inst * sz + (int64_t)l * N, i, j, n, w);
    acc -= (C)(tab.tau * tab.L[stage * ns + l]) * stiff9<C>(w);
  }
  st<T, C>(out + inst * so + p, acc);
}

// t_0 = r_0;  t_{m+1} = r_{m+1} + tau M sum_i b_i z_{V,m,i}   (r_v - Psi1 z_V)
template <class T>
__global__ __launch_bounds__(TPB) void k_fe_schur_coupling(const double* __restrict__ r, const T* __restrict__ zV,
                                                           T* __restrict__ t, int n, int ns, double mh, Tab tab) {
  using C = typename Acc<T>::type;
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int step = blockIdx.y;
  const int64_t NN = N;
  double acc = r[(int64_t)step * NN + p];
  if (step > 0) {
    double u[3][3], w[3][3];
    for (int rr = 0; rr < 3; ++rr)
      for (int qq = 0; qq < 3; ++qq) u[rr][qq] = 0.0;
    for (int q = 0; q < ns; ++q) {
      gather9<T, double>(zV + ((int64_t)(step - 1) * ns + q) * NN, i, j, n, w);
      axpy9<double>(u, tab.b[q], w);
    }
    acc += tab.tau * mass9<double>(u, mh);
  }
  st<T, C>(t + (int64_t)step * NN + p, (C)acc);
}

// out_{b,i} = K zin_b for every stage i
template <class T>
__global__ __launch_bounds__(TPB) void k_fe_schur_kz(const T* __restrict__ zin, int64_t szin, T* __restrict__ out,
                                                     int64_t sout, int n, int ns) {
  using C = typename Acc<T>::type;
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  const int64_t b = blockIdx.y;
  C w[3][3];
  gather9<T, C>(zin + b * szin, i, j, n, w);
  const C kz = stiff9<C>(w);
  for (int q = 0; q < ns; ++q) st<T, C>(out + b * sout + (int64_t)q * N + p, kz);
}

// One step of the Chebyshev semi-iteration for M y = t on B blocks:
// out = w (y - yprev + D^{-1} (t - M y) / theta) + yprev, or, on the first
// step, out = D^{-1} t / theta; yprev may be null (a zero y_{k-1}).  out may
// alias t or yprev (each element reads only its own entry of those); it
// never aliases y, whose neighbours other threads read.
template <class T>
__global__ __launch_bounds__(TPB) void k_fe_cheb(const T* t, const T* __restrict__ y, const T* yprev, T* out, int n,
                                                 typename Acc<T>::type mh, typename Acc<T>::type dth,
                                                 typename Acc<T>::type w, int first) {
  using C = typename Acc<T>::type;
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int64_t off = (int64_t)blockIdx.y * N + p;
  const C tv = ld<T, C>(t + off);
  if (first) {
    st<T, C>(out + off, dth * tv);
    return;
  }
  const int i = p % n, j = p / n;
  C v[3][3];
  gather9<T, C>(y + (int64_t)blockIdx.y * N, i, j, n, v);
  const C yp = yprev ? ld<T, C>(yprev + off) : C(0);
  st<T, C>(out + off, w * (v[1][1] - yp + dth * (tv - mass9<C>(v, mh))) + yp);
}

// out_b = M in_b, B blocks (FP64)
__global__ __launch_bounds__(TPB) void k_fe_mass(const double* __restrict__ in, double* __restrict__ out, int n,
                                                 double mh) {
  const int N = n * n;
  const int p = blockIdx.x * TPB + threadIdx.x;
  if (p >= N) return;
  const int i = p % n, j = p / n;
  double v[3][3];
  gather9<double, double>(in + (int64_t)blockIdx.y * N, i, j, n, v);
  out[(int64_t)blockIdx.y * N + p] = mass9<double>(v, mh);
}

inline dim3 fe_grid(int64_t N, int64_t B) { return dim3((unsigned)((N + TPB - 1) / TPB), (unsigned)B); }

inline double fe_mh(const aao_problem* h) { return h->h * h->h / 36.0; }

#define AAO_FE_S(s_, M) \
  do {                  \
    if ((s_) == 1) M(1); \
    else if ((s_) == 2) M(2); \
    else M(3);          \
  } while (0)

}  // namespace

template <class TX>
hipError_t fe_apply_A(const aao_problem* h, const TX* x, double* y, bool transpose, hipStream_t st) {
  const dim3 g = fe_grid(h->N, (int64_t)(h->nt + 1) + (int64_t)h->nt * h->s);
  const double mh = fe_mh(h);
#define AAO_GO(S_)                                                                                               \
  do {                                                                                                           \
    if (transpose) hipLaunchKernelGGL((k_fe_apply_AT<S_, TX>), g, dim3(TPB), 0, st, x, y, h->n, h->nt, mh, h->tab); \
    else hipLaunchKernelGGL((k_fe_apply_A<S_, TX>), g, dim3(TPB), 0, st, x, y, h->n, h->nt, mh, h->tab);          \
  } while (0)
  AAO_FE_S(h->s, AAO_GO);
#undef AAO_GO
  return hipGetLastError();
}

template <class T>
hipError_t fe_theta_apply(const aao_problem* h, const Tab& tab, const T* z, int64_t sz, T* w, int64_t sw, int B,
                          hipStream_t st) {
  using C = typename Acc<T>::type;
  const dim3 g = fe_grid(h->N, B);
  const C mh = (C)fe_mh(h);
#define AAO_GO(S_) hipLaunchKernelGGL((k_fe_theta<S_, T>), g, dim3(TPB), 0, st, z, sz, w, sw, h->n, mh, tab)
  AAO_FE_S(h->s, AAO_GO);
#undef AAO_GO
  return hipGetLastError();
}

template <class T>
hipError_t fe_rana_rhs(const aao_problem* h, const Tab& tab, int i, const T* v, int64_t sv, const T* z, int64_t sz,
                       T* out, int64_t so, int B, hipStream_t st) {
  hipLaunchKernelGGL((k_fe_rana_rhs<T>), fe_grid(h->N, B), dim3(TPB), 0, st, v, sv, z, sz, out, so, h->n, i, h->s,
                     tab);
  return hipGetLastError();
}

template <class T>
hipError_t fe_schur_coupling(const aao_problem* h, const double* r, const T* zV, T* t, hipStream_t st) {
  hipLaunchKernelGGL((k_fe_schur_coupling<T>), fe_grid(h->N, h->nt + 1), dim3(TPB), 0, st, r, zV, t, h->n, h->s,
                     fe_mh(h), h->tab);
  return hipGetLastError();
}

template <class T>
hipError_t fe_schur_kz(const aao_problem* h, const T* zin, int64_t szin, T* out, int64_t sout, int B,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_fe_schur_kz<T>), fe_grid(h->N, B), dim3(TPB), 0, st, zin, szin, out, sout, h->n, h->s);
  return hipGetLastError();
}

// t <- (CHEB_STEPS steps of Chebyshev semi-iteration with the Jacobi
// splitting) M^{-1} t on B consecutive blocks of N values, in place; ya, yb:
// two scratch vectors of B N values.  The spectrum of D^{-1} M of Q1 squares
// lies in [1/4, 9/4] (D = diag M = 4 h^2 / 9); theta = 5/4 its centre, rho
// = 4/5 the radius of the Jacobi iteration matrix I - D^{-1} M / theta.
template <class T>
hipError_t fe_mass_solve(const aao_problem* h, T* t, T* ya, T* yb, int B, hipStream_t st) {
  using C = typename Acc<T>::type;
  const double alpha = 0.25, beta = 2.25;
  const double theta = 0.5 * (alpha + beta), rho = (beta - alpha) / (beta + alpha);
  const double dinv = 9.0 / (4.0 * h->h * h->h);
  const C mh = (C)fe_mh(h), dth = (C)(dinv / theta);
  const dim3 g = fe_grid(h->N, B);
  const int n = h->n;
  // y_1 -> ya; then y_{k+1} overwrites y_{k-1}; the last step writes into t
  hipLaunchKernelGGL((k_fe_cheb<T>), g, dim3(TPB), 0, st, (const T*)t, (const T*)nullptr, (const T*)nullptr, ya, n,
                     mh, dth, C(1), 1);
  T* cur = ya;
  T* prev = yb;
  double w = 1.0;
  for (int k = 1; k < FE_CHEB_STEPS; ++k) {
    w = k == 1 ? 1.0 / (1.0 - rho * rho / 2.0) : 1.0 / (1.0 - rho * rho * w / 4.0);
    const bool last = k + 1 == FE_CHEB_STEPS;
    T* out = last ? t : prev;
    hipLaunchKernelGGL((k_fe_cheb<T>), g, dim3(TPB), 0, st, (const T*)t, (const T*)cur,
                       k == 1 ? (const T*)nullptr : (const T*)prev, out, n, mh, dth, (C)w, 0);
    prev = cur;
    cur = out;
  }
  return hipGetLastError();
}

hipError_t fe_assemble_rhs(const aao_problem* h, const double* f, const double* u0, double* rhs, hipStream_t st) {
  const int64_t N = h->N;
  hipLaunchKernelGGL(k_fe_mass, fe_grid(N, 1), dim3(TPB), 0, st, u0, rhs, h->n, fe_mh(h));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_fill<double>(rhs + N, 0.0, (int64_t)h->nt * N, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fe_mass, fe_grid(N, (int64_t)h->nt * h->s), dim3(TPB), 0, st, f,
                     rhs + (int64_t)(h->nt + 1) * N, h->n, fe_mh(h));
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
  template hipError_t fe_apply_A<T>(const aao_problem*, const T*, double*, bool, hipStream_t);
AAO_FE_INST(double)
AAO_FE_INST(float)
AAO_FE_INST(__half)
#undef AAO_FE_INST

}  // namespace aao

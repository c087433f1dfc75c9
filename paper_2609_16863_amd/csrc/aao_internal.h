// Internal declarations of the all-at-once heat solver library (not part of
// the C ABI).  Kernels live in kern_*.hip, host orchestration in solver.hip,
// the ABI in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "aao_heat.h"

namespace aao {

constexpr int SMAX = 3;          // Radau IIA stages supported by the kernels
constexpr int KMAX = 12;         // inner GMRES iterations per application
constexpr int MMAX = 120;        // outer FGMRES restart length
constexpr int DOTS_PER_PASS = 16;
constexpr int RED_THREADS = 256;
constexpr int COARSE_MAX = 256;        // default size of the exactly solved coarsest multigrid level
constexpr int COARSE_DENSE_MAX = 256;  // largest coarsest level solved with a dense inverse
constexpr int COARSE_FD_MAX = 1024;    // largest coarsest level solved by fast diagonalization (2D)

// ---------------------------------------------------------------------------
// Parameters passed to kernels by value
// ---------------------------------------------------------------------------
struct Tab {                     // Runge--Kutta data (Sec. 2)
  int s;
  double tau;
  double A[SMAX * SMAX];         // A_RK, row-major
  double b[SMAX];
  double L[SMAX * SMAX];         // Crout lower factor (Rana's preconditioner)
};

// Face diffusivities for variable kappa: minus/plus side of every node along
// each axis (already divided by h^2 is NOT applied here).  All null when
// kappa = 1.
template <class C>
struct Faces {
  const C* m[3];
  const C* p[3];
};

// One multigrid level's operator.  Level 0: I + a K (matrix-free 5/7-point).
// Level >= 1, constant kappa: Galerkin operator M(x)M(x..) + a sum T(x)M..,
// from 1D tridiagonal factors tri = [Mlo, Md, Mup, Tlo, Td, Tup] (each n).
template <class C>
struct LevelOp {
  int n;
  int64_t N;
  C a;             // shift tau * L_ii
  C ih2;           // 1/h^2 (level 0 only)
  const C* tri;    // 6 * n (level >= 1)
  const C* st9;    // level >= 1, variable kappa (2D): 9 * N Galerkin stencil of K, else null
  Faces<C> faces;  // level 0, variable kappa
};

// Precision of storage types.
template <class T> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

template <class T> __host__ __device__ inline float to_f(T v);
template <> __host__ __device__ inline float to_f<float>(float v) { return v; }
template <> __host__ __device__ inline float to_f<double>(double v) { return (float)v; }

template <class T, class C> __device__ __forceinline__ C ld(const T* p) { return (C)(*p); }
template <> __device__ __forceinline__ float ld<__half, float>(const __half* p) { return __half2float(*p); }
template <> __device__ __forceinline__ float ld<__hip_bfloat16, float>(const __hip_bfloat16* p) {
  return __bfloat162float(*p);
}
template <class T, class C> __device__ __forceinline__ void st(T* p, C v) { *p = (T)v; }
template <> __device__ __forceinline__ void st<__half, float>(__half* p, float v) { *p = __float2half_rn(v); }
template <> __device__ __forceinline__ void st<__hip_bfloat16, float>(__hip_bfloat16* p, float v) {
  *p = __float2bfloat16(v);
}

// Strided batch of vectors: instance b starts at ptr + b * stride.
template <class T>
struct BVec {
  T* ptr;
  int64_t stride;
  __host__ __device__ T* at(int b) const { return ptr + (int64_t)b * stride; }
};

}  // namespace aao

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct aao_problem {
  int dim = 2, n = 0, s = 1, nt = 1;
  double T = 1.0, tau = 1.0, h = 1.0, ih2 = 1.0;
  int64_t N = 0, U = 0, UV = 0;
  aao::Tab tab{};
  double c[aao::SMAX] = {0, 0, 0};
  double LT[aao::SMAX * aao::SMAX] = {0};   // Crout lower factor of A_RK^T
  aao_opts opts{};
  double omega = 0.8;
  bool vark = false;
  bool fe = false;                           // finite elements (AAO_DISC_Q1 or AAO_DISC_Q2)
  int fe_order = 0;                          // 1: bilinear (Q1), 2: biquadratic (Q2)
  std::vector<double> kappa;                 // host copy (N) when vark

  // multigrid levels (sizes per axis), shared by all stages
  std::vector<int> lev_n;
  std::vector<int64_t> lev_N;
  std::vector<double> tri_host;              // concatenated 6*n_l per level
  std::vector<size_t> tri_off;               // element offset per level
  std::vector<double> cinv_host;             // coarsest-level inverses: [transpose][stage] N_c^2 each
  int64_t cinv_N = 0;
  std::vector<double> faces_host;            // 2*dim*N when vark
  std::vector<double> fd_host;               // coarsest level, constant kappa (2D): V (n_c^2) then lam (n_c)
  int fd_n = 0;                              // n_c when fd_host is set
  std::vector<double> st9_host;              // Galerkin stencils of K, levels >= 1 (2D, vark)
  std::vector<size_t> st9_off;               // element offset per level (levels >= 1)

  // workspace plan (byte offsets)
  size_t ws_need = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  struct Plan {
    size_t tri_d, tri_f, faces_d, faces_f, cinv_d, cinv_f, st9_d, st9_f, fd_d, fd_f;
    size_t outV, outZ, outW, outY;           // outer FGMRES
    size_t outPb;                            // P-tilde^{-1} b (left / split preconditioning)
    size_t gIn, gOut;                        // fixed input/output of the captured P-tilde
    size_t inV, inZ, inW, inX;               // inner GMRES (nt instances)
    size_t rana;                              // Rana right-hand side (nt*N)
    size_t schurRhs, schurY;                  // S-tilde steps (s*N per instance)
    size_t mgritT, mgritG, mgritE;            // MGRIT: t (nt+1 blocks), C-point values, corrections
    size_t feA, feB;                          // finite elements: Chebyshev mass-solve iterates (nt+1 blocks each)
    std::vector<size_t> mgX, mgT, mgB, mgR;   // per level, nt instances
    size_t partial, dscal, counters;          // reductions / device scalars / tickets
    size_t partial_bytes, dscal_bytes;
  } plan{};
  // Multigrid launch shapes (aao_autotune): blocks per launch from which the
  // FP32 tiled level kernels use their tall tiles, and whether the register
  // tail also takes a 64 x 64 level.  Neither changes the algorithm.
  struct Tune {
    int tall_min_b = 8;
    bool tail_extend = true;
  } tune;
  int pi_bytes = 8;                           // inner (GMRES) storage bytes
  int pm_bytes = 8;                           // multigrid storage bytes
  double mg_scale = 1.0;                      // coarse-level vectors are stored times this (FP16 storage)

  hipStream_t stream = nullptr;
  size_t lds_budget = 65536;                  // LDS bytes per workgroup for the multigrid tail
  struct GraphEntry {
    bool transpose;
    int k, cycles, phase;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;             // captured P-tilde applications
  hipStream_t capture_stream = nullptr;
  hipEvent_t phase_ev[3] = {nullptr, nullptr, nullptr};   // P-tilde phase timing
  double* hpin = nullptr;                     // pinned host scalars
  // Set while a call runs in the library's static scratch memory: no graph
  // capture, no events, and host reads go through hpage instead of hpin.
  bool no_alloc = false;
  double hpage[4096];
  double* host_scalars() { return no_alloc || !hpin ? hpage : hpin; }
  std::string err;
};

// ---------------------------------------------------------------------------
// Host-side helpers implemented in setup.cpp / solver.hip / kern_*.hip
// ---------------------------------------------------------------------------
namespace aao {

// setup.cpp (host only)
bool radau_iia(int s, double* A, double* b, double* c);
void crout_lower(int s, const double* A, double* L);
void galerkin_1d(int n, int dim, double h, int coarse_max, int fe, std::vector<int>& sizes,
                 std::vector<std::vector<double>>& tri);
bool tensor_eigen(int n, const std::vector<double>& tri, std::vector<double>& V, std::vector<double>& lam);
void galerkin_stencils_2d(const std::vector<int>& sizes, const std::vector<double>& faces, double ih2,
                          std::vector<std::vector<double>>& st9);
bool coarse_inverse(int dim, int n, const std::vector<double>& tri, double a, bool fine, double ih2,
                    const double* faces, const double* st9, std::vector<double>& invT);
void face_coefficients(int dim, int n, const double* kappa, std::vector<double>& faces);

int status_from_hip(aao_problem* h, hipError_t e, const char* what);

// kern_allatonce.hip
template <class TX>
hipError_t launch_apply_A(const aao_problem* h, const TX* x, double* y, hipStream_t st);
template <class TX>
hipError_t launch_apply_AT(const aao_problem* h, const TX* x, double* y, hipStream_t st);
hipError_t launch_sub_from(const double* a, double* y, int64_t n, hipStream_t st);
template <class TY, class TX>
hipError_t launch_scale(TY* y, const TX* x, double alpha, int64_t n, hipStream_t st);
hipError_t launch_assemble_rhs(const aao_problem* h, const double* f, const double* u0, double* rhs,
                               hipStream_t st);
hipError_t launch_grad_logkappa(const aao_problem* h, const double* x, const double* lam, double* g,
                                hipStream_t st);
template <class TD, class TS>
hipError_t launch_copy_cast(TD* dst, const TS* src, int64_t n, hipStream_t st);
// out = a - b (b may be null), converted to TO
template <class TO, class TA>
hipError_t launch_diff(TO* out, const TA* a, const TA* b, int64_t n, hipStream_t st);
template <class T>
hipError_t launch_fill(T* dst, T v, int64_t n, hipStream_t st);
// x <- x rounded to FP32 (nearest even) and back: simulated single precision
hipError_t launch_round_f32(double* x, int64_t n, hipStream_t st);
// x <- x rounded to FP32, then to BF16 (nearest even), and back
hipError_t launch_round_bf16(double* x, int64_t n, hipStream_t st);

// kern_mg.hip
size_t mg_configure_lds();

// api.hip: copy the handle's constant tables into its workspace (h->ws) and
// clear its counters, on the handle's stream (not synchronised).
hipError_t upload_tables(aao_problem* h);

// solver.hip
void release_graphs(aao_problem* h);
int apply_P(aao_problem* h, const double* r, double* z, int inner_k, int cycles, bool transpose);
int solve(aao_problem* h, const double* rhs, double* x, aao_stats* st, bool transpose);
// `cycles` V-cycles on count blocks of (I + tau L_ii K), L = Crout factor of
// A (or A^T); r, z in the preconditioner's working type.
hipError_t apply_mg(aao_problem* h, bool transpose, int stage, int count, int cycles, const void* r, void* z);
// One V-cycle from zero on `count` blocks of stage `stage`: labels of its
// launches and their mean microseconds in situ (event after every launch)
// and alone (each launch replayed by itself from a graph), and the mean
// microseconds of the whole cycle replayed as a graph.
hipError_t profile_vcycle(aao_problem* h, int stage, int count, int reps, std::vector<std::string>& labels,
                          std::vector<double>& us_situ, std::vector<double>& us_alone, double& total_us);
// Capture (without launching) the HIP graph of the handle's P-tilde (or its
// transpose) so that later solves only replay it.
hipError_t prepare_graph(aao_problem* h, bool transpose);
// First multigrid level handled by the one-workgroup tail.
int mg_tail_level(aao_problem* h);

}  // namespace aao

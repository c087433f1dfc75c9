// C ABI of the all-at-once heat solver (declared in include/aao_heat.h).
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "aao_internal.h"

namespace {

std::string g_create_error;

int fail(aao_problem* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lay out every device buffer of the handle inside one workspace.
void plan_workspace(aao_problem* h) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = align256(off);
    off = o + align256(bytes);
    return o;
  };
  auto& P = h->plan;
  const int64_t N = h->N, U = h->U, UV = h->UV;
  const int L = (int)h->lev_n.size();
  P.tri_d = take(h->tri_host.size() * sizeof(double));
  P.tri_f = take(h->tri_host.size() * sizeof(float));
  P.cinv_d = take(h->cinv_host.size() * sizeof(double));
  P.cinv_f = take(h->cinv_host.size() * sizeof(float));
  P.fd_d = take(h->fd_host.size() * sizeof(double));
  P.fd_f = take(h->fd_host.size() * sizeof(float));
  P.st9_d = take(h->st9_host.size() * sizeof(double));
  P.st9_f = take(h->st9_host.size() * sizeof(float));
  // faces (2*dim*N) followed by nodal kappa (N)
  P.faces_d = take(h->vark ? (size_t)(2 * h->dim + 1) * N * sizeof(double) : 0);
  P.faces_f = take(h->vark ? (size_t)(2 * h->dim + 1) * N * sizeof(float) : 0);
  const int m = h->opts.restart;
  const int k = h->opts.inner_k;
  const size_t pi = (size_t)h->pi_bytes, pm = (size_t)h->pm_bytes;
  P.outV = take((size_t)(m + 1) * U * sizeof(double));
  P.outZ = take((size_t)m * U * pi);
  P.outW = take((size_t)U * sizeof(double));
  P.outY = take((size_t)U * pi);
  P.outPb = take(h->opts.side != AAO_SIDE_RIGHT ? (size_t)U * pi : 0);
  P.gIn = take(h->opts.use_graph ? (size_t)U * sizeof(double) : 0);
  P.gOut = take(h->opts.use_graph ? (size_t)U * pi : 0);
  P.inV = take((size_t)(k + 1) * UV * pi);
  P.inZ = take((size_t)k * UV * pi);
  P.inW = take((size_t)UV * pi);
  P.inX = take((size_t)UV * pi);
  P.rana = take((size_t)h->nt * N * pi);
  // S-tilde step buffers: one instance for the substitution, one per coarse
  // interval for MGRIT's batched relaxation; MGRIT keeps t, the C-point
  // values g and the coarse corrections e apart
  const bool mgrit = h->opts.schur == AAO_SCHUR_MGRIT;
  const int64_t Kc = mgrit ? (h->nt + h->opts.mgrit_cf - 1) / h->opts.mgrit_cf : 1;
  P.schurRhs = take((size_t)Kc * h->s * N * pi);
  P.schurY = take((size_t)Kc * h->s * N * pi);
  P.mgritT = take(mgrit ? (size_t)(h->nt + 1) * N * pi : 0);
  P.mgritG = take(mgrit ? (size_t)Kc * N * pi : 0);
  P.mgritE = take(mgrit ? (size_t)Kc * N * pi : 0);
  P.feA = take(h->fe ? (size_t)(h->nt + 1) * N * pi : 0);
  P.feB = take(h->fe ? (size_t)(h->nt + 1) * N * pi : 0);
  P.mgX.assign(L, 0);
  P.mgT.assign(L, 0);
  P.mgB.assign(L, 0);
  P.mgR.assign(L, 0);
  // coarse levels the precision schedule may keep in the level-0 format
  const bool sched = h->opts.mg_low_from > 1 || h->opts.mg_coarse_fp32;
  for (int l = 0; l < L; ++l) {
    const size_t bytes = (size_t)h->nt * h->lev_N[l] * (l == 0 || sched ? pi : pm);
    if (l > 0) {
      P.mgX[l] = take(bytes);
      P.mgB[l] = take(bytes);
    }
    P.mgT[l] = take(bytes);
    P.mgR[l] = take(bytes);
  }
  P.partial_bytes = (size_t)8192 * aao::DOTS_PER_PASS * sizeof(double) + (size_t)h->nt * 64 *
                    (aao::KMAX + 2) * sizeof(double);
  P.partial = take(P.partial_bytes);
  P.dscal_bytes = (size_t)(h->nt + 1) * 512 * sizeof(double) + (aao::MMAX + 8) * 8 * sizeof(double);
  P.dscal = take(P.dscal_bytes);
  P.counters = take((size_t)(h->nt + 2) * sizeof(unsigned));
  h->ws_need = align256(off);
}

// The tables that depend on the diffusivity, for nodal values `kappa`
// (empty for kappa = 1): face coefficients and the Galerkin stencils of the
// coarse levels (variable kappa), and the exact inverses of the coarsest
// level when it is not solved by fast diagonalization -- for the shifts
// tau L_ii of P-tilde and tau LT_ii of its transpose (sets 0, 1) and, with
// MGRIT, those of its coarse step of mgrit_cf tau (sets 2, 3).  Written into
// the handle only when all of them could be built.
bool kappa_tables(aao_problem* h, const std::vector<double>& kappa, std::string& why) {
  std::vector<double> faces, st9_all, cinv;
  std::vector<size_t> st9_off;
  std::vector<std::vector<double>> st9;
  const int L = (int)h->lev_n.size();
  if (!kappa.empty()) {
    for (double kv : kappa)
      if (!(kv > 0.0) || !std::isfinite(kv)) {
        why = "kappa must be finite and > 0";
        return false;
      }
    aao::face_coefficients(h->dim, h->n, kappa.data(), faces);
    aao::galerkin_stencils_2d(h->lev_n, faces, h->ih2, st9);
    st9_off.assign(L, 0);
    for (int l = 1; l < L; ++l) {
      st9_off[l] = st9_all.size();
      st9_all.insert(st9_all.end(), st9[l].begin(), st9[l].end());
    }
  }
  if (h->fd_n == 0) {
    const int lc = L - 1;
    const std::vector<double> tri(h->tri_host.begin() + h->tri_off[lc],
                                  h->tri_host.begin() + h->tri_off[lc] + 6 * h->lev_n[lc]);
    const int nsets = h->opts.schur == AAO_SCHUR_MGRIT ? 4 : 2;
    for (int set = 0; set < nsets; ++set)
      for (int i = 0; i < h->s; ++i) {
        const double* Lf = (set & 1) ? h->LT : h->tab.L;
        const double a = (set >= 2 ? h->opts.mgrit_cf : 1) * h->tau * Lf[i * h->s + i];
        std::vector<double> inv;
        if (!aao::coarse_inverse(h->dim, h->lev_n[lc], tri, a, lc == 0 && !h->fe, h->ih2,
                                 kappa.empty() ? nullptr : faces.data(),
                                 (!kappa.empty() && lc > 0) ? st9[lc].data() : nullptr, inv)) {
          why = "singular coarsest multigrid level";
          return false;
        }
        cinv.insert(cinv.end(), inv.begin(), inv.end());
      }
  }
  h->faces_host.swap(faces);
  h->st9_host.swap(st9_all);
  h->st9_off.swap(st9_off);
  h->cinv_host.swap(cinv);
  if (h->fd_n == 0) h->cinv_N = h->lev_N[L - 1];
  return true;
}

bool valid_opts(const aao_opts* o, std::string& why) {
  if (o->restart < 1 || o->restart > aao::MMAX) { why = "restart must be in [1, 120]"; return false; }
  if (o->maxit < 1) { why = "maxit must be >= 1"; return false; }
  if (!(o->tol > 0.0)) { why = "tol must be > 0"; return false; }
  if (o->inner_k < 1 || o->inner_k > aao::KMAX) { why = "inner_k must be in [1, 12]"; return false; }
  if (o->cycles < 1 || o->cycles > 64) { why = "cycles must be in [1, 64]"; return false; }
  if (o->nu1 < 1 || o->nu2 < 1 || o->nu1 > 16 || o->nu2 > 16) { why = "nu1, nu2 must be in [1, 16]"; return false; }
  if (o->precision < AAO_PREC_FP64 || o->precision > AAO_PREC_FP16_ALL) { why = "unknown precision"; return false; }
  if (o->omega < 0.0 || o->omega >= 2.0) { why = "omega must be in [0, 2)"; return false; }
  if (o->mg_tail_max < 0) { why = "mg_tail_max must be >= 0"; return false; }
  if (o->coarse_max < 0 || o->coarse_max > aao::COARSE_FD_MAX) { why = "coarse_max must be in [0, 1024]"; return false; }
  if (!(o->inner_tol >= 0.0 && o->inner_tol < 1.0)) { why = "inner_tol must be in [0, 1)"; return false; }
  if (o->schur != AAO_SCHUR_SWEEP && o->schur != AAO_SCHUR_MGRIT) { why = "unknown schur"; return false; }
  if (o->mgrit_cf != 0 && (o->mgrit_cf < 2 || o->mgrit_cf > 64)) { why = "mgrit_cf must be in [2, 64]"; return false; }
  if (o->mgrit_iters < 0) { why = "mgrit_iters must be >= 0"; return false; }
  if (o->mgrit_fcf != 0 && o->mgrit_fcf != 1) { why = "mgrit_fcf must be 0 or 1"; return false; }
  if (o->side < AAO_SIDE_RIGHT || o->side > AAO_SIDE_SPLIT) { why = "unknown side"; return false; }
  if (o->outer_precision != AAO_OUTER_FP64 && o->outer_precision != AAO_OUTER_FP32) {
    why = "unknown outer_precision";
    return false;
  }
  if (o->mg_low_from < 0) { why = "mg_low_from must be >= 0"; return false; }
  if (o->mg_coarse_fp32 != 0 && o->mg_coarse_fp32 != 1) { why = "mg_coarse_fp32 must be 0 or 1"; return false; }
  if (o->relax_matvec != 0 && o->relax_matvec != 1) { why = "relax_matvec must be 0 or 1"; return false; }
  if (o->mgrit_coarse_k < 0 || o->mgrit_coarse_k > aao::KMAX) { why = "mgrit_coarse_k must be in [0, 12]"; return false; }
  if (o->schur_k < 0 || o->schur_k > aao::KMAX) { why = "schur_k must be in [0, 12]"; return false; }
  if (o->inner_orth != AAO_ORTH_CGS2 && o->inner_orth != AAO_ORTH_CGS1) { why = "inner_orth must be CGS2 or CGS1"; return false; }
  if (o->outer_orth != AAO_ORTH_CGS2 && o->outer_orth != AAO_ORTH_GRAM) { why = "outer_orth must be CGS2 or GRAM"; return false; }
  return true;
}

}  // namespace

namespace aao {
int status_from_hip(aao_problem* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return AAO_OK;
  return fail(h, AAO_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
// FP64 table from the host to ws + off_d, and its FP32 copy at ws + off_f.
hipError_t upload_pair(aao_problem* h, const double* host, size_t count, size_t off_d, size_t off_f) {
  if (count == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(h->ws + off_d, host, count * sizeof(double), hipMemcpyHostToDevice, h->stream);
  if (e != hipSuccess) return e;
  return launch_copy_cast<float, double>(reinterpret_cast<float*>(h->ws + off_f),
                                         reinterpret_cast<const double*>(h->ws + off_d), (int64_t)count, h->stream);
}
}  // namespace

hipError_t upload_tables(aao_problem* h) {
  const auto& P = h->plan;
  hipError_t e = upload_pair(h, h->tri_host.data(), h->tri_host.size(), P.tri_d, P.tri_f);
  if (e == hipSuccess) e = upload_pair(h, h->cinv_host.data(), h->cinv_host.size(), P.cinv_d, P.cinv_f);
  if (e == hipSuccess) e = upload_pair(h, h->fd_host.data(), h->fd_host.size(), P.fd_d, P.fd_f);
  if (e == hipSuccess) e = upload_pair(h, h->st9_host.data(), h->st9_host.size(), P.st9_d, P.st9_f);
  if (e == hipSuccess && h->vark) {
    // faces (2 dim N) followed by the nodal kappa (N)
    const size_t nf = h->faces_host.size();
    e = hipMemcpyAsync(h->ws + P.faces_d, h->faces_host.data(), nf * sizeof(double), hipMemcpyHostToDevice,
                       h->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->ws + P.faces_d + nf * sizeof(double), h->kappa.data(), h->N * sizeof(double),
                         hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
      e = launch_copy_cast<float, double>(reinterpret_cast<float*>(h->ws + P.faces_f),
                                          reinterpret_cast<const double*>(h->ws + P.faces_d),
                                          (int64_t)(nf + h->N), h->stream);
  }
  if (e == hipSuccess)
    e = launch_fill<unsigned>(reinterpret_cast<unsigned*>(h->ws + P.counters), 0u, h->nt + 2, h->stream);
  return e;
}
}  // namespace aao

extern "C" {

void aao_default_opts(aao_opts* o) {
  if (!o) return;
  o->restart = 30;
  o->maxit = 100;
  o->tol = 1e-8;
  o->inner_k = 3;
  o->cycles = 1;
  o->nu1 = 2;
  o->nu2 = 2;
  o->omega = 0.0;
  o->precision = AAO_PREC_FP64;
  o->use_graph = 1;
  o->mg_tail_max = 0;
  o->coarse_max = 0;
  o->inner_tol = 0.0;
  o->schur = AAO_SCHUR_SWEEP;
  o->mgrit_cf = 8;
  o->mgrit_iters = 1;
  o->mgrit_fcf = 0;
  o->side = AAO_SIDE_RIGHT;
  o->outer_precision = AAO_OUTER_FP64;
  o->mg_low_from = 0;
  o->mg_coarse_fp32 = 0;
  o->relax_matvec = 0;
  o->mgrit_coarse_k = 0;
  o->schur_k = 0;
  o->inner_orth = AAO_ORTH_CGS2;
  o->outer_orth = AAO_ORTH_CGS2;
}

int aao_create_problem(const aao_desc* d, const aao_opts* o, aao_problem** out) {
  if (!d || !out) return fail(nullptr, AAO_INVALID_ARG, "null argument");
  *out = nullptr;
  if (d->dim != 2 && d->dim != 3) return fail(nullptr, AAO_INVALID_ARG, "dim must be 2 or 3");
  if (d->n < 2) return fail(nullptr, AAO_INVALID_ARG, "n must be >= 2");
  if (d->s < 1 || d->s > aao::SMAX) return fail(nullptr, AAO_INVALID_ARG, "s must be 1, 2 or 3");
  if (d->nt < 1 || d->nt > 65535) return fail(nullptr, AAO_INVALID_ARG, "nt must be in [1, 65535]");
  if (!(d->T > 0.0) || !std::isfinite(d->T)) return fail(nullptr, AAO_INVALID_ARG, "T must be > 0");
  if (d->disc != AAO_DISC_FD && d->disc != AAO_DISC_Q1 && d->disc != AAO_DISC_Q2)
    return fail(nullptr, AAO_INVALID_ARG, "unknown disc");
  const bool fe = d->disc != AAO_DISC_FD;
  if (d->disc == AAO_DISC_FD && d->length != 0.0 && d->length != 1.0)
    return fail(nullptr, AAO_INVALID_ARG, "finite differences live on the unit domain (length 0 or 1)");
  if (fe) {
    if (d->dim != 2 || d->kappa) return fail(nullptr, AAO_INVALID_ARG, "finite elements: 2D and constant kappa");
    if ((int64_t)(d->nt + 1) + (int64_t)d->nt * d->s > 65535)
      return fail(nullptr, AAO_INVALID_ARG, "finite elements: (nt + 1) + nt s must be <= 65535");
    if (d->length < 0.0 || !std::isfinite(d->length)) return fail(nullptr, AAO_INVALID_ARG, "length must be > 0");
    if (d->disc == AAO_DISC_Q2 && (d->n < 3 || d->n % 2 == 0))
      return fail(nullptr, AAO_INVALID_ARG, "Q2 elements: n must be odd and >= 3");
  }
  const double Nd = std::pow((double)d->n, d->dim);
  if (Nd > 1.5e9) return fail(nullptr, AAO_INVALID_ARG, "grid too large (N must fit in int32)");
  aao_opts opts;
  aao_default_opts(&opts);
  if (o) opts = *o;
  std::string why;
  if (!valid_opts(&opts, why)) return fail(nullptr, AAO_INVALID_ARG, why);
  if (opts.mgrit_cf == 0) opts.mgrit_cf = 8;
  if (opts.mgrit_iters == 0) opts.mgrit_iters = 1;
  if (opts.mgrit_iters > d->nt) return fail(nullptr, AAO_INVALID_ARG, "mgrit_iters must be <= nt");
  if (fe && (opts.nu1 > 3 || opts.nu2 > 3))
    return fail(nullptr, AAO_INVALID_ARG, "finite elements: nu1, nu2 <= 3");

  aao_problem* h = new (std::nothrow) aao_problem();
  if (!h) return fail(nullptr, AAO_INVALID_ARG, "out of host memory");
  h->dim = d->dim;
  h->n = d->n;
  h->s = d->s;
  h->nt = d->nt;
  h->T = d->T;
  h->tau = d->T / d->nt;
  h->fe = fe;
  h->fe_order = d->disc == AAO_DISC_Q2 ? 2 : (fe ? 1 : 0);
  h->h = (h->fe && d->length > 0.0 ? d->length : 1.0) / (d->n + 1);
  h->ih2 = 1.0 / (h->h * h->h);
  h->N = (int64_t)std::llround(Nd);
  h->U = h->N * ((int64_t)d->nt * (d->s + 1) + 1);
  h->UV = h->N * (int64_t)d->nt * d->s;
  h->opts = opts;
  h->omega = opts.omega > 0.0 ? opts.omega : (d->dim == 2 ? 0.8 : 6.0 / 7.0);
  h->pi_bytes = opts.precision == AAO_PREC_FP64 ? 8 : (opts.precision == AAO_PREC_FP16_ALL ? 2 : 4);
  h->pm_bytes = opts.precision == AAO_PREC_FP64 ? 8 : (opts.precision == AAO_PREC_FP32 ? 4 : 2);
  // FP16 multigrid storage: the V-cycle's right-hand sides are unit-norm
  // Krylov vectors over s N entries, so their entries are near (s N)^{-1/2};
  // the coarse levels store their vectors times the power of two nearest to
  // (s N)^{1/2}, which keeps them near 1, well inside FP16's normal range
  // (the cycle is linear below level 0, so only the level-0 transfers see it).
  if (opts.precision == AAO_PREC_FP16)
    h->mg_scale = std::ldexp(1.0, (int)std::lround(0.5 * std::log2((double)d->s * (double)h->N)));

  h->tab.s = d->s;
  h->tab.tau = h->tau;
  if (!aao::radau_iia(d->s, h->tab.A, h->tab.b, h->c)) {
    delete h;
    return fail(nullptr, AAO_INVALID_ARG, "Radau IIA construction failed");
  }
  aao::crout_lower(d->s, h->tab.A, h->tab.L);
  double At[aao::SMAX * aao::SMAX];
  for (int i = 0; i < d->s; ++i)
    for (int j = 0; j < d->s; ++j) At[i * d->s + j] = h->tab.A[j * d->s + i];
  aao::crout_lower(d->s, At, h->LT);
  for (int i = 0; i < d->s; ++i)
    if (!(h->tab.L[i * d->s + i] > 0.0) || !(h->LT[i * d->s + i] > 0.0)) {
      delete h;
      return fail(nullptr, AAO_INVALID_ARG, "non-positive Crout pivot");
    }

  if (d->kappa) {
    h->vark = true;
    h->kappa.assign(d->kappa, d->kappa + h->N);
    for (double kv : h->kappa)
      if (!(kv > 0.0) || !std::isfinite(kv)) {
        delete h;
        return fail(nullptr, AAO_INVALID_ARG, "kappa must be finite and > 0");
      }
    if (d->dim == 3) {
      delete h;
      return fail(nullptr, AAO_INVALID_ARG, "variable kappa is supported in 2D only");
    }
  }

  // 2D constant kappa solves the coarsest level by fast diagonalization (up
  // to 1024 nodes); otherwise by a dense inverse (up to 256 nodes)
  const int cmax = opts.coarse_max > 0 ? opts.coarse_max : aao::COARSE_MAX;
  const bool fd_ok = d->dim == 2 && !d->kappa;
  if (!fd_ok && cmax > aao::COARSE_DENSE_MAX) {
    delete h;
    return fail(nullptr, AAO_INVALID_ARG, "coarse_max above 256 needs 2D and constant kappa");
  }
  std::vector<std::vector<double>> tri;
  aao::galerkin_1d(d->n, d->dim, h->h, cmax, h->fe_order, h->lev_n, tri);
  h->lev_N.resize(h->lev_n.size());
  h->tri_off.assign(h->lev_n.size(), 0);
  for (size_t l = 0; l < h->lev_n.size(); ++l) {
    h->lev_N[l] = (int64_t)std::llround(std::pow((double)h->lev_n[l], d->dim));
    h->tri_off[l] = h->tri_host.size();
    h->tri_host.insert(h->tri_host.end(), tri[l].begin(), tri[l].end());
  }
  // fast diagonalization of the coarsest level (2D, constant kappa)
  if (fd_ok) {
    const int lc = (int)h->lev_n.size() - 1;
    std::vector<double> V, lam;
    if (aao::tensor_eigen(h->lev_n[lc], tri[lc], V, lam)) {
      h->fd_n = h->lev_n[lc];
      h->fd_host = V;
      h->fd_host.insert(h->fd_host.end(), lam.begin(), lam.end());
    } else if (h->lev_N.back() > aao::COARSE_DENSE_MAX) {
      delete h;
      return fail(nullptr, AAO_INVALID_ARG, "coarsest multigrid level not diagonalizable");
    }
  }
  if (!kappa_tables(h, h->kappa, why)) {
    delete h;
    return fail(nullptr, AAO_INVALID_ARG, why);
  }
  plan_workspace(h);
  *out = h;
  return AAO_OK;
}

int aao_workspace_size(const aao_problem* h, size_t* bytes) {
  if (!h || !bytes) return AAO_INVALID_ARG;
  *bytes = h->ws_need;
  return AAO_OK;
}

int aao_set_workspace(aao_problem* h, void* dev_ptr, size_t bytes) {
  if (!h) return AAO_INVALID_ARG;
  if (!dev_ptr) return fail(h, AAO_INVALID_ARG, "null workspace");
  if (((uintptr_t)dev_ptr & 255) != 0) return fail(h, AAO_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < h->ws_need) return fail(h, AAO_WORKSPACE_TOO_SMALL, "workspace too small");
  hipError_t e = hipSuccess;
  if (!h->hpin) {
    e = hipHostMalloc((void**)&h->hpin, 4096 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
      h->hpin = nullptr;
      return aao::status_from_hip(h, e, "pinned host scalars");
    }
  }
  // captured P-tilde graphs hold the previous workspace's addresses
  if (h->ws != static_cast<char*>(dev_ptr)) aao::release_graphs(h);
  h->ws = static_cast<char*>(dev_ptr);
  h->ws_bytes = bytes;
  h->lds_budget = aao::mg_configure_lds();
  e = aao::upload_tables(h);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->ws = nullptr;
    return aao::status_from_hip(h, e, "workspace upload");
  }
  return AAO_OK;
}

int aao_set_kappa(aao_problem* h, const double* values, int is_log) {
  if (!h) return AAO_INVALID_ARG;
  if (!values) return fail(h, AAO_INVALID_ARG, "null kappa");
  if (!h->vark) return fail(h, AAO_INVALID_ARG, "the handle was created with constant kappa");
  if (is_log != 0 && is_log != 1) return fail(h, AAO_INVALID_ARG, "is_log must be 0 or 1");
  std::vector<double> kap((size_t)h->N);
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(kap.data(), values, kap.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return aao::status_from_hip(h, e, "set_kappa");
  if (is_log)
    for (double& v : kap) v = std::exp(v);
  const size_t nf = h->faces_host.size(), ns = h->st9_host.size(), nc = h->cinv_host.size();
  std::string why;
  if (!kappa_tables(h, kap, why)) return fail(h, AAO_INVALID_ARG, why);
  if (h->faces_host.size() != nf || h->st9_host.size() != ns || h->cinv_host.size() != nc)
    return fail(h, AAO_INVALID_ARG, "internal: diffusivity tables changed size");
  h->kappa.swap(kap);
  if (!h->ws) return AAO_OK;
  // same sizes and places in the workspace: the captured graphs stay valid
  e = aao::upload_tables(h);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return aao::status_from_hip(h, e, "set_kappa upload");
}

int aao_set_stream(aao_problem* h, void* stream) {
  if (!h) return AAO_INVALID_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  return AAO_OK;
}

int aao_destroy(aao_problem* h) {
  if (!h) return AAO_INVALID_ARG;
  aao::release_graphs(h);
  for (hipEvent_t& ev : h->phase_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (h->hpin) (void)hipHostFree(h->hpin);
  delete h;
  return AAO_OK;
}

int aao_get_tableau(const aao_problem* h, double* A, double* b, double* c) {
  if (!h) return AAO_INVALID_ARG;
  for (int i = 0; i < h->s; ++i) {
    if (b) b[i] = h->tab.b[i];
    if (c) c[i] = h->c[i];
    for (int j = 0; j < h->s; ++j)
      if (A) A[i * h->s + j] = h->tab.A[i * h->s + j];
  }
  return AAO_OK;
}

int aao_sizes(const aao_problem* h, int64_t* N, int64_t* U) {
  if (!h) return AAO_INVALID_ARG;
  if (N) *N = h->N;
  if (U) *U = h->U;
  return AAO_OK;
}

int aao_apply_A(aao_problem* h, const double* x, double* y) {
  if (!h) return AAO_INVALID_ARG;
  if (!x || !y || x == y) return fail(h, AAO_INVALID_ARG, "x, y must be distinct device pointers");
  if (h->vark && !h->ws) return fail(h, AAO_NO_WORKSPACE, "variable kappa needs the workspace");
  return aao::status_from_hip(h, aao::launch_apply_A<double>(h, x, y, h->stream), "apply_A");
}

int aao_apply_AT(aao_problem* h, const double* x, double* y) {
  if (!h) return AAO_INVALID_ARG;
  if (!x || !y || x == y) return fail(h, AAO_INVALID_ARG, "x, y must be distinct device pointers");
  if (h->vark && !h->ws) return fail(h, AAO_NO_WORKSPACE, "variable kappa needs the workspace");
  return aao::status_from_hip(h, aao::launch_apply_AT<double>(h, x, y, h->stream), "apply_AT");
}

int aao_apply_P(aao_problem* h, const double* r, double* z) {
  if (!h) return AAO_INVALID_ARG;
  return aao_apply_P_with(h, r, z, h->opts.inner_k, h->opts.cycles);
}

int aao_apply_P_with(aao_problem* h, const double* r, double* z, int inner_k, int cycles) {
  if (!h) return AAO_INVALID_ARG;
  if (!r || !z || r == z) return fail(h, AAO_INVALID_ARG, "r, z must be distinct device pointers");
  if (inner_k < 1 || inner_k > h->opts.inner_k) return fail(h, AAO_INVALID_ARG, "inner_k out of range");
  if (cycles < 1 || cycles > 64) return fail(h, AAO_INVALID_ARG, "cycles out of range");
  if (!h->ws) return fail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  return aao::apply_P(h, r, z, inner_k, cycles, false);
}

int aao_mg_levels(const aao_problem* h, int cap, int64_t* nodes, int* levels, int* tail_level) {
  if (!h) return AAO_INVALID_ARG;
  aao_problem* hm = const_cast<aao_problem*>(h);
  if (!levels || !tail_level || cap < 0 || (cap > 0 && !nodes)) return fail(hm, AAO_INVALID_ARG, "null pointer");
  const int L = (int)h->lev_N.size();
  *levels = L;
  for (int l = 0; l < L && l < cap; ++l) nodes[l] = h->lev_N[l];
  if (!h->ws) return fail(hm, AAO_NO_WORKSPACE, "the tail level depends on the device: aao_set_workspace first");
  *tail_level = aao::mg_tail_level(hm);
  return AAO_OK;
}

int aao_apply_mg(aao_problem* h, int transpose, int stage, int count, int cycles, const void* r, void* z) {
  if (!h) return AAO_INVALID_ARG;
  if (!r || !z) return fail(h, AAO_INVALID_ARG, "null pointer");
  if (transpose != 0 && transpose != 1) return fail(h, AAO_INVALID_ARG, "transpose must be 0 or 1");
  if (stage < 0 || stage >= h->s) return fail(h, AAO_INVALID_ARG, "stage out of range");
  if (count < 1 || count > h->nt) return fail(h, AAO_INVALID_ARG, "count must be in [1, nt]");
  if (cycles < 1 || cycles > 64) return fail(h, AAO_INVALID_ARG, "cycles out of range");
  const size_t bytes = (size_t)count * (size_t)h->N * (size_t)h->pi_bytes;
  const char* rb = static_cast<const char*>(r);
  const char* zb = static_cast<const char*>(z);
  if (rb < zb + bytes && zb < rb + bytes) return fail(h, AAO_INVALID_ARG, "r and z overlap");
  if (!h->ws) return fail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  return aao::status_from_hip(h, aao::apply_mg(h, transpose == 1, stage, count, cycles, r, z), "apply_mg");
}

int aao_assemble_rhs(aao_problem* h, const double* f, const double* u0, double* rhs) {
  if (!h) return AAO_INVALID_ARG;
  if (!f || !u0 || !rhs) return fail(h, AAO_INVALID_ARG, "null pointer");
  return aao::status_from_hip(h, aao::launch_assemble_rhs(h, f, u0, rhs, h->stream), "assemble_rhs");
}

int aao_solve(aao_problem* h, const double* rhs, double* x, aao_stats* st) {
  if (!h) return AAO_INVALID_ARG;
  if (!rhs || !x || rhs == x) return fail(h, AAO_INVALID_ARG, "rhs, x must be distinct device pointers");
  if (!h->ws) return fail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  return aao::solve(h, rhs, x, st, false);
}

int aao_solve_adjoint(aao_problem* h, const double* g, double* lam, aao_stats* st) {
  if (!h) return AAO_INVALID_ARG;
  if (!g || !lam || g == lam) return fail(h, AAO_INVALID_ARG, "g, lam must be distinct device pointers");
  if (!h->ws) return fail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  return aao::solve(h, g, lam, st, true);
}

int aao_grad_logkappa(aao_problem* h, const double* x, const double* lam, double* g) {
  if (!h) return AAO_INVALID_ARG;
  if (!x || !lam || !g) return fail(h, AAO_INVALID_ARG, "null pointer");
  if (h->fe) return fail(h, AAO_INVALID_ARG, "finite elements: the kappa gradient is not available");
  if (h->vark && !h->ws) return fail(h, AAO_NO_WORKSPACE, "aao_set_workspace first");
  return aao::status_from_hip(h, aao::launch_grad_logkappa(h, x, lam, g, h->stream), "grad_logkappa");
}

const char* aao_last_error(const aao_problem* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// Host-side setup: Radau IIA tableau, Crout factor for Rana's stage
// preconditioner, 1D Galerkin factors of the multigrid hierarchy, and face
// diffusivities.  No device code.
#include <algorithm>
#include <cmath>
#include <vector>

#include "aao_internal.h"

namespace aao {

namespace {

// Legendre polynomial P_k(t) by the three-term recurrence.
double legendre(int k, double t) {
  if (k == 0) return 1.0;
  double p0 = 1.0, p1 = t;
  for (int m = 1; m < k; ++m) {
    double p2 = ((2.0 * m + 1.0) * t * p1 - m * p0) / (m + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Right Radau polynomial on [-1, 1]: its zeros map to the Radau IIA nodes.
double radau_poly(int s, double t) { return legendre(s, t) - legendre(s - 1, t); }

// Solve the dense s x s system M x = r in place (partial pivoting).
bool dense_solve(int s, std::vector<double> M, std::vector<double>& r) {
  for (int k = 0; k < s; ++k) {
    int piv = k;
    for (int i = k + 1; i < s; ++i)
      if (std::fabs(M[i * s + k]) > std::fabs(M[piv * s + k])) piv = i;
    if (M[piv * s + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < s; ++j) std::swap(M[k * s + j], M[piv * s + j]);
      std::swap(r[k], r[piv]);
    }
    for (int i = k + 1; i < s; ++i) {
      double f = M[i * s + k] / M[k * s + k];
      for (int j = k; j < s; ++j) M[i * s + j] -= f * M[k * s + j];
      r[i] -= f * r[k];
    }
  }
  for (int k = s - 1; k >= 0; --k) {
    double acc = r[k];
    for (int j = k + 1; j < s; ++j) acc -= M[k * s + j] * r[j];
    r[k] = acc / M[k * s + k];
  }
  return true;
}

}  // namespace

// Radau IIA: nodes are the zeros of P_s(t) - P_{s-1}(t) mapped by x = (1+t)/2
// (the last one is x = 1); the coefficients satisfy the collocation
// conditions sum_j a_ij c_j^{q-1} = c_i^q / q, q = 1..s; b = last row of A.
bool radau_iia(int s, double* A, double* b, double* c) {
  if (s < 1 || s > SMAX) return false;
  std::vector<double> nodes;
  const int samples = 20000;
  double tprev = -1.0, fprev = radau_poly(s, tprev);
  for (int k = 1; k <= samples && (int)nodes.size() < s - 1; ++k) {
    double t = -1.0 + 2.0 * k / samples * (1.0 - 1e-6);
    double f = radau_poly(s, t);
    if (fprev == 0.0) {
      nodes.push_back(tprev);
    } else if (fprev * f < 0.0) {
      double lo = tprev, hi = t, flo = fprev;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), fm = radau_poly(s, mid);
        if (fm == 0.0) { lo = hi = mid; break; }
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      nodes.push_back(0.5 * (lo + hi));
    }
    tprev = t;
    fprev = f;
  }
  if ((int)nodes.size() != s - 1) return false;
  nodes.push_back(1.0);
  for (int i = 0; i < s; ++i) c[i] = 0.5 * (1.0 + nodes[i]);
  c[s - 1] = 1.0;
  // collocation: rows i of A from the transposed Vandermonde system
  std::vector<double> Vt(s * s);
  for (int q = 0; q < s; ++q)
    for (int j = 0; j < s; ++j) Vt[q * s + j] = std::pow(c[j], q);
  for (int i = 0; i < s; ++i) {
    std::vector<double> r(s);
    for (int q = 0; q < s; ++q) r[q] = std::pow(c[i], q + 1) / (q + 1);
    if (!dense_solve(s, Vt, r)) return false;
    for (int j = 0; j < s; ++j) A[i * s + j] = r[j];
  }
  for (int j = 0; j < s; ++j) b[j] = A[(s - 1) * s + j];
  return true;
}

// Crout: A = L U with U unit upper triangular; returns L (row-major s x s).
void crout_lower(int s, const double* A, double* L) {
  std::vector<double> U(s * s, 0.0);
  for (int i = 0; i < s * s; ++i) L[i] = 0.0;
  for (int i = 0; i < s; ++i) U[i * s + i] = 1.0;
  for (int j = 0; j < s; ++j) {
    for (int i = j; i < s; ++i) {
      double acc = A[i * s + j];
      for (int k = 0; k < j; ++k) acc -= L[i * s + k] * U[k * s + j];
      L[i * s + j] = acc;
    }
    for (int i = j + 1; i < s; ++i) {
      double acc = A[j * s + i];
      for (int k = 0; k < j; ++k) acc -= L[j * s + k] * U[k * s + i];
      U[j * s + i] = acc / L[j * s + j];
    }
  }
}

// 1D Galerkin factors of the hierarchy.  Level 0: M_0 = I,
// T_0 = tridiag(-1, 2, -1)/h^2 on n nodes for finite differences (fe = 0);
// for bilinear elements (fe = 1) the 1D mass and stiffness matrices
// M_0 = h tridiag(1/6, 2/3, 1/6), T_0 = tridiag(-1, 2, -1)/h; for
// biquadratic elements (fe = 2, n odd, element side H = 2h) the quadratic
// ones, whose rows at element vertices (odd 0-based index) couple five
// nodes, M: H/30 (-1, 2, 8, 2, -1), T: (1, -8, 14, -8, 1)/(3H), and whose
// rows at edge midpoints couple three, M: H/30 (2, 16, 2), T: (-8, 16, -8)/(3H).
// The tensor form M(x)M + a (T(x)M + M(x)T) of these is the finite-element
// matrix M + a K.  Coarse nodes are the fine nodes 2, 4, ..., 2 floor(n/2)
// (1-based; for Q2 the element vertices), P is linear interpolation (zero
// boundary values), and M_{l+1} = P^T M_l P / 2, T_{l+1} = P^T T_l P / 2, so
// that in d dimensions R = P^T / 2^d and the Galerkin operator R A_l P of
// A_l = M(x)M + a (T(x)M + M(x)T) is again of that form; from level 1 on the
// factors are tridiagonal (for Q2 a midpoint row, the only one reaching a
// vertex two nodes away, never lies under two coarse nodes' supports).
// Coarsening stops once a level has at most coarse_max nodes (that level is
// solved exactly); Q2 coarsens at least once, so that level 0 is never the
// exactly solved one.
// tri[l] = [Mlo, Md, Mup, Tlo, Td, Tup], each n_l long; for Q2, tri[0] =
// [M(i,i-2), .., M(i,i+2), T(i,i-2), .., T(i,i+2)], ten arrays of n.
void galerkin_1d(int n, int dim, double h, int coarse_max, int fe, std::vector<int>& sizes,
                 std::vector<std::vector<double>>& tri) {
  sizes.assign(1, n);
  int nf = n;
  std::vector<double> M(nf * nf, 0.0), T(nf * nf, 0.0);
  int band = 1;
  if (fe == 2) {
    band = 2;
    const double H = 2.0 * h;
    static const double mv[5] = {-1, 2, 8, 2, -1}, tv[5] = {1, -8, 14, -8, 1};
    static const double mm[5] = {0, 2, 16, 2, 0}, tm[5] = {0, -8, 16, -8, 0};
    for (int i = 0; i < nf; ++i) {
      const bool vertex = i & 1;
      for (int d = -2; d <= 2; ++d) {
        if (i + d < 0 || i + d >= nf) continue;
        M[i * nf + i + d] = H / 30.0 * (vertex ? mv : mm)[d + 2];
        T[i * nf + i + d] = (vertex ? tv : tm)[d + 2] / (3.0 * H);
      }
    }
  } else {
    const double ts = fe ? 1.0 / h : 1.0 / (h * h);
    for (int i = 0; i < nf; ++i) {
      M[i * nf + i] = fe ? 2.0 * h / 3.0 : 1.0;
      if (fe && i > 0) M[i * nf + i - 1] = h / 6.0;
      if (fe && i + 1 < nf) M[i * nf + i + 1] = h / 6.0;
      T[i * nf + i] = 2.0 * ts;
      if (i > 0) T[i * nf + i - 1] = -ts;
      if (i + 1 < nf) T[i * nf + i + 1] = -ts;
    }
  }
  auto pack = [](const std::vector<double>& Mx, const std::vector<double>& Tx, int m) {
    std::vector<double> t(6 * m, 0.0);
    for (int i = 0; i < m; ++i) {
      t[0 * m + i] = i > 0 ? Mx[i * m + i - 1] : 0.0;
      t[1 * m + i] = Mx[i * m + i];
      t[2 * m + i] = i + 1 < m ? Mx[i * m + i + 1] : 0.0;
      t[3 * m + i] = i > 0 ? Tx[i * m + i - 1] : 0.0;
      t[4 * m + i] = Tx[i * m + i];
      t[5 * m + i] = i + 1 < m ? Tx[i * m + i + 1] : 0.0;
    }
    return t;
  };
  auto pack5 = [](const std::vector<double>& Mx, const std::vector<double>& Tx, int m) {
    std::vector<double> t(10 * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int d = -2; d <= 2; ++d) {
        if (i + d < 0 || i + d >= m) continue;
        t[(d + 2) * m + i] = Mx[i * m + i + d];
        t[(d + 7) * m + i] = Tx[i * m + i + d];
      }
    return t;
  };
  tri.assign(1, band == 2 ? pack5(M, T, nf) : pack(M, T, nf));
  auto npow = [dim](int m) { double v = 1.0; for (int a = 0; a < dim; ++a) v *= m; return v; };
  while ((npow(nf) > coarse_max || (fe == 2 && sizes.size() == 1)) && nf > 1) {
    int nc = nf / 2;
    // P: nf x nc, coarse J at fine 2J+1 (0-based), neighbours 2J and 2J+2
    std::vector<double> P(nf * nc, 0.0);
    for (int J = 0; J < nc; ++J) {
      int f = 2 * J + 1;
      P[f * nc + J] = 1.0;
      P[(f - 1) * nc + J] = 0.5;
      if (f + 1 < nf) P[(f + 1) * nc + J] = 0.5;
    }
    auto rap = [&](const std::vector<double>& X) {
      std::vector<double> XP(nf * nc, 0.0), out(nc * nc, 0.0);
      for (int i = 0; i < nf; ++i)
        for (int k = std::max(0, i - band); k <= std::min(nf - 1, i + band); ++k) {
          double x = X[i * nf + k];
          if (x == 0.0) continue;
          for (int J = 0; J < nc; ++J) XP[i * nc + J] += x * P[k * nc + J];
        }
      for (int I = 0; I < nc; ++I)
        for (int i = 0; i < nf; ++i) {
          double p = P[i * nc + I];
          if (p == 0.0) continue;
          for (int J = 0; J < nc; ++J) out[I * nc + J] += 0.5 * p * XP[i * nc + J];
        }
      return out;
    };
    std::vector<double> Mc = rap(M), Tc = rap(T);
    sizes.push_back(nc);
    tri.push_back(pack(Mc, Tc, nc));
    M.swap(Mc);
    T.swap(Tc);
    nf = nc;
    band = 1;
  }
}

// Generalized eigenvectors of the pair (T, M) of 1D factors of one level
// (both symmetric tridiagonal, M positive definite): T V = M V diag(lam) with
// V^T M V = I.  Then M(x)M + a (T(x)M + M(x)T) = (V(x)V)^{-T} D (V(x)V)^{-1}
// with D = I + a (lam(x)1 + 1(x)lam), so its inverse is applied by four
// small matrix products and a diagonal scaling (fast diagonalization, Lynch,
// Rice and Thomas 1964).  Computed as V = L^{-T} Q with M = L L^T and Q the
// eigenvectors of L^{-1} T L^{-T} by cyclic Jacobi rotations.  V is returned
// row-major (V[i n + k] = component i of vector k).
bool tensor_eigen(int n, const std::vector<double>& tri, std::vector<double>& V, std::vector<double>& lam) {
  std::vector<double> M((size_t)n * n, 0.0), T((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int d = -1; d <= 1; ++d) {
      const int j = i + d;
      if (j < 0 || j >= n) continue;
      M[(size_t)i * n + j] = tri[(1 + d) * n + i];
      T[(size_t)i * n + j] = tri[(4 + d) * n + i];
    }
  // Cholesky M = L L^T
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    L[(size_t)j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / L[(size_t)j * n + j];
    }
  }
  // Linv = L^{-1} (lower triangular)
  std::vector<double> Li((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * Li[(size_t)k * n + c];
      Li[(size_t)i * n + c] = v / L[(size_t)i * n + i];
    }
  // C = Linv T Linv^T
  std::vector<double> W((size_t)n * n, 0.0), C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += Li[(size_t)i * n + k] * T[(size_t)k * n + j];
      W[(size_t)i * n + j] = v;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += W[(size_t)i * n + k] * Li[(size_t)j * n + k];
      C[(size_t)i * n + j] = v;
    }
  // cyclic Jacobi: C = Q diag Q^T
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double c2 = C[(size_t)i * n + j] * C[(size_t)i * n + j];
        tot += c2;
        if (i != j) off += c2;
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {   // C <- C J (columns p, q)
          const double ckp = C[(size_t)k * n + p], ckq = C[(size_t)k * n + q];
          C[(size_t)k * n + p] = c * ckp - sn * ckq;
          C[(size_t)k * n + q] = sn * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {   // C <- J^T C (rows p, q)
          const double cpk = C[(size_t)p * n + k], cqk = C[(size_t)q * n + k];
          C[(size_t)p * n + k] = c * cpk - sn * cqk;
          C[(size_t)q * n + k] = sn * cpk + c * cqk;
        }
        for (int k = 0; k < n; ++k) {   // Q <- Q J
          const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = c * qkp - sn * qkq;
          Q[(size_t)k * n + q] = sn * qkp + c * qkq;
        }
      }
  }
  lam.assign(n, 0.0);
  for (int k = 0; k < n; ++k) lam[k] = C[(size_t)k * n + k];
  // V = L^{-T} Q
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double v = 0.0;
      for (int m = 0; m < n; ++m) v += Li[(size_t)m * n + i] * Q[(size_t)m * n + k];
      V[(size_t)i * n + k] = v;
    }
  return true;
}

// Galerkin stencils of K on the coarse levels for variable diffusivity (2D).
// K_0 is the 5-point operator with the face diffusivities (scaled by 1/h^2);
// K_{l+1} = P^T K_l P / 4 with the tensor-linear interpolation P of
// galerkin_1d (coarse node J at fine 2J+1, weights 1/2, 1, 1/2), so level l
// applies I-part M_l (x) M_l (from the 1D factors) plus a K_l.  A 9-point
// stencil stays 9-point under this product.  st9[l] (l >= 1) holds 9 N_l
// values: entry (dj+1)*3 + (di+1) of node p at [((dj+1)*3 + di+1) N_l + p];
// st9[0] is left empty (the fine level applies the faces directly).
void galerkin_stencils_2d(const std::vector<int>& sizes, const std::vector<double>& faces, double ih2,
                          std::vector<std::vector<double>>& st9) {
  const int L = (int)sizes.size();
  st9.assign(L, {});
  int n = sizes[0];
  int64_t N = (int64_t)n * n;
  std::vector<double> K((size_t)9 * N, 0.0);
  for (int64_t p = 0; p < N; ++p) {
    const int i = (int)(p % n), j = (int)(p / n);
    const double m0 = faces[p], p0 = faces[N + p], m1 = faces[2 * N + p], p1 = faces[3 * N + p];
    K[4 * N + p] = ih2 * (m0 + p0 + m1 + p1);
    if (i > 0) K[3 * N + p] = -ih2 * m0;
    if (i + 1 < n) K[5 * N + p] = -ih2 * p0;
    if (j > 0) K[1 * N + p] = -ih2 * m1;
    if (j + 1 < n) K[7 * N + p] = -ih2 * p1;
  }
  // coarse nodes whose interpolation reaches fine index i, with weights
  auto coarse_of = [](int i, int nc, int* I, double* w) {
    if (i & 1) {
      I[0] = (i - 1) / 2;
      w[0] = 1.0;
      return 1;
    }
    int c = 0;
    if (i / 2 - 1 >= 0) { I[c] = i / 2 - 1; w[c] = 0.5; ++c; }
    if (i / 2 < nc) { I[c] = i / 2; w[c] = 0.5; ++c; }
    return c;
  };
  for (int l = 1; l < L; ++l) {
    const int nc = sizes[l];
    const int64_t Nc = (int64_t)nc * nc;
    std::vector<double> Kc((size_t)9 * Nc, 0.0);
    for (int64_t f = 0; f < N; ++f) {
      const int i = (int)(f % n), j = (int)(f / n);
      int Ix[2], Jy[2];
      double wx[2], wy[2];
      const int cxn = coarse_of(i, nc, Ix, wx), cyn = coarse_of(j, nc, Jy, wy);
      if (cxn == 0 || cyn == 0) continue;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const double kv = K[(size_t)((dj + 1) * 3 + di + 1) * N + f];
          if (kv == 0.0) continue;
          const int gi = i + di, gj = j + dj;
          int Gx[2], Gy[2];
          double gx[2], gy[2];
          const int gxn = coarse_of(gi, nc, Gx, gx), gyn = coarse_of(gj, nc, Gy, gy);
          for (int a = 0; a < cyn; ++a)
            for (int b = 0; b < cxn; ++b) {
              const int64_t C = (int64_t)Jy[a] * nc + Ix[b];
              const double wf = 0.25 * wy[a] * wx[b] * kv;
              for (int c = 0; c < gyn; ++c)
                for (int e = 0; e < gxn; ++e) {
                  const int dJ = Gy[c] - Jy[a], dI = Gx[e] - Ix[b];
                  Kc[(size_t)((dJ + 1) * 3 + dI + 1) * Nc + C] += wf * gy[c] * gx[e];
                }
            }
        }
    }
    st9[l] = Kc;
    K.swap(Kc);
    n = nc;
    N = Nc;
  }
}

// Dense inverse of the coarsest level's operator, stored transposed
// (invT[c * Nc + r] = (A^{-1})_{rc}) so that threads reading consecutive rows
// read consecutive addresses.  The operator is the tensor Galerkin form
// M(x)M(x..) + a sum T(x)M.. built from the level's 1D factors; when the
// coarsest level is the fine level it is I + a K with the face diffusivities
// (faces may be null for kappa = 1); with a Galerkin stencil st9 of K (2D,
// variable kappa) it is M(x)M + a K.
bool coarse_inverse(int dim, int n, const std::vector<double>& tri, double a, bool fine, double ih2,
                    const double* faces, const double* st9, std::vector<double>& invT) {
  int N = 1;
  for (int d = 0; d < dim; ++d) N *= n;
  std::vector<double> A((size_t)N * N, 0.0);
  auto m1 = [&](int q, int i) { return tri[q * n + i]; };   // q: 0 lo, 1 d, 2 up (M); 3..5 (T)
  auto coord = [&](int p, int* c) { c[0] = p % n; c[1] = (p / n) % n; c[2] = dim == 3 ? p / (n * n) : 0; };
  for (int p = 0; p < N; ++p) {
    int c[3];
    coord(p, c);
    for (int q = 0; q < N; ++q) {
      int e[3];
      coord(q, e);
      bool near = true;
      int off[3] = {0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        off[d] = e[d] - c[d];
        if (off[d] < -1 || off[d] > 1) near = false;
      }
      if (!near) continue;
      double v;
      if (fine) {
        int nz = 0;
        for (int d = 0; d < dim; ++d) nz += off[d] != 0;
        if (nz > 1) continue;
        if (nz == 0) {
          double sum = 0.0;
          for (int d = 0; d < dim; ++d)
            sum += faces ? faces[(size_t)(2 * d) * N + p] + faces[(size_t)(2 * d + 1) * N + p] : 2.0;
          v = 1.0 + a * ih2 * sum;
        } else {
          int d = 0;
          while (off[d] == 0) ++d;
          const double f = faces ? faces[(size_t)(2 * d + (off[d] > 0 ? 1 : 0)) * N + p] : 1.0;
          v = -a * ih2 * f;
        }
      } else if (st9) {      // 2D Galerkin level with a stencil for K
        const double mm = m1(1 + off[0], c[0]) * m1(1 + off[1], c[1]);
        v = mm + a * st9[(size_t)((off[1] + 1) * 3 + off[0] + 1) * N + p];
      } else {
        double mm = 1.0, sumT = 0.0;
        for (int d = 0; d < dim; ++d) mm *= m1(1 + off[d], c[d]);
        for (int d = 0; d < dim; ++d) {
          double t = m1(4 + off[d], c[d]);
          for (int d2 = 0; d2 < dim; ++d2)
            if (d2 != d) t *= m1(1 + off[d2], c[d2]);
          sumT += t;
        }
        v = mm + a * sumT;
      }
      A[(size_t)p * N + q] = v;
    }
  }
  // Gauss-Jordan with partial pivoting
  std::vector<double> inv((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i) inv[(size_t)i * N + i] = 1.0;
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (std::fabs(A[(size_t)i * N + k]) > std::fabs(A[(size_t)piv * N + k])) piv = i;
    if (A[(size_t)piv * N + k] == 0.0) return false;
    if (piv != k)
      for (int j = 0; j < N; ++j) {
        std::swap(A[(size_t)k * N + j], A[(size_t)piv * N + j]);
        std::swap(inv[(size_t)k * N + j], inv[(size_t)piv * N + j]);
      }
    const double dk = 1.0 / A[(size_t)k * N + k];
    for (int j = 0; j < N; ++j) {
      A[(size_t)k * N + j] *= dk;
      inv[(size_t)k * N + j] *= dk;
    }
    for (int i = 0; i < N; ++i) {
      if (i == k) continue;
      const double f = A[(size_t)i * N + k];
      if (f == 0.0) continue;
      for (int j = 0; j < N; ++j) {
        A[(size_t)i * N + j] -= f * A[(size_t)k * N + j];
        inv[(size_t)i * N + j] -= f * inv[(size_t)k * N + j];
      }
    }
  }
  invT.assign((size_t)N * N, 0.0);
  for (int r = 0; r < N; ++r)
    for (int cidx = 0; cidx < N; ++cidx) invT[(size_t)cidx * N + r] = inv[(size_t)r * N + cidx];
  return true;
}

// Face diffusivities (not divided by h^2): harmonic mean between interior
// nodes, the node's own value on faces to the boundary.
// faces[(2a) N + p] = minus side of p along axis a, faces[(2a+1) N + p] = plus side.
void face_coefficients(int dim, int n, const double* kappa, std::vector<double>& faces) {
  int64_t N = 1;
  for (int a = 0; a < dim; ++a) N *= n;
  faces.assign((size_t)2 * dim * N, 0.0);
  int64_t strides[3] = {1, n, (int64_t)n * n};
  for (int64_t p = 0; p < N; ++p) {
    int64_t coord[3] = {p % n, (p / n) % n, dim == 3 ? p / ((int64_t)n * n) : 0};
    for (int a = 0; a < dim; ++a) {
      double kp = kappa[p];
      double km = coord[a] > 0 ? kappa[p - strides[a]] : kp;
      double kq = coord[a] + 1 < n ? kappa[p + strides[a]] : kp;
      faces[(2 * a) * N + p] = coord[a] > 0 ? 2.0 * kp * km / (kp + km) : kp;
      faces[(2 * a + 1) * N + p] = coord[a] + 1 < n ? 2.0 * kp * kq / (kp + kq) : kp;
    }
  }
}

}  // namespace aao

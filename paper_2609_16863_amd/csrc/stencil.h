// Device helpers shared by the kernels: grid coordinates, the 5/7-point
// operator K = -div(kappa grad)_h (times h^2), and compile-time dispatch.
#pragma once

#include "aao_internal.h"

namespace aao {

template <int DIM>
__device__ __forceinline__ void node_coords(int p, int n, int& i, int& j, int& k) {
  if (DIM == 2) {
    j = p / n;
    i = p - j * n;
    k = 0;
  } else {
    const int nn = n * n;
    k = p / nn;
    const int r = p - k * nn;
    j = r / n;
    i = r - j * n;
  }
}

// h^2 (K f)_p for the field f (values outside the grid are zero).
template <int DIM, bool VK, class T, class C>
__device__ __forceinline__ C stencil_K(const T* __restrict__ f, int p, int i, int j, int k, int n,
                                       int N, const Faces<C>& fc) {
  const C c0 = ld<T, C>(f + p);
  const C xm = i > 0 ? ld<T, C>(f + p - 1) : C(0);
  const C xp = i + 1 < n ? ld<T, C>(f + p + 1) : C(0);
  const C ym = j > 0 ? ld<T, C>(f + p - n) : C(0);
  const C yp = j + 1 < n ? ld<T, C>(f + p + n) : C(0);
  C zm = C(0), zp = C(0);
  if (DIM == 3) {
    const int nn = n * n;
    zm = k > 0 ? ld<T, C>(f + p - nn) : C(0);
    zp = k + 1 < n ? ld<T, C>(f + p + nn) : C(0);
  }
  if (!VK) {
    C acc = C(2 * DIM) * c0 - xm - xp - ym - yp;
    if (DIM == 3) acc -= zm + zp;
    return acc;
  }
  C acc = fc.m[0][p] * (c0 - xm) + fc.p[0][p] * (c0 - xp) + fc.m[1][p] * (c0 - ym) +
          fc.p[1][p] * (c0 - yp);
  if (DIM == 3) acc += fc.m[2][p] * (c0 - zm) + fc.p[2][p] * (c0 - zp);
  return acc;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8, each XCD with its own L2).  xcd_tile(b, B) is the logical
// tile of workgroup b of B such that each XCD walks one contiguous range of
// logical tiles: tiles that share halo lines (neighbours in the same block)
// then meet in one L2.  A bijection on [0, B).
constexpr int NXCD = 8;

__device__ __forceinline__ int xcd_tile(int b, int B) {
  const int q = B / NXCD, r = B % NXCD, k = b % NXCD;
  return k * q + (k < r ? k : r) + b / NXCD;
}

// Diagonal of h^2 K at p.
template <int DIM, bool VK, class C>
__device__ __forceinline__ C stencil_K_diag(int p, const Faces<C>& fc) {
  if (!VK) return C(2 * DIM);
  C d = fc.m[0][p] + fc.p[0][p] + fc.m[1][p] + fc.p[1][p];
  if (DIM == 3) d += fc.m[2][p] + fc.p[2][p];
  return d;
}

}  // namespace aao

// Dispatch a macro M(DIM, S, VK) over the runtime (dim, s, vark).
#define DISPATCH_DSV(dim_, s_, vk_, M)              \
  do {                                              \
    if ((dim_) == 2) {                              \
      if (vk_) {                                    \
        if ((s_) == 1) M(2, 1, true);               \
        else if ((s_) == 2) M(2, 2, true);          \
        else M(2, 3, true);                         \
      } else {                                      \
        if ((s_) == 1) M(2, 1, false);              \
        else if ((s_) == 2) M(2, 2, false);         \
        else M(2, 3, false);                        \
      }                                             \
    } else {                                        \
      if (vk_) {                                    \
        if ((s_) == 1) M(3, 1, true);               \
        else if ((s_) == 2) M(3, 2, true);          \
        else M(3, 3, true);                         \
      } else {                                      \
        if ((s_) == 1) M(3, 1, false);              \
        else if ((s_) == 2) M(3, 2, false);         \
        else M(3, 3, false);                        \
      }                                             \
    }                                               \
  } while (0)

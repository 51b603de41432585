// Shared device-side helpers for the polyspectrum kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ps {

template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
// multiply by +i (s > 0) or -i (s < 0)
template <typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a, int s) {
  return s > 0 ? cplx<T>{-a.im, a.re} : cplx<T>{a.im, -a.re};
}

// Geometry of the pruned transforms.  The ball of modes with |q| < K_e is held in
// a dense "box" of (2Kc+1) x (Kc+1) x (2Kc+1) complex values indexed
// [a = q0 + Kc][c = q2][e = q1 + Kc] (half space q2 >= 0), Kc the largest integer
// component below K_e.  Intermediates between 1-D passes:
//   H1[z][x1][c][a]   (after the q1 -> x1 transform),  N * B2 * B0 values
//   H2[z][x0][x1][c]  (after the q0 -> x0 transform),  N * N * H2s values: rows of B2
//                     entries at a stride H2s of B2 rounded up to 16, so that the runs of
//                     16 consecutive c written by the q0 -> x0 pass are whole 128-byte lines
// A slab restricts the last two transforms to the planes x1_0 <= x1 < x1_0 + S1 (the
// whole grid is the slab x1_0 = 0, S1 = N): H2 and the real output then hold S1
// planes, [z][x0][x1 - x1_0][c] and [z][x0][x1 - x1_0][x2].
// z enumerates (batch, shell) pairs of one launch: batch = z / spb, shell =
// shell_base + z % spb (spb = shells per batch; spb = 0 means one unmasked field
// per batch, batch = z, shell 0).
struct Geom {
  int N;
  int Kc;
  int B0;   // 2Kc+1 (also the q1 extent of the box)
  int B2;   // Kc+1
  int H2s;  // row stride of H2: B2 rounded up to a multiple of 16
  int spb;
  int shell_base;
  int n_shells;
  int S1;     // x1 planes of the slab (N for the whole grid)
  int x1_0;   // first x1 plane of the slab
  int fold;   // fields per shell set: field f of a batch is shell shell_base + f % fold
  int ell;    // multipole plans: fields f >= fold carry the weight L_ell(mu); -1 otherwise
};

__device__ __forceinline__ int geom_shell(const Geom& g, int z) {
  return g.spb > 0 ? g.shell_base + (z % g.spb) % g.fold : 0;
}
// Multipole plans: whether field z is the Legendre-weighted copy of its shell.
__device__ __forceinline__ bool geom_weighted(const Geom& g, int z) {
  return g.ell >= 0 && g.spb > 0 && (z % g.spb) >= g.fold;
}
// Legendre polynomial L_ell(mu) by the three-term recurrence.
template <typename T>
__device__ __forceinline__ T legendre(int ell, T mu) {
  T p0 = (T)1, p1 = mu;
  if (ell == 0) return p0;
  for (int n = 1; n < ell; ++n) {
    const T p2 = ((T)(2 * n + 1) * mu * p1 - (T)n * p0) / (T)(n + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}
__device__ __forceinline__ int geom_batch(const Geom& g, int z) {
  return g.spb > 0 ? z / g.spb : z;
}

}  // namespace ps

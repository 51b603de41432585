// Stockham FFT building blocks shared by the transform passes and the fused
// epilogue of the adjoint: small DFTs, the padded LDS pencil layout, per-stage
// twiddle tables and a full length-N transform of P pencils by NT threads.
#pragma once

#include "common.h"

namespace ps {

constexpr int kFftThreads = 256;

// ---------------------------------------------------------------------------
// small DFTs, X[r] = sum_t x[t] exp(S * 2 pi i r t / R), S = +1 (inverse) or -1
// ---------------------------------------------------------------------------
template <typename T, int S>
__device__ __forceinline__ void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, int S>
__device__ __forceinline__ void dft4(cplx<T>& x0, cplx<T>& x1, cplx<T>& x2, cplx<T>& x3) {
  cplx<T> a = cadd(x0, x2), b = csub(x0, x2);
  cplx<T> c = cadd(x1, x3), d = cmul_i(csub(x1, x3), S);
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, d);
  x3 = csub(b, d);
}

template <typename T, int S>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, S>(e0, e1, e2, e3);
  dft4<T, S>(o0, o1, o2, o3);
  const T h = (T)0.70710678118654752440084436210484903928;
  // w8^r = exp(S 2 pi i r / 8)
  cplx<T> t1 = cmul(o1, cplx<T>{h, (T)S * h});
  cplx<T> t2 = cmul_i(o2, S);
  cplx<T> t3 = cmul(o3, cplx<T>{-h, (T)S * h});
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

template <typename T, int S, int R>
__device__ __forceinline__ void dftR(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, S>(v);
  else if constexpr (R == 4) dft4<T, S>(v[0], v[1], v[2], v[3]);
  else dft8<T, S>(v);
}

// LDS position of element i of a pencil: one pad slot after every 8 elements, so the
// stride-8 writes of the first radix-8 stage fall in distinct banks.
__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }

// Pencil stride in LDS: padded length plus one, so that neighbouring pencils start
// in different banks.
template <int N>
constexpr int pencil_stride() { return N + N / 8 + 1; }

// Twiddles of every stage but the first (whose twiddles are all 1), laid out
// [stage][r - 1][k] so that lanes handling consecutive k read consecutive words.
template <int N>
constexpr int stage_tw_size() {
  int l2 = 0;
  while ((1 << l2) < N) ++l2;
  int p = 1, tot = 0;
  for (int s = 0; s < l2 / 3; ++s) {
    if (p > 1) tot += 7 * p;
    p *= 8;
  }
  if (l2 % 3) tot += (l2 % 3 == 2 ? 3 : 1) * p;
  return tot;
}

template <typename T, int N, int NT = kFftThreads>
__device__ __forceinline__ void build_stage_twiddles(cplx<T>* stw, const cplx<T>* __restrict__ tw) {
  constexpr int L2 = __builtin_ctz(N), N8 = L2 / 3, REM = L2 % 3;
  int off = 0, p = 1;
  for (int st = 0; st < N8; ++st) {
    if (p > 1) {
      for (int i = threadIdx.x; i < 7 * p; i += NT) {
        const int r = i / p + 1, k = i % p;
        stw[off + i] = tw[k * r * (N / (p * 8))];
      }
      off += 7 * p;
    }
    p *= 8;
  }
  if constexpr (REM != 0) {
    constexpr int R = REM == 2 ? 4 : 2;
    for (int i = threadIdx.x; i < (R - 1) * p; i += NT) {
      const int r = i / p + 1, k = i % p;
      stw[off + i] = tw[k * r * (N / (p * R))];
    }
  }
}

// One Stockham stage of radix R over P pencils of length N stored with stride NS.
// After the stage every run of p*R consecutive outputs is a finished sub-DFT.
// tws: this stage's twiddle table, entry (r - 1) * p + k = exp(2 pi i k r / (p R)).
template <typename T, int N, int P, int NS, int R, int S, int NT = kFftThreads>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int p, const cplx<T>* tws) {
  constexpr int NB = N / R;
  constexpr int BPT = (P * NB) / NT;
  static_assert(BPT >= 1 && (P * NB) % NT == 0, "block shape");
  cplx<T> v[BPT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    const int pen = b / NB, i = b % NB;
    const int k = i & (p - 1);
    const cplx<T>* base = buf + pen * NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx<T> x = base[pad8(i + r * NB)];
      if (r > 0 && p > 1) {
        cplx<T> w = tws[(r - 1) * p + k];
        if (S < 0) w.im = -w.im;
        x = cmul(x, w);
      }
      v[u][r] = x;
    }
    dftR<T, S, R>(v[u]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int b = tid + u * NT;
    const int pen = b / NB, i = b % NB;
    const int k = i & (p - 1);
    const int j = (i - k) * R + k;
    cplx<T>* base = buf + pen * NS;
#pragma unroll
    for (int r = 0; r < R; ++r) base[pad8(j + r * p)] = v[u][r];
  }
  __syncthreads();
}

// Full length-N transform of the P pencils in buf (caller has synchronised).
template <typename T, int N, int P, int NS, int S, int NT = kFftThreads>
__device__ __forceinline__ void fft_block(cplx<T>* buf, const cplx<T>* stw) {
  int p = 1, off = 0;
  constexpr int L2 = __builtin_ctz(N);
  constexpr int N8 = L2 / 3;
  constexpr int REM = L2 % 3;
#pragma unroll
  for (int st = 0; st < N8; ++st) {
    fft_stage<T, N, P, NS, 8, S, NT>(buf, p, stw + off);
    if (p > 1) off += 7 * p;
    p *= 8;
  }
  if constexpr (REM == 2) fft_stage<T, N, P, NS, 4, S, NT>(buf, p, stw + off);
  if constexpr (REM == 1) fft_stage<T, N, P, NS, 2, S, NT>(buf, p, stw + off);
}

}  // namespace ps

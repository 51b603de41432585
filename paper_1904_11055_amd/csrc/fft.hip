// Pruned, batched 3-D FFT passes for shell fields (gfx950).
//
// A shell field d_s[x] = sum_q [s(q) = s] delta_hat[q] e^{+2 pi i q.x/N} is the
// unnormalised inverse transform of the density restricted to one spherical shell
// (the paper's I_k(x), Sec. 2; FFTW(I~) in Appendix A).  Only the ball |q| < K_e is
// non-zero, so the inverse 3-D transform runs as three 1-D passes that never touch
// the empty part of the spectrum:
//   P1  q1 -> x1 on the (2Kc+1)(Kc+1) columns that meet the shell (masked gather),
//   P2  q0 -> x0 on N (Kc+1) pencils,
//   P3  q2 -> x2 complex-to-real on N^2 rows, two rows per complex transform.
// The forward (real-to-complex) direction runs the same passes in reverse and keeps
// only the ball (input transform) or only one shell's modes (adjoint).
//
// Every block transforms P pencils of length N held in LDS (pencil stride N+1 to
// spread banks) with a Stockham autosort FFT of radix-8 stages plus one radix-4 or
// radix-2 stage; twiddles exp(2 pi i e / N) come from a table computed on the host
// in double precision.
#include "common.h"
#include "fft_core.h"

namespace ps {

constexpr int kAbsmaxSpread = 256;   // partial maxima per field (spreads the atomics)

// Complex values held by one block: column passes (P1, P2, Q2, Q1) take more
// pencils per block so that their strided global accesses come in longer runs;
// row passes (P3, Q3) take fewer, for more resident blocks per CU.
template <typename T>
struct FftCfg;
template <>
struct FftCfg<float> {
  static constexpr int kElems = 4096;
  static constexpr int kColElems = 8192;   // P2: 16 pencils at N = 512, so runs of 128 bytes
  static constexpr int kRowElems = 2048;
};
template <>
struct FftCfg<double> {
  static constexpr int kElems = 2048;
  static constexpr int kColElems = 2048;
  static constexpr int kRowElems = 2048;
};

__device__ __forceinline__ int freq_of(int n, int N) { return n < N / 2 ? n : n - N; }

// ---------------------------------------------------------------------------
// Inverse direction (ball -> real grid)
// ---------------------------------------------------------------------------

// P1: columns (a, c) of the box, transform q1 -> x1, masked by shell s(z).
// UNIT: the input is the unit shell (1 inside, 0 outside) instead of the box.
// Multipole plans: the weighted fields also take L_ell(mu), mu = q2 / |q| (the line of
// sight along the third axis; q2 is the column index c).
// grid (ceil(B0/P), B2, nz)
template <typename T, int N, bool UNIT>
__global__ __launch_bounds__(kFftThreads) void c2r_p1(const cplx<float>* __restrict__ box,
                                                      const int16_t* __restrict__ shell_of_q,
                                                      const int* __restrict__ qmax,
                                                      cplx<T>* __restrict__ H1,
                                                      const cplx<T>* __restrict__ tw, Geom g) {
  constexpr int P = FftCfg<T>::kElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int s = geom_shell(g, z);
  const int b = geom_batch(g, z);
  const bool weighted = !UNIT && geom_weighted(g, z);
  const int a0 = blockIdx.x * P;
  const int c = blockIdx.y;
  const int Kc = g.Kc;
  const int qm = qmax[s];
  {
    // columns of the block that miss the shell's outer sphere are never read by P2
    const int qa = a0 - Kc, qb = min(a0 + P - 1, g.B0 - 1) - Kc;
    const int qmin0 = (qa <= 0 && qb >= 0) ? 0 : min(qa * qa, qb * qb);
    if (qmin0 + c * c > qm) return;
  }
  const size_t box_sz = (size_t)g.B0 * g.B2 * g.B0;
  const cplx<float>* bx = box + (size_t)b * box_sz;
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, n = u % N;
    const int a = a0 + pp;
    const int q1 = freq_of(n, N);
    cplx<T> val{(T)0, (T)0};
    if (a < g.B0 && q1 >= -Kc && q1 <= Kc) {
      const int q0 = a - Kc;
      const int Q = q0 * q0 + q1 * q1 + c * c;
      if (Q <= qm) {
        const int sid = shell_of_q[Q];
        const bool in = (s == 0) ? (sid > 0) : (sid == s);
        if (in) {
          if (UNIT) {
            val.re = (T)1;
          } else {
            cplx<float> v = bx[((size_t)a * g.B2 + c) * g.B0 + (q1 + Kc)];
            val.re = (T)v.re;
            val.im = (T)v.im;
            if (weighted) {
              const T lw = legendre<T>(g.ell, (T)c / sqrt((T)Q));
              val.re *= lw;
              val.im *= lw;
            }
          }
        }
      }
    }
    buf[pp * NS + pad8(n)] = val;
  }
  __syncthreads();
  fft_block<T, N, P, NS, +1>(buf, stw);
  // store H1[z][x1][c][a0 + pp]
  cplx<T>* out = H1 + (size_t)z * N * g.B2 * g.B0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u % P, x1 = u / P;
    const int a = a0 + pp;
    if (a < g.B0) out[((size_t)x1 * g.B2 + c) * g.B0 + a] = buf[pp * NS + pad8(x1)];
  }
}

// P2: pencils (x1, c), transform q0 -> x0, for the x1 planes of the slab.
// grid (ceil(B2/P), S1, nz).  One plane per block: looping a block over neighbouring
// planes (as pass 3 does over rows) was measured slower here (3.6 -> 5.4 ms at 512^3).
template <typename T, int N>
__global__ __launch_bounds__(kFftThreads) void c2r_p2(const cplx<T>* __restrict__ H1,
                                                      const int* __restrict__ qmax,
                                                      cplx<T>* __restrict__ H2,
                                                      const cplx<T>* __restrict__ tw, Geom g) {
  constexpr int P = FftCfg<T>::kColElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int s = geom_shell(g, z);
  const int c0 = blockIdx.x * P;
  const int xs = blockIdx.y;          // plane within the slab
  const int x1 = g.x1_0 + xs;
  const int Kc = g.Kc;
  const int qm = qmax[s];
  if (c0 * c0 > qm) return;  // every column of this chunk lies outside the shell
  const cplx<T>* in = H1 + (size_t)z * N * g.B2 * g.B0 + (size_t)x1 * g.B2 * g.B0;
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, n = u % N;
    const int c = c0 + pp;
    const int q0 = freq_of(n, N);
    cplx<T> val{(T)0, (T)0};
    if (c < g.B2 && q0 >= -Kc && q0 <= Kc && q0 * q0 + c * c <= qm)
      val = in[(size_t)c * g.B0 + (q0 + Kc)];
    buf[pp * NS + pad8(n)] = val;
  }
  __syncthreads();
  fft_block<T, N, P, NS, +1>(buf, stw);
  cplx<T>* out = H2 + (size_t)z * N * g.S1 * g.H2s;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u % P, x0 = u / P;
    const int c = c0 + pp;
    if (c < g.B2 && c * c <= qm) out[((size_t)x0 * g.S1 + xs) * g.H2s + c] = buf[pp * NS + pad8(x0)];
  }
}


// Z[n] of the packed two-row spectrum Z = A + iB from rows A, B staged in LDS
// (half spectra with entries c = 0..cm; zero above).
template <typename T>
__device__ __forceinline__ cplx<T> two_row_spectrum(const cplx<T>* rowA, const cplx<T>* rowB, int n, int N,
                                                    int cm) {
  const int c = n <= N / 2 ? n : N - n;
  if (c > cm) return cplx<T>{(T)0, (T)0};
  cplx<T> A = rowA[c], B = rowB[c];
  if (c == 0) {  // the DC term of a real row is real
    A.im = 0;
    B.im = 0;
  }
  if (n > N / 2) {  // Z[-c] = conj(A[c]) + i conj(B[c])
    A.im = -A.im;
    B.im = -B.im;
  }
  return cplx<T>{A.re - B.im, A.im + B.re};
}

// Largest q2 index that can be non-zero for shell s.
__device__ __forceinline__ int col_max(const Geom& g, int qm) {
  int cm = g.Kc;
  while (cm * cm > qm) --cm;
  return cm;
}

// P3: rows (x0, x1) of the slab in pairs, complex-to-real over x2.
// out[z * N S1 N + row * N + x2]; optional |value| maximum per z (as float bits).
// Dynamic LDS: the 2P input rows, 2P (Kc + 1) complex values.
// grid (N*S1/2/P/REPS, 1, nz): each block transforms REPS consecutive groups of 2P
// rows, so that its stage twiddles are built once for all of them (a compile-time
// count: the same loop with a run-time count measured 9.6 instead of 8.7 ms at 512^3).
template <int N, int REPS>
__global__ __launch_bounds__(kFftThreads) void c2r_p3(const cplx<float>* __restrict__ H2,
                                                      const int* __restrict__ qmax,
                                                      float* __restrict__ out,
                                                      unsigned* __restrict__ absmax,
                                                      const cplx<float>* __restrict__ tw, Geom g) {
  using T = float;
  constexpr int P = FftCfg<T>::kRowElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  extern __shared__ cplx<float> raw[];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int cm = col_max(g, qmax[geom_shell(g, z)]);
  const int W = cm + 1;
  const size_t rows = (size_t)N * g.S1;   // rows (x0, x1) of the slab
  const size_t G = rows * N;
  float amax = 0.f;
  for (int it = 0; it < REPS; ++it) {
  if (it > 0) __syncthreads();          // the previous group's output has left the LDS
  const int row0 = (blockIdx.x * REPS + it) * 2 * P;  // first of the group's 2P rows
  const cplx<T>* in = H2 + (size_t)z * rows * g.H2s + (size_t)row0 * g.H2s;
  for (int u = threadIdx.x; u < 2 * P * W; u += kFftThreads) {
    const int r = u / W, c = u - r * W;
    raw[u] = in[(size_t)r * g.H2s + c];
  }
  __syncthreads();
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, n = u % N;
    buf[pp * NS + pad8(n)] = two_row_spectrum<T>(raw + (2 * pp) * W, raw + (2 * pp + 1) * W, n, N, cm);
  }
  __syncthreads();
  fft_block<T, N, P, NS, +1>(buf, stw);
  float* o = out + (size_t)z * G + (size_t)row0 * N;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    // one LDS read gives both rows of the pair: the real part is row 2 pp, the imaginary row 2 pp + 1
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, x2 = u % N;
    const cplx<T> v = buf[pp * NS + pad8(x2)];
    o[(size_t)(2 * pp) * N + x2] = v.re;
    o[(size_t)(2 * pp + 1) * N + x2] = v.im;
    amax = fmaxf(amax, fmaxf(fabsf(v.re), fabsf(v.im)));
  }
  }
  if (absmax != nullptr) {
    // block maximum, then one atomic into one of kAbsmaxSpread words of this field
    __shared__ float wmax[kFftThreads / 64];
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = wmax[0];
      for (int w = 1; w < kFftThreads / 64; ++w) m = fmaxf(m, wmax[w]);
      atomicMax(absmax + (size_t)z * kAbsmaxSpread + (blockIdx.x % kAbsmaxSpread), __float_as_uint(m));
    }
  }
}

// absmax[z] = max over the kAbsmaxSpread partial maxima of field z (float bits).
__global__ void reduce_absmax(const unsigned* __restrict__ part, unsigned* __restrict__ absmax, int nz) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  unsigned m = 0;
  for (int i = 0; i < kAbsmaxSpread; ++i) m = max(m, part[(size_t)z * kAbsmaxSpread + i]);
  absmax[z] = m;
}

// P3 (symmetry wedge, float64): rows from a list, outputs x2 in [x1, N/2] only,
// written compactly at out[z * nwedge + off(row) + x2 - x1].  rows[] holds
// (x0, x1, off) triples; rows are processed two at a time.  Dynamic LDS: the 2P
// input rows.  grid (ceil(nrows/2/P), 1, nz)
template <int N>
__global__ __launch_bounds__(kFftThreads) void c2r_p3_wedge(const cplx<double>* __restrict__ H2,
                                                            const int* __restrict__ qmax,
                                                            const int* __restrict__ rows, int nrows,
                                                            double* __restrict__ out, long long nwedge,
                                                            const cplx<double>* __restrict__ tw,
                                                            Geom g) {
  using T = double;
  constexpr int P = FftCfg<T>::kRowElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  extern __shared__ cplx<double> rawd[];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int cm = col_max(g, qmax[geom_shell(g, z)]);
  const int W = cm + 1;
  const int r0 = blockIdx.x * 2 * P;
  const cplx<T>* in = H2 + (size_t)z * N * N * g.H2s;
  for (int u = threadIdx.x; u < 2 * P * W; u += kFftThreads) {
    const int r = u / W, c = u - r * W;
    const int rr = min(r0 + r, nrows - 1);  // rows past the end repeat the last one (unused)
    rawd[u] = in[((size_t)rows[3 * rr] * N + rows[3 * rr + 1]) * g.H2s + c];
  }
  __syncthreads();
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, n = u % N;
    buf[pp * NS + pad8(n)] = two_row_spectrum<T>(rawd + (2 * pp) * W, rawd + (2 * pp + 1) * W, n, N, cm);
  }
  __syncthreads();
  fft_block<T, N, P, NS, +1>(buf, stw);
  double* o = out + (size_t)z * nwedge;
  for (int u = threadIdx.x; u < 2 * P * (N / 2 + 1); u += kFftThreads) {
    const int r = u / (N / 2 + 1), x2 = u % (N / 2 + 1);
    const int rr = r0 + r;
    if (rr >= nrows) continue;
    const int x1 = rows[3 * rr + 1], off = rows[3 * rr + 2];
    if (x2 < x1) continue;
    const cplx<T> v = buf[(r >> 1) * NS + pad8(x2)];
    o[off + x2 - x1] = (r & 1) ? v.im : v.re;
  }
}

// ---------------------------------------------------------------------------
// Forward direction (real grid -> ball)
// ---------------------------------------------------------------------------

// Q3: rows (x0, x1) of the slab in pairs, real-to-complex over x2, keep c = 0..Kc.
// in[z * N S1 N + row * N + x2]; grid (N*S1/2/P, 1, nz).
// grid (N*N/2/P, 1, nz)
template <int N>
__global__ __launch_bounds__(kFftThreads) void r2c_q3(const float* __restrict__ in,
                                                      cplx<float>* __restrict__ H2,
                                                      const cplx<float>* __restrict__ tw, Geom g) {
  using T = float;
  constexpr int P = FftCfg<T>::kRowElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const size_t rows = (size_t)N * g.S1;   // rows (x0, x1) of the slab
  const size_t G = rows * N;
  const int row0 = blockIdx.x * 2 * P;
  const float* src = in + (size_t)z * G + (size_t)row0 * N;
  constexpr int E = P * N / kFftThreads;
  float ra[E], rb[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, x2 = u % N;
    ra[m] = src[(size_t)(2 * pp) * N + x2];
    rb[m] = src[(size_t)(2 * pp + 1) * N + x2];
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u / N, x2 = u % N;
    buf[pp * NS + pad8(x2)] = cplx<T>{ra[m], rb[m]};
  }
  __syncthreads();
  fft_block<T, N, P, NS, -1>(buf, stw);
  cplx<T>* o = H2 + (size_t)z * rows * g.H2s + (size_t)row0 * g.H2s;
  for (int u = threadIdx.x; u < 2 * P * g.B2; u += kFftThreads) {
    const int r = u / g.B2, c = u % g.B2;
    const int pp = r >> 1;
    const cplx<T> Zp = buf[pp * NS + pad8(c)];
    const cplx<T> Zm = buf[pp * NS + pad8(((N - c) & (N - 1)))];
    cplx<T> v;
    if ((r & 1) == 0) {  // A = (Z[c] + conj(Z[-c])) / 2
      v = cplx<T>{(T)0.5 * (Zp.re + Zm.re), (T)0.5 * (Zp.im - Zm.im)};
    } else {  // B = (Z[c] - conj(Z[-c])) / (2i)
      v = cplx<T>{(T)0.5 * (Zp.im + Zm.im), (T)0.5 * (Zm.re - Zp.re)};
    }
    o[(size_t)r * g.H2s + c] = v;
  }
}

// Q2: pencils (x1, c) for the x1 planes of the slab, transform x0 -> q0, keep
// |q0| <= Kc; writes rows x1 of the whole H1.  grid (ceil(B2/P), S1/reps, nz): a
// block takes `reps` consecutive planes.
template <int N>
__global__ __launch_bounds__(kFftThreads) void r2c_q2(const cplx<float>* __restrict__ H2,
                                                      cplx<float>* __restrict__ H1,
                                                      const cplx<float>* __restrict__ tw, Geom g, int reps) {
  using T = float;
  constexpr int P = FftCfg<T>::kElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int c0 = blockIdx.x * P;
  for (int it = 0; it < reps; ++it) {
  if (it > 0) __syncthreads();          // the previous plane's output has left the LDS
  const int xs = blockIdx.y * reps + it;   // plane within the slab
  const int x1 = g.x1_0 + xs;
  const cplx<T>* in = H2 + (size_t)z * N * g.S1 * g.H2s;
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u % P, x0 = u / P;
    const int c = c0 + pp;
    buf[pp * NS + pad8(x0)] = (c < g.B2) ? in[((size_t)x0 * g.S1 + xs) * g.H2s + c] : cplx<T>{0, 0};
  }
  __syncthreads();
  fft_block<T, N, P, NS, -1>(buf, stw);
  cplx<T>* o = H1 + (size_t)z * N * g.B2 * g.B0 + (size_t)x1 * g.B2 * g.B0;
  for (int u = threadIdx.x; u < P * g.B0; u += kFftThreads) {
    const int pp = u / g.B0, a = u % g.B0;
    const int c = c0 + pp;
    if (c >= g.B2) continue;
    const int q0 = a - g.Kc;
    o[(size_t)c * g.B0 + a] = buf[pp * NS + pad8((q0 & (N - 1)))];
  }
  }
}

// Q1: pencils (a, c), transform x1 -> q1, keep |q1| <= Kc and write into the box.
// MASK: write only the modes of shell s(z) (other box entries untouched);
// otherwise write every box entry of the column (the input transform).
// grid (ceil(B0/P), B2, nz)
template <int N, bool MASK>
__global__ __launch_bounds__(kFftThreads) void r2c_q1(const cplx<float>* __restrict__ H1,
                                                      const int16_t* __restrict__ shell_of_q,
                                                      const int* __restrict__ qmax,
                                                      cplx<float>* __restrict__ box,
                                                      const cplx<float>* __restrict__ tw, Geom g) {
  using T = float;
  constexpr int P = FftCfg<T>::kElems / N;
  constexpr int NS = pencil_stride<N>();
  __shared__ cplx<T> buf[P * NS];
  __shared__ cplx<T> stw[stage_tw_size<N>()];
  build_stage_twiddles<T, N>(stw, tw);
  const int z = blockIdx.z;
  const int s = geom_shell(g, z);
  const int b = geom_batch(g, z);
  const int a0 = blockIdx.x * P;
  const int c = blockIdx.y;
  const int Kc = g.Kc;
  const int qm = qmax[s];
  if (MASK) {
    // skip the block when none of its columns reaches shell s
    const int qa = a0 - Kc, qb = a0 + P - 1 - Kc;
    const int qmin0 = (qa <= 0 && qb >= 0) ? 0 : min(qa * qa, qb * qb);
    if (qmin0 + c * c > qm) return;
  }
  const cplx<T>* in = H1 + (size_t)z * N * g.B2 * g.B0;
  constexpr int E = P * N / kFftThreads;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int u = threadIdx.x + m * kFftThreads;
    const int pp = u % P, x1 = u / P;
    const int a = a0 + pp;
    buf[pp * NS + pad8(x1)] = (a < g.B0) ? in[((size_t)x1 * g.B2 + c) * g.B0 + a] : cplx<T>{0, 0};
  }
  __syncthreads();
  fft_block<T, N, P, NS, -1>(buf, stw);
  cplx<float>* o = box + (size_t)b * g.B0 * g.B2 * g.B0;
  for (int u = threadIdx.x; u < P * g.B0; u += kFftThreads) {
    const int pp = u / g.B0, e = u % g.B0;
    const int a = a0 + pp;
    if (a >= g.B0) continue;
    const int q0 = a - Kc, q1 = e - Kc;
    const int Q = q0 * q0 + q1 * q1 + c * c;
    const size_t idx = ((size_t)a * g.B2 + c) * g.B0 + e;
    const cplx<T> v = buf[pp * NS + pad8((q1 & (N - 1)))];
    if (MASK) {
      if (Q <= qm && shell_of_q[Q] == s) o[idx] = v;
    } else {
      o[idx] = v;
    }
  }
}

// Gather the box from a caller's half spectrum complex64 [batch][N][N][N/2+1].
__global__ void box_from_half_spectrum(const cplx<float>* __restrict__ hs, cplx<float>* __restrict__ box,
                                       Geom g) {
  const int N = g.N;
  const size_t box_sz = (size_t)g.B0 * g.B2 * g.B0;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= box_sz) return;
  const int e = i % g.B0;
  const int c = (i / g.B0) % g.B2;
  const int a = i / ((size_t)g.B0 * g.B2);
  const int q0 = a - g.Kc, q1 = e - g.Kc;
  const size_t src = (((size_t)(q0 & (N - 1)) * N) + (q1 & (N - 1))) * (N / 2 + 1) + c;
  box[b * box_sz + i] = hs[(size_t)b * N * N * (N / 2 + 1) + src];
}

// Gradient with respect to a half-spectrum input X[q0][q1][c] (complex64
// [batch][N][N][N/2+1]) from the ball box g of sum_m [s(q) = m] R2C(a_m)[q].  The
// inverse real transform reads X[q] once for c = 0 and, through its conjugate mirror,
// twice for 0 < c < N/2, so dL/dRe X + i dL/dIm X = w_c g[q] with w_0 = 1 and w_c = 2
// (the box never reaches c = N/2).  Every output element is written: zero outside
// the box.
__global__ void half_spectrum_from_box(const cplx<float>* __restrict__ box, cplx<float>* __restrict__ hs, Geom g) {
  const int N = g.N, H = N / 2 + 1;
  const size_t per = (size_t)N * N * H;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= per) return;
  const int c = (int)(i % H);
  const int i1 = (int)((i / H) % N);
  const int i0 = (int)(i / ((size_t)H * N));
  const int q0 = freq_of(i0, N), q1 = freq_of(i1, N);
  cplx<float> v{0.f, 0.f};
  if (c <= g.Kc && q0 >= -g.Kc && q0 <= g.Kc && q1 >= -g.Kc && q1 <= g.Kc) {
    const size_t box_sz = (size_t)g.B0 * g.B2 * g.B0;
    v = box[(size_t)b * box_sz + ((size_t)(q0 + g.Kc) * g.B2 + c) * g.B0 + (q1 + g.Kc)];
    if (c > 0) {
      v.re *= 2.f;
      v.im *= 2.f;
    }
  }
  hs[(size_t)b * per + i] = v;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T>
int fft_pencils_per_block(int N) { return FftCfg<T>::kElems / N; }

// Work items per block for the looping passes: a power of two up to `cap` that
// divides the items and keeps at least 16K blocks in the launch (the per-block setup
// -- stage twiddles in LDS, block start -- is then paid once per `reps` items).
int loop_reps(size_t items, int nz, int cap = 16) {
  int reps = 1;
  while (reps < cap && items % (2 * (size_t)reps) == 0 && items / (2 * (size_t)reps) * (size_t)nz >= 16384)
    reps *= 2;
  return reps;
}

#define PS_FOR_EACH_N(M) M(16) M(32) M(64) M(128) M(256) M(512) M(1024)

template <typename T, bool UNIT>
hipError_t launch_c2r_p1(const cplx<float>* box, const int16_t* sq, const int* qmax, cplx<T>* H1,
                         const cplx<T>* tw, Geom g, int nz, hipStream_t st) {
  const int P = FftCfg<T>::kElems / g.N;
  dim3 grid((g.B0 + P - 1) / P, g.B2, nz);
  switch (g.N) {
#define CASE(n) \
  case n: hipLaunchKernelGGL((c2r_p1<T, n, UNIT>), grid, dim3(kFftThreads), 0, st, box, sq, qmax, H1, tw, g); break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c2r_p2(const cplx<T>* H1, const int* qmax, cplx<T>* H2, const cplx<T>* tw, Geom g, int nz,
                         hipStream_t st) {
  const int P = FftCfg<T>::kColElems / g.N;
  if (g.S1 < 1 || g.x1_0 < 0 || g.x1_0 + g.S1 > g.N) return hipErrorInvalidValue;
  dim3 grid((g.B2 + P - 1) / P, g.S1, nz);
  switch (g.N) {
#define CASE(n) case n: hipLaunchKernelGGL((c2r_p2<T, n>), grid, dim3(kFftThreads), 0, st, H1, qmax, H2, tw, g); break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_c2r_p3(const cplx<float>* H2, const int* qmax, float* out, unsigned* absmax,
                         const cplx<float>* tw, Geom g, int nz, hipStream_t st) {
  const int P = FftCfg<float>::kRowElems / g.N;
  if (g.S1 < 1 || g.x1_0 < 0 || g.x1_0 + g.S1 > g.N || ((size_t)g.N * g.S1) % (2 * P) != 0)
    return hipErrorInvalidValue;
  const size_t groups = (size_t)g.N * g.S1 / 2 / P;
  // 16 groups per block when that still leaves a few thousand blocks, else one
  const bool loop = groups % 16 == 0 && groups / 16 * (size_t)nz >= 4096;
  dim3 grid((unsigned)(groups / (loop ? 16 : 1)), 1, nz);
  const size_t shm = (size_t)2 * P * g.B2 * sizeof(cplx<float>);
  switch (g.N) {
#define CASE(n)                                                                                                  \
  case n:                                                                                                        \
    if (loop) hipLaunchKernelGGL((c2r_p3<n, 16>), grid, dim3(kFftThreads), shm, st, H2, qmax, out, absmax, tw, g); \
    else hipLaunchKernelGGL((c2r_p3<n, 1>), grid, dim3(kFftThreads), shm, st, H2, qmax, out, absmax, tw, g);       \
    break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_c2r_p3_wedge(const cplx<double>* H2, const int* qmax, const int* rows, int nrows,
                               double* out, long long nwedge, const cplx<double>* tw, Geom g, int nz,
                               hipStream_t st) {
  const int P = FftCfg<double>::kRowElems / g.N;
  dim3 grid((nrows + 2 * P - 1) / (2 * P), 1, nz);
  const size_t shm = (size_t)2 * P * g.B2 * sizeof(cplx<double>);
  switch (g.N) {
#define CASE(n)                                                                                         \
  case n:                                                                                               \
    hipLaunchKernelGGL((c2r_p3_wedge<n>), grid, dim3(kFftThreads), shm, st, H2, qmax, rows, nrows, out, \
                       nwedge, tw, g);                                                                  \
    break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_r2c_q3(const float* in, cplx<float>* H2, const cplx<float>* tw, Geom g, int nz,
                         hipStream_t st) {
  const int P = FftCfg<float>::kRowElems / g.N;
  if (g.S1 < 1 || g.x1_0 < 0 || g.x1_0 + g.S1 > g.N || ((size_t)g.N * g.S1) % (2 * P) != 0)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((size_t)g.N * g.S1 / 2 / P), 1, nz);
  switch (g.N) {
#define CASE(n) case n: hipLaunchKernelGGL((r2c_q3<n>), grid, dim3(kFftThreads), 0, st, in, H2, tw, g); break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_r2c_q2(const cplx<float>* H2, cplx<float>* H1, const cplx<float>* tw, Geom g, int nz,
                         hipStream_t st) {
  const int P = FftCfg<float>::kElems / g.N;
  if (g.S1 < 1 || g.x1_0 < 0 || g.x1_0 + g.S1 > g.N) return hipErrorInvalidValue;
  const int cb = (g.B2 + P - 1) / P;
  const int reps = loop_reps(g.S1, cb * nz);
  dim3 grid(cb, g.S1 / reps, nz);
  switch (g.N) {
#define CASE(n) case n: hipLaunchKernelGGL((r2c_q2<n>), grid, dim3(kFftThreads), 0, st, H2, H1, tw, g, reps); break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool MASK>
hipError_t launch_r2c_q1(const cplx<float>* H1, const int16_t* sq, const int* qmax, cplx<float>* box,
                         const cplx<float>* tw, Geom g, int nz, hipStream_t st) {
  const int P = FftCfg<float>::kElems / g.N;
  dim3 grid((g.B0 + P - 1) / P, g.B2, nz);
  switch (g.N) {
#define CASE(n) \
  case n: hipLaunchKernelGGL((r2c_q1<n, MASK>), grid, dim3(kFftThreads), 0, st, H1, sq, qmax, box, tw, g); break;
    PS_FOR_EACH_N(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_absmax(const unsigned* part, unsigned* absmax, int nz, hipStream_t st) {
  hipLaunchKernelGGL(reduce_absmax, dim3((nz + 255) / 256), dim3(256), 0, st, part, absmax, nz);
  return hipGetLastError();
}

hipError_t launch_box_from_half_spectrum(const cplx<float>* hs, cplx<float>* box, Geom g, int batch,
                                         hipStream_t st) {
  const size_t box_sz = (size_t)g.B0 * g.B2 * g.B0;
  dim3 grid((unsigned)((box_sz + 255) / 256), batch);
  hipLaunchKernelGGL(box_from_half_spectrum, grid, dim3(256), 0, st, hs, box, g);
  return hipGetLastError();
}

hipError_t launch_half_spectrum_from_box(const cplx<float>* box, cplx<float>* hs, Geom g, int batch,
                                         hipStream_t st) {
  const size_t per = (size_t)g.N * g.N * (g.N / 2 + 1);
  dim3 grid((unsigned)((per + 255) / 256), batch);
  hipLaunchKernelGGL(half_spectrum_from_box, grid, dim3(256), 0, st, box, hs, g);
  return hipGetLastError();
}

template hipError_t launch_c2r_p1<float, false>(const cplx<float>*, const int16_t*, const int*, cplx<float>*,
                                                const cplx<float>*, Geom, int, hipStream_t);
template hipError_t launch_c2r_p1<double, true>(const cplx<float>*, const int16_t*, const int*, cplx<double>*,
                                                const cplx<double>*, Geom, int, hipStream_t);
template hipError_t launch_c2r_p2<float>(const cplx<float>*, const int*, cplx<float>*, const cplx<float>*, Geom,
                                         int, hipStream_t);
template hipError_t launch_c2r_p2<double>(const cplx<double>*, const int*, cplx<double>*, const cplx<double>*,
                                          Geom, int, hipStream_t);
template hipError_t launch_r2c_q1<true>(const cplx<float>*, const int16_t*, const int*, cplx<float>*,
                                        const cplx<float>*, Geom, int, hipStream_t);
template hipError_t launch_r2c_q1<false>(const cplx<float>*, const int16_t*, const int*, cplx<float>*,
                                         const cplx<float>*, Geom, int, hipStream_t);

}  // namespace ps

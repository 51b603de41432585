// Host-side launchers of the device kernels (fft.hip, contract.hip, util.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace ps {

// fft.hip
template <typename T>
int fft_pencils_per_block(int N);
template <typename T, bool UNIT>
hipError_t launch_c2r_p1(const cplx<float>* box, const int16_t* shell_of_q, const int* qmax, cplx<T>* H1,
                         const cplx<T>* tw, Geom g, int nz, hipStream_t st);
template <typename T>
hipError_t launch_c2r_p2(const cplx<T>* H1, const int* qmax, cplx<T>* H2, const cplx<T>* tw, Geom g, int nz,
                         hipStream_t st);
hipError_t launch_c2r_p3(const cplx<float>* H2, const int* qmax, float* out, unsigned* absmax,
                         const cplx<float>* tw, Geom g, int nz, hipStream_t st);
hipError_t launch_c2r_p3_wedge(const cplx<double>* H2, const int* qmax, const int* rows, int nrows, double* out,
                               long long nwedge, const cplx<double>* tw, Geom g, int nz, hipStream_t st);
hipError_t launch_r2c_q3(const float* in, cplx<float>* H2, const cplx<float>* tw, Geom g, int nz, hipStream_t st);
hipError_t launch_r2c_q2(const cplx<float>* H2, cplx<float>* H1, const cplx<float>* tw, Geom g, int nz,
                         hipStream_t st);
template <bool MASK>
hipError_t launch_r2c_q1(const cplx<float>* H1, const int16_t* shell_of_q, const int* qmax, cplx<float>* box,
                         const cplx<float>* tw, Geom g, int nz, hipStream_t st);
constexpr int kAbsmaxSpreadHost = 256;
hipError_t launch_reduce_absmax(const unsigned* part, unsigned* absmax, int nz, hipStream_t st);
hipError_t launch_box_from_half_spectrum(const cplx<float>* hs, cplx<float>* box, Geom g, int batch,
                                         hipStream_t st);
hipError_t launch_half_spectrum_from_box(const cplx<float>* box, cplx<float>* hs, Geom g, int batch,
                                         hipStream_t st);

// contract.hip
struct CtrParams {
  const float* D;
  const int* pair_uv;
  const int* slot_uni;     // [n_groups][waves][kSlots / 4]: one byte per slot
  const int* slot_lane;    // [n_groups][waves][16 rows][kSlots]: pair shells per lane
  const int* slot_tile;
  const int* slot_blk;     // [n_groups][waves][kSlotsMax]: A pair block | B pair block << 16
  const unsigned* absmax;
  float* partials;
  long long G;
  int n_shells;
  int n_blk;
  int n_pairs_padded;
  int n_tiles;
  int ksteps;
  int n_chunks;
  int n_pair_blocks;       // order 4, FP16: pair operands formed once per K-step in LDS (0: per slot)
  const int* grp_blk;      // or null: [n_groups][kMaxPairBlocksHost] the group's own pair blocks (global ids)
  const int* grp_nblk;     // [n_groups]: how many (then slot_blk holds indices into that list)
};
// Order 4, split FP16: pair blocks that fit the workgroup's LDS as shared operands
// beside the staged shell operands (28 blocks of 16 pairs: up to 29 shells).
constexpr int kMaxPairBlocksHost = 28;
constexpr int kCtrWavesHost = 16;
constexpr int kSlotsHost = 14;
constexpr int kSlots4Host = 10;
constexpr int kSlots56Host = 8;
constexpr int kSlots6Host = 7;
constexpr int kMaxShells56 = 32;    // orders 5 and 6: shells per plan (row tables stay small)
constexpr int kSlots2Host = 4;
constexpr int kSlotsMaxHost = 16;   // per-wave stride of the slot tables
constexpr int kStagePtsHost = 64;
constexpr int kMaxBlkHost = 4;       // the shell-block aligned order-3 kernel (<= 64 shells)
constexpr int kMaxTileBlkHost = 8;   // the tile kernel, orders 2 to 4 (<= 128 shells)
constexpr int kAdjPtsHost = 512;   // grid points per adjoint workgroup
constexpr int kCntTuplesPerGroup = 1024;
constexpr int kCntStageHost = 32;

hipError_t launch_contract(int prec, int order, const CtrParams& p, int n_groups, int batch, hipStream_t st);

// Order 3 with pair blocks aligned to shell blocks: wave w of kJWaves owns the shells
// j = w + kJWaves q (q = 0..7, shell block jb = q / 2) and the tiles (ib <= jb, kb >= jb)
// of each, at most kJSlots per wave, numbered by jslot().
constexpr int kJWaves = 8;
constexpr int kJSlots = 40;
__host__ __device__ constexpr int jslot(int q, int ib, int kb) {
  int s = 0;
  for (int qq = 0; qq < q; ++qq) s += (qq / 2 + 1) * (4 - qq / 2);
  return s + ib * (4 - q / 2) + (kb - q / 2);
}
struct CtrJParams {
  const float* D;
  const unsigned* absmax;
  const int* tile_of_slot;   // [kJWaves][kJSlots]: compact tile id, or -1
  const unsigned* slot_mask; // [kJWaves][2]: bit s set when slot s holds a tile
  float* partials;
  long long G;
  int n_shells;
  int n_blk;
  int n_tiles;
  int ksteps;
  int n_chunks;
};
hipError_t launch_contract_j3(int prec, const CtrJParams& p, int batch, hipStream_t st);
hipError_t launch_reduce_f32(const float* part, double* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                             bool accumulate, const int* closing_of_entry, const int* bins, int order,
                             const unsigned* absmax, int n_shells, int prec, int batch, hipStream_t st);
hipError_t launch_reduce_f64(const double* part, double* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                             int batch, hipStream_t st);
hipError_t launch_gather(const double* tmp, int n_groups, long long n_ent, const int* ent_idx, const int* bins,
                         int order, const double* fnorm, int n_closing, const unsigned* absmax, int n_shells,
                         int prec, double* out, double* raw, int* nonfinite, int batch, hipStream_t st);
hipError_t launch_counts_wedge(int order, const double* cw, long long nwedge, const unsigned char* wmult,
                               const int* cand, int n_cand, int n_shells, int stages_per_chunk, int n_chunks,
                               double2* part, hipStream_t st);
hipError_t launch_reduce_dd(const double2* part, double2* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                            hipStream_t st);
// Adjoint products (adjoint.h).  FP16 (prec 2) scales every weight row m by its own
// power of two, found from rowmax[b][64] (float64 bits, written by the weights launch);
// absmax holds the per-shell field maxima of the forward's FP16 scaling.
hipError_t launch_adjoint_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                  int n_closing, int prec, const unsigned* absmax, unsigned long long* rowmax,
                                  uint4* W, int batch, hipStream_t st);
// N <= 512: the adjoint kernel also runs the first (x2 -> q2) transform of its fields
// and writes H2 (A must be null); otherwise it writes the fields to A (H2 null).
inline bool adjoint_fuses_rows(int N) { return N <= 512; }
hipError_t launch_adjoint_gemm(int prec, const float* D, const uint4* W, const int* vmask, const unsigned* absmax,
                               const unsigned long long* rowmax, int n_shells, long long G, float* A,
                               cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st);
// Order 4 (n_shells <= kAdj4MaxShells): W4[b][item (w, v <= w)][uc][mb][hi, lo][lane],
// item = w (w + 1) / 2 + v, over NC = 2 chunks of u and one 32-row block of m up to 32
// shells, NC = 4 chunks and two blocks above.
constexpr int kAdj4MaxShells = 64;
constexpr int kAdj3MaxShells = 64;
__host__ __device__ constexpr int adj4_chunks(int n_shells) { return n_shells <= 32 ? 2 : 4; }
__host__ __device__ constexpr int adj4_words_per_item(int n_shells) {
  return adj4_chunks(n_shells) * (adj4_chunks(n_shells) / 2) * 2 * 64;
}
hipError_t launch_adjoint4_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                   int n_closing, int prec, const unsigned* absmax, unsigned long long* rowmax,
                                   uint4* W, int batch, hipStream_t st);
hipError_t launch_adjoint4_gemm(int prec, const float* D, const uint4* W, const int* imask, const unsigned* absmax,
                                const unsigned long long* rowmax, int n_shells, long long G, float* A,
                                cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st);

// util.hip
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;   // polyspec_forward_static's workspace
constexpr int kMaxDevices = 64;
// Device address of this device's static scratch (looked up once per device, with that
// device current).
hipError_t static_scratch_address(int device, void** ptr);
hipError_t launch_fill_u32(void* dst, unsigned value, size_t n_words, hipStream_t st);
hipError_t launch_fields_absmax(const float* x, long long G, int nz, unsigned* part, int spread, hipStream_t st);

}  // namespace ps

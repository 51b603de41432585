// Host side of the polyspectrum library: descriptor validation, shell and tuple
// tables, tile scheduling, workspace, plan-time polygon counts and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/polyspec.h"
#include "kernels.h"

using ps::cplx;
using ps::Geom;

namespace {

thread_local std::string g_plan_error;

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

// Exact dyadic representation of the shell width: width = m * 2^e with m odd.
struct Dyadic {
  int64_t m = 0;
  int e = 0;
};

bool to_dyadic(double w, Dyadic* out) {
  if (!(w > 0.0) || !std::isfinite(w)) return false;
  int ex = 0;
  double fr = std::frexp(w, &ex);            // w = fr * 2^ex, fr in [0.5, 1)
  double mm = std::ldexp(fr, 53);            // integer
  int64_t m = (int64_t)mm;
  int e = ex - 53;
  while ((m & 1) == 0) {
    m >>= 1;
    ++e;
  }
  out->m = m;
  out->e = e;
  return true;
}

using u128 = unsigned __int128;

// Smallest integer Q with 4 Q >= (k * width)^2, k >= 1 odd; width = m 2^e, m < 2^24.
int64_t ceil_quarter_square(int64_t k, const Dyadic& d) {
  u128 num = (u128)(k * d.m) * (u128)(k * d.m);  // (k m)^2 < 2^70
  int sh = 2 * d.e - 2;                            // Q >= num * 2^(2e) / 4
  if (sh >= 0) return (int64_t)(num << sh);
  int r = -sh;
  if (r >= 127) return num ? 1 : 0;
  u128 q = num >> r;
  if ((q << r) != num) ++q;
  return (int64_t)q;
}

}  // namespace

struct polyspec_plan_s {
  polyspec_desc desc{};
  hipStream_t stream = nullptr;
  std::string last_error;
  int device = -1;                 // current device when the plan was made
  void* static_scratch = nullptr;  // that device's static scratch (polyspec_forward_static)
  hipError_t static_scratch_status = hipSuccess;

  int N = 0, order = 0, nb = 0, batch = 0, prec = 0;
  int Kc = 0, B0 = 0, B2 = 0, n_blk = 0;
  long long G = 0;
  bool alias_free = true;
  // streamed mode: the last two inverse passes and the contraction run one slab of
  // S1 x1-planes at a time, so only a slab of every shell field is ever stored
  bool streamed = false;
  int S1 = 0, n_slabs = 1;

  std::vector<int64_t> thr;        // T_1..T_{nb+1}
  std::vector<int16_t> shell_of_q;
  std::vector<int> qmax;           // [nb+1]

  // tuples (0-based shells)
  std::vector<int> cand;           // [n_cand][order]
  std::vector<double> cand_quot;   // C_t / N^3
  std::vector<int64_t> cand_count;
  std::vector<int> closing;        // candidate index of each closing tuple
  std::vector<int> cl_bins;        // [n_closing][order]
  std::vector<int64_t> cl_counts;
  std::vector<double> fnorm_base;  // f / (N^3 n_t) of each closing tuple

  // multipole plans (POLYSPEC_MULTIPOLE): nb counts fields, ns shells; fields 0..ns-1 are
  // the shells, ns..2ns-1 their L_ell-weighted copies, and tuples are (u, v, ns + w)
  bool mp = false;
  int ns = 0;
  int ell = 0;

  // contraction tiling
  int n_pairs = 0, n_pairs_padded = 0, n_tiles = 0, n_groups = 0, ksteps = 0, n_chunks = 0;
  int red_groups = 0, red_cpg = 0;
  int n_adj_active = 0;
  std::vector<int> pair_uv;
  // shell-block aligned order-3 schedule (FP16 split)
  std::vector<int> wmask_host;     // adjoint: per v, bits 2 uc + mb of weight blocks
  bool jsched = false;
  int n_tiles_j = 0, ksteps_j = 0, n_chunks_j = 0;

  // device tables
  DevBuf tw32, shell_q, qmax_d, pairs_d, slots_d, slot_lane_d, slot_tile_d, slot_blk_d, ent_d, bins_d, fnorm_d, lookup_d,
      wmask_d, flag_d;
  DevBuf jtile_d, jmask_d, ent_j_d;
  // order 4 with more pair blocks than one workgroup's LDS holds: each tile group's own
  // pair blocks (global ids, kMaxPairBlocksHost per group) and their count
  bool pair_groups = false;
  DevBuf grp_blk_d, grp_nblk_d;
  DevBuf closing_of_ent_d, closing_of_ent_j_d;   // streamed plans: tile entry -> closing tuple (or -1)
  // workspace carving
  DevBuf own_ws;
  char* ws = nullptr;
  size_t ws_size = 0;
  cplx<float>* box = nullptr;
  cplx<float>* gbox = nullptr;
  cplx<float>* H1 = nullptr;
  cplx<float>* H1a = nullptr;   // streamed backward: the adjoint's x1 rows (H1 keeps the forward's)
  cplx<float>* H2 = nullptr;
  float* D = nullptr;
  float* A = nullptr;
  float* partials = nullptr;
  double* red = nullptr;
  unsigned* absmax = nullptr;       // per-field max |d| (float bits), FP16 scaling
  unsigned* absmax_part = nullptr;  // partial maxima written by the shell transform
  bool absmax_valid = false;
  float* W = nullptr;
  unsigned long long* rowmax = nullptr;   // adjoint, FP16: per weight row maximum (float64 bits)
  bool have_fields = false;

  // per-kernel timing with HIP events on the plan's stream
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double prof_ms[POLYSPEC_N_PHASES] = {};
  int64_t prof_calls[POLYSPEC_N_PHASES] = {};

  polyspec_status fail(polyspec_status st, const std::string& msg) {
    last_error = msg;
    return st;
  }
};

namespace {

polyspec_status dev_alloc(polyspec_plan_s* p, DevBuf* b, size_t n) {
  b->n = n;
  if (n == 0) {
    b->p = nullptr;
    return POLYSPEC_OK;
  }
  hipError_t e = hipMalloc(&b->p, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b->p = nullptr;
    return p->fail(e == hipErrorOutOfMemory ? POLYSPEC_ERR_OUT_OF_MEMORY : POLYSPEC_ERR_DEVICE,
                   std::string("hipMalloc of ") + std::to_string(n) + " bytes failed: " + hipGetErrorString(e));
  }
  return POLYSPEC_OK;
}

void dev_free(DevBuf* b) {
  if (b->p) (void)hipFree(b->p);
  b->p = nullptr;
  b->n = 0;
}

template <typename T>
polyspec_status upload(polyspec_plan_s* p, DevBuf* b, const std::vector<T>& v) {
  polyspec_status st = dev_alloc(p, b, v.size() * sizeof(T));
  if (st != POLYSPEC_OK || v.empty()) return st;
  hipError_t e = hipMemcpy(b->p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return p->fail(POLYSPEC_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return POLYSPEC_OK;
}

#define PS_HIP(p, ...)                                                                                     \
  do {                                                                                                     \
    hipError_t e_ = (__VA_ARGS__);                                                                            \
    if (e_ != hipSuccess) {                                                                                \
      (void)hipGetLastError();                                                                             \
      return (p)->fail(POLYSPEC_ERR_DEVICE, std::string(#__VA_ARGS__) + " failed: " + hipGetErrorString(e_));     \
    }                                                                                                      \
  } while (0)

#define PS_TRY(expr)                     \
  do {                                   \
    polyspec_status s_ = (expr);         \
    if (s_ != POLYSPEC_OK) return s_;    \
  } while (0)

hipEvent_t ev_get(polyspec_plan_s* p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Launch with optional start/stop events around it (phase ph).
#define PS_TIMED(p, ph, ...)                                                  \
  do {                                                                        \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                  \
    if ((p)->prof) {                                                          \
      e0_ = ev_get(p);                                                        \
      e1_ = ev_get(p);                                                        \
      if (e0_ && e1_) PS_HIP(p, hipEventRecord(e0_, (p)->stream));            \
    }                                                                         \
    PS_HIP(p, __VA_ARGS__);                                                   \
    if ((p)->prof && e0_ && e1_) {                                            \
      PS_HIP(p, hipEventRecord(e1_, (p)->stream));                            \
      (p)->ev_pending.push_back({(ph), {e0_, e1_}});                          \
    }                                                                         \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Row stride of H2 (see Geom): B2 rounded up to 16 entries.
size_t h2_stride(const polyspec_plan_s* p) { return ((size_t)p->B2 + 15) & ~(size_t)15; }

// The adjoint product exists for orders 3 and 4 up to 64 shells.
bool has_adjoint(const polyspec_plan_s* p) {
  if (p->mp) return false;
  return (p->order == 3 && p->nb <= ps::kAdj3MaxShells) || (p->order == 4 && p->nb <= ps::kAdj4MaxShells);
}

Geom make_geom(const polyspec_plan_s* p, int spb, int shell_base) {
  Geom g;
  g.N = p->N;
  g.Kc = p->Kc;
  g.B0 = p->B0;
  g.B2 = p->B2;
  g.H2s = h2_stride(p);
  g.spb = spb;
  g.shell_base = shell_base;
  g.n_shells = p->nb;
  g.S1 = p->N;
  g.x1_0 = 0;
  g.fold = p->mp ? p->ns : std::max(spb, 1);
  g.ell = p->mp ? p->ell : -1;
  return g;
}

// Grid points of one contraction launch: the whole grid, or one slab.
long long launch_points(const polyspec_plan_s* p) { return p->streamed ? (long long)p->N * p->N * p->S1 : p->G; }

// Chunking of one contraction launch into workgroups of ksteps 64-point stages.
void set_chunking(polyspec_plan_s* p) {
  const long long steps = launch_points(p) / ps::kStagePtsHost;
  long long ks = steps / 512;
  ks = std::max(1LL, std::min(256LL, ks));
  while (steps % ks) --ks;
  p->ksteps = (int)ks;
  p->n_chunks = (int)(steps / ks);
  // the shell-block aligned kernel works on whole 256-point stages
  long long ksj = std::max(4LL, ks);
  while (steps % ksj) ++ksj;
  p->ksteps_j = (int)ksj;
  p->n_chunks_j = (int)(steps / ksj);
  p->red_cpg = 64;
  p->red_groups = (p->n_chunks + p->red_cpg - 1) / p->red_cpg;
}

// Smallest slab the last pass accepts: N S1 rows must split into pairs of P-row blocks.
int min_slab_planes(int N) {
  const int P = 2048 / N;
  int s1 = 1;
  while (((long long)N * s1) % (2 * P) != 0) s1 *= 2;
  return s1;
}

template <typename T>
std::vector<cplx<T>> twiddles(int N) {
  std::vector<cplx<T>> tw(N);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int e = 0; e < N; ++e) {
    long double a = two_pi * (long double)e / (long double)N;
    tw[e].re = (T)std::cos(a);
    tw[e].im = (T)std::sin(a);
  }
  // exact values on the axes and diagonals
  for (int e = 0; e < N; e += N / 4) {
    int q = e / (N / 4);
    tw[e].re = (T)(q == 0 ? 1 : q == 2 ? -1 : 0);
    tw[e].im = (T)(q == 1 ? 1 : q == 3 ? -1 : 0);
  }
  return tw;
}

// Sizes of the workspace pieces, in carving order.
struct WsLayout {
  size_t box, gbox, H1, H1a, H2, D, A, partials, red, absmax, W, rowmax, total;
};

WsLayout layout_of(const polyspec_plan_s* p) {
  WsLayout L{};
  const size_t box_elems = (size_t)p->B0 * p->B2 * p->B0;
  const size_t zf = (size_t)p->batch * p->nb;
  L.box = align256((size_t)p->batch * box_elems * sizeof(cplx<float>));
  const bool adjoint = has_adjoint(p);
  const size_t planes = p->streamed ? p->S1 : p->N;   // x1 planes held of H2 and of the fields
  L.gbox = adjoint ? L.box : 0;
  L.H1 = align256(zf * p->N * p->B2 * p->B0 * sizeof(cplx<float>));
  L.H1a = (adjoint && p->streamed) ? L.H1 : 0;
  // H2 also takes the input's first transform, batch x N^2 x B2, when a slab is smaller
  L.H2 = align256(std::max(zf * p->N * planes, (size_t)p->batch * p->N * p->N) * h2_stride(p) * sizeof(cplx<float>));
  L.D = align256(zf * (size_t)p->N * planes * p->N * sizeof(float));
  L.A = (adjoint && !ps::adjoint_fuses_rows(p->N)) ? L.D : 0;   // adjoint fields only when not fused
  const size_t tiles = (size_t)std::max(p->n_tiles, p->n_tiles_j);
  L.partials = align256((size_t)p->batch * p->n_chunks * tiles * 256 * sizeof(float));
  L.red = align256((size_t)p->batch * p->red_groups * tiles * 256 * sizeof(double));
  L.absmax = align256(zf * sizeof(unsigned)) + align256(zf * ps::kAbsmaxSpreadHost * sizeof(unsigned));
  L.W = !adjoint ? 0
        : p->order == 3 ? align256((size_t)p->batch * p->nb * 4 * 2 * 2 * 64 * 16)
        : adjoint ? align256((size_t)p->batch * (p->nb * (p->nb + 1) / 2) * ps::adj4_words_per_item(p->nb) * 16)
                  : 0;
  L.rowmax = adjoint ? align256((size_t)p->batch * 64 * sizeof(unsigned long long)) : 0;
  L.total = L.box + L.gbox + L.H1 + L.H1a + L.H2 + L.D + L.A + L.partials + L.red + L.absmax + L.W + L.rowmax;
  return L;
}

void carve(polyspec_plan_s* p, char* base) {
  WsLayout L = layout_of(p);
  char* c = base;
  p->box = (cplx<float>*)c; c += L.box;
  p->gbox = L.gbox ? (cplx<float>*)c : nullptr; c += L.gbox;
  p->H1 = (cplx<float>*)c; c += L.H1;
  p->H1a = L.H1a ? (cplx<float>*)c : nullptr; c += L.H1a;
  p->H2 = (cplx<float>*)c; c += L.H2;
  p->D = (float*)c; c += L.D;
  p->A = L.A ? (float*)c : nullptr; c += L.A;
  p->partials = (float*)c; c += L.partials;
  p->red = (double*)c; c += L.red;
  p->absmax = (unsigned*)c;
  p->absmax_part = (unsigned*)(c + align256((size_t)p->batch * p->nb * sizeof(unsigned)));
  c += L.absmax;
  p->W = L.W ? (float*)c : nullptr; c += L.W;
  p->rowmax = L.rowmax ? (unsigned long long*)c : nullptr; c += L.rowmax;
}

polyspec_status ensure_workspace(polyspec_plan_s* p) {
  if (p->ws) return POLYSPEC_OK;
  WsLayout L = layout_of(p);
  PS_TRY(dev_alloc(p, &p->own_ws, L.total));
  p->ws = (char*)p->own_ws.p;
  p->ws_size = L.total;
  carve(p, p->ws);
  return POLYSPEC_OK;
}

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
void build_tuples(polyspec_plan_s* p) {
  const int n = p->order, nb = p->nb;
  std::vector<int> t(n, 0);
  // lexicographic enumeration of t_0 <= ... <= t_{n-1}, last index fastest
  while (true) {
    bool ok = true;
    if (p->alias_free) {
      // 1-based: t_n < sum_{j<n} t_j + n/2  <=>  2 t_n < 2 sum + n
      long long s = 0;
      for (int j = 0; j < n - 1; ++j) s += t[j] + 1;
      ok = 2LL * (t[n - 1] + 1) < 2 * s + n;
    }
    if (ok)
      for (int j = 0; j < n; ++j) p->cand.push_back(t[j]);
    int j = n - 1;
    while (j >= 0 && t[j] == nb - 1) --j;
    if (j < 0) break;
    ++t[j];
    for (int k = j + 1; k < n; ++k) t[k] = t[j];
  }
}

// Pairs (i <= j) ordered by j, then i: a block of 16 consecutive pairs spans few
// values of j, so few shell blocks k >= j close triangles with it.
void build_pairs(polyspec_plan_s* p, std::vector<int>* pidx) {
  const int nb = p->nb;
  p->n_pairs = nb * (nb + 1) / 2;
  p->n_pairs_padded = (p->n_pairs + 31) / 32 * 32;
  const int zrow = p->n_blk * 16;
  p->pair_uv.assign(p->n_pairs_padded, zrow | (zrow << 16));
  pidx->assign(nb * nb, -1);
  int k = 0;
  for (int j = 0; j < nb; ++j)
    for (int i = 0; i <= j; ++i) {
      p->pair_uv[k] = i | (j << 16);
      (*pidx)[i * nb + j] = k;
      ++k;
    }
}

struct TileKey {
  int a, b;
  bool operator<(const TileKey& o) const { return a != o.a ? a < o.a : b < o.b; }
};

// Entry of output (row, col) of a 16x16 tile in the dumped accumulator layout:
// lane 16 (row / 4) + col, register row % 4.
inline int tile_entry(int row, int col) { return 4 * (16 * (row / 4) + col) + (row % 4); }

// Triples (i <= j <= k) for the row blocks of orders 5 and 6, packed as shell bytes
// i | j << 8 | k << 16, padded with the zero row.  The B side is ordered by its
// smallest shell (then j, k) and the A side of order 6 by its largest (then j, i):
// the needed tuples pair an A row whose largest shell is at most the B row's
// smallest, so both orders keep the needed tiles in a dense staircase.
void build_triples(const polyspec_plan_s* p, bool by_largest, std::vector<int>* rows, std::vector<int>* tidx) {
  const int nb = p->nb, zrow = p->n_blk * 16;
  rows->clear();
  tidx->assign((size_t)nb * nb * nb, -1);
  std::vector<std::array<int, 3>> tl;
  for (int i = 0; i < nb; ++i)
    for (int j = i; j < nb; ++j)
      for (int k = j; k < nb; ++k) tl.push_back({i, j, k});
  if (by_largest)
    std::stable_sort(tl.begin(), tl.end(), [](const std::array<int, 3>& a, const std::array<int, 3>& b) {
      return a[2] != b[2] ? a[2] < b[2] : a[1] != b[1] ? a[1] < b[1] : a[0] < b[0];
    });
  for (const auto& t : tl) {
    (*tidx)[((size_t)t[0] * nb + t[1]) * nb + t[2]] = (int)rows->size();
    rows->push_back(t[0] | (t[1] << 8) | (t[2] << 16));
  }
  while (rows->size() % 16) rows->push_back(zrow | (zrow << 8) | (zrow << 16));
}

polyspec_status build_tiles(polyspec_plan_s* p, std::vector<int>* ent_of_cand) {
  std::vector<int> pidx;
  build_pairs(p, &pidx);
  const int n = p->order, nb = p->nb;
  const size_t nc = p->cand.size() / n;
  // shell bytes of every A and B row (orders 5 and 6)
  std::vector<int> arows, brows, aidx, bidx;
  if (n >= 5) {
    build_triples(p, false, &brows, &bidx);
    if (n == 6) {
      build_triples(p, true, &arows, &aidx);
    } else {
      for (int w : p->pair_uv) arows.push_back((w & 0xff) | (((w >> 16) & 0xff) << 8));
    }
  }
  std::map<TileKey, int> tiles;
  std::vector<std::array<int, 4>> loc(nc);  // ablk, bblk, row, col
  for (size_t c = 0; c < nc; ++c) {
    const int* t = &p->cand[c * n];
    int ra, rb;
    if (n == 2) {
      ra = t[0];
      rb = t[1];
    } else if (n == 3) {
      ra = pidx[t[0] * nb + t[1]];
      rb = t[2];
    } else if (n == 4) {
      ra = pidx[t[0] * nb + t[1]];
      rb = pidx[t[2] * nb + t[3]];
    } else if (n == 5) {
      ra = pidx[t[0] * nb + t[1]];
      rb = bidx[((size_t)t[2] * nb + t[3]) * nb + t[4]];
    } else {
      ra = aidx[((size_t)t[0] * nb + t[1]) * nb + t[2]];
      rb = bidx[((size_t)t[3] * nb + t[4]) * nb + t[5]];
    }
    loc[c] = {ra / 16, rb / 16, ra % 16, rb % 16};
    tiles[TileKey{ra / 16, rb / 16}] = 0;
  }
  int id = 0;
  std::vector<TileKey> tlist;
  for (auto& kv : tiles) {
    kv.second = id++;
    tlist.push_back(kv.first);
  }
  p->n_tiles = id;
  ent_of_cand->resize(nc);
  for (size_t c = 0; c < nc; ++c) {
    const int t = tiles[TileKey{loc[c][0], loc[c][1]}];
    (*ent_of_cand)[c] = t * 256 + tile_entry(loc[c][2], loc[c][3]);
  }
  // units: runs of tiles sharing the A block, cut into pieces that fit one wave
  const int cap = n == 2   ? ps::kSlots2Host
                  : n == 3 ? ps::kSlotsHost
                  : n == 4 ? ps::kSlots4Host
                  : n == 5 ? ps::kSlots56Host
                           : ps::kSlots6Host;
  std::vector<std::pair<int, int>> units;  // [first tile, count]
  for (int t = 0; t < id;) {
    int u = t;
    while (u < id && tlist[u].a == tlist[t].a) ++u;
    for (int f = t; f < u; f += cap) units.push_back({f, std::min(cap, u - f)});
    t = u;
  }
  struct Wave {
    std::vector<int> tiles;
    double load = 0;
  };
  std::vector<std::vector<Wave>> groups;
  auto new_group = [&]() { groups.emplace_back(ps::kCtrWavesHost); };
  // Order 4 in split FP16 with more pair blocks than fit one workgroup's LDS as shared
  // operands: tile groups over rectangles of ka A blocks by kb B blocks (ka + kb within the
  // LDS), the rectangle sizes that give the fewest groups; each group then forms only its
  // own blocks, once per K-step.  Tiles go to the waves in (A, B) order, a contiguous run
  // each.  The grouping follows the precision the plan is made with: the FP32 and BF16
  // contractions, which form pair products per tile, run faster on the greedy groups
  // below (40 shells at 256^3, FP32: 77 against 83 ms); after a switch of precision the
  // plan keeps its grouping (a plan made in FP32 then contracts FP16 without the sharing).
  const int npb = p->n_pairs_padded / 16;
  const int lmax = ps::kMaxPairBlocksHost;
  p->pair_groups = n == 4 && p->prec == POLYSPEC_SPLIT_FP16 && p->n_blk <= 4 && npb > lmax;
  std::vector<int> grp_blk, grp_nblk;
  if (p->pair_groups) {
    int best = -1, bka = 0, bkb = 0;
    for (int ka = 1; ka < lmax; ++ka)
      for (int kb = 1; ka + kb <= lmax; ++kb) {
        std::map<std::pair<int, int>, int> cnt;
        for (const TileKey& k : tlist) ++cnt[{k.a / ka, k.b / kb}];
        int ng = 0;
        for (const auto& kv : cnt) ng += (kv.second + 16 * cap - 1) / (16 * cap);
        if (best < 0 || ng < best) { best = ng; bka = ka; bkb = kb; }
      }
    std::map<std::pair<int, int>, std::vector<int>> rect;   // tiles in (A, B) order
    for (int t = 0; t < id; ++t) rect[{tlist[t].a / bka, tlist[t].b / bkb}].push_back(t);
    for (const auto& kv : rect) {
      const std::vector<int>& tl = kv.second;
      for (size_t f = 0; f < tl.size(); f += 16 * cap) {
        const int cnt = (int)std::min(tl.size() - f, (size_t)16 * cap);
        new_group();
        const int per = (cnt + ps::kCtrWavesHost - 1) / ps::kCtrWavesHost;
        for (int k = 0; k < cnt; ++k) groups.back()[k / per].tiles.push_back(tl[f + k]);
        std::vector<int> blocks;
        for (int k = 0; k < cnt; ++k) {
          blocks.push_back(tlist[tl[f + k]].a);
          blocks.push_back(tlist[tl[f + k]].b);
        }
        std::sort(blocks.begin(), blocks.end());
        blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
        if ((int)blocks.size() > lmax) return p->fail(POLYSPEC_ERR_UNSUPPORTED, "tile group exceeds its pair blocks");
        grp_nblk.push_back((int)blocks.size());
        blocks.resize(lmax, -1);
        grp_blk.insert(grp_blk.end(), blocks.begin(), blocks.end());
      }
    }
  } else {
    // greedy: largest units first, onto the least loaded wave with room
    std::vector<int> order(units.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return units[x].second > units[y].second; });
    new_group();
    for (int ui : order) {
      const int cnt = units[ui].second;
      if (cnt > cap) return p->fail(POLYSPEC_ERR_UNSUPPORTED, "tile unit larger than a wave");
      Wave* best = nullptr;
      for (auto& grp : groups)
        for (auto& w : grp)
          if ((int)w.tiles.size() + cnt <= cap && (!best || w.load < best->load)) best = &w;
      if (!best) {
        new_group();
        best = &groups.back()[0];
      }
      for (int k = 0; k < cnt; ++k) best->tiles.push_back(units[ui].first + k);
      best->load += 1.0 + cnt * (n >= 5 ? 3.0 : n == 4 ? 2.0 : 1.0);   // one A formation + the tiles
    }
  }
  p->n_groups = (int)groups.size();
  // slot tables (see contract_tiles): a uniform byte per slot and per-lane pair shells,
  // laid out with the fixed per-wave stride kSlotsMaxHost
  const int S = ps::kSlotsMaxHost;
  std::vector<int> uni((size_t)p->n_groups * ps::kCtrWavesHost * (S / 4), 0);
  std::vector<int> lanew((size_t)p->n_groups * ps::kCtrWavesHost * 16 * S, 0);
  std::vector<int> slot_tile((size_t)p->n_groups * ps::kCtrWavesHost * S, -1);
  std::vector<int> slot_blk((size_t)p->n_groups * ps::kCtrWavesHost * S, 0);   // A | B << 16 pair blocks
  auto uv8 = [&](int pair) {
    const int w = p->pair_uv[pair];
    return (w & 0xff) | (((w >> 16) & 0xff) << 8);
  };
  for (int gi = 0; gi < p->n_groups; ++gi)
    for (int w = 0; w < ps::kCtrWavesHost; ++w) {
      auto& tl = groups[gi][w].tiles;
      std::sort(tl.begin(), tl.end());
      const size_t gw = (size_t)gi * ps::kCtrWavesHost + w;
      int prev_a = -1;
      for (int s = 0; s < S; ++s) {
        int info = 0x80;
        if (s >= cap) {  // beyond this order's slot count: never read
          uni[gw * (S / 4) + s / 4] |= info << (8 * (s % 4));
          continue;
        }
        if (s < (int)tl.size()) {
          const TileKey k = tlist[tl[s]];
          const int form = k.a != prev_a ? 1 : 0;
          prev_a = k.a;
          info = (n >= 4 ? 0 : (k.b & 7)) | (n == 2 ? (k.a & 7) << 3 : 0) | (form << 6);
          slot_tile[gw * S + s] = tl[s];
          if (p->pair_groups) {   // the group's local block indices
            const int* gb = &grp_blk[(size_t)gi * lmax];
            const int la = (int)(std::find(gb, gb + lmax, k.a) - gb), lb = (int)(std::find(gb, gb + lmax, k.b) - gb);
            slot_blk[gw * S + s] = la | (lb << 16);
          } else {
            slot_blk[gw * S + s] = k.a | (k.b << 16);
          }
          for (int r = 0; r < 16; ++r) {
            int* row_words = &lanew[(gw * 16 + r) * S];
            if (n == 3) row_words[s / 2] |= uv8(16 * k.a + r) << (16 * (s % 2));
            if (n == 4) row_words[s] = uv8(16 * k.a + r) | (uv8(16 * k.b + r) << 16);
            if (n >= 5) {
              row_words[2 * s] = arows[16 * k.a + r];
              row_words[2 * s + 1] = brows[16 * k.b + r];
            }
          }
        }
        uni[gw * (S / 4) + s / 4] |= info << (8 * (s % 4));
      }
    }
  PS_TRY(upload(p, &p->slots_d, uni));
  PS_TRY(upload(p, &p->slot_lane_d, lanew));
  PS_TRY(upload(p, &p->slot_tile_d, slot_tile));
  PS_TRY(upload(p, &p->slot_blk_d, slot_blk));
  PS_TRY(upload(p, &p->pairs_d, p->pair_uv));
  if (p->pair_groups) {
    PS_TRY(upload(p, &p->grp_blk_d, grp_blk));
    PS_TRY(upload(p, &p->grp_nblk_d, grp_nblk));
  }
  return POLYSPEC_OK;
}

// Order 3, shell-block aligned schedule: candidate (i <= j <= k) lives in slot
// jslot(j / 8, i / 16, k / 16) of wave j % 8; used slots get compact tile ids.
polyspec_status build_jsched(polyspec_plan_s* p, std::vector<int>* ent_of_cand) {
  p->jsched = p->order == 3 && p->n_blk <= ps::kMaxBlkHost;
  if (!p->jsched) return POLYSPEC_OK;
  const size_t nc = p->cand.size() / 3;
  std::vector<int> tile((size_t)ps::kJWaves * ps::kJSlots, -1);
  std::vector<unsigned> mask((size_t)ps::kJWaves * 2, 0u);
  auto slot_of = [&](const int* t) {
    return (t[1] % ps::kJWaves) * ps::kJSlots + ps::jslot(t[1] / ps::kJWaves, t[0] / 16, t[2] / 16);
  };
  for (size_t c = 0; c < nc; ++c) tile[slot_of(&p->cand[c * 3])] = 0;
  int id = 0;
  for (int w = 0; w < ps::kJWaves; ++w)
    for (int s = 0; s < ps::kJSlots; ++s) {
      int& t = tile[(size_t)w * ps::kJSlots + s];
      if (t < 0) continue;
      t = id++;
      mask[2 * w + s / 32] |= 1u << (s % 32);
    }
  p->n_tiles_j = id;
  ent_of_cand->resize(nc);
  for (size_t c = 0; c < nc; ++c) {
    const int* t = &p->cand[c * 3];
    (*ent_of_cand)[c] = tile[slot_of(t)] * 256 + tile_entry(t[0] % 16, t[2] % 16);
  }
  PS_TRY(upload(p, &p->jtile_d, tile));
  PS_TRY(upload(p, &p->jmask_d, mask));
  return POLYSPEC_OK;
}

// Plan-time counts: unit-shell fields in float64 on the symmetry wedge, then
// C_t = sum over the wedge of orbit size times the product.
polyspec_status compute_counts(polyspec_plan_s* p) {
  const int N = p->N, h = N / 2, nb = p->nb, n = p->order;
  std::vector<int> rows;
  std::vector<unsigned char> wmult;
  long long off = 0;
  for (int x0 = 0; x0 <= h; ++x0)
    for (int x1 = x0; x1 <= h; ++x1) {
      rows.push_back(x0);
      rows.push_back(x1);
      rows.push_back((int)off);
      for (int x2 = x1; x2 <= h; ++x2) {
        int signs = (x0 != 0 && x0 != h ? 2 : 1) * (x1 != 0 && x1 != h ? 2 : 1) * (x2 != 0 && x2 != h ? 2 : 1);
        int perms = (x0 == x1 && x1 == x2) ? 1 : (x0 == x1 || x1 == x2) ? 3 : 6;
        wmult.push_back((unsigned char)(signs * perms));
      }
      off += h - x1 + 1;
    }
  const long long nwedge = off;
  const int nrows = (int)(rows.size() / 3);
  const size_t n_cand = p->cand.size() / n;

  DevBuf tw64, rows_d, wm_d, cand_d, cw, H1d, H2d, part, tmp;
  auto cleanup = [&]() {
    dev_free(&tw64); dev_free(&rows_d); dev_free(&wm_d); dev_free(&cand_d); dev_free(&cw);
    dev_free(&H1d); dev_free(&H2d); dev_free(&part); dev_free(&tmp);
  };
  polyspec_status st = POLYSPEC_OK;
  do {
    if ((st = upload(p, &tw64, twiddles<double>(N))) != POLYSPEC_OK) break;
    if ((st = upload(p, &rows_d, rows)) != POLYSPEC_OK) break;
    if ((st = upload(p, &wm_d, wmult)) != POLYSPEC_OK) break;
    if ((st = upload(p, &cand_d, p->cand)) != POLYSPEC_OK) break;
    if ((st = dev_alloc(p, &cw, (size_t)nb * nwedge * sizeof(double))) != POLYSPEC_OK) break;
    // shells per group: keep the float64 intermediates near 4 GiB
    const size_t per_shell = ((size_t)N * p->B2 * p->B0 + (size_t)N * N * h2_stride(p)) * sizeof(cplx<double>);
    int gs = (int)std::max<size_t>(1, std::min<size_t>(nb, ((size_t)4 << 30) / std::max<size_t>(per_shell, 1)));
    gs = std::max(1, std::min(gs, nb));
    if ((st = dev_alloc(p, &H1d, (size_t)gs * N * p->B2 * p->B0 * sizeof(cplx<double>))) != POLYSPEC_OK) break;
    if ((st = dev_alloc(p, &H2d, (size_t)gs * N * N * h2_stride(p) * sizeof(cplx<double>))) != POLYSPEC_OK) break;
    hipError_t e = hipSuccess;
    for (int s0 = 0; s0 < nb && e == hipSuccess; s0 += gs) {
      const int cnt = std::min(gs, nb - s0);
      Geom g = make_geom(p, cnt, s0 + 1);
      e = ps::launch_c2r_p1<double, true>(nullptr, (const int16_t*)p->shell_q.p, (const int*)p->qmax_d.p,
                                          (cplx<double>*)H1d.p, (const cplx<double>*)tw64.p, g, cnt, p->stream);
      if (e == hipSuccess)
        e = ps::launch_c2r_p2<double>((const cplx<double>*)H1d.p, (const int*)p->qmax_d.p, (cplx<double>*)H2d.p,
                                      (const cplx<double>*)tw64.p, g, cnt, p->stream);
      if (e == hipSuccess)
        e = ps::launch_c2r_p3_wedge((const cplx<double>*)H2d.p, (const int*)p->qmax_d.p, (const int*)rows_d.p,
                                    nrows, (double*)cw.p + (size_t)s0 * nwedge, nwedge,
                                    (const cplx<double>*)tw64.p, g, cnt, p->stream);
    }
    if (e != hipSuccess) {
      st = p->fail(POLYSPEC_ERR_DEVICE, std::string("count-field transform: ") + hipGetErrorString(e));
      break;
    }
    dev_free(&H1d);
    dev_free(&H2d);
    // contraction over the wedge
    const int spc = 64;  // 32-point stages per chunk: 2048 wedge points
    const long long pts_per_chunk = (long long)spc * ps::kCntStageHost;
    const int n_chunks = (int)((nwedge + pts_per_chunk - 1) / pts_per_chunk);
    if ((st = dev_alloc(p, &part, (size_t)n_chunks * n_cand * sizeof(double2))) != POLYSPEC_OK) break;
    e = ps::launch_counts_wedge(n, (const double*)cw.p, nwedge, (const unsigned char*)wm_d.p, (const int*)cand_d.p,
                                (int)n_cand, nb, spc, n_chunks, (double2*)part.p, p->stream);
    if (e != hipSuccess) {
      st = p->fail(POLYSPEC_ERR_DEVICE, std::string("count contraction: ") + hipGetErrorString(e));
      break;
    }
    const int cpg = 64;
    const int ngr = (n_chunks + cpg - 1) / cpg;
    if ((st = dev_alloc(p, &tmp, (size_t)ngr * n_cand * sizeof(double2))) != POLYSPEC_OK) break;
    e = ps::launch_reduce_dd((const double2*)part.p, (double2*)tmp.p, n_chunks, cpg, ngr, (long long)n_cand, p->stream);
    if (e != hipSuccess) {
      st = p->fail(POLYSPEC_ERR_DEVICE, std::string("count reduction: ") + hipGetErrorString(e));
      break;
    }
    std::vector<double2> host((size_t)ngr * n_cand);
    e = hipMemcpyAsync(host.data(), tmp.p, host.size() * sizeof(double2), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
      st = p->fail(POLYSPEC_ERR_DEVICE, std::string("count readback: ") + hipGetErrorString(e));
      break;
    }
    // N^3 is a power of two, so (hi, lo) / N^3 is exact and the distance to the
    // nearest integer is computed without cancellation
    const double N3 = (double)N * N * N;
    p->cand_quot.assign(n_cand, 0.0);
    p->cand_count.assign(n_cand, 0);
    // Allowed distance to the nearest integer: 1e-3, widened to |q| 2^-46 for
    // large counts, where the FP64 rounding of the count fields themselves (not of
    // the sum, which is compensated) reaches 1e-3.  Counts of 2^44 or more would
    // need a tolerance of 1/4 and are refused.
    double worst = 0.0;
    size_t worst_at = 0;
    bool too_large = false;
    for (size_t c = 0; c < n_cand; ++c) {
      double hi = 0.0, lo = 0.0;
      for (int gi = 0; gi < ngr; ++gi) {
        const double2 v = host[(size_t)gi * n_cand + c];
        const double s = hi + v.x;
        const double bb = s - hi;
        lo += (hi - (s - bb)) + (v.x - bb) + v.y;
        hi = s;
      }
      const double qh = hi / N3, ql = lo / N3;
      const double r = std::rint(qh + ql);
      const double frac = (qh - r) + ql;
      const double tol = std::max(1e-3, std::ldexp(std::fabs(qh), -46));
      p->cand_quot[c] = qh + ql;
      p->cand_count[c] = (int64_t)r;
      if (std::fabs(qh) >= std::ldexp(1.0, 44)) too_large = true;
      if (std::fabs(frac) / tol > worst) {
        worst = std::fabs(frac) / tol;
        worst_at = c;
      }
    }
    if (too_large) {
      st = p->fail(POLYSPEC_ERR_COUNT_NOT_INTEGRAL, "a polygon count reaches 2^44, beyond exact FP64 recovery");
      break;
    }
    if (!(worst < 1.0)) {
      st = p->fail(POLYSPEC_ERR_COUNT_NOT_INTEGRAL,
                   "polygon count quotient " + std::to_string(p->cand_quot[worst_at]) + " of candidate " +
                       std::to_string(worst_at) + " is not within max(1e-3, |q| 2^-46) of an integer");
      break;
    }
  } while (false);
  cleanup();
  return st;
}

// Multipole plans: every closing-candidate triangle (a <= b <= c) of the shells gives a
// tuple for each distinct choice of its weighted side w, (u, v, ns + w) with (u, v) the
// other two sides in order, over the 2 ns fields; lexicographic order, the triangle's
// count and quotient.
void expand_multipoles(polyspec_plan_s* p) {
  const int ns = p->ns;
  std::map<std::array<int, 3>, std::pair<int64_t, double>> rows;
  const size_t nc = p->cand.size() / 3;
  for (size_t c = 0; c < nc; ++c) {
    const int a = p->cand[3 * c], b = p->cand[3 * c + 1], e = p->cand[3 * c + 2];
    const std::pair<int64_t, double> v{p->cand_count[c], p->cand_quot[c]};
    rows[{b, e, a}] = v;
    rows[{a, e, b}] = v;
    rows[{a, b, e}] = v;
  }
  p->cand.clear();
  p->cand_count.clear();
  p->cand_quot.clear();
  for (const auto& kv : rows) {
    p->cand.push_back(kv.first[0]);
    p->cand.push_back(kv.first[1]);
    p->cand.push_back(ns + kv.first[2]);
    p->cand_count.push_back(kv.second.first);
    p->cand_quot.push_back(kv.second.second);
  }
  p->nb = 2 * ns;
  p->n_blk = (p->nb + 15) / 16;
}

polyspec_status build_plan(polyspec_plan_s* p) {
  const polyspec_desc& d = p->desc;
  if (d.N < 32 || d.N > 1024 || (d.N & (d.N - 1)) != 0)
    return p->fail(POLYSPEC_ERR_INVALID_ARG, "N must be a power of two in [32, 1024]");
  if (d.order < 2 || d.order > 6) return p->fail(POLYSPEC_ERR_INVALID_ARG, "order must be 2 to 6");
  if (d.n_shells < 1) return p->fail(POLYSPEC_ERR_INVALID_ARG, "n_shells must be >= 1");
  if (d.batch < 1) return p->fail(POLYSPEC_ERR_INVALID_ARG, "batch must be >= 1");
  if (d.precision < 0 || d.precision > 2) return p->fail(POLYSPEC_ERR_INVALID_ARG, "unknown precision");
  if (!(d.box_length >= 0.0) || !std::isfinite(d.box_length))
    return p->fail(POLYSPEC_ERR_INVALID_ARG, "box_length must be finite and >= 0");
  const uint32_t known = POLYSPEC_INPUT_HALF_SPECTRUM | POLYSPEC_ALLOW_ALIASING | POLYSPEC_NAN_GUARD |
                         POLYSPEC_STREAM_SLABS | POLYSPEC_MULTIPOLE;
  if (d.flags & ~known) return p->fail(POLYSPEC_ERR_INVALID_ARG, "unknown flag bits");
  Dyadic w;
  if (!to_dyadic(d.shell_width, &w)) return p->fail(POLYSPEC_ERR_INVALID_ARG, "shell_width must be finite and > 0");
  if (w.m >= (1LL << 24) || w.e < -40 || w.e > 20)
    return p->fail(POLYSPEC_ERR_INVALID_ARG, "shell_width must be a binary fraction with at most 24 significant bits");
  p->N = d.N;
  p->order = d.order;
  p->nb = d.n_shells;   // shells; a multipole plan doubles it into fields once its counts are known
  p->ns = d.n_shells;
  p->mp = (d.flags & POLYSPEC_MULTIPOLE) != 0;
  if (p->mp) {
    if (d.order != 3) return p->fail(POLYSPEC_ERR_UNSUPPORTED, "multipoles are implemented for order 3");
    if (d.flags & POLYSPEC_STREAM_SLABS) return p->fail(POLYSPEC_ERR_UNSUPPORTED, "multipole plans are not streamed");
    if (2 * d.n_shells > 16 * ps::kMaxTileBlkHost)
      return p->fail(POLYSPEC_ERR_UNSUPPORTED, "a multipole plan handles at most 64 shells");
  }
  p->batch = d.batch;
  p->prec = d.precision;
  p->G = (long long)d.N * d.N * d.N;
  // (2 nb + 1) width <= N: the last shell's outer edge stays below Nyquist
  {
    const long double ke2 = (long double)(2 * d.n_shells + 1) * (long double)d.shell_width;
    if (ke2 > (long double)d.N)
      return p->fail(POLYSPEC_ERR_INVALID_ARG, "(n_shells + 1/2) * shell_width exceeds N/2");
    const long double alias = (long double)d.order * ke2;
    p->alias_free = alias <= 2.0L * (long double)d.N;
    if (!p->alias_free && !(d.flags & POLYSPEC_ALLOW_ALIASING))
      return p->fail(POLYSPEC_ERR_ALIASING,
                     "order * (n_shells + 1/2) * shell_width > N; set POLYSPEC_ALLOW_ALIASING for the mod-N estimator");
  }
  if (d.n_shells > 16 * ps::kMaxTileBlkHost)
    return p->fail(POLYSPEC_ERR_UNSUPPORTED, "the matrix-core contraction handles at most 128 shells");
  if (d.order >= 5 && d.n_shells > ps::kMaxShells56)
    return p->fail(POLYSPEC_ERR_UNSUPPORTED, "orders 5 and 6 handle at most 32 shells");
  if ((d.flags & POLYSPEC_INPUT_HALF_SPECTRUM) && (d.N * (size_t)d.N * (d.N / 2 + 1)) == 0)
    return p->fail(POLYSPEC_ERR_INVALID_ARG, "bad half-spectrum size");

  // shell thresholds: shell s (1-based) holds T_s <= |q|^2 < T_{s+1}
  p->thr.resize(p->nb + 1);
  for (int s = 1; s <= p->nb + 1; ++s) p->thr[s - 1] = ceil_quarter_square(2 * s - 1, w);
  const int64_t qtop = p->thr[p->nb] - 1;  // largest |q|^2 inside the ball
  int Kc = 0;
  while ((int64_t)(Kc + 1) * (Kc + 1) <= qtop) ++Kc;
  p->Kc = Kc;
  p->B0 = 2 * Kc + 1;
  p->B2 = Kc + 1;
  p->n_blk = (p->nb + 15) / 16;
  const int64_t qtab = 3LL * Kc * Kc + 1;
  p->shell_of_q.assign(qtab, 0);
  for (int64_t Q = 0; Q < qtab; ++Q) {
    int s = 0;
    while (s < p->nb && p->thr[s] <= Q) ++s;  // s = number of thresholds <= Q
    p->shell_of_q[Q] = (int16_t)((Q < p->thr[p->nb] && s >= 1) ? s : 0);
  }
  p->qmax.resize(p->nb + 1);
  p->qmax[0] = (int)qtop;
  for (int s = 1; s <= p->nb; ++s) p->qmax[s] = (int)(p->thr[s] - 1);

  build_tuples(p);
  if (p->mp) {
    // the triangles' counts over the shells first, then the weighted-leg tuples
    PS_TRY(upload(p, &p->shell_q, p->shell_of_q));
    PS_TRY(upload(p, &p->qmax_d, p->qmax));
    PS_TRY(compute_counts(p));
    expand_multipoles(p);
  }
  std::vector<int> ent_of_cand;
  PS_TRY(build_tiles(p, &ent_of_cand));
  std::vector<int> ent_j_of_cand;
  PS_TRY(build_jsched(p, &ent_j_of_cand));

  // streamed mode: the largest power-of-two slab whose shell fields take at most
  // 2 GiB (polyspec_set_slab_planes overrides it before the first use)
  p->streamed = (d.flags & POLYSPEC_STREAM_SLABS) != 0;
  if (p->streamed) {
    int s1 = p->N;
    while (s1 > min_slab_planes(p->N) && (size_t)p->batch * p->nb * s1 * (size_t)p->N * p->N * 4 > ((size_t)2 << 30))
      s1 /= 2;
    p->S1 = s1;
    p->n_slabs = p->N / s1;
  }
  set_chunking(p);

  PS_TRY(upload(p, &p->tw32, twiddles<float>(p->N)));
  if (!p->mp) {
    PS_TRY(upload(p, &p->shell_q, p->shell_of_q));
    PS_TRY(upload(p, &p->qmax_d, p->qmax));
    PS_TRY(compute_counts(p));
  }

  const size_t nc = p->cand.size() / p->order;
  std::vector<int> ent, ent_j;
  std::vector<double> fnorm;
  const double N3 = (double)p->N * p->N * p->N;
  double phys = 1.0;
  if (d.box_length > 0) {
    const double V = d.box_length * d.box_length * d.box_length;
    phys = std::pow(V, p->order - 1) / std::pow((double)p->N, 3 * p->order);
  }
  std::vector<int> lookup;
  const bool adj3 = has_adjoint(p) && p->order == 3, adj4 = has_adjoint(p) && p->order == 4;
  if (adj3) lookup.assign((size_t)p->nb * p->nb * p->nb, -1);
  if (adj4) lookup.assign((size_t)p->nb * p->nb * p->nb * p->nb, -1);
  for (size_t c = 0; c < nc; ++c) {
    if (p->cand_count[c] <= 0) continue;
    const int k = (int)p->closing.size();
    p->closing.push_back((int)c);
    for (int j = 0; j < p->order; ++j) p->cl_bins.push_back(p->cand[c * p->order + j]);
    p->cl_counts.push_back(p->cand_count[c]);
    ent.push_back(ent_of_cand[c]);
    if (p->jsched) ent_j.push_back(ent_j_of_cand[c]);
    fnorm.push_back(phys / (N3 * (double)p->cand_count[c]) * (p->mp ? 2.0 * p->ell + 1.0 : 1.0));
    p->fnorm_base.push_back(phys / (N3 * (double)p->cand_count[c]));
    if (adj3) {
      const int* t = &p->cand[c * 3];
      lookup[((size_t)t[0] * p->nb + t[1]) * p->nb + t[2]] = k;
    }
    if (adj4) {
      const int* t = &p->cand[c * 4];
      lookup[(((size_t)t[0] * p->nb + t[1]) * p->nb + t[2]) * p->nb + t[3]] = k;
    }
  }
  PS_TRY(upload(p, &p->ent_d, ent));
  if (p->jsched) PS_TRY(upload(p, &p->ent_j_d, ent_j));
  if (p->streamed) {
    // the reduction of a streamed slab unscales each entry with its tuple's exponents
    std::vector<int> inv((size_t)p->n_tiles * 256, -1);
    for (size_t k = 0; k < ent.size(); ++k) inv[ent[k]] = (int)k;
    PS_TRY(upload(p, &p->closing_of_ent_d, inv));
    if (p->jsched) {
      std::vector<int> inv_j((size_t)p->n_tiles_j * 256, -1);
      for (size_t k = 0; k < ent_j.size(); ++k) inv_j[ent_j[k]] = (int)k;
      PS_TRY(upload(p, &p->closing_of_ent_j_d, inv_j));
    }
  }
  PS_TRY(upload(p, &p->bins_d, p->cl_bins));
  PS_TRY(upload(p, &p->fnorm_d, fnorm));
  PS_TRY(dev_alloc(p, &p->flag_d, 256));
  if (adj3) {
    PS_TRY(upload(p, &p->lookup_d, lookup));
    // for each v: which (16-shell chunk of u, 32-shell block of m) of W[m][(u, v)] can
    // be non-zero, as bits 2 uc + mb (the adjoint GEMM skips the others)
    std::vector<int> wmask(p->nb, 0);
    for (int v = 0; v < p->nb; ++v)
      for (int u = 0; u <= v; ++u)
        for (int m = 0; m < p->nb; ++m) {
          int t[3] = {m, u, v};
          std::sort(t, t + 3);
          if (lookup[((size_t)t[0] * p->nb + t[1]) * p->nb + t[2]] >= 0) wmask[v] |= 1 << (2 * (u / 16) + m / 32);
        }
    p->n_adj_active = p->nb;
    p->wmask_host = wmask;
    PS_TRY(upload(p, &p->wmask_d, wmask));
  }
  if (adj4) {
    PS_TRY(upload(p, &p->lookup_d, lookup));
    // for each item (w, v <= w): which (16-shell chunk uc of u <= v, 32-row block mb of
    // m) hold a weight W4[m][(u, v, w)] (bit 2 uc + mb): each closing tuple, with each of
    // its positions taken by m and the other three (u <= v <= w); the order-4 adjoint
    // skips items without any, and blocks of m without any
    const int nb = p->nb;
    std::vector<int> imask(nb * (nb + 1) / 2, 0);
    for (size_t k = 0; k < p->closing.size(); ++k) {
      const int* t = &p->cl_bins[k * 4];
      for (int pos = 0; pos < 4; ++pos) {
        int rest[3], r = 0;
        for (int j = 0; j < 4; ++j)
          if (j != pos) rest[r++] = t[j];
        imask[rest[2] * (rest[2] + 1) / 2 + rest[1]] |= 1 << (2 * (rest[0] / 16) + t[pos] / 32);
      }
    }
    p->wmask_host = imask;
    PS_TRY(upload(p, &p->wmask_d, imask));
  }
  return POLYSPEC_OK;
}

void release(polyspec_plan_s* p) {
  for (auto& pe : p->ev_pending) {
    p->ev_pool.push_back(pe.second.first);
    p->ev_pool.push_back(pe.second.second);
  }
  p->ev_pending.clear();
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  p->ev_pool.clear();
  DevBuf* bufs[] = {&p->tw32, &p->shell_q, &p->qmax_d, &p->pairs_d, &p->slots_d, &p->slot_lane_d, &p->slot_tile_d, &p->slot_blk_d, &p->ent_d,
                    &p->bins_d, &p->fnorm_d, &p->lookup_d, &p->wmask_d, &p->flag_d, &p->jtile_d, &p->jmask_d,
                    &p->ent_j_d, &p->closing_of_ent_d, &p->closing_of_ent_j_d, &p->grp_blk_d, &p->grp_nblk_d,
                    &p->own_ws};
  for (DevBuf* b : bufs) dev_free(b);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* polyspec_status_string(polyspec_status st) {
  switch (st) {
    case POLYSPEC_OK: return "ok";
    case POLYSPEC_ERR_INVALID_ARG: return "invalid argument";
    case POLYSPEC_ERR_ALIASING: return "configuration aliases";
    case POLYSPEC_ERR_OUT_OF_MEMORY: return "out of memory";
    case POLYSPEC_ERR_DEVICE: return "device error";
    case POLYSPEC_ERR_COUNT_NOT_INTEGRAL: return "polygon count not integral";
    case POLYSPEC_ERR_STATE: return "call out of order";
    case POLYSPEC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* polyspec_last_error(polyspec_plan_t plan) {
  return plan ? plan->last_error.c_str() : g_plan_error.c_str();
}

polyspec_status polyspec_plan(const polyspec_desc* desc, void* stream, polyspec_plan_t* out) {
  g_plan_error.clear();
  if (!desc || !out) {
    g_plan_error = "null descriptor or output pointer";
    return POLYSPEC_ERR_INVALID_ARG;
  }
  *out = nullptr;
  polyspec_plan_s* p = new (std::nothrow) polyspec_plan_s;
  if (!p) {
    g_plan_error = "host allocation failed";
    return POLYSPEC_ERR_OUT_OF_MEMORY;
  }
  p->desc = *desc;
  p->stream = (hipStream_t)stream;
  // the static scratch of this device, looked up once per device with it current
  if (hipGetDevice(&p->device) == hipSuccess) {
    p->static_scratch_status = ps::static_scratch_address(p->device, &p->static_scratch);
  } else {
    (void)hipGetLastError();
    p->static_scratch_status = hipErrorInvalidDevice;
  }
  polyspec_status st;
  try {
    st = build_plan(p);
  } catch (const std::bad_alloc&) {
    st = p->fail(POLYSPEC_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    st = p->fail(POLYSPEC_ERR_INVALID_ARG, "unexpected failure while building the plan");
  }
  if (st != POLYSPEC_OK) {
    g_plan_error = p->last_error;
    release(p);
    delete p;
    return st;
  }
  *out = p;
  return POLYSPEC_OK;
}

polyspec_status polyspec_workspace_size(polyspec_plan_t p, size_t* bytes) {
  if (!p || !bytes) return POLYSPEC_ERR_INVALID_ARG;
  *bytes = layout_of(p).total;
  return POLYSPEC_OK;
}

polyspec_status polyspec_set_workspace(polyspec_plan_t p, void* d_ptr, size_t bytes) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (p->ws) return p->fail(POLYSPEC_ERR_STATE, "workspace already set or allocated");
  if (!d_ptr || ((uintptr_t)d_ptr & 255)) return p->fail(POLYSPEC_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < layout_of(p).total) return p->fail(POLYSPEC_ERR_INVALID_ARG, "workspace too small");
  p->ws = (char*)d_ptr;
  p->ws_size = bytes;
  carve(p, p->ws);
  return POLYSPEC_OK;
}

polyspec_status polyspec_set_precision(polyspec_plan_t p, int32_t precision) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (precision < 0 || precision > 2) return p->fail(POLYSPEC_ERR_INVALID_ARG, "unknown precision");
  p->prec = precision;
  return POLYSPEC_OK;
}

polyspec_status polyspec_set_slab_planes(polyspec_plan_t p, int32_t planes) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!p->streamed) return p->fail(POLYSPEC_ERR_STATE, "slab planes apply to plans made with POLYSPEC_STREAM_SLABS");
  if (p->ws) return p->fail(POLYSPEC_ERR_STATE, "the workspace is already sized");
  if (planes < min_slab_planes(p->N) || planes > p->N || (planes & (planes - 1)) != 0)
    return p->fail(POLYSPEC_ERR_INVALID_ARG, "planes must be a power of two between " +
                                                 std::to_string(min_slab_planes(p->N)) + " and N");
  p->S1 = planes;
  p->n_slabs = p->N / planes;
  set_chunking(p);
  return POLYSPEC_OK;
}

polyspec_status polyspec_slab_planes(polyspec_plan_t p, int32_t* planes) {
  if (!p || !planes) return POLYSPEC_ERR_INVALID_ARG;
  *planes = p->streamed ? p->S1 : p->N;
  return POLYSPEC_OK;
}

// The contraction scales every shell field by a power of two (from its largest
// magnitude) for the FP16 split, and at orders 5 and 6 for every precision.
static bool scaled_contraction(const polyspec_plan_s* p) {
  return p->prec == POLYSPEC_SPLIT_FP16 || p->order >= 5;
}

// Last two inverse passes for the x1-planes [x1_0, x1_0 + S1) of every shell (the whole
// grid when not streamed), optionally with the per-field maxima.
static polyspec_status shell_slab(polyspec_plan_t p, int slab, unsigned* absmax_part) {
  Geom gs = make_geom(p, p->nb, 1);
  if (p->streamed) {
    gs.S1 = p->S1;
    gs.x1_0 = slab * p->S1;
  }
  const int nz = p->batch * p->nb;
  hipStream_t st = p->stream;
  PS_TIMED(p, POLYSPEC_PH_SHELL_P2, ps::launch_c2r_p2<float>(p->H1, (const int*)p->qmax_d.p, p->H2, (const cplx<float>*)p->tw32.p, gs, nz,
                                     st));
  PS_TIMED(p, POLYSPEC_PH_SHELL_P3, ps::launch_c2r_p3(p->H2, (const int*)p->qmax_d.p, p->D, absmax_part,
                                                      (const cplx<float>*)p->tw32.p, gs, nz, st));
  return POLYSPEC_OK;
}

// Per-field maxima of resident shell fields (the scaling of the contraction's operands).
static polyspec_status field_maxima(polyspec_plan_t p) {
  const int nz = p->batch * p->nb;
  hipStream_t st = p->stream;
  PS_HIP(p, ps::launch_fill_u32(p->absmax_part, 0u, (size_t)nz * ps::kAbsmaxSpreadHost, st));
  PS_HIP(p, ps::launch_fields_absmax(p->D, p->G, nz, p->absmax_part, ps::kAbsmaxSpreadHost, st));
  PS_HIP(p, ps::launch_reduce_absmax(p->absmax_part, p->absmax, nz, st));
  p->absmax_valid = true;
  return POLYSPEC_OK;
}

// a0-a2 into the carved workspace (which the caller has provided or allocated).
static polyspec_status shells_impl(polyspec_plan_t p, const void* d_delta) {
  const int nz = p->batch * p->nb;
  hipStream_t st = p->stream;
  Geom gin = make_geom(p, 0, 0);
  if (p->desc.flags & POLYSPEC_INPUT_HALF_SPECTRUM) {
    PS_HIP(p, ps::launch_box_from_half_spectrum((const cplx<float>*)d_delta, p->box, gin, p->batch, st));
  } else {
    // the input transform uses H2 and H1 as scratch (sized for it in streamed plans too)
    PS_TIMED(p, POLYSPEC_PH_INPUT_Q3, ps::launch_r2c_q3((const float*)d_delta, p->H2, (const cplx<float>*)p->tw32.p, gin, p->batch, st));
    PS_TIMED(p, POLYSPEC_PH_INPUT_Q2, ps::launch_r2c_q2(p->H2, p->H1, (const cplx<float>*)p->tw32.p, gin, p->batch, st));
    PS_TIMED(p, POLYSPEC_PH_INPUT_Q1, ps::launch_r2c_q1<false>(p->H1, (const int16_t*)p->shell_q.p, (const int*)p->qmax_d.p, p->box,
                                       (const cplx<float>*)p->tw32.p, gin, p->batch, st));
  }
  Geom gs = make_geom(p, p->nb, 1);
  PS_TIMED(p, POLYSPEC_PH_SHELL_P1, ps::launch_c2r_p1<float, false>(p->box, (const int16_t*)p->shell_q.p, (const int*)p->qmax_d.p, p->H1,
                                            (const cplx<float>*)p->tw32.p, gs, nz, st));
  p->absmax_valid = false;
  if (!p->streamed) {   // a streamed plan makes its fields slab by slab in polyspec_contract
    const bool want_max = scaled_contraction(p);
    if (want_max) PS_HIP(p, ps::launch_fill_u32(p->absmax_part, 0u, (size_t)nz * ps::kAbsmaxSpreadHost, st));
    PS_TRY(shell_slab(p, 0, want_max ? p->absmax_part : nullptr));
    if (want_max) PS_HIP(p, ps::launch_reduce_absmax(p->absmax_part, p->absmax, nz, st));
    p->absmax_valid = want_max;
  }
  p->have_fields = true;
  return POLYSPEC_OK;
}

polyspec_status polyspec_shells(polyspec_plan_t p, const void* d_delta) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!d_delta) return p->fail(POLYSPEC_ERR_INVALID_ARG, "null input");
  PS_TRY(ensure_workspace(p));
  return shells_impl(p, d_delta);
}

// One contraction launch over the fields in D (the whole grid or one slab) and its
// FP64 reduction over chunks into p->red, added to what is there when `accumulate`.
// Returns the tile entries and entry table that the gather needs.
static polyspec_status contract_launch(polyspec_plan_t p, bool accumulate, long long* n_ent, int* groups,
                                       const int** ent) {
  hipStream_t st = p->stream;
  int n_chunks;
  if (p->jsched && p->prec == POLYSPEC_SPLIT_FP16 && p->ksteps_j % 4 == 0) {   // whole 256-point stages
    ps::CtrJParams jp;
    jp.D = p->D;
    jp.absmax = p->absmax;
    jp.tile_of_slot = (const int*)p->jtile_d.p;
    jp.slot_mask = (const unsigned*)p->jmask_d.p;
    jp.partials = p->partials;
    jp.G = launch_points(p);
    jp.n_shells = p->nb;
    jp.n_blk = p->n_blk;
    jp.n_tiles = p->n_tiles_j;
    jp.ksteps = p->ksteps_j;
    jp.n_chunks = p->n_chunks_j;
    PS_TIMED(p, POLYSPEC_PH_CONTRACT, ps::launch_contract_j3(p->prec, jp, p->batch, st));
    *n_ent = (long long)p->n_tiles_j * 256;
    n_chunks = p->n_chunks_j;
    *ent = (const int*)p->ent_j_d.p;
  } else {
    ps::CtrParams cp;
    cp.D = p->D;
    cp.pair_uv = (const int*)p->pairs_d.p;
    cp.slot_uni = (const int*)p->slots_d.p;
    cp.slot_lane = (const int*)p->slot_lane_d.p;
    cp.slot_tile = (const int*)p->slot_tile_d.p;
    cp.slot_blk = (const int*)p->slot_blk_d.p;
    cp.absmax = p->absmax;
    cp.partials = p->partials;
    cp.G = launch_points(p);
    cp.n_shells = p->nb;
    cp.n_blk = p->n_blk;
    cp.n_pairs_padded = p->n_pairs_padded;
    cp.n_tiles = p->n_tiles;
    cp.ksteps = p->ksteps;
    cp.n_chunks = p->n_chunks;
    // order 4 in split FP16: every pair operand formed once per K-step, shared through LDS
    // (with more pair blocks than fit, each tile group's own blocks)
    const int npb = p->n_pairs_padded / 16;
    const bool plds = p->order == 4 && p->prec == POLYSPEC_SPLIT_FP16 && p->n_blk <= 4;
    cp.n_pair_blocks = !plds ? 0 : p->pair_groups ? ps::kMaxPairBlocksHost : npb;
    cp.grp_blk = plds && p->pair_groups ? (const int*)p->grp_blk_d.p : nullptr;
    cp.grp_nblk = plds && p->pair_groups ? (const int*)p->grp_nblk_d.p : nullptr;
    PS_TIMED(p, POLYSPEC_PH_CONTRACT, ps::launch_contract(p->prec, p->order, cp, p->n_groups, p->batch, st));
    *n_ent = (long long)p->n_tiles * 256;
    n_chunks = p->n_chunks;
    *ent = (const int*)p->ent_d.p;
  }
  // chunk groups of red_cpg chunks; the aligned kernel has at most as many chunks
  *groups = (n_chunks + p->red_cpg - 1) / p->red_cpg;
  // a streamed slab's operands carry the slab's own scales: removed here, per entry
  const int* closing_of_entry = nullptr;
  if (p->streamed && scaled_contraction(p))
    closing_of_entry = (const int*)(*ent == (const int*)p->ent_j_d.p ? p->closing_of_ent_j_d.p : p->closing_of_ent_d.p);
  PS_TIMED(p, POLYSPEC_PH_REDUCE, ps::launch_reduce_f32(p->partials, p->red, n_chunks, p->red_cpg, *groups, *n_ent,
                                                        accumulate, closing_of_entry, (const int*)p->bins_d.p,
                                                        p->order, p->absmax, p->nb, p->prec, p->batch, st));
  return POLYSPEC_OK;
}

polyspec_status polyspec_contract(polyspec_plan_t p, double* d_out, double* d_raw_sums) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!d_out) return p->fail(POLYSPEC_ERR_INVALID_ARG, "null output");
  if (!p->have_fields) return p->fail(POLYSPEC_ERR_STATE, "polyspec_contract before polyspec_shells");
  hipStream_t st = p->stream;
  const bool scaled = scaled_contraction(p);
  if (scaled && !p->streamed && !p->absmax_valid) PS_TRY(field_maxima(p));  // precision switched after shells
  long long n_ent = 0;
  int groups = 0;
  const int* ent = nullptr;
  if (p->streamed) {
    // slab by slab: the slab's fields (and, when the operands are scaled, the slab's own
    // per-field maxima), its contraction, and its sums unscaled and added in FP64 in
    // slab order (a fixed order, so reruns are bitwise equal)
    const int nz = p->batch * p->nb;
    for (int k = 0; k < p->n_slabs; ++k) {
      if (scaled) PS_HIP(p, ps::launch_fill_u32(p->absmax_part, 0u, (size_t)nz * ps::kAbsmaxSpreadHost, st));
      PS_TRY(shell_slab(p, k, scaled ? p->absmax_part : nullptr));
      if (scaled) PS_HIP(p, ps::launch_reduce_absmax(p->absmax_part, p->absmax, nz, st));
      PS_TRY(contract_launch(p, k > 0, &n_ent, &groups, &ent));
    }
  } else {
    PS_TRY(contract_launch(p, false, &n_ent, &groups, &ent));
  }
  const bool guard = p->desc.flags & POLYSPEC_NAN_GUARD;
  if (guard) PS_HIP(p, ps::launch_fill_u32(p->flag_d.p, 0u, 1, st));
  const int ncl = (int)p->closing.size();
  if (ncl > 0)
    PS_TIMED(p, POLYSPEC_PH_GATHER, ps::launch_gather(p->red, groups, n_ent, ent, (const int*)p->bins_d.p,
                                p->order, (const double*)p->fnorm_d.p, ncl, p->streamed ? nullptr : p->absmax,
                                p->nb, p->prec, d_out,
                                d_raw_sums, guard ? (int*)p->flag_d.p : nullptr, p->batch, st));
  if (guard) {
    int flag = 0;
    PS_HIP(p, hipMemcpyAsync(&flag, p->flag_d.p, sizeof(int), hipMemcpyDeviceToHost, st));
    PS_HIP(p, hipStreamSynchronize(st));
    if (flag) return p->fail(POLYSPEC_ERR_DEVICE, "non-finite polyspectrum value");
  }
  return POLYSPEC_OK;
}

// The workspace pointers carved from the plan's workspace, and the state that refers to
// them: saved and restored around a call that runs on the static scratch instead.
namespace {
struct CarvedState {
  char* ws;
  size_t ws_size;
  cplx<float>*box, *gbox, *H1, *H1a, *H2;
  float *D, *A, *partials, *W;
  double* red;
  unsigned *absmax, *absmax_part;
  unsigned long long* rowmax;
  bool have_fields, absmax_valid, prof;
};
CarvedState save_carved(const polyspec_plan_s* p) {
  return {p->ws, p->ws_size, p->box, p->gbox, p->H1, p->H1a, p->H2, p->D, p->A, p->partials, p->W,
          p->red, p->absmax, p->absmax_part, p->rowmax, p->have_fields, p->absmax_valid, p->prof};
}
void restore_carved(polyspec_plan_s* p, const CarvedState& c) {
  p->ws = c.ws; p->ws_size = c.ws_size; p->box = c.box; p->gbox = c.gbox; p->H1 = c.H1; p->H1a = c.H1a;
  p->H2 = c.H2; p->D = c.D; p->A = c.A; p->partials = c.partials; p->W = c.W; p->red = c.red;
  p->absmax = c.absmax; p->absmax_part = c.absmax_part; p->rowmax = c.rowmax;
  p->have_fields = c.have_fields; p->absmax_valid = c.absmax_valid; p->prof = c.prof;
}
}  // namespace

static_assert(POLYSPEC_STATIC_SCRATCH_BYTES == ps::kStaticScratchBytes, "header and library agree on the scratch size");

polyspec_status polyspec_forward_static(polyspec_plan_t p, const void* d_delta, double* d_out, double* d_raw_sums) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!d_delta || !d_out) return p->fail(POLYSPEC_ERR_INVALID_ARG, "null input or output");
  const size_t need = layout_of(p).total;
  if (need > ps::kStaticScratchBytes)
    return p->fail(POLYSPEC_ERR_UNSUPPORTED, "the plan needs " + std::to_string(need) +
                                                 " bytes of workspace; the static scratch holds " +
                                                 std::to_string(ps::kStaticScratchBytes));
  if (p->static_scratch_status != hipSuccess || p->static_scratch == nullptr)
    return p->fail(POLYSPEC_ERR_DEVICE, std::string("static scratch unavailable: ") +
                                            hipGetErrorString(p->static_scratch_status));
  int cur = -1;
  PS_HIP(p, hipGetDevice(&cur));
  if (cur != p->device) return p->fail(POLYSPEC_ERR_INVALID_ARG, "the plan's device is not the current device");
  // run shells + contract on the static scratch; the plan's own workspace (if any) and
  // the fields kept in it are untouched.  Event timing is off for the call (it would
  // create events).
  const CarvedState saved = save_carved(p);
  p->ws = (char*)p->static_scratch;
  p->ws_size = ps::kStaticScratchBytes;
  carve(p, p->ws);
  p->prof = false;
  polyspec_status st = shells_impl(p, d_delta);
  if (st == POLYSPEC_OK) st = polyspec_contract(p, d_out, d_raw_sums);
  restore_carved(p, saved);
  return st;
}

polyspec_status polyspec_backward(polyspec_plan_t p, const double* d_grad_out, void* d_grad_delta) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!has_adjoint(p))
    return p->fail(POLYSPEC_ERR_UNSUPPORTED,
                   "backward is implemented for orders 3 and 4 with at most 64 shells "
                   "(not for multipole plans)");
  if (!d_grad_out || !d_grad_delta) return p->fail(POLYSPEC_ERR_INVALID_ARG, "null pointer");
  if (!p->have_fields) return p->fail(POLYSPEC_ERR_STATE, "polyspec_backward before polyspec_shells");
  hipStream_t st = p->stream;
  const int nz = p->batch * p->nb;
  const int ncl = (int)p->closing.size();
  // adjoint arithmetic: FP32, or the split of the plan's precision; a streamed plan's
  // field scales are per slab, so its FP16 mode takes the BF16 split (no scaling needed)
  const int aprec = p->prec == POLYSPEC_FP32 ? 0 : (p->prec == POLYSPEC_SPLIT_FP16 && !p->streamed) ? 2 : 1;
  if (aprec == 2 && !p->absmax_valid) PS_TRY(field_maxima(p));   // precision switched after shells
  Geom gs = make_geom(p, p->nb, 1);
  const cplx<float>* tw = (const cplx<float>*)p->tw32.p;
  const bool fused = ps::adjoint_fuses_rows(p->N);   // the kernel also runs the x2 -> q2 pass
  if (p->order == 3) {
    PS_TIMED(p, POLYSPEC_PH_ADJ_WEIGHTS,
             ps::launch_adjoint_weights(d_grad_out, (const double*)p->fnorm_d.p, (const int*)p->lookup_d.p, p->nb,
                                        ncl, aprec, p->absmax, p->rowmax, (uint4*)p->W, p->batch, st));
  } else {
    PS_TIMED(p, POLYSPEC_PH_ADJ_WEIGHTS,
             ps::launch_adjoint4_weights(d_grad_out, (const double*)p->fnorm_d.p, (const int*)p->lookup_d.p, p->nb,
                                         ncl, aprec, p->absmax, p->rowmax, (uint4*)p->W, p->batch, st));
  }
  // a streamed plan keeps the forward's first pass in H1 for the next slabs, so the
  // adjoint's x1 rows go to a buffer of their own
  cplx<float>* H1x = p->streamed ? p->H1a : p->H1;
  // a_m on the fields in D (the whole grid, or one slab), then its x2 and x0 transforms
  // into rows x1 of H1x
  auto adjoint_rows = [&](int slab) -> polyspec_status {
    Geom gk = gs;
    if (p->streamed) {
      gk.S1 = p->S1;
      gk.x1_0 = slab * p->S1;
    }
    const long long Gk = launch_points(p);
    if (p->order == 3)
      PS_TIMED(p, POLYSPEC_PH_ADJ_GEMM,
               ps::launch_adjoint_gemm(aprec, p->D, (const uint4*)p->W, (const int*)p->wmask_d.p, p->absmax,
                                       p->rowmax, p->nb, Gk, fused ? nullptr : p->A, fused ? p->H2 : nullptr, tw,
                                       gk, p->batch, st));
    else
      PS_TIMED(p, POLYSPEC_PH_ADJ_GEMM,
               ps::launch_adjoint4_gemm(aprec, p->D, (const uint4*)p->W, (const int*)p->wmask_d.p, p->absmax,
                                        p->rowmax, p->nb, Gk, fused ? nullptr : p->A, fused ? p->H2 : nullptr, tw,
                                        gk, p->batch, st));
    if (!fused) PS_TIMED(p, POLYSPEC_PH_ADJ_Q3, ps::launch_r2c_q3(p->A, p->H2, tw, gk, nz, st));
    PS_TIMED(p, POLYSPEC_PH_ADJ_Q2, ps::launch_r2c_q2(p->H2, H1x, tw, gk, nz, st));
    return POLYSPEC_OK;
  };
  if (p->streamed) {
    for (int k = 0; k < p->n_slabs; ++k) {   // the slab's fields again, then its adjoint rows
      PS_TRY(shell_slab(p, k, nullptr));
      PS_TRY(adjoint_rows(k));
    }
  } else {
    PS_TRY(adjoint_rows(0));
  }
  const size_t box_elems = (size_t)p->B0 * p->B2 * p->B0;
  PS_HIP(p, ps::launch_fill_u32(p->gbox, 0u, (size_t)p->batch * box_elems * 2, st));
  PS_TIMED(p, POLYSPEC_PH_ADJ_Q1, ps::launch_r2c_q1<true>(H1x, (const int16_t*)p->shell_q.p, (const int*)p->qmax_d.p, p->gbox, tw, gs,
                                    nz, st));
  Geom gall = make_geom(p, 0, 0);
  if (p->desc.flags & POLYSPEC_INPUT_HALF_SPECTRUM) {
    // the gradient stays in the input's space: the half spectrum, weighted by how often
    // the inverse real transform reads each entry
    PS_HIP(p, ps::launch_half_spectrum_from_box(p->gbox, (cplx<float>*)d_grad_delta, gall, p->batch, st));
    return POLYSPEC_OK;
  }
  float* grad_x = (float*)d_grad_delta;
  PS_TIMED(p, POLYSPEC_PH_GRAD_P1, ps::launch_c2r_p1<float, false>(p->gbox, (const int16_t*)p->shell_q.p, (const int*)p->qmax_d.p, H1x,
                                            tw, gall, p->batch, st));
  PS_TIMED(p, POLYSPEC_PH_GRAD_P2, ps::launch_c2r_p2<float>(H1x, (const int*)p->qmax_d.p, p->H2, tw, gall, p->batch, st));
  PS_TIMED(p, POLYSPEC_PH_GRAD_P3, ps::launch_c2r_p3(p->H2, (const int*)p->qmax_d.p, grad_x, nullptr, tw, gall, p->batch, st));
  return POLYSPEC_OK;
}

polyspec_status polyspec_tuples(polyspec_plan_t p, int64_t* n_closing, int32_t* h_bins, int64_t* h_counts) {
  if (!p || !n_closing) return POLYSPEC_ERR_INVALID_ARG;
  *n_closing = (int64_t)p->closing.size();
  if (h_bins)   // 1-based shells (a multipole plan's last, weighted field reported as its shell)
    for (size_t i = 0; i < p->cl_bins.size(); ++i) h_bins[i] = p->cl_bins[i] % (p->mp ? p->ns : 1 << 30) + 1;
  if (h_counts) std::memcpy(h_counts, p->cl_counts.data(), p->cl_counts.size() * sizeof(int64_t));
  return POLYSPEC_OK;
}

polyspec_status polyspec_candidates(polyspec_plan_t p, int64_t* n_candidates, int32_t* h_bins, double* h_quotients) {
  if (!p || !n_candidates) return POLYSPEC_ERR_INVALID_ARG;
  *n_candidates = (int64_t)(p->cand.size() / p->order);
  if (h_bins)
    for (size_t i = 0; i < p->cand.size(); ++i) h_bins[i] = p->cand[i] % (p->mp ? p->ns : 1 << 30) + 1;
  if (h_quotients) std::memcpy(h_quotients, p->cand_quot.data(), p->cand_quot.size() * sizeof(double));
  return POLYSPEC_OK;
}

polyspec_status polyspec_set_multipole(polyspec_plan_t p, int32_t ell) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  if (!p->mp) return p->fail(POLYSPEC_ERR_STATE, "the plan was not made with POLYSPEC_MULTIPOLE");
  if (ell < 0 || ell > 16 || (ell & 1)) return p->fail(POLYSPEC_ERR_INVALID_ARG, "ell must be even, 0 to 16");
  std::vector<double> fnorm(p->fnorm_base.size());
  for (size_t k = 0; k < fnorm.size(); ++k) fnorm[k] = p->fnorm_base[k] * (2.0 * ell + 1.0);
  // on the plan's stream, after any gather still reading the factors
  PS_HIP(p, hipMemcpyAsync(p->fnorm_d.p, fnorm.data(), fnorm.size() * sizeof(double), hipMemcpyHostToDevice,
                           p->stream));
  PS_HIP(p, hipStreamSynchronize(p->stream));
  p->ell = ell;
  p->have_fields = false;   // the weighted fields of the previous ell are stale
  p->absmax_valid = false;
  return POLYSPEC_OK;
}

polyspec_status polyspec_fields(polyspec_plan_t p, const float** d_fields) {
  if (!p || !d_fields) return POLYSPEC_ERR_INVALID_ARG;
  if (!p->have_fields) return p->fail(POLYSPEC_ERR_STATE, "no shell fields yet");
  if (p->streamed) return p->fail(POLYSPEC_ERR_STATE, "a streamed plan keeps no whole shell fields");
  *d_fields = p->D;
  return POLYSPEC_OK;
}

polyspec_status polyspec_profile(polyspec_plan_t p, int32_t enable) {
  if (!p) return POLYSPEC_ERR_INVALID_ARG;
  p->prof = enable != 0;
  return POLYSPEC_OK;
}

polyspec_status polyspec_profile_read(polyspec_plan_t p, double* h_ms, int64_t* h_launches) {
  if (!p || !h_ms) return POLYSPEC_ERR_INVALID_ARG;
  PS_HIP(p, hipStreamSynchronize(p->stream));
  for (auto& pe : p->ev_pending) {
    float ms = 0.f;
    PS_HIP(p, hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
    p->prof_ms[pe.first] += ms;
    p->prof_calls[pe.first] += 1;
    p->ev_pool.push_back(pe.second.first);
    p->ev_pool.push_back(pe.second.second);
  }
  p->ev_pending.clear();
  for (int i = 0; i < POLYSPEC_N_PHASES; ++i) {
    h_ms[i] = p->prof_ms[i];
    if (h_launches) h_launches[i] = p->prof_calls[i];
    p->prof_ms[i] = 0.0;
    p->prof_calls[i] = 0;
  }
  return POLYSPEC_OK;
}

polyspec_status polyspec_issued_flops(polyspec_plan_t p, int32_t phase, double* flops) {
  if (!p || !flops) return POLYSPEC_ERR_INVALID_ARG;
  if (phase < 0 || phase >= POLYSPEC_N_PHASES) return p->fail(POLYSPEC_ERR_INVALID_ARG, "unknown phase");
  const double terms = p->prec == POLYSPEC_FP32 ? 1.0 : 3.0;   // split: hi*hi + hi*lo + lo*hi
  const double pts = (double)p->G * p->batch;
  *flops = 0.0;
  if (phase == POLYSPEC_PH_CONTRACT) {
    // a 16 x 16 tile is 2 * 256 flops per grid point and product term
    const bool aligned = p->jsched && p->prec == POLYSPEC_SPLIT_FP16 && p->ksteps_j % 4 == 0;
    *flops = (aligned ? p->n_tiles_j : p->n_tiles) * 512.0 * terms * pts;
  } else if (phase == POLYSPEC_PH_ADJ_GEMM && p->order == 4 && p->nb <= ps::kAdj4MaxShells) {
    // per item (w, v): the 16-shell chunks of u <= v, for each 32-row block of m with a
    // weight (the only block up to 32 shells)
    double blocks = 0.0;
    const int mbn = p->nb > 32 ? 2 : 1;
    for (int w = 0; w < p->nb; ++w)
      for (int v = 0; v <= w; ++v) {
        const int mask = p->wmask_host[w * (w + 1) / 2 + v];
        if (!mask) continue;
        for (int mb = 0; mb < mbn; ++mb)
          if (mbn == 1 || (mask & (0x55 << mb))) blocks += v / 16 + 1;
      }
    *flops = blocks * 32.0 * 32.0 * 16.0 * 2.0 / 32.0 * terms * pts;
  } else if (phase == POLYSPEC_PH_ADJ_GEMM && p->order == 3 && has_adjoint(p)) {
    // per partner shell v, 32 x 32 x 16 products per 32 grid points: for v >= 16 in FP32
    // and BF16 every (16-shell chunk u <= v, 32-row block of m); otherwise the blocks
    // that hold a weight (the adjoint's arithmetic is that of backward())
    const bool fp16 = p->prec == POLYSPEC_SPLIT_FP16 && !p->streamed;
    const int mbn = p->nb > 32 ? 2 : 1;
    double blocks = 0.0;
    for (int v = 0; v < p->nb; ++v) {
      const int mask = p->wmask_host[v];
      if (!mask) continue;
      if (!fp16 && v >= 16) {
        blocks += mbn * (v / 16 + 1);
        continue;
      }
      for (int mb = 0; mb < mbn; ++mb)
        for (int uc = 0; uc <= v / 16; ++uc) blocks += (mask >> (2 * uc + mb)) & 1;
    }
    *flops = blocks * 32.0 * 32.0 * 16.0 * 2.0 / 32.0 * terms * pts;
  }
  return POLYSPEC_OK;
}

polyspec_status polyspec_destroy(polyspec_plan_t p) {
  if (!p) return POLYSPEC_OK;
  (void)hipStreamSynchronize(p->stream);
  release(p);
  delete p;
  return POLYSPEC_OK;
}

}  // extern "C"

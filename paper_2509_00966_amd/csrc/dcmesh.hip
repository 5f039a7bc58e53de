// Host side of the C ABI declared in include/dcmesh.h: argument validation,
// workspace layout, work lists, kernel sequencing and graph capture.
//
// One call = one "plan": the domain descriptors and the per-kernel work lists
// are built on the host, copied into the head of the caller's workspace from a
// pinned staging buffer, and every kernel launch then covers all domains of
// the call at once (one launch per kernel family and tile variant).
#include "dcmesh.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"
#include "gemm_split.hpp"
#include "reduce.hpp"
#include "stencil.hpp"

using namespace dcm;

// Device scratch of the allocation-free entry point dcmesh_step_noalloc (its
// maximum workspace size; see dcmesh.h).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(DCMESH_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

bool is_fp64(int prec) { return prec == DCMESH_FP64; }
bool is_split(int prec) { return prec == DCMESH_SPLIT_BF16 || prec == DCMESH_SPLIT_FP16; }
size_t real_size(int prec) { return is_fp64(prec) ? 8 : 4; }

// ---------------------------------------------------------------------------
// Tile variants and tuning overrides
// ---------------------------------------------------------------------------
struct StencilVariant { int oc, tx, ty, nt; };
// variants 6 and 7 prefetch two planes ahead with a double-buffered LDS plane
// variants 8-12 fetch each plane's halo with its interior: 8 with the queues
// shifted per plane (k_stencil_sweep3), 9-12 with unrolled register rings
// (k_stencil_sweep4); FP32 variant 12 runs the 8 x 8 tile on 16 waves, one
// column per thread (FP64 runs it as 11)
const StencilVariant kStencilF32[] = {{16, 16, 8, 256}, {8, 16, 8, 256}, {16, 8, 8, 256},
                                      {4, 16, 16, 256}, {16, 8, 8, 512}, {16, 16, 8, 512},
                                      {16, 8, 8, 512}, {16, 8, 8, 256}, {16, 8, 8, 512},
                                      {16, 8, 8, 512}, {16, 8, 8, 256}, {16, 16, 8, 512},
                                      {16, 8, 8, 1024}};
const StencilVariant kStencilF64[] = {{8, 16, 8, 256}, {8, 8, 8, 256}, {4, 16, 8, 256},
                                      {16, 8, 4, 256}, {8, 8, 8, 512}, {8, 16, 8, 512},
                                      {8, 8, 8, 512}, {8, 8, 8, 256}, {8, 8, 8, 512},
                                      {8, 8, 8, 512}, {8, 8, 8, 256}, {8, 16, 8, 512},
                                      {8, 16, 8, 512}};
constexpr int kNStencil = 13;
constexpr int kFirstSweep3 = 8;
constexpr int kFirstSweep4 = 9;   // variants 9-12: the ring sweep (k_stencil_sweep4)
constexpr int kStencilFallback = 2;
constexpr int kStencilDefaultF32 = 11;   // measured best at 64^3 / 128 orbitals
constexpr int kStencilDefaultF64 = 2;    // the 16-wide FP64 ring sweep spills
// z planes per sweep segment: 0 = chosen from the block count, else fixed
const int kZsegOpt[] = {0, 8, 16, 32, 1 << 20};
constexpr int kNZseg = 5;

struct GemmVariant { int bm, bn; };
// FP32 variant 0 of each product is the three-product (Gauss) kernel; its tile
// in complex orbitals is half the real-column tile listed here.
const GemmVariant kProjF32[] = {{128, 128}, {64, 64}, {64, 128}, {128, 256}};
const GemmVariant kProjF64[] = {{64, 64}, {32, 32}, {64, 32}, {32, 64}};
// FP32 variants 4 and 5: the three-product kernel with direct LDS loads on
// 128 and 64 projectors; variant 7: the three-product kernel through
// registers on 64 projectors x 32 complex orbitals (any row length); variant
// 8: every orbital of a domain (up to 96) in one block, 64 projectors.  Split
// variants 4, 5 and 6: the projector planes loaded into LDS directly, on four
// waves with two stages (128 x 128), on eight waves with three (128 x 256),
// and on four waves with two stages (64 x 64).  Other modes run variants 5
// and 6 as 4 (FP64) or 5 and 4 (FP32), and 7 as 1 (FP64) or 6 (split).
constexpr int kNProj = 9;
constexpr int kProjDirect = 8; // its launch key
const GemmVariant kCorrF32[] = {{64, 256}, {64, 128}, {64, 64}, {128, 256}};
// split-precision kernels (variant 2 of each stages twice as much per LDS pass)
const GemmVariant kProjSplit[] = {{128, 128}, {64, 64}, {128, 128}, {128, 256}, {128, 128}, {128, 256}, {64, 64}};
const GemmVariant kCorrSplit[] = {{64, 256}, {64, 128}, {64, 256}, {128, 256}, {64, 256}, {128, 256}};
const GemmVariant kCorrF64[] = {{64, 64}, {32, 64}, {64, 32}, {32, 32}};
// FP32 variants 4 and 5: the three-product kernel with the Q tile loaded into
// LDS directly, on 128 and 64 complex columns; variant 6: as 5 with the output
// tile requested before the reduction; variant 7: every orbital of a domain
// (up to 96) in one block of 64 grid rows.  Split variants 4 and 5: both tiles
// loaded into LDS directly, on four waves with two stages and on eight waves
// with three (split runs variant 6 as 5, FP64 runs 5 and 6 as 4).
constexpr int kNCorr = 8;
constexpr int kProjKG = 16;

std::atomic<int> g_tune[5] = {{-1}, {-1}, {-1}, {-1}, {-1}};

// Per-shape tile choices (dcmesh_set_tuning_shape): (kernel, precision, nx, ny,
// nz, fd_order, n_orb, n_proj) -> variant.  A global choice (g_tune) takes
// precedence; shapes without an entry use the built-in rules.
using ShapeKey = std::array<int, 8>;
std::mutex g_shape_mu;
std::map<ShapeKey, int> g_shape_tune;
std::atomic<int> g_shape_count{0};

ShapeKey shape_key(int kernel, int prec, const dcmesh_domain& d) {
  return {kernel, prec, d.nx, d.ny, d.nz, d.fd_order, d.n_orb, d.n_proj};
}
// The tuned variant of this family for this domain: the global choice, else
// the per-shape entry, else -1.
int tuned(int kernel, int prec, const dcmesh_domain& d) {
  const int t = g_tune[kernel].load();
  if (t >= 0 || g_shape_count.load() == 0) return t;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  auto it = g_shape_tune.find(shape_key(kernel, prec, d));
  return it == g_shape_tune.end() ? -1 : it->second;
}

// The sweep3 variants address a plane of u with 32-bit byte offsets; a domain
// whose plane spans 2^32 bytes or more uses the default sweep instead.
// FP32 default: the 8 x 8 sweep on 16 waves, one column per thread
// (variant 12), for domains of x and y edges up to 40, and for larger ones
// where the 16 x 8 tile pads the x edge enough to outweigh the narrower
// tile's larger halo share (1.15x per useful point); else the 16 x 8 tile on
// 8 waves.  On the batch of 512 domains with edges 20-40 the 16-wave sweep is
// 3.4% faster than the 8-wave 8 x 8 and 16 x 8 sweeps it replaced; on the
// 64^3 domain it takes two rounds of blocks (one 16-wave block per CU) and is
// 3% slower than the 16 x 8 tile.
int stencil_default_f32(const dcmesh_domain& d) {
  auto waste = [&](int tx, int ty) {
    return (double)(cdiv(d.nx, tx) * tx) * (double)(cdiv(d.ny, ty) * ty) / ((double)d.nx * d.ny);
  };
  if (d.nx <= 40 && d.ny <= 40) return 12;
  return 1.15 * waste(8, 8) < waste(16, 8) ? 12 : kStencilDefaultF32;
}
int stencil_variant(const dcmesh_domain& d, int prec) {
  const int t = tuned(DCMESH_KERNEL_STENCIL, prec, d);
  const int v = t >= 0 ? t : (is_fp64(prec) ? kStencilDefaultF64 : stencil_default_f32(d));
  const long long plane_bytes = (long long)d.nx * d.ny * d.n_orb * (is_fp64(prec) ? 16 : 8);
  return (v >= kFirstSweep3 && plane_bytes >= (1LL << 32)) ? kStencilFallback : v;
}
// FP32 projector products load rows with 16-byte vectors when every row
// length is a multiple of 4 floats, else with 8-byte (one complex) vectors;
// the launch key carries that choice as variant + 4.
int wide_proj(const dcmesh_domain& d, int prec) {
  return (!is_fp64(prec) && !is_split(prec) && d.n_proj % 2 == 0 && d.n_orb % 2 == 0) ? 4 : 0;
}
int wide_corr(const dcmesh_domain& d, int prec) {
  return (!is_fp64(prec) && !is_split(prec) && d.n_proj % 2 == 0) ? 4 : 0;
}
int proj_variant_base(const dcmesh_domain& d, int prec);
int corr_variant_base(const dcmesh_domain& d, int prec);
// The direct-LDS projection moves 16-byte chunks of whole rows (even n_proj
// and n_orb) and addresses a split's rows with 32-bit byte offsets.
bool direct_proj_ok(const dcmesh_domain& d, int prec) {
  const long long rows = 2048;   // the longest split
  return prec == DCMESH_FP32 && wide_proj(d, prec) && rows * 8 * d.n_proj < (1LL << 31) &&
         rows * 8 * d.n_orb < (1LL << 31);
}
// The direct-LDS split projection addresses 128 rows of the transposed
// projector planes (2 ldbt bytes each) with 32-bit offsets.
bool direct_split_proj_ok(const dcmesh_domain& d) {
  const long long ldbt = (2LL * d.nx * d.ny * d.nz + 7) / 8 * 8;
  return 128 * 2 * ldbt + 4 * ldbt < (1LL << 31);
}
// The narrow FP32 products cover all orbitals of a domain in one block of
// 16 NB orbitals, NB <= kNarrowMax.
constexpr int kNarrowMax = 6;
bool narrow_ok(const dcmesh_domain& d, int prec) { return prec == DCMESH_FP32 && d.n_orb <= 16 * kNarrowMax; }
int narrow_nb(const dcmesh_domain& d) { return (d.n_orb + 15) / 16; }
constexpr int kProjNarrow = 12, kCorrNarrow = 16;   // first launch keys (+ 2 (NB - 1) + wide)
constexpr int kSplitNarrow = 8;                     // split modes: first launch key (+ NB - 1)
bool narrow_split_ok(const dcmesh_domain& d, int prec) { return is_split(prec) && d.n_orb <= 16 * kNarrowMax; }
// The narrow kernels are the default where they pad the orbitals less than a
// 64-orbital tile does (n_orb mod 64 in 1..48): where both pad to the same
// width the 64-orbital direct-LDS kernels are faster (measured per
// orbital-count class on the batch, and on 64 orbitals of the 48^3 domain).
// In split modes only the correction takes them: the split projection's own
// kernels were as fast or faster in every class.
bool narrow_pays(const dcmesh_domain& d, int prec) {
  return (narrow_ok(d, prec) || narrow_split_ok(d, prec)) && d.n_orb % 64 != 0 && d.n_orb % 64 <= 48;
}

int proj_variant(const dcmesh_domain& d, int prec) {
  int base = proj_variant_base(d, prec);
  if (base == 8) {
    // every orbital in one block, 64 projectors per block: FP32 launch keys
    // 12 + 2 (NB - 1) + wide, split 8 + NB - 1; larger orbital counts and FP64
    // run 4
    if (narrow_ok(d, prec)) return kProjNarrow + 2 * (narrow_nb(d) - 1) + (wide_proj(d, prec) ? 1 : 0);
    if (narrow_split_ok(d, prec)) return kSplitNarrow + narrow_nb(d) - 1;
    base = 4;
  }
  if (base == 7) {
    // FP32: the three-product kernel on 64 projectors x 32 complex orbitals
    // (launch keys 10 and 11: 8-byte and 16-byte loads), for any row length;
    // other modes run it as 6 (split) or 1 (FP64)
    if (prec == DCMESH_FP32) return 10 + (wide_proj(d, prec) ? 1 : 0);
    base = is_split(prec) ? 6 : 1;
  }
  if (base == 6) {
    if (is_split(prec)) return direct_split_proj_ok(d) ? 6 : 1;
    base = 4;
  }
  if (base == 5) {
    if (is_split(prec)) return direct_split_proj_ok(d) ? 5 : 0;
    // FP32: the three-product kernel with direct LDS loads on 64 projectors
    // (launch key kProjDirect + 1); FP64 runs it as variant 4
    if (prec == DCMESH_FP32) return direct_proj_ok(d, prec) ? kProjDirect + 1 : 1 + wide_proj(d, prec);
    base = 4;
  }
  if (base == 4) {
    if (is_split(prec)) return direct_split_proj_ok(d) ? 4 : 0;
    return direct_proj_ok(d, prec) ? kProjDirect : wide_proj(d, prec);
  }
  return base + wide_proj(d, prec);
}
// The direct-LDS correction (launch keys 8 and 12: 8-byte and 16-byte
// loads of the projector rows) addresses each Q plane with 32-bit offsets.
bool direct_corr_ok(const dcmesh_domain& d, int prec) {
  const long long ldq3 = (d.n_orb + 3) / 4 * 4;
  return prec == DCMESH_FP32 && (long long)d.n_proj * ldq3 * 4 < (1LL << 31);
}
int corr_variant(const dcmesh_domain& d, int prec) {
  int base = corr_variant_base(d, prec);
  if (base == 7) {
    // every orbital in one block, 64 grid rows per block: FP32 launch keys
    // 16 + 2 (NB - 1) + wide, split 8 + NB - 1; larger orbital counts and FP64
    // run 5
    if (narrow_ok(d, prec)) return kCorrNarrow + 2 * (narrow_nb(d) - 1) + (wide_corr(d, prec) ? 1 : 0);
    if (narrow_split_ok(d, prec)) return kSplitNarrow + narrow_nb(d) - 1;
    base = 5;
  }
  if (base == 6) {
    if (is_split(prec)) return 5;
    // FP32: the 64-complex-column direct-LDS kernel with the output tile
    // requested before the reduction (launch keys 11 and 15)
    if (prec == DCMESH_FP32) return direct_corr_ok(d, prec) ? (wide_corr(d, prec) ? 15 : 11) : 1 + wide_corr(d, prec);
    base = 4;
  }
  if (base == 5) {
    if (is_split(prec)) return 5;
    // FP32: the direct-LDS three-product kernel on 64 complex columns
    // (launch keys 10 and 14); FP64 runs it as variant 4
    if (prec == DCMESH_FP32) return direct_corr_ok(d, prec) ? (wide_corr(d, prec) ? 14 : 10) : 1 + wide_corr(d, prec);
    base = 4;
  }
  if (base == 4) {
    if (is_split(prec)) return 4;   // the split kernel with both tiles loaded into LDS directly
    return direct_corr_ok(d, prec) ? (wide_corr(d, prec) ? 12 : 8) : wide_corr(d, prec);
  }
  return base + wide_corr(d, prec);
}
// Padded output area of a tile grid over the n_proj x 2 n_orb projection,
// relative to the useful area.
double proj_waste(const dcmesh_domain& d, int bm, int bn) {
  const double m = d.n_proj, n = 2.0 * d.n_orb;
  return (double)(cdiv(d.n_proj, bm) * bm) * (double)(cdiv(2 * d.n_orb, bn) * bn) / (m * n);
}
int proj_variant_base(const dcmesh_domain& d, int prec) {
  const int t = tuned(DCMESH_KERNEL_PROJECT, prec, d);
  if (t >= 0) return t;
  if (is_fp64(prec)) return (d.n_proj >= 48 || 2 * d.n_orb >= 48) ? 0 : 1;
  // The cheapest of a few candidates by padded area times the kernel's time
  // per useful flop without padding (relative; measured on the 64^3 domain and
  // on batches of equal small domains).  FP32: 4 and 5 = the three-product
  // kernel with direct LDS loads, 128 x 128 and 64 x 128 (proj_variant falls
  // back where it cannot run), 1 = 64 x 64, 2 = 64 x 128.  Split: 5 = three stages
  // on eight waves, 128 x 256; 4 and 6 = two stages, 128 x 128 and 64 x 64.
  struct Cand { int v, bm, bn; double cost; };
  // FP32 domains whose orbitals a 64-orbital tile would pad: every orbital in one block
  if (prec == DCMESH_FP32 && narrow_pays(d, prec)) return 8;
  static const Cand kF32[] = {{4, 128, 128, 1.0}, {5, 64, 128, 1.01}, {1, 64, 64, 1.43}, {2, 64, 128, 1.36}};
  static const Cand kSplit[] = {{5, 128, 256, 1.0}, {4, 128, 128, 1.15}, {6, 64, 64, 1.59}};
  const Cand* c = is_split(prec) ? kSplit : kF32;
  const int nc = is_split(prec) ? 3 : 4;
  int best = c[0].v;
  double best_cost = 1e300;
  for (int k = 0; k < nc; ++k) {
    const double cost = c[k].cost * proj_waste(d, c[k].bm, c[k].bn);
    if (cost < best_cost) { best_cost = cost; best = c[k].v; }
  }
  return best;
}
int corr_variant_base(const dcmesh_domain& d, int prec) {
  const int t = tuned(DCMESH_KERNEL_CORRECT, prec, d);
  if (t >= 0) return t;
  if (is_fp64(prec)) return 2 * d.n_orb > 32 ? 0 : 2;
  // domains whose orbitals a 64-orbital tile would pad: every orbital in one block
  if (narrow_pays(d, prec)) return 7;
  // large tiles: both tiles loaded into LDS directly, three stages on eight waves
  if (is_split(prec)) return 2 * d.n_orb > 128 ? 5 : 1;
  const int n2 = 2 * d.n_orb;
  // the three-product kernel with the Q tile loaded into LDS directly on 64
  // complex columns: never more padding than the 128-column tile, and three
  // waves per SIMD instead of two (corr_variant falls back where it cannot run)
  return n2 > 64 ? 5 : 2;
}

// ---------------------------------------------------------------------------
// Validation (host only, before any HIP call)
// ---------------------------------------------------------------------------
int validate_domains(const dcmesh_domain* doms, int32_t n_dom, int32_t prec) {
  if (!doms) return fail(DCMESH_ERR_INVALID_ARGUMENT, "doms is NULL");
  if (n_dom < 1) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_dom must be >= 1");
  if (prec < DCMESH_FP64 || prec > DCMESH_SPLIT_FP16)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "unknown precision " + std::to_string(prec));
  for (int i = 0; i < n_dom; ++i) {
    const dcmesh_domain& d = doms[i];
    const std::string at = " (domain " + std::to_string(i) + ")";
    if (d.fd_order != 2 && d.fd_order != 4 && d.fd_order != 6)
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "fd_order must be 2, 4 or 6" + at);
    const int need = d.fd_order + 1;
    if (d.nx < need || d.ny < need || d.nz < need)
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "grid edges must be >= fd_order + 1" + at);
    if ((long long)d.nx * d.ny * d.nz > (1LL << 31))
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "grid too large (more than 2^31 points)" + at);
    if (d.n_orb < 1 || d.n_orb > (1 << 16)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_orb must be in [1, 65536]" + at);
    if (d.n_proj < 0 || d.n_proj > (1 << 20)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_proj must be in [0, 2^20]" + at);
    if (!(d.h > 0.0) || !std::isfinite(d.h)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "h must be finite and > 0" + at);
    if (!d.psi || !d.v_loc || !d.occ) return fail(DCMESH_ERR_INVALID_ARGUMENT, "psi, v_loc and occ are required" + at);
    if (d.n_proj > 0 && (!d.proj || !d.d)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "proj and d are required when n_proj > 0" + at);
  }
  return DCMESH_OK;
}

int validate_work(void* work, size_t work_bytes, size_t need) {
  if (!work) return fail(DCMESH_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(work) % kAlign) return fail(DCMESH_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (work_bytes < need)
    return fail(DCMESH_ERR_WORKSPACE, "workspace too small: " + std::to_string(work_bytes) + " < " + std::to_string(need));
  return DCMESH_OK;
}

// ---------------------------------------------------------------------------
// Plans: descriptors, work lists and workspace layout
// ---------------------------------------------------------------------------
struct Launch {
  int variant;       // tile variant of the family
  size_t first;      // offset (in items) of this launch's list
  int count;
};

struct Plan {
  int prec = 0, n_dom = 0;
  std::vector<DomDesc> desc;
  std::vector<Item> items;
  std::vector<Launch> stencil, proj, reduce, corr, dens, elem, energy, ovl_proj, ovl_reduce;
  std::vector<Launch> presplit, absmax_b, absmax_u, splitq;   // split-precision modes
  std::vector<Launch> dfinish;                                 // density partials -> rho, j
  std::vector<Launch> rows;                                    // 256-point row blocks (column norms)
  std::vector<Launch> occ_rows;                                // 4 reference orbitals per block
  size_t bytes_tables = 0, bytes_total = 0;
  size_t off_items = 0, off_flag = 0;
  bool any_proj = false;
  // the adjoint's gradient partials come from its stencil sweeps (every
  // domain on a ring-sweep variant, FP32 or split); else from k_grad_partial
  bool grad_fused = false;
};

// Elements per thread of the elementwise kernels.
constexpr int kEPT = 4;

void group_launch(std::vector<Launch>& out, std::vector<Item>& items, int n_dom,
                  const std::function<int(int)>& variant_of,
                  const std::function<void(int, std::vector<Item>&)>& emit,
                  const std::function<void(int, int)>& on_first = nullptr) {
  std::map<int, std::vector<int>> groups;
  for (int i = 0; i < n_dom; ++i) {
    const int v = variant_of(i);
    if (v >= 0) groups[v].push_back(i);
  }
  for (auto& kv : groups) {
    Launch L{kv.first, items.size(), 0};
    for (int i : kv.second) {
      if (on_first) on_first(i, (int)(items.size() - L.first));
      emit(i, items);
    }
    L.count = (int)(items.size() - L.first);
    if (L.count > 0) out.push_back(L);
  }
}

// Reorders items [begin, end), made of consecutive clusters of cs items, so
// that each cluster lands on one XCD: work-groups are dealt to the 8 XCDs
// round-robin by index, so position t*8 + c of every run of 8 clusters goes to
// XCD c.  Items of one cluster share operand rows (a split-K slice, or the
// halo planes of one z segment), which then meet in that XCD's L2.
void xcd_interleave(std::vector<Item>& items, size_t begin, size_t end, size_t cs) {
  const size_t n = end - begin;
  if (cs == 0 || n % cs) return;
  const size_t nclus = n / cs;
  std::vector<Item> out;
  out.reserve(n);
  for (size_t c0 = 0; c0 < nclus; c0 += 8) {
    const size_t cn = std::min<size_t>(8, nclus - c0);
    for (size_t t = 0; t < cs; ++t)
      for (size_t c = 0; c < cn; ++c) out.push_back(items[begin + (c0 + c) * cs + t]);
  }
  std::copy(out.begin(), out.end(), items.begin() + begin);
}

// Stencil work orders (DCMESH_KERNEL_SORDER): 0 keeps each domain's items as
// emitted, its orbital chunks dealt over the XCDs by xcd_interleave; 1 and 2
// make every (domain, z segment) a cluster that runs on one XCD, with its items
// in (y tile, x tile, chunk) order (1: the blocks resident together on an XCD
// hold every chunk of a few tiles) or (chunk, y tile, x tile) order (2: whole
// chunks).  A cluster then holds both the halo planes its tiles share and the
// cache lines that two chunks of a grid point share when a point's orbitals do
// not fill whole lines.  Clusters go to the least loaded of the 8 XCD queues in
// launch order, and the queues are dealt round-robin, so position 8 t + x of
// the launch runs on XCD x until the shortest queue runs out.
constexpr int kNSorder = 3;
void stencil_deal(std::vector<Item>& items, size_t first, size_t count, int mode) {
  if (mode == 0 || count == 0) return;
  std::vector<Item> v(items.begin() + first, items.begin() + first + count);
  auto key = [&](const Item& a) {
    const int zs = a.c >> 16, ch = a.c & 0xffff;
    return mode == 1 ? std::array<int, 5>{a.dom, zs, a.b, a.a, ch} : std::array<int, 5>{a.dom, zs, ch, a.b, a.a};
  };
  std::stable_sort(v.begin(), v.end(), [&](const Item& x, const Item& y) { return key(x) < key(y); });
  std::vector<std::vector<Item>> q(8);
  std::array<size_t, 8> load{};
  for (size_t i = 0; i < v.size();) {
    size_t j = i;
    while (j < v.size() && v[j].dom == v[i].dom && (v[j].c >> 16) == (v[i].c >> 16)) ++j;
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    q[x].insert(q[x].end(), v.begin() + i, v.begin() + j);
    load[x] += j - i;
    i = j;
  }
  size_t pos = first;
  for (size_t t = 0; pos < first + count; ++t)
    for (int x = 0; x < 8; ++x)
      if (t < q[x].size()) items[pos++] = q[x][t];
}

// Builds the plan for these domains.  Pointers into the workspace are set when
// work != nullptr; otherwise only sizes are computed.
void build_plan(Plan& P, const dcmesh_domain* doms, int n_dom, int prec, char* work) {
  P = Plan();
  P.prec = prec;
  P.n_dom = n_dom;
  P.desc.resize(n_dom);
  const size_t rs = real_size(prec), cs = 2 * rs;
  const size_t acc = rs;  // accumulation type of the projector products

  // work lists
  // stencil launches are keyed by (radius, tile variant): variant + 4 r
  auto sv = [&](int i) { return stencil_variant(doms[i], prec) + 16 * (doms[i].fd_order / 2); };
  auto stile = [&](int v) { return is_fp64(prec) ? kStencilF64[v % 16] : kStencilF32[v % 16]; };
  long long stencil_blocks_xy = 0;
  for (int i = 0; i < n_dom; ++i) {
    const StencilVariant t = stile(sv(i));
    stencil_blocks_xy += cdiv(doms[i].nx, t.tx) * cdiv(doms[i].ny, t.ty) * cdiv(doms[i].n_orb, t.oc);
  }
  for (int i = 0; i < n_dom; ++i) {
    DomDesc& D = P.desc[i];
    const dcmesh_domain& d = doms[i];
    std::memset(&D, 0, sizeof(D));
    D.nx = d.nx; D.ny = d.ny; D.nz = d.nz; D.r = d.fd_order / 2;
    D.n_orb = d.n_orb; D.n_proj = d.n_proj;
    D.n_grid = (long long)d.nx * d.ny * d.nz;
    D.h = d.h;
    // z segments: aim at >= 1024 stencil blocks in total, segments of >= 16
    // planes (or the tuned fixed length)
    const int zt = g_tune[DCMESH_KERNEL_ZSEG].load();
    if (zt > 0) {
      D.zseg = std::min(d.nz, kZsegOpt[zt]);
    } else {
      // whole z columns (no re-read of the 2r boundary planes) once the
      // column tiles give every CU a block; shorter segments only to fill it
      const long long want = std::max<long long>(1, cdiv(256, std::max<long long>(1, stencil_blocks_xy)));
      D.zseg = (int)std::min<long long>(d.nz, std::max<long long>(16, cdiv(d.nz, want)));
    }
    // split-K length depends on the domain alone (its sizes, not the tile
    // variant), so a domain gives the same bits whether it runs alone or inside
    // a batch: enough splits that the projection has about 512 blocks over
    // nominal 128 x 128 tiles (and at least 32 splits), 512 to 2048 points each
    const long long tiles = cdiv(D.n_proj, 128) * cdiv(2LL * D.n_orb, 128);
    const long long want_splits = std::max<long long>(32, cdiv(512, std::max<long long>(1, tiles)));
    D.split_len = (int)std::min<long long>(
        2048, std::max<long long>(512, cdiv(cdiv(D.n_grid, want_splits), kProjKG) * kProjKG));
    D.n_split = (int)cdiv(D.n_grid, D.split_len);
    D.a_stride = 3;
    D.ldq = (2 * D.n_orb + 3) / 4 * 4;
    D.ldq3 = (D.n_orb + 3) / 4 * 4;
    // whole 32-half stages of the split correction (zero padded)
    D.ldbs = D.ldqt = (2 * (long long)D.n_proj + 31) / 32 * 32;
    D.ldbt = (2 * D.n_grid + 7) / 8 * 8;
  }
  P.any_proj = false;
  for (int i = 0; i < n_dom; ++i) P.any_proj |= doms[i].n_proj > 0;

  group_launch(P.stencil, P.items, n_dom, sv,
               [&](int i, std::vector<Item>& it) {
                 const StencilVariant t = stile(sv(i));
                 DomDesc& D = P.desc[i];
                 const int nzs = (int)cdiv(D.nz, D.zseg), nch = (int)cdiv(D.n_orb, t.oc);
                 D.n_chunks = nch;
                 const size_t b0 = it.size();
                 const int nyt = (int)cdiv(D.ny, t.ty), nxt = (int)cdiv(D.nx, t.tx);
                 for (int zs = 0; zs < nzs; ++zs)
                   for (int ch = 0; ch < nch; ++ch)
                     for (int yt = 0; yt < nyt; ++yt)
                       for (int xt = 0; xt < nxt; ++xt) it.push_back({i, xt, yt, (zs << 16) | ch});
                 xcd_interleave(it, b0, it.size(), (size_t)nyt * nxt);
               },
               nullptr);
  {
    // built-in order: one XCD per (domain, z segment) once a launch has a
    // cluster for every XCD (the batch of small domains: 9% less stencil time,
    // half the HBM reads); a launch of fewer clusters keeps the chunk deal,
    // which spreads a single large domain over all eight
    const int so = g_tune[DCMESH_KERNEL_SORDER].load();
    for (const Launch& L : P.stencil) {
      long long clusters = 0;
      for (int k = 0; k < L.count; ++k) {
        const Item& a = P.items[L.first + k];
        clusters += (a.a == 0 && a.b == 0 && (a.c & 0xffff) == 0);   // one first tile per (domain, segment)
      }
      stencil_deal(P.items, L.first, L.count, so >= 0 ? so : (clusters >= 8 ? 1 : 0));
    }
  }
  for (const Launch& L : P.stencil)
    for (int k = 0; k < L.count; ++k) P.desc[P.items[L.first + k].dom].n_e_loc++;

  auto pv = [&](int i) { return doms[i].n_proj > 0 ? proj_variant(doms[i], prec) : -1; };
  group_launch(P.proj, P.items, n_dom, pv, [&](int i, std::vector<Item>& it) {
    // FP32 launch key kProjDirect + 1: the direct-LDS kernel on 64 projectors x 64 complex orbitals
    const int v = pv(i);
    const GemmVariant t = is_fp64(prec)  ? kProjF64[v % 4]
                          : is_split(prec) ? (v >= kSplitNarrow ? GemmVariant{64, 32 * (v - kSplitNarrow + 1)}
                                                                : kProjSplit[v])
                          : v == kProjDirect + 1 ? GemmVariant{64, 128}
                          : (v == 10 || v == 11) ? GemmVariant{64, 64}
                          : v >= kProjNarrow ? GemmVariant{64, 32 * ((v - kProjNarrow) / 2 + 1)}
                                                 : kProjF32[v % 4];
    const DomDesc& D = P.desc[i];
    const size_t b0 = it.size();
    const int nmt = (int)cdiv(D.n_proj, t.bm), nnt = (int)cdiv(2 * D.n_orb, t.bn);
    for (int s = 0; s < D.n_split; ++s)
      for (int mt = 0; mt < nmt; ++mt)
        for (int nt = 0; nt < nnt; ++nt) it.push_back({i, mt, nt, s});
    xcd_interleave(it, b0, it.size(), (size_t)nmt * nnt);
  });
  group_launch(P.reduce, P.items, n_dom, [&](int i) { return doms[i].n_proj > 0 ? 0 : -1; },
               [&](int i, std::vector<Item>& it) {
                 const DomDesc& D = P.desc[i];
                 for (long long b = 0; b < cdiv((long long)D.n_proj * D.n_orb, kBlock); ++b) it.push_back({i, (int)b, 0, 0});
               },
               [&](int i, int first) { P.desc[i].item0_reduce = first; });
  for (const Launch& L : P.reduce)
    for (int k = 0; k < L.count; ++k) P.desc[P.items[L.first + k].dom].n_e_nl++;
  auto cv = [&](int i) { return doms[i].n_proj > 0 ? corr_variant(doms[i], prec) : -1; };
  group_launch(P.corr, P.items, n_dom, cv, [&](int i, std::vector<Item>& it) {
    // FP32 launch keys 8 and 12: the direct-LDS kernel on the tile of variant
    // 0; keys 10 and 14: on 64 complex columns
    const int v = cv(i);
    const GemmVariant t = is_fp64(prec)  ? kCorrF64[v % 4]
                          : is_split(prec) ? (v >= kSplitNarrow ? GemmVariant{64, 32 * (v - kSplitNarrow + 1)}
                                                                : kCorrSplit[v])
                          : v >= kCorrNarrow ? GemmVariant{64, 32 * ((v - kCorrNarrow) / 2 + 1)}
                          : (v == 10 || v == 11 || v == 14 || v == 15) ? GemmVariant{64, 128}
                                                 : kCorrF32[v % 4];
    const DomDesc& D = P.desc[i];
    const size_t b0 = it.size();
    const int nnt = (int)cdiv(2 * D.n_orb, t.bn);
    for (long long gt = 0; gt < cdiv(D.n_grid, t.bm); ++gt)
      for (int nt = 0; nt < nnt; ++nt) it.push_back({i, (int)gt, nt, 0});
    // the column tiles of a row block share its B rows: one XCD, one L2
    if (nnt > 1) xcd_interleave(it, b0, it.size(), (size_t)nnt);
  });
  group_launch(P.dens, P.items, n_dom, [](int) { return 0; },
               [&](int i, std::vector<Item>& it) {
                 DomDesc& D = P.desc[i];
                 D.n_dens = (int)cdiv(D.n_grid, 4);
                 for (long long b = 0; b < D.n_dens; ++b) it.push_back({i, (int)b, 0, 0});
               },
               [&](int i, int first) { P.desc[i].item0_dens = first; });
  group_launch(P.elem, P.items, n_dom, [](int) { return 0; },
               [&](int i, std::vector<Item>& it) {
                 const DomDesc& D = P.desc[i];
                 for (long long b = 0; b < cdiv(D.n_grid * D.n_orb, (long long)kBlock * kEPT); ++b) it.push_back({i, (int)b, 0, 0});
               },
               [&](int i, int first) { P.desc[i].item0_elem = first; });
  for (const Launch& L : P.elem)
    for (int k = 0; k < L.count; ++k) P.desc[P.items[L.first + k].dom].n_g_part++;
  P.grad_fused = !is_fp64(prec);
  for (int i = 0; i < n_dom; ++i) P.grad_fused &= (sv(i) % 16) >= kFirstSweep4;
  if (P.grad_fused)
    for (int i = 0; i < n_dom; ++i) P.desc[i].n_g_part = P.desc[i].n_e_loc;
  group_launch(P.dfinish, P.items, n_dom, [](int) { return 0; }, [&](int i, std::vector<Item>& it) {
    for (long long b = 0; b < cdiv(P.desc[i].n_grid, kBlock); ++b) it.push_back({i, (int)b, 0, 0});
  });
  group_launch(P.rows, P.items, n_dom, [](int) { return 0; },
               [&](int i, std::vector<Item>& it) {
                 DomDesc& D = P.desc[i];
                 D.n_rows_blocks = (int)cdiv(D.n_grid, kBlock);
                 for (int b = 0; b < D.n_rows_blocks; ++b) it.push_back({i, b, 0, 0});
               },
               [&](int i, int first) { P.desc[i].item0_rows = first; });
  group_launch(P.energy, P.items, n_dom, [](int) { return 0; },
               [&](int i, std::vector<Item>& it) { it.push_back({i, 0, 0, 0}); });
  // overlap S = h^3 Psi^H Psi (always FP64 arithmetic)
  group_launch(P.ovl_proj, P.items, n_dom, [](int) { return 0; }, [&](int i, std::vector<Item>& it) {
    const DomDesc& D = P.desc[i];
    for (int s = 0; s < D.n_split; ++s)
      for (int mt = 0; mt < cdiv(D.n_orb, 64); ++mt)
        for (int nt = 0; nt < cdiv(2 * D.n_orb, 64); ++nt) it.push_back({i, mt, nt, s});
  });
  group_launch(P.ovl_reduce, P.items, n_dom, [](int) { return 0; }, [&](int i, std::vector<Item>& it) {
    const DomDesc& D = P.desc[i];
    for (long long b = 0; b < cdiv((long long)D.n_orb * D.n_orb, kBlock); ++b) it.push_back({i, (int)b, 0, 0});
  });
  group_launch(P.occ_rows, P.items, n_dom, [](int) { return 0; },
               [&](int i, std::vector<Item>& it) {
                 for (int b = 0; b < cdiv(P.desc[i].n_orb, kBlock / kWave); ++b) it.push_back({i, b, 0, 0});
               },
               [&](int i, int first) { P.desc[i].item0_occ = first; });

  if (is_split(prec)) {
    auto has_p = [&](int i) { return doms[i].n_proj > 0 ? 0 : -1; };
    group_launch(P.presplit, P.items, n_dom, has_p, [&](int i, std::vector<Item>& it) {
      const DomDesc& D = P.desc[i];
      const long long ngt = std::max(cdiv(D.n_grid, 32), cdiv(D.ldbt, 64));
      const long long npt = std::max(cdiv(D.n_proj, 32), cdiv(D.ldbs, 64));
      for (long long gt = 0; gt < ngt; ++gt)
        for (int pt = 0; pt < npt; ++pt) it.push_back({i, (int)gt, pt, 0});
    });
    group_launch(P.absmax_b, P.items, n_dom, has_p, [&](int i, std::vector<Item>& it) {
      const DomDesc& D = P.desc[i];
      for (long long b = 0; b < cdiv(D.n_grid * 2 * D.n_proj, (long long)kBlock * kAbsPer); ++b) it.push_back({i, (int)b, 0, 0});
    });
    group_launch(P.absmax_u, P.items, n_dom, has_p, [&](int i, std::vector<Item>& it) {
      const DomDesc& D = P.desc[i];
      for (long long b = 0; b < cdiv(D.n_grid * 2 * D.n_orb, (long long)kBlock * kAbsPer); ++b) it.push_back({i, (int)b, 0, 0});
    });
    group_launch(P.splitq, P.items, n_dom, has_p, [&](int i, std::vector<Item>& it) {
      const DomDesc& D = P.desc[i];
      for (long long b = 0; b < cdiv(2LL * D.n_orb * D.ldqt, kBlock); ++b) it.push_back({i, (int)b, 0, 0});
    });
  }

  // Workspace layout.  The item tables and the stencil's energy partials get
  // room for the largest count any tile variant could produce (smallest
  // tiles: stencil 8 x 4 columns x 4 orbitals over segments of >= min(nz, 8)
  // planes; projector products in 32 x 32 tiles), so the workspace size does
  // not depend on the tuning.
  auto stencil_bound = [](const DomDesc& D) {
    return cdiv(D.nx, 8) * cdiv(D.ny, 4) * cdiv(D.n_orb, 4) * cdiv(D.nz, std::min(D.nz, 8));
  };
  size_t variable = 0, bound = 0;
  for (const auto* fam : {&P.stencil, &P.proj, &P.corr})
    for (const Launch& L : *fam) variable += L.count;
  for (int i = 0; i < n_dom; ++i) {
    const DomDesc& D = P.desc[i];
    bound += (size_t)stencil_bound(D);
    if (D.n_proj > 0) {
      bound += (size_t)(D.n_split * cdiv(D.n_proj, 32) * cdiv(2 * D.n_orb, 32));
      bound += (size_t)(cdiv(D.n_grid, 32) * cdiv(2 * D.n_orb, 32));
    }
  }
  const size_t item_room = P.items.size() - variable + std::max(bound, variable);
  size_t off = 0;
  off += align_up(sizeof(DomDesc) * n_dom);
  P.off_items = off;
  off += align_up(sizeof(Item) * item_room);
  P.off_flag = off;
  off += kAlign;
  P.bytes_tables = off;
  auto take = [&](size_t bytes) -> char* {
    char* p = work ? work + off : nullptr;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  };
  for (int i = 0; i < n_dom; ++i) {
    DomDesc& D = P.desc[i];
    const size_t psi_bytes = (size_t)D.n_grid * D.n_orb * cs;
    for (int s = SLOT_B0; s <= SLOT_B4; ++s) D.slot[s] = as_global(take(psi_bytes));
    const size_t no2 = 2 * (size_t)D.n_orb;
    const size_t part = std::max((size_t)D.n_split * D.n_proj * no2 * acc, (size_t)D.n_split * D.n_orb * no2 * 8);
    D.ppart = as_global(take(part));
    D.pmat = as_global(take((size_t)D.n_proj * no2 * acc));
    D.qmat = as_global(take(2 * (size_t)D.n_proj * D.ldq * acc));
    // three-product (Gauss) planes of coef D P for the FP32 correction
    D.qmat3 = as_global(prec == DCMESH_FP32 ? take(3 * (size_t)D.n_proj * D.ldq3 * sizeof(float)) : (char*)nullptr);
    D.e_loc = as_global((double*)take(sizeof(double) * (size_t)std::max<long long>(D.n_e_loc, stencil_bound(D))));
    D.e_nl = as_global((double*)take(sizeof(double) * std::max(1, D.n_e_nl)));
    // gradient partials: one per elementwise item, or one per stencil item when
    // the sweeps form them; room for either, whatever the tile variant
    const long long g_room = std::max<long long>(cdiv(D.n_grid * D.n_orb, (long long)kBlock * kEPT), stencil_bound(D));
    D.g_part = as_global((double*)take(3 * sizeof(double) * (size_t)std::max<long long>(1, g_room)));
    // sized for the smallest orbital chunk of any stencil variant, so the
    // workspace does not depend on the tile choice
    D.dpart = as_global(take((size_t)cdiv(D.n_orb, 4) * D.n_grid * 4 * rs));
    D.cn_part = as_global((double*)take(sizeof(double) * (size_t)D.n_rows_blocks * D.n_orb));
    D.cn_inv = as_global((double*)take(sizeof(double) * D.n_orb));
    D.smat = as_global((double*)take(16 * (size_t)D.n_orb * D.n_orb));
    D.jpart = as_global((double*)take(4 * sizeof(double) * (size_t)std::max(1, D.n_dens)));
    D.jnl_part = as_global((double*)take(3 * sizeof(double) * (size_t)std::max(1, D.n_e_nl)));
    D.cur = as_global((double*)take(3 * sizeof(double)));
    if (is_split(prec) && D.n_proj > 0) {
      const size_t nbs = (size_t)D.n_grid * D.ldbs * 2, nbt = (size_t)D.n_proj * D.ldbt * 2;   // 16-bit values
      D.bs_hi = as_global(take(nbs)); D.bs_lo = as_global(take(nbs));
      D.bt_hi = as_global(take(nbt)); D.bt_lo = as_global(take(nbt));
      const size_t nq = (size_t)2 * D.n_orb * D.ldqt * 2;
      D.qt_hi = as_global(take(nq)); D.qt_lo = as_global(take(nq));
      D.maxbits = as_global((unsigned*)take(4 * sizeof(unsigned)));
    }
  }
  P.bytes_total = off;
}

// Pinned staging copies of the tables, cached by content so that identical
// tables never overwrite a buffer that a queued copy may still read.
struct Staging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  int graph_refs = 0;            // captured graphs that read this buffer
  ~Staging() {
    if (done) (void)hipEventDestroy(done);
    if (host) (void)hipHostFree(host);
  }
};

std::mutex g_stage_mu;
std::map<std::pair<size_t, size_t>, std::shared_ptr<Staging>> g_stage;   // (hash, bytes) -> buffer

// Finds or creates the pinned copy of the tables.  A buffer whose last copy
// has completed and that no graph references is rewritten for new contents, so
// repeated calls with changing pointers (chunked runs, the adjoint sweep) reuse
// a handful of allocations.  Allocation is not allowed under stream capture,
// so graph creation stages its tables before capturing.
// The head of the workspace as the kernels read it: domain descriptors, then
// the work lists.
std::vector<char> table_image(const Plan& P) {
  std::vector<char> img(P.bytes_tables, 0);
  std::memcpy(img.data(), P.desc.data(), sizeof(DomDesc) * P.n_dom);
  std::memcpy(img.data() + P.off_items, P.items.data(), sizeof(Item) * P.items.size());
  return img;
}

int get_staging(const Plan& P, bool capturing, std::shared_ptr<Staging>* out) {
  const size_t bytes = P.bytes_tables;
  const std::vector<char> img = table_image(P);
  const size_t hsh = std::hash<std::string>()(std::string(img.data(), img.size()));
  std::shared_ptr<Staging> st;
  std::lock_guard<std::mutex> lk(g_stage_mu);
  auto itr = g_stage.find({hsh, bytes});
  if (itr != g_stage.end() && std::memcmp(itr->second->host, img.data(), bytes) == 0) st = itr->second;
  if (!st) {
    if (capturing)
      return fail(DCMESH_ERR_UNSUPPORTED,
                  "these tables were not staged before capture: use dcmesh_graph_create to record steps");
    // reuse an idle buffer of sufficient size
    for (auto e = g_stage.begin(); e != g_stage.end(); ++e) {
      Staging& c = *e->second;
      if (c.graph_refs == 0 && e->second.use_count() == 1 && c.bytes >= bytes &&
          (!c.done || hipEventQuery(c.done) == hipSuccess)) {
        st = e->second;
        g_stage.erase(e);
        break;
      }
    }
    if (!st) {
      st = std::make_shared<Staging>();
      HIPCHK(hipHostMalloc(&st->host, bytes, hipHostMallocDefault));
      st->bytes = bytes;
      HIPCHK(hipEventCreateWithFlags(&st->done, hipEventDisableTiming));
    }
    std::memcpy(st->host, img.data(), bytes);
    g_stage[{hsh, bytes}] = st;
    // bound the number of idle buffers kept
    if (g_stage.size() > 64) {
      for (auto e = g_stage.begin(); e != g_stage.end() && g_stage.size() > 64;) {
        if (e->second != st && e->second->graph_refs == 0 && e->second.use_count() == 1 &&
            (!e->second->done || hipEventQuery(e->second->done) == hipSuccess))
          e = g_stage.erase(e);
        else
          ++e;
      }
    }
  }
  *out = st;
  return DCMESH_OK;
}

int stage_tables(const Plan& P, char* work, hipStream_t s, bool capturing, std::shared_ptr<Staging>* keep) {
  std::shared_ptr<Staging> st;
  int rc = get_staging(P, capturing, &st);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(work, st->host, P.bytes_tables, hipMemcpyHostToDevice, s));
  if (!capturing && st->done) HIPCHK(hipEventRecord(st->done, s));
  if (keep) *keep = st;
  return DCMESH_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of dcmesh_step_noalloc
// ---------------------------------------------------------------------------
// Callers that cannot allocate device memory (work under graph capture, tight
// serving loops) get the workspace from this array instead; each GPU the
// library runs on holds its own copy until the process ends.  Its device
// address comes from hipGetSymbolAddress, once per device: in host code the
// array's name is not a device address.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Tables reach the scratch through kernel arguments (no pinned staging buffer
// is allocated): one launch per chunk, in stream order before the work.
constexpr int kUploadChunk = 1024;
struct UploadChunk { unsigned char b[kUploadChunk]; };
__global__ void k_upload(unsigned char* dst, UploadChunk c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.b[i];
}

// Device address of this device's copy of the scratch array.  Looked up
// once per device with that device current (the caller's current device).
int scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DCMESH_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DCMESH_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DCMESH_OK;
}

int upload_tables(const Plan& P, char* dst, hipStream_t s) {
  const std::vector<char> img = table_image(P);
  UploadChunk c;
  for (size_t off = 0; off < img.size(); off += kUploadChunk) {
    const int n = (int)std::min<size_t>(kUploadChunk, img.size() - off);
    std::memcpy(c.b, img.data() + off, n);
    k_upload<<<1, kBlock, 0, s>>>((unsigned char*)dst + off, c, n);
  }
  HIPCHK(hipGetLastError());
  return DCMESH_OK;
}

int check_device() {
  static std::once_flag once;
  static int status = DCMESH_OK;
  static std::string msg;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      status = DCMESH_ERR_HIP;
      msg = "no HIP device";
      return;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
      status = DCMESH_ERR_UNSUPPORTED;
      msg = std::string("this library is built for gfx950, found ") + prop.gcnArchName;
    }
  });
  return status == DCMESH_OK ? DCMESH_OK : fail(status, msg);
}

// ---------------------------------------------------------------------------
// Kernel profiling: HIP events around each launch family (DCMESH_FLAG_PROFILE)
// ---------------------------------------------------------------------------
struct ProfRec { int fam; hipEvent_t a, b; };
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;
thread_local bool t_prof_on = false;

hipEvent_t prof_event() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct ProfScope {
  int fam;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(int f, hipStream_t st) : fam(f), s(st) {
    if (t_prof_on) {
      a = prof_event();
      (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({fam, a, b});
  }
};

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
struct Ctx {
  const Plan* P;
  const DomDesc* d_desc;
  const Item* d_items;
  hipStream_t s;
};

template <typename T, int R>
void launch_stencil_r(const Ctx& c, const Launch& L, const StencilArgs& a) {
  const Item* it = c.d_items + L.first;
  const dim3 g(L.count);
  if constexpr (sizeof(T) == 4) {
    if (a.grad_slot < SLOT_NONE) {
      // the adjoint's ring sweeps with the gradient partials (the plan asks
      // for them only when every stencil launch is a ring sweep)
      switch (L.variant) {
        case 9: k_stencil_sweep4<T, R, 16, 8, 8, 512, true><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
        case 10: k_stencil_sweep4<T, R, 16, 8, 8, 256, true><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
        case 12: k_stencil_sweep4<T, R, 16, 8, 8, 1024, true><<<g, 1024, 0, c.s>>>(c.d_desc, it, a); break;
        default: k_stencil_sweep4<T, R, 16, 16, 8, 512, true><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      }
      return;
    }
    switch (L.variant) {
      case 0: k_stencil_sweep<T, R, 16, 16, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 1: k_stencil_sweep<T, R, 8, 16, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 2: k_stencil_sweep<T, R, 16, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 3: k_stencil_sweep<T, R, 4, 16, 16, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 4: k_stencil_sweep<T, R, 16, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 5: k_stencil_sweep<T, R, 16, 16, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 6: k_stencil_sweep2<T, R, 16, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 7: k_stencil_sweep2<T, R, 16, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 8: k_stencil_sweep3<T, R, 16, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 9: k_stencil_sweep4<T, R, 16, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 10: k_stencil_sweep4<T, R, 16, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 12: k_stencil_sweep4<T, R, 16, 8, 8, 1024><<<g, 1024, 0, c.s>>>(c.d_desc, it, a); break;
      default: k_stencil_sweep4<T, R, 16, 16, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
    }
  } else {
    switch (L.variant) {
      case 0: k_stencil_sweep<T, R, 8, 16, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 1: k_stencil_sweep<T, R, 8, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 2: k_stencil_sweep<T, R, 4, 16, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 3: k_stencil_sweep<T, R, 16, 8, 4, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 4: k_stencil_sweep<T, R, 8, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 5: k_stencil_sweep<T, R, 8, 16, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 6: k_stencil_sweep2<T, R, 8, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 7: k_stencil_sweep2<T, R, 8, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      case 8: k_stencil_sweep3<T, R, 8, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 9: k_stencil_sweep4<T, R, 8, 8, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
      case 10: k_stencil_sweep4<T, R, 8, 8, 8, 256><<<g, 256, 0, c.s>>>(c.d_desc, it, a); break;
      default: k_stencil_sweep4<T, R, 8, 16, 8, 512><<<g, 512, 0, c.s>>>(c.d_desc, it, a); break;
    }
  }
}

// Stencil launches are keyed by variant + 16 r, so every domain of a launch
// shares the stencil radius.
template <typename T>
void launch_stencil(const Ctx& c, const StencilArgs& a) {
  ProfScope prof_(DCMESH_FAM_STENCIL, c.s);
  for (const Launch& L : c.P->stencil) {
    Launch l2 = L;
    l2.variant = L.variant % 16;
    switch (L.variant / 16) {
      case 1: launch_stencil_r<T, 1>(c, l2, a); break;
      case 2: launch_stencil_r<T, 2>(c, l2, a); break;
      default: launch_stencil_r<T, 3>(c, l2, a); break;
    }
  }
}

template <typename T>
void launch_project(const Ctx& c, int u_slot, int a_slot = -1) {
  ProfScope prof_(DCMESH_FAM_PROJECT, c.s);
  ProjArgs a{a_slot, u_slot, 0};
  for (const Launch& L : c.P->proj) {
    const Item* it = c.d_items + L.first;
    const dim3 g(L.count), b(kBlock);
    if constexpr (sizeof(T) == 4) {
      switch (L.variant) {
        case 0: k_project3m<128, 64, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 1: k_project<T, T, 64, 64, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 2: k_project<T, T, 64, 128, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 3: k_project<T, T, 128, 256, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 4: k_project3m<128, 64, kProjKG, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 5: k_project<T, T, 64, 64, kProjKG, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 6: k_project<T, T, 64, 128, kProjKG, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 7: k_project<T, T, 128, 256, kProjKG, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 9: k_project3m_dl<64, 64, kProjKG><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 10: k_project3m<64, 32, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 11: k_project3m<64, 32, kProjKG, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
#define DCM_PN(NB)                                                                                  \
  case kProjNarrow + 2 * (NB - 1): k_project3m_n<NB, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break; \
  case kProjNarrow + 2 * (NB - 1) + 1: k_project3m_n<NB, 4><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        DCM_PN(1) DCM_PN(2) DCM_PN(3) DCM_PN(4) DCM_PN(5) DCM_PN(6)
#undef DCM_PN
        default: k_project3m_dl<128, 64, kProjKG><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
      }
    } else {
      switch (L.variant) {
        case 0: k_project<T, T, 64, 64, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 1: k_project<T, T, 32, 32, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        case 2: k_project<T, T, 64, 32, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
        default: k_project<T, T, 32, 64, kProjKG, 2><<<g, b, 0, c.s>>>(c.d_desc, it, a); break;
      }
    }
  }
}

template <typename T>
void launch_reduce(const Ctx& c, double cre, double cim, int occ_scale, int want_energy, int unit_d = 0) {
  ProfScope prof_(DCMESH_FAM_REDUCE, c.s);
  ReduceArgs a{cre, cim, occ_scale, want_energy, 0, c.P->prec == DCMESH_SPLIT_FP16 ? 1 : 0, unit_d};
  for (const Launch& L : c.P->reduce)
    k_reduce<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, a);
}

template <typename T>
void launch_correct(const Ctx& c, int out_slot) {
  ProfScope prof_(DCMESH_FAM_CORRECT, c.s);
  for (const Launch& L : c.P->corr) {
    const Item* it = c.d_items + L.first;
    const dim3 g(L.count), b(kBlock);
    if constexpr (sizeof(T) == 4) {
      switch (L.variant) {
        case 0: k_correct3m<64, 128, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 1: k_correct<T, T, 64, 128, 32, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 2: k_correct<T, T, 64, 64, 32, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 3: k_correct<T, T, 128, 256, 32, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 4: k_correct3m<64, 128, 16, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 5: k_correct<T, T, 64, 128, 32, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 6: k_correct<T, T, 64, 64, 32, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 7: k_correct<T, T, 128, 256, 32, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 8: k_correct3m_dl<64, 128, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 10: k_correct3m_dl<64, 64, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 11: k_correct3m_dl<64, 64, 16, 2, true><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 14: k_correct3m_dl<64, 64, 16, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 15: k_correct3m_dl<64, 64, 16, 4, true><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
#define DCM_CN(NB)                                                                                         \
  case kCorrNarrow + 2 * (NB - 1): k_correct3m_n<NB, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break; \
  case kCorrNarrow + 2 * (NB - 1) + 1: k_correct3m_n<NB, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        DCM_CN(1) DCM_CN(2) DCM_CN(3) DCM_CN(4) DCM_CN(5) DCM_CN(6)
#undef DCM_CN
        default: k_correct3m_dl<64, 128, 16, 4><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
      }
    } else {
      switch (L.variant) {
        case 0: k_correct<T, T, 64, 64, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 1: k_correct<T, T, 32, 64, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        case 2: k_correct<T, T, 64, 32, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
        default: k_correct<T, T, 32, 32, 16, 2><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot); break;
      }
    }
  }
}

// ---- split-precision launches ----
void launch_zero_maxbits(const Ctx& c, int which) {
  for (const Launch& L : c.P->energy)
    k_zero_maxbits<<<cdiv(L.count, kBlock), kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, L.count, which);
}

// Once per call: the 16-bit hi/lo planes of the projectors (and, for FP16,
// the max |B| that fixes their scale).
void launch_presplit(const Ctx& c) {
  ProfScope prof_(DCMESH_FAM_SPLIT, c.s);
  const bool f16 = c.P->prec == DCMESH_SPLIT_FP16;
  if (f16) {
    launch_zero_maxbits(c, 0);
    for (const Launch& L : c.P->absmax_b) k_absmax<<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, 0, 0);
  }
  for (const Launch& L : c.P->presplit) {
    if (f16)
      k_presplit<1><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
    else
      k_presplit<0><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  }
}

// umax_known (FP16): maxbits[1] already holds max |u| of every domain,
// gathered by the correction that wrote u
template <int MODE>
void launch_project_split(const Ctx& c, int u_slot, bool umax_known = false) {
  if (MODE == 1 && !umax_known) {
    ProfScope prof_(DCMESH_FAM_SPLIT, c.s);
    launch_zero_maxbits(c, 1);
    for (const Launch& L : c.P->absmax_u)
      k_absmax<<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, 1, u_slot);
  }
  ProfScope prof_(DCMESH_FAM_PROJECT, c.s);
  for (const Launch& L : c.P->proj) {
    const Item* it = c.d_items + L.first;
    const dim3 g(L.count), b(kBlock);
    switch (L.variant) {
      case 0: k_project_split<MODE, 128, 128, 16><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      case 1: k_project_split<MODE, 64, 64, 16><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      case 2: k_project_split<MODE, 128, 128, 32><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      case 3: k_project_split<MODE, 128, 256, 16><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      case 4: k_project_split_dl<MODE, 128, 128><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      case 6: k_project_split_dl<MODE, 64, 64><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
#define DCM_SPN(NB) \
  case kSplitNarrow + NB - 1: k_project_split_n<MODE, NB><<<g, b, 0, c.s>>>(c.d_desc, it, u_slot); break;
      DCM_SPN(1) DCM_SPN(2) DCM_SPN(3) DCM_SPN(4) DCM_SPN(5) DCM_SPN(6)
#undef DCM_SPN
      default: k_project_split_dl3<MODE><<<g, dim3(kBlockProj3), 0, c.s>>>(c.d_desc, it, u_slot); break;
    }
  }
}

// umax (FP16): the correction kernels also gather max |out| into maxbits[1]
// (cleared here; the projection that read it was launched before), the scale
// source of the next projection when out is its input
template <int MODE>
void launch_correct_split(const Ctx& c, int out_slot, bool umax = false) {
  const int um = (MODE == 1 && umax) ? 1 : 0;
  if (um) launch_zero_maxbits(c, 1);
  {
    ProfScope prof_(DCMESH_FAM_SPLIT, c.s);
    for (const Launch& L : c.P->splitq) k_split_q<MODE><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  }
  ProfScope prof_(DCMESH_FAM_CORRECT, c.s);
  for (const Launch& L : c.P->corr) {
    const Item* it = c.d_items + L.first;
    const dim3 g(L.count), b(kBlock);
    switch (L.variant) {
      case 0: k_correct_split<MODE, 64, 256, 32><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
      case 1: k_correct_split<MODE, 64, 128, 32><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
      case 2: k_correct_split<MODE, 64, 256, 64><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
      case 3: k_correct_split<MODE, 128, 256, 32><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
      case 4: k_correct_split_dl<MODE, 64, 256><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
#define DCM_SCN(NB) \
  case kSplitNarrow + NB - 1: k_correct_split_n<MODE, NB><<<g, b, 0, c.s>>>(c.d_desc, it, out_slot, um); break;
      DCM_SCN(1) DCM_SCN(2) DCM_SCN(3) DCM_SCN(4) DCM_SCN(5) DCM_SCN(6)
#undef DCM_SCN
      default: k_correct_split_dl3<MODE><<<g, dim3(kBlockCorr3), 0, c.s>>>(c.d_desc, it, out_slot, um); break;
    }
  }
}

// out = base + coef * f^occ * H(A_step) u   (full H: local sweep, then the
// projector correction added in place).
// fp16_scale (FP16 mode): bit 0 = maxbits[1] already holds max |u| (the
// correction that wrote u gathered it), bit 1 = gather max |out| for the next
// stage
constexpr int kScaleKnown = 1, kScaleGather = 2;
template <typename T>
void apply_stage(const Ctx& c, int u_slot, int base_slot, int out_slot, double cre, double cim,
                 int occ_scale, int step, int want_energy, int want_density = 0, bool nonlocal = true,
                 int fp16_scale = 0, int grad_slot = SLOT_NONE, double gre = 0.0, double gim = 0.0) {
  const int prec = c.P->prec;
  const bool nl = nonlocal && c.P->any_proj;
  if (nl) {
    if (prec == DCMESH_SPLIT_BF16) {
      launch_project_split<0>(c, u_slot);
    } else if (prec == DCMESH_SPLIT_FP16) {
      launch_project_split<1>(c, u_slot, (fp16_scale & kScaleKnown) != 0);
      launch_zero_maxbits(c, 2);
    } else {
      launch_project<T>(c, u_slot);
    }
    launch_reduce<T>(c, cre, cim, occ_scale, want_energy);
  }
  // grad_slot: only the adjoint's FP32 / split sweeps of mu ask for gradient
  // partials, with no base term, energy or density (the gradient sweep kernel
  // has none of them)
  StencilArgs sa{u_slot, base_slot, out_slot, cre, cim, occ_scale, step, want_energy, want_density,
                 grad_slot, gre, gim};
  launch_stencil<T>(c, sa);
  if (nl) {
    if (prec == DCMESH_SPLIT_BF16)
      launch_correct_split<0>(c, out_slot);
    else if (prec == DCMESH_SPLIT_FP16)
      launch_correct_split<1>(c, out_slot, (fp16_scale & kScaleGather) != 0);
    else
      launch_correct<T>(c, out_slot);
  }
}

template <typename T>
void launch_energy(const Ctx& c, int obs) {
  ProfScope prof_(DCMESH_FAM_ENERGY, c.s);
  for (const Launch& L : c.P->energy) k_energy_final<<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, obs);
}

template <typename T>
void launch_density(const Ctx& c, int step, int obs) {
  ProfScope prof_(DCMESH_FAM_DENSITY, c.s);
  for (const Launch& L : c.P->dens) k_density<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, step, obs);
}

template <typename T>
void launch_density_finish(const Ctx& c, int step, int obs) {
  ProfScope prof_(DCMESH_FAM_DENSITY, c.s);
  for (const Launch& L : c.P->dfinish)
    k_density_finish<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, step, obs);
}

template <typename T>
void launch_axpy(const Ctx& c, int x_slot, int out_slot) {
  ProfScope prof_(DCMESH_FAM_ADJOINT, c.s);
  for (const Launch& L : c.P->elem) k_axpy<T, kEPT><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, x_slot, out_slot);
}

template <typename T>
void launch_grad(const Ctx& c, int mu_slot, int u_slot, double cre, double cim) {
  ProfScope prof_(DCMESH_FAM_ADJOINT, c.s);
  for (const Launch& L : c.P->elem)
    k_grad_partial<T, kEPT><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, mu_slot, u_slot, cre, cim);
}

// S = h^3 A^H Psi into D.overlap, FP64 accumulation, for A the psi-sized
// buffer in a_slot (Psi itself for the orbital overlap).
template <typename T>
void launch_overlap(const Ctx& c, int a_slot = SLOT_PSI) {
  ProfScope prof_(DCMESH_FAM_OVERLAP, c.s);
  ProjArgs a{a_slot, SLOT_PSI, 1};
  for (const Launch& L : c.P->ovl_proj)
    k_project<T, double, 64, 64, kProjKG, 2><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, a);
  ReduceArgs r{1.0, 0.0, 0, 0, 1, 0, 0};
  for (const Launch& L : c.P->ovl_reduce) k_reduce<double><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, r);
}

// Macroscopic current of psi into D.cur: block sums of rho and the
// paramagnetic current; with the position-weighted projectors, P = h^3 B^H psi
// (left in D.pmat by the reduce) and the three products h^3 B_d^H psi reduced
// against it; then the final sum.  step >= 0: the field is the Maxwell state's.
template <typename T>
void launch_current(const Ctx& c, int step, bool nonlocal) {
  launch_density<T>(c, 0, 0);
  if (nonlocal) {
    launch_project<T>(c, SLOT_PSI);
    launch_reduce<T>(c, 1.0, 0.0, 0, 0);
    for (int d = 0; d < 3; ++d) {
      launch_project<T>(c, SLOT_PSI, -2 - d);
      ProfScope prof_(DCMESH_FAM_REDUCE, c.s);
      for (const Launch& L : c.P->reduce) k_jnl_partial<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, d);
    }
  }
  ProfScope prof_(DCMESH_FAM_DENSITY, c.s);
  for (const Launch& L : c.P->energy)
    k_current_final<<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, step, nonlocal ? 1 : 0);
}

// f_s and n_exc from the cross overlap with the reference orbitals in
// SLOT_LAMBDA.
template <typename T>
void launch_occupations(const Ctx& c) {
  launch_overlap<T>(c, SLOT_LAMBDA);
  ProfScope prof_(DCMESH_FAM_OVERLAP, c.s);
  for (const Launch& L : c.P->rows) k_colnorm_partial<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  for (const Launch& L : c.P->occ_rows) k_occ_rows<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  for (const Launch& L : c.P->energy) k_occ_final<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
}

// ---------------------------------------------------------------------------
// Entry-point bodies
// ---------------------------------------------------------------------------
struct CallSetup {
  Plan P;
  Ctx c;
  std::shared_ptr<Staging> keep;
};

// use_static: the workspace is the static scratch (dcmesh_step_noalloc; work
// and work_bytes are ignored), with the tables uploaded through kernel
// arguments instead of a pinned staging copy.
int prepare(CallSetup& cs, const dcmesh_domain* doms, int32_t n_dom, int32_t prec, void* work,
            size_t work_bytes, hipStream_t s, uint32_t flags, const std::function<void(Plan&)>& fill,
            bool use_static = false) {
  Plan& P = cs.P;
  int rc;
  if (use_static) {
    if (flags & DCMESH_FLAG_PROFILE)
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "PROFILE creates events: not available without allocation");
    build_plan(P, doms, n_dom, prec, nullptr);
    if (P.bytes_total > kScratchBytes)
      return fail(DCMESH_ERR_WORKSPACE, "these domains need " + std::to_string(P.bytes_total) +
                                            " bytes of workspace; the static scratch holds " +
                                            std::to_string(kScratchBytes));
    rc = check_device();
    if (rc) return rc;
    rc = scratch_address(&work);
    if (rc) return rc;
    work_bytes = kScratchBytes;
  }
  build_plan(P, doms, n_dom, prec, (char*)work);
  rc = validate_work(work, work_bytes, P.bytes_total);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  fill(P);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(s, &cap));
  if ((flags & DCMESH_FLAG_PROFILE) && cap != hipStreamCaptureStatusNone)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "PROFILE cannot be used under stream capture");
  t_prof_on = (flags & DCMESH_FLAG_PROFILE) != 0;
  rc = use_static ? upload_tables(P, (char*)work, s)
                  : stage_tables(P, (char*)work, s, cap != hipStreamCaptureStatusNone, &cs.keep);
  if (rc) return rc;
  cs.c = Ctx{&P, (const DomDesc*)work, (const Item*)((char*)work + P.off_items), s};
  return DCMESH_OK;
}

// psi <- psi / |psi_n| column by column (fixed-order FP64 norms).
template <typename T>
void launch_normalise(const Ctx& c) {
  ProfScope prof_(DCMESH_FAM_REDUCE, c.s);
  for (const Launch& L : c.P->rows) k_colnorm_partial<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  for (const Launch& L : c.P->energy) k_colnorm_final<<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
  for (const Launch& L : c.P->rows) k_colnorm_scale<T><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first);
}

// Eq. 2 with the nonlocal operator of Eq. 5: per step N T4(-i dt h_loc(A_k)) N,
// N psi = normalise(psi - delta Psi0 h^3 Psi0^H psi), delta = i dt v_nl / 2.
// The domain descriptors carry Psi0 as their projector array (n_proj = n_orb).
template <typename T>
int run_step_eq2(CallSetup& cs, int32_t n_steps, double dt, double v_nl) {
  const Ctx& c = cs.c;
  auto half = [&]() {
    launch_project<T>(c, SLOT_PSI);
    launch_reduce<T>(c, 0.0, -0.5 * dt * v_nl, 0, 0, 1);     // coef = -delta, D = 1
    launch_correct<T>(c, SLOT_PSI);
    launch_normalise<T>(c);
  };
  for (int k = 0; k < n_steps; ++k) {
    half();
    apply_stage<T>(c, SLOT_PSI, SLOT_PSI, SLOT_B0, 0.0, -dt / 4, 0, k, 0, 0, false);
    apply_stage<T>(c, SLOT_B0, SLOT_PSI, SLOT_B1, 0.0, -dt / 3, 0, k, 0, 0, false);
    apply_stage<T>(c, SLOT_B1, SLOT_PSI, SLOT_B0, 0.0, -dt / 2, 0, k, 0, 0, false);
    apply_stage<T>(c, SLOT_B0, SLOT_PSI, SLOT_PSI, 0.0, -dt, 0, k, 0, 0, false);
    half();
  }
  return DCMESH_OK;
}

// One Taylor-4 step with the field sample k.
template <typename T>
void one_step(const Ctx& c, int k, double dt, bool want_rho_j, bool want_e) {
  // stage 4 applies H to psi_k: it also yields E_k and the rho/j partials of psi_k
  // FP16 scales: every correction gathers max |out|, the input of the next
  // stage (of the next step, for the last); from the second step of a call on,
  // psi's max is the one the previous step's last correction gathered
  const int first = (k > 0 ? kScaleKnown : 0) | kScaleGather, next = kScaleKnown | kScaleGather;
  apply_stage<T>(c, SLOT_PSI, SLOT_PSI, SLOT_B0, 0.0, -dt / 4, 0, k, want_e ? 1 : 0, want_rho_j ? 1 : 0, true,
                 first);
  if (want_rho_j) launch_density_finish<T>(c, k, k);
  apply_stage<T>(c, SLOT_B0, SLOT_PSI, SLOT_B1, 0.0, -dt / 3, 0, k, 0, 0, true, next);
  apply_stage<T>(c, SLOT_B1, SLOT_PSI, SLOT_B0, 0.0, -dt / 2, 0, k, 0, 0, true, next);
  apply_stage<T>(c, SLOT_B0, SLOT_PSI, SLOT_PSI, 0.0, -dt, 0, k, 0, 0, true, next);
  if (want_e) launch_energy<T>(c, k);
}

template <typename T>
int run_step(CallSetup& cs, int32_t n_steps, double dt, bool want_rho_j, bool want_e) {
  const Ctx& c = cs.c;
  if (is_split(c.P->prec) && c.P->any_proj && n_steps > 0) launch_presplit(c);
  for (int k = 0; k < n_steps; ++k) one_step<T>(c, k, dt, want_rho_j, want_e);
  return DCMESH_OK;
}

// n steps coupled to the Maxwell update: per step the current of psi_k in the
// field A_ext(t_k) + A_ind, the leapfrog update (which writes the step field
// into D.amid = D.a), then the Taylor step.
template <typename T>
int run_step_maxwell(CallSetup& cs, int32_t n_steps, double dt, bool nonlocal) {
  const Ctx& c = cs.c;
  for (int k = 0; k < n_steps; ++k) {
    launch_current<T>(c, k, nonlocal);
    for (const Launch& L : c.P->energy) k_field_update<<<L.count, 1, 0, c.s>>>(c.d_desc, c.d_items + L.first, k, dt);
    one_step<T>(c, k, dt, false, false);
  }
  return DCMESH_OK;
}

int finish(CallSetup& cs, uint32_t flags) {
  t_prof_on = false;
  HIPCHK(hipGetLastError());
  if (flags & DCMESH_FLAG_CHECK_FINITE) {
    const Ctx& c = cs.c;
    int* flag = (int*)((char*)c.d_desc + cs.P.off_flag);
    k_fill_int<<<1, 1, 0, c.s>>>(flag, 0);
    for (const Launch& L : cs.P.elem) {
      if (is_fp64(cs.P.prec))
        k_nonfinite<double, kEPT><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, flag);
      else
        k_nonfinite<float, kEPT><<<L.count, kBlock, 0, c.s>>>(c.d_desc, c.d_items + L.first, flag);
    }
    int host = 0;
    HIPCHK(hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, c.s));
    HIPCHK(hipStreamSynchronize(c.s));
    if (host) return fail(DCMESH_ERR_NONFINITE, "psi holds a NaN or Inf after the call");
  }
  return DCMESH_OK;
}

int step_impl(const dcmesh_domain* doms, int32_t n_dom, int32_t prec, const double* a_dev,
              int32_t a_per_domain, int64_t a_stride, double dt, int32_t n_steps, const dcmesh_obs* obs,
              void* work, size_t work_bytes, uint32_t flags, hipStream_t s, CallSetup& cs,
              bool use_static = false) {
  int rc = validate_domains(doms, n_dom, prec);
  if (rc) return rc;
  if (n_steps < 0) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_steps must be >= 0");
  if (n_steps > 0 && !a_dev) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_dev is NULL");
  if (a_stride < n_steps) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_stride must be >= n_steps");
  if (!std::isfinite(dt)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "dt must be finite");
  bool want_rho_j = false, want_e = false;
  if (obs)
    for (int i = 0; i < n_dom; ++i) {
      want_rho_j |= obs[i].rho != nullptr || obs[i].j != nullptr;
      want_e |= obs[i].energy != nullptr;
    }
  rc = prepare(cs, doms, n_dom, prec, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.v = as_global(doms[i].v_loc);
      D.proj = as_global(doms[i].proj);
      D.d = as_global(doms[i].d);
      D.occ = as_global(doms[i].occ);
      D.a = as_global(a_dev + (a_per_domain ? (long long)i * a_stride * 3 : 0));
      if (obs) {
        D.rho = as_global(obs[i].rho);
        D.jcur = as_global(obs[i].j);
        D.energy = as_global(obs[i].energy);
      }
    }
  }, use_static);
  if (rc) return rc;
  if (is_fp64(prec))
    rc = run_step<double>(cs, n_steps, dt, want_rho_j, want_e);
  else
    rc = run_step<float>(cs, n_steps, dt, want_rho_j, want_e);
  if (rc) return rc;
  return finish(cs, flags);
}

struct GraphHandle {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::shared_ptr<Staging> keep;
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* dcmesh_last_error(void) { return g_err.c_str(); }

int dcmesh_workspace_bytes(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, uint32_t flags,
                           size_t* bytes) {
  if (!bytes) return fail(DCMESH_ERR_INVALID_ARGUMENT, "bytes is NULL");
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  std::vector<dcmesh_domain> eq2;
  if (flags & DCMESH_FLAG_EQ2) {     // the reference orbitals take the place of the projectors
    eq2.assign(doms, doms + n_dom);
    for (auto& d : eq2) {
      d.n_proj = d.n_orb;
      d.proj = d.psi;
      d.d = d.occ;
    }
    doms = eq2.data();
  }
  Plan P;
  build_plan(P, doms, n_dom, precision, nullptr);
  *bytes = P.bytes_total;
  return DCMESH_OK;
}

int dcmesh_step(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const double* a_dev,
                int32_t a_per_domain, int64_t a_stride, double dt, int32_t n_steps, const dcmesh_obs* obs,
                void* work, size_t work_bytes, uint32_t flags, void* stream) {
  CallSetup cs;
  return step_impl(doms, n_dom, precision, a_dev, a_per_domain, a_stride, dt, n_steps, obs, work, work_bytes,
                   flags, (hipStream_t)stream, cs);
}

int dcmesh_step_noalloc(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const double* a_dev,
                        int32_t a_per_domain, int64_t a_stride, double dt, int32_t n_steps,
                        const dcmesh_obs* obs, uint32_t flags, void* stream) {
  CallSetup cs;
  return step_impl(doms, n_dom, precision, a_dev, a_per_domain, a_stride, dt, n_steps, obs, nullptr, 0, flags,
                   (hipStream_t)stream, cs, true);
}

int dcmesh_step_eq2(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const void* const* psi0,
                    double v_nl, const double* a_dev, int32_t a_per_domain, int64_t a_stride, double dt,
                    int32_t n_steps, void* work, size_t work_bytes, uint32_t flags, void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (precision != DCMESH_FP64 && precision != DCMESH_FP32)
    return fail(DCMESH_ERR_UNSUPPORTED, "dcmesh_step_eq2 runs in FP64 or FP32");
  if (!psi0) return fail(DCMESH_ERR_INVALID_ARGUMENT, "psi0 is NULL");
  for (int i = 0; i < n_dom; ++i)
    if (!psi0[i]) return fail(DCMESH_ERR_INVALID_ARGUMENT, "psi0[" + std::to_string(i) + "] is NULL");
  if (n_steps < 0) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_steps must be >= 0");
  if (n_steps > 0 && !a_dev) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_dev is NULL");
  if (a_stride < n_steps) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_stride must be >= n_steps");
  if (!std::isfinite(dt) || !std::isfinite(v_nl)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "dt and v_nl must be finite");
  std::vector<dcmesh_domain> eq2(doms, doms + n_dom);
  for (int i = 0; i < n_dom; ++i) {
    eq2[i].n_proj = eq2[i].n_orb;
    eq2[i].proj = psi0[i];
    eq2[i].d = eq2[i].occ;      // not read: the reduce runs with D = 1
  }
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, eq2.data(), n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(eq2[i].psi);
      D.v = as_global(eq2[i].v_loc);
      D.proj = as_global(eq2[i].proj);
      D.d = as_global(eq2[i].d);
      D.occ = as_global(eq2[i].occ);
      D.a = as_global(a_dev + (a_per_domain ? (long long)i * a_stride * 3 : 0));
    }
  });
  if (rc) return rc;
  if (precision == DCMESH_FP64)
    rc = run_step_eq2<double>(cs, n_steps, dt, v_nl);
  else
    rc = run_step_eq2<float>(cs, n_steps, dt, v_nl);
  if (rc) return rc;
  return finish(cs, flags);
}

int dcmesh_density(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const double* a_dev,
                   int32_t a_per_domain, const dcmesh_density_out* out, void* work, size_t work_bytes,
                   uint32_t flags, void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (!a_dev) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_dev is NULL");
  if (!out) return fail(DCMESH_ERR_INVALID_ARGUMENT, "out is NULL");
  bool rho_j = false, e = false, hpsi = false, ovl = false;
  for (int i = 0; i < n_dom; ++i) {
    rho_j |= out[i].rho || out[i].j;
    e |= out[i].energy != nullptr;
    hpsi |= out[i].hpsi_occ != nullptr;
    ovl |= out[i].overlap != nullptr;
  }
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, doms, n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.slot[SLOT_HPSI] = out[i].hpsi_occ ? as_global(out[i].hpsi_occ) : D.slot[SLOT_B0];
      D.v = as_global(doms[i].v_loc);
      D.proj = as_global(doms[i].proj);
      D.d = as_global(doms[i].d);
      D.occ = as_global(doms[i].occ);
      D.a = as_global(a_dev + (a_per_domain ? (long long)i * 3 : 0));
      D.rho = as_global(out[i].rho);
      D.jcur = as_global(out[i].j);
      D.energy = as_global(out[i].energy);
      D.overlap = as_global(out[i].overlap);
      D.jpart = nullptr;
    }
  });
  if (rc) return rc;
  const bool f64 = is_fp64(precision);
  if (is_split(precision) && cs.P.any_proj && (e || hpsi)) launch_presplit(cs.c);
  if (rho_j) f64 ? launch_density<double>(cs.c, 0, 0) : launch_density<float>(cs.c, 0, 0);
  if (e || hpsi) {
    if (f64) {
      apply_stage<double>(cs.c, SLOT_PSI, SLOT_NONE, SLOT_HPSI, 1.0, 0.0, 1, 0, e ? 1 : 0);
      if (e) launch_energy<double>(cs.c, 0);
    } else {
      apply_stage<float>(cs.c, SLOT_PSI, SLOT_NONE, SLOT_HPSI, 1.0, 0.0, 1, 0, e ? 1 : 0);
      if (e) launch_energy<float>(cs.c, 0);
    }
  }
  if (ovl) f64 ? launch_overlap<double>(cs.c) : launch_overlap<float>(cs.c);
  return finish(cs, flags);
}

int dcmesh_occupations(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const void* const* psi0,
                       double* const* overlap, double* const* f_out, double* n_exc, void* work,
                       size_t work_bytes, uint32_t flags, void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (!psi0 || !f_out || !n_exc) return fail(DCMESH_ERR_INVALID_ARGUMENT, "psi0, f_out and n_exc are required");
  for (int i = 0; i < n_dom; ++i)
    if (!psi0[i] || !f_out[i])
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "psi0[" + std::to_string(i) + "] or f_out[" + std::to_string(i) + "] is NULL");
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, doms, n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.slot[SLOT_LAMBDA] = as_global(const_cast<void*>(psi0[i]));
      D.occ = as_global(doms[i].occ);
      D.overlap = overlap && overlap[i] ? as_global(overlap[i]) : D.smat;
      D.f_occ = as_global(f_out[i]);
      D.n_exc = as_global(n_exc + i);
    }
  });
  if (rc) return rc;
  is_fp64(precision) ? launch_occupations<double>(cs.c) : launch_occupations<float>(cs.c);
  return finish(cs, flags);
}

namespace {
int check_proj_r(const dcmesh_domain* doms, int32_t n_dom, const void* const* proj_r) {
  if (!proj_r) return DCMESH_OK;
  for (int i = 0; i < n_dom; ++i)
    if (doms[i].n_proj > 0 && !proj_r[i])
      return fail(DCMESH_ERR_INVALID_ARGUMENT, "proj_r[" + std::to_string(i) + "] is NULL for a domain with projectors");
  return DCMESH_OK;
}
}  // namespace

int dcmesh_current(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const double* a_dev,
                   int32_t a_per_domain, const void* const* proj_r, double* current, void* work,
                   size_t work_bytes, uint32_t flags, void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (precision != DCMESH_FP64 && precision != DCMESH_FP32)
    return fail(DCMESH_ERR_UNSUPPORTED, "dcmesh_current runs in FP64 or FP32");
  if (!a_dev || !current) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_dev and current are required");
  rc = check_proj_r(doms, n_dom, proj_r);
  if (rc) return rc;
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, doms, n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.v = as_global(doms[i].v_loc);
      D.proj = as_global(doms[i].proj);
      D.proj_r = proj_r ? as_global(proj_r[i]) : nullptr;
      D.d = as_global(doms[i].d);
      D.occ = as_global(doms[i].occ);
      D.a = as_global(a_dev + (a_per_domain ? (long long)i * 3 : 0));
      D.cur = as_global(current + (long long)i * 3);
    }
  });
  if (rc) return rc;
  const bool nl = proj_r != nullptr && cs.P.any_proj;
  precision == DCMESH_FP64 ? launch_current<double>(cs.c, -1, nl) : launch_current<float>(cs.c, -1, nl);
  return finish(cs, flags);
}

int dcmesh_step_maxwell(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const void* const* proj_r,
                        const double* a_ext, int32_t a_per_domain, double dt, int32_t n_steps, double* field,
                        double* a_mid, double* current, void* work, size_t work_bytes, uint32_t flags,
                        void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (precision != DCMESH_FP64 && precision != DCMESH_FP32)
    return fail(DCMESH_ERR_UNSUPPORTED, "dcmesh_step_maxwell runs in FP64 or FP32");
  if (n_steps < 0) return fail(DCMESH_ERR_INVALID_ARGUMENT, "n_steps must be >= 0");
  if (!a_ext || !field || !a_mid) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_ext, field and a_mid are required");
  if (!std::isfinite(dt)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "dt must be finite");
  rc = check_proj_r(doms, n_dom, proj_r);
  if (rc) return rc;
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, doms, n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.v = as_global(doms[i].v_loc);
      D.proj = as_global(doms[i].proj);
      D.proj_r = proj_r ? as_global(proj_r[i]) : nullptr;
      D.d = as_global(doms[i].d);
      D.occ = as_global(doms[i].occ);
      D.a_ext = as_global(a_ext + (a_per_domain ? (long long)i * (n_steps + 1) * 3 : 0));
      D.amid = as_global(a_mid + (long long)i * n_steps * 3);
      D.a = D.amid;
      D.a_stride = 3;
      D.field = as_global(field + (long long)i * 6);
      D.cur_out = current ? as_global(current + (long long)i * n_steps * 3) : nullptr;
    }
  });
  if (rc) return rc;
  const bool nl = proj_r != nullptr && cs.P.any_proj;
  rc = precision == DCMESH_FP64 ? run_step_maxwell<double>(cs, n_steps, dt, nl)
                                : run_step_maxwell<float>(cs, n_steps, dt, nl);
  if (rc) return rc;
  return finish(cs, flags);
}

int dcmesh_adjoint_step(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, void* const* lambda,
                        const double* a_dev, int32_t a_per_domain, double dt, double* grad_dev, void* work,
                        size_t work_bytes, uint32_t flags, void* stream) {
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  if (!lambda) return fail(DCMESH_ERR_INVALID_ARGUMENT, "lambda is NULL");
  for (int i = 0; i < n_dom; ++i)
    if (!lambda[i]) return fail(DCMESH_ERR_INVALID_ARGUMENT, "lambda[" + std::to_string(i) + "] is NULL");
  if (!a_dev || !grad_dev) return fail(DCMESH_ERR_INVALID_ARGUMENT, "a_dev and grad_dev are required");
  if (!std::isfinite(dt)) return fail(DCMESH_ERR_INVALID_ARGUMENT, "dt must be finite");
  CallSetup cs;
  hipStream_t s = (hipStream_t)stream;
  rc = prepare(cs, doms, n_dom, precision, work, work_bytes, s, flags, [&](Plan& P) {
    for (int i = 0; i < n_dom; ++i) {
      DomDesc& D = P.desc[i];
      D.slot[SLOT_PSI] = as_global(doms[i].psi);
      D.slot[SLOT_LAMBDA] = as_global(lambda[i]);
      D.v = as_global(doms[i].v_loc);
      D.proj = as_global(doms[i].proj);
      D.d = as_global(doms[i].d);
      D.occ = as_global(doms[i].occ);
      D.a = as_global(a_dev + (a_per_domain ? (long long)i * 3 : 0));
      D.grad = as_global(grad_dev + (a_per_domain ? (long long)i * 3 : 0));
    }
  });
  if (rc) return rc;
  auto body = [&](auto tag) {
    using T = decltype(tag);
    const Ctx& c = cs.c;
    if (is_split(precision) && c.P->any_proj) launch_presplit(c);
    // forward Horner intermediates: u3 -> B0, u2 -> B1, u1 -> B2 (u4 = psi)
    apply_stage<T>(c, SLOT_PSI, SLOT_PSI, SLOT_B0, 0.0, -dt / 4, 0, 0, 0);
    apply_stage<T>(c, SLOT_B0, SLOT_PSI, SLOT_B1, 0.0, -dt / 3, 0, 0, 0);
    apply_stage<T>(c, SLOT_B1, SLOT_PSI, SLOT_B2, 0.0, -dt / 2, 0, 0, 0);
    // mu_0 = lambda; mu_j = conj(c_j) H mu_{j-1}, added into lambda as soon as
    // it exists (mu_{j-1} is not needed afterwards); before that,
    // grad += 2 Re <mu_{j-1}, c_j dH/dA u_j>, c_j = -i dt / j.
    const int u_of[5] = {-1, SLOT_B2, SLOT_B1, SLOT_B0, SLOT_PSI};
    const int bufs[2] = {SLOT_B3, SLOT_B4};
    int mu_prev = SLOT_LAMBDA;
    // With the ring sweep the partials come from the sweep that applies H to
    // mu_{j-1}, as Re(c_j sum conj((-i D1 + A) mu_{j-1}) u_j) (the operator is
    // Hermitian); otherwise a separate pass forms them before that sweep.
    for (int j = 1; j <= 4; ++j) {
      const int mu_new = bufs[(j - 1) % 2];
      if (c.P->grad_fused) {
        apply_stage<T>(c, mu_prev, SLOT_NONE, mu_new, 0.0, dt / j, 0, 0, 0, 0, true, 0, u_of[j], 0.0, -dt / j);
      } else {
        launch_grad<T>(c, mu_prev, u_of[j], 0.0, -dt / j);
      }
      {
        ProfScope prof_(DCMESH_FAM_ADJOINT, c.s);
        k_grad_final<<<a_per_domain ? n_dom : 1, kBlock, 0, c.s>>>(c.d_desc, n_dom, a_per_domain ? 0 : 1);
      }
      if (!c.P->grad_fused) apply_stage<T>(c, mu_prev, SLOT_NONE, mu_new, 0.0, dt / j, 0, 0, 0);
      launch_axpy<T>(c, mu_new, SLOT_LAMBDA);
      mu_prev = mu_new;
    }
  };
  if (is_fp64(precision))
    body(double());
  else
    body(float());
  return finish(cs, flags);
}

int dcmesh_graph_create(const dcmesh_domain* doms, int32_t n_dom, int32_t precision, const double* a_dev,
                        int32_t a_per_domain, int64_t a_stride, double dt, int32_t n_steps, const dcmesh_obs* obs,
                        void* work, size_t work_bytes, uint32_t flags, void* stream, void** graph_out) {
  if (!graph_out) return fail(DCMESH_ERR_INVALID_ARGUMENT, "graph_out is NULL");
  if (flags & DCMESH_FLAG_CHECK_FINITE)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "CHECK_FINITE cannot be captured into a graph");
  int rc = validate_domains(doms, n_dom, precision);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<GraphHandle> g(new GraphHandle());
  {
    // stage the tables (pinned allocation) before capturing: a dry pass with
    // zero steps builds the same plan and queues only the table copy
    CallSetup pre;
    rc = step_impl(doms, n_dom, precision, a_dev, a_per_domain, a_stride, dt, 0, obs, work, work_bytes, flags,
                   s, pre);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    pre.keep->graph_refs += 1;
    g->keep = pre.keep;
  }
  CallSetup cs;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  rc = step_impl(doms, n_dom, precision, a_dev, a_per_domain, a_stride, dt, n_steps, obs, work, work_bytes, flags,
                 s, cs);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (rc || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g->keep->graph_refs -= 1;
    return rc ? rc : fail(DCMESH_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  g->graph = graph;
  const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g->keep->graph_refs -= 1;
    return fail(DCMESH_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  *graph_out = g.release();
  return DCMESH_OK;
}

int dcmesh_graph_launch(void* graph, void* stream) {
  if (!graph) return fail(DCMESH_ERR_INVALID_ARGUMENT, "graph is NULL");
  GraphHandle* g = (GraphHandle*)graph;
  HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return DCMESH_OK;
}

int dcmesh_graph_destroy(void* graph) {
  if (!graph) return fail(DCMESH_ERR_INVALID_ARGUMENT, "graph is NULL");
  GraphHandle* g = (GraphHandle*)graph;
  if (g->exec) HIPCHK(hipGraphExecDestroy(g->exec));
  if (g->graph) HIPCHK(hipGraphDestroy(g->graph));
  if (g->keep) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    g->keep->graph_refs -= 1;
  }
  delete g;
  return DCMESH_OK;
}

int dcmesh_profile_collect(double* total_ms, int64_t* launches, int32_t n) {
  if (!total_ms || !launches || n < 0 || n > DCMESH_N_FAMILIES)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "bad profile buffers");
  for (int i = 0; i < n; ++i) { total_ms[i] = 0; launches[i] = 0; }
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    recs.swap(g_prof);
  }
  int rc = DCMESH_OK;
  for (const ProfRec& r : recs) {
    float ms = 0;
    if (rc == DCMESH_OK) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) rc = fail(DCMESH_ERR_HIP, std::string("profile events: ") + hipGetErrorString(e));
    }
    if (r.fam < n) { total_ms[r.fam] += ms; launches[r.fam] += 1; }
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (const ProfRec& r : recs) { g_prof_pool.push_back(r.a); g_prof_pool.push_back(r.b); }
  return rc;
}

int dcmesh_set_tuning(int32_t kernel, int32_t variant) {
  int count = 0;
  int rc = dcmesh_tuning_options(kernel, &count);
  if (rc) return rc;
  if (variant < -1 || variant >= count) return fail(DCMESH_ERR_INVALID_ARGUMENT, "variant out of range");
  g_tune[kernel].store(variant);
  return DCMESH_OK;
}

int dcmesh_set_tuning_shape(int32_t kernel, int32_t precision, const dcmesh_domain* shape, int32_t variant) {
  if (!shape) return fail(DCMESH_ERR_INVALID_ARGUMENT, "shape is NULL");
  if (precision < DCMESH_FP64 || precision > DCMESH_SPLIT_FP16)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "unknown precision " + std::to_string(precision));
  if (kernel == DCMESH_KERNEL_ZSEG || kernel == DCMESH_KERNEL_SORDER)
    return fail(DCMESH_ERR_INVALID_ARGUMENT, "the z segment and the stencil work order are not set per shape");
  int count = 0;
  int rc = dcmesh_tuning_options(kernel, &count);
  if (rc) return rc;
  if (variant < -1 || variant >= count) return fail(DCMESH_ERR_INVALID_ARGUMENT, "variant out of range");
  std::lock_guard<std::mutex> lk(g_shape_mu);
  const ShapeKey k = shape_key(kernel, precision, *shape);
  if (variant < 0)
    g_shape_tune.erase(k);
  else
    g_shape_tune[k] = variant;
  g_shape_count.store((int)g_shape_tune.size());
  return DCMESH_OK;
}

int dcmesh_clear_tuning_shapes(void) {
  std::lock_guard<std::mutex> lk(g_shape_mu);
  g_shape_tune.clear();
  g_shape_count.store(0);
  return DCMESH_OK;
}

int dcmesh_tuning_options(int32_t kernel, int32_t* count) {
  if (!count) return fail(DCMESH_ERR_INVALID_ARGUMENT, "count is NULL");
  switch (kernel) {
    case DCMESH_KERNEL_STENCIL: *count = kNStencil; return DCMESH_OK;
    case DCMESH_KERNEL_PROJECT: *count = kNProj; return DCMESH_OK;
    case DCMESH_KERNEL_CORRECT: *count = kNCorr; return DCMESH_OK;
    case DCMESH_KERNEL_ZSEG: *count = kNZseg; return DCMESH_OK;
    case DCMESH_KERNEL_SORDER: *count = kNSorder; return DCMESH_OK;
    default: return fail(DCMESH_ERR_INVALID_ARGUMENT, "unknown kernel family");
  }
}

}  // extern "C"

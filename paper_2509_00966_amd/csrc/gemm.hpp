// Projector products of the nonlocal term (Sec. V.B.5) on the matrix cores.
//
//   projection  P = h^3 B^H u        M = n_proj, N = n_orb, K = N_g   (split-K)
//   correction  out += B Q            M = N_g,   N = n_orb, K = n_proj
//
// Complex products are written as one real product on the interleaved
// (re, im) storage, so both operands are read straight from the complex arrays:
//   projection: rows p, columns j = (n, c), reduction index (g, c'):
//       A[p][(g,0)] = Re B[g][p], A[p][(g,1)] = Im B[g][p]
//       X[(g,0)][j] = u_raw[g][j],  X[(g,1)][(n,0)] = Im u, X[(g,1)][(n,1)] = -Re u
//   giving Re/Im of sum_g conj(B) u in columns (n,0)/(n,1);
//   correction: out_raw[g][j] += sum_k B_raw[g][k] Q'[k][j] with the real form
//       Q'[(p,0)][(n,0)] = Re Q, Q'[(p,1)][(n,0)] = -Im Q,
//       Q'[(p,0)][(n,1)] = Im Q, Q'[(p,1)][(n,1)] = Re Q.
// A complex product therefore costs 8 M N K real flops, all on MFMA.
//
// Both kernels stream their tiles with 16-byte (VW = 4 floats / 2 doubles) or
// 8-byte (VW = 2 floats, odd row lengths) global loads into registers, one
// chunk ahead of the MFMA work on the chunk held in LDS.
//
// MFMA shape: 16x16x4.  Operand lane l holds row/column l % 16 and reduction
// index l / 16 for both FP32 and FP64.  The accumulator lane l holds column
// l % 16 and four rows: 4 (l / 16) + i for FP32, (l / 16) + 4 i for FP64
// (i = 0..3), as measured on gfx950.
#pragma once

#include "common.hpp"

namespace dcm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename TC> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = f32x4;
  __device__ __forceinline__ static acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lk, int i) { return 4 * lk + i; }
};
template <> struct Mfma<double> {
  using acc_t = f64x4;
  __device__ __forceinline__ static acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lk, int i) { return lk + 4 * i; }
};

// A short vector of VW elements of T moved as one load / store.
template <typename T, int VW> struct alignas(sizeof(T) * VW) Vec { T v[VW]; };

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> vload(const T* p) { return *reinterpret_cast<const Vec<T, VW>*>(p); }

template <typename T, int VW>
__device__ __forceinline__ Vec<T, VW> vzero() {
  Vec<T, VW> z;
#pragma unroll
  for (int i = 0; i < VW; ++i) z.v[i] = (T)0;
  return z;
}

struct ProjArgs {
  int a_slot;        // left operand (proj_operand): slot >= 0 (overlap), -1 B, -2 - d B_d
  int u_slot;        // right operand
  int out_overlap;   // unused by the kernel (kept for the launch record)
};

// Items: (dom, p tile, j tile, split).  Block = 4 waves in 2 x 2, each wave a
// (BM/2) x (BN/2) tile of 16 x 16 MFMA blocks.  KG grid points per LDS stage.
// VW: vector width of the global loads (row lengths 2 np and 2 n_orb must be
// multiples of VW).
template <typename TIn, typename TC, int BM, int BN, int KG, int VW>
__global__ __launch_bounds__(kBlock) void k_project(const DomDesc* __restrict__ doms,
                                                    const Item* __restrict__ items, ProjArgs args) {
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int LA = 2 * BM + 4, LB = BN + 4;          // padded LDS rows
  constexpr int VA = KG * 2 * BM / VW, VB = KG * BN / VW;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) TC sA[KG * LA];
  __shared__ __align__(16) TC sB[KG * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = args.a_slot < 0 ? D.n_proj : D.n_orb;
  const int no2 = 2 * D.n_orb;
  const TIn* __restrict__ Bsrc = (const TIn*)proj_operand<sizeof(TIn)>(D, args.a_slot);
  const TIn* __restrict__ U = (const TIn*)D.slot[args.u_slot];
  const int p0 = it.a * BM, j0 = it.b * BN;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BM / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  using acc_t = typename Mfma<TC>::acc_t;
  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  Vec<TIn, VW> ra[RA], rb[RB];
  auto load = [&](long long gc) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
      const long long g = gc + gl;
      const int p2 = 2 * p0 + c;
      ra[q] = (idx < VA && g < g_end && p2 < 2 * np) ? vload<TIn, VW>(Bsrc + g * (2 * np) + p2) : vzero<TIn, VW>();
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (BN / VW), c = (idx % (BN / VW)) * VW;
      const long long g = gc + gl;
      const int j = j0 + c;
      rb[q] = (idx < VB && g < g_end && j < no2) ? vload<TIn, VW>(U + g * no2 + j) : vzero<TIn, VW>();
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) sA[gl * LA + c + e] = (TC)ra[q].v[e];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (BN / VW), c = (idx % (BN / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) sB[gl * LB + c + e] = (TC)rb[q].v[e];
      }
    }
  };

  // Lane constants of the operand reads.  A: row wm0 + 16 i + ll, reduction
  // index (g, c) with c = lk & 1.  X: for c = 0 column col of u; for c = 1 the
  // partner column (col + 1 for a real part, col - 1 for an imaginary part,
  // negated) -- col has the parity of ll since wn0 and 16 j are even.
  const int cc = lk & 1;
  const int a_off = 2 * (wm0 + ll) + cc;
  const int b_off = wn0 + ll + (cc == 0 ? 0 : ((ll & 1) == 0 ? 1 : -1));
  const TC b_sign = (cc == 1 && (ll & 1)) ? (TC)-1 : (TC)1;

  load(g_begin);
  for (long long gc = g_begin; gc < g_end; gc += KG) {
    store();
    __syncthreads();
    if (gc + KG < g_end) load(gc + KG);
#pragma unroll 2
    for (int ks = 0; ks < KG / 2; ++ks) {
      const int gl = 2 * ks + (lk >> 1);
      TC a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = sA[gl * LA + a_off + 2 * i * 16];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = b_sign * sB[gl * LB + b_off + j * 16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<TC>::run(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  TC* __restrict__ part = (TC*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + Mfma<TC>::row(lk, r);
        const int jj = j0 + wn0 + j * 16 + ll;
        if (p < np && jj < no2) part[(long long)p * no2 + jj] = acc[i][j][r];
      }
}

struct ReduceArgs {
  double cre, cim;     // coef folded into Q = coef D P (f^s)
  int occ_scale;       // fold f_n into Q
  int want_energy;     // nonlocal energy partials sum f D |P|^2
  int write_overlap;   // overlap mode: write h^3 * sum to D.overlap (complex128)
  int want_qmax;       // gather max |Q'| into D.maxbits[2] (FP16 split scaling)
  int unit_d;          // D = 1 (the reference-orbital projector of Eq. 5)
};

// Sum over the split-K partials of entry (p, n) of an np x n_orb complex
// product: (re, im) of split s at ppart[s np 2 n_orb + p 2 n_orb + 2 n].  One
// pair per load, eight splits in flight, summed in split order.
template <typename TC>
__device__ __forceinline__ void split_sum(const DomDesc& D, int np, int p, int n, TC& sr, TC& si) {
  const long long no2 = 2LL * D.n_orb;
  const TC* part = (const TC*)D.ppart + (long long)p * no2 + 2 * n;
  const long long stride = (long long)np * no2;
  sr = 0;
  si = 0;
  int s = 0;
  for (; s + 8 <= D.n_split; s += 8) {
    Vec<TC, 2> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = vload<TC, 2>(part + (s + u) * stride);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sr += v[u].v[0];
      si += v[u].v[1];
    }
  }
  for (; s < D.n_split; ++s) {
    const Vec<TC, 2> v = vload<TC, 2>(part + s * stride);
    sr += v.v[0];
    si += v.v[1];
  }
}

// Items: (dom, block index over n_proj * n_orb pairs).  Deterministic: the
// split-K partials are summed in split order.  Q' rows are D.ldq apart.
template <typename TC>
__global__ __launch_bounds__(kBlock) void k_reduce(const DomDesc* __restrict__ doms,
                                                   const Item* __restrict__ items, ReduceArgs args) {
  __shared__ double red[4];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = args.write_overlap ? D.n_orb : D.n_proj;
  const int no = D.n_orb, no2 = 2 * no;
  const long long idx = (long long)it.a * kBlock + threadIdx.x;
  const bool ok = idx < (long long)np * no;
  double e = 0.0;
  float qmax = 0.f;
  if (ok) {
    const int p = (int)(idx / no), n = (int)(idx % no);
    TC sr, si;
    split_sum<TC>(D, np, p, n, sr, si);
    const double h3 = D.h * D.h * D.h;
    if (args.write_overlap) {
      D.overlap[((long long)p * no + n) * 2] = h3 * (double)sr;
      D.overlap[((long long)p * no + n) * 2 + 1] = h3 * (double)si;
    } else {
      const TC pr = (TC)(h3 * (double)sr), pi = (TC)(h3 * (double)si);
      TC* P = (TC*)D.pmat;
      P[(long long)p * no2 + 2 * n] = pr;
      P[(long long)p * no2 + 2 * n + 1] = pi;
      const TC dp = args.unit_d ? (TC)1 : ((const TC*)D.d)[p];
      const TC fn = ((const TC*)D.occ)[n];
      const TC sc = args.occ_scale ? dp * fn : dp;
      const TC qr = sc * ((TC)args.cre * pr - (TC)args.cim * pi);
      const TC qi = sc * ((TC)args.cre * pi + (TC)args.cim * pr);
      TC* Q = (TC*)D.qmat;
      const long long ldq = D.ldq;
      Q[(long long)(2 * p) * ldq + 2 * n] = qr;
      Q[(long long)(2 * p) * ldq + 2 * n + 1] = qi;
      Q[(long long)(2 * p + 1) * ldq + 2 * n] = -qi;
      Q[(long long)(2 * p + 1) * ldq + 2 * n + 1] = qr;
      if (D.qmat3) {
        TC* Q3 = (TC*)D.qmat3;
        const long long pl = (long long)np * D.ldq3;
        Q3[(long long)p * D.ldq3 + n] = qr;
        Q3[pl + (long long)p * D.ldq3 + n] = qi - qr;
        Q3[2 * pl + (long long)p * D.ldq3 + n] = qr + qi;
      }
      if (args.want_energy) e = (double)fn * (double)dp * ((double)pr * pr + (double)pi * pi);
      qmax = fmaxf(fabsf((float)qr), fabsf((float)qi));
    }
  }
  if (args.want_qmax) {
    float m = qmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&D.maxbits[2], __float_as_uint(m));
  }
  if (args.want_energy) {
    const double s = block_sum(e, red);
    if (threadIdx.x == 0) D.e_nl[blockIdx.x - D.item0_reduce] = s;
  }
}

// Nonlocal current of one axis d: with P = h^3 B^H u in D.pmat (left by
// k_reduce) and the split-K partials of h^3 B_d^H u in D.ppart, the block sums
// of f_n D_p Im(conj(P_pn) R_pn), R summed over the splits in order, go to
// jnl_part[d][item].  Items: those of k_reduce.
template <typename TC>
__global__ __launch_bounds__(kBlock) void k_jnl_partial(const DomDesc* __restrict__ doms,
                                                        const Item* __restrict__ items, int d) {
  __shared__ double red[kBlock / kWave];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, no2 = 2 * no;
  const long long idx = (long long)it.a * kBlock + threadIdx.x;
  double v = 0.0;
  if (idx < (long long)np * no) {
    const int p = (int)(idx / no), n = (int)(idx % no);
    TC sr, si;
    split_sum<TC>(D, np, p, n, sr, si);
    const double h3 = D.h * D.h * D.h;
    const double rr = h3 * (double)sr, ri = h3 * (double)si;
    const TC* P = (const TC*)D.pmat;
    const double pr = (double)P[(long long)p * no2 + 2 * n], pi = (double)P[(long long)p * no2 + 2 * n + 1];
    v = (double)((const TC*)D.occ)[n] * (double)((const TC*)D.d)[p] * (pr * ri - pi * rr);
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) D.jnl_part[(long long)d * D.n_e_nl + (blockIdx.x - D.item0_reduce)] = v;
}

// Items: (dom, g tile, j tile).  out_raw[g][j] += sum_k B_raw[g][k] Q'[k][j].
// Block = 4 waves in 2 x 2; KC real reduction indices per LDS stage.  VW: load
// width for the rows of B (2 n_proj must be a multiple of VW); Q' rows are
// padded to a multiple of 4 elements (D.ldq) and zero in the padding.
template <typename TIn, typename TC, int BMG, int BN, int KC, int VW>
__global__ __launch_bounds__(kBlock) void k_correct(const DomDesc* __restrict__ doms,
                                                    const Item* __restrict__ items, int out_slot) {
  constexpr int TM = BMG / 32, TN = BN / 32;
  // LDS row pads: A rows of KC + 2 keep the 16 rows x 2 reduction indices of a
  // half-wave on distinct banks; B rows of BN + 16 (FP32) put the two
  // reduction rows of a half-wave 16 banks apart.
  constexpr int LA = KC + 2, LB = BN + (sizeof(TC) == 4 ? 16 : 4);
  constexpr int QW = 16 / sizeof(TC);                   // Q' vector width (rows padded)
  constexpr int VA = BMG * KC / VW, VB = KC * BN / QW;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) TC sA[BMG * LA];
  __shared__ __align__(16) TC sB[KC * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int K = 2 * D.n_proj, no2 = 2 * D.n_orb;
  const long long ldq = D.ldq;
  const long long g0 = (long long)it.a * BMG;
  const int j0 = it.b * BN;
  const TIn* __restrict__ Braw = (const TIn*)D.proj;
  const TC* __restrict__ Q = (const TC*)D.qmat;
  TIn* __restrict__ out = (TIn*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BMG / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  using acc_t = typename Mfma<TC>::acc_t;
  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  Vec<TIn, VW> ra[RA];
  Vec<TC, QW> rb[RB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KC / VW), c = (idx % (KC / VW)) * VW;
      const long long g = g0 + r;
      const int k = k0 + c;
      ra[q] = (idx < VA && g < D.n_grid && k < K) ? vload<TIn, VW>(Braw + g * K + k) : vzero<TIn, VW>();
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (BN / QW), c = (idx % (BN / QW)) * QW;
      const int k = k0 + r, j = j0 + c;
      rb[q] = (idx < VB && k < K && j < ldq) ? vload<TC, QW>(Q + (long long)k * ldq + j) : vzero<TC, QW>();
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (KC / VW), c = (idx % (KC / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) sA[r * LA + c + e] = (TC)ra[q].v[e];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int r = idx / (BN / QW), c = (idx % (BN / QW)) * QW;
        *reinterpret_cast<Vec<TC, QW>*>(&sB[r * LB + c]) = rb[q];
      }
    }
  };

  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    store();
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll 2
    for (int ks = 0; ks < KC / 4; ++ks) {
      TC a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = sA[(wm0 + i * 16 + ll) * LA + ks * 4 + lk];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = sB[(ks * 4 + lk) * LB + wn0 + j * 16 + ll];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mfma<TC>::run(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  // out += acc: every read is issued before the first write, so the reads
  // overlap instead of each waiting behind the previous write
  TIn prev[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + Mfma<TC>::row(lk, r);
        const int jj = j0 + wn0 + j * 16 + ll;
        prev[i][j][r] = (g < D.n_grid && jj < no2) ? out[g * no2 + jj] : (TIn)0;
      }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + Mfma<TC>::row(lk, r);
        const int jj = j0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && jj < no2) out[g * no2 + jj] = (TIn)((TC)prev[i][j][r] + acc[i][j][r]);
      }
}

}  // namespace dcm

namespace dcm {

// ---------------------------------------------------------------------------
// FP32 projector products with three real products per complex product
// (Gauss's form), on the complex operands as stored:
//   (a + ib)(c + id):  k1 = c (a + b'), k2 = a (d - c), k3 = b' (c + d),
//                      Re = k1 - k3, Im = k1 + k2   (b' = b, or -b for conj(a + ib)).
// Projection P = B^H u: a = Re B, b' = -Im B, c = Re u, d = Im u.
// Correction B Q:       a = Re B, b' =  Im B, c = Re Q, d = Im Q, with the
// three combinations of Q stored by the reduce kernel as planes
// Q3[0] = Re Q, Q3[1] = Im Q - Re Q, Q3[2] = Re Q + Im Q.
// Each complex multiply-add costs 6 real flops on MFMA instead of 8.
// ---------------------------------------------------------------------------

// Items: (dom, p tile, complex-orbital tile, split).  Block = 4 waves in 2 x 2,
// wave tile (BM/2) projectors x (BNC/2) orbitals; KG grid points per LDS stage.
template <int BM, int BNC, int KG, int VW>
__global__ __launch_bounds__(kBlock) void k_project3m(const DomDesc* __restrict__ doms,
                                                      const Item* __restrict__ items, ProjArgs args) {
  constexpr int TM = BM / 32, TN = BNC / 32;
  constexpr int LA = 2 * BM + 8, LB = 2 * BNC + 8;
  constexpr int VA = KG * 2 * BM / VW, VB = KG * 2 * BNC / VW;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[KG * LA];
  __shared__ __align__(16) float sB[KG * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, no2 = 2 * no;
  const float* __restrict__ Bsrc = (const float*)proj_operand<4>(D, args.a_slot);
  const float* __restrict__ U = (const float*)D.slot[args.u_slot];
  const int p0 = it.a * BM, n0 = it.b * BNC;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BM / 2), wn0 = (wv % 2) * (BNC / 2);
  const int ll = lane % 16, lk = lane / 16;
  f32x4 k1[TM][TN], k2[TM][TN], k3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) k1[i][j] = k2[i][j] = k3[i][j] = f32x4{0, 0, 0, 0};

  Vec<float, VW> ra[RA], rb[RB];
  auto load = [&](long long gc) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
      const long long g = gc + gl;
      const int p2 = 2 * p0 + c;
      ra[q] = (idx < VA && g < g_end && p2 < 2 * np) ? vload<float, VW>(Bsrc + g * (2 * np) + p2) : vzero<float, VW>();
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (2 * BNC / VW), c = (idx % (2 * BNC / VW)) * VW;
      const long long g = gc + gl;
      const int j = 2 * n0 + c;
      rb[q] = (idx < VB && g < g_end && j < no2) ? vload<float, VW>(U + g * no2 + j) : vzero<float, VW>();
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
        *reinterpret_cast<Vec<float, VW>*>(&sA[gl * LA + c]) = ra[q];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (2 * BNC / VW), c = (idx % (2 * BNC / VW)) * VW;
        *reinterpret_cast<Vec<float, VW>*>(&sB[gl * LB + c]) = rb[q];
      }
    }
  };

  load(g_begin);
  for (long long gc = g_begin; gc < g_end; gc += KG) {
    store();
    __syncthreads();
    if (gc + KG < g_end) load(gc + KG);
#pragma unroll 2
    for (int ks = 0; ks < KG / 4; ++ks) {
      const int gl = 4 * ks + lk;
      float a1[TM], a2[TM], a3[TM], b1[TN], b2[TN], b3[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const float2 v = *reinterpret_cast<const float2*>(&sA[gl * LA + 2 * (wm0 + i * 16 + ll)]);
        a1[i] = v.x - v.y;   // a + b' with b' = -Im B
        a2[i] = v.x;
        a3[i] = -v.y;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const float2 v = *reinterpret_cast<const float2*>(&sB[gl * LB + 2 * (wn0 + j * 16 + ll)]);
        b1[j] = v.x;
        b2[j] = v.y - v.x;
        b3[j] = v.x + v.y;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          k1[i][j] = Mfma<float>::run(a1[i], b1[j], k1[i][j]);
          k2[i][j] = Mfma<float>::run(a2[i], b2[j], k2[i][j]);
          k3[i][j] = Mfma<float>::run(a3[i], b3[j], k3[i][j]);
        }
    }
    __syncthreads();
  }
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        if (p < np && n < no)
          *reinterpret_cast<float2*>(&part[(long long)p * no2 + 2 * n]) =
              make_float2(k1[i][j][r] - k3[i][j][r], k1[i][j][r] + k2[i][j][r]);
      }
}

// Raw buffer resource over [base, base + bytes): reads at or past the end
// return zero (gfx9 descriptor word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(const DCM_GLOBAL void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
}

// 16 bytes per lane from a buffer into LDS: lane i's bytes land at
// dst + 16 i (one wave moves 1 KB); dst is wave-uniform.
__device__ __forceinline__ void load_lds16(__amdgpu_buffer_rsrc_t r, float* dst, unsigned voffset) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)dst, 16, voffset, 0, 0, 0);
}

// The three-product projection with the operand tiles moved from memory
// straight into LDS (buffer loads with an LDS destination), double-buffered:
// no staging registers and one barrier per stage.  A stage holds KG grid
// points: KG rows of 2 BM floats of B (1 KB, one wave instruction each) and KG
// rows of 2 BNC floats of u (512 B; one instruction moves two).  The buffers
// start at the block's first grid point and end at its last, so rows past the
// split read as zero; columns past n_proj or n_orb (read from the next row, or
// zero) reach only outputs that are not stored.  Items as k_project3m.
template <int BM, int BNC, int KG>
__global__ __launch_bounds__(kBlock) void k_project3m_dl(const DomDesc* __restrict__ doms,
                                                         const Item* __restrict__ items, ProjArgs args) {
  constexpr int TM = BM / 32, TN = BNC / 32;
  constexpr int RA = 2 * BM, RB = 2 * BNC;             // floats per LDS row
  // one wave instruction moves 1 KB: RPA rows of B (LPA lanes each), RPB of u
  constexpr int RPA = 256 / RA, LPA = RA / 4, RPB = 256 / RB, LPB = RB / 4;
  static_assert((RA == 256 || RA == 128) && RB == 128, "rows of 1 KB or 512 B (B) and 512 B (u)");
  static_assert(RPA * LPA == kWave && RPB * LPB == kWave, "whole rows per wave instruction");
  static_assert(KG % 8 == 0, "whole wave instructions per stage");
  constexpr int SA = KG * RA, SB = KG * RB;
  __shared__ __align__(16) float sA0[SA], sA1[SA];
  __shared__ __align__(16) float sB0[SB], sB1[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, no2 = 2 * no;
  const int p0 = it.a * BM, n0 = it.b * BNC;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);
  const int n_st = (int)((g_end - g_begin + KG - 1) / KG);
  const unsigned rowA = 8u * (unsigned)np, rowB = 8u * (unsigned)no;     // bytes per grid point
  const DCM_GLOBAL char* Bsrc = proj_operand<4>(D, args.a_slot) + g_begin * rowA;
  const DCM_GLOBAL char* Usrc = (const DCM_GLOBAL char*)D.slot[args.u_slot] + g_begin * rowB;
  const __amdgpu_buffer_rsrc_t ra = buffer_over(Bsrc, (unsigned)(g_end - g_begin) * rowA);
  const __amdgpu_buffer_rsrc_t rb = buffer_over(Usrc, (unsigned)(g_end - g_begin) * rowB);

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 2) * (BM / 2), wn0 = (wv % 2) * (BNC / 2);
  const int ll = lane % 16, lk = lane / 16;
  const unsigned colA = 4u * (2u * p0 + 4u * (lane % LPA));      // this lane's 16 bytes of a B row
  const unsigned colB = 4u * (2u * n0 + 4u * (lane % LPB));      // ... of a u row
  f32x4 k1[TM][TN], k2[TM][TN], k3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) k1[i][j] = k2[i][j] = k3[i][j] = f32x4{0, 0, 0, 0};

  auto issue = [&](int st, float* sA, float* sB) {
#pragma unroll
    for (int r = wv; r < KG / RPA; r += 4)
      load_lds16(ra, sA + RPA * r * RA, (unsigned)(st * KG + RPA * r + lane / LPA) * rowA + colA);
#pragma unroll
    for (int r2 = wv; r2 < KG / RPB; r2 += 4)
      load_lds16(rb, sB + RPB * r2 * RB, (unsigned)(st * KG + RPB * r2 + lane / LPB) * rowB + colB);
  };
  auto compute = [&](const float* sA, const float* sB) {
#pragma unroll 2
    for (int ks = 0; ks < KG / 4; ++ks) {
      const int gl = 4 * ks + lk;
      float a1[TM], a2[TM], a3[TM], b1[TN], b2[TN], b3[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const float2 v = *reinterpret_cast<const float2*>(&sA[gl * RA + 2 * (wm0 + i * 16 + ll)]);
        a1[i] = v.x - v.y;
        a2[i] = v.x;
        a3[i] = -v.y;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const float2 v = *reinterpret_cast<const float2*>(&sB[gl * RB + 2 * (wn0 + j * 16 + ll)]);
        b1[j] = v.x;
        b2[j] = v.y - v.x;
        b3[j] = v.x + v.y;
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          k1[i][j] = Mfma<float>::run(a1[i], b1[j], k1[i][j]);
          k2[i][j] = Mfma<float>::run(a2[i], b2[j], k2[i][j]);
          k3[i][j] = Mfma<float>::run(a3[i], b3[j], k3[i][j]);
        }
    }
  };
  // stage st computes from buffer st % 2 while stage st + 1 streams into the
  // other; the barrier after each wait makes a stage's rows visible to every
  // wave and retires the readers of the buffer about to be refilled
  if (n_st > 0) issue(0, sA0, sB0);
  int st = 0;
  for (; st + 1 < n_st; st += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    issue(st + 1, sA1, sB1);
    compute(sA0, sB0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (st + 2 < n_st) issue(st + 2, sA0, sB0);
    compute(sA1, sB1);
  }
  if (st < n_st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    compute(sA0, sB0);
  }
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        if (p < np && n < no)
          *reinterpret_cast<float2*>(&part[(long long)p * no2 + 2 * n]) =
              make_float2(k1[i][j][r] - k3[i][j][r], k1[i][j][r] + k2[i][j][r]);
      }
}

// Items: (dom, g tile, complex-orbital tile).  out[g][n] += sum_p B[g][p] Q[p][n]
// with Q from the three planes D.qmat3 (rows of D.ldq3 floats).  Block = 4
// waves in 2 x 2, wave tile (BMG/2) grid points x (BNC/2) orbitals; KC
// projectors per LDS stage.
template <int BMG, int BNC, int KC, int VW>
__global__ __launch_bounds__(kBlock) void k_correct3m(const DomDesc* __restrict__ doms,
                                                      const Item* __restrict__ items, int out_slot) {
  constexpr int TM = BMG / 32, TN = BNC / 32;
  constexpr int LA = 2 * KC + 2, LB = BNC + 16;
  constexpr int VA = BMG * 2 * KC / VW, VB = 3 * KC * BNC / 4;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[BMG * LA];
  __shared__ __align__(16) float sB[3 * KC * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, K2 = 2 * np;
  const long long ldq3 = D.ldq3;
  const long long g0 = (long long)it.a * BMG;
  const int n0 = it.b * BNC;
  const float* __restrict__ Braw = (const float*)D.proj;
  const float* __restrict__ Q3 = (const float*)D.qmat3;
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BMG / 2), wn0 = (wv % 2) * (BNC / 2);
  const int ll = lane % 16, lk = lane / 16;
  f32x4 k1[TM][TN], k2[TM][TN], k3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) k1[i][j] = k2[i][j] = k3[i][j] = f32x4{0, 0, 0, 0};

  Vec<float, VW> ra[RA];
  Vec<float, 4> rb[RB];
  auto load = [&](int p0) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
      const long long g = g0 + r;
      const int k = 2 * p0 + c;
      ra[q] = (idx < VA && g < D.n_grid && k < K2) ? vload<float, VW>(Braw + g * K2 + k) : vzero<float, VW>();
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int row = idx / (BNC / 4), c = (idx % (BNC / 4)) * 4;   // row = plane * KC + p_local
      const int pl = row / KC, p = p0 + row % KC, n = n0 + c;
      rb[q] = (idx < VB && p < np && n < ldq3) ? vload<float, 4>(Q3 + ((long long)pl * np + p) * ldq3 + n)
                                               : vzero<float, 4>();
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; e += 2)
          *reinterpret_cast<float2*>(&sA[r * LA + c + e]) = make_float2(ra[q].v[e], ra[q].v[e + 1]);
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int row = idx / (BNC / 4), c = (idx % (BNC / 4)) * 4;
        *reinterpret_cast<Vec<float, 4>*>(&sB[row * LB + c]) = rb[q];
      }
    }
  };

  load(0);
  for (int p0 = 0; p0 < np; p0 += KC) {
    store();
    __syncthreads();
    if (p0 + KC < np) load(p0 + KC);
#pragma unroll 2
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int pl = 4 * ks + lk;
      float a1[TM], a2[TM], a3[TM], b1[TN], b2[TN], b3[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const float2 v = *reinterpret_cast<const float2*>(&sA[(wm0 + i * 16 + ll) * LA + 2 * pl]);
        a1[i] = v.x + v.y;
        a2[i] = v.x;
        a3[i] = v.y;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn0 + j * 16 + ll;
        b1[j] = sB[(0 * KC + pl) * LB + n];
        b2[j] = sB[(1 * KC + pl) * LB + n];
        b3[j] = sB[(2 * KC + pl) * LB + n];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          k1[i][j] = Mfma<float>::run(a1[i], b1[j], k1[i][j]);
          k2[i][j] = Mfma<float>::run(a2[i], b2[j], k2[i][j]);
          k3[i][j] = Mfma<float>::run(a3[i], b3[j], k3[i][j]);
        }
    }
    __syncthreads();
  }
  // out += result, one 16-row tile at a time: the tile's reads are all issued
  // before its first write, so they overlap instead of each waiting behind the
  // previous write (a whole-block batch would cost the registers of a second
  // wave per SIMD)
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float2 prev[TN][4];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        prev[j][r] = (g < D.n_grid && n < no) ? *reinterpret_cast<const float2*>(out + (g * no + n) * 2)
                                               : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && n < no)
          *reinterpret_cast<float2*>(out + (g * no + n) * 2) =
              make_float2(prev[j][r].x + (k1[i][j][r] - k3[i][j][r]), prev[j][r].y + (k1[i][j][r] + k2[i][j][r]));
      }
  }
}

// The three-product correction with the Q tile moved from memory straight
// into LDS (buffer loads with an LDS destination) and both tiles
// double-buffered (one barrier per stage).  A stage holds KC projectors: the
// three Q planes give 3 KC rows of BNC floats (BNC = 128: 512 B, one wave
// instruction moves two rows; BNC = 64: 256 B, four rows), and the projector
// rows of B are staged through registers into padded LDS rows as in
// k_correct3m.  Odd Q rows are stored rotated by 16 floats, so the two 16-lane
// quarters of a half-wave, which read consecutive rows, use disjoint LDS banks.  Each plane's buffer ends after n_proj rows, so rows past it read
// as zero; columns past n_orb reach only outputs that are not stored.
template <int BMG, int BNC, int KC, int VW, bool PF = false>
__global__ __launch_bounds__(kBlock) void k_correct3m_dl(const DomDesc* __restrict__ doms,
                                                         const Item* __restrict__ items, int out_slot) {
  constexpr int TM = BMG / 32, TN = BNC / 32;
  constexpr int LA = 2 * KC + 2;
  static_assert(BNC == 128 || BNC == 64, "Q rows of 512 B or 256 B");
  constexpr int RPI = 256 / BNC;                                 // Q rows per wave instruction (1 KB)
  static_assert(KC % RPI == 0, "Q rows move in whole instructions");
  constexpr int VA = BMG * 2 * KC / VW;
  constexpr int RA = (VA + kBlock - 1) / kBlock;
  constexpr int SB = 3 * KC * BNC;
  __shared__ __align__(16) float sA0[BMG * LA], sA1[BMG * LA];
  __shared__ __align__(16) float sB0[SB], sB1[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, K2 = 2 * np;
  const long long ldq3 = D.ldq3;
  const long long g0 = (long long)it.a * BMG;
  const int n0 = it.b * BNC;
  const float* __restrict__ Braw = (const float*)D.proj;
  float* __restrict__ out = (float*)D.slot[out_slot];
  const unsigned qrow = 4u * (unsigned)ldq3;                     // bytes per Q row
  __amdgpu_buffer_rsrc_t rq[3];
#pragma unroll
  for (int pl = 0; pl < 3; ++pl)
    rq[pl] = buffer_over((const DCM_GLOBAL char*)D.qmat3 + (long long)pl * np * qrow, (unsigned)np * qrow);

  // the wave index is uniform: buffer descriptors and LDS destinations chosen
  // by it stay in scalar registers
  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 2) * (BMG / 2), wn0 = (wv % 2) * (BNC / 2);
  const int ll = lane % 16, lk = lane / 16;
  // one instruction moves RPI consecutive rows (BNC / 4 lanes each); odd rows
  // are stored rotated by 16 floats
  constexpr int LPR = BNC / 4;                                   // lanes per row
  static_assert(LPR * RPI == kWave, "one wave instruction moves RPI whole rows");
  const int qt = lane % LPR, qodd = (lane / LPR) & 1;
  const unsigned qcol = 4u * (unsigned)(n0 + 4 * (qodd ? (qt + 4) % LPR : qt));
  const int bshift = (lk & 1) ? 16 : 0;                          // this lane reads odd rows
  f32x4 k1[TM][TN], k2[TM][TN], k3[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) k1[i][j] = k2[i][j] = k3[i][j] = f32x4{0, 0, 0, 0};
  // PF: the output tile this lane adds into is requested before the
  // reduction, so that its latency is spent under the products (a short
  // reduction, as in small domains, otherwise ends on a full memory round
  // trip); it costs about 40 registers, one wave per SIMD
  float2 prev[TM][TN][4];
  auto load_prev = [&](int i) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        prev[i][j][r] = (g < D.n_grid && n < no) ? *reinterpret_cast<const float2*>(out + (g * no + n) * 2)
                                                  : make_float2(0.f, 0.f);
      }
  };
  if constexpr (PF) {
#pragma unroll
    for (int i = 0; i < TM; ++i) load_prev(i);
  }

  Vec<float, VW> ra[RA];
  auto load_a = [&](int st) {
    const int p0 = st * KC;
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
      const long long g = g0 + r;
      const int k = 2 * p0 + c;
      ra[q] = (idx < VA && g < D.n_grid && k < K2) ? vload<float, VW>(Braw + g * K2 + k) : vzero<float, VW>();
    }
  };
  auto store_a = [&](float* sA) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; e += 2)
          *reinterpret_cast<float2*>(&sA[r * LA + c + e]) = make_float2(ra[q].v[e], ra[q].v[e + 1]);
      }
    }
  };
  auto issue_q = [&](int st, float* sB) {
    // row groups (plane, RPI m .. RPI m + RPI - 1): 3 KC / RPI instructions per stage
#pragma unroll
    for (int pr = wv; pr < 3 * KC / RPI; pr += 4) {
      const int pl = pr / (KC / RPI), m = pr % (KC / RPI);
      const int row = st * KC + RPI * m + lane / LPR;
      load_lds16(rq[pl], sB + (pl * KC + RPI * m) * BNC, (unsigned)row * qrow + qcol);
    }
  };
  auto compute = [&](const float* sA, const float* sB) {
#pragma unroll 2
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int pl = 4 * ks + lk;
      float a1[TM], a2[TM], a3[TM], b1[TN], b2[TN], b3[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const float2 v = *reinterpret_cast<const float2*>(&sA[(wm0 + i * 16 + ll) * LA + 2 * pl]);
        a1[i] = v.x + v.y;
        a2[i] = v.x;
        a3[i] = v.y;
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int pos = (wn0 + j * 16 + ll - bshift) & (BNC - 1);
        b1[j] = sB[(0 * KC + pl) * BNC + pos];
        b2[j] = sB[(1 * KC + pl) * BNC + pos];
        b3[j] = sB[(2 * KC + pl) * BNC + pos];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          k1[i][j] = Mfma<float>::run(a1[i], b1[j], k1[i][j]);
          k2[i][j] = Mfma<float>::run(a2[i], b2[j], k2[i][j]);
          k3[i][j] = Mfma<float>::run(a3[i], b3[j], k3[i][j]);
        }
    }
  };
  // stage st reads buffer st % 2; the wait + barrier at its top publishes its
  // tiles and retires the readers of the buffers about to be refilled
  const int n_st = (np + KC - 1) / KC;
  if (n_st > 0) {
    load_a(0);
    issue_q(0, sB0);
  }
  int st = 0;
  for (; st + 1 < n_st; st += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    store_a(sA0);
    __syncthreads();
    load_a(st + 1);
    issue_q(st + 1, sB1);
    compute(sA0, sB0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_a(sA1);
    __syncthreads();
    if (st + 2 < n_st) {
      load_a(st + 2);
      issue_q(st + 2, sB0);
    }
    compute(sA1, sB1);
  }
  if (st < n_st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_a(sA0);
    __syncthreads();
    compute(sA0, sB0);
  }
  // out += result, one 16-row tile at a time (reads before writes)
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    if constexpr (!PF) load_prev(i);
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int n = n0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && n < no)
          *reinterpret_cast<float2*>(out + (g * no + n) * 2) =
              make_float2(prev[i][j][r].x + (k1[i][j][r] - k3[i][j][r]),
                          prev[i][j][r].y + (k1[i][j][r] + k2[i][j][r]));
      }
  }
}

// ---------------------------------------------------------------------------
// FP32 three-product products with every orbital of a domain in one block,
// for domains with at most 16 NB orbitals.  Four waves are stacked along the
// long operand's rows (16 rows each), and each wave covers all NB 16-orbital
// column blocks, so the orbital padding stays below 16 columns: on the batch of
// domains with 16-96 orbitals, 64-orbital tiles do 1.5x (correction) and 1.8x
// (projection) the useful products.  Both tiles pass through registers into
// double-buffered LDS; the loads are issued a stage ahead (the projection's,
// over long reductions, two stages ahead in two register sets) and stay in
// flight across the LDS-only barriers.
// ---------------------------------------------------------------------------

// Row stride (floats) of an LDS tile of 16 NB columns: consecutive rows start
// on opposite halves of the banks for the two 16-lane quarters of a half-wave.
template <int NB>
constexpr int narrow_ld() { return 16 * NB + (NB % 2 == 0 ? 16 : 0); }

// Correction out += B Q (Q as the three planes of qmat3) on 64-row tiles.
// Items: (dom, 64-row tile, 0, 0).  A stage holds KC = 16 projectors.  The
// output tile is requested before the reduction, so its latency is spent
// under the products.
template <int NB, int VW>
__global__ __launch_bounds__(kBlock) void k_correct3m_n(const DomDesc* __restrict__ doms,
                                                        const Item* __restrict__ items, int out_slot) {
  constexpr int KC = 16, BMG = 64, BNC = 16 * NB;
  constexpr int LA = 2 * KC + 2, LB = narrow_ld<NB>();
  constexpr int VA = BMG * 2 * KC / VW, RA = (VA + kBlock - 1) / kBlock;
  constexpr int VQ = 3 * KC * BNC / 4, RQ = (VQ + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[2][BMG * LA];
  __shared__ __align__(16) float sB[2][3 * KC * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, K2 = 2 * np;
  const long long ldq3 = D.ldq3;
  const long long g0 = (long long)it.a * BMG;
  const float* __restrict__ Braw = (const float*)D.proj;
  const float* __restrict__ Q3 = (const float*)D.qmat3;
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = wv * 16;
  const int ll = lane % 16, lk = lane / 16;
  f32x4 k1[NB], k2[NB], k3[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) k1[j] = k2[j] = k3[j] = f32x4{0, 0, 0, 0};
  float2 prev[NB][4];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long g = g0 + wm0 + 4 * lk + r;
      const int n = j * 16 + ll;
      prev[j][r] = (g < D.n_grid && n < no) ? *reinterpret_cast<const float2*>(out + (g * no + n) * 2)
                                             : make_float2(0.f, 0.f);
    }

  // one register set, loaded a stage ahead (the reductions are short: two
  // register sets cost occupancy and measured slower)
  Vec<float, VW> ra[1][RA];
  Vec<float, 4> rq[1][RQ];
  auto load = [&](int set, int st) {
    const int p0 = st * KC;
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
      const long long g = g0 + r;
      const int k = 2 * p0 + c;
      ra[set][q] = (idx < VA && g < D.n_grid && k < K2) ? vload<float, VW>(Braw + g * K2 + k) : vzero<float, VW>();
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int row = idx / (BNC / 4), c = (idx % (BNC / 4)) * 4;    // row = plane * KC + projector
      const int pl = row / KC, p = p0 + row % KC;
      rq[set][q] = (idx < VQ && p < np && c < ldq3) ? vload<float, 4>(Q3 + ((long long)pl * np + p) * ldq3 + c)
                                                    : vzero<float, 4>();
    }
  };
  auto store = [&](int set, int b) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (2 * KC / VW), c = (idx % (2 * KC / VW)) * VW;
#pragma unroll
        for (int e = 0; e < VW; e += 2)
          *reinterpret_cast<float2*>(&sA[b][r * LA + c + e]) = make_float2(ra[set][q].v[e], ra[set][q].v[e + 1]);
      }
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VQ) {
        const int row = idx / (BNC / 4), c = (idx % (BNC / 4)) * 4;
        *reinterpret_cast<Vec<float, 4>*>(&sB[b][row * LB + c]) = rq[set][q];
      }
    }
  };
  auto compute = [&](int b) {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int pl = 4 * ks + lk;
      const float2 v = *reinterpret_cast<const float2*>(&sA[b][(wm0 + ll) * LA + 2 * pl]);
      const float a1 = v.x + v.y, a2 = v.x, a3 = v.y;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int col = j * 16 + ll;
        k1[j] = Mfma<float>::run(a1, sB[b][(0 * KC + pl) * LB + col], k1[j]);
        k2[j] = Mfma<float>::run(a2, sB[b][(1 * KC + pl) * LB + col], k2[j]);
        k3[j] = Mfma<float>::run(a3, sB[b][(2 * KC + pl) * LB + col], k3[j]);
      }
    }
  };
  // stage st: LDS buffer st % 2, whose last readers (stage st - 2) finished
  // before the barrier of stage st - 1
  const int n_st = (np + KC - 1) / KC;
  load(0, 0);
  for (int st = 0; st < n_st; ++st) {
    store(0, st & 1);
    lds_barrier();
    if (st + 1 < n_st) load(0, st + 1);
    compute(st & 1);
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long g = g0 + wm0 + 4 * lk + r;
      const int n = j * 16 + ll;
      if (g < D.n_grid && n < no)
        *reinterpret_cast<float2*>(out + (g * no + n) * 2) =
            make_float2(prev[j][r].x + (k1[j][r] - k3[j][r]), prev[j][r].y + (k1[j][r] + k2[j][r]));
    }
}

// Projection partials P_split = h^3-free sum over the split's grid points of
// conj(B) u (the h^3 and D factors are applied by k_reduce), for 64
// projectors per block.  Items: (dom, 64-projector tile, 0, split).  A stage
// holds KG = 16 grid points.  Waves whose 16 projectors lie past n_proj load
// and synchronise with the others but skip their products.
template <int NB, int VW>
__global__ __launch_bounds__(kBlock) void k_project3m_n(const DomDesc* __restrict__ doms,
                                                        const Item* __restrict__ items, ProjArgs args) {
  constexpr int KG = 16, BM = 64, BNC = 16 * NB;
  constexpr int LA = 2 * BM + 8, LB = 2 * narrow_ld<NB>();
  constexpr int VA = KG * 2 * BM / VW, RA = (VA + kBlock - 1) / kBlock;
  constexpr int VB = KG * 2 * BNC / VW, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) float sA[2][KG * LA];
  __shared__ __align__(16) float sB[2][KG * LB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no = D.n_orb, no2 = 2 * no;
  const float* __restrict__ Bsrc = (const float*)proj_operand<4>(D, args.a_slot);
  const float* __restrict__ U = (const float*)D.slot[args.u_slot];
  const int p0 = it.a * BM;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = wv * 16;
  const bool active = p0 + wm0 < np;          // wave-uniform
  const int ll = lane % 16, lk = lane / 16;
  f32x4 k1[NB], k2[NB], k3[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) k1[j] = k2[j] = k3[j] = f32x4{0, 0, 0, 0};

  // two register sets: stage st is loaded into set st % 2 two stages ahead
  Vec<float, VW> ra[2][RA], rb[2][RB];
  auto load = [&](int set, long long gc) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
      const long long g = gc + gl;
      const int p2 = 2 * p0 + c;
      ra[set][q] = (idx < VA && g < g_end && p2 < 2 * np) ? vload<float, VW>(Bsrc + g * (2 * np) + p2)
                                                          : vzero<float, VW>();
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (2 * BNC / VW), c = (idx % (2 * BNC / VW)) * VW;
      const long long g = gc + gl;
      rb[set][q] = (idx < VB && g < g_end && c < no2) ? vload<float, VW>(U + g * no2 + c) : vzero<float, VW>();
    }
  };
  auto store = [&](int set) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int gl = idx / (2 * BM / VW), c = (idx % (2 * BM / VW)) * VW;
        *reinterpret_cast<Vec<float, VW>*>(&sA[set][gl * LA + c]) = ra[set][q];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (2 * BNC / VW), c = (idx % (2 * BNC / VW)) * VW;
        *reinterpret_cast<Vec<float, VW>*>(&sB[set][gl * LB + c]) = rb[set][q];
      }
    }
  };
  auto compute = [&](int b) {
#pragma unroll
    for (int ks = 0; ks < KG / 4; ++ks) {
      const int gl = 4 * ks + lk;
      const float2 v = *reinterpret_cast<const float2*>(&sA[b][gl * LA + 2 * (wm0 + ll)]);
      const float a1 = v.x - v.y, a2 = v.x, a3 = -v.y;   // conj(B): b' = -Im B
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const float2 w = *reinterpret_cast<const float2*>(&sB[b][gl * LB + 2 * (j * 16 + ll)]);
        k1[j] = Mfma<float>::run(a1, w.x, k1[j]);
        k2[j] = Mfma<float>::run(a2, w.y - w.x, k2[j]);
        k3[j] = Mfma<float>::run(a3, w.x + w.y, k3[j]);
      }
    }
  };
  // stage st: registers and LDS buffer st % 2 (as in k_correct3m_n)
  const int n_st = (int)((g_end - g_begin + KG - 1) / KG);
  load(0, g_begin);
  if (n_st > 1) load(1, g_begin + KG);
  for (int st = 0; st < n_st; st += 2) {
    store(0);
    lds_barrier();
    if (st + 2 < n_st) load(0, g_begin + (long long)(st + 2) * KG);
    if (active) compute(0);
    if (st + 1 >= n_st) break;
    store(1);
    lds_barrier();
    if (st + 3 < n_st) load(1, g_begin + (long long)(st + 3) * KG);
    if (active) compute(1);
  }
  if (!active) return;
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = p0 + wm0 + 4 * lk + r;
      const int n = j * 16 + ll;
      if (p < np && n < no)
        *reinterpret_cast<float2*>(&part[(long long)p * no2 + 2 * n]) =
            make_float2(k1[j][r] - k3[j][r], k1[j][r] + k2[j][r]);
    }
}

}  // namespace dcm


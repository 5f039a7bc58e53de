// Split-precision projector products (the hi+lo BF16 / FP16 modes of
// Sec. VI.C, here with two terms per operand): every FP32 operand value x is
// written as hi + lo with hi = round16(x) and lo = round16(x - hi), and each
// real product is accumulated in FP32 as hi*hi + hi*lo + lo*hi on the 16-bit
// matrix cores (v_mfma_f32_16x16x32_{bf16,f16}).  FP16 operands are first
// scaled by a power of two 2^s chosen from the operand's largest magnitude
// (max |x| 2^s in [2^14, 2^15)) so both terms stay in FP16 range; the sums are
// scaled back by 2^-(s_a + s_b).
//
// Operand storage (all 16-bit, hi and lo in separate planes, rows padded with
// zeros to a multiple of 8 halves so every tile row moves as 16-byte loads):
//   Bs[g][k]   k = 2p + c : the projectors as stored (correction, A operand)
//   Bt[p][k]   k = 2g + c : transposed (projection, A operand)
//   Qt[j][k]   k = 2p + c : transposed real form of coef D P (correction, B operand)
// and the projection's right operand u is split while it is staged into LDS.
// MFMA 16x16x32 lane layout: operand lane l holds row/column l % 16 and the 8
// consecutive reduction indices 8 (l / 16) .. 8 (l / 16) + 7; accumulator lane
// l holds column l % 16, rows 4 (l / 16) + i.
#pragma once

#include "common.hpp"
#include "gemm.hpp"

namespace dcm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int MODE> struct Half;
template <> struct Half<0> {   // BF16
  using T = __bf16;
  using V8 = bf16x8;
  __device__ __forceinline__ static f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Half<1> {   // FP16
  using T = _Float16;
  using V8 = f16x8;
  __device__ __forceinline__ static f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Two adjacent 16-bit values moved as one 4-byte store.
template <typename T> struct alignas(4) Pair { T a, b; };

// hi/lo of x * 2^s (s = 0 for BF16)
template <int MODE>
__device__ __forceinline__ void split2(float x, float scale, typename Half<MODE>::T& hi, typename Half<MODE>::T& lo) {
  using T = typename Half<MODE>::T;
  const float xs = x * scale;
  hi = (T)xs;
  lo = (T)(xs - (float)hi);
}

// Power-of-two scale from the bits of a max |x| (FP16 mode): s = 15 - e with
// max = m 2^e, m in [0.5, 1).  Returns 2^s; 1 when max is 0.
__device__ __forceinline__ float fp16_scale_from_bits(unsigned bits) {
  const float m = __uint_as_float(bits);
  if (m == 0.0f) return 1.0f;
  int e;
  (void)frexpf(m, &e);
  return ldexpf(1.0f, 15 - e);
}

// max |x| over a real array of n values into *bits (atomic max on the float
// bits, exact and order independent).  Items: (dom, block of kBlock kAbsPer
// values); which: 0 = B, 1 = slot u.  A block whose max does not exceed the
// value already stored skips its atomic, so the thousands of blocks of a
// large array do not queue on one address.
constexpr int kAbsPer = 64;
__global__ __launch_bounds__(kBlock) void k_absmax(const DomDesc* __restrict__ doms, const Item* __restrict__ items,
                                                   int which, int u_slot) {
  __shared__ float red[kBlock / kWave];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const DCM_GLOBAL float* x = which == 0 ? (const DCM_GLOBAL float*)D.proj : (const DCM_GLOBAL float*)D.slot[u_slot];
  const long long n = which == 0 ? D.n_grid * 2 * D.n_proj : D.n_grid * 2 * D.n_orb;
  const long long base = (long long)it.a * kBlock * kAbsPer;
  float m = 0.f;
  if ((reinterpret_cast<uintptr_t>(x) & 15) == 0 && base + kBlock * kAbsPer <= n) {
    const DCM_GLOBAL float4* x4 = (const DCM_GLOBAL float4*)(x + base);
#pragma unroll
    for (int i = 0; i < kAbsPer / 4; ++i) {
      const float4 v = x4[i * kBlock + threadIdx.x];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  } else {
    for (int i = 0; i < kAbsPer; ++i) {
      const long long e = base + (long long)i * kBlock + threadIdx.x;
      if (e < n) m = fmaxf(m, fabsf(x[e]));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = red[0];
    for (int w = 1; w < kBlock / kWave; ++w) b = fmaxf(b, red[w]);
    unsigned* dst = &D.maxbits[which == 0 ? 0 : 1];
    const unsigned bits = __float_as_uint(b);
    if (bits > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, bits);
  }
}

// Clears maxbits[which] of every domain.  Items: one per domain.
__global__ void k_zero_maxbits(const DomDesc* __restrict__ doms, const Item* __restrict__ items, int n_items,
                               int which) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_items) {
    unsigned* m = doms[items[i].dom].maxbits;
    if (m) m[which] = 0u;
  }
}

// Pre-split of the projectors: Bs (natural layout) and Bt (transposed), hi and
// lo, including the zero padding of both.  Items: (dom, 32-row g tile, 32-column
// p tile); the tiles cover the padded extents.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_presplit(const DomDesc* __restrict__ doms, const Item* __restrict__ items) {
  using T = typename Half<MODE>::T;
  __shared__ float tile[32][65];     // 32 g x (32 p x re/im)
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, k2 = 2 * np;
  const long long g0 = (long long)it.a * 32;
  const int p0 = it.b * 32;
  const float scale = MODE == 1 ? fp16_scale_from_bits(D.maxbits[0]) : 1.0f;
  const float* B = (const float*)D.proj;
  for (int idx = threadIdx.x; idx < 32 * 64; idx += kBlock) {
    const int r = idx / 64, c = idx % 64;
    const long long g = g0 + r;
    const int k = 2 * p0 + c;
    float v = 0.f;
    if (g < D.n_grid && k < k2) v = B[g * k2 + k];
    if (g < D.n_grid && k < D.ldbs) {
      T hi, lo;
      split2<MODE>(v, scale, hi, lo);
      ((T*)D.bs_hi)[g * D.ldbs + k] = hi;
      ((T*)D.bs_lo)[g * D.ldbs + k] = lo;
    }
    tile[r][c] = v;
  }
  __syncthreads();
  // transposed: Bt[p][2g + c]; the last g tile also clears the row padding
  for (int idx = threadIdx.x; idx < 32 * 64; idx += kBlock) {
    const int pr = idx / 64, q = idx % 64;      // q = 2 * g_local + c
    const int p = p0 + pr;
    const long long k = 2 * g0 + q;
    if (p < np && k < D.ldbt) {
      T hi, lo;
      split2<MODE>(tile[q / 2][2 * pr + q % 2], scale, hi, lo);   // zero past N_g
      ((T*)D.bt_hi)[(long long)p * D.ldbt + k] = hi;
      ((T*)D.bt_lo)[(long long)p * D.ldbt + k] = lo;
    }
  }
}

// Projection partials: part[s][p][j] = sum over the split's grid points of the
// real-form product, from Bt (16-bit, pre-split) and u (FP32, split here).
// Items: (dom, p tile, j tile, split).  KG grid points (2 KG reduction indices)
// per LDS stage; 2 KG must be a multiple of 32.  Global tiles are prefetched
// into registers one stage ahead.
template <int MODE, int BM, int BN, int KG>
__global__ __launch_bounds__(kBlock) void k_project_split(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items, int u_slot) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int KK = 2 * KG;                 // reduction indices per stage
  constexpr int LK = KK + 8;                 // padded row (halves)
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int VA = BM * KK / 8;            // 16-byte vectors per plane of the A tile
  constexpr int RA = (VA + kBlock - 1) / kBlock;
  constexpr int VB = KG * BN / 2;            // complex values of the u tile
  constexpr int RB = (VB + kBlock - 1) / kBlock;
  static_assert(KK % 32 == 0, "stage must hold whole MFMA steps");
  __shared__ __align__(16) T sAh[BM * LK];
  __shared__ __align__(16) T sAl[BM * LK];
  __shared__ __align__(16) T sBh[BN * LK];
  __shared__ __align__(16) T sBl[BN * LK];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no2 = 2 * D.n_orb;
  const long long ldbt = D.ldbt;
  const int p0 = it.a * BM, j0 = it.b * BN;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);
  const float2* __restrict__ U = (const float2*)D.slot[u_slot];
  const T* __restrict__ bth = (const T*)D.bt_hi;
  const T* __restrict__ btl = (const T*)D.bt_lo;
  const float su = MODE == 1 ? fp16_scale_from_bits(D.maxbits[1]) : 1.0f;
  const float sbs = MODE == 1 ? fp16_scale_from_bits(D.maxbits[0]) : 1.0f;

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BM / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  V8 rah[RA], ral[RA];
  float2 rb[RB];
  const V8 z8 = {};
  auto load = [&](long long gc) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KK / 8), c = (idx % (KK / 8)) * 8;
      const int p = p0 + r;
      const long long k = 2 * gc + c;
      const bool ok = idx < VA && p < np && k < 2 * g_end;   // rows are zero padded to ldbt
      rah[q] = ok ? *(const V8*)(bth + (long long)p * ldbt + k) : z8;
      ral[q] = ok ? *(const V8*)(btl + (long long)p * ldbt + k) : z8;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (BN / 2), nn = idx % (BN / 2);
      const long long g = gc + gl;
      const int j = j0 + 2 * nn;
      rb[q] = (idx < VB && g < g_end && j < no2) ? U[g * (no2 / 2) + j / 2] : make_float2(0.f, 0.f);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (KK / 8), c = (idx % (KK / 8)) * 8;
        *(V8*)&sAh[r * LK + c] = rah[q];
        *(V8*)&sAl[r * LK + c] = ral[q];
      }
    }
    // column j, k = 2 g_local + c: c = 0 -> u[g][j]; c = 1 -> (j even: u[g][j+1], j odd: -u[g][j-1]);
    // the two reduction indices of a grid point are adjacent, so each column
    // receives one 4-byte pair per plane
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (BN / 2), nn = idx % (BN / 2);
        T rh, rl, ih, il;
        split2<MODE>(rb[q].x, su, rh, rl);
        split2<MODE>(rb[q].y, su, ih, il);
        const T nrh = (T)(-(float)rh), nrl = (T)(-(float)rl);
        const int c0 = (2 * nn) * LK + 2 * gl, c1 = (2 * nn + 1) * LK + 2 * gl;
        *(Pair<T>*)&sBh[c0] = Pair<T>{rh, ih};
        *(Pair<T>*)&sBh[c1] = Pair<T>{ih, nrh};
        *(Pair<T>*)&sBl[c0] = Pair<T>{rl, il};
        *(Pair<T>*)&sBl[c1] = Pair<T>{il, nrl};
      }
    }
  };

  load(g_begin);
  for (long long gc = g_begin; gc < g_end; gc += KG) {
    store();
    __syncthreads();
    if (gc + KG < g_end) load(gc + KG);
#pragma unroll
    for (int ks = 0; ks < KK / 32; ++ks) {
      V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = (wm0 + i * 16 + ll) * LK + ks * 32 + 8 * lk;
        ah[i] = *(const V8*)&sAh[o];
        al[i] = *(const V8*)&sAl[o];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = (wn0 + j * 16 + ll) * LK + ks * 32 + 8 * lk;
        bh[j] = *(const V8*)&sBh[o];
        bl[j] = *(const V8*)&sBl[o];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
          acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
          acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
        }
    }
    __syncthreads();
  }
  const float unscale = 1.0f / (su * sbs);
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (p < np && jj < no2) part[(long long)p * no2 + jj] = acc[i][j][r] * unscale;
      }
}

// Q'^T hi/lo (rows of ldqt halves, zero padded) from the FP32 real form Q'
// written by k_reduce.  FP16 mode uses the max of |Q'| gathered with an atomic
// by the same k_reduce launch.  Items: (dom, block over 2 n_orb x ldqt entries).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_split_q(const DomDesc* __restrict__ doms, const Item* __restrict__ items) {
  using T = typename Half<MODE>::T;
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int k2 = 2 * D.n_proj, no2 = 2 * D.n_orb;
  const long long ldqt = D.ldqt;
  const long long idx = (long long)it.a * kBlock + threadIdx.x;
  if (idx >= (long long)no2 * ldqt) return;
  const int j = (int)(idx / ldqt), k = (int)(idx % ldqt);
  const float scale = MODE == 1 ? fp16_scale_from_bits(D.maxbits[2]) : 1.0f;
  const float v = k < k2 ? ((const float*)D.qmat)[(long long)k * D.ldq + j] : 0.f;
  T hi, lo;
  split2<MODE>(v, scale, hi, lo);
  ((T*)D.qt_hi)[idx] = hi;
  ((T*)D.qt_lo)[idx] = lo;
}

// FP16 mode: the max |x| of the values a wave has written into maxbits[1],
// the scale source of the next projection, whose input they are (an atomic max
// on the float bits, skipped where the stored value is already as large).
// Every lane of the wave calls it.
__device__ __forceinline__ void wave_umax(const DomDesc& D, float m) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) {
    unsigned* dst = &D.maxbits[1];
    const unsigned bits = __float_as_uint(m);
    if (bits > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, bits);
  }
}

// out[g][j] += sum_k Bs[g][k] Qt[j][k] (hi*hi + hi*lo + lo*hi), unscaled.
// Items: (dom, g tile, j tile).  KC reduction indices per LDS stage.
template <int MODE, int BMG, int BN, int KC>
__global__ __launch_bounds__(kBlock) void k_correct_split(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items, int out_slot, int umax) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int LK = KC + 8;
  constexpr int TM = BMG / 32, TN = BN / 32;
  constexpr int VA = BMG * KC / 8, VB = BN * KC / 8;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  static_assert(KC % 32 == 0, "stage must hold whole MFMA steps");
  __shared__ __align__(16) T sAh[BMG * LK];
  __shared__ __align__(16) T sAl[BMG * LK];
  __shared__ __align__(16) T sBh[BN * LK];
  __shared__ __align__(16) T sBl[BN * LK];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long ldbs = D.ldbs, ldqt = D.ldqt;
  const int no2 = 2 * D.n_orb;
  const long long g0 = (long long)it.a * BMG;
  const int j0 = it.b * BN;
  const T* __restrict__ ah_g = (const T*)D.bs_hi;
  const T* __restrict__ al_g = (const T*)D.bs_lo;
  const T* __restrict__ bh_g = (const T*)D.qt_hi;
  const T* __restrict__ bl_g = (const T*)D.qt_lo;
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int wm0 = (wv / 2) * (BMG / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  V8 rah[RA], ral[RA], rbh[RB], rbl[RB];
  const V8 z8 = {};
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
      const long long g = g0 + r;
      const int k = k0 + c;
      const bool ok = idx < VA && g < D.n_grid && k < ldbs;
      rah[q] = ok ? *(const V8*)(ah_g + g * ldbs + k) : z8;
      ral[q] = ok ? *(const V8*)(al_g + g * ldbs + k) : z8;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
      const int j = j0 + r, k = k0 + c;
      const bool ok = idx < VB && j < no2 && k < ldqt;
      rbh[q] = ok ? *(const V8*)(bh_g + (long long)j * ldqt + k) : z8;
      rbl[q] = ok ? *(const V8*)(bl_g + (long long)j * ldqt + k) : z8;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
        *(V8*)&sAh[r * LK + c] = rah[q];
        *(V8*)&sAl[r * LK + c] = ral[q];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
        *(V8*)&sBh[r * LK + c] = rbh[q];
        *(V8*)&sBl[r * LK + c] = rbl[q];
      }
    }
  };

  const int K = (int)ldbs;   // zero padded: the padding contributes nothing
  load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
    store();
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = (wm0 + i * 16 + ll) * LK + ks * 32 + 8 * lk;
        ah[i] = *(const V8*)&sAh[o];
        al[i] = *(const V8*)&sAl[o];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = (wn0 + j * 16 + ll) * LK + ks * 32 + 8 * lk;
        bh[j] = *(const V8*)&sBh[o];
        bl[j] = *(const V8*)&sBl[o];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
          acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
          acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
        }
    }
    __syncthreads();
  }
  const float unscale = MODE == 1 ? 1.0f / (fp16_scale_from_bits(D.maxbits[0]) * fp16_scale_from_bits(D.maxbits[2]))
                                  : 1.0f;
  // out += acc: every read is issued before the first write, so the reads
  // overlap instead of each waiting behind the previous write
  float prev[TM][TN][4];
  float vmax = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        prev[i][j][r] = (g < D.n_grid && jj < no2) ? out[g * no2 + jj] : 0.f;
      }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && jj < no2) {
          const float v = prev[i][j][r] + acc[i][j][r] * unscale;
          out[g * no2 + jj] = v;
          vmax = fmaxf(vmax, fabsf(v));
        }
      }
  if (MODE == 1 && umax) wave_umax(D, vmax);
}

// The split correction with both pre-split operands moved from memory
// straight into LDS (buffer loads with an LDS destination), double-buffered
// (one barrier per stage).  A stage covers 32 reduction indices: every row of
// Bs and Qt contributes 64 B per plane, four 16-byte chunks.  One wave
// instruction moves 16 rows; within a row, chunk c sits in slot c ^ ((r / 2) % 4)
// so that the 16-byte fragment reads of eight consecutive rows fall on
// distinct LDS banks.  The row length ldbs is a multiple of 32 halves (zero
// padded), so no stage runs past it; rows past the grid or past 2 n_orb read
// as zero and reach only outputs that are not stored.
template <int MODE, int BMG, int BN>
__global__ __launch_bounds__(kBlock) void k_correct_split_dl(const DomDesc* __restrict__ doms,
                                                             const Item* __restrict__ items, int out_slot, int umax) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int KC = 32;
  constexpr int TM = BMG / 32, TN = BN / 32;
  constexpr int SA = BMG * KC, SB = BN * KC;
  static_assert(BMG % 64 == 0 && BN % 64 == 0, "whole instructions per wave");
  __shared__ __align__(16) T sA0h[SA], sA0l[SA], sA1h[SA], sA1l[SA];
  __shared__ __align__(16) T sB0h[SB], sB0l[SB], sB1h[SB], sB1l[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long ldbs = D.ldbs, ldqt = D.ldqt;
  const int no2 = 2 * D.n_orb;
  const long long g0 = (long long)it.a * BMG;
  const int j0 = it.b * BN;
  const unsigned rowA = 2u * (unsigned)ldbs, rowB = 2u * (unsigned)ldqt;     // bytes per row
  const unsigned nA = (unsigned)min((long long)BMG, D.n_grid - g0), nB = (unsigned)min(BN, no2 - j0);
  const __amdgpu_buffer_rsrc_t rah = buffer_over((const DCM_GLOBAL char*)D.bs_hi + g0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t ral = buffer_over((const DCM_GLOBAL char*)D.bs_lo + g0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t rbh = buffer_over((const DCM_GLOBAL char*)D.qt_hi + (long long)j0 * rowB, nB * rowB);
  const __amdgpu_buffer_rsrc_t rbl = buffer_over((const DCM_GLOBAL char*)D.qt_lo + (long long)j0 * rowB, nB * rowB);
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 2) * (BMG / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  // this lane's row within an instruction's 16 rows and the chunk it moves
  const int lr = lane / 4;
  const unsigned lchunk = (unsigned)((lane % 4) ^ ((lr >> 1) & 3));
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  auto issue = [&](int st, T* ah, T* al, T* bh, T* bl) {
    const unsigned kb = (unsigned)st * (2u * KC) + 16u * lchunk;            // byte offset in the row
#pragma unroll
    for (int r0 = wv * 16; r0 < BMG; r0 += 64) {
      const unsigned off = (unsigned)(r0 + lr) * rowA + kb;
      load_lds16(rah, (float*)(ah + r0 * KC), off);
      load_lds16(ral, (float*)(al + r0 * KC), off);
    }
#pragma unroll
    for (int r0 = wv * 16; r0 < BN; r0 += 64) {
      const unsigned off = (unsigned)(r0 + lr) * rowB + kb;
      load_lds16(rbh, (float*)(bh + r0 * KC), off);
      load_lds16(rbl, (float*)(bl + r0 * KC), off);
    }
  };
  auto frag = [&](const T* s, int r) -> V8 {
    return *(const V8*)&s[r * KC + 8 * (lk ^ ((r >> 1) & 3))];
  };
  auto compute = [&](const T* ah_s, const T* al_s, const T* bh_s, const T* bl_s) {
    V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      ah[i] = frag(ah_s, wm0 + i * 16 + ll);
      al[i] = frag(al_s, wm0 + i * 16 + ll);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      bh[j] = frag(bh_s, wn0 + j * 16 + ll);
      bl[j] = frag(bl_s, wn0 + j * 16 + ll);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
      }
  };
  const int n_st = (int)(ldbs / KC);
  if (n_st > 0) issue(0, sA0h, sA0l, sB0h, sB0l);
  int st = 0;
  for (; st + 1 < n_st; st += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    issue(st + 1, sA1h, sA1l, sB1h, sB1l);
    compute(sA0h, sA0l, sB0h, sB0l);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (st + 2 < n_st) issue(st + 2, sA0h, sA0l, sB0h, sB0l);
    compute(sA1h, sA1l, sB1h, sB1l);
  }
  if (st < n_st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    compute(sA0h, sA0l, sB0h, sB0l);
  }
  const float unscale = MODE == 1 ? 1.0f / (fp16_scale_from_bits(D.maxbits[0]) * fp16_scale_from_bits(D.maxbits[2]))
                                  : 1.0f;
  // out += acc, one 16-row tile at a time (reads before writes)
  float vmax = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float prev[TN][4];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        prev[j][r] = (g < D.n_grid && jj < no2) ? out[g * no2 + jj] : 0.f;
      }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && jj < no2) {
          const float v = prev[j][r] + acc[i][j][r] * unscale;
          out[g * no2 + jj] = v;
          vmax = fmaxf(vmax, fabsf(v));
        }
      }
  }
  if (MODE == 1 && umax) wave_umax(D, vmax);
}

// The split correction on eight waves with a three-deep ring of LDS stages:
// the Bs rows of a stage are requested two stages ahead (straight into LDS),
// which hides the memory latency that one stage of compute cannot; the small
// Qt tile comes from L2 one stage ahead through registers.  A 128 x 256 tile
// (waves 2 x 4, each 64 x 64); per stage every wave moves one 16-row group of
// each Bs plane.  Layout, swizzle and zero fill as k_correct_split_dl.  512
// threads.
constexpr int kBlockCorr3 = 512;
template <int MODE>
__global__ __launch_bounds__(kBlockCorr3) void k_correct_split_dl3(const DomDesc* __restrict__ doms,
                                                                   const Item* __restrict__ items, int out_slot, int umax) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int BMG = 128, BN = 256, KC = 32, NW = kBlockCorr3 / kWave;
  constexpr int TM = 4, TN = 4;
  constexpr int SA = BMG * KC, SB = BN * KC;
  __shared__ __align__(16) T sA0h[SA], sA0l[SA], sA1h[SA], sA1l[SA], sA2h[SA], sA2l[SA];
  __shared__ __align__(16) T sB0h[SB], sB0l[SB], sB1h[SB], sB1l[SB], sB2h[SB], sB2l[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long ldbs = D.ldbs, ldqt = D.ldqt;
  const int no2 = 2 * D.n_orb;
  const long long g0 = (long long)it.a * BMG;
  const int j0 = it.b * BN;
  const unsigned rowA = 2u * (unsigned)ldbs, rowB = 2u * (unsigned)ldqt;     // bytes per row
  const unsigned nA = (unsigned)min((long long)BMG, D.n_grid - g0), nB = (unsigned)min(BN, no2 - j0);
  const __amdgpu_buffer_rsrc_t rah = buffer_over((const DCM_GLOBAL char*)D.bs_hi + g0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t ral = buffer_over((const DCM_GLOBAL char*)D.bs_lo + g0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t rbh = buffer_over((const DCM_GLOBAL char*)D.qt_hi + (long long)j0 * rowB, nB * rowB);
  const __amdgpu_buffer_rsrc_t rbl = buffer_over((const DCM_GLOBAL char*)D.qt_lo + (long long)j0 * rowB, nB * rowB);
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 4) * 64, wn0 = (wv % 4) * 64;
  const int ll = lane % 16, lk = lane / 16;
  const int lr = lane / 4;
  const unsigned lchunk = (unsigned)((lane % 4) ^ ((lr >> 1) & 3));
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  // Qt tile rows through registers (it sits in L2): 4 x 16 bytes per thread
  // per stage, stored into LDS swizzled like the Bs rows
  const DCM_GLOBAL T* qh = (const DCM_GLOBAL T*)D.qt_hi + (long long)j0 * ldqt;
  const DCM_GLOBAL T* ql = (const DCM_GLOBAL T*)D.qt_lo + (long long)j0 * ldqt;
  V8 rq[4];
  const V8 z8 = {};
  auto load_b = [&](int st) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = (q % 2) * kBlockCorr3 + threadIdx.x;
      const int row = idx / 4, ch = idx % 4;
      // rows past the tile read the last valid row; store_b zeroes them
      const int rr = min(row, (int)nB - 1);
      rq[q] = *(const DCM_GLOBAL V8*)((q < 2 ? qh : ql) + (long long)rr * ldqt + st * KC + 8 * ch);
    }
  };
  auto store_b = [&](T* bh, T* bl) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = (q % 2) * kBlockCorr3 + threadIdx.x;
      const int row = idx / 4, ch = idx % 4;
      *(V8*)&(q < 2 ? bh : bl)[row * KC + 8 * (ch ^ ((row >> 1) & 3))] = row < (int)nB ? rq[q] : z8;
    }
  };
  auto issue_a = [&](int st, T* ah, T* al) {
    const unsigned kb = (unsigned)st * (2u * KC) + 16u * lchunk;
    const int ra = wv * 16;
    const unsigned oa = (unsigned)(ra + lr) * rowA + kb;
    load_lds16(rah, (float*)(ah + ra * KC), oa);
    load_lds16(ral, (float*)(al + ra * KC), oa);
  };
  auto frag = [&](const T* s, int r) -> V8 {
    return *(const V8*)&s[r * KC + 8 * (lk ^ ((r >> 1) & 3))];
  };
  auto compute = [&](const T* ah_s, const T* al_s, const T* bh_s, const T* bl_s) {
    V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      ah[i] = frag(ah_s, wm0 + i * 16 + ll);
      al[i] = frag(al_s, wm0 + i * 16 + ll);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      bh[j] = frag(bh_s, wn0 + j * 16 + ll);
      bl[j] = frag(bl_s, wn0 + j * 16 + ll);
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
      }
  };
  // Stage st: its Bs part was requested two stages earlier (the only load
  // that may still be in flight is the one of stage st + 1: two per wave) and
  // its Qt part was stored by this wave at the end of stage st - 1.  After
  // the barrier: request Qt of st + 1 and Bs of st + 2 (into the buffer that
  // stage st - 1 read), multiply, store Qt of st + 1.  The barrier is the
  // bare instruction between two compiler memory clobbers: a workgroup fence
  // would wait for every load in flight.
  const int n_st = (int)(ldbs / KC);    // >= 1: the kernel runs only where n_proj > 0
  issue_a(0, sA0h, sA0l);
  load_b(0);
  if (n_st > 1) issue_a(1, sA1h, sA1l);
  store_b(sB0h, sB0l);
#define DCM_SYNC(MORE)                                                              \
  do {                                                                              \
    if (MORE)                                                                       \
      __builtin_amdgcn_s_waitcnt(0x0072);   /* vmcnt(2) lgkmcnt(0) */               \
    else                                                                            \
      __builtin_amdgcn_s_waitcnt(0x0070);   /* vmcnt(0) lgkmcnt(0) */               \
    asm volatile("" ::: "memory");                                                  \
    __builtin_amdgcn_s_barrier();                                                   \
    asm volatile("" ::: "memory");                                                  \
  } while (0)
#define DCM_STAGE_FULL(ST, C, N, NB)                                                \
  do {                                                                              \
    DCM_SYNC(true);                                                                 \
    load_b((ST) + 1);                                                               \
    __builtin_amdgcn_sched_barrier(0);   /* Qt loads retire before the Bs ones */   \
    issue_a((ST) + 2, sA##N##h, sA##N##l);                                          \
    compute(sA##C##h, sA##C##l, sB##C##h, sB##C##l);                                \
    __builtin_amdgcn_sched_barrier(0);                                              \
    store_b(sB##NB##h, sB##NB##l);                                                  \
  } while (0)
#define DCM_STAGE_TAIL(ST, C, N, NB)                                                \
  do {                                                                              \
    DCM_SYNC((ST) + 1 < n_st);                                                      \
    if ((ST) + 1 < n_st) load_b((ST) + 1);                                          \
    __builtin_amdgcn_sched_barrier(0);                                              \
    if ((ST) + 2 < n_st) issue_a((ST) + 2, sA##N##h, sA##N##l);                     \
    compute(sA##C##h, sA##C##l, sB##C##h, sB##C##l);                                \
    __builtin_amdgcn_sched_barrier(0);                                              \
    if ((ST) + 1 < n_st) store_b(sB##NB##h, sB##NB##l);                             \
  } while (0)
  int st = 0;
  for (; st + 4 < n_st; st += 3) {
    DCM_STAGE_FULL(st, 0, 2, 1);
    DCM_STAGE_FULL(st + 1, 1, 0, 2);
    DCM_STAGE_FULL(st + 2, 2, 1, 0);
  }
  if (st < n_st) DCM_STAGE_TAIL(st, 0, 2, 1);
  if (st + 1 < n_st) DCM_STAGE_TAIL(st + 1, 1, 0, 2);
  if (st + 2 < n_st) DCM_STAGE_TAIL(st + 2, 2, 1, 0);
  if (st + 3 < n_st) DCM_STAGE_TAIL(st + 3, 0, 2, 1);
#undef DCM_STAGE_FULL
#undef DCM_STAGE_TAIL
#undef DCM_SYNC
  const float unscale = MODE == 1 ? 1.0f / (fp16_scale_from_bits(D.maxbits[0]) * fp16_scale_from_bits(D.maxbits[2]))
                                  : 1.0f;
  float vmax = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    float prev[TN][4];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        prev[j][r] = (g < D.n_grid && jj < no2) ? out[g * no2 + jj] : 0.f;
      }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long g = g0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (g < D.n_grid && jj < no2) {
          const float v = prev[j][r] + acc[i][j][r] * unscale;
          out[g * no2 + jj] = v;
          vmax = fmaxf(vmax, fabsf(v));
        }
      }
  }
  if (MODE == 1 && umax) wave_umax(D, vmax);
}

// The split projection with the pre-split projector planes Bt moved from
// memory straight into LDS (buffer loads with an LDS destination, rows of 64 B
// per stage, chunks swizzled as in k_correct_split_dl) and u split on the way
// into LDS as in k_project_split; both tiles double-buffered (one barrier per
// stage).  Reduction indices past the split's last grid point meet a zero u
// tile; rows past n_proj read as zero.  Items as k_project_split.
template <int MODE, int BM, int BN>
__global__ __launch_bounds__(kBlock) void k_project_split_dl(const DomDesc* __restrict__ doms,
                                                             const Item* __restrict__ items, int u_slot) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int KG = 16, KK = 2 * KG;        // grid points and reduction indices per stage
  constexpr int LK = KK + 8;                 // padded u rows (halves)
  constexpr int TM = BM / 32, TN = BN / 32;
  constexpr int VB = KG * BN / 2;
  constexpr int RB = (VB + kBlock - 1) / kBlock;
  constexpr int SA = BM * KK, SB = BN * LK;
  static_assert(BM % 64 == 0, "whole instructions per wave");
  __shared__ __align__(16) T sA0h[SA], sA0l[SA], sA1h[SA], sA1l[SA];
  __shared__ __align__(16) T sB0h[SB], sB0l[SB], sB1h[SB], sB1l[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no2 = 2 * D.n_orb;
  const int p0 = it.a * BM, j0 = it.b * BN;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);
  const int n_st = (int)((g_end - g_begin + KG - 1) / KG);
  const unsigned rowA = 2u * (unsigned)D.ldbt;                           // bytes per Bt row
  const unsigned nA = (unsigned)min(BM, np - p0);
  const long long kb0 = 2 * (2 * g_begin);                                // byte offset of the split in a row
  const __amdgpu_buffer_rsrc_t rah = buffer_over((const DCM_GLOBAL char*)D.bt_hi + (long long)p0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t ral = buffer_over((const DCM_GLOBAL char*)D.bt_lo + (long long)p0 * rowA, nA * rowA);
  const float2* __restrict__ U = (const float2*)D.slot[u_slot];
  const float su = MODE == 1 ? fp16_scale_from_bits(D.maxbits[1]) : 1.0f;
  const float sbs = MODE == 1 ? fp16_scale_from_bits(D.maxbits[0]) : 1.0f;

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 2) * (BM / 2), wn0 = (wv % 2) * (BN / 2);
  const int ll = lane % 16, lk = lane / 16;
  const int lr = lane / 4;
  const unsigned lchunk = (unsigned)((lane % 4) ^ ((lr >> 1) & 3));
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  float2 rb[RB];
  auto issue_a = [&](int st, T* ah, T* al) {
    const unsigned kb = (unsigned)(kb0 + (long long)st * (2 * KK)) + 16u * lchunk;
#pragma unroll
    for (int r0 = wv * 16; r0 < BM; r0 += 64) {
      const unsigned off = (unsigned)(r0 + lr) * rowA + kb;
      load_lds16(rah, (float*)(ah + r0 * KK), off);
      load_lds16(ral, (float*)(al + r0 * KK), off);
    }
  };
  auto load_b = [&](int st) {
    const long long gc = g_begin + (long long)st * KG;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (BN / 2), nn = idx % (BN / 2);
      const long long g = gc + gl;
      const int j = j0 + 2 * nn;
      rb[q] = (idx < VB && g < g_end && j < no2) ? U[g * (no2 / 2) + j / 2] : make_float2(0.f, 0.f);
    }
  };
  auto store_b = [&](T* bh, T* bl) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (BN / 2), nn = idx % (BN / 2);
        T rh, rl, ih, il;
        split2<MODE>(rb[q].x, su, rh, rl);
        split2<MODE>(rb[q].y, su, ih, il);
        const T nrh = (T)(-(float)rh), nrl = (T)(-(float)rl);
        const int c0 = (2 * nn) * LK + 2 * gl, c1 = (2 * nn + 1) * LK + 2 * gl;
        *(Pair<T>*)&bh[c0] = Pair<T>{rh, ih};
        *(Pair<T>*)&bh[c1] = Pair<T>{ih, nrh};
        *(Pair<T>*)&bl[c0] = Pair<T>{rl, il};
        *(Pair<T>*)&bl[c1] = Pair<T>{il, nrl};
      }
    }
  };
  auto compute = [&](const T* ah_s, const T* al_s, const T* bh_s, const T* bl_s) {
    V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm0 + i * 16 + ll;
      const int o = r * KK + 8 * (lk ^ ((r >> 1) & 3));
      ah[i] = *(const V8*)&ah_s[o];
      al[i] = *(const V8*)&al_s[o];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int o = (wn0 + j * 16 + ll) * LK + 8 * lk;
      bh[j] = *(const V8*)&bh_s[o];
      bl[j] = *(const V8*)&bl_s[o];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
      }
  };
  if (n_st > 0) {
    issue_a(0, sA0h, sA0l);
    load_b(0);
  }
  // the scheduling barriers keep the split of the next u tile (which waits
  // for its loads) behind the products of the current one
  int st = 0;
  for (; st + 1 < n_st; st += 2) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    store_b(sB0h, sB0l);
    __syncthreads();
    issue_a(st + 1, sA1h, sA1l);
    load_b(st + 1);
    compute(sA0h, sA0l, sB0h, sB0l);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_b(sB1h, sB1l);
    __syncthreads();
    if (st + 2 < n_st) {
      issue_a(st + 2, sA0h, sA0l);
      load_b(st + 2);
    }
    compute(sA1h, sA1l, sB1h, sB1l);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (st < n_st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    store_b(sB0h, sB0l);
    __syncthreads();
    compute(sA0h, sA0l, sB0h, sB0l);
  }
  const float unscale = 1.0f / (su * sbs);
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (p < np && jj < no2) part[(long long)p * no2 + jj] = acc[i][j][r] * unscale;
      }
}

// The split projection on eight waves with the ring of k_correct_split_dl3:
// the Bt rows of a stage (the large operand) are requested two stages ahead
// straight into a three-deep LDS ring; u comes one stage ahead through
// registers and is split into hi/lo on its way into a two-deep ring (a
// buffer is free once the barrier after its last reader has passed), so the
// loop is unrolled by six.  A 128 x 256 tile (waves 2 x 4, each 64 x 64); a
// stage covers 16 grid points.  Reduction indices past the split meet a zero
// u tile; rows past n_proj read as zero.  Items as k_project_split; 512
// threads.
constexpr int kBlockProj3 = 512;
template <int MODE>
__global__ __launch_bounds__(kBlockProj3) void k_project_split_dl3(const DomDesc* __restrict__ doms,
                                                                   const Item* __restrict__ items, int u_slot) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int BM = 128, BN = 256, KG = 16, KK = 2 * KG, LK = KK + 8;
  constexpr int TM = 4, TN = 4;
  constexpr int SA = BM * KK, SB = BN * LK;
  constexpr int RB = KG * (BN / 2) / kBlockProj3;      // complex values of u per thread and stage
  __shared__ __align__(16) T sA0h[SA], sA0l[SA], sA1h[SA], sA1l[SA], sA2h[SA], sA2l[SA];
  __shared__ __align__(16) T sB0h[SB], sB0l[SB], sB1h[SB], sB1l[SB];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no2 = 2 * D.n_orb, no = D.n_orb;
  const int p0 = it.a * BM, j0 = it.b * BN;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);
  const int n_st = (int)((g_end - g_begin + KG - 1) / KG);              // >= 1
  const unsigned rowA = 2u * (unsigned)D.ldbt;
  const unsigned nA = (unsigned)min(BM, np - p0);
  const long long kb0 = 2 * (2 * g_begin);
  const __amdgpu_buffer_rsrc_t rah = buffer_over((const DCM_GLOBAL char*)D.bt_hi + (long long)p0 * rowA, nA * rowA);
  const __amdgpu_buffer_rsrc_t ral = buffer_over((const DCM_GLOBAL char*)D.bt_lo + (long long)p0 * rowA, nA * rowA);
  const DCM_GLOBAL float2* U = (const DCM_GLOBAL float2*)D.slot[u_slot];
  const float su = MODE == 1 ? fp16_scale_from_bits(D.maxbits[1]) : 1.0f;
  const float sbs = MODE == 1 ? fp16_scale_from_bits(D.maxbits[0]) : 1.0f;

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = (wv / 4) * 64, wn0 = (wv % 4) * 64;
  const int ll = lane % 16, lk = lane / 16;
  const int lr = lane / 4;
  const unsigned lchunk = (unsigned)((lane % 4) ^ ((lr >> 1) & 3));
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};

  // thread -> (grid point gl of the stage, complex column nn of the tile)
  float2 rb[RB];
  auto load_b = [&](int st) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = q * kBlockProj3 + threadIdx.x;
      const int gl = idx / (BN / 2), nn = idx % (BN / 2);
      // out-of-range points and columns load an in-range value; store_b zeroes them
      const long long g = min(g_begin + (long long)st * KG + gl, g_end - 1);
      const int c = min(j0 / 2 + nn, no - 1);
      rb[q] = U[g * no + c];
    }
  };
  auto store_b = [&](int st, T* bh, T* bl) {
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = q * kBlockProj3 + threadIdx.x;
      const int gl = idx / (BN / 2), nn = idx % (BN / 2);
      const bool ok = g_begin + (long long)st * KG + gl < g_end && j0 + 2 * nn < no2;
      const float2 v = ok ? rb[q] : make_float2(0.f, 0.f);
      T rh, rl, ih, il;
      split2<MODE>(v.x, su, rh, rl);
      split2<MODE>(v.y, su, ih, il);
      const T nrh = (T)(-(float)rh), nrl = (T)(-(float)rl);
      const int c0 = (2 * nn) * LK + 2 * gl, c1 = (2 * nn + 1) * LK + 2 * gl;
      *(Pair<T>*)&bh[c0] = Pair<T>{rh, ih};
      *(Pair<T>*)&bh[c1] = Pair<T>{ih, nrh};
      *(Pair<T>*)&bl[c0] = Pair<T>{rl, il};
      *(Pair<T>*)&bl[c1] = Pair<T>{il, nrl};
    }
  };
  auto issue_a = [&](int st, T* ah, T* al) {
    const unsigned kb = (unsigned)(kb0 + (long long)st * (2 * KK)) + 16u * lchunk;
    const int ra = wv * 16;
    const unsigned off = (unsigned)(ra + lr) * rowA + kb;
    load_lds16(rah, (float*)(ah + ra * KK), off);
    load_lds16(ral, (float*)(al + ra * KK), off);
  };
  auto compute = [&](const T* ah_s, const T* al_s, const T* bh_s, const T* bl_s) {
    V8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm0 + i * 16 + ll;
      const int o = r * KK + 8 * (lk ^ ((r >> 1) & 3));
      ah[i] = *(const V8*)&ah_s[o];
      al[i] = *(const V8*)&al_s[o];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int o = (wn0 + j * 16 + ll) * LK + 8 * lk;
      bh[j] = *(const V8*)&bh_s[o];
      bl[j] = *(const V8*)&bl_s[o];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        acc[i][j] = Half<MODE>::mma(ah[i], bh[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(ah[i], bl[j], acc[i][j]);
        acc[i][j] = Half<MODE>::mma(al[i], bh[j], acc[i][j]);
      }
  };
  issue_a(0, sA0h, sA0l);
  load_b(0);
  if (n_st > 1) issue_a(1, sA1h, sA1l);
  store_b(0, sB0h, sB0l);
  // stage ST reads A ring slot CA and B ring slot CB; it requests stage ST + 2
  // into A slot NA and stores stage ST + 1 into B slot NB
#define DCM_SYNC(MORE)                                                              \
  do {                                                                              \
    if (MORE)                                                                       \
      __builtin_amdgcn_s_waitcnt(0x0072);   /* vmcnt(2) lgkmcnt(0) */               \
    else                                                                            \
      __builtin_amdgcn_s_waitcnt(0x0070);   /* vmcnt(0) lgkmcnt(0) */               \
    asm volatile("" ::: "memory");                                                  \
    __builtin_amdgcn_s_barrier();                                                   \
    asm volatile("" ::: "memory");                                                  \
  } while (0)
#define DCM_PSTAGE_FULL(ST, CA, NA, CB, NB)                                         \
  do {                                                                              \
    DCM_SYNC(true);                                                                 \
    load_b((ST) + 1);                                                               \
    __builtin_amdgcn_sched_barrier(0);                                              \
    issue_a((ST) + 2, sA##NA##h, sA##NA##l);                                        \
    compute(sA##CA##h, sA##CA##l, sB##CB##h, sB##CB##l);                            \
    __builtin_amdgcn_sched_barrier(0);                                              \
    store_b((ST) + 1, sB##NB##h, sB##NB##l);                                        \
  } while (0)
#define DCM_PSTAGE_TAIL(ST, CA, NA, CB, NB)                                         \
  do {                                                                              \
    DCM_SYNC((ST) + 1 < n_st);                                                      \
    if ((ST) + 1 < n_st) load_b((ST) + 1);                                          \
    __builtin_amdgcn_sched_barrier(0);                                              \
    if ((ST) + 2 < n_st) issue_a((ST) + 2, sA##NA##h, sA##NA##l);                   \
    compute(sA##CA##h, sA##CA##l, sB##CB##h, sB##CB##l);                            \
    __builtin_amdgcn_sched_barrier(0);                                              \
    if ((ST) + 1 < n_st) store_b((ST) + 1, sB##NB##h, sB##NB##l);                   \
  } while (0)
  int st = 0;
  for (; st + 7 < n_st; st += 6) {
    DCM_PSTAGE_FULL(st, 0, 2, 0, 1);
    DCM_PSTAGE_FULL(st + 1, 1, 0, 1, 0);
    DCM_PSTAGE_FULL(st + 2, 2, 1, 0, 1);
    DCM_PSTAGE_FULL(st + 3, 0, 2, 1, 0);
    DCM_PSTAGE_FULL(st + 4, 1, 0, 0, 1);
    DCM_PSTAGE_FULL(st + 5, 2, 1, 1, 0);
  }
  if (st < n_st) DCM_PSTAGE_TAIL(st, 0, 2, 0, 1);
  if (st + 1 < n_st) DCM_PSTAGE_TAIL(st + 1, 1, 0, 1, 0);
  if (st + 2 < n_st) DCM_PSTAGE_TAIL(st + 2, 2, 1, 0, 1);
  if (st + 3 < n_st) DCM_PSTAGE_TAIL(st + 3, 0, 2, 1, 0);
  if (st + 4 < n_st) DCM_PSTAGE_TAIL(st + 4, 1, 0, 0, 1);
  if (st + 5 < n_st) DCM_PSTAGE_TAIL(st + 5, 2, 1, 1, 0);
  if (st + 6 < n_st) DCM_PSTAGE_TAIL(st + 6, 0, 2, 0, 1);
#undef DCM_PSTAGE_FULL
#undef DCM_PSTAGE_TAIL
#undef DCM_SYNC
  const float unscale = 1.0f / (su * sbs);
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = p0 + wm0 + i * 16 + 4 * lk + r;
        const int jj = j0 + wn0 + j * 16 + ll;
        if (p < np && jj < no2) part[(long long)p * no2 + jj] = acc[i][j][r] * unscale;
      }
}

// ---------------------------------------------------------------------------
// Split products with every orbital of a domain in one block (at most 16 NB
// orbitals, 32 NB real columns), as the FP32 kernels of the same name: four
// waves stacked along the long operand's rows, 16 rows each, every wave over
// all 2 NB 16-column blocks.  Registers are loaded a stage ahead into
// double-buffered LDS, one LDS-only barrier per stage.
// ---------------------------------------------------------------------------

// out[g][j] += sum_k Bs[g][k] Qt[j][k], 64 grid rows per block.  Items: (dom,
// 64-row tile, 0, 0).  KC = 32 reduction indices per stage.
template <int MODE, int NB>
__global__ __launch_bounds__(kBlock) void k_correct_split_n(const DomDesc* __restrict__ doms,
                                                            const Item* __restrict__ items, int out_slot, int umax) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int KC = 32, LK = KC + 8, BMG = 64, BN = 32 * NB, TN = 2 * NB;
  constexpr int VA = BMG * KC / 8, VB = BN * KC / 8;
  constexpr int RA = (VA + kBlock - 1) / kBlock, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) T sAh[2][BMG * LK], sAl[2][BMG * LK];
  __shared__ __align__(16) T sBh[2][BN * LK], sBl[2][BN * LK];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long ldbs = D.ldbs, ldqt = D.ldqt;
  const int no2 = 2 * D.n_orb;
  const long long g0 = (long long)it.a * BMG;
  const T* __restrict__ ah_g = (const T*)D.bs_hi;
  const T* __restrict__ al_g = (const T*)D.bs_lo;
  const T* __restrict__ bh_g = (const T*)D.qt_hi;
  const T* __restrict__ bl_g = (const T*)D.qt_lo;
  float* __restrict__ out = (float*)D.slot[out_slot];

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = wv * 16;
  const int ll = lane % 16, lk = lane / 16;
  f32x4 acc[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) acc[j] = f32x4{0, 0, 0, 0};
  // the output tile, requested before the reduction
  float prev[TN][4];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long g = g0 + wm0 + 4 * lk + r;
      const int jj = j * 16 + ll;
      prev[j][r] = (g < D.n_grid && jj < no2) ? out[g * no2 + jj] : 0.f;
    }

  V8 rah[RA], ral[RA], rbh[RB], rbl[RB];
  const V8 z8 = {};
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
      const long long g = g0 + r;
      const int k = k0 + c;
      const bool ok = idx < VA && g < D.n_grid && k < ldbs;
      rah[q] = ok ? *(const V8*)(ah_g + g * ldbs + k) : z8;
      ral[q] = ok ? *(const V8*)(al_g + g * ldbs + k) : z8;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
      const int k = k0 + c;
      const bool ok = idx < VB && r < no2 && k < ldqt;
      rbh[q] = ok ? *(const V8*)(bh_g + (long long)r * ldqt + k) : z8;
      rbl[q] = ok ? *(const V8*)(bl_g + (long long)r * ldqt + k) : z8;
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
        *(V8*)&sAh[b][r * LK + c] = rah[q];
        *(V8*)&sAl[b][r * LK + c] = ral[q];
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int r = idx / (KC / 8), c = (idx % (KC / 8)) * 8;
        *(V8*)&sBh[b][r * LK + c] = rbh[q];
        *(V8*)&sBl[b][r * LK + c] = rbl[q];
      }
    }
  };
  auto compute = [&](int b) {
    const int oa = (wm0 + ll) * LK + 8 * lk;
    const V8 ah = *(const V8*)&sAh[b][oa], al = *(const V8*)&sAl[b][oa];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int o = (j * 16 + ll) * LK + 8 * lk;
      const V8 bh = *(const V8*)&sBh[b][o], bl = *(const V8*)&sBl[b][o];
      acc[j] = Half<MODE>::mma(ah, bh, acc[j]);
      acc[j] = Half<MODE>::mma(ah, bl, acc[j]);
      acc[j] = Half<MODE>::mma(al, bh, acc[j]);
    }
  };
  // stage st: LDS buffer st % 2, whose last readers (stage st - 2) finished
  // before the barrier of stage st - 1
  const int n_st = (int)(ldbs / KC);   // ldbs: a multiple of 32, zero padded
  load(0);
  for (int st = 0; st < n_st; ++st) {
    store(st & 1);
    lds_barrier();
    if (st + 1 < n_st) load((st + 1) * KC);
    compute(st & 1);
  }
  const float unscale = MODE == 1 ? 1.0f / (fp16_scale_from_bits(D.maxbits[0]) * fp16_scale_from_bits(D.maxbits[2]))
                                  : 1.0f;
  float vmax = 0.f;
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long g = g0 + wm0 + 4 * lk + r;
      const int jj = j * 16 + ll;
      if (g < D.n_grid && jj < no2) {
        const float v = prev[j][r] + acc[j][r] * unscale;
        out[g * no2 + jj] = v;
        vmax = fmaxf(vmax, fabsf(v));
      }
    }
  if (MODE == 1 && umax) wave_umax(D, vmax);
}

// Projection partials from Bt (pre-split) and u (split while staged), 64
// projectors per block.  Items: (dom, 64-projector tile, 0, split).  KG = 16
// grid points (32 reduction indices) per stage.  Waves whose 16 projectors
// lie past n_proj load and synchronise but skip their products.
template <int MODE, int NB>
__global__ __launch_bounds__(kBlock) void k_project_split_n(const DomDesc* __restrict__ doms,
                                                            const Item* __restrict__ items, int u_slot) {
  using T = typename Half<MODE>::T;
  using V8 = typename Half<MODE>::V8;
  constexpr int KG = 16, KK = 2 * KG, LK = KK + 8, BM = 64, BN = 32 * NB, TN = 2 * NB;
  constexpr int VA = BM * KK / 8, RA = (VA + kBlock - 1) / kBlock;
  constexpr int VB = KG * BN / 2, RB = (VB + kBlock - 1) / kBlock;
  __shared__ __align__(16) T sAh[2][BM * LK], sAl[2][BM * LK];
  __shared__ __align__(16) T sBh[2][BN * LK], sBl[2][BN * LK];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int np = D.n_proj, no2 = 2 * D.n_orb;
  const long long ldbt = D.ldbt;
  const int p0 = it.a * BM;
  const long long g_begin = (long long)it.c * D.split_len;
  const long long g_end = min(g_begin + (long long)D.split_len, D.n_grid);
  const float2* __restrict__ U = (const float2*)D.slot[u_slot];
  const T* __restrict__ bth = (const T*)D.bt_hi;
  const T* __restrict__ btl = (const T*)D.bt_lo;
  const float su = MODE == 1 ? fp16_scale_from_bits(D.maxbits[1]) : 1.0f;
  const float sbs = MODE == 1 ? fp16_scale_from_bits(D.maxbits[0]) : 1.0f;

  const int lane = threadIdx.x % kWave, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm0 = wv * 16;
  const bool active = p0 + wm0 < np;      // wave-uniform
  const int ll = lane % 16, lk = lane / 16;
  f32x4 acc[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) acc[j] = f32x4{0, 0, 0, 0};

  V8 rah[RA], ral[RA];
  float2 rb[RB];
  const V8 z8 = {};
  auto load = [&](long long gc) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int r = idx / (KK / 8), c = (idx % (KK / 8)) * 8;
      const int p = p0 + r;
      const long long k = 2 * gc + c;
      const bool ok = idx < VA && p < np && k < 2 * g_end;   // rows are zero padded to ldbt
      rah[q] = ok ? *(const V8*)(bth + (long long)p * ldbt + k) : z8;
      ral[q] = ok ? *(const V8*)(btl + (long long)p * ldbt + k) : z8;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      const int gl = idx / (BN / 2), nn = idx % (BN / 2);
      const long long g = gc + gl;
      rb[q] = (idx < VB && g < g_end && 2 * nn < no2) ? U[g * (no2 / 2) + nn] : make_float2(0.f, 0.f);
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VA) {
        const int r = idx / (KK / 8), c = (idx % (KK / 8)) * 8;
        *(V8*)&sAh[b][r * LK + c] = rah[q];
        *(V8*)&sAl[b][r * LK + c] = ral[q];
      }
    }
    // column j, k = 2 g_local + c: c = 0 -> u[g][j]; c = 1 -> (j even: u[g][j+1],
    // j odd: -u[g][j-1]), one 4-byte pair per plane and column
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int idx = threadIdx.x + q * kBlock;
      if (idx < VB) {
        const int gl = idx / (BN / 2), nn = idx % (BN / 2);
        T rh, rl, ih, il;
        split2<MODE>(rb[q].x, su, rh, rl);
        split2<MODE>(rb[q].y, su, ih, il);
        const T nrh = (T)(-(float)rh), nrl = (T)(-(float)rl);
        const int c0 = (2 * nn) * LK + 2 * gl, c1 = (2 * nn + 1) * LK + 2 * gl;
        *(Pair<T>*)&sBh[b][c0] = Pair<T>{rh, ih};
        *(Pair<T>*)&sBh[b][c1] = Pair<T>{ih, nrh};
        *(Pair<T>*)&sBl[b][c0] = Pair<T>{rl, il};
        *(Pair<T>*)&sBl[b][c1] = Pair<T>{il, nrl};
      }
    }
  };
  auto compute = [&](int b) {
    const int oa = (wm0 + ll) * LK + 8 * lk;
    const V8 ah = *(const V8*)&sAh[b][oa], al = *(const V8*)&sAl[b][oa];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int o = (j * 16 + ll) * LK + 8 * lk;
      const V8 bh = *(const V8*)&sBh[b][o], bl = *(const V8*)&sBl[b][o];
      acc[j] = Half<MODE>::mma(ah, bh, acc[j]);
      acc[j] = Half<MODE>::mma(ah, bl, acc[j]);
      acc[j] = Half<MODE>::mma(al, bh, acc[j]);
    }
  };
  const int n_st = (int)((g_end - g_begin + KG - 1) / KG);
  load(g_begin);
  for (int st = 0; st < n_st; ++st) {
    store(st & 1);
    lds_barrier();
    if (st + 1 < n_st) load(g_begin + (long long)(st + 1) * KG);
    if (active) compute(st & 1);
  }
  if (!active) return;
  const float unscale = 1.0f / (su * sbs);
  float* __restrict__ part = (float*)D.ppart + (long long)it.c * np * no2;
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = p0 + wm0 + 4 * lk + r;
      const int jj = j * 16 + ll;
      if (p < np && jj < no2) part[(long long)p * no2 + jj] = acc[j][r] * unscale;
    }
}

}  // namespace dcm


// Reductions over orbitals and over the grid: density and local current,
// energy finalisation, the gradient inner products of the adjoint step, and
// small elementwise helpers.  Orbital reductions give one wave per grid point
// (lanes over orbitals, wave shuffles to combine); grid reductions write one
// FP64 partial per block and are finished in a fixed order, so every result is
// bitwise reproducible.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace dcm {

// rho = sum_n f_n |psi_n|^2, j_d = sum_n f_n [Im(conj psi_n D1_d psi_n) + A_d |psi_n|^2].
// Items: (dom, block of 4 grid points).  step: A sample; obs: output row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_density(const DomDesc* __restrict__ doms,
                                                    const Item* __restrict__ items, int step, int obs) {
  using C = Cplx<T>;
  __shared__ double red[kBlock / kWave];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long g = (long long)it.a * 4 + threadIdx.x / kWave;
  const bool valid = g < D.n_grid;
  const int lane = threadIdx.x % kWave;
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb, r = D.r;
  const int x = (int)(g % nx), y = (int)((g / nx) % ny), z = (int)(g / ((long long)nx * ny));
  const C* __restrict__ psi = (const C*)D.slot[SLOT_PSI];
  const T* __restrict__ occ = (const T*)D.occ;
  const double ih = 1.0 / D.h;
  double rho = 0, j0 = 0, j1 = 0, j2 = 0;
  for (int n = lane; valid && n < no; n += kWave) {
    const double f = (double)occ[n];
    const C c = psi[g * no + n];
    rho += f * ((double)c.re * c.re + (double)c.im * c.im);
    double jd[3] = {0, 0, 0};
    for (int m = 1; m <= r; ++m) {
      const double am = fd1(r, m) * ih;
      const long long gxp = ((long long)z * ny + y) * nx + wrap(x + m, nx);
      const long long gxm = ((long long)z * ny + y) * nx + wrap(x - m, nx);
      const long long gyp = ((long long)z * ny + wrap(y + m, ny)) * nx + x;
      const long long gym = ((long long)z * ny + wrap(y - m, ny)) * nx + x;
      const long long gzp = ((long long)wrap(z + m, nz) * ny + y) * nx + x;
      const long long gzm = ((long long)wrap(z - m, nz) * ny + y) * nx + x;
      const long long nb[3][2] = {{gxp, gxm}, {gyp, gym}, {gzp, gzm}};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const C up = psi[nb[d][0] * no + n], um = psi[nb[d][1] * no + n];
        const double tr = (double)up.re - um.re, ti = (double)up.im - um.im;
        // Im(conj(c) * t) = c.re t.im - c.im t.re
        jd[d] += am * ((double)c.re * ti - (double)c.im * tr);
      }
    }
    j0 += f * jd[0];
    j1 += f * jd[1];
    j2 += f * jd[2];
  }
  rho = wave_sum(rho);
  j0 = wave_sum(j0);
  j1 = wave_sum(j1);
  j2 = wave_sum(j2);
  if (lane == 0 && valid) {
    const double* A = D.a + (long long)step * D.a_stride;
    if (D.rho) ((T*)D.rho)[(long long)obs * D.n_grid + g] = (T)rho;
    if (D.jcur) {
      T* j = (T*)D.jcur + ((long long)obs * D.n_grid + g) * 3;
      j[0] = (T)(j0 + A[0] * rho);
      j[1] = (T)(j1 + A[1] * rho);
      j[2] = (T)(j2 + A[2] * rho);
    }
  }
  if (D.jpart) {
    // block sums (four grid points, fixed order) of rho and the paramagnetic
    // current for the macroscopic current
    double* out = D.jpart + (long long)(blockIdx.x - D.item0_dens) * 4;
    const double v[4] = {rho, j0, j1, j2};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (lane == 0) red[threadIdx.x / kWave] = v[i];
      __syncthreads();
      if (threadIdx.x == 0) out[i] = (red[0] + red[1]) + (red[2] + red[3]);
      __syncthreads();
    }
  }
}

// energy[obs] = h^3 sum(e_loc) + sum(e_nl).  Items: (dom); one block per domain.
__global__ __launch_bounds__(kBlock) void k_energy_final(const DomDesc* __restrict__ doms,
                                                         const Item* __restrict__ items, int obs) {
  __shared__ double red[4];
  const DomDesc& D = doms[items[blockIdx.x].dom];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < D.n_e_loc; i += kBlock) a += D.e_loc[i];
  for (int i = threadIdx.x; i < D.n_e_nl; i += kBlock) b += D.e_nl[i];
  const double sa = block_sum(a, red);
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0 && D.energy) D.energy[obs] = D.h * D.h * D.h * sa + sb;
}

// Gradient partials: for each d, sum Re(conj(mu) * coef * (-i D1_d u + A_d u)).
// Items: (dom, element block); EPT elements per thread.
template <typename T, int EPT>
__global__ __launch_bounds__(kBlock) void k_grad_partial(const DomDesc* __restrict__ doms,
                                                         const Item* __restrict__ items, int mu_slot,
                                                         int u_slot, double cre, double cim) {
  using C = Cplx<T>;
  __shared__ double red[4];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb, r = D.r;
  const long long total = D.n_grid * no;
  const C* __restrict__ mu = (const C*)D.slot[mu_slot];
  const C* __restrict__ u = (const C*)D.slot[u_slot];
  const double* A = D.a;
  const double ih = 1.0 / D.h;
  double acc[3] = {0, 0, 0};
  // I: the index type, 32-bit when the domain's element count allows it (a
  // uniform branch per block; the divisions dominate the kernel otherwise)
  auto run = [&](auto tag, auto rc) {
    using I = decltype(tag);
    constexpr int R = decltype(rc)::value;   // the stencil radius, so the neighbour loads unroll
    const I xy = (I)nx * (I)ny;
    for (int i = 0; i < EPT; ++i) {
      const long long e = ((long long)it.a * EPT + i) * kBlock + threadIdx.x;
      if (e >= total) break;
      const I ei = (I)e;
      const I g = ei / (I)no;
      const int n = (int)(ei - g * (I)no);
      const int z = (int)(g / xy);
      const I rem = g - (I)z * xy;
      const int y = (int)(rem / (I)nx);
      const int x = (int)(rem - (I)y * (I)nx);
      const C m = mu[ei], c = u[ei];
      // w = conj(mu) * coef
      const double wr = (double)m.re * cre + (double)m.im * cim;
      const double wi = (double)m.re * cim - (double)m.im * cre;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double dr = 0, di = 0;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          I gp, gm;
          if (d == 0) {
            gp = g - (I)x + (I)wrap(x + k, nx);
            gm = g - (I)x + (I)wrap(x - k, nx);
          } else if (d == 1) {
            gp = g + ((I)wrap(y + k, ny) - (I)y) * (I)nx;
            gm = g + ((I)wrap(y - k, ny) - (I)y) * (I)nx;
          } else {
            gp = g + ((I)wrap(z + k, nz) - (I)z) * xy;
            gm = g + ((I)wrap(z - k, nz) - (I)z) * xy;
          }
          const C up = u[gp * (I)no + (I)n], um = u[gm * (I)no + (I)n];
          const double ak = fd1(R, k) * ih;
          dr += ak * ((double)up.re - um.re);
          di += ak * ((double)up.im - um.im);
        }
        // t = -i D1 u + A_d u
        const double tr = di + A[d] * c.re;
        const double ti = -dr + A[d] * c.im;
        acc[d] += wr * tr - wi * ti;
      }
    }
  };
  auto by_radius = [&](auto tag) {
    if (r == 1)
      run(tag, std::integral_constant<int, 1>{});
    else if (r == 2)
      run(tag, std::integral_constant<int, 2>{});
    else
      run(tag, std::integral_constant<int, 3>{});
  };
  if (total < (1LL << 31))
    by_radius(0u);
  else
    by_radius(0LL);
  for (int d = 0; d < 3; ++d) {
    const double s = block_sum(acc[d], red);
    if (threadIdx.x == 0) D.g_part[(long long)(blockIdx.x - D.item0_elem) * 3 + d] = s;
  }
}

// grad[d] += 2 h^3 sum(partials).  When the field is shared (one gradient for
// all domains) a single block walks every domain in order.
__global__ __launch_bounds__(kBlock) void k_grad_final(const DomDesc* __restrict__ doms, int n_dom,
                                                       int shared) {
  __shared__ double red[4];
  const int d0 = shared ? 0 : blockIdx.x, d1 = shared ? n_dom : blockIdx.x + 1;
  double s[3] = {0, 0, 0};
  for (int dm = d0; dm < d1; ++dm) {
    const DomDesc& D = doms[dm];
    double a[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < D.n_g_part; i += kBlock)
      for (int d = 0; d < 3; ++d) a[d] += D.g_part[(long long)i * 3 + d];
    const double h3 = D.h * D.h * D.h;
    for (int d = 0; d < 3; ++d) s[d] += 2.0 * h3 * block_sum(a[d], red);
  }
  if (threadIdx.x == 0) {
    double* g = doms[d0].grad;
    for (int d = 0; d < 3; ++d) g[d] += s[d];
  }
}

// out += x over psi-sized slots.  Items: (dom, element block).
template <typename T, int EPT>
__global__ __launch_bounds__(kBlock) void k_axpy(const DomDesc* __restrict__ doms,
                                                 const Item* __restrict__ items, int x_slot, int out_slot) {
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long total = D.n_grid * D.n_orb * 2;
  const T* __restrict__ x = (const T*)D.slot[x_slot];
  T* __restrict__ out = (T*)D.slot[out_slot];
  for (int i = 0; i < 2 * EPT; ++i) {
    const long long e = ((long long)it.a * 2 * EPT + i) * kBlock + threadIdx.x;
    if (e < total) out[e] += x[e];
  }
}

// Sets *flag to 1 if any value of the psi slot is not finite.
template <typename T, int EPT>
__global__ __launch_bounds__(kBlock) void k_nonfinite(const DomDesc* __restrict__ doms,
                                                      const Item* __restrict__ items, int* flag) {
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long total = D.n_grid * D.n_orb * 2;
  const T* __restrict__ x = (const T*)D.slot[SLOT_PSI];
  int bad = 0;
  for (int i = 0; i < 2 * EPT; ++i) {
    const long long e = ((long long)it.a * 2 * EPT + i) * kBlock + threadIdx.x;
    if (e < total && !isfinite(x[e])) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_fill_int(int* p, int v) { *p = v; }

}  // namespace dcm

namespace dcm {

// Column norms of the psi slot: partial sums of |psi[g][n]|^2 over 256 grid
// rows per block, one FP64 value per (block, orbital), in a fixed order.
// Items: (dom, row block).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_colnorm_partial(const DomDesc* __restrict__ doms,
                                                            const Item* __restrict__ items) {
  using C = Cplx<T>;
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int no = D.n_orb;
  const long long g0 = (long long)it.a * kBlock, g1 = min(g0 + kBlock, D.n_grid);
  const C* __restrict__ psi = (const C*)D.slot[SLOT_PSI];
  const int rows = (int)(g1 - g0);
  double* __restrict__ part = D.cn_part + (long long)(blockIdx.x - D.item0_rows) * no;
  if (no > kBlock / 2) {
    for (int n = threadIdx.x; n < no; n += kBlock) {
      // rows in order; unrolled so that eight loads are in flight per thread
      double s = 0;
      const C* __restrict__ col = psi + g0 * no + n;
#pragma unroll 8
      for (int r = 0; r < rows; ++r) {
        const C c = col[(long long)r * no];
        s += (double)c.re * c.re + (double)c.im * c.im;
      }
      part[n] = s;
    }
    return;
  }
  // no <= 128: ph = kBlock / no threads per orbital, thread (p, n) summing rows
  // p, p + ph, ... (so a wave's loads cover whole consecutive rows); the ph
  // sums of an orbital are then added in p order
  __shared__ double red[kBlock];
  const int ph = kBlock / no, p = threadIdx.x / no, n = threadIdx.x % no;
  double s = 0;
  if (p < ph) {
    const C* __restrict__ col = psi + g0 * no + n;
#pragma unroll 8
    for (int r = p; r < rows; r += ph) {
      const C c = col[(long long)r * no];
      s += (double)c.re * c.re + (double)c.im * c.im;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < no) {
    double t = 0;
    for (int q = 0; q < ph; ++q) t += red[q * no + threadIdx.x];
    part[threadIdx.x] = t;
  }
}

// inv[n] = 1 / sqrt(h^3 sum_blocks partial[blk][n]) in block order.  Items: one per domain.
__global__ __launch_bounds__(kBlock) void k_colnorm_final(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items) {
  const DomDesc& D = doms[items[blockIdx.x].dom];
  const int no = D.n_orb;
  const double h3 = D.h * D.h * D.h;
  const int nb = D.n_rows_blocks;
  for (int n = threadIdx.x; n < no; n += kBlock) {
    // block order; unrolled so that sixteen loads are in flight per thread
    double s = 0;
    const double* __restrict__ col = D.cn_part + n;
#pragma unroll 16
    for (int b = 0; b < nb; ++b) s += col[(long long)b * no];
    D.cn_inv[n] = 1.0 / sqrt(h3 * s);
  }
}

// psi[g][n] *= inv[n].  Items: (dom, row block).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_colnorm_scale(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items) {
  using C = Cplx<T>;
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int no = D.n_orb;
  const long long g0 = (long long)it.a * kBlock, g1 = min(g0 + kBlock, D.n_grid);
  C* __restrict__ psi = (C*)D.slot[SLOT_PSI] + g0 * no;
  // element e of the block's rows is orbital e mod no; stepping e by the block
  // size steps the orbital by kBlock mod no (one conditional wrap), so no
  // 64-bit division per element
  const int count = (int)((g1 - g0) * no), step = kBlock % no;
  int n = threadIdx.x % no;
  for (int e = threadIdx.x; e < count; e += kBlock) {
    const T s = (T)D.cn_inv[n];
    psi[e].re *= s;
    psi[e].im *= s;
    n += step;
    if (n >= no) n -= no;
  }
}

// Occupations of the reference orbitals from the cross overlap
// S_sn = h^3 <psi0_s|psi_n> (in D.overlap, complex128):
//     f_s = sum_n f_n |S_sn|^2.
// One wave per reference orbital s; the lanes take n in a fixed order and the
// wave sum has a fixed shape.  Items: (dom, block of 4 rows).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_occ_rows(const DomDesc* __restrict__ doms,
                                                     const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int no = D.n_orb;
  const int s = it.a * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (s >= no) return;                 // whole waves leave together
  const T* __restrict__ occ = (const T*)D.occ;
  const double* __restrict__ S = D.overlap + (long long)s * no * 2;
  double acc = 0.0;
  for (int n = lane; n < no; n += kWave) {
    const double re = S[2 * n], im = S[2 * n + 1];
    acc += (double)occ[n] * (re * re + im * im);
  }
  acc = wave_sum(acc);
  if (lane == 0) D.f_occ[s] = acc;
}

// n_exc = sum_n f_n (h^3 |psi_n|^2 - sum_s |S_sn|^2), the occupation-weighted
// norm outside the reference span.  The column norms come from the
// k_colnorm_partial block partials, summed in block order.  One block per domain.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_occ_final(const DomDesc* __restrict__ doms,
                                                      const Item* __restrict__ items) {
  __shared__ double red[kBlock / kWave];
  const DomDesc& D = doms[items[blockIdx.x].dom];
  const int no = D.n_orb;
  const double h3 = D.h * D.h * D.h;
  const T* __restrict__ occ = (const T*)D.occ;
  double t = 0.0;
  for (int n = threadIdx.x; n < no; n += kBlock) {
    double nrm = 0.0, col = 0.0;
    for (int b = 0; b < D.n_rows_blocks; ++b) nrm += D.cn_part[(long long)b * no + n];
    for (int s = 0; s < no; ++s) {
      const double re = D.overlap[((long long)s * no + n) * 2], im = D.overlap[((long long)s * no + n) * 2 + 1];
      col += re * re + im * im;
    }
    t += (double)occ[n] * (h3 * nrm - col);
  }
  t = block_sum(t, red);
  if (threadIdx.x == 0) D.n_exc[0] = t;
}

// Macroscopic current density of a domain,
//   J = (h^3 sum_g [j_para(g) + A rho(g)] - 2 sum f D Im(conj(P) R)) / Omega,
// from the block sums of k_density and k_jnl_partial (summed in a fixed order).
// A: the field of the state, D.a_ext[step] + field[0..2] for a Maxwell step
// (step >= 0), else D.a.  Items: one per domain.
__global__ __launch_bounds__(kBlock) void k_current_final(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items, int step, int nonlocal) {
  __shared__ double red[kBlock / kWave];
  const DomDesc& D = doms[items[blockIdx.x].dom];
  double s[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) s[i] = 0.0;
  for (int b = threadIdx.x; b < D.n_dens; b += kBlock)
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += D.jpart[(long long)b * 4 + i];
  if (nonlocal)
    for (int b = threadIdx.x; b < D.n_e_nl; b += kBlock)
#pragma unroll
      for (int d = 0; d < 3; ++d) s[4 + d] += D.jnl_part[(long long)d * D.n_e_nl + b];
#pragma unroll
  for (int i = 0; i < 7; ++i) s[i] = block_sum(s[i], red);
  if (threadIdx.x == 0) {
    double A[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) A[d] = step >= 0 ? D.a_ext[(long long)step * 3 + d] + D.field[d] : D.a[d];
    const double h3 = D.h * D.h * D.h, vol = (double)D.n_grid * h3;
#pragma unroll
    for (int d = 0; d < 3; ++d) D.cur[d] = (h3 * (s[1 + d] + A[d] * s[0]) - 2.0 * s[4 + d]) / vol;
  }
}

// Leapfrog update of the induced field of a uniform vector potential driven by
// the macroscopic particle current J_k (in D.cur):
//   b <- b - 4 pi dt J_k,  A_ind' = A_ind + dt b,
//   step field = (A_ext[k] + A_ext[k + 1]) / 2 + (A_ind + A_ind') / 2.
// One thread per domain (items: one per domain).
__global__ void k_field_update(const DomDesc* __restrict__ doms, const Item* __restrict__ items, int step,
                               double dt) {
  const DomDesc& D = doms[items[blockIdx.x].dom];
  if (threadIdx.x != 0) return;
  const double pi4 = 4.0 * 3.14159265358979323846;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double j = D.cur[d];
    const double b = D.field[3 + d] - pi4 * dt * j;
    const double a0 = D.field[d], a1 = a0 + dt * b;
    D.amid[(long long)step * 3 + d] =
        0.5 * (D.a_ext[(long long)step * 3 + d] + D.a_ext[(long long)(step + 1) * 3 + d]) + 0.5 * (a0 + a1);
    D.field[d] = a1;
    D.field[3 + d] = b;
    if (D.cur_out) D.cur_out[(long long)step * 3 + d] = j;
  }
}

}  // namespace dcm

// Local part of H: the finite-difference kinetic term with the vector
// potential, and the pointwise potential (Eq. 3 in atomic units),
//     H_loc u = -1/2 Lap_h u - i A.grad_h u + (v_loc + 1/2 |A|^2) u,
// fused with the Taylor-stage update out = base + coef * f^s * H_loc u.
//
// Layout: u[g][n] complex with the orbital index fastest (Sec. V.B.2).  A block
// owns a TX x TY tile of (x, y) columns and an orbital chunk of OC orbitals, and
// marches along z over a segment of planes.  The z-neighbours of every owned
// point-orbital sit in a register queue of 2r+1 planes; the x/y neighbours of
// the centre plane are staged through LDS with an r-wide halo (only the star
// arms, no corners).  All global reads of plane z+1 (queue head, halo strips,
// base values, potential) are issued before plane z is computed, so their
// latency overlaps the arithmetic and stores of plane z.  Each u value leaves
// HBM about once per sweep plus the halo strips, and the lanes of a wave touch
// OC consecutive orbitals of consecutive points.
//
// With want_density the sweep also produces, per (grid point, orbital chunk),
// the partial sums sum_n f_n |u_n|^2 and sum_n f_n Im(conj(u_n) D1_d u_n) of
// the density and the paramagnetic current (reduced over the chunk's lanes
// with DPP row operations); k_density_finish adds the chunks in order.
#pragma once

#include <utility>

#include "common.hpp"

namespace dcm {

struct StencilArgs {
  int u_slot, base_slot, out_slot;  // base_slot == SLOT_NONE: no base term
  double cre, cim;                  // coef
  int occ_scale;                    // multiply H_loc u by f_n
  int step;                         // A sample index
  int want_energy;                  // accumulate f_n Re(conj(u) H_loc u)
  int want_density;                 // write density / current partials of u
  // pulse-gradient partials formed in the sweep (ring sweep only): with v the
  // psi-sized buffer in grad_slot and g the gradient coefficient, block
  // partials of Re(g sum conj((-i D1_d + A_d) u) v), d = x, y, z, go to
  // D.g_part at the item's slot.  (-i D1_d + A_d) is Hermitian on the periodic
  // grid, so the sum equals Re(g sum conj(u) (-i D1_d + A_d) v).
  int grad_slot = SLOT_NONE;
  double gre = 0, gim = 0;
};

template <typename T>
struct StencilW {
  T alpha[3];       // -1/2 c_m / h^2, m = 1..r
  T a1[3];          // a_m / h
  T A[3];           // vector potential
  T centre;         // -3/2 c_0 / h^2 + 1/2 |A|^2
};

template <typename T>
__device__ __forceinline__ StencilW<T> stencil_weights(const DomDesc& D, int step) {
  StencilW<T> w;
  const double* A = D.a + (long long)step * D.a_stride;
  const double a0 = A[0], a1 = A[1], a2 = A[2];
  const double ih2 = 1.0 / (D.h * D.h), ih = 1.0 / D.h;
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    const bool on = m <= D.r;
    w.alpha[m - 1] = on ? (T)(-0.5 * fd2(D.r, m) * ih2) : (T)0;
    w.a1[m - 1] = on ? (T)(fd1(D.r, m) * ih) : (T)0;
  }
  w.A[0] = (T)a0;
  w.A[1] = (T)a1;
  w.A[2] = (T)a2;
  w.centre = (T)(-1.5 * fd2(D.r, 0) * ih2 + 0.5 * (a0 * a0 + a1 * a1 + a2 * a2));
  return w;
}

template <int R, int OC, int TX, int TY, int NT>
struct SweepCfg {
  static constexpr int kCols = TX * TY;            // (x, y) columns per tile
  static constexpr int kThrCols = NT / OC;         // columns covered by one pass of the block
  static constexpr int kPer = kCols / kThrCols;    // columns per thread
  static constexpr int kLX = TX + 2 * R;           // LDS plane with halo
  static constexpr int kLY = TY + 2 * R;
  static constexpr int kQ = 2 * R + 1;             // z queue depth
  static constexpr int kHx = 2 * R * TY, kHy = 2 * R * TX, kH = kHx + kHy;   // halo columns
  static constexpr int kHPer = (kH + kThrCols - 1) / kThrCols;               // halo columns per thread
  static_assert(NT % OC == 0 && kCols % kThrCols == 0, "tile does not fit the block");
};

// LDS coordinates of halo column hidx (x strips, then y strips).
template <int R, int TX, int TY>
__device__ __forceinline__ void halo_xy(int hidx, int& lx, int& ly) {
  constexpr int kHx = 2 * R * TY;
  if (hidx < kHx) {
    const int side = hidx / (R * TY), rem = hidx % (R * TY);
    ly = rem / R + R;
    lx = side == 0 ? rem % R : TX + R + rem % R;
  } else {
    const int h2 = hidx - kHx;
    const int side = h2 / (R * TX), rem = h2 % (R * TX);
    lx = rem % TX + R;
    ly = side == 0 ? rem / TX : TY + R + rem / TX;
  }
}

// Slot of an item's local-energy partial in D.e_loc: its index in the
// domain's (z segment, orbital chunk, y tile, x tile) order, whatever the
// position of the item in its launch.
template <int TX, int TY>
__device__ __forceinline__ int e_loc_slot(const DomDesc& D, const Item& it) {
  const int nxt = (D.nx + TX - 1) / TX, nyt = (D.ny + TY - 1) / TY;
  return (((it.c >> 16) * D.n_chunks + (it.c & 0xffff)) * nyt + it.b) * nxt + it.a;
}

// Items: (dom, x tile, y tile, (z segment << 16) | orbital chunk).
// D.zseg planes per segment.  Energy partials: one per item, at
// e_loc[e_loc_slot].  Density partials at
// dpart[chunk][g][0..3] (rho, j_x, j_y, j_z without the A rho term).
template <typename T, int R, int OC, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_stencil_sweep(const DomDesc* __restrict__ doms,
                                                      const Item* __restrict__ items,
                                                      StencilArgs args) {
  using C = Cplx<T>;
  using Cfg = SweepCfg<R, OC, TX, TY, NT>;
  constexpr int KP = Cfg::kPer, KQ = Cfg::kQ, KH = Cfg::kHPer;
  __shared__ C lds[Cfg::kLY * Cfg::kLX * OC];
  __shared__ double red[NT / kWave];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb;
  const int x0 = it.a * TX, y0 = it.b * TY;
  const int chunk = it.c & 0xffff;
  const int zseg = it.c >> 16, oc0 = chunk * OC;
  const int z_begin = zseg * D.zseg, z_end = min(z_begin + D.zseg, nz);

  const C* __restrict__ u = (const C*)D.slot[args.u_slot];
  const C* __restrict__ base = args.base_slot < SLOT_NONE ? (const C*)D.slot[args.base_slot] : nullptr;
  C* __restrict__ out = (C*)D.slot[args.out_slot];
  const T* __restrict__ V = (const T*)D.v;
  const T* __restrict__ occ = (const T*)D.occ;

  const StencilW<T> w = stencil_weights<T>(D, args.step);
  const T cre = (T)args.cre, cim = (T)args.cim;

  const int o = threadIdx.x % OC;
  const int tc = threadIdx.x / OC;
  const int n = oc0 + o;
  const bool n_ok = n < no;
  const T fn = n_ok ? occ[n] : (T)0;
  const long long plane = (long long)nx * ny;

  // Columns of this thread.  Loads use wrapped coordinates so that slots past
  // the domain edge hold the periodic images needed by the last valid column.
  int lxk[KP], lyk[KP];
  int gcol[KP];                    // y * nx + x of the column (N_g < 2^31)
  bool ok[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int col = tc + k * Cfg::kThrCols;
    lxk[k] = col % TX;
    lyk[k] = col / TX;
    const int x = x0 + lxk[k], y = y0 + lyk[k];
    ok[k] = n_ok && x < nx && y < ny;
    gcol[k] = wrap(y, ny) * nx + wrap(x, nx);
  }
  // Halo columns of this thread
  int hl[KH];
  int hcol[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hidx = tc + k * Cfg::kThrCols;
    int lx = 0, ly = 0;
    if (hidx < Cfg::kH) halo_xy<R, TX, TY>(hidx, lx, ly);
    hl[k] = hidx < Cfg::kH ? (ly * Cfg::kLX + lx) * OC + o : -1;
    hcol[k] = wrap(y0 + ly - R, ny) * nx + wrap(x0 + lx - R, nx);
  }

  auto ldu = [&](int z, int col) -> C {
    return n_ok ? u[((long long)z * plane + col) * no + n] : C{0, 0};
  };

  C q[KP][KQ];      // q[k][s] = plane z - R + s
  C qn[KP];         // plane z + R + 1 (prefetch)
  C hpf[KH];        // halo of plane z + 1 (prefetch)
  C bcur[KP], bpf[KP];
  T vcur[KP], vpf[KP];

  // prologue: queue, centre plane of z_begin into LDS, its base and potential
#pragma unroll
  for (int k = 0; k < KP; ++k) {
#pragma unroll
    for (int s = 0; s < KQ; ++s) q[k][s] = ldu(wrap(z_begin - R + s, nz), gcol[k]);
    const long long g = (long long)z_begin * plane + gcol[k];
    bcur[k] = (base && ok[k]) ? base[g * no + n] : C{0, 0};
    vcur[k] = ok[k] ? V[g] : (T)0;
    lds[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
  }
#pragma unroll
  for (int k = 0; k < KH; ++k)
    if (hl[k] >= 0) lds[hl[k]] = ldu(z_begin, hcol[k]);
  __syncthreads();

  double e_acc = 0.0;
  for (int z = z_begin; z < z_end; ++z) {
    const bool more = z + 1 < z_end;
    if (more) {
      const int zq = wrap(z + 1 + R, nz);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        qn[k] = ldu(zq, gcol[k]);
        const long long g1 = (long long)(z + 1) * plane + gcol[k];
        bpf[k] = (base && ok[k]) ? base[g1 * no + n] : C{0, 0};
        vpf[k] = ok[k] ? V[g1] : (T)0;
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) hpf[k] = hl[k] >= 0 ? ldu(z + 1, hcol[k]) : C{0, 0};
    }

#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int cx = lxk[k] + R, cy = lyk[k] + R;
      const C c0 = q[k][R];
      // per axis: S = sum_m alpha_m (u+ + u-), G = sum_m (a_m / h) (u+ - u-)
      C S{0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const C xp = lds[(cy * Cfg::kLX + cx + m) * OC + o], xm = lds[(cy * Cfg::kLX + cx - m) * OC + o];
        const C yp = lds[((cy + m) * Cfg::kLX + cx) * OC + o], ym = lds[((cy - m) * Cfg::kLX + cx) * OC + o];
        const C zp = q[k][R + m], zm = q[k][R - m];
        const T al = w.alpha[m - 1], am = w.a1[m - 1];
        S.re += al * ((xp.re + xm.re) + (yp.re + ym.re) + (zp.re + zm.re));
        S.im += al * ((xp.im + xm.im) + (yp.im + ym.im) + (zp.im + zm.im));
        G[0].re += am * (xp.re - xm.re); G[0].im += am * (xp.im - xm.im);
        G[1].re += am * (yp.re - ym.re); G[1].im += am * (yp.im - ym.im);
        G[2].re += am * (zp.re - zm.re); G[2].im += am * (zp.im - zm.im);
      }
      // H_loc u = S - i A.G + (centre + V) c0
      const T cv = w.centre + vcur[k];
      C acc{S.re + cv * c0.re + (w.A[0] * G[0].im + w.A[1] * G[1].im + w.A[2] * G[2].im),
            S.im + cv * c0.im - (w.A[0] * G[0].re + w.A[1] * G[1].re + w.A[2] * G[2].re)};
      if (args.want_density) {
        // f |c0|^2 and f Im(conj(c0) G_d), summed over the chunk's OC lanes
        T dv[4] = {fn * (c0.re * c0.re + c0.im * c0.im), fn * (c0.re * G[0].im - c0.im * G[0].re),
                   fn * (c0.re * G[1].im - c0.im * G[1].re), fn * (c0.re * G[2].im - c0.im * G[2].re)};
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[i] = group_sum<OC>(dv[i]);
        const int x = x0 + lxk[k], y = y0 + lyk[k];
        if (o == 0 && x < nx && y < ny) {
          const long long g = (long long)z * plane + gcol[k];
          T* dp = (T*)D.dpart + ((long long)chunk * D.n_grid + g) * 4;
          dp[0] = dv[0]; dp[1] = dv[1]; dp[2] = dv[2]; dp[3] = dv[3];
        }
      }
      if (ok[k]) {
        if (args.want_energy) e_acc += (double)fn * ((double)c0.re * acc.re + (double)c0.im * acc.im);
        if (args.occ_scale) { acc.re *= fn; acc.im *= fn; }
        C r{cre * acc.re - cim * acc.im, cre * acc.im + cim * acc.re};
        r.re += bcur[k].re;
        r.im += bcur[k].im;
        const long long g = (long long)z * plane + gcol[k];
        out[g * no + n] = r;
      }
    }
    if (!more) break;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KP; ++k) {
#pragma unroll
      for (int s = 0; s < KQ - 1; ++s) q[k][s] = q[k][s + 1];
      q[k][KQ - 1] = qn[k];
      bcur[k] = bpf[k];
      vcur[k] = vpf[k];
      lds[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
    }
#pragma unroll
    for (int k = 0; k < KH; ++k)
      if (hl[k] >= 0) lds[hl[k]] = hpf[k];
    __syncthreads();
  }
  if (args.want_energy) {
    const double s = block_sum<double, NT / kWave>(e_acc, red);
    if (threadIdx.x == 0) D.e_loc[e_loc_slot<TX, TY>(D, it)] = s;
  }
}

// Same sweep with the global reads issued two planes ahead and the centre
// plane double-buffered in LDS (one barrier per plane).  The plane loop is
// unrolled by two so the two prefetch register sets are addressed statically.
template <typename T, int R, int OC, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_stencil_sweep2(const DomDesc* __restrict__ doms,
                                                       const Item* __restrict__ items,
                                                       StencilArgs args) {
  using C = Cplx<T>;
  using Cfg = SweepCfg<R, OC, TX, TY, NT>;
  constexpr int KP = Cfg::kPer, KQ = Cfg::kQ, KH = Cfg::kHPer;
  constexpr int PLANE = Cfg::kLY * Cfg::kLX * OC;
  __shared__ C lds[2 * PLANE];
  __shared__ double red[NT / kWave];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb;
  const int x0 = it.a * TX, y0 = it.b * TY;
  const int chunk = it.c & 0xffff;
  const int zseg = it.c >> 16, oc0 = chunk * OC;
  const int z_begin = zseg * D.zseg, z_end = min(z_begin + D.zseg, nz);

  const C* __restrict__ u = (const C*)D.slot[args.u_slot];
  const C* __restrict__ base = args.base_slot < SLOT_NONE ? (const C*)D.slot[args.base_slot] : nullptr;
  C* __restrict__ out = (C*)D.slot[args.out_slot];
  const T* __restrict__ V = (const T*)D.v;
  const T* __restrict__ occ = (const T*)D.occ;

  const StencilW<T> w = stencil_weights<T>(D, args.step);
  const T cre = (T)args.cre, cim = (T)args.cim;

  const int o = threadIdx.x % OC;
  const int tc = threadIdx.x / OC;
  const int n = oc0 + o;
  const bool n_ok = n < no;
  const T fn = n_ok ? occ[n] : (T)0;
  const long long plane = (long long)nx * ny;

  int lxk[KP], lyk[KP], gcol[KP];
  bool ok[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int col = tc + k * Cfg::kThrCols;
    lxk[k] = col % TX;
    lyk[k] = col / TX;
    const int x = x0 + lxk[k], y = y0 + lyk[k];
    ok[k] = n_ok && x < nx && y < ny;
    gcol[k] = wrap(y, ny) * nx + wrap(x, nx);
  }
  int hl[KH], hcol[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hidx = tc + k * Cfg::kThrCols;
    int lx = 0, ly = 0;
    if (hidx < Cfg::kH) halo_xy<R, TX, TY>(hidx, lx, ly);
    hl[k] = hidx < Cfg::kH ? (ly * Cfg::kLX + lx) * OC + o : -1;
    hcol[k] = wrap(y0 + ly - R, ny) * nx + wrap(x0 + lx - R, nx);
  }
  auto ldu = [&](int z, int col) -> C {
    return n_ok ? u[((long long)z * plane + col) * no + n] : C{0, 0};
  };

  struct Pf {   // everything plane z needs that is not already in the queue
    C qh[KP];   // queue head: plane z + R
    C h[KH];    // halo of plane z
    C b[KP];    // base of plane z
    T v[KP];    // potential of plane z
  };
  auto fetch = [&](Pf& f, int z) {
    const int zq = wrap(z + R, nz);
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      f.qh[k] = ldu(zq, gcol[k]);
      const long long g = (long long)z * plane + gcol[k];
      f.b[k] = (base && ok[k]) ? base[g * no + n] : C{0, 0};
      f.v[k] = ok[k] ? V[g] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < KH; ++k) f.h[k] = hl[k] >= 0 ? ldu(z, hcol[k]) : C{0, 0};
  };

  C q[KP][KQ];       // q[k][s] = plane z - R + s
  C bcur[KP];
  T vcur[KP];
  // prologue: queue of z_begin, its centre plane and halo in LDS buffer 0
#pragma unroll
  for (int k = 0; k < KP; ++k) {
#pragma unroll
    for (int s = 0; s < KQ; ++s) q[k][s] = ldu(wrap(z_begin - R + s, nz), gcol[k]);
    const long long g = (long long)z_begin * plane + gcol[k];
    bcur[k] = (base && ok[k]) ? base[g * no + n] : C{0, 0};
    vcur[k] = ok[k] ? V[g] : (T)0;
    lds[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
  }
#pragma unroll
  for (int k = 0; k < KH; ++k)
    if (hl[k] >= 0) lds[hl[k]] = ldu(z_begin, hcol[k]);
  Pf pa, pb;
  if (z_begin + 1 < z_end) fetch(pa, z_begin + 1);
  __syncthreads();

  double e_acc = 0.0;
  // one plane: compute z from LDS buffer cur; fetch z + 2 into fnext; move the
  // prefetched plane z + 1 (fcur) into the queue and LDS buffer 1 - cur.
  auto plane_step = [&](int z, int cur, Pf& fcur, Pf& fnext) {
    if (z + 2 < z_end) fetch(fnext, z + 2);
    const C* L = lds + cur * PLANE;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int cx = lxk[k] + R, cy = lyk[k] + R;
      const C c0 = q[k][R];
      C S{0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const C xp = L[(cy * Cfg::kLX + cx + m) * OC + o], xm = L[(cy * Cfg::kLX + cx - m) * OC + o];
        const C yp = L[((cy + m) * Cfg::kLX + cx) * OC + o], ym = L[((cy - m) * Cfg::kLX + cx) * OC + o];
        const C zp = q[k][R + m], zm = q[k][R - m];
        const T al = w.alpha[m - 1], am = w.a1[m - 1];
        S.re += al * ((xp.re + xm.re) + (yp.re + ym.re) + (zp.re + zm.re));
        S.im += al * ((xp.im + xm.im) + (yp.im + ym.im) + (zp.im + zm.im));
        G[0].re += am * (xp.re - xm.re); G[0].im += am * (xp.im - xm.im);
        G[1].re += am * (yp.re - ym.re); G[1].im += am * (yp.im - ym.im);
        G[2].re += am * (zp.re - zm.re); G[2].im += am * (zp.im - zm.im);
      }
      const T cv = w.centre + vcur[k];
      C acc{S.re + cv * c0.re + (w.A[0] * G[0].im + w.A[1] * G[1].im + w.A[2] * G[2].im),
            S.im + cv * c0.im - (w.A[0] * G[0].re + w.A[1] * G[1].re + w.A[2] * G[2].re)};
      if (args.want_density) {
        T dv[4] = {fn * (c0.re * c0.re + c0.im * c0.im), fn * (c0.re * G[0].im - c0.im * G[0].re),
                   fn * (c0.re * G[1].im - c0.im * G[1].re), fn * (c0.re * G[2].im - c0.im * G[2].re)};
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[i] = group_sum<OC>(dv[i]);
        const int x = x0 + lxk[k], y = y0 + lyk[k];
        if (o == 0 && x < nx && y < ny) {
          const long long g = (long long)z * plane + gcol[k];
          T* dp = (T*)D.dpart + ((long long)chunk * D.n_grid + g) * 4;
          dp[0] = dv[0]; dp[1] = dv[1]; dp[2] = dv[2]; dp[3] = dv[3];
        }
      }
      if (ok[k]) {
        if (args.want_energy) e_acc += (double)fn * ((double)c0.re * acc.re + (double)c0.im * acc.im);
        if (args.occ_scale) { acc.re *= fn; acc.im *= fn; }
        C r{cre * acc.re - cim * acc.im, cre * acc.im + cim * acc.re};
        r.re += bcur[k].re;
        r.im += bcur[k].im;
        out[((long long)z * plane + gcol[k]) * no + n] = r;
      }
    }
    if (z + 1 < z_end) {
      C* Ln = lds + (1 - cur) * PLANE;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
#pragma unroll
        for (int s = 0; s < KQ - 1; ++s) q[k][s] = q[k][s + 1];
        q[k][KQ - 1] = fcur.qh[k];
        bcur[k] = fcur.b[k];
        vcur[k] = fcur.v[k];
        Ln[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
      }
#pragma unroll
      for (int k = 0; k < KH; ++k)
        if (hl[k] >= 0) Ln[hl[k]] = fcur.h[k];
    }
    __syncthreads();
  };
  for (int z = z_begin; z < z_end; z += 2) {
    plane_step(z, 0, pa, pb);
    if (z + 1 < z_end) plane_step(z + 1, 1, pb, pa);
  }
  if (args.want_energy) {
    const double s = block_sum<double, NT / kWave>(e_acc, red);
    if (threadIdx.x == 0) D.e_loc[e_loc_slot<TX, TY>(D, it)] = s;
  }
}

// Same sweep with every global read of a plane issued in one step: the halo
// strips of plane z + R + 1 are fetched together with its interior (the queue
// head) and wait in a register queue of R planes until that plane becomes the
// centre.  Neighbouring tiles fetch the same plane at about the same time, so
// the strips are served from L2 instead of being fetched again from memory a
// few planes later.  The centre plane is double-buffered in LDS (one barrier
// per plane).  When the base buffer is u itself (the first Horner stage) the
// base term is the queue's centre and is not read again.  Addresses are a
// per-plane base (uniform) plus a fixed 32-bit byte offset per column, which
// requires a plane of u, nx ny n_orb complex values, to span < 2^32 bytes.
template <typename T, int R, int OC, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_stencil_sweep3(const DomDesc* __restrict__ doms,
                                                       const Item* __restrict__ items,
                                                       StencilArgs args) {
  using C = Cplx<T>;
  using Cfg = SweepCfg<R, OC, TX, TY, NT>;
  constexpr int KP = Cfg::kPer, KQ = Cfg::kQ, KH = Cfg::kHPer;
  constexpr int PLANE = Cfg::kLY * Cfg::kLX * OC;
  __shared__ C lds[2 * PLANE];
  __shared__ double red[NT / kWave];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb;
  const int x0 = it.a * TX, y0 = it.b * TY;
  const int chunk = it.c & 0xffff;
  const int zseg = it.c >> 16, oc0 = chunk * OC;
  const int z_begin = zseg * D.zseg, z_end = min(z_begin + D.zseg, nz);

  const bool base_is_u = args.base_slot == args.u_slot;
  const char* __restrict__ ub = (const char*)D.slot[args.u_slot];
  const char* __restrict__ bb =
      (args.base_slot < SLOT_NONE && !base_is_u) ? (const char*)D.slot[args.base_slot] : nullptr;
  char* __restrict__ ob = (char*)D.slot[args.out_slot];
  const char* __restrict__ vb = (const char*)D.v;
  const T* __restrict__ occ = (const T*)D.occ;
  const long long plane = (long long)nx * ny;
  const long long pbytes = plane * no * (long long)sizeof(C);      // one plane of u
  const long long vbytes = plane * (long long)sizeof(T);           // one plane of V

  const StencilW<T> w = stencil_weights<T>(D, args.step);
  const T cre = (T)args.cre, cim = (T)args.cim;

  const int o = threadIdx.x % OC;
  const int tc = threadIdx.x / OC;
  const int n = oc0 + o;
  const bool n_ok = n < no;
  const int nl = n_ok ? n : no - 1;        // lanes past the last orbital read a valid element
  const T fn = n_ok ? occ[n] : (T)0;

  int lxk[KP], lyk[KP];
  unsigned co[KP], cv[KP];                 // byte offsets of the column in a plane of u / of V
  bool ok[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int col = tc + k * Cfg::kThrCols;
    lxk[k] = col % TX;
    lyk[k] = col / TX;
    const int x = x0 + lxk[k], y = y0 + lyk[k];
    ok[k] = n_ok && x < nx && y < ny;
    const unsigned gc = (unsigned)(wrap(y, ny) * nx + wrap(x, nx));
    co[k] = (gc * (unsigned)no + (unsigned)nl) * (unsigned)sizeof(C);
    cv[k] = gc * (unsigned)sizeof(T);
  }
  int hl[KH];
  unsigned ho[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hidx = tc + k * Cfg::kThrCols;
    int lx = R, ly = R;
    if (hidx < Cfg::kH) halo_xy<R, TX, TY>(hidx, lx, ly);
    hl[k] = hidx < Cfg::kH ? (ly * Cfg::kLX + lx) * OC + o : -1;
    const unsigned gc = (unsigned)(wrap(y0 + ly - R, ny) * nx + wrap(x0 + lx - R, nx));
    ho[k] = (gc * (unsigned)no + (unsigned)nl) * (unsigned)sizeof(C);
  }
  auto at = [&](const char* b, int z, unsigned off) -> C {
    return *(const C*)(b + (long long)z * pbytes + off);
  };
  auto vat = [&](int z, unsigned off) -> T { return *(const T*)(vb + (long long)z * vbytes + off); };

  C q[KP][KQ];          // q[k][s] = plane z - R + s
  C hq[KH][R + 1];      // hq[k][j] = halo of plane z + 1 + j; j = R receives the prefetch
  C qn[KP];             // prefetch of the queue head, plane z + R + 1
  C bcur[KP], bpf[KP];
  T vcur[KP], vpf[KP];

  // prologue: the queue of z_begin; its centre plane (interior and halo) into
  // LDS buffer 0; the halo of the next R planes into the halo queue
#pragma unroll
  for (int k = 0; k < KP; ++k) {
#pragma unroll
    for (int s = 0; s < KQ; ++s) q[k][s] = at(ub, wrap(z_begin - R + s, nz), co[k]);
    bcur[k] = bb ? at(bb, z_begin, co[k]) : C{0, 0};
    vcur[k] = vat(z_begin, cv[k]);
    lds[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
  }
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    if (hl[k] >= 0) lds[hl[k]] = at(ub, z_begin, ho[k]);
#pragma unroll
    for (int j = 0; j < R; ++j) hq[k][j] = at(ub, wrap(z_begin + 1 + j, nz), ho[k]);
  }
  lds_barrier();

  double e_acc = 0.0;
  for (int z = z_begin; z < z_end; ++z) {
    const bool more = z + 1 < z_end;
    const C* L = lds + ((z - z_begin) & 1) * PLANE;
    if (more) {
      const int zq = wrap(z + 1 + R, nz);
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        qn[k] = at(ub, zq, co[k]);
        bpf[k] = bb ? at(bb, z + 1, co[k]) : C{0, 0};
        vpf[k] = vat(z + 1, cv[k]);
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) hq[k][R] = at(ub, zq, ho[k]);
    }

#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int cx = lxk[k] + R, cy = lyk[k] + R;
      const C c0 = q[k][R];
      C S{0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const C xp = L[(cy * Cfg::kLX + cx + m) * OC + o], xm = L[(cy * Cfg::kLX + cx - m) * OC + o];
        const C yp = L[((cy + m) * Cfg::kLX + cx) * OC + o], ym = L[((cy - m) * Cfg::kLX + cx) * OC + o];
        const C zp = q[k][R + m], zm = q[k][R - m];
        const T al = w.alpha[m - 1], am = w.a1[m - 1];
        S.re += al * ((xp.re + xm.re) + (yp.re + ym.re) + (zp.re + zm.re));
        S.im += al * ((xp.im + xm.im) + (yp.im + ym.im) + (zp.im + zm.im));
        G[0].re += am * (xp.re - xm.re); G[0].im += am * (xp.im - xm.im);
        G[1].re += am * (yp.re - ym.re); G[1].im += am * (yp.im - ym.im);
        G[2].re += am * (zp.re - zm.re); G[2].im += am * (zp.im - zm.im);
      }
      const T cvk = w.centre + vcur[k];
      C acc{S.re + cvk * c0.re + (w.A[0] * G[0].im + w.A[1] * G[1].im + w.A[2] * G[2].im),
            S.im + cvk * c0.im - (w.A[0] * G[0].re + w.A[1] * G[1].re + w.A[2] * G[2].re)};
      if (args.want_density) {
        T dv[4] = {fn * (c0.re * c0.re + c0.im * c0.im), fn * (c0.re * G[0].im - c0.im * G[0].re),
                   fn * (c0.re * G[1].im - c0.im * G[1].re), fn * (c0.re * G[2].im - c0.im * G[2].re)};
#pragma unroll
        for (int i = 0; i < 4; ++i) dv[i] = group_sum<OC>(dv[i]);
        const int x = x0 + lxk[k], y = y0 + lyk[k];
        if (o == 0 && x < nx && y < ny) {
          const long long g = (long long)z * plane + (long long)(cv[k] / sizeof(T));
          T* dp = (T*)D.dpart + ((long long)chunk * D.n_grid + g) * 4;
          dp[0] = dv[0]; dp[1] = dv[1]; dp[2] = dv[2]; dp[3] = dv[3];
        }
      }
      if (ok[k]) {
        if (args.want_energy) e_acc += (double)fn * ((double)c0.re * acc.re + (double)c0.im * acc.im);
        if (args.occ_scale) { acc.re *= fn; acc.im *= fn; }
        const C b = base_is_u ? c0 : bcur[k];
        C r{cre * acc.re - cim * acc.im + b.re, cre * acc.im + cim * acc.re + b.im};
        *(C*)(ob + (long long)z * pbytes + co[k]) = r;
      }
    }
    if (!more) break;
    // plane z + 1 becomes the centre: its interior (queue slot R + 1) and halo
    // (halo-queue slot 0) go to the other LDS buffer, whose last readers
    // finished before the previous barrier
    C* Ln = lds + ((z + 1 - z_begin) & 1) * PLANE;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
#pragma unroll
      for (int s = 0; s < KQ - 1; ++s) q[k][s] = q[k][s + 1];
      q[k][KQ - 1] = qn[k];
      bcur[k] = bpf[k];
      vcur[k] = vpf[k];
      Ln[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
    }
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      if (hl[k] >= 0) Ln[hl[k]] = hq[k][0];
#pragma unroll
      for (int j = 0; j < R; ++j) hq[k][j] = hq[k][j + 1];
    }
    lds_barrier();
  }
  if (args.want_energy) {
    const double s = block_sum<double, NT / kWave>(e_acc, red);
    if (threadIdx.x == 0) D.e_loc[e_loc_slot<TX, TY>(D, it)] = s;
  }
}

// The sweep of k_stencil_sweep3 with every plane-to-plane move taken out of
// the loop.  The plane loop is unrolled by U = 2 (R + 1): the z queue becomes a
// ring of U register slots (plane p in slot (p - z_begin + R) mod U), the halo
// queue a ring of R + 1 slots, base and potential rings of two, and the LDS
// centre plane alternates between two buffers, so every index is static and
// each prefetch lands directly in the slot its plane will occupy.  GM selects
// which gradient axes are formed (bit d: axis d): the x and y axes are skipped
// when neither the field's component along them nor the current needs them.
// Calls f(integral_constant<int, 0>, ..., integral_constant<int, U - 1>).
template <typename F, int... Ps>
__device__ __forceinline__ void with_phases(F&& f, std::integer_sequence<int, Ps...>) {
  f(std::integral_constant<int, Ps>{}...);
}

template <typename T, int R, int OC, int TX, int TY, int NT, int GM, bool HB, bool EN, bool GR>
__device__ __forceinline__ void sweep4_body(const DomDesc& D, const Item& it, const StencilArgs& args,
                                            const StencilW<T>& w, Cplx<T>* lds, double* red) {
  using C = Cplx<T>;
  using Cfg = SweepCfg<R, OC, TX, TY, NT>;
  constexpr int KP = Cfg::kPer, KH = Cfg::kHPer, U = 2 * (R + 1), H = R + 1;
  constexpr int PLANE = Cfg::kLY * Cfg::kLX * OC;

  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb;
  const int x0 = it.a * TX, y0 = it.b * TY;
  const int chunk = it.c & 0xffff;
  const int zseg = it.c >> 16, oc0 = chunk * OC;
  const int z_begin = zseg * D.zseg, z_end = min(z_begin + D.zseg, nz);

  // HB: a base other than u is read (otherwise the base is u, or none)
  const bool base_is_u = args.base_slot == args.u_slot;
  const char* __restrict__ ub = (const char*)D.slot[args.u_slot];
  const char* __restrict__ bb = HB ? (const char*)D.slot[args.base_slot] : nullptr;
  // GR: the gradient partner v, read at each owned point (needs all three axes)
  static_assert(!GR || GM == 7, "the gradient partials need every axis");
  const char* __restrict__ gb = GR ? (const char*)D.slot[args.grad_slot] : nullptr;
  char* __restrict__ ob = (char*)D.slot[args.out_slot];
  const char* __restrict__ vb = (const char*)D.v;
  const T* __restrict__ occ = (const T*)D.occ;
  const long long plane = (long long)nx * ny;
  const long long pbytes = plane * no * (long long)sizeof(C);
  const long long vbytes = plane * (long long)sizeof(T);
  const T cre = (T)args.cre, cim = (T)args.cim;

  const int o = threadIdx.x % OC;
  const int tc = threadIdx.x / OC;
  const int n = oc0 + o;
  const bool n_ok = n < no;
  const int nl = n_ok ? n : no - 1;
  const T fn = n_ok ? occ[n] : (T)0;

  int lc[KP];                      // LDS index of the column's centre cell
  unsigned co[KP], cv[KP];
  bool ok[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int col = tc + k * Cfg::kThrCols;
    const int lx = col % TX, ly = col / TX;
    const int x = x0 + lx, y = y0 + ly;
    ok[k] = n_ok && x < nx && y < ny;
    lc[k] = ((ly + R) * Cfg::kLX + (lx + R)) * OC + o;
    const unsigned gc = (unsigned)(wrap(y, ny) * nx + wrap(x, nx));
    co[k] = (gc * (unsigned)no + (unsigned)nl) * (unsigned)sizeof(C);
    cv[k] = gc * (unsigned)sizeof(T);
  }
  // halo cells: slots past the strips write a scratch cell past both planes,
  // so every LDS store and every load is unconditional (straight-line code
  // lets the compiler wait for each prefetch by count)
  int hl[KH];
  unsigned ho[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hidx = tc + k * Cfg::kThrCols;
    int lx = R, ly = R;
    if (hidx < Cfg::kH) halo_xy<R, TX, TY>(hidx, lx, ly);
    hl[k] = hidx < Cfg::kH ? (ly * Cfg::kLX + lx) * OC + o : 2 * PLANE + o;
    const unsigned gc = (unsigned)(wrap(y0 + ly - R, ny) * nx + wrap(x0 + lx - R, nx));
    ho[k] = (gc * (unsigned)no + (unsigned)nl) * (unsigned)sizeof(C);
  }
  auto at = [&](const char* b, int z, unsigned off) -> C {
    return *(const C*)(b + (long long)z * pbytes + off);
  };
  auto vat = [&](int z, unsigned off) -> T { return *(const T*)(vb + (long long)z * vbytes + off); };

  C q[KP][U];          // plane p in slot (p - z_begin + R) % U
  C hq[KH][H];         // halo of plane p in slot (p - z_begin) % H
  C bq[KP][2];         // base of plane p in slot (p - z_begin) % 2
  T vq[KP][2];         // potential of plane p in slot (p - z_begin) % 2
  C gq[KP][2];         // GR: gradient partner of plane p in slot (p - z_begin) % 2

#pragma unroll
  for (int k = 0; k < KP; ++k) {
#pragma unroll
    for (int s = 0; s < 2 * R + 1; ++s) q[k][s] = at(ub, wrap(z_begin - R + s, nz), co[k]);
    if constexpr (HB) bq[k][0] = at(bb, z_begin, co[k]);
    if constexpr (GR) gq[k][0] = at(gb, z_begin, co[k]);
    vq[k][0] = vat(z_begin, cv[k]);
    lds[lc[k]] = q[k][R];
  }
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    lds[hl[k]] = at(ub, z_begin, ho[k]);
#pragma unroll
    for (int j = 1; j <= R; ++j) hq[k][j] = at(ub, wrap(z_begin + j, nz), ho[k]);
  }
  lds_barrier();

  double e_acc = 0.0;
  double g_acc[3] = {0.0, 0.0, 0.0};
  // one plane at phase P = (z - z_begin) % U; false once the segment is done
  auto plane_step = [&](auto PC, int z) -> bool {
    constexpr int P = decltype(PC)::value;
    const bool more = z + 1 < z_end;
    {
      // the next plane's loads, issued on the segment's last plane too (a
      // plane that exists: z + 1 clamped to the segment), unused then
      const int zq = wrap(z + 1 + R, nz), zn = more ? z + 1 : z;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        q[k][(P + 2 * R + 1) % U] = at(ub, zq, co[k]);
        if constexpr (HB) bq[k][(P + 1) % 2] = at(bb, zn, co[k]);
        if constexpr (GR) gq[k][(P + 1) % 2] = at(gb, zn, co[k]);
        vq[k][(P + 1) % 2] = vat(zn, cv[k]);
      }
#pragma unroll
      for (int k = 0; k < KH; ++k) hq[k][P % H] = at(ub, zq, ho[k]);
    }
    const C* L = lds + (P % 2) * PLANE;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const C c0 = q[k][(P + R) % U];
      C S{0, 0}, G[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        const C xp = L[lc[k] + m * OC], xm = L[lc[k] - m * OC];
        const C yp = L[lc[k] + m * Cfg::kLX * OC], ym = L[lc[k] - m * Cfg::kLX * OC];
        const C zp = q[k][(P + R + m) % U], zm = q[k][(P + R - m) % U];
        const T al = w.alpha[m - 1], am = w.a1[m - 1];
        S.re += al * ((xp.re + xm.re) + (yp.re + ym.re) + (zp.re + zm.re));
        S.im += al * ((xp.im + xm.im) + (yp.im + ym.im) + (zp.im + zm.im));
        if constexpr (GM & 1) { G[0].re += am * (xp.re - xm.re); G[0].im += am * (xp.im - xm.im); }
        if constexpr (GM & 2) { G[1].re += am * (yp.re - ym.re); G[1].im += am * (yp.im - ym.im); }
        if constexpr (GM & 4) { G[2].re += am * (zp.re - zm.re); G[2].im += am * (zp.im - zm.im); }
      }
      const T cvk = w.centre + vq[k][P % 2];
      T agi = 0, agr = 0;                    // A.G (imaginary and real parts)
      if constexpr (GM & 1) { agi += w.A[0] * G[0].im; agr += w.A[0] * G[0].re; }
      if constexpr (GM & 2) { agi += w.A[1] * G[1].im; agr += w.A[1] * G[1].re; }
      if constexpr (GM & 4) { agi += w.A[2] * G[2].im; agr += w.A[2] * G[2].re; }
      C acc{S.re + cvk * c0.re + agi, S.im + cvk * c0.im - agr};
      if constexpr (GM == 7) {
        if (args.want_density) {
          T dv[4] = {fn * (c0.re * c0.re + c0.im * c0.im), fn * (c0.re * G[0].im - c0.im * G[0].re),
                     fn * (c0.re * G[1].im - c0.im * G[1].re), fn * (c0.re * G[2].im - c0.im * G[2].re)};
#pragma unroll
          for (int i = 0; i < 4; ++i) dv[i] = group_sum<OC>(dv[i]);
          const int col = tc + k * Cfg::kThrCols;
          const int x = x0 + col % TX, y = y0 + col / TX;
          if (o == 0 && x < nx && y < ny) {
            const long long g = (long long)z * plane + (long long)(cv[k] / sizeof(T));
            T* dp = (T*)D.dpart + ((long long)chunk * D.n_grid + g) * 4;
            dp[0] = dv[0]; dp[1] = dv[1]; dp[2] = dv[2]; dp[3] = dv[3];
          }
        }
      }
      if (ok[k]) {
        if constexpr (GR) {
          // t_d = (-i D1_d + A_d) u at this point; conj(t_d) v, times the coefficient
          const C v = gq[k][P % 2];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const T tre = w.A[d] * c0.re + G[d].im, tim = w.A[d] * c0.im - G[d].re;
            const double pr = (double)tre * v.re + (double)tim * v.im;
            const double pi = (double)tre * v.im - (double)tim * v.re;
            g_acc[d] += args.gre * pr - args.gim * pi;
          }
        }
        if constexpr (EN) e_acc += (double)fn * ((double)c0.re * acc.re + (double)c0.im * acc.im);
        if (args.occ_scale) { acc.re *= fn; acc.im *= fn; }
        C b = base_is_u ? c0 : C{0, 0};
        if constexpr (HB) b = bq[k][P % 2];
        *(C*)(ob + (long long)z * pbytes + co[k]) =
            C{cre * acc.re - cim * acc.im + b.re, cre * acc.im + cim * acc.re + b.im};
      }
    }
    if (!more) return false;
    // plane z + 1 becomes the centre: its interior and halo go to the other
    // LDS buffer, whose readers finished before the previous barrier
    C* Ln = lds + ((P + 1) % 2) * PLANE;
#pragma unroll
    for (int k = 0; k < KP; ++k) Ln[lc[k]] = q[k][(P + R + 1) % U];
#pragma unroll
    for (int k = 0; k < KH; ++k) Ln[hl[k]] = hq[k][(P + 1) % H];
    lds_barrier();
    return true;
  };
  auto run = [&](auto... PCs) {
    for (int z = z_begin; z < z_end; z += U)
      if (!(plane_step(PCs, z + decltype(PCs)::value) && ...)) break;
  };
  with_phases(run, std::make_integer_sequence<int, U>{});
  if constexpr (EN) {
    const double s = block_sum<double, NT / kWave>(e_acc, red);
    if (threadIdx.x == 0) D.e_loc[e_loc_slot<TX, TY>(D, it)] = s;
  }
  if constexpr (GR) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double s = block_sum<double, NT / kWave>(g_acc[d], red);
      if (threadIdx.x == 0) D.g_part[(long long)e_loc_slot<TX, TY>(D, it) * 3 + d] = s;
    }
  }
}

// GRK: the adjoint's sweep (every axis, no base, energy or density, the
// pulse-gradient partials of args.grad_slot formed in passing); a kernel of its
// own, so the extra registers it needs do not weigh on the other sweeps.
template <typename T, int R, int OC, int TX, int TY, int NT, bool GRK = false>
__global__ __launch_bounds__(NT) void k_stencil_sweep4(const DomDesc* __restrict__ doms,
                                                       const Item* __restrict__ items,
                                                       StencilArgs args) {
  using Cfg = SweepCfg<R, OC, TX, TY, NT>;
  // two centre planes, then one scratch cell per orbital lane for the halo
  // slots past the strips
  __shared__ Cplx<T> lds[2 * Cfg::kLY * Cfg::kLX * OC + OC];
  __shared__ double red[NT / kWave];
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const StencilW<T> w = stencil_weights<T>(D, args.step);
  const bool hb = args.base_slot < SLOT_NONE && args.base_slot != args.u_slot;
  // The energy flag is a template argument: as a run-time flag the compiler
  // evaluates every point's FP64 energy term and discards it with a select.
  // The twelve bodies are forced inline: left to itself the compiler outlines
  // them as calls with a private stack.
  auto body = [&](auto hbc, auto enc) __attribute__((always_inline)) {
    constexpr bool HB = decltype(hbc)::value, EN = decltype(enc)::value;
    if (args.want_density || w.A[0] != (T)0 || w.A[1] != (T)0)
      sweep4_body<T, R, OC, TX, TY, NT, 7, HB, EN, false>(D, it, args, w, lds, red);
    else if (w.A[2] != (T)0)
      sweep4_body<T, R, OC, TX, TY, NT, 4, HB, EN, false>(D, it, args, w, lds, red);
    else
      sweep4_body<T, R, OC, TX, TY, NT, 0, HB, EN, false>(D, it, args, w, lds, red);
  };
  auto with_en = [&](auto hbc) __attribute__((always_inline)) {
    if (args.want_energy)
      body(hbc, std::true_type{});
    else
      body(hbc, std::false_type{});
  };
  if constexpr (GRK) {
    // the adjoint applies H to mu with no base term (the host passes none)
    sweep4_body<T, R, OC, TX, TY, NT, 7, false, false, true>(D, it, args, w, lds, red);
  } else if (hb) {
    with_en(std::true_type{});
  } else {
    with_en(std::false_type{});
  }
}

// rho[g] = sum_chunks dpart[c][g][0];  j[g][d] = sum_chunks dpart[c][g][1 + d] + A_d rho.
// Items: (dom, block of 256 grid points).  step: A sample; obs: output row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_density_finish(const DomDesc* __restrict__ doms,
                                                           const Item* __restrict__ items, int step, int obs) {
  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const long long g = (long long)it.a * kBlock + threadIdx.x;
  if (g >= D.n_grid) return;
  const int nch = D.n_chunks;
  T s[4] = {0, 0, 0, 0};
  for (int c = 0; c < nch; ++c) {
    const T* dp = (const T*)D.dpart + ((long long)c * D.n_grid + g) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += dp[i];
  }
  const double* A = D.a + (long long)step * D.a_stride;
  if (D.rho) ((T*)D.rho)[(long long)obs * D.n_grid + g] = s[0];
  if (D.jcur) {
    T* j = (T*)D.jcur + ((long long)obs * D.n_grid + g) * 3;
    j[0] = s[1] + (T)A[0] * s[0];
    j[1] = s[2] + (T)A[1] * s[0];
    j[2] = s[3] + (T)A[2] * s[0];
  }
}

}  // namespace dcm

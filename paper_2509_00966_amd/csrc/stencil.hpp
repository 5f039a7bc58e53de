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
// arms, no corners).  Each u value leaves HBM about once per sweep plus the
// halo strips, and the lanes of a wave touch OC consecutive orbitals of
// consecutive points.
#pragma once

#include "common.hpp"

namespace dcm {

struct StencilArgs {
  int u_slot, base_slot, out_slot;  // base_slot == SLOT_NONE: no base term
  double cre, cim;                  // coef
  int occ_scale;                    // multiply H_loc u by f_n
  int step;                         // A sample index
  int want_energy;                  // accumulate f_n Re(conj(u) H_loc u)
};

template <typename T>
struct StencilW {
  T alpha[3];       // -1/2 c_m / h^2, m = 1..r
  T beta[3][3];     // A_d a_m / h
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
    w.beta[0][m - 1] = on ? (T)(a0 * fd1(D.r, m) * ih) : (T)0;
    w.beta[1][m - 1] = on ? (T)(a1 * fd1(D.r, m) * ih) : (T)0;
    w.beta[2][m - 1] = on ? (T)(a2 * fd1(D.r, m) * ih) : (T)0;
  }
  w.centre = (T)(-1.5 * fd2(D.r, 0) * ih2 + 0.5 * (a0 * a0 + a1 * a1 + a2 * a2));
  return w;
}

// m-th neighbour pair along one axis: alpha (u+ + u-) - i beta (u+ - u-)
template <typename T>
__device__ __forceinline__ void pair_add(Cplx<T>& acc, Cplx<T> up, Cplx<T> um, T alpha, T beta) {
  const T sr = up.re + um.re, si = up.im + um.im;
  const T tr = up.re - um.re, ti = up.im - um.im;
  acc.re += alpha * sr + beta * ti;
  acc.im += alpha * si - beta * tr;
}

template <int R, int OC, int TX, int TY>
struct SweepCfg {
  static constexpr int kCols = TX * TY;            // (x, y) columns per tile
  static constexpr int kThrCols = kBlock / OC;     // columns covered by one pass of the block
  static constexpr int kPer = kCols / kThrCols;    // columns per thread
  static constexpr int kLX = TX + 2 * R;           // LDS plane with halo
  static constexpr int kLY = TY + 2 * R;
  static constexpr int kQ = 2 * R + 1;             // z queue depth
  static_assert(kBlock % OC == 0 && kCols % kThrCols == 0, "tile does not fit the block");
};

// Items: (dom, x tile, y tile, (z segment << 16) | orbital chunk).
// D.zseg planes per segment.  Energy partials: one per item, at
// e_loc[blockIdx.x - D.item0_stencil].
template <typename T, int R, int OC, int TX, int TY>
__global__ __launch_bounds__(kBlock) void k_stencil_sweep(const DomDesc* __restrict__ doms,
                                                          const Item* __restrict__ items,
                                                          StencilArgs args) {
  using C = Cplx<T>;
  using Cfg = SweepCfg<R, OC, TX, TY>;
  __shared__ C lds[Cfg::kLY * Cfg::kLX * OC];
  __shared__ double red[4];

  const Item it = items[blockIdx.x];
  const DomDesc& D = doms[it.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz, no = D.n_orb;
  const int x0 = it.a * TX, y0 = it.b * TY;
  const int zseg = it.c >> 16, oc0 = (it.c & 0xffff) * OC;
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

  // Columns of this thread.  Loads use wrapped coordinates so that slots past
  // the domain edge hold the periodic images needed by the last valid column.
  int lxk[Cfg::kPer], lyk[Cfg::kPer];
  long long gcol[Cfg::kPer];       // (y*nx + x) of the column, wrapped
  bool ok[Cfg::kPer];
#pragma unroll
  for (int k = 0; k < Cfg::kPer; ++k) {
    const int col = tc + k * Cfg::kThrCols;
    lxk[k] = col % TX;
    lyk[k] = col / TX;
    const int x = x0 + lxk[k], y = y0 + lyk[k];
    ok[k] = n_ok && x < nx && y < ny;
    gcol[k] = (long long)wrap(y, ny) * nx + wrap(x, nx);
  }
  const long long plane = (long long)nx * ny;

  C q[Cfg::kPer][Cfg::kQ];   // q[k][s] = plane z - R + s
#pragma unroll
  for (int k = 0; k < Cfg::kPer; ++k)
#pragma unroll
    for (int s = 0; s < Cfg::kQ - 1; ++s) {
      const int zz = wrap(z_begin - R + s, nz);
      q[k][s + 1] = n_ok ? u[((long long)zz * plane + gcol[k]) * no + n] : C{0, 0};
    }

  double e_acc = 0.0;
  for (int z = z_begin; z < z_end; ++z) {
    const int zf = wrap(z + R, nz);
#pragma unroll
    for (int k = 0; k < Cfg::kPer; ++k) {
#pragma unroll
      for (int s = 0; s < Cfg::kQ - 1; ++s) q[k][s] = q[k][s + 1];
      q[k][Cfg::kQ - 1] = n_ok ? u[((long long)zf * plane + gcol[k]) * no + n] : C{0, 0};
      lds[((lyk[k] + R) * Cfg::kLX + (lxk[k] + R)) * OC + o] = q[k][R];
    }
    constexpr int kHx = 2 * R * TY, kHy = 2 * R * TX, kH = kHx + kHy;
    for (int hidx = tc; hidx < kH; hidx += Cfg::kThrCols) {
      int lx, ly;
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
      const int xx = wrap(x0 + lx - R, nx), yy = wrap(y0 + ly - R, ny);
      lds[(ly * Cfg::kLX + lx) * OC + o] =
          n_ok ? u[(((long long)z * ny + yy) * nx + xx) * no + n] : C{0, 0};
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < Cfg::kPer; ++k) {
      const int cx = lxk[k] + R, cy = lyk[k] + R;
      const C c0 = q[k][R];
      const long long g = (long long)z * plane + gcol[k];
      const T vg = ok[k] ? V[g] : (T)0;
      C acc{(w.centre + vg) * c0.re, (w.centre + vg) * c0.im};
#pragma unroll
      for (int m = 1; m <= R; ++m) {
        pair_add(acc, lds[(cy * Cfg::kLX + cx + m) * OC + o], lds[(cy * Cfg::kLX + cx - m) * OC + o],
                 w.alpha[m - 1], w.beta[0][m - 1]);
        pair_add(acc, lds[((cy + m) * Cfg::kLX + cx) * OC + o], lds[((cy - m) * Cfg::kLX + cx) * OC + o],
                 w.alpha[m - 1], w.beta[1][m - 1]);
        pair_add(acc, q[k][R + m], q[k][R - m], w.alpha[m - 1], w.beta[2][m - 1]);
      }
      if (ok[k]) {
        if (args.want_energy) e_acc += (double)fn * ((double)c0.re * acc.re + (double)c0.im * acc.im);
        if (args.occ_scale) { acc.re *= fn; acc.im *= fn; }
        C r{cre * acc.re - cim * acc.im, cre * acc.im + cim * acc.re};
        if (base) { const C b = base[g * no + n]; r.re += b.re; r.im += b.im; }
        out[g * no + n] = r;
      }
    }
    __syncthreads();
  }
  if (args.want_energy) {
    const double s = block_sum(e_acc, red);
    if (threadIdx.x == 0) D.e_loc[blockIdx.x - D.item0_stencil] = s;
  }
}

}  // namespace dcm

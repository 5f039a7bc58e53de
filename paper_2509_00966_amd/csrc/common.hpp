// Shared device-side types for the Kohn-Sham step kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcm {

constexpr int kWave = 64;
constexpr int kBlock = 256;   // four waves per block everywhere

// Buffers a kernel can address through a domain descriptor.
enum Slot : int {
  SLOT_PSI = 0,     // caller's orbitals
  SLOT_B0 = 1,      // workspace psi-sized buffers
  SLOT_B1 = 2,
  SLOT_B2 = 3,
  SLOT_B3 = 4,
  SLOT_B4 = 5,
  SLOT_LAMBDA = 6,  // caller's adjoint state
  SLOT_HPSI = 7,    // caller's f_n H psi_n output
  SLOT_NONE = 8,
  N_SLOTS = 8
};

// Every pointer a kernel reaches through a domain descriptor addresses device
// memory.  The device pass declares the descriptor's pointer fields in the
// global address space, so that the compiler emits global (not flat) loads and
// stores for everything derived from them: a flat access also counts against
// the LDS wait counter, which would make each LDS wait in a kernel wait for its
// outstanding prefetches too.  The host pass sees the same layout with plain
// pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define DCM_GLOBAL __attribute__((address_space(1)))
#else
#define DCM_GLOBAL
#endif

// Host code stores device addresses into descriptor fields through this cast.
template <typename T>
__host__ __device__ inline DCM_GLOBAL T* as_global(T* p) { return (DCM_GLOBAL T*)p; }

// One domain as the kernels see it.  Built on the host, copied into the head
// of the workspace once per call.
struct DomDesc {
  int nx, ny, nz, r;            // grid edges, stencil half-width
  int n_orb, n_proj;
  long long n_grid;
  double h;
  DCM_GLOBAL void* slot[N_SLOTS];          // psi-sized complex buffers
  const DCM_GLOBAL void* v;                // [N_g] real
  const DCM_GLOBAL void* proj;             // [N_g][n_proj] complex
  const DCM_GLOBAL void* d;                // [n_proj] real
  const DCM_GLOBAL void* occ;              // [n_orb] real
  const DCM_GLOBAL double* a;              // A samples of this domain, [.][3]
  long long a_stride;           // doubles between steps (3) -- kept general
  // workspace (accumulation type of the projector products)
  DCM_GLOBAL void* ppart;                  // [n_split][n_proj][2 n_orb] split-K partials
  DCM_GLOBAL void* pmat;                   // [n_proj][2 n_orb]  P = h^3 B^H u
  DCM_GLOBAL void* qmat;                   // [2 n_proj][ldq] real form of coef D P
  long long ldq;                // row stride of qmat: 2 n_orb rounded up to 4
  DCM_GLOBAL void* qmat3;                  // FP32: [3][n_proj][ldq3] Re Q, Im Q - Re Q, Re Q + Im Q (null otherwise)
  long long ldq3;               // n_orb rounded up to 4
  DCM_GLOBAL double* e_loc;                // [n_stencil_items] local-energy partials
  DCM_GLOBAL double* e_nl;                 // [n_reduce_items] nonlocal-energy partials
  DCM_GLOBAL double* g_part;               // [n_grad_items][3] gradient partials
  int n_split;                  // projection split-K count
  int split_len;                // grid points per split
  int zseg;                     // z planes per stencil sweep segment
  int n_e_loc, n_e_nl, n_g_part;
  int item0_reduce;             // ... in its reduce launch
  int item0_elem;               // ... in its elementwise launch
  int n_chunks;                 // orbital chunks of the stencil sweep
  int item0_rows;               // first item of this domain in its row-block launch
  int n_rows_blocks;            // row blocks (256 grid points) of the domain
  DCM_GLOBAL double* cn_part;              // [n_rows_blocks][n_orb] column-norm partials
  DCM_GLOBAL double* cn_inv;               // [n_orb] inverse column norms
  DCM_GLOBAL void* dpart;                  // [n_chunks][N_g][4] density / current partials
  // per-step observables (may be null)
  DCM_GLOBAL void* rho;                    // [.][N_g]
  DCM_GLOBAL void* jcur;                   // [.][N_g][3]
  DCM_GLOBAL double* energy;               // [.]
  DCM_GLOBAL double* grad;                 // [3] gradient accumulator (adjoint)
  DCM_GLOBAL double* overlap;              // [n_orb][n_orb] complex128
  DCM_GLOBAL double* smat;                 // workspace [n_orb][n_orb] complex128 (cross overlap)
  DCM_GLOBAL double* f_occ;                // [n_orb] occupations of the reference orbitals
  DCM_GLOBAL double* n_exc;                // one value: electrons outside the reference span
  int item0_occ;                // first item of this domain in its occupation-row launch
  // macroscopic current and the Maxwell update of the field
  const DCM_GLOBAL void* proj_r;   // [3][N_g][n_proj] complex position-weighted projectors (or null)
  const DCM_GLOBAL double* a_ext;  // [n_steps + 1][3] external field at the step times (Maxwell steps)
  DCM_GLOBAL double* jpart;        // [n_dens_items][4] block sums of rho and the paramagnetic current
  DCM_GLOBAL double* jnl_part;     // [3][n_e_nl] block sums of the nonlocal current
  DCM_GLOBAL double* cur;          // [3] macroscopic current density
  DCM_GLOBAL double* cur_out;      // [n_steps][3] per-step currents (Maxwell steps, or null)
  DCM_GLOBAL double* field;        // [6] induced field and its rate (Maxwell steps)
  DCM_GLOBAL double* amid;         // [n_steps][3] step fields written by the Maxwell update
  int item0_dens;                  // first item of this domain in its density launch
  int n_dens;                      // density items of this domain
  // split-precision operands (16-bit hi and lo planes), null otherwise
  DCM_GLOBAL void* bs_hi; DCM_GLOBAL void* bs_lo;    // [N_g][ldbs]       projectors as stored
  DCM_GLOBAL void* bt_hi; DCM_GLOBAL void* bt_lo;    // [n_proj][ldbt]    projectors transposed
  DCM_GLOBAL void* qt_hi; DCM_GLOBAL void* qt_lo;    // [2 n_orb][ldqt]   transposed real form of coef D P
  DCM_GLOBAL unsigned* maxbits;            // [4]: max |B|, max |u|, max |Q'| as float bits (FP16 scaling)
  long long ldbs, ldbt, ldqt;   // row strides (halves) of bs, bt, qt: multiples of 8, zero padded
};

// A unit of work: which domain, and up to three tile coordinates.
struct Item {
  int dom, a, b, c;
};

template <typename T> struct Cplx { T re, im; };

// Central finite-difference weights (second and first derivative), indexed by
// half-width r = 1..3: c[0] is the centre weight of the second derivative.
__device__ __forceinline__ double fd2(int r, int m) {
  // r = 1: (-2, 1); r = 2: (-5/2, 4/3, -1/12); r = 3: (-49/18, 3/2, -3/20, 1/90)
  if (r == 1) return m == 0 ? -2.0 : 1.0;
  if (r == 2) return m == 0 ? -2.5 : (m == 1 ? 4.0 / 3.0 : -1.0 / 12.0);
  return m == 0 ? -49.0 / 18.0 : (m == 1 ? 1.5 : (m == 2 ? -0.15 : 1.0 / 90.0));
}
__device__ __forceinline__ double fd1(int r, int m) {
  // r = 1: (1/2); r = 2: (2/3, -1/12); r = 3: (3/4, -3/20, 1/60)
  if (r == 1) return 0.5;
  if (r == 2) return m == 1 ? 2.0 / 3.0 : -1.0 / 12.0;
  return m == 1 ? 0.75 : (m == 2 ? -0.15 : 1.0 / 60.0);
}

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// x as read from another lane of the same 16-lane row (DPP lane selection
// CTRL), for any 4-byte-multiple type.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_mov(T x) {
  static_assert(sizeof(T) % 4 == 0, "DPP moves 32-bit words");
  struct Words { int w[sizeof(T) / 4]; };
  Words a = __builtin_bit_cast(Words, x);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) a.w[i] = __builtin_amdgcn_mov_dpp(a.w[i], CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(T, a);
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8 or 16), valid in every
// lane of the group: swaps within pairs and quads, then the mirrored half of
// each 8 and of each 16 lanes.  Lane 0 of a group adds in the same order as
// the xor butterfly (v0 + v1) + (v2 + v3) + ..., with no LDS traffic.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  if constexpr (G >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  if constexpr (G >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
  if constexpr (G >= 16) v += dpp_mov<0x140>(v);  // row_mirror
  return v;
}

// Left operand of a projection: a psi-sized slot (a_slot >= 0), the
// projectors B (-1), or component d of the position-weighted projectors
// B_d = (r - R_atom)_d B (-2 - d).  ES: bytes of one real element.
template <int ES>
__device__ __forceinline__ const DCM_GLOBAL char* proj_operand(const DomDesc& D, int a_slot) {
  if (a_slot >= 0) return (const DCM_GLOBAL char*)D.slot[a_slot];
  if (a_slot == -1) return (const DCM_GLOBAL char*)D.proj;
  return (const DCM_GLOBAL char*)D.proj_r + (long long)(-2 - a_slot) * D.n_grid * D.n_proj * 2 * ES;
}

// Barrier for an LDS exchange: waits for this wave's own LDS reads and
// writes (lgkmcnt(0)), then for the other waves.  Global loads stay in flight
// across it: a __syncthreads() fence would also wait for every prefetch in
// flight, draining the memory pipeline at each stage.  The registers those
// loads fill are waited for where they are used.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt not waited
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Sum over a block of NW waves (lds holds NW values); result valid in
// thread 0, added in wave order.
template <typename T, int NW = kBlock / kWave>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
  __syncthreads();
  T s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; ++i) s += lds[i];
  __syncthreads();
  return s;
}

}  // namespace dcm

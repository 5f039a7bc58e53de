/*
 * dcmesh.h -- C ABI of the MI355X real-time Kohn-Sham step library.
 *
 * The library advances complex Kohn-Sham orbitals on periodic real-space grids
 * ("domains" of the divide-and-conquer scheme, Sec. V.A.1) by the step
 *     psi <- T4(-i dt H(A_k)) psi,   T4(z) = sum_{m=0}^{4} z^m / m!,
 * the fourth-order Taylor form of exp(-i dt H) (Eq. 2 with the full H), with
 *     H(A) = -1/2 Lap_h - i A.grad_h + 1/2 |A|^2 + v_loc + B diag(D) h^3 B^H
 * (Eq. 3 in atomic units: hbar = m = 1, e/c folded into A; the nonlocal part as
 * the two dense products of Sec. V.B.5).  Lap_h and grad_h are periodic central
 * finite differences of order 2, 4 or 6.  A_k is the vector potential at the
 * step midpoint t_k + dt/2 (the midpoint rule of Eq. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid point g = (z*ny + y)*nx + x sits at r = h*(x, y, z).  Inner product
 * <a|b> = h^3 sum_g conj(a_g) b_g.
 * Layouts (row-major, the orbital index fastest: the structure-of-arrays
 * layout of Sec. V.B.2):
 *     psi   [N_g][n_orb]  complex (interleaved re, im)
 *     proj  [N_g][n_proj] complex  (columns beta_p)
 *     v_loc [N_g], d [n_proj], occ [n_orb]  real
 * Element types follow the precision mode:
 *     DCMESH_FP64                         complex128 / float64
 *     DCMESH_FP32, DCMESH_SPLIT_BF16/FP16  complex64  / float32
 * Energies, gradients, overlaps and A samples are always float64.
 *
 * Ownership: every pointer inside a call's arguments is caller-owned device
 * memory (unless stated as host) and must stay valid until the work queued on
 * the stream has finished.  The library allocates no device memory; scratch
 * space is the caller's workspace, sized by dcmesh_workspace_bytes, whose
 * contents are private to the library between calls.  The library keeps no
 * device pointer after a call returns, except inside a graph handle.
 *
 * Work lists: each call copies its domain descriptors and tile lists into the
 * head of the workspace from pinned host memory that the library keeps
 * between calls, one buffer per distinct table content (at most 64 idle ones
 * are kept).  A call whose tables are not staged yet allocates such a buffer
 * (hipHostMalloc) and an event; nothing else is allocated.
 *
 * Streams: all work is queued on the given stream (a hipStream_t passed as
 * void*, NULL = the default stream) and calls return without waiting for it.
 * No entry point synchronises or reads device memory on the host unless
 * DCMESH_FLAG_CHECK_FINITE is set.  A call made under stream capture must find
 * its tables staged (the allocation above is not allowed there):
 * dcmesh_graph_create stages them before it captures, and dcmesh_step_noalloc
 * needs no staging.
 *
 * Errors: each entry point returns a DCMESH_* status; 0 means success.  All
 * arguments are validated on the host before any HIP call, so an invalid
 * argument leaves the stream untouched.  dcmesh_last_error() gives a message
 * for the calling thread's last failure.
 */
#ifndef DCMESH_H
#define DCMESH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum dcmesh_status {
  DCMESH_OK = 0,
  DCMESH_ERR_INVALID_ARGUMENT = 1,  /* a null pointer, a bad size or order */
  DCMESH_ERR_UNSUPPORTED = 2,       /* a valid request this build cannot run */
  DCMESH_ERR_WORKSPACE = 3,         /* workspace missing, too small or misaligned */
  DCMESH_ERR_HIP = 4,               /* a HIP runtime call failed */
  DCMESH_ERR_NONFINITE = 5          /* CHECK_FINITE found a NaN/Inf in psi */
};

enum dcmesh_precision {
  DCMESH_FP64 = 0,        /* complex128 everywhere, FP64 matrix cores */
  DCMESH_FP32 = 1,        /* complex64; projector products on FP32 matrix cores */
  DCMESH_SPLIT_BF16 = 2,  /* complex64; projector products as BF16 hi+lo, FP32 accumulation */
  DCMESH_SPLIT_FP16 = 3   /* complex64; projector products as FP16 hi+lo (power-of-two scaled) */
};

/* Flags (bitwise or). */
#define DCMESH_FLAG_CHECK_FINITE 0x1u  /* synchronise after the call and test psi for NaN/Inf */
#define DCMESH_FLAG_PROFILE 0x2u       /* bracket every kernel launch with HIP events on the
                                          call's stream; read with dcmesh_profile_collect */
#define DCMESH_FLAG_EQ2 0x4u           /* dcmesh_workspace_bytes: size for dcmesh_step_eq2 */

/* Kernel families reported by dcmesh_profile_collect. */
enum dcmesh_family {
  DCMESH_FAM_STENCIL = 0,   /* local H sweep fused with the Taylor-stage update */
  DCMESH_FAM_PROJECT = 1,   /* P = h^3 B^H u, split-K partials */
  DCMESH_FAM_REDUCE = 2,    /* split-K sum, coef D P and its real form */
  DCMESH_FAM_CORRECT = 3,   /* out += B (coef D P) */
  DCMESH_FAM_DENSITY = 4,   /* rho and j */
  DCMESH_FAM_ENERGY = 5,    /* energy finalisation */
  DCMESH_FAM_ADJOINT = 6,   /* gradient inner products and lambda accumulation */
  DCMESH_FAM_OVERLAP = 7,   /* S = h^3 Psi^H Psi */
  DCMESH_FAM_SPLIT = 8,     /* hi/lo operand preparation of the split modes */
  DCMESH_N_FAMILIES = 9
};

/* One periodic domain.  nx, ny, nz >= fd_order + 1; fd_order in {2, 4, 6};
 * n_orb >= 1; n_proj >= 0 (0: no nonlocal term, proj and d may be NULL). */
typedef struct dcmesh_domain {
  int32_t nx, ny, nz;
  int32_t fd_order;
  int32_t n_orb;
  int32_t n_proj;
  double h;               /* mesh spacing (bohr), > 0 */
  void* psi;              /* [N_g][n_orb] complex, in/out */
  const void* v_loc;      /* [N_g] real (Ha) */
  const void* proj;       /* [N_g][n_proj] complex */
  const void* d;          /* [n_proj] real (Ha) */
  const void* occ;        /* [n_orb] real occupations f_n */
} dcmesh_domain;

/* Per-step observables of one domain for dcmesh_step.  Entry k refers to the
 * state entering step k, evaluated with that step's field A_k.  Any pointer may
 * be NULL (not computed).
 *   rho    [n_steps][N_g]     real   rho = sum_n f_n |psi_n|^2
 *   j      [n_steps][N_g][3]  real   j = sum_n f_n [Im(conj psi_n grad_h psi_n) + A |psi_n|^2]
 *   energy [n_steps]          float64  E = h^3 sum_n f_n <psi_n|H(A_k)|psi_n> */
typedef struct dcmesh_obs {
  void* rho;
  void* j;
  double* energy;
} dcmesh_obs;

/* Outputs of dcmesh_density for one domain (any may be NULL).
 *   rho [N_g], j [N_g][3]  real, as in dcmesh_obs
 *   energy                 one float64, E = h^3 sum_n f_n <psi_n|H(A)|psi_n>
 *   hpsi_occ [N_g][n_orb]  complex, f_n H(A) psi_n (the adjoint seed of E)
 *   overlap [n_orb][n_orb] complex128, S = h^3 Psi^H Psi accumulated in FP64 */
typedef struct dcmesh_density_out {
  void* rho;
  void* j;
  double* energy;
  void* hpsi_occ;
  double* overlap;
} dcmesh_density_out;

/* Not in the paper (the caller-owned scratch of the calls below).
 * Workspace needed by every entry point below (one size serves all, except
 * dcmesh_step_eq2: DCMESH_FLAG_EQ2) for these domains and precision.  Host-only; writes
 * *bytes.  Workspace pointers must be 256-byte aligned. */
int dcmesh_workspace_bytes(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                           uint32_t flags, size_t* bytes);

/* Advance every domain by n_steps Taylor-4 steps (Eq. 2 structure, full H).
 *   doms      host array [n_dom]
 *   a_dev     device float64 A samples, [n_a][a_stride][3] with n_a = n_dom if
 *             a_per_domain else 1; step k of this call uses a_dev[.][k][:]
 *   dt        time step (a.u.); n_steps >= 0
 *   obs       NULL or host array [n_dom] of per-step observable outputs
 *   work      device workspace of work_bytes >= dcmesh_workspace_bytes(...)
 *   stream    hipStream_t */
int dcmesh_step(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                const double* a_dev, int32_t a_per_domain, int64_t a_stride,
                double dt, int32_t n_steps, const dcmesh_obs* obs,
                void* work, size_t work_bytes, uint32_t flags, void* stream);

/* dcmesh_step without a workspace argument, for callers that cannot allocate
 * device memory: work recorded under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The workspace is a static device array of
 * 64 MiB (2^26 bytes) that every GPU the library runs on holds until the
 * process ends; domains that need more (dcmesh_workspace_bytes) make the call
 * fail with DCMESH_ERR_WORKSPACE before any HIP call.  The call allocates
 * nothing: no device memory, no pinned staging buffer (the work lists reach the
 * array through kernel arguments), no events (DCMESH_FLAG_PROFILE is
 * rejected).  The array keeps the last call's contents; every call writes
 * whatever it later reads, so nothing needs clearing between calls.  All calls
 * on one GPU share its array: calls that overlap on one GPU (two streams, two
 * threads) race, and the caller must serialise them.  Other arguments,
 * results and errors as dcmesh_step (bitwise the same results). */
int dcmesh_step_noalloc(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                        const double* a_dev, int32_t a_per_domain, int64_t a_stride,
                        double dt, int32_t n_steps, const dcmesh_obs* obs,
                        uint32_t flags, void* stream);

/* Eq. 2 with the nonlocal operator of Eq. 5: every step applies
 *     N T4(-i dt h_loc(A_k)) N,   N psi = (psi - delta Psi0 h^3 Psi0^H psi) / |.|,
 *     delta = i dt v_nl / 2,
 * i.e. normalised half-steps of the reference-orbital projector v_nl
 * |Psi0><Psi0| (Eq. 5's Psi(t) -= delta Psi(0) Psi^H(0) Psi(t), each orbital
 * rescaled to unit norm) around the fourth-order Taylor propagator of the local
 * Hamiltonian.  The domains' proj and d are ignored.  psi0: host array [n_dom]
 * of device pointers, [N_g][n_orb] complex, the reference orbitals.  FP64 and
 * FP32 only.  Workspace: dcmesh_workspace_bytes with DCMESH_FLAG_EQ2. */
int dcmesh_step_eq2(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                    const void* const* psi0, double v_nl,
                    const double* a_dev, int32_t a_per_domain, int64_t a_stride,
                    double dt, int32_t n_steps,
                    void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Observables of the current orbitals for the field a_dev ([n_a][3], float64,
 * device): the density and current that couple the orbitals to the field
 * (Sec. V.B.5), the energy E = h^3 sum_n f_n <psi_n|H|psi_n> of Eq. 3's H, its
 * adjoint seed f_n H psi_n, and the FP64 overlap S = h^3 Psi^H Psi (the
 * orthonormality check; Sec. V.B.5's overlap product).  out: host array
 * [n_dom]. */
int dcmesh_density(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                   const double* a_dev, int32_t a_per_domain,
                   const dcmesh_density_out* out,
                   void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Occupations of the reference orbitals and the number of excited electrons,
 * the quantities the local field dynamics hands to the atomic dynamics
 * (Sec. V.A.3 and V.A.8).  With the reference orbitals psi0 (Eq. 5's Psi(0)):
 *     S_sn  = h^3 <psi0_s | psi_n>                          (FP64 accumulation)
 *     f_s   = sum_n f_n |S_sn|^2
 *     n_exc = sum_n f_n (h^3 <psi_n|psi_n> - sum_s |S_sn|^2)
 * n_exc is the occupation-weighted norm of the orbitals outside the span of
 * orthonormal reference orbitals (the paper gives the quantities, not the
 * formula; this is the projection form).
 *   psi0     host array [n_dom] of device pointers, [N_g][n_orb] complex in the
 *            precision's storage type (as psi); read only
 *   overlap  NULL, or host array [n_dom] whose non-NULL entries receive S,
 *            device [n_orb][n_orb] complex128 (row s, column n)
 *   f_out    host array [n_dom] of device float64 [n_orb] outputs
 *   n_exc    device float64 [n_dom] output
 * Deterministic (fixed summation orders).  Workspace as dcmesh_step. */
int dcmesh_occupations(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                       const void* const* psi0, double* const* overlap,
                       double* const* f_out, double* n_exc,
                       void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Macroscopic particle current density of each domain (the current that the
 * Maxwell equations for the field take, Sec. V.B.5: its nonlocal correction is
 * formed with projector products):
 *     J = (h^3 sum_g j(g) + J_nl) / Omega,   Omega = N_g h^3,
 *     j(g) = sum_n f_n [Im(conj psi_n D1 psi_n) + A |psi_n|^2]   (as dcmesh_density)
 *     J_nl,d = sum_n f_n <psi_n| i[V_nl, r_d] |psi_n>
 *            = -2 sum_{n,p} f_n D_p Im(conj(P_pn) R_d,pn),
 *     P = h^3 B^H Psi,  R_d = h^3 B_d^H Psi,
 * with B_d = (r - R_atom)_d B the position-weighted projectors, r measured from
 * each projector's atom (any per-projector origin gives the same commutator).
 *   a_dev    device float64 [n_a][3], the field of the state (n_a = n_dom or 1)
 *   proj_r   NULL (no nonlocal part), or host array [n_dom] of device pointers to
 *            [3][N_g][n_proj] complex in the precision's storage type; entries
 *            may be NULL only for domains without projectors
 *   current  device float64 [n_dom][3] output
 * FP64 and FP32.  Workspace as dcmesh_step.  Deterministic. */
int dcmesh_current(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                   const double* a_dev, int32_t a_per_domain, const void* const* proj_r,
                   double* current, void* work, size_t work_bytes, uint32_t flags, void* stream);

/* n_steps Taylor-4 steps coupled to the Maxwell equation of a uniform vector
 * potential: the field is A = A_ext + A_ind with d^2 A_ind / dt^2 = -4 pi J
 * (J the macroscopic particle current density of dcmesh_current, atomic units,
 * e/c folded into A).  Per step k, with A_ind at the step times and its rate b
 * at the half steps:
 *     J_k = J(psi_k, A_ext(t_k) + A_ind);  b -= 4 pi dt J_k;  A_ind' = A_ind + dt b
 *     psi_k+1 = T4(-i dt H(A_mid)) psi_k,
 *     A_mid = (A_ext(t_k) + A_ext(t_k+1)) / 2 + (A_ind + A_ind') / 2.
 *   a_ext    device float64 [n_a][n_steps + 1][3] at the step times
 *   field    device float64 [n_dom][6] in/out: A_ind (3), then b (3)
 *   a_mid    device float64 [n_dom][n_steps][3] output: the step fields
 *   current  NULL or device float64 [n_dom][n_steps][3] output: J_k
 *   proj_r   as dcmesh_current (NULL: local current only)
 * FP64 and FP32.  Workspace as dcmesh_step.  No host synchronisation. */
int dcmesh_step_maxwell(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                        const void* const* proj_r, const double* a_ext, int32_t a_per_domain,
                        double dt, int32_t n_steps, double* field, double* a_mid, double* current,
                        void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Not in the paper: the pulse-gradient extension (the gradient of an
 * absorbed energy with respect to the vector-potential samples).
 * One step of the adjoint recursion for the gradient of a loss L(psi_N):
 *     lambda_k = U_k^H lambda_{k+1} = T4(+i dt H(A_k)) lambda_{k+1}
 *     grad[d] += 2 Re <lambda_{k+1}, (dU_k/dA_d) psi_k>,  dH/dA_d = -i D1_d + A_d
 * doms[i].psi holds psi_k (read only).  lambda: host array [n_dom] of device
 * pointers, [N_g][n_orb] complex, overwritten in place.  a_dev: A_k,
 * [n_a][3] float64.  grad_dev: device float64 [n_a][3], accumulated (+=). */
int dcmesh_adjoint_step(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                        void* const* lambda, const double* a_dev, int32_t a_per_domain,
                        double dt, double* grad_dev,
                        void* work, size_t work_bytes, uint32_t flags, void* stream);

/* Not in the paper (launch plumbing for many steps of many domains).
 * Record the work of one dcmesh_step call (same arguments) into a HIP graph
 * owned by the returned handle; replay it with dcmesh_graph_launch.  The
 * handle keeps the pointers it was built with. */
int dcmesh_graph_create(const dcmesh_domain* doms, int32_t n_dom, int32_t precision,
                        const double* a_dev, int32_t a_per_domain, int64_t a_stride,
                        double dt, int32_t n_steps, const dcmesh_obs* obs,
                        void* work, size_t work_bytes, uint32_t flags, void* stream,
                        void** graph_out);
int dcmesh_graph_launch(void* graph, void* stream);
int dcmesh_graph_destroy(void* graph);

/* Not in the paper (tile plumbing).
 * Tile choices: dcmesh_set_tuning selects a kernel variant for a kernel family
 * (DCMESH_KERNEL_*) and value (see dcmesh_tuning_options); -1 restores the
 * built-in heuristic.  Process-wide; takes effect for calls made afterwards.
 * DCMESH_KERNEL_ZSEG picks the z-segment length of the stencil sweep (0: from
 * the block count; 1..4: 8, 16, 32 planes, whole columns).
 * DCMESH_KERNEL_SORDER picks the order of the stencil's work-groups (0: each
 * domain's orbital chunks dealt over the 8 XCDs; 1, 2: each (domain, z
 * segment) on one XCD, tiles before chunks or chunks before tiles; built in:
 * 1 for a launch of 8 or more (domain, z segment) pairs, else 0).  The
 * workspace size does not depend on these choices, and results do not depend
 * on the order. */
enum dcmesh_kernel { DCMESH_KERNEL_STENCIL = 0, DCMESH_KERNEL_PROJECT = 1, DCMESH_KERNEL_CORRECT = 2,
                     DCMESH_KERNEL_ZSEG = 3, DCMESH_KERNEL_SORDER = 4 };
int dcmesh_set_tuning(int32_t kernel, int32_t variant);
int dcmesh_tuning_options(int32_t kernel, int32_t* count);

/* Per-shape tile choices, the table an autotuner fills (not in the paper):
 * domains of exactly shape's nx, ny, nz, fd_order, n_orb and n_proj (its
 * pointers are not read) in this precision use this variant of the kernel
 * family (values as dcmesh_set_tuning; the z segment and the stencil work
 * order are not per shape);
 * -1 removes the entry.  A global dcmesh_set_tuning choice takes precedence;
 * shapes without an entry use the built-in rules.  Process-wide; for calls
 * made afterwards.  dcmesh_clear_tuning_shapes empties the table. */
int dcmesh_set_tuning_shape(int32_t kernel, int32_t precision, const dcmesh_domain* shape, int32_t variant);
int dcmesh_clear_tuning_shapes(void);

/* Not in the paper (measurement plumbing).
 * Waits for the events recorded by calls made with DCMESH_FLAG_PROFILE (since
 * the last collect), and writes per family the summed kernel time in ms and
 * the number of launches.  total_ms and launches: host arrays of n entries
 * (n <= DCMESH_N_FAMILIES).  Synchronises with the recorded events. */
int dcmesh_profile_collect(double* total_ms, int64_t* launches, int32_t n);

/* Not in the paper.  Message for the calling thread's last failed call ("" if
 * none). */
const char* dcmesh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DCMESH_H */

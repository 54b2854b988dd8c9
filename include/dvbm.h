/*
 * dvbm.h -- C ABI of the MI355X (gfx950) double-distribution quasi-equilibrium
 * discrete velocity Boltzmann (DDF-QE DVBM) library.
 *
 * The library advances the mass/momentum distribution f and the energy
 * distribution g of Strassle, Hosseini & Karlin, "Consistent kinetic modeling
 * of compressible flows with variable Prandtl numbers: double-distribution
 * quasi-equilibrium approach" (arXiv 2510.04197), on a uniform 2-D grid with
 * the fully discrete update of Eq. (finalDiscretePDE) (Sec. III A 1):
 *
 *   X(t+dt) = X - dt/dV sum_faces F_i - dt/tau_1 (X - X*) - dt/tau_2 (X* - X^eq),
 *   X in {f_i, g_i},
 *
 * with Grad-Hermite equilibria and quasi-equilibria (Sec. II D 2-4, Table I,
 * App. D), the tensor-product Gauss-Hermite velocity sets D2Q16 (total energy
 * split I) and D2Q25 (internal non-translational energy split II) of App. G,
 * and NND face values with the generalised van Leer limiter (Sec. III A 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All pointers named "device" are device (HBM) addresses on the current
 *    HIP device; they are owned by the caller.  The library never allocates
 *    or frees device memory (the fixed scratch of dvbm_adjoint_step_noalloc
 *    is a static device array of the loaded code object).  Pointers named
 *    "host" are host addresses.
 *  - Macroscopic fields are dense row-major float64 arrays of ny*nx values,
 *    element (y, x) at index y*nx + x; cell (y, x) has its centre at
 *    ((x + 1/2) dx, (y + 1/2) dy).
 *  - Population buffers hold each distribution row by row, the Q planes of a
 *    row side by side:
 *        element (d, i, y, x) at index ((d*ny + y)*Q + i)*pitch + x,
 *    d = 0 for f and d = 1 for g, pitch = dvbm_pitch(p) elements.  The dense
 *    float64 arrays of dvbm_load_populations, dvbm_store_populations and the
 *    adjoint cotangents are [2][Q][ny][nx] instead.
 *    Population i = a*q1 + b has velocity sqrt(R T_ref) (xi_a, xi_b) and
 *    weight w_a w_b, with the 1-D Gauss-Hermite nodes xi ascending
 *    (q1 = 4 for split I, Q = 16; q1 = 5 for split II, Q = 25).
 *  - Storage DVBM_F64 / DVBM_F32 stores X itself.  DVBM_BF16_DEV /
 *    DVBM_FP16_DEV / DVBM_F32_DEV store the deviation (X_i - X_ref_i) / w_i
 *    rounded to nearest-even, where X_ref is the rest equilibrium (rho = 1, u = 0,
 *    T = T_ref): f_ref_i = w_i; g_ref_i = w_i (Cv - R) T_ref (split II) or
 *    w_i (Cv T_ref + R T_ref (|xi_i|^2 - 2) / 2) (split I).  F64 computes in
 *    float64; the other formats compute in float32 with float64 per-node
 *    moment sums.
 *  - Every call is asynchronous on the stream given to dvbm_init unless its
 *    description says it synchronises.
 *  - Every int-returning call returns DVBM_OK (0) or a negative DVBM_E*
 *    code; dvbm_last_error() then describes the failure (thread-local).
 *    A kernel fault surfaces at the next synchronising call as DVBM_EHIP.
 */
#ifndef DVBM_H
#define DVBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DVBM_OK 0
#define DVBM_EINVAL (-1) /* invalid argument or parameter */
#define DVBM_EHIP (-2)   /* HIP runtime error (message from hipGetErrorString) */
#define DVBM_ENAN (-3)   /* non-finite or non-physical state (rho <= 0, T <= 0) */
#define DVBM_ESTIFF (-4) /* dt / tau_1 > 2 for the initial state */

/* DVBM_F32_DEV keeps float32's bytes but stores the deviation: near the rest
 * state its values are small, so a rounding of the stored value is that much
 * finer than one of X itself.  The step kernels also do their arithmetic
 * in deviation units.  The adjoint takes this format as well as F64 and F32
 * (it differentiates the map of the populations X, decoded to float64). */
enum dvbm_storage { DVBM_F64 = 0, DVBM_F32 = 1, DVBM_BF16_DEV = 2, DVBM_FP16_DEV = 3, DVBM_F32_DEV = 4 };
/* Boundaries: periodic; zero-gradient (two ghost layers copy the nearest
 * interior cell); DVBM_WALL (bc_y only): no-slip walls on the faces below row
 * 0 and above row ny-1 with temperatures wall_T and x velocities wall_ux
 * (thermal Couette flow, Sec. IV).  The wall's two ghost rows take the fields
 * of the first two interior rows reflected through the wall values,
 * rho_G = rho_B, u_G = 2 u_W - u_B, T_G = 2 T_W - T_B, and the populations
 * X^eq(G) + (X_B - X^eq(B)).  Walls run on the per-cell kernel, need the
 * larger workspace dvbm_workspace_bytes() reports for them, and have no
 * adjoint (EINVAL). */
enum dvbm_bc { DVBM_PERIODIC = 0, DVBM_ZERO_GRADIENT = 1, DVBM_WALL = 2 };
enum dvbm_visc { DVBM_CONST_MU = 0, DVBM_CONST_TAU = 1 };
/* Step kernel (all compute the same update; the choice only affects speed):
 * AUTO picks the column sweep on grids of at least 3 * 2^18 cells (for
 * 32/16-bit storage only when one distribution fits 2 GiB), else the LDS
 * tile kernel for DVBM_F64 and the per-cell kernel for the other storages.
 * SWEEP with 32/16-bit storage requires a distribution of at most 2 GiB. */
enum dvbm_kernel { DVBM_KERNEL_AUTO = 0, DVBM_KERNEL_CELL = 1, DVBM_KERNEL_SWEEP = 2, DVBM_KERNEL_TILE = 3 };

/*
 * Simulation parameters (Sec. III A 3).  dvbm_params_default() fills the
 * paper's defaults: split II, F32, periodic, CONST_MU, AUTO kernel, R = 1, gamma = 1.4,
 * Pr = 0.71, mu = 5e-5 (tau_ref = 5e-5 with p_ref = 1), T_ref = 1,
 * beta = 1.2, CFL = 0.01, dt = 0 (CFL rule).
 *
 * Relaxation times (Sec. II C, Eqs. visc_shear_1 .. Pr_times_cases): the
 * shear time is tau_nu = tau_ref * p_ref / p(node) for DVBM_CONST_MU (fixed
 * dynamic viscosity mu = tau_ref * p_ref) or tau_nu = tau_ref for
 * DVBM_CONST_TAU; tau_alpha = tau_nu / Pr; tau_1 = min, tau_2 = max of the two.
 */
typedef struct dvbm_params {
  int32_t nx, ny;      /* cells, each >= 4 (the flux stencil has radius 2) */
  int32_t split;       /* 1 = total energy split (D2Q16), 2 = internal non-translational (D2Q25) */
  int32_t storage;     /* enum dvbm_storage */
  int32_t bc_x, bc_y;  /* enum dvbm_bc; zero-gradient copies the nearest interior cell into 2 ghost layers */
  int32_t visc_mode;   /* enum dvbm_visc */
  int32_t kernel;      /* enum dvbm_kernel (0 = AUTO) */
  double dx, dy;       /* cell sizes, > 0 */
  double R, gamma;     /* gas constant > 0; 1 < gamma <= 2 (split II needs Cv >= D R / 2) */
  double Pr;           /* Prandtl number > 0 */
  double tau_ref;      /* > 0, see above */
  double p_ref;        /* > 0 */
  double T_ref;        /* lattice reference temperature > 0 */
  double beta;         /* limiter parameter in [1, 2] */
  double cfl;          /* > 0; used when dt <= 0 */
  double dt;           /* > 0 overrides dt = cfl * min(dx, dy) / max(|u| + sqrt(gamma R T)) */
  double wall_T[2];    /* bc_y == DVBM_WALL: temperature (> 0) of the lower and the upper wall (default 1) */
  double wall_ux[2];   /* bc_y == DVBM_WALL: x velocity of the lower and the upper wall (default 0) */
} dvbm_params;

typedef struct dvbm_handle dvbm_handle;

/* Fill *p with the defaults above (nx = ny = 0: the caller sets the grid). */
void dvbm_params_default(dvbm_params* p);

/* Number of populations per distribution (16 or 25), or DVBM_EINVAL. */
int dvbm_num_populations(int32_t split);

/* The library's velocity set (App. G, Tables II-III) for checks: writes Q
 * velocities to v_host[2*i], v_host[2*i+1] and weights to w_host[i]
 * (both host arrays of at least 25 entries).  Returns Q or DVBM_EINVAL. */
int dvbm_velocity_set(int32_t split, double R, double T_ref, double* v_host, double* w_host);

/* Row pitch in elements of the population layout (nx rounded up to 64). */
int64_t dvbm_pitch(const dvbm_params* p);

/* Bytes of ONE population buffer (f and g) for these parameters; 0 if invalid. */
size_t dvbm_buffer_bytes(const dvbm_params* p);

/* Bytes of the caller-provided device workspace (reduction partials, and the
 * wall ghost rows when bc_y == DVBM_WALL). */
size_t dvbm_workspace_bytes(const dvbm_params* p);

/*
 * Create a solver on two caller-owned device buffers of dvbm_buffer_bytes()
 * each (ping-pong; 256-byte aligned) and a device workspace of
 * dvbm_workspace_bytes(), and fill buf0 with the equilibrium populations of
 * the device float64 fields rho, ux, uy, T (Sec. III A 3: initial conditions
 * are equilibrium populations).  stream is a hipStream_t (NULL = default).
 * Computes dt from the fields when p->dt <= 0 (device reduction, then host
 * arithmetic).  Synchronises.  Errors: EINVAL (parameters, NULL pointers),
 * ENAN (rho <= 0 or T <= 0 or non-finite input), ESTIFF (dt/tau_1 > 2 at
 * some node), EHIP.  On success *out owns only host memory.
 */
int dvbm_init(const dvbm_params* p, const double* rho, const double* ux, const double* uy,
              const double* T, void* buf0, void* buf1, void* workspace, void* stream,
              dvbm_handle** out);

/* Advance nsteps >= 0 time steps of Eq. (finalDiscretePDE) (one fused kernel
 * launch per step, ping-ponging between the two buffers).  Asynchronous. */
int dvbm_step(dvbm_handle* h, int64_t nsteps);

/* One time step from the population buffer src into dst (device buffers of
 * dvbm_buffer_bytes() in the layout above, e.g. checkpoint copies; they must
 * not overlap).  The handle's own state and buffers are not touched.
 * Asynchronous. */
int dvbm_step_from(dvbm_handle* h, const void* src, void* dst);

/*
 * Macroscopic fields and global sums of the current state (Eqs.
 * eq_quadratur1-3).  rho, ux, uy, T: device float64 arrays of ny*nx or NULL.
 * sums_host (may be NULL): host double[4] = sum over cells of rho, rho ux,
 * rho uy and total energy E, accumulated in float64 in a fixed order
 * (deterministic).  Synchronises when sums_host != NULL; returns ENAN if a
 * sum is not finite.
 */
int dvbm_moments(dvbm_handle* h, double* rho, double* ux, double* uy, double* T, double* sums_host);

/* Overwrite the current state with populations given as a dense device
 * float64 array X[2][Q][ny][nx] (encoded to the storage format). */
int dvbm_load_populations(dvbm_handle* h, const double* X);

/* Decode the current state into a dense device float64 array X[2][Q][ny][nx]. */
int dvbm_store_populations(dvbm_handle* h, double* X);

/* Time step in use (host value). */
double dvbm_get_dt(const dvbm_handle* h);

/* Device address of the buffer holding the current state (buf0 or buf1),
 * and its index 0/1. */
void* dvbm_state(const dvbm_handle* h);
int dvbm_state_index(const dvbm_handle* h);

/* Make buffer index (0 or 1) the current state, e.g. after the caller copied
 * a checkpoint into it. */
int dvbm_set_state_index(dvbm_handle* h, int index);

/*
 * Discrete adjoint (reverse-mode derivative of the update above; it is not
 * part of the paper and follows the discretise-then-differentiate rule: the
 * limiter is differentiated on the branch the forward step takes, and dt is
 * held fixed).  Supported for DVBM_F64, DVBM_F32 and DVBM_F32_DEV storage
 * (EINVAL otherwise); the arithmetic is float64.  Cotangents lam are dense device
 * float64 arrays lam[2][Q][ny][nx] of dvbm_adjoint_bytes() bytes.
 */
size_t dvbm_adjoint_bytes(const dvbm_params* p);

/* Bytes of the device work array of dvbm_adjoint_step (14 float64 values per
 * cell: the cotangents of the 13 node moments and 1 - dt/tau_1); 0 if the
 * parameters are invalid. */
size_t dvbm_adjoint_work_bytes(const dvbm_params* p);

/* lam_n = (dX_{n+1}/dX_n)^T lam_np1 for the step that maps state_n (a device
 * buffer in the population layout above, e.g. a checkpoint copy) to
 * X_{n+1}.  When dparams != NULL (device double[2]) it is incremented by
 * (dX_{n+1}/dtau_ref)^T lam_np1 and (dX_{n+1}/dPr)^T lam_np1 (at Pr == 1,
 * where Table I has no quasi-equilibrium, the Pr entry is 0), summed in a
 * fixed order through the handle's workspace.  work is a caller-owned device
 * array of dvbm_adjoint_work_bytes() bytes (contents overwritten).  Calls on
 * one handle, or sharing one work array, must not overlap; lam_np1 and lam_n
 * must not overlap.  Asynchronous. */
int dvbm_adjoint_step(dvbm_handle* h, const void* state_n, const double* lam_np1, double* lam_n,
                      double* dparams, void* work);

/* dvbm_adjoint_step with the cotangents stored in float32: lam_np1 and lam_n
 * are dense device float arrays lam[2][Q][ny][nx] (half of
 * dvbm_adjoint_bytes()).  Values are widened to float64 on load, all
 * arithmetic, the work array and dparams are float64, and lam_n is rounded to
 * nearest once on store, so a step adds one float32 rounding (2^-24 relative)
 * per value; it halves the cotangent traffic of a reverse sweep.  Arguments,
 * errors and ordering as for dvbm_adjoint_step.  Asynchronous. */
int dvbm_adjoint_step_f32(dvbm_handle* h, const void* state_n, const float* lam_np1, float* lam_n,
                          double* dparams, void* work);

/* dvbm_adjoint_step for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with no work argument.  The work rows and
 * the reduction partials live in a fixed scratch array of 16 MiB that the
 * library holds on each device it runs on until the process ends (its device
 * address is looked up once per device in dvbm_init); the call itself makes
 * no allocation and no runtime call besides its kernel launches.  Grids
 * needing more than the scratch's 16 MiB - 64 KiB of work rows (nx*ny above
 * 149,211 cells) are rejected with DVBM_EINVAL.  Every call on one device
 * uses that device's one array: calls that overlap in time on one GPU (other
 * streams, other threads, other handles) race and give wrong results;
 * consecutive calls are safe (each clears the counter it needs).  Other
 * arguments, errors and ordering as for dvbm_adjoint_step (float64
 * cotangents; f64, f32 and f32_dev storage).  Asynchronous. */
int dvbm_adjoint_step_noalloc(dvbm_handle* h, const void* state_n, const double* lam_np1, double* lam_n,
                              double* dparams);

/* lam = sum of (d field / dX)^T d_field over the macroscopic fields of state
 * (rho, u_x, u_y, T of Eqs. eq_quadratur1-3); any d_* may be NULL (zero).
 * d_* are device float64 arrays of ny*nx.  Asynchronous. */
int dvbm_adjoint_moments(dvbm_handle* h, const void* state, const double* d_rho, const double* d_ux,
                         const double* d_uy, const double* d_T, double* lam);

/* Cotangents of the initial fields through the equilibrium initialisation:
 * d_field = (dX_0/d field)^T lam0 for the device float64 fields rho, ux, uy,
 * T (the values given to dvbm_init); outputs that are NULL are skipped.
 * Asynchronous. */
int dvbm_adjoint_init(dvbm_handle* h, const double* lam0, const double* rho, const double* ux,
                      const double* uy, const double* T, double* d_rho, double* d_ux, double* d_uy,
                      double* d_T);

/* Limiter branches of the step from state (a device buffer in the
 * population layout, float64 storage only; EINVAL otherwise or with walls),
 * for derivative checks: central differences X(p + h) - X(p - h) measure
 * the derivative only while both runs take the same branch of the limiter
 * phi (Sec. III A 2) at every face.  For every face the step reconstructs
 * (the face above each cell along each axis with a non-zero velocity
 * component, from its upwind side), branch 0 (r <= 0), 1 (beta r),
 * 2 ((1 + r)/2) or 3 (beta) is mixed with the face's index by the SplitMix64
 * output function, and the sum of these terms modulo 2^64 is ADDED to the
 * device uint64 *sig (the caller zeroes it).  Equal branch patterns give
 * equal sums; a different pattern differs except for a 2^-64 collision.
 * Asynchronous. */
int dvbm_limiter_signature(dvbm_handle* h, const void* state, uint64_t* sig);

/* Streaming probe (not part of the method): plain grid-stride kernels that
 * bound the HBM bandwidth any kernel reaches on this GPU.  mode 0 copies
 * bytes from src to dst, 1 reads src (dst receives at most one element),
 * 2 writes dst (src unused, may be NULL); mode + 4 makes the accesses
 * non-temporal; width 16 or 4 is the bytes each lane moves per access.  src and dst are caller-owned device buffers of
 * `bytes` bytes (a positive multiple of width, both aligned to width);
 * stream is a hipStream_t.  EINVAL on a bad argument.  Asynchronous. */
int dvbm_stream_probe(const void* src, void* dst, size_t bytes, int32_t mode, int32_t width, void* stream);

/* Release the handle (host memory only).  NULL is ignored. */
void dvbm_destroy(dvbm_handle* h);

/* Message describing the last failure on this thread ("" if none). */
const char* dvbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DVBM_H */

/*
 * fsib.h -- C ABI of the MI355X (gfx950) Fourier spectral immersed boundary (FSIB) hot path.
 *
 * Method: Chen & Peskin, "A Fourier spectral immersed boundary method with exact translation
 * invariance, improved boundary resolution, and a divergence-free velocity field".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named X, c, fhat, F, S, U, uhat, ... are DEVICE pointers owned by the caller, unless
 *    a comment says "host".  The library never frees or keeps them after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).  Every call that
 *    takes a stream only enqueues work on it and returns without synchronising, except
 *    fsib_plan_create (allocates and synchronises once) and fsib_plan_check (synchronises).
 *  - The truncated mode set K_N (Sec. 3.1, eq. kNh): per axis m in [-N/2, N/2-1] (even N) or
 *    [-(N-1)/2, (N-1)/2] (odd N), k = 2*pi*m/L.  Spectral arrays are in FFT order (m = 0, 1, ...,
 *    then the negative modes; the zero mode first) with the x index fastest, then y, then z.
 *  - "Full" spectral array of one transform: N_z*N_y*N_x complex values (2D: N_y*N_x).
 *    "Half" spectral array of one real field: N_z*N_y*H_x complex values, H_x = floor(N_x/2)+1,
 *    holding m_x = 0..H_x-1 (the other half is the complex conjugate).  For even N_x the last
 *    entry is the wavenumber +N_x/2, the conjugate partner of the K_N modes with m_x = -N_x/2:
 *    fsib_force_spread fills it, fsib_fluid_step sets it to zero and fsib_velocity_interp
 *    requires it to be zero.  Vector fields are component-major: d consecutive scalar arrays
 *    (d = dim).
 *  - Complex values are interleaved (re, im) pairs of the plan precision: double for FSIB_F64,
 *    float for FSIB_F32.  "prec" below means that scalar type.
 *  - Positions X are always double, shape (M, dim) row-major, any real values: the L-periodicity
 *    is applied inside (x is folded to [0, L) in double before any rounding to prec).
 *  - Argument checks happen before anything is enqueued; on error nothing is written and the
 *    status says why (fsib_last_error() gives a message, per thread).  HIP failures map to
 *    FSIB_ERR_HIP.
 *  - The compute entry points allocate no memory: the plan owns its workspace, sized at creation
 *    for dim, N, precision, ntrans and max_points.
 *  - A plan is not thread-safe: calls that share a plan must be issued in order on one stream.
 */
#ifndef FSIB_H
#define FSIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsib_plan_s* fsib_plan;

typedef enum { FSIB_F64 = 0, FSIB_F32 = 1 } fsib_prec;

typedef enum {
  FSIB_OK = 0,
  FSIB_ERR_ARG = 1,        /* invalid argument (null pointer, size out of range, unsupported option) */
  FSIB_ERR_TOL = 2,        /* requested tolerance not reachable in the plan precision */
  FSIB_ERR_NO_DEVICE = 3,  /* no HIP device visible */
  FSIB_ERR_OOM = 4,        /* workspace allocation failed at plan creation */
  FSIB_ERR_HIP = 5,        /* a HIP runtime call failed; fsib_last_error() holds its message */
  FSIB_ERR_NONFINITE = 6,  /* a NaN/Inf position was seen since the last fsib_plan_check */
  FSIB_ERR_STATE = 7       /* the plan lacks the workspace this call needs (see fsib_plan_opts) */
} fsib_status;

typedef struct {
  int dim;              /* 2 or 3 */
  int64_t n_modes[3];   /* N per axis (x, y, z), each >= 2; n_modes[2] ignored in 2D */
  double L;             /* period of the box [0, L)^dim, > 0 */
  int prec;             /* fsib_prec: arithmetic of grids, FFTs, spectral update, U */
  double tol;           /* relative l2 accuracy asked of the nonuniform transforms:
                           FP64 in [1e-14, 1e-1], FP32 in [1e-6, 1e-1] (else FSIB_ERR_TOL) */
  double upsampfac;     /* fine-grid oversampling sigma: 2.0, 1.5 or 1.25.  Below 2 the fine grid
                           is smaller (1.5: about 2.4x fewer grid bytes in 3D; 1.25: about 4x) and
                           the kernel wider; the per-axis error tol/(2 dim) must stay reachable with
                           w <= 16 (1.25: tol >= about 1e-8; 1.5: about 1e-11), and the
                           deconvolution lifts FP32 rounding by up to ~10x (1.5) or ~100x (1.25), so
                           FP32 plans need tol >= 1e-5 at 1.5 and >= 1e-3 at 1.25, else
                           FSIB_ERR_TOL.  0 = automatic: for 3D plans with max_points <= N_x N_y N_z
                           / 20, 1.5 in FP64 at tol >= 1e-6 and in FP32 at tol >= 1e-4; else 2.0
                           (fsib_plan_info reports n_fine) */
  int ntrans;           /* complex transforms per fsib_spread / fsib_interp call, >= 1 */
  int64_t max_points;   /* largest M accepted by any call, >= 0 */
  int fluid;            /* 0: NUFFT only; 1: also the FSIB workspace (force spread, velocity
                           interp, fluid step, time step) */
  int navier_stokes;    /* with fluid = 1: 1 also allocates the dealiasing workspace (Sec. 3.1) */
  int ninst;            /* independent simulations held by the plan, all with these n_modes, L, prec
                           and tol (0 or 1: one).  ninst > 1 needs fluid = 1, navier_stokes = 0 and
                           ntrans = 1 (Stokes instances); every stage of a step then runs as one
                           launch over all instances.  Points are given instance after instance
                           (fsib_plan_set_instances), half spectra as [ninst][dim][...]. */
  int deterministic;    /* 0: points inside a spreading bin are ordered as the sort's atomic run claims
                           arrive, so spreading sums agree between runs to rounding only; 1: every bin
                           lists its points in ascending original index (one more pass over the points
                           per sort), so every output of every call is bitwise reproducible for the same
                           inputs, including across HIP graph replays and checkpoint/resume of fsib_step
                           trajectories (Sec. 5: the method itself is deterministic). */
} fsib_plan_opts;

/* Read-only facts about a plan (host struct filled by fsib_plan_info). */
typedef struct {
  int w;                /* kernel width in fine-grid cells */
  double beta;          /* Kaiser-Bessel shape parameter (App. A, eq. kernel_KB) */
  int degree;           /* degree of the piecewise polynomial that evaluates the kernel */
  int64_t n_fine[3];    /* fine (oversampled) grid per axis */
  int64_t n_dealias[3]; /* dealiasing grid per axis (0 unless navier_stokes) */
  int64_t tile[3];      /* spreading tile (= bin) size per axis in fine cells */
  int64_t workspace_bytes;
} fsib_plan_info_t;

/* Launch-shape knobs of a plan (results do not depend on them, only speed). */
typedef struct {
  int xcd_chunk_interp;  /* interpolation workgroups kept together on one XCD (0: plain order) */
  int xcd_chunk_spread;  /* spreading tiles kept together on one XCD (0: plain order) */
  int split;             /* candidate points per part of a heavy spreading tile */
  int overlap;           /* Navier-Stokes steps: 1 runs the point side of each half step (positions,
                            force, sort, spreading, interpolation) on a second stream of the plan,
                            concurrently with the dealiased products; 0 runs everything on the
                            caller's stream.  1 by default. */
  int interp_points;     /* points per interpolation wavefront: 1, 2, 4 (default), 8 or 16, rounded
                            up to the points a kernel sums together (up to 4) */
  int spread_threads;    /* spreading variant: threads per 16 x 16 tile of a 2D plan, 64 (4 cells
                            per lane), 128 (2) or 256 (1); 0 picks the default (64 in FP32, 128 in
                            FP64).  3D plans take 0 or 256 (16 x 8 x 8 tiles, 4 cells per lane). */
  int nl_stages;         /* Navier-Stokes plans whose dealiasing grid has 192 points along x (128
                            modes): FFT stages of the fused x pass of the dealiased products (Sec.
                            3.1), 2 (16 x 12, registers between the stages; fastest alone) or 3 (8 x 8
                            x 3 through LDS; lower peak demand on memory and LDS, which leaves more of
                            the GPU to a point side running beside it); 0 picks 3 for the first half
                            step of FP64 steps whose point side overlaps (overlap = 1), where that side
                            is the critical path, and 2 otherwise.  Other plans take any of 0, 2, 3
                            and ignore it. */
} fsib_tuning;

typedef enum { FSIB_STOKES = 0, FSIB_NAVIER_STOKES = 1 } fsib_model;

typedef struct {
  int model;            /* fsib_model */
  double rho, mu, dt;   /* density, viscosity (> 0), time step */
  double body[3];       /* NAVIER_STOKES: uniform body force density f0 added to the zero mode of fhat
                           (the channel-flow driving force of Sec. 6.2.2); 0 for none.  STOKES
                           ignores it (its zero mode is 0). */
} fsib_fluid_params;

typedef enum {
  FSIB_FORCE_CURVE_TENSION = 0,
  FSIB_FORCE_SURFACE_TENSION = 1,
  FSIB_FORCE_EDGE_SPRINGS = 2,
  FSIB_FORCE_TARGET = 3
} fsib_force_kind;

typedef struct {
  int kind;                 /* fsib_force_kind */
  double K;                 /* stiffness K (curve tension) or surface tension gamma */
  const int32_t* tris;      /* SURFACE_TENSION: device (ntris, 3) vertex indices, counter-clockwise
                               seen from outside */
  int64_t ntris;
  const int32_t* v2t_ptr;   /* device CSR (M+1) offsets: triangles incident to each vertex
                               (EDGE_SPRINGS: the neighbours of each vertex) */
  const int32_t* v2t_idx;   /* device CSR (3*ntris) triangle ids (EDGE_SPRINGS: neighbour ids) */
  const double* aux;        /* EDGE_SPRINGS: device stiffness per CSR entry (K_ij, both directions);
                               TARGET: device (M, dim) target positions.  NULL otherwise. */
} fsib_force;

/* ---- library ------------------------------------------------------------------------------- */
const char* fsib_version(void);
const char* fsib_status_string(fsib_status s);
const char* fsib_last_error(void);  /* message of the last failing call on this thread */
int fsib_device_count(void);        /* visible HIP devices (0 when none or no driver) */

/* ---- plans ---------------------------------------------------------------------------------- */
/* Chooses the kernel width/shape for `tol` (App. A.3), the fine grid (upsampfac * N rounded to a
 * 2^a 3^b 5^c multiple of the tile), twiddle and deconvolution tables, and allocates the workspace
 * on the current device.  *out is written only on success. */
fsib_status fsib_plan_create(const fsib_plan_opts* opts, fsib_plan* out);
/* Point ranges of the instances of a plan with ninst > 1: instance i owns points
 * [offsets[i], offsets[i+1]) of X, U (host array of ninst + 1, offsets[0] = 0, non-decreasing,
 * offsets[ninst] <= max_points).  A set-up call: copies to the device and synchronises.  Until it is
 * made, fsib_step and fsib_velocity fail with FSIB_ERR_STATE on such plans; afterwards their M must
 * be offsets[ninst].  Errors: FSIB_ERR_ARG for bad offsets, FSIB_ERR_STATE for ninst = 1 plans. */
fsib_status fsib_plan_set_instances(fsib_plan plan, const int64_t* offsets);
fsib_status fsib_plan_destroy(fsib_plan plan);  /* waits for the plan's work, frees the workspace */
fsib_status fsib_plan_info(fsib_plan plan, fsib_plan_info_t* info /* host */);
/* Synchronises `stream`; returns FSIB_ERR_NONFINITE (and clears the flag) if any call since the
 * last check saw a non-finite position (such points are treated as x = 0), else FSIB_OK. */
fsib_status fsib_plan_check(fsib_plan plan, void* stream);

/* Kernel timing with HIP events (for roofline measurement): while enabled, every launch of the
 * chosen kernel class by this plan is bracketed by an event pair on its stream, for at most
 * max_launches launches, and its algorithmic bytes (each input and output element of the launch
 * counted once; for spreading the grid written once plus the point records and strengths; for
 * interpolation the point records plus w^d cells per point) are accumulated.
 * fsib_plan_profile synchronises the device and (re)creates the events; kernel_class -1 disables.
 * fsib_plan_profile_read waits for the recorded launches, returns the summed elapsed time (ms),
 * the launch count and the bytes (host outputs), and starts a new tally. */
typedef enum {
  FSIB_PROF_FFT_STRIDED = 1,  /* batched FFT passes along y and z */
  FSIB_PROF_SPREAD = 2,       /* spreading onto the fine grid */
  FSIB_PROF_INTERP = 3,       /* interpolation from the fine grid */
  FSIB_PROF_FFT_X = 4,        /* real-data FFT passes along x */
  FSIB_PROF_NL_X = 5          /* fused x pass of the dealiased products */
} fsib_prof_class;
fsib_status fsib_plan_profile(fsib_plan plan, int kernel_class, int max_launches);
/* Read (get = 1) or set (get = 0) the launch-shape knobs, e.g. for a timed autotuning search.
 * Results are identical up to the summation order of spreading.  split may not go below the value
 * the plan was created with (its scratch is sized for it).  The creation value is 256 for plans of
 * at most 2^18 points (128 for FP32 Navier-Stokes ones), else 512; the environment variable
 * FSIB_SPREAD_SPLIT, read at plan creation, replaces it (clamped to [64, 2^20]), and
 * FSIB_XCD_CHUNK_INTERP and FSIB_XCD_CHUNK_SPREAD likewise replace the two chunk defaults (values
 * outside [0, 4096] ignored).  Errors:
 * FSIB_ERR_ARG for NULL or out-of-range values (chunks in [0, 4096], split in [creation, 1 << 20],
 * overlap 0 or 1, interp_points 1, 2, 4, 8 or 16, spread_threads as above, nl_stages 0, 2 or 3). */
fsib_status fsib_plan_tuning(fsib_plan plan, fsib_tuning* tuning, int get);
fsib_status fsib_plan_profile_read(fsib_plan plan, double* total_ms /* host */, int64_t* launches /* host */,
                                   double* bytes /* host */);

/* ---- nonuniform transforms (App. A) --------------------------------------------------------- */
/* Type-1 (App. A, eq. type1; with scale = L^-d it is eq. force_spreading_quad):
 *   fhat[t][k] = scale * sum_j c[t][j] exp(-i k.X_j),  k in K_N,  t < ntrans.
 * c: ntrans x M complex prec (transform-major); fhat: ntrans full spectral arrays.
 * Computed by spreading onto the fine grid with the plan kernel, an FFT, truncation to K_N and
 * division by the kernel transform (eqs. type1_conv, type1_deco); relative l2 error ~ tol. */
fsib_status fsib_spread(fsib_plan plan, int64_t M, const double* X, const void* c, void* fhat,
                        double scale, void* stream);
/* Type-2 (App. A, eq. type2): c[t][j] = sum_{k in K_N} fhat[t][k] exp(+i k.X_j).
 * fhat: ntrans full spectral arrays; c: ntrans x M complex prec (eqs. type2_divi, type2_conv). */
fsib_status fsib_interp(fsib_plan plan, int64_t M, const double* X, const void* fhat, void* c,
                        void* stream);

/* ---- Type-1 without allocation ----------------------------------------------------------------
 * For callers that cannot allocate device memory at call time or hold a plan's per-call workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): fsib_spread
 * with every per-call buffer (point sort, spreading work list and partial tiles, fine grid, FFT
 * intermediates) carved from a static device array of FSIB_NOALLOC_SCRATCH_BYTES per GPU, held by
 * the library from its first use on that GPU until the process ends.  Makes no hipMalloc, hipFree
 * or other allocating call.  Same arguments, layout and results as fsib_spread (to rounding; bitwise
 * on deterministic plans) with these differences:
 *   - M may exceed the plan's max_points; the buffers for (M, the plan's grid and ntrans) must fit the
 *     static array, else FSIB_ERR_ARG with the number of bytes needed (nothing is enqueued);
 *   - the plan must have fluid = 0 (FSIB_ERR_STATE otherwise) and be used on its own device
 *     (FSIB_ERR_ARG otherwise); its own workspace is neither read nor written;
 *   - every call on one GPU shares that GPU's array and leaves its contents behind: calls that may
 *     overlap in time on one GPU (different streams, threads or plans) race and must be ordered by
 *     the caller.  Nothing in the array needs to be cleared by the caller. */
#define FSIB_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
fsib_status fsib_spread_noalloc(fsib_plan plan, int64_t M, const double* X, const void* c, void* fhat,
                                double scale, void* stream);

/* ---- Adjoint building blocks (gradients of the transforms) ------------------------------------
 * For a real loss, the gradient of the strengths of type-1 is a type-2 sum of the gradient of its
 * output (and vice versa), and the gradient of the positions needs the phase derivative
 * d/dx_a exp(+-i k.x) = +-i k_a exp(+-i k.x) (App. A, eqs. type1 and type2).  Gradients of complex
 * arrays are dL/dRe + i dL/dIm. */
/* out = scale * in (axis = -1) or out = scale * i k_axis * in (axis in [0, dim)), k_a = 2 pi m_a / L,
 * elementwise on spectral arrays (device, complex prec, in place allowed):
 *   layout 0: ntrans full spectral arrays (FFT order, x fastest), as fsib_spread / fsib_interp;
 *   layout 1: dim half spectral arrays of real fields (fluid plans), as fsib_velocity_interp --
 *             i k_a uhat is the half spectrum of the derivative d/dx_a of the field.
 * Errors: FSIB_ERR_ARG for a bad layout or axis, NULL arrays, a non-finite scale; FSIB_ERR_STATE for
 * layout 1 on a plan without fluid. */
fsib_status fsib_spectral_scale(fsib_plan plan, int layout, int axis, double scale, const void* in, void* out,
                                void* stream);
/* Per-point combination of gradient terms into column `axis` of gX ((M, dim) double, device):
 *   kind 0: gX[j][axis] = scale * sum_{t < ntrans} Re( conj(u[t][j]) v[t][j] ),  u, v: ntrans x M complex;
 *   kind 1: gX[j][axis] = scale * sum_a ( u[j][a] v[j][a] + u2[j][a] v2[j][a] ),  u, v, u2, v2: (M, dim)
 *           real prec; u2 and v2 may both be NULL.
 * Errors: FSIB_ERR_ARG for M outside [0, max_points], a bad kind or axis, NULL arrays, non-finite scale. */
fsib_status fsib_grad_combine(fsib_plan plan, int64_t M, int kind, const void* u, const void* v, const void* u2,
                              const void* v2, double scale, double* gX, int axis, void* stream);

/* ---- FSIB coupling (Sec. 3.1); plans created with fluid = 1 ---------------------------------- */
/* Force spreading of real vector strengths S (M, dim) prec (S_j = w_j F_j):
 *   fhat[a][k] = scale * sum_j S[j][a] exp(-i k.X_j)   (eq. force_spreading_quad, scale = L^-d),
 * written as dim half spectral arrays. */
fsib_status fsib_force_spread(fsib_plan plan, int64_t M, const double* X, const void* S,
                              void* fhat_half, double scale, void* stream);
/* Velocity interpolation U[j][a] = sum_{k in K_N} uhat_a(k) exp(i k.X_j) (eq. velo_intp_fini)
 * from dim half spectral arrays (the field is real: uhat(-k) = conj uhat(k)); modes with any
 * m_a = -N_a/2 (even N_a) must be zero -- the fluid step guarantees it -- and are ignored.
 * U: (M, dim) prec. */
fsib_status fsib_velocity_interp(fsib_plan plan, int64_t M, const double* X, const void* uhat_half,
                                 void* U, void* stream);
/* Fourier-space fluid update on half spectral arrays (dim components each).
 *  NAVIER_STOKES (Alg. 1, eqs. spatial_2 and spatial_3, with V-hat of Alg. 2 and the dealiased
 *  nonlinear term of eq. nonlinear_kspace; plan needs navier_stokes = 1):
 *    uhat_mid = (dt/2 V(fhat, uhat) + uhat)/(1+a);  uhat <- (dt V(fhat, uhat_mid) + (1-a) uhat)/(1+a),
 *    a = mu dt |k|^2 / (2 rho);  uhat_mid may be NULL.
 *  STOKES (Sec. 6.1, eq. stokeslet): uhat <- (1/mu)(I/|k|^2 - k k^T/|k|^4) fhat, uhat(0) = 0;
 *    uhat_mid, if not NULL, receives the same.
 * fhat is the output of fsib_force_spread with scale L^-d.  Every output has the modes with any
 * m_a = -N_a/2 (even N_a) set to zero. */
fsib_status fsib_fluid_step(fsib_plan plan, const fsib_fluid_params* params, const void* fhat_half,
                            void* uhat_half, void* uhat_mid, void* stream);
/* Nodal force F(X) of a built-in model, double (M, dim):
 *  CURVE_TENSION (dim 2, Sec. 6.2.1 eq. elstic_force_2d): F_j = K (X_{j+1}+X_{j-1}-2X_j)/dtheta^2,
 *    dtheta = 2 pi / M (force per unit theta; quadrature weight dtheta).
 *  SURFACE_TENSION (dim 3, Sec. 6.2.3): F_i = -(K/2) sum_{(i,j,k)} (X_j - X_k) x n_ijk (nodal force,
 *    weight 1).  Needs tris and the vertex->triangle CSR.
 *  EDGE_SPRINGS (dim 2 or 3, Sec. 6.2.3 elastic sphere): F_i = K sum_{j linked with i} K_ij (X_j - X_i)
 *    (nodal force, weight 1); the CSR lists each vertex's neighbours, aux the K_ij of each entry (the
 *    cotangent stiffness of the reference triangulation for sigma = 1, K = sigma).
 *  TARGET (dim 2 or 3, Sec. 6.2.2 channel walls): F_i = K (Xtarget_i - X_i), aux = Xtarget (nodal
 *    force, weight 1). */
fsib_status fsib_compute_force(const fsib_force* force, int dim, int64_t M, const double* X,
                               double* F, void* stream);
/* Directional derivative out = dF(X)[V] of the force law ((M, dim) double arrays, device).  Both
 * laws are minus the gradient of an energy (Sec. 6.2.1: (K/2) sum |X_{j+1} - X_j|^2 / dtheta;
 * Sec. 6.2.3: K times the surface area), so the Jacobian is symmetric and out is also the transpose
 * product dF(X)^T V that the adjoint of a time step needs.  CURVE_TENSION is linear in X: out = F(V).
 * out must not alias X or V.  Errors as fsib_compute_force. */
fsib_status fsib_force_jvp(const fsib_force* force, int dim, int64_t M, const double* X, const double* V,
                           double* out, void* stream);
/* Stiffness of the elastic sphere's edge springs from the reference configuration X0 (Sec. 6.2.3),
 * for sigma = 1 (the EDGE_SPRINGS force takes sigma as K): entry e = (i -> j) of the neighbour CSR
 * (nbr_ptr (M+1), nbr_idx) receives sum over the triangles holding edge ij of
 * (a0^2 + b0^2 - c0^2) / (8 S0) = (cot C1 + cot C2) / 2.  X0 (M, 3) double, tris (T, 3), the
 * vertex->triangle CSR and the neighbour CSR are device arrays; kij (device, nbr_ptr[M] doubles) is
 * written.  A set-up call: it allocates 4 bytes and synchronises the device.  Errors: FSIB_ERR_ARG for
 * NULL arrays or a triangle edge absent from the neighbour lists. */
fsib_status fsib_spring_stiffness(int64_t M, const double* X0, const int32_t* tris, const int32_t* v2t_ptr,
                                  const int32_t* v2t_idx, const int32_t* nbr_ptr, const int32_t* nbr_idx,
                                  double* kij);
/* Pressure (Sec. 3, eq. pressure_poisson_k; Stokes: Sec. 6.1, eq. stokeslet), half spectrum of one real
 * field (prec, device, N_z x N_y x H_x):
 *   NAVIER_STOKES: phat = -i k.(fhat - rho shat(uhat)) / |k|^2, shat the dealiased nonlinear term of
 *                  uhat (as in fsib_fluid_step);
 *   STOKES:        phat = -i k.fhat / |k|^2.
 * phat(0) = 0 (the pressure has zero mean) and the modes with some m_a = -N_a/2 are zero.  fhat as for
 * fsib_fluid_step; uhat_half may be NULL for STOKES.  Errors: FSIB_ERR_STATE without fluid,
 * FSIB_ERR_ARG for NULL arrays or bad params. */
fsib_status fsib_pressure(fsib_plan plan, const fsib_fluid_params* params, const void* fhat_half,
                          const void* uhat_half, void* phat_half, void* stream);
/* Boundary velocity at X for the current state:  NAVIER_STOKES: U = interp(uhat, X) (uhat is
 * input).  STOKES: uhat <- Stokeslet(spread(w F(X))), U = interp(uhat, X) (uhat is output).
 * This gives U^0 for the first fsib_step. */
fsib_status fsib_velocity(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force,
                          int64_t M, const double* X, void* U, void* uhat_half, void* stream);
/* One time step of Alg. 1 (Sec. 3.3): X (double, in/out), U (prec, in U^m, out U^{m+1}),
 * uhat_half (in/out).  X^{m+1/2} = X^m + dt/2 U^m; F^{m+1/2} = F(X^{m+1/2}); fhat from the spread;
 * the fluid update; U^{m+1/2} = interp(uhat^{m+1/2}, X^{m+1/2}); X^{m+1} = X^m + dt U^{m+1/2};
 * U^{m+1} = interp(uhat^{m+1}, X^{m+1}).  STOKES: uhat is a function of X (see fsib_velocity).
 * X stays double in both precisions.  Ordering: the call is asynchronous in the order of `stream`;
 * NAVIER_STOKES steps fork their point side (positions, force, sort, spreading, interpolation at
 * X^{m+1/2}) onto the plan's second stream with an event and join it back with another before
 * returning, so all outputs are ready in the order of `stream` and a captured step records both
 * branches (tuning knob overlap = 0 keeps everything on `stream`).  Calls on one plan must not
 * overlap.  diag (device, nullable) receives FSIB_DIAG_COUNT doubles:
 *   [0..2] sum_j w_j F_j^{m+1/2}          (Sec. 5.3; [2] = 0 in 2D)
 *   [3..5] Re uhat^{m+1}(k = 0)
 *   [6]    E_K = rho/2 L^d sum_k |uhat^{m+1}|^2                     (Sec. 5.4)
 *   [7]    mu L^d sum_k |k|^2 |uhat^{m+1}|^2 (viscous dissipation)   (Sec. 5.4)
 *   [8]    sum_j w_j F_j^{m+1/2} . U_j^{m+1/2} (power)               (Sec. 5.4)
 *   [9]    max_k |k . uhat^{m+1}(k)| / max_k |k| |uhat^{m+1}(k)|     (Sec. 5.1)
 *   [10]   area (2D, shoelace) or volume (3D, signed tetrahedra) enclosed by X^{m+1} (Sec. 6.2) */
#define FSIB_DIAG_COUNT 11
fsib_status fsib_step(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force,
                      int64_t M, double* X, void* U, void* uhat_half, double* diag, void* stream);
/* nsteps >= 0 consecutive steps of Alg. 1, exactly as nsteps calls of fsib_step (results equal to
 * rounding: spreading sums in the order the sort leaves), with the same arguments; diag, if given,
 * is that of the last step.  Between the steps of one call the interpolation of U^{m+1} runs on the
 * plan's second stream (tuning knob overlap) beside the products of uhat^{m+1} that open the next
 * step; U, X and uhat_half are complete in the order of `stream` when the last step has run.
 * Errors as fsib_step; FSIB_ERR_ARG for nsteps < 0. */
fsib_status fsib_steps(fsib_plan plan, const fsib_fluid_params* params, const fsib_force* force,
                       int64_t M, double* X, void* U, void* uhat_half, int nsteps, double* diag,
                       void* stream);

/* ---- groups: many Stokes simulations of different sizes advanced together ----
 * Alg. 1 (Sec. 3.3) with the Stokes velocity of Sec. 6.1 (eq. stokeslet) is independent per
 * simulation; a group lets simulations of different N (each plan may itself hold ninst equal-N
 * instances) share every launch of a step: each stage of the step (positions, force, point sort,
 * spreading, the FFT passes, the Stokeslet, interpolation) is one kernel launch whose workgroups are
 * divided among the plans, each plan's part with that plan's own arguments and grid.  Stages whose
 * plans need different workgroup sizes (FFT lengths without a common thread count) fall back to one
 * launch per plan.
 *
 * fsib_group_create: nplans in [1, 8] distinct plans (host array) with fluid = 1, navier_stokes = 0,
 * and one device, dim, prec and kernel width w (the same tol and upsampfac give the same w).
 * Deterministic plans keep their bitwise reproducibility in a group (their ranking passes run as
 * launches of their own).  The group keeps the plan handles, not copies: the plans must outlive the group and
 * are not used on their own while a group call on them may still run.  Errors: FSIB_ERR_ARG. */
typedef struct fsib_group_s* fsib_group;
fsib_status fsib_group_create(int nplans, const fsib_plan* plans, fsib_group* out);
fsib_status fsib_group_destroy(fsib_group group);
/* nsteps >= 0 Stokes steps of every plan of the group, each as fsib_steps of that plan would run them
 * (same arithmetic per plan; spreading sums in the order the sort leaves).  Host arrays of nplans
 * entries, entry g for plan g: params (model STOKES, each plan its own mu and dt), forces, M, and
 * the device pointers X (double, in/out), U (prec, in U^m, out U^{m+1}) and uhat_half (in/out), as
 * for fsib_step.  No diagnostics.  Asynchronous in the order of `stream`; allocates nothing, so a
 * call can be captured in a HIP graph.  Errors as fsib_step, checked for every plan before any
 * launch. */
fsib_status fsib_group_steps(fsib_group group, const fsib_fluid_params* params, const fsib_force* forces,
                             const int64_t* M, double* const* X, void* const* U, void* const* uhat_half,
                             int nsteps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FSIB_H */

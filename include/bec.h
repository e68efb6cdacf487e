/*
 * bec.h -- C ABI of the MI355X (gfx950) PCG-ATKM ground-state library.
 *
 * Problem (paper Sec. 1, eqs. "DipGPE0", "Vpoten", "DDI-3D", "energy", "groundDef"):
 * minimise the discrete energy
 *   E(phi) = < -1/2 [[Lap]]phi + V phi + beta/2 |phi|^2 phi + lambda/2 Phi phi - Omega [[L_z]]phi, phi >
 * over the unit sphere ||phi|| = 1 (Sec. 2.3, eq. "mp"), with V the harmonic trap, Phi the dipolar
 * potential U_dip * |phi|^2 evaluated by the anisotropic truncated kernel method (Sec. 2.2), and
 * the Riemannian preconditioned conjugate gradient of Algorithm 1 (PCG-ATKM, Sec. 2.3).
 *
 * Conventions shared by every entry point:
 *  - Grid: box prod_a [-a_a, a_a) with N_a even points, x_j = -a + j h, h = 2a/N (Sec. 2.1).
 *  - Fields: contiguous C order [Nx][Ny][Nz], z fastest. Complex fields are interleaved
 *    (re, im): complex128 (double2) on BEC_FP64 grids, complex64 (float2) on BEC_FP32 grids.
 *    Real fields (Phi) are double / float accordingly. All field pointers are device pointers.
 *  - Inner product <u, v> = Re(h_x h_y h_z sum u conj(v)) (eq. "innerPro"); ||.||_inf unweighted.
 *  - Ownership: the caller owns every device buffer and the workspace (it asks
 *    bec_workspace_bytes for the size and allocates it). The handle holds host metadata and
 *    views into the workspace (twiddle and quadrature tables included); the library never
 *    allocates device memory. bec_pcg_solve creates and destroys a private stream, an event
 *    and a HIP graph per call.
 *  - Streams: all work is enqueued on the stream given to bec_init_grid (a hipStream_t, or
 *    NULL for the default stream) and is asynchronous, except calls that return host data
 *    (bec_energy with out_on_host, bec_pcg_solve), which synchronise that stream.
 *    A handle must not be used from two threads at once.
 *  - Batches: a grid may hold `batch` independent solves on the same box and grid (see
 *    bec_init_grid_batched). Then every `bec_params*` argument points to `batch` parameter
 *    sets, every field argument holds `batch` fields back to back ([batch][Nx][Ny][Nz]), and
 *    every per-solve output (mu, energies, results) has `batch` entries. One launch per phase
 *    serves the whole batch. bec_init_grid is the batch = 1 case.
 *  - Errors: arguments are validated before any launch; nothing throws or aborts. A HIP
 *    failure marks the handle (BEC_EHIP) and every later call on it returns BEC_EHIP.
 *    bec_last_error() gives a thread-local message for the last failing call.
 */
#ifndef BEC_H
#define BEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BEC_OK = 0,
    BEC_EINVAL = -1,    /* bad argument (odd/too small N, a <= 0, |n| != 1, NULL, ...) */
    BEC_ENOMEM = -2,    /* workspace too small */
    BEC_EHIP = -3,      /* HIP runtime error; the handle is unusable afterwards */
    BEC_ENOTCONV = -4,  /* max_iter reached; phi and the result are still written */
    BEC_ENUMERIC = -5,  /* NaN/Inf met; phi is rolled back to the last accepted iterate */
    BEC_ESTALL = -6     /* reserved */
};

/* BEC_MIXED is another name for BEC_FP32: a BEC_FP32 grid holds FP64 and FP32 fields and its
 * solves run the FP32 bulk phase, then the FP64 polish. */
typedef enum { BEC_FP64 = 0, BEC_FP32 = 1, BEC_MIXED = 1 } bec_precision;

/* Box and grid (Sec. 2.1): N_a even, 4 <= N_a <= 2048, each N_a = 2^i 3^j 5^k. */
typedef struct { int32_t n[3]; double a[3]; } bec_grid_desc;

/* Physical parameters (eqs. "DipGPE0", "Vpoten", "DDI-3D"): trap frequencies gamma, contact
 * strength beta, dipolar strength lambda, dipole axis n (unit; normalised if within 1e-12),
 * rotation speed Omega. */
typedef struct { double gamma[3]; double beta, lambda; double n[3]; double omega; } bec_params;

/* Energy parts (Sec. 3: E_kin, E_pot, E_int, E_dip, E_rot), chemical potential
 * mu = <H phi, phi> (eq. "EL"), mass h^3 sum |phi|^2 and virial residual
 * 2 E_kin - 2 E_pot + 3 E_int + 3 E_dip (eq. "vir_iden"). */
typedef struct { double E, Ekin, Epot, Eint, Edip, Erot, mu, mass, virial; } bec_energies;

/* Options of Algorithm 1. */
typedef struct {
    double tol_res_inf;    /* stop when ||H phi - mu phi||_inf <= tol (default 1e-8)          */
    double tol_step_inf;   /* 0 = off; the paper's rule ||phi_{n+1} - phi_n||_inf <= tol       */
    int32_t max_iter;      /* default 20000                                                   */
    int32_t max_halvings;  /* step halvings before a forced accept (default 30)               */
    double t_default;      /* step when the quadratic model is not convex (default 0.3)       */
    double tau_E_ulps;     /* energy-test slack in ulps of sum |E parts| (default 64)         */
    double switch_res;     /* mixed precision: FP32 -> FP64 when ||r||_inf <= this (1e-5),    */
                           /* times |mu| when switch_relative is set                          */
    int32_t check_every;   /* host polls the device state every k iterations (default 16)     */
    int32_t debug_flags;   /* bit0: force first trial step debug_t; bit1: force c2 = debug_c2 */
    double debug_t;
    double debug_c2;
    int32_t stall_window;  /* mixed: switch to FP64 if ||r||_inf has not improved this long   */
    int32_t use_graph;     /* 1: replay iterations from a captured HIP graph (default 1)     */
    int32_t switch_relative; /* 1 (default): the FP32 -> FP64 switch is ||r||_inf <= switch_res |mu| */
    int32_t branches;      /* 1 (default): passes that do not depend on each other run on a second */
                           /* stream beside the others; 0: every launch in order on one stream    */
} bec_pcg_opts;

typedef struct {
    int32_t status;        /* BEC_OK, BEC_ENOTCONV or BEC_ENUMERIC                             */
    int32_t iters, halvings, psd_resets, forced_accepts, fp32_iters;
    double res_inf, step_inf;
    bec_energies e;
} bec_pcg_result;

typedef struct bec_grid_s* bec_grid;

const char* bec_status_string(int status);
const char* bec_last_error(void);
int bec_version(void);

/* Workspace size in bytes for a grid and precision (one solve / `batch` solves). */
int bec_workspace_bytes(const bec_grid_desc* desc, int precision, size_t* bytes);
int bec_workspace_bytes_batched(const bec_grid_desc* desc, int precision, int batch, size_t* bytes);

/* Creates a handle over a caller-owned device workspace (>= bec_workspace_bytes, 256-byte
 * aligned) on `hip_stream`. Computes nothing yet. */
int bec_init_grid(const bec_grid_desc* desc, int precision, void* d_workspace, size_t ws_bytes,
                  void* hip_stream, bec_grid* out);
/* Same for a batch of 1..65535 independent solves on one box and grid (parameter sweeps,
 * training-set generation). The truncated-kernel symbol is shared by the batch. */
int bec_init_grid_batched(const bec_grid_desc* desc, int precision, int batch, void* d_workspace,
                          size_t ws_bytes, void* hip_stream, bec_grid* out);
int bec_grid_batch(bec_grid g);
int bec_destroy_grid(bec_grid g);

/* Truncated-kernel Fourier integral U_k of U = 1/(4 pi |y|) over the twofold box (Sec. 2.2,
 * eq. "FUk"; precomputed once per box and grid, Remark after eq. "U_TrunFour"), in FP64 on
 * every grid. It is real and even in each frequency, independent of the dipole axis; stored
 * as the octant [Nx+1][Ny+1][Nz+1] (index k_a = 0..N_a of the 2N_a-point padded axis).
 * Written to the workspace; also copied to d_uhat_octant if it is not NULL. */
int bec_atkm_symbol(bec_grid g, double* d_uhat_octant);

/* Dipolar potential Phi = U_dip * |phi|^2 on the grid by ATKM (Sec. 2.2, eqs. "DDI2Cou3D",
 * "fouriercoeff", "U_TrunFour"). Needs bec_atkm_symbol first. */
int bec_dipolar(bec_grid g, const bec_params* p, const void* d_phi, void* d_Phi);

/* H_phi phi = -1/2[[Lap]]phi + (V + beta|phi|^2 + lambda Phi)phi - Omega [[L_z]]phi
 * (Sec. 2.3, Euclidean gradient). d_hphi must not alias d_phi. Optional outputs: d_Phi (real
 * field) and d_mu (one double on the device, mu = <H phi, phi>). */
int bec_apply_H(bec_grid g, const bec_params* p, const void* d_phi, void* d_hphi,
                void* d_Phi, double* d_mu);

/* bec_apply_H for callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): no handle and no workspace argument. The
 * workspace is a static device array of bec_static_scratch_bytes() bytes (64 MiB), one per GPU,
 * held until the process ends; the grid's workspace (bec_workspace_bytes for BEC_FP64) must fit
 * in it, else BEC_EINVAL. FP64 fields only (complex128 d_phi, d_hphi; double d_Phi). The truncated-
 * kernel symbol is computed on the first call for a grid and kept until a call with another grid
 * or box. Work is enqueued on `hip_stream` (a hipStream_t or NULL), on the current device. All
 * calls on one GPU share its array: calls that overlap in time on one GPU (other streams or
 * threads without ordering) race and must be serialised by the caller. The first call on a device,
 * and a call whose grid differs from the previous call's, also upload twiddle tables and may
 * compute the symbol (synchronous copies); repeated calls on one grid only launch kernels. */
int bec_apply_H_static(const bec_grid_desc* desc, const bec_params* p, const void* d_phi, void* d_hphi,
                       void* d_Phi, double* d_mu, void* hip_stream);
int bec_static_scratch_bytes(size_t* bytes);

/* Energy parts of phi (Sec. 2.3 discrete energy; Sec. 3 virial identity). `out` is a host
 * pointer if out_on_host != 0 (the call then synchronises), else a device pointer. */
int bec_energy(bec_grid g, const bec_params* p, const void* d_phi, bec_energies* out,
               int out_on_host);

/* Algorithm 1 (PCG-ATKM) from the guess in d_phi (complex128, normalised by the caller) to
 * ||H phi - mu phi||_inf <= tol_res_inf. On BEC_FP64 grids every field is FP64. On BEC_FP32
 * grids the bulk runs on FP32 fields (FP64 reductions, energies and step coefficients) until
 * ||r||_inf <= switch_res or the residual stalls, then the same grid's FP64 buffers polish
 * from the renormalised FP32 result with a CG restart. Overwrites d_phi with the result.
 * `opts` may be NULL (defaults). Returns BEC_OK, BEC_ENOTCONV or BEC_ENUMERIC (the result
 * struct is filled in all three cases). Synchronises. */
int bec_pcg_solve(bec_grid g, const bec_params* p, void* d_phi, const bec_pcg_opts* opts,
                  bec_pcg_result* h_result);
/* Algorithm 1 for every solve of a batched grid at once: `p` holds `batch` parameter sets,
 * d_phi `batch` guesses, h_results `batch` results. Finished solves stop costing work (their
 * blocks return at once); the call returns when all are done. Returns the worst status
 * (BEC_ENUMERIC over BEC_ENOTCONV over BEC_OK). */
int bec_pcg_solve_batched(bec_grid g, const bec_params* p, void* d_phi, const bec_pcg_opts* opts,
                          bec_pcg_result* h_results);
/* Algorithm 1 for several grids of different sizes in one call (parameter sweeps over uneven
 * grids, e.g. the transverse resolution growing with Omega): grids[k] is a handle with its own
 * box, grid, precision and batch, params[k] its `batch` parameter sets, d_phis[k] its
 * [batch][Nx][Ny][Nz] complex128 guesses (overwritten with the results). Each grid runs on a
 * private stream of its own; the host issues every grid's iterations up to its next check of
 * the device states, then reads the grids in turn, so the grids' iterations run side by side on
 * the GPU and finished grids drop out. The handles must be distinct and use distinct
 * workspaces. h_results receives sum_k batch_k results in grid order. Each solve's result is the
 * one bec_pcg_solve_batched gives on its grid alone, bit for bit. Returns the worst status as
 * bec_pcg_solve_batched, or the first error. A project addition (no passage of the paper; the
 * sweeps are those of Sec. 3, critical rotational frequency). Synchronises. */
int bec_pcg_solve_ragged(bec_grid* grids, const bec_params* const* params, void* const* d_phis, int ngrids,
                         const bec_pcg_opts* opts, bec_pcg_result* h_results);
int bec_pcg_default_opts(bec_pcg_opts* opts);

/* 3-D C2C FFT on the N grid (unnormalised; dir = -1 forward exp(-2 pi i jk/N), +1 inverse),
 * the transform of the Fourier coefficients (eq. "FourphiCo") used by the operators. */
int bec_fft3d(bec_grid g, const void* d_in, void* d_out, int dir);

/* Spectral (trigonometric) interpolation of `batch` fields from grid src to grid dst on the
 * same box (Algorithm 2, step 2: hand-over of a ground state to another mesh; the paper leaves
 * the interpolant open, this is the Fourier series of eq. "Fourphi" evaluated on the new
 * points). Modes with |f_a| < min(N_src,a, N_dst,a)/2 are kept on every axis (both Nyquist
 * modes dropped); refining zero-pads the spectrum, coarsening truncates it. d_in holds src
 * fields in in_precision, d_out receives dst fields in out_precision (BEC_FP64: complex128,
 * BEC_FP32: complex64). Batch sizes must match. Runs on src's stream (synchronising it when
 * dst uses another stream); uses the FFT scratch and device state of both handles. */
int bec_interp_spectral(bec_grid src, bec_grid dst, const void* d_in, int in_precision, void* d_out,
                        int out_precision);
/* Scales each complex128 field of the batch to unit mass h_x h_y h_z sum |phi|^2 = 1
 * (the constraint of eq. "groundDef"). */
int bec_normalize(bec_grid g, void* d_phi);
/* Removes the global phase, which leaves the energy unchanged (Sec. 3, accuracy study):
 * each complex128 field is multiplied by a unit complex number so that sum phi G is real and
 * positive, G = exp(-(gamma_x x^2 + gamma_y y^2 + gamma_z z^2)/2) from p[b].gamma. A field with
 * sum phi G = 0 is left unchanged. */
int bec_gauge_fix(bec_grid g, const bec_params* p, void* d_phi);

/* Rotation about the z axis (Sec. 3, rotation-aligned error of vortex states): d_out(x) =
 * d_in(R_alpha x) for every complex128 field of the batch, R_alpha the rotation by alpha about
 * z through the box centre, evaluated exactly on the Fourier interpolant by three one-axis
 * Fourier shears (shear decomposition; angles beyond pi/2 are split into equal parts). Needs
 * N_x = N_y and a_x = a_y; the field is treated as periodic on the box, so it should have decayed
 * at the boundary. d_out may equal d_in. Runs with the solves of the handle marked active (it
 * clears the handle's device state). */
int bec_rotate_z(bec_grid g, const void* d_in, void* d_out, double alpha);

/* Measurement helper: runs one stage of the hot path `reps` times on the grid's stream and
 * returns the mean duration per run from HIP events (milliseconds). which = 0: the ATKM
 * padded x pass (forward, symbol multiply, inverse); 1: the whole ATKM potential of |phi|^2;
 * 2: the whole H phi apply; 3: the 3-D FFT of phi (forward); 4: a plain copy of one complex
 * field (bandwidth calibration); 5: the ATKM padded y forward pass; 6: the two-density
 * padded x Parseval pass of the step model. 0, 5 and 6 are timed as inside the iteration:
 * before each run the kernels that produce the pass's input run again, untimed, and the pass
 * kernel is launched with start and stop events of its own, so the mean is the kernel's
 * duration. Needs bec_atkm_symbol except for 3 and 4. Synchronises. */
int bec_time_stage(bec_grid g, const bec_params* p, const void* d_phi, int which, int reps, double* avg_ms);

/* Launch sites of one iteration of Algorithm 1, as reported by bec_pcg_profile. */
enum {
    BEC_SITE_CONTROL = 0,  /* single-thread control kernels and the energy finish of the apply   */
    BEC_SITE_FINISH,       /* ordered finishes of the FP64 block partial sums                     */
    BEC_SITE_PREC_Z,       /* r = H phi - mu phi, ||r||_inf, sqrt(P_V) r, forward z transform     */
    BEC_SITE_PREC_Y,       /* preconditioner y forward and inverse transforms (2 launches)       */
    BEC_SITE_PREC_X,       /* preconditioner x: forward, division by alpha + |nu|^2/2, inverse    */
    BEC_SITE_PREC_ZI,      /* inverse z, times sqrt(P_V) -> P r, direction inner products         */
    BEC_SITE_DIR_Z,        /* direction update p, z R2C of Re(conj(phi) p) and |p|^2, step sums  */
    BEC_SITE_Y_FWD,        /* ATKM padded y forward (2 for the step model, 1 in the apply)        */
    BEC_SITE_X_PARS2,      /* two-density padded x Parseval pass of the step model               */
    BEC_SITE_P_LINES,      /* kinetic and rotation Parseval sums of p along z, y, x (3 launches) */
    BEC_SITE_RETRACT,      /* retraction phi <- cos(t||p||) phi + sin(t||p||) p / ||p||           */
    BEC_SITE_ATKM_Z,       /* ATKM z R2C of |phi|^2 (pairs of real lines)                         */
    BEC_SITE_X_ATKM,       /* ATKM padded x pass: forward, symbol multiply, inverse              */
    BEC_SITE_Y_INV,        /* ATKM padded y inverse and crop                                      */
    BEC_SITE_ATKM_ZI,      /* ATKM z C2R and crop -> Phi                                          */
    BEC_SITE_H_Z,          /* kinetic line operator along z                                       */
    BEC_SITE_H_Y,          /* kinetic + rotation line operator along y                            */
    BEC_SITE_H_X,          /* kinetic + rotation line operator along x, assembles H phi           */
    BEC_SITE_OTHER,        /* renormalisation of the FP32 phase and anything else                 */
    BEC_NSITES
};

/* Measurement helper: runs `iters` iterations of Algorithm 1 from d_phi (overwritten with the
 * iterate reached) with no stopping test, launching every kernel eagerly with start and stop
 * events of its own on the stream it runs on, and accumulates per launch site (BEC_SITE_*)
 * the summed kernel durations in site_ms[BEC_NSITES] (milliseconds) and the launch counts in
 * site_launches[BEC_NSITES] (host arrays). flags bit 0: run the independent passes on a second
 * stream as the solver does (durations then include the sharing of the GPU); clear: every
 * launch in order on one stream (each kernel's own duration). On BEC_FP32 grids the iterations
 * are those of the FP32 bulk phase. The initial H phi apply is not counted. Synchronises. */
int bec_pcg_profile(bec_grid g, const bec_params* p, void* d_phi, int iters, int flags, double* site_ms,
                    int32_t* site_launches);

/* Launch-shape variants of the register-resident FFT kernels, per launch site (BEC_SITE_*):
 * 0 is the default shape; bit 0 halves the points per thread in blocks of twice the threads;
 * bit 1 exchanges whole complex values through LDS where the default exchanges one component at
 * a time (larger LDS tile, fewer barriers); bit 2 doubles the lines per block (blocks of twice
 * the threads, twice the LDS) for the lengths 256 and 512. For the
 * two-density Parseval pass bit 0 selects the line kernels' shape instead of its own (its two
 * transforms then run one after the other; its default runs them side by side, each butterfly's
 * twiddles formed once for both), and the other bits change nothing. Radices and every butterfly
 * stay the same, so fields are identical bit for bit under every variant; block sums group the
 * points by thread and block, so reductions change at rounding level. Variants exist for the
 * power-of-two lengths of at least 16 points per thread, for 256 and 512, and for lengths whose
 * default tile uses the split exchange; other sites ignore the setting. Values are
 * 0 .. BEC_KERNEL_VARIANTS-1. A project addition (performance only, no passage of the paper).
 * Arrays hold BEC_NSITES entries. */
#define BEC_KERNEL_VARIANTS 8
int bec_set_kernel_variants(bec_grid g, const int32_t* variants);
int bec_get_kernel_variants(bec_grid g, int32_t* variants);
/* Times every variant on every launch site with `iters` event-timed iterations of Algorithm 1
 * each (as bec_pcg_profile on one stream, from d_phi, which is overwritten), keeps per site that
 * has variants the fastest one if it beats the default by more than 2 % (of variants that launch
 * the same kernels at a site only the lowest counts), leaves the choice on
 * the grid and
 * returns it in variants_out; ms_default / ms_best receive the per-iteration milliseconds of
 * each site under the default and the chosen variant (all three nullable). Synchronises. */
int bec_autotune_kernels(bec_grid g, const bec_params* p, void* d_phi, int iters, int32_t* variants_out,
                         double* ms_default, double* ms_best);

/* Line tiles of the runtime-length FFT kernels: lengths without register kernels (those have
 * 32..1024 powers of two and 48, 96, 192, 384, 160, 320), or every length when the register
 * kernels are switched off. These kernels hold one tile of at
 * most 4096 complex values per block, 2048 for two-field passes. div[a] (a = 0: x, 1: y, 2: z)
 * divides the number of lines per block of every pass along axis a, padded passes included.
 * div[a] must be a power of two in [1, 16]; the default is 1. Tiles change the partition of the
 * lines among blocks and the order of the block partial sums, nothing else: fields are
 * unchanged bit for bit, and reductions change at rounding level. A project addition
 * (performance only, no passage of the paper). Takes effect from the next call on the handle. */
int bec_set_line_tiles(bec_grid g, const int32_t div[3]);
/* Current divisors; tunable (nullable) receives 1 for the axes that run a runtime-length pass. */
int bec_get_line_tiles(bec_grid g, int32_t div[3], int32_t tunable[3]);
/* Searches the divisors one axis at a time (z, y, x) over 1, 2, 4, 8, 16. Each candidate is
 * timed with HIP events as one H phi apply plus one two-density padded x Parseval pass on d_phi
 * and p, `reps` runs after a warm-up. Leaves the fastest set on the grid and returns it in
 * div_out (nullable) with its time in ms_out (nullable). Axes without a runtime-length pass are
 * skipped. Needs bec_atkm_symbol. Synchronises. */
int bec_autotune_line_tiles(bec_grid g, const bec_params* p, const void* d_phi, int reps, int32_t div_out[3],
                            double* ms_out);

#ifdef __cplusplus
}
#endif

#endif /* BEC_H */

/*
 * besselfdtd — MI355X (gfx950) FDTD solver for the Bessel-antenna method of
 * Ardaneh, Giust, Morel and Courvoisier, "Generation of a Bessel beam in FDTD
 * using a cylindrical antenna" (Opt. Express; arXiv 2102.12978).
 *
 * C ABI. Plain pointers and sizes only. Unless a call says otherwise:
 *   - host pointers are read (or written) during the call only, never kept;
 *   - the library owns every context and every device buffer it allocates;
 *   - a context is used by one host thread at a time;
 *   - fdtd_step and the adjoint/batch step calls are asynchronous on the
 *     stream given at creation; every read-back synchronises that stream;
 *   - no C++ exception or abort crosses the ABI: failures return a negative
 *     code and fdtd_last_error(ctx) holds a message.
 *
 * Units. Inputs are SI (metres, seconds, radians). Internally lengths are in
 * Δx, time in Δx/c, c = ε0 = μ0 = 1 and H is stored as H̃ = η0 H. Field
 * arrays on the host side are float32, indexed [k][j][i] = [z][y][x]
 * (x fastest), component order Ex, Ey, Ez, Hx, Hy, Hz.
 *
 * Discretisation (paper §4): standard second-order Yee scheme; E_x at
 * (i+½, j, k), E_y (i, j+½, k), E_z (i, j, k+½), H_x (i, j+½, k+½),
 * H_y (i+½, j, k+½), H_z (i+½, j+½, k). One step takes (E^n, H̃^{n+½}) to
 * (E^{n+1}, H̃^{n+3/2}): E update, then the E soft source at t_{n+1}, then the
 * H update, then the H soft source at t_{n+3/2}. z is periodic; x and y end
 * on PEC walls backed by a convolutional PML (CPML, §4), or are periodic in
 * the test mode FDTD_BC_PERIODIC.
 */
#ifndef BESSELFDTD_FDTD_H
#define BESSELFDTD_FDTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define FDTD_OK         0
#define FDTD_EINVAL    (-1)   /* bad argument (nothing was changed)          */
#define FDTD_ENOMEM    (-2)   /* device or host allocation failed            */
#define FDTD_EDEVICE   (-3)   /* a HIP call failed (no GPU, launch error)    */
#define FDTD_ESTATE    (-4)   /* call out of order (e.g. no injector set)   */
#define FDTD_EUNSTABLE (-5)   /* NaN/Inf or energy blow-up detected          */

/* ---- transverse boundary (x and y) ------------------------------------- */
#define FDTD_BC_CPML     0    /* CPML of cpml_cells cells, PEC behind it      */
#define FDTD_BC_PEC      1    /* bare PEC walls (cpml_cells must be 0)        */
#define FDTD_BC_PERIODIC 2    /* x and y periodic (test mode, no CPML)        */

/* ---- temporal envelope f(t) of the injected fields (§4) ---------------- */
#define FDTD_RAMP_SIN2  0     /* f = sin²(π t / 2 T_r) for t < T_r, then 1    */
#define FDTD_RAMP_GAUSS 1     /* f = exp(-(t - T0)² / T²), phase e^{-iω(t-T0)}*/
#define FDTD_RAMP_CW    2     /* f = 1                                        */

/* ---- polarisation of the injected beam (§3.1) ----------------------------
 * Hertz potential Π along x, y or z, J_m(K r) e^{imφ} e^{iβz}, Q = ∇×Π,
 * R = ∇×Q (the printed Cartesian forms of §3.1), paired as
 *   TE (the E2/H2 solution): Ẽ = i (E0/k) Q, H̃ = (E0/k²) R;
 *   TM (the E1/H1 solution): Ẽ = (E0/k²) R, H̃ = -i (E0/k) Q.
 * Π_x TE is the linearly y-polarised beam of the paper's runs, Π_y TE the
 * x-polarised one; Π_z gives for m = 0 the azimuthal (TE) and radial (TM)
 * polarisations. */
#define FDTD_POL_X_TE 0
#define FDTD_POL_Y_TE 1
#define FDTD_POL_Z_TE 2
#define FDTD_POL_X_TM 3
#define FDTD_POL_Y_TM 4
#define FDTD_POL_Z_TM 5

/* ---- injector flags (fdtd_injector.flags) ---------------------------------
 * FDTD_INJ_ALLOW_Z_MISFIT: accept a z length that holds a fractional number
 * of axial periods λ_z = λ / cos θ (for example nz from the truncation
 * int(p λ_z / Δz) of §4's sampling rule instead of fdtd_fit_periodic_z). z
 * stays periodic, so the injected phase e^{iβz} then jumps where the box
 * wraps; without the flag such a box is rejected. */
#define FDTD_INJ_ALLOW_Z_MISFIT 1

/* ---- kernel choice ------------------------------------------------------ */
#define FDTD_KERNEL_AUTO  0   /* fused kernel, tile shape from the autotuner  */
#define FDTD_KERNEL_SPLIT 1   /* two kernels per step (E, then H)            */
#define FDTD_KERNEL_FUSED 2   /* one fused E-then-H kernel per step           */

/* ---- state arrays for fdtd_get_state / fdtd_set_state ------------------
 * Fields: [nz][ny][nx]. CPML memories ψ live only in the slabs: the x-slab
 * arrays (ψ of the x derivatives: EYX, EZX, HYX, HZX) are [nz][ny][2*cpml]
 * holding x = 0..cpml-1 then x = nx-cpml..nx-1; the y-slab arrays (EXY, EZY,
 * HXY, HZY) are [nz][2*cpml][nx] holding y = 0..cpml-1 then ny-cpml..ny-1.  */
#define FDTD_EX 0
#define FDTD_EY 1
#define FDTD_EZ 2
#define FDTD_HX 3
#define FDTD_HY 4
#define FDTD_HZ 5
#define FDTD_PSI_EXY 6
#define FDTD_PSI_EYX 7
#define FDTD_PSI_EZX 8
#define FDTD_PSI_EZY 9
#define FDTD_PSI_HXY 10
#define FDTD_PSI_HYX 11
#define FDTD_PSI_HZX 12
#define FDTD_PSI_HZY 13

/* ---- diagnostics mask (fdtd_set_diagnostics) ---------------------------- */
#define FDTD_DIAG_EX2    1u   /* accumulate E_x² on the plane                */
#define FDTD_DIAG_EY2    2u   /* accumulate E_y² on the plane (§5 intensity) */
#define FDTD_DIAG_EZ2    4u   /* accumulate E_z² on the plane                */
#define FDTD_DIAG_ENERGY 8u   /* W^{n+1} = Σ(E^{n+1})² + Σ H̃^{n+½}·H̃^{n+3/2}  */

typedef struct fdtd_ctx fdtd_ctx;

typedef struct fdtd_grid {
    int32_t nx, ny, nz;       /* cells; nx, ny >= 2, nz >= 1                  */
    double dx, dy, dz;        /* cell sizes (m); dz normally from              */
                              /* fdtd_fit_periodic_z                           */
    double courant;           /* S = c Δt / Δx; S·sqrt(1+(Δx/Δy)²+(Δx/Δz)²)<1 */
    int32_t bc_xy;            /* FDTD_BC_*                                     */
    int32_t cpml_cells;       /* CPML thickness (cells), 1 <= cpml <= n/2      */
    double cpml_grade;        /* polynomial grade g of σ and κ                 */
    double cpml_sigma_scale;  /* σ_max in units of 0.8 (g+1) / (η0 Δ)          */
    double cpml_kappa_max;    /* κ at the PEC wall (>= 1)                      */
    double cpml_alpha_max;    /* CFS α at the interface, α Δx / (ε0 c)          */
    int32_t kernel;           /* FDTD_KERNEL_*                                 */
    int32_t reserved;         /* set to 0                                      */
    void *stream;             /* hipStream_t to run on; NULL = null stream     */
} fdtd_grid;

typedef struct fdtd_injector {
    double wavelength;        /* λ (m)                                         */
    double theta;             /* cone angle θ (rad), 0 < θ < π/2               */
    int32_t order;            /* Bessel order m >= 0 (the paper's m)           */
    int32_t ramp_kind;        /* FDTD_RAMP_*                                   */
    double e0;                /* amplitude E0 of the injected TE Π_x beam      */
    double r_outer;           /* outer antenna radius R_B (m)                  */
    double thickness;         /* antenna thickness δs (m), 0 < δs < R_B        */
    double axis_x, axis_y;    /* beam axis from the x = 0 / y = 0 walls (m);   */
                              /* NaN = grid centre                             */
    double ramp_a;            /* SIN2: T_r (s); GAUSS: T (s)                   */
    double ramp_b;            /* GAUSS: T0 (s)                                 */
    int32_t n_sectors;        /* 0, or number of angular sectors of weights    */
    int32_t polarization;     /* FDTD_POL_* (0: Π_x TE, the paper's runs)      */
    const double *sector_amp;   /* host [n_sectors] amplitudes a_s, or NULL    */
    const double *sector_phase; /* host [n_sectors] phases φ_s (rad), or NULL  */
    int32_t flags;            /* FDTD_INJ_* bits; 0 = none                       */
} fdtd_injector;

typedef struct fdtd_info {
    int32_t nx, ny, nz, pitch;   /* pitch: floats between x rows on device   */
    double sx, sy, sz;           /* S Δx/Δ_d                                  */
    double k, beta, kr, omega;   /* normalised (1/Δx, 1/(Δx/c))              */
    int32_t n_source[6];         /* antenna points per component per plane   */
    int32_t n_slots;             /* antenna columns                          */
    int32_t kernel;              /* kernel in use                            */
    int32_t tile_rows;           /* fused kernel: y rows per wavefront        */
    int32_t tile_zchunk;         /* fused kernel: z planes per wavefront      */
    int64_t step;                /* completed steps                           */
    int64_t device_bytes;        /* device memory held by the context         */
    int64_t interior_cells;      /* cells per step updated by the fused kernel */
    int32_t frame;               /* FDTD_FRAME_* used around the interior     */
    int32_t xalign;              /* interior x origin multiple (32 or 64)     */
    int32_t frame_rows;          /* rows per fused frame tile (2 or 4)        */
    int32_t time_block;          /* steps per pass (1, 2 or 3)                */
    int32_t tb_rows;             /* 2-/3-step kernel: y rows per wavefront    */
    int32_t tb_zchunk;           /* 2-/3-step kernel: z planes per chunk      */
} fdtd_info;

/* Library version string (static storage). */
const char *fdtd_version(void);

/* Periodic z fit (§4 sampling rule, z-periodic box): the box holds
 * p = max(1, round(nz_hint Δx / λ_z)) whole axial periods λ_z = λ / cos θ;
 * *nz = round(p λ_z / Δx) and *dz = p λ_z / *nz exactly (rounding half up).
 * Pure host function; returns FDTD_EINVAL for non-positive inputs or θ
 * outside (0, π/2). */
int fdtd_fit_periodic_z(double wavelength, double theta, double dx, int32_t nz_hint,
                        int32_t *nz, double *dz);

/* The antenna's source points as fdtd_set_injector would install them for
 * this grid (§4 antenna: R_B - δs < r <= R_B at each component's own
 * staggered position; tangential E on a PEC wall excluded; §3.1 sector
 * weights indexed by s = floor(n_sectors φ / 2π), φ in [0, 2π) the point's
 * azimuth about the axis). Pure host function (no GPU call). out receives
 * 4 int32 per point, in the library's slot order (columns y-major, then
 * component Ex..Hz): component, i, j, sector (-1 when n_sectors is 0).
 * *count is set to the number of points; FDTD_EINVAL when cap (points) is
 * smaller, or for a grid or injector that fdtd_create / fdtd_set_injector
 * would reject. */
int fdtd_antenna_points(const fdtd_grid *grid, const fdtd_injector *inj, int32_t *out,
                        int64_t cap, int64_t *count);

/* Create a solver (§4: Yee grid, CPML on x/y, periodic z). Validates the
 * grid (sizes, Courant condition, CPML thickness) before touching the GPU,
 * then allocates the ping-pong field and CPML buffers on the current HIP
 * device and zeroes them. On success *out owns everything; free it with
 * fdtd_destroy. On failure *out is NULL. */
int fdtd_create(const fdtd_grid *grid, fdtd_ctx **out);

/* Field layout of a grid on the device (pure host function; no GPU call).
 * A field component is nz x ny rows of *pitch floats, x fastest; *pitch is
 * nx rounded up to a multiple of 64 (256-byte rows) and the cells x >= nx of
 * a row are padding that no kernel reads or writes. One parity holds the six
 * components Ex, Ey, Ez, Hx, Hy, Hz in that order, one after another:
 * *parity_floats = 6 nz ny pitch. Returns FDTD_EINVAL for a grid that
 * fdtd_create would reject or NULL outputs. */
int fdtd_field_layout(const fdtd_grid *grid, int32_t *pitch, int64_t *parity_floats);

/* fdtd_create with the two ping-pong parities of the six field components in
 * caller-owned device memory (for example two torch tensors), for callers
 * that want the fields without copies. dev_fields[0] and dev_fields[1] each
 * hold fdtd_field_layout's parity_floats floats; they must be device memory
 * of the current device, 256-byte aligned and disjoint, and each must lie
 * inside one device allocation (checked: FDTD_EINVAL otherwise; a buffer
 * that is too short but sits inside a larger allocation, as a slice of a
 * caching allocator's block can, is not detected and is overrun). The
 * library zeroes them on the grid's stream during this call, reads and
 * writes them on that stream while stepping and never frees them: they must
 * outlive the context. The CPML memories, tables and every other buffer stay
 * library-owned and count in fdtd_info.device_bytes; the two field buffers
 * do not. Everything else behaves as for fdtd_create. */
int fdtd_create_ext(const fdtd_grid *grid, float *const dev_fields[2], fdtd_ctx **out);

/* Device address of the parity buffer that holds the current state
 * (E^n and H̃^{n+1/2} after n steps; six components in the fdtd_field_layout
 * layout): one of the two buffers of fdtd_create_ext, or a library-owned one.
 * It changes with every step call (a two- or three-step pass flips the
 * parity once per pass), so query it after stepping; the contents are complete once the
 * grid's stream has finished the steps. */
int fdtd_current_fields(const fdtd_ctx *ctx, float **dev_ptr);

/* Free the context and all its device memory (not the caller's buffers of
 * fdtd_create_ext). NULL-safe. */
int fdtd_destroy(fdtd_ctx *ctx);

/* Message of the last failure on ctx (or of the last failed fdtd_create when
 * ctx is NULL). Static or context-owned storage; valid until the next call. */
const char *fdtd_last_error(const fdtd_ctx *ctx);

/* Install the Bessel antenna (§3.1 TE fields of the Π_x potential, §4 antenna
 * and soft source): every component location with R_B - δs < r <= R_B from
 * the axis becomes a source point for the whole z length; its complex
 * amplitude Ã_c (Ẽ = i (E0/k) Q, H̃ = (E0/k²) R) is computed in double
 * precision, J_ν from std::cyl_bessel_j. Each step adds
 * Re{w_s Ã_c e^{iβ z_c} f(t) e^{-iω(t - T0)}} to that component. With
 * n_sectors > 0 the weight w_s = a_s e^{iφ_s} of the sector
 * s = floor(n_sectors φ_c / 2π) of the point's azimuth multiplies Ã_c.
 * Requires an integer number of axial periods in the box (|β nz Δz / 2π -
 * round| <= 1e-6) unless inj->flags holds FDTD_INJ_ALLOW_Z_MISFIT; unknown
 * flag bits are rejected. inj == NULL removes the antenna. */
int fdtd_set_injector(fdtd_ctx *ctx, const fdtd_injector *inj);

/* Replace the sector weights of the installed antenna (host arrays of n
 * doubles). n must equal the injector's n_sectors. */
int fdtd_set_sector_weights(fdtd_ctx *ctx, int32_t n, const double *amp, const double *phase);

/* Diagnostics (§5). For every step n >= window_begin_step (0-based step
 * index; E^{n+1} is accumulated) the selected squares of E on plane
 * k = k_plane are summed in double precision; fdtd_fluence returns their
 * mean. Also resets the sums and the count. FDTD_DIAG_ENERGY records W after
 * every step. */
int fdtd_set_diagnostics(fdtd_ctx *ctx, int32_t k_plane, int64_t window_begin_step,
                         uint32_t mask);

/* Advance nsteps leapfrog steps on the context's stream (asynchronous). */
int fdtd_step(fdtd_ctx *ctx, int64_t nsteps);

/* fdtd_step for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same steps, kernels
 * and results (bit for bit) as fdtd_step, but the call allocates, frees and
 * creates nothing: the energy diagnostic's per-workgroup partial sums go to
 * a 2 MiB static device array (at most 262,144 partials: FDTD_EINVAL, with
 * nothing stepped, when a grid and tile need more), the two-step kernel's
 * boundary launches run on the context's stream after the interior one,
 * no profiling marks are taken, and the time tables are not grown (steps
 * past their end: FDTD_ESTATE, nothing stepped; fdtd_set_injector builds
 * them 1024 steps ahead and fdtd_step grows them). The static array is
 * shared by every context on a device and keeps the last call's contents
 * (each energy step clears the part it uses): calls that overlap on one GPU,
 * from two host threads or on two streams, race. */
int fdtd_step_static(fdtd_ctx *ctx, int64_t nsteps);

/* Mean over the window of one plane quantity (FDTD_DIAG_EX2, _EY2 or _EZ2),
 * written to host_out[ny*nx] (x fastest). Synchronises. n = capacity.
 * Returns FDTD_EUNSTABLE (after writing host_out) if any sum is NaN or
 * infinite. */
int fdtd_fluence(fdtd_ctx *ctx, uint32_t quantity, float *host_out, int64_t n);

/* Number of steps accumulated in the fluence sums. */
int fdtd_fluence_count(const fdtd_ctx *ctx, int64_t *count);

/* W after the most recent step (FDTD_DIAG_ENERGY must be on). Synchronises;
 * returns FDTD_EUNSTABLE if W is not finite. */
int fdtd_energy(fdtd_ctx *ctx, double *out);

/* Copy one state array (FDTD_EX .. FDTD_PSI_HZY) to / from the host; n is
 * the element count of the host array and must match the array's size
 * (nz*ny*nx for fields, the slab sizes above for ψ). Synchronises. */
int fdtd_get_state(fdtd_ctx *ctx, int32_t which, float *host, int64_t n);
int fdtd_set_state(fdtd_ctx *ctx, int32_t which, const float *host, int64_t n);

/* Zero fields, CPML memories, diagnostics and the step counter. */
int fdtd_reset(fdtd_ctx *ctx);

/* Sizes, derived constants, antenna counts, kernel choice. */
int fdtd_get_info(const fdtd_ctx *ctx, fdtd_info *out);

/* Analytic reference on the diagnostic plane: ½ E0² cos²θ J_m²(K r) at the
 * E_y positions (the time average of E_y² of the CW beam, §3.1/§5), written
 * to host_out[ny*nx]. Requires an injector of polarisation FDTD_POL_X_TE
 * (FDTD_ESTATE otherwise). */
int fdtd_analytic_ey2(fdtd_ctx *ctx, float *host_out, int64_t n);

/* Select the fused kernel's tile shape explicitly: y rows per wavefront in
 * {4, 8} (a wavefront covers 64 x cells and marches along z); z chunk in
 * planes per wavefront, 0 = the whole z extent. Returns FDTD_EINVAL
 * otherwise. A new context starts with 4 rows and the z
 * chunk that gives the interior kernel about 32 workgroups per compute unit
 * (at least 4 planes; the whole z when that already suffices). */
int fdtd_set_tile(fdtd_ctx *ctx, int32_t rows, int32_t zchunk);

/* How the fused kernel's frame (the CPML slabs, walls and the cells the
 * interior's tiles leave over) is stepped:
 *   FDTD_FRAME_SPLIT: the split E and H kernels, one thread per cell;
 *   FDTD_FRAME_FUSED: one launch of the fused step over the 64 x `rows`
 *     tiles (rows 2 or 4) that hold frame cells, each cell through the same
 *     per-cell boundary code as the split kernels, marching a z chunk like
 *     the interior.
 * xalign (32 or 64) rounds the interior's x origin up to a multiple of that
 * many cells; 64 makes the frame's x strips whole tiles. */
#define FDTD_FRAME_SPLIT 0
#define FDTD_FRAME_FUSED 1
int fdtd_set_frame(fdtd_ctx *ctx, int32_t kind, int32_t xalign, int32_t rows);

/* Steps per pass over the fields (temporal blocking). steps = 1: every
 * step runs the one-step kernels. steps = 2: pairs of steps run the
 * two-step kernel over the whole grid (the Yee update of §4 with its CPML
 * and soft source applied twice in registers: each field and CPML memory
 * is read and written once per pair, 24 B of fields per cell-update), on
 * tiles of 60 x cells by `rows` (2 or 4) rows marching through z chunks of
 * zchunk planes (0 = the whole z; corner and y-wall tiles take at most 8
 * and 16 planes); tiles free of walls and CPML, tiles at the x walls, at
 * the y walls and at the corners run as four launches, the three boundary
 * ones on streams the context creates, concurrent with the interior one
 * (forked from and joined back into the context's stream by events). No
 * buffer is allocated. The result is bit-identical to one-step runs. Pairs
 * fall back to single steps for the split kernel choice, the periodic test
 * mode, and while the energy diagnostic or a plane record is on; an odd
 * last step runs alone. steps = 3: triples of steps run the three-step
 * kernel (the update applied three times in registers, 16 B of fields per
 * cell-update) on tiles of 58 x cells by `rows` rows in the same four
 * launches and under the same fallbacks; a remainder of two steps runs as a
 * pair through the two-step kernel, one step alone. Other values:
 * FDTD_EINVAL. */
int fdtd_set_time_block(fdtd_ctx *ctx, int32_t steps, int32_t rows, int32_t zchunk);

/* Whether the two- and three-step kernels' three boundary launches run beside the
 * interior one on the context's side streams (on = 1, the default) or one
 * after another on the context's stream (on = 0), for example to time each
 * launch alone with fdtd_profile_enable. Results are the same bit for bit
 * either way. FDTD_EINVAL for other values. */
int fdtd_set_concurrency(fdtd_ctx *ctx, int32_t on);

/* Time candidate tile shapes and frame choices on the live problem (the state
 * is restored) and keep the fastest: the one-step kernel's rows x z chunks x
 * frames, and, except in the periodic test mode, the two-step and the
 * three-step kernels (fdtd_set_time_block) at rows {4, 2} x z chunks {nz/8,
 * nz/16, nz/4, nz/2, whole} (rounded up, repeats dropped). Each
 * candidate is timed over at least steps_per_trial steps, and over more
 * until the timed span reaches about 2 ms. One-step trials read what the
 * previous trial wrote, as a run does: they go back and forth between the
 * free parity and a scratch set of fields and CPML memories that this call
 * allocates and frees (when the device lacks the memory, each trial re-runs
 * the same step from the live state instead). *best_rows / *best_zchunk (may
 * be NULL) receive the one-step kernel's tile; fdtd_get_info reports
 * whether the two- or three-step kernel won (time_block) and its tile. */
int fdtd_autotune(fdtd_ctx *ctx, int32_t steps_per_trial, int32_t *best_rows,
                  int32_t *best_zchunk);

/* ---- kernel timing --------------------------------------------------------
 * With profiling on, every kernel the context launches is bracketed by HIP
 * events on its stream; fdtd_profile_read synchronises and returns, per
 * kernel name, the number of launches and their summed duration (ms). */
typedef struct fdtd_kernel_profile {
    char name[48];
    int64_t launches;
    double total_ms;
} fdtd_kernel_profile;

/* Turn per-launch timing on (1) or off (0); either way the counters reset. */
int fdtd_profile_enable(fdtd_ctx *ctx, int32_t on);

/* Copy up to max entries; *count receives the number of kernel names. */
int fdtd_profile_read(fdtd_ctx *ctx, fdtd_kernel_profile *out, int32_t max, int32_t *count);

/* ---- memory-roofline probe ------------------------------------------------
 * Not part of the method: the measurement that the Yee kernels' HBM
 * fraction is read against. Allocates two device buffers of `bytes` bytes
 * each (freed before returning), then times `reps` passes of a plain
 * streaming kernel on `stream` (NULL: the null stream) with HIP events:
 *   FDTD_PROBE_COPY  reads one buffer and writes the other (2·bytes moved);
 *   FDTD_PROBE_READ  reads one buffer (bytes moved);
 *   FDTD_PROBE_WRITE writes one buffer (bytes moved).
 * bytes must be a positive multiple of 16; reps in [1, 1000]. On success
 * *ms_per_pass is the mean pass time and *gbs the moved bytes per second
 * in GB/s. Synchronous; returns FDTD_ENOMEM if the buffers cannot be had. */
#define FDTD_PROBE_COPY  0
#define FDTD_PROBE_READ  1
#define FDTD_PROBE_WRITE 2
int fdtd_stream_probe(int32_t kind, int64_t bytes, int32_t reps, void *stream,
                      double *ms_per_pass, double *gbs);

/* ---- adjoint: gradient of an intensity loss w.r.t. the sector weights ----
 * The scheme is linear in (E, H̃, ψ) plus an additive source, so reverse-
 * mode differentiation is the transposed step run backwards in time: for a
 * forward curl term ψ' = bψ + cΔ, u' = u + σ S_d((1/κ)Δ + ψ'), the transpose
 * is μ = σ S_d λ_u', λ_Δ = (1/κ + c)μ + cλ_ψ', λ_ψ = b(μ + λ_ψ'), and the
 * differenced field receives the transposed difference of λ_Δ (PEC-held
 * components contribute nothing). The loss L(Ī) depends on the window mean
 * Ī of E_y² on one plane (§5 intensity); ∂L/∂Ī comes from the caller. The
 * gradient with respect to a sector weight w_s = a_s e^{iφ_s} (set with
 * fdtd_set_injector / fdtd_set_sector_weights, §4 amplitudes) is
 *   ∂L/∂a_s = Σ_{points of s} Re{e^{iφ_s} Ã G},  ∂L/∂φ_s = -Σ Im{w_s Ã G},
 *   G = Σ_n T(t) Σ_k λ(k) e^{iβ z(k)}  (T the time factor of that half step).
 * The forward run stores the full state every checkpoint_every steps; the
 * reverse sweep regenerates, segment by segment from those checkpoints, the
 * E_y planes the loss needs, so only one segment of planes is held. */
typedef struct fdtd_adjoint fdtd_adjoint;

typedef struct fdtd_adjoint_info {
    int32_t checkpoint_every;
    int32_t checkpoints;         /* state snapshots held                        */
    int32_t antenna_columns;     /* slots of the per-point correlations G       */
    int32_t reserved;
    int64_t forward_steps;       /* steps of the last fdtd_adjoint_forward      */
    int64_t recompute_steps;     /* forward steps redone by the last backward   */
    int64_t device_bytes;        /* λ state, checkpoints, plane records, G      */
    int64_t forward_runs;        /* completed fdtd_adjoint_forward calls        */
} fdtd_adjoint_info;

/* Attach an adjoint to a forward context (which it borrows). Destroying the
 * forward context first detaches the adjoint: its calls then return
 * FDTD_ESTATE, and fdtd_adjoint_destroy still frees it. Allocates λ (two parities of fields and CPML memories,
 * like the forward state) and one segment of plane records.
 * checkpoint_every >= 1. The transposed step follows the forward context's
 * kernel choice: with the fused kernel its interior runs through the fused
 * interior kernel (the forward step with negated Courant factors) and the
 * transposed CPML kernels take the frame. */
int fdtd_adjoint_create(fdtd_ctx *fwd, int32_t checkpoint_every, fdtd_adjoint **out);

/* Free the adjoint's device memory. NULL-safe. */
int fdtd_adjoint_destroy(fdtd_adjoint *a);

/* Message of the last failure on a (or of the last failed create). */
const char *fdtd_adjoint_last_error(const fdtd_adjoint *a);

/* Reset the forward context and run nsteps steps from zero fields with
 * Ī = window mean of E_y² on plane k_plane over steps >= window_begin
 * (fdtd_fluence(fwd, FDTD_DIAG_EY2) reads it), storing a checkpoint every
 * checkpoint_every steps. Requires an injector. */
int fdtd_adjoint_forward(fdtd_adjoint *a, int64_t nsteps, int32_t k_plane, int64_t window_begin);

/* Reverse sweep for ∂L/∂Ī = dl_dI[ny*nx] (host, x fastest; n = ny*nx):
 * writes ∂L/∂a_s and ∂L/∂φ_s of the n_sectors sector weights to
 * grad_amp / grad_phase. Synchronises. Returns FDTD_ESTATE, changing
 * nothing, when fdtd_set_injector or fdtd_set_sector_weights ran on the
 * forward context after the last fdtd_adjoint_forward (the checkpoints
 * belong to the old antenna). The forward context is left at the
 * end of the last recomputed segment (its fluence sums are untouched). */
int fdtd_adjoint_backward(fdtd_adjoint *a, const float *dl_dI, int64_t n, int32_t n_sectors,
                          double *grad_amp, double *grad_phase);

/* Per-point correlations G of the last backward: [slot][component][re, im]
 * (n = 12 * antenna_columns doubles; slots in the antenna's column order,
 * components Ex, Ey, Ez, Hx, Hy, Hz). */
int fdtd_adjoint_source_correlation(fdtd_adjoint *a, double *host, int64_t n);

/* nsteps source-free transposed steps applied to the λ state as it is (for
 * transposition checks). */
int fdtd_adjoint_transpose(fdtd_adjoint *a, int64_t nsteps);

/* λ arrays, same ids, host layouts and sizes as fdtd_get_state. */
int fdtd_adjoint_get_state(fdtd_adjoint *a, int32_t which, float *host, int64_t n);
int fdtd_adjoint_set_state(fdtd_adjoint *a, int32_t which, const float *host, int64_t n);

int fdtd_adjoint_get_info(const fdtd_adjoint *a, fdtd_adjoint_info *out);

/* ---- batch: many independent instances advanced together -----------------
 * A batch owns `count` solver contexts of uneven grid size, cone angle and
 * order (each made as by fdtd_create with FDTD_KERNEL_SPLIT on the batch's
 * stream, then fdtd_set_injector) and advances them in lockstep. Every step
 * walks a single flattened list of work items covering all instances with a
 * persistent grid: by default an E launch and an H launch over blocks of
 * flattened columns, or one fused launch over tiles (instance, 64 x cells,
 * 4 rows, z chunk). Either way the per-cell arithmetic is that of the
 * split kernels, so every instance evolves bit-identically to a
 * single-domain FDTD_KERNEL_SPLIT run of the same problem. Runs of
 * graph_steps steps are recorded once into a HIP graph and replayed; the
 * step index lives in a device counter so a replay stays valid. */
typedef struct fdtd_batch fdtd_batch;

typedef struct fdtd_batch_info {
    int32_t count;               /* instances                                  */
    int32_t tile_cols;           /* columns per work item (= workgroup size)  */
    int32_t tile_zchunk;         /* z planes per work item, 0 = whole z        */
    int32_t work_items;          /* flattened work list length                 */
    int32_t blocks;              /* persistent grid (workgroups per launch)    */
    int32_t graph_steps;         /* steps per graph replay, 0 = no graphs      */
    int64_t cells;               /* sum of nx*ny*nz over the instances         */
    int64_t step;                /* completed steps                            */
    int64_t device_bytes;        /* device memory held by batch and instances  */
    int32_t kernel;              /* FDTD_KERNEL_FUSED or FDTD_KERNEL_SPLIT      */
    int32_t reserved;
    int32_t time_block;          /* steps per pass (2: the two-step kernel)     */
    int32_t tb_rows;             /* two-step kernel: rows per wavefront         */
    int32_t tb_zchunk;           /* two-step kernel: z planes per work item     */
    int32_t tb_items;            /* two-step kernel: work items per pair        */
} fdtd_batch_info;

/* Create a batch. grids[count] (their stream and kernel fields are ignored:
 * the batch's stream and the split kernel choice are used); injectors is
 * NULL (no antennas) or holds count entries. Every instance is validated as
 * by fdtd_create / fdtd_set_injector; the first failure is returned with
 * the instance index in fdtd_batch_last_error(NULL). On failure *out is
 * NULL and nothing is kept. */
int fdtd_batch_create(int32_t count, const fdtd_grid *grids, const fdtd_injector *injectors,
                      void *stream, fdtd_batch **out);

/* Free the batch and its instances. NULL-safe. */
int fdtd_batch_destroy(fdtd_batch *b);

/* Message of the last failure on b (or of the last failed create when b is
 * NULL). */
const char *fdtd_batch_last_error(const fdtd_batch *b);

/* Borrowed handle of instance q (NULL when out of range), valid until the
 * batch is destroyed. Read-backs (fdtd_get_state, fdtd_fluence, _count,
 * fdtd_get_info, fdtd_analytic_ey2), fdtd_set_state, fdtd_set_diagnostics
 * (window steps count from the batch's step 0), fdtd_set_injector and
 * fdtd_set_sector_weights work on it as on any context; fdtd_step,
 * fdtd_reset, fdtd_set_tile, fdtd_set_frame, fdtd_set_time_block,
 * fdtd_autotune and fdtd_destroy return
 * FDTD_ESTATE. The energy diagnostic is not computed for batch instances. */
fdtd_ctx *fdtd_batch_instance(fdtd_batch *b, int32_t q);

/* Advance every instance nsteps steps (asynchronous on the batch's stream). */
int fdtd_batch_step(fdtd_batch *b, int64_t nsteps);

/* Step kernel: FDTD_KERNEL_SPLIT (default: an E launch and an H launch
 * over flattened columns) or FDTD_KERNEL_FUSED (one launch per step over
 * tiles of 64 x cells by `rows` rows (2 or 4; ignored by the split kernel)
 * marching through a z chunk, the boundary cases handled per cell;
 * bit-identical to the split kernels). The autotuner tries both. */
int fdtd_batch_set_kernel(fdtd_batch *b, int32_t kernel, int32_t rows);

/* Work-item shape: cols in {64, 128, 256} (split kernel only), zchunk >= 0
 * (z planes per work item, 0 = whole z; for the split kernel 1 launches one
 * workgroup per column block and plane instead of the persistent grid). */
int fdtd_batch_set_tile(fdtd_batch *b, int32_t cols, int32_t zchunk);

/* Steps per pass (temporal blocking), as fdtd_set_time_block for a single
 * context: steps = 2 runs pairs of steps of every instance through the
 * two-step kernel over each whole grid (walls and CPML included; four
 * launches per pair, one per tile class, over work items (instance, 60-cell
 * x segment, row group of 4 * rows rows, z chunk of zchunk planes, 0 = the
 * whole z)); an odd last step runs the step kernel of fdtd_batch_set_kernel.
 * Bit-identical to one-step runs. rows: 2 or 4. Refused (FDTD_EINVAL) when
 * an instance is in the periodic test mode. */
int fdtd_batch_set_time_block(fdtd_batch *b, int32_t steps, int32_t rows, int32_t zchunk);

/* Steps recorded per graph: an even number in [2, 1000], or 0 to launch
 * every step directly. */
int fdtd_batch_set_graph_steps(fdtd_batch *b, int32_t steps);

/* Time every kernel and work-item shape (fused with zchunk in
 * {0, 32, 16, 8}; split with cols x zchunk in {64, 128, 256} x
 * {0, 16, 8, 4, 1}; and, without periodic instances, the two-step kernel at
 * rows {2, 4} x zchunk {16, 32, 8, 0}) for steps_per_trial steps on the live
 * state and keep the fastest (fdtd_batch_get_info reports whether the
 * two-step kernel won); *best_cols is 0 when the fused kernel wins among the
 * one-step kernels, which odd steps use. Trials write only the buffers of
 * the next parity, so the state is unchanged. */
int fdtd_batch_autotune(fdtd_batch *b, int32_t steps_per_trial, int32_t *best_cols,
                        int32_t *best_zchunk);

int fdtd_batch_get_info(const fdtd_batch *b, fdtd_batch_info *out);

#ifdef __cplusplus
}
#endif

#endif /* BESSELFDTD_FDTD_H */

/*
 * zda.h -- C ABI of the MI355X (gfx950) library for one zone of zoned discrete
 * axisymmetry (ZDA), arXiv 2501.07979: the cylindrical (r, phi, z) Yee FDTD
 * of one annular-sector zone with n-fold Bloch periodicity in phi, CPML in r
 * and z, a soft pulsed current source, on-the-fly multi-frequency DFT
 * monitors, and the adjoint run with the permittivity-gradient overlap.
 *
 * Conventions shared by every call
 *  - Units eps0 = mu0 = c = 1, mu = 1.  Cell (i, j, k): i radial in [0, nr),
 *    j azimuthal in [0, nphi), k axial in [0, nz).  r_p = r_in + p dr,
 *    dphi = 2 pi / (n_fold nphi), dt = courant * min(dr, dz).
 *  - Every 3-D array is [nz][nr][nphi] (phi fastest), row-major, FP32.
 *    Complex arrays are interleaved (re, im) pairs of float.
 *  - Component samples sit on the staggered Yee grid: E_r (i+1/2, j, k),
 *    E_phi (i, j+1/2, k), E_z (i, j, k+1/2), H_r (i, j+1/2, k+1/2),
 *    H_phi (i+1/2, j, k+1/2), H_z (i+1/2, j+1/2, k).  The stored field is the
 *    physical Bloch field; crossing the wedge boundary multiplies by
 *    exp(+-i m 2 pi / n_fold) (eq. 1-2 of the paper).
 *  - Pointers flagged *_on_device are HIP device pointers on the zone's
 *    device, otherwise host pointers.  Input buffers are copied; the caller
 *    keeps ownership of everything it passes.  The zone owns all its device
 *    memory and frees it in zda_zone_destroy.
 *  - Every zone has a stream (a hipStream_t, NULL = the default stream):
 *    the stream of its last zda_fdtd_run / zda_adjoint_grad, or the one given
 *    to zda_zone_set_stream.  Calls that take a `stream` make it the zone's
 *    stream.  All work of a zone is ordered on its stream and asynchronous;
 *    a call waits for the stream only when it reads into host memory, takes
 *    host input that it must copy before returning, or is zda_zone_sync.
 *    Device inputs must stay valid until the stream has consumed them.
 *    Calls on one zone must not overlap; different zones are independent.
 *  - Device memory is allocated with hipMalloc, or through the functions
 *    registered with zda_set_allocator.
 *  - Every call returns a zda_status; no exception or abort crosses the ABI.
 *    zda_last_error() gives a message for the last failure on the calling
 *    thread.
 */
#ifndef ZDA_H
#define ZDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZDA_OK = 0,
    ZDA_ERR_ARG = 1,          /* bad sizes, indices, NULL pointer, buffer too small */
    ZDA_ERR_CFL = 2,          /* Courant number at or above the stability bound */
    ZDA_ERR_UNSUPPORTED = 3,  /* r_in <= 0 (axis zone) or an unsupported preset */
    ZDA_ERR_OOM = 4,          /* device allocation failed */
    ZDA_ERR_STATE = 5,        /* call out of order (e.g. gradient without forward volume DFT) */
    ZDA_ERR_HIP = 6,          /* a HIP runtime call failed */
    ZDA_ERR_DIVERGED = 7      /* non-finite or exploding fields found by the watchdog */
} zda_status;

#define ZDA_MAX_FREQ 8        /* frequencies per run (K) */

/*
 * Zone description (a zone is radii, wedge angle 2 pi / n, height, grid steps
 * and an eps map: Fig. 2 caption and the section on the cylindrical solver).
 * pml_* widths are cells (0 = bare PEC wall on that face).  pml_sigma_max
 * <= 0 selects 0.8 (order + 1) / step; pml_alpha is the constant CFS shift.
 * The inner r-layer is the regularised one (radius stretched with |Sigma|).
 * k_mon: exit-plane monitor index in [1, nz).  Design layer k in
 * [design_k0, design_k1) over all i, j; eq. (6) maps rho to
 * eps = eps_bg + rho (eps_hi - eps_bg).
 */
typedef struct {
    double r_in;            /* inner radius (> 0), length units; dr / 2 for an axis zone */
    int nr, nphi, nz;       /* cells */
    int n_fold;             /* wedge angle tau = 2 pi / n_fold; 0 = continuous zone (nphi = 1) */
    int m;                  /* Bloch angular momentum of the forward run */
    double dr, dz;          /* grid steps */
    double courant;         /* dt = courant * min(dr, dz) */
    int pml_r_in, pml_r_out, pml_z_lo, pml_z_hi;
    double pml_order, pml_sigma_max_r, pml_sigma_max_z, pml_alpha;
    int k_mon;
    int design_k0, design_k1;
    double eps_bg, eps_hi;
    int single_buffer;      /* 1: one field set only (in-place split kernels; half the memory) */
    int axis;               /* 1: the zone contains the axis (r_in = dr / 2, no inner r-layer) */
} zda_zone_desc;

typedef struct zda_zone zda_zone;

/* Fill *d with defaults (PML 8 cells everywhere, order 3, alpha 0.05,
 * courant 0.5, eps_bg 1, eps_hi 6.25); sizes are left zero.  The zone's
 * parameters are those of the Fig. 2 caption (radii, wedge angle, height,
 * steps); the PML constants are this library's reading of the section on
 * the cylindrical solver, which says only that stretched-coordinate PMLs
 * surround the zone in r and z. */
void zda_zone_desc_default(zda_zone_desc *d);

/*
 * Device allocator for zone and batch memory, so that a host framework's
 * caching allocator can back it.  alloc_fn(bytes, device, ctx) returns a
 * device pointer on `device` (the zone's device, current when it is called)
 * or NULL (the call that needed it fails with ZDA_ERR_OOM); free_fn(ptr,
 * bytes, device, ctx) takes back what alloc_fn gave.  Both NULL restores
 * hipMalloc / hipFree; one NULL is ZDA_ERR_ARG.  Process-wide: zones and
 * batches created afterwards use it (each keeps the pair it was created
 * with and frees through it, in zda_zone_destroy or when a buffer grows; the
 * library first waits for the zone's stream, so nothing in flight reads the
 * memory it hands back).  Called on the thread that calls the library.
 * Pinned host staging buffers, streams and events do not go through it.
 */
typedef void *(*zda_alloc_fn)(size_t bytes, int device, void *ctx);
typedef void (*zda_free_fn)(void *ptr, size_t bytes, int device, void *ctx);
zda_status zda_set_allocator(zda_alloc_fn alloc_fn, zda_free_fn free_fn, void *ctx);

/*
 * Create a zone (section "Zoned discrete axisymmetry"; Fig. 2 caption).
 * Zones of the first radial band (the paper's zone 1 and its neighbours;
 * the section on the cylindrical solver closes the lens centre with loop
 * integrals and puts only an outer r-PML on the zone that holds r = 0):
 *  - axis = 1: the axis is the radial half-point r_{-1/2} = 0, so
 *    r_in = dr / 2 and nothing is stored on it.  The z components there are
 *    single-valued scalars, which the Bloch condition forces to zero unless
 *    exp(i m tau) = 1; the first row is then updated like any other (H_z on
 *    the axis = 0, the H_phi term at r_{-1/2} has weight 0) instead of being a
 *    PEC wall.  Runs whose seam phase is 1 (m = 0 mod n, or m = 0 in a
 *    continuous zone) are refused (ZDA_ERR_UNSUPPORTED).
 *  - n_fold = 0: continuous zone, the n -> infinity limit: nphi = 1, the
 *    fields carry exp(i m phi) exactly (seam factors 1 +- i m, dphi = 1, so
 *    the phi differences are exactly +-i m F / r), every component at phi = 0.
 * Create a zone on the current HIP device.  eps: nz*nr*nphi FP32 [k][i][j]
 * (may be NULL: eps = 1).  Errors: ZDA_ERR_ARG (sizes < 1, n_fold < 0,
 * n_fold = 0 with nphi != 1, PML wider than half the extent, k_mon or design
 * layer out of range, axis with r_in != dr/2 or an inner r-layer),
 * ZDA_ERR_CFL (courant * min(dr,dz) * sqrt(1/dr^2 + q^2 + 1/dz^2) >= 1 with
 * q = 1/(r_in dphi), or |m|/(2 r_in) in a continuous zone), ZDA_ERR_UNSUPPORTED
 * (r_in <= 0), ZDA_ERR_OOM.
 */
zda_status zda_zone_create(const zda_zone_desc *d, const float *eps, int eps_on_device,
                           zda_zone **out);

/* NULL-safe; waits for the device to finish the zone's work, then frees its
 * memory. */
void zda_zone_destroy(zda_zone *z);

/* Replace the permittivity map of the zone (Fig. 2 caption: a zone carries its
 * eps map; one eps per cell, applied to the cell's three E samples):
 * nz*nr*nphi FP32 [k][i][j] (NULL: eps = 1).  Ordered on the zone's stream;
 * host input is copied before the call returns (it waits for the stream). */
zda_status zda_zone_set_eps(zda_zone *z, const float *eps, int on_device);

/* eq. (6) inside the design layer: rho is (design_k1-design_k0)*nr*nphi FP32
 * in [0, 1] (values are not clamped), eps = eps_bg + rho (eps_hi - eps_bg).
 * Ordered on the zone's stream; host input is copied before the call
 * returns. */
zda_status zda_zone_set_design(zda_zone *z, const float *rho, int on_device);

/* Make `stream` the zone's stream (see the conventions above).  The next
 * call that takes a stream replaces it. */
zda_status zda_zone_set_stream(zda_zone *z, void *stream);

/*
 * Wait for the zone's stream.  Returns ZDA_ERR_DIVERGED if a divergence check
 * since the last run that reset the zone found a field sample that is not
 * finite or whose magnitude exceeds 1e18 (the regularised r-PML of the
 * section on the cylindrical solver exists because unregularised layers
 * diverge; the checks catch a run that does anyway).  Checks run inside the
 * time loop every ZDA_OPT_WATCHDOG steps (all six fields) and on every
 * monitor that zda_dft_fields reads; calls into host memory report the flag
 * themselves.
 */
zda_status zda_zone_sync(zda_zone *z);

/* Source presets (the normally incident plane wave decomposes into m = +-1,
 * section "Results and Discussion"). */
typedef enum {
    ZDA_SRC_PLANE_CIRC = 0,   /* J_r = -g e^{i m phi_j}/dz, J_phi = -i sgn(m) g e^{i m phi_{j+1/2}}/dz; |m| = 1 */
    ZDA_SRC_RADIAL = 1,       /* J_r = -g / dz; m = 0 */
    ZDA_SRC_CUSTOM = 2        /* n_profiles patterns, each [2][nr][nphi] complex (J_r, J_phi) */
} zda_src_kind;

/*
 * Soft current sheet on plane k_src (in [1, nz)):
 * J^{n+1/2}(x) = sum_p pattern_p(x) profile_p(n).  For presets the profile
 * is the pulse g(t) = sin(omega_c (t - t0)) exp(-(t - t0)^2 / (2 width^2)),
 * t = (n + 1/2) dt, t0 = (n0 + 1/2) dt, n0 < 0 selects round(6 width / dt),
 * g = 0 for n > 2 n0.  CUSTOM: patterns (device or host, per
 * patterns_on_device) and profiles (host, complex [n_profiles][nsteps],
 * interleaved doubles); at most ZDA_MAX_FREQ profiles.
 */
typedef struct {
    int kind;                 /* zda_src_kind */
    int k_src;
    double omega_c, width;
    int n0;
    int n_profiles;           /* CUSTOM only */
    const float *patterns;    /* CUSTOM only */
    int patterns_on_device;
    const double *profiles;   /* CUSTOM only, host */
} zda_source;

/* dft_flags */
#define ZDA_DFT_PLANE   1     /* exit plane k_mon: E_r, E_phi */
#define ZDA_DFT_VOLUME  2     /* design layer: E_r, E_phi, E_z (needed by zda_adjoint_grad) */
#define ZDA_RUN_CONTINUE 4    /* keep fields/aux/DFTs from the previous call (no reset) */
#define ZDA_RUN_TIMING   8    /* bracket every update kernel with HIP events (zda_zone_last_timing) */

/*
 * The time loop (section on the cylindrical solver: Yee leap-frog of eq. 3-5
 * on the staggered grid, PMLs in r and z; the DTFT monitors of its adjoint
 * paragraph, all frequencies extracted in one run).  Time-steps nsteps
 * leap-frog steps (H half-step, then E half-step with the soft source sheet)
 * and accumulates Ehat(w_k) = dt sum_{n=1..T} E^n e^{i w_k n dt} for
 * K <= ZDA_MAX_FREQ angular frequencies omega[] (host) on the monitors that
 * dft_flags selects.  Resets fields, auxiliaries, DFTs and the divergence
 * flag first unless ZDA_RUN_CONTINUE (then the monitors keep accumulating and
 * the pulse continues from the zone's step count).  Asynchronous on `stream`
 * (the zone's stream from then on); host arrays (omega, profiles, host
 * patterns) are copied before the call returns.  Errors: ZDA_ERR_ARG,
 * ZDA_ERR_STATE (ZDA_DFT_VOLUME without a design layer), ZDA_ERR_UNSUPPORTED
 * (preset and m disagree; axis zone with seam phase 1), ZDA_ERR_OOM,
 * ZDA_ERR_HIP.  Divergence is reported by zda_zone_sync.
 */
zda_status zda_fdtd_run(zda_zone *z, const zda_source *s, int nsteps, const double *omega, int K,
                        int dft_flags, void *stream);

/*
 * zda_fdtd_run for callers that cannot allocate (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same run with
 * the same kernels and results, whose per-run staging (source patterns,
 * pulse profiles, DFT twiddles, the two-step tile list) goes to a fixed
 * device scratch array of the library, ZDA_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the first call on that GPU until the process ends.  It calls no
 * hipMalloc / hipFree, no pinned-host allocation and no allocator registered
 * with zda_set_allocator; the zone (created beforehand) brings its own field
 * memory, and a ZDA_DFT_VOLUME run needs the design-layer buffer that a
 * first zda_fdtd_run with ZDA_DFT_VOLUME allocates (ZDA_ERR_STATE
 * otherwise).  Limits, each refused with ZDA_ERR_ARG before any work is
 * enqueued: source patterns * 2 * nr * nphi <= ZDA_NOALLOC_PATTERN complex
 * samples, nsteps * patterns <= ZDA_NOALLOC_STEPS and nsteps * K <=
 * ZDA_NOALLOC_STEPS, at most ZDA_NOALLOC_TILES two-step tiles; ZDA_RUN_TIMING
 * is refused.  The staging is written from the zone's pageable host vectors,
 * and the call waits for `stream` before it returns so that the next call
 * may rewrite them.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (on different streams or threads) race and must
 * not be made.  The concurrent layer-tile stream option is not used here.
 */
/*
 * The forward leap-frog of zda_fdtd_run (section on the cylindrical solver:
 * eq. 3-5 with the zone's PMLs, the soft source sheet, the exit-plane DTFT)
 * in FP64: fields, layer auxiliaries, coefficients, source and DFT all in
 * double precision, stepped by the in-place H and E kernel pair.  It exists
 * for finite-difference checks of the FP32 adjoint gradient (eq. 6 overlap):
 * the objective change from one design pixel lies below FP32 rounding, not
 * below FP64's.  eps: nz*nr*nphi FP64 permittivity [k][i][j] (host or device;
 * the zone's own FP32 map is not used, so a check can move a pixel by less
 * than an FP32 ulp); the zone supplies geometry, layers and k_mon.  Preset
 * sources only (ZDA_ERR_UNSUPPORTED otherwise); 1 <= K <= ZDA_MAX_FREQ.
 * plane_out: [K][2][nr][nphi] complex FP64 (2*K*2*nr*nphi doubles), host or
 * device.  The first call allocates the FP64 state (six complex FP64 fields,
 * dt/eps, auxiliaries: about 104 B per cell), kept until zda_zone_destroy;
 * the zone's FP32 state is untouched.  Waits for `stream` before it returns.
 */
zda_status zda_fdtd_run_fp64(zda_zone *z, const double *eps, int eps_on_device, const zda_source *s, int nsteps,
                             const double *omega, int K, double *plane_out, int out_on_device, void *stream);

#define ZDA_NOALLOC_PATTERN (1u << 20)   /* complex samples (8 MiB) */
#define ZDA_NOALLOC_STEPS (1u << 17)     /* complex samples each for profiles and twiddles (1 MiB each) */
#define ZDA_NOALLOC_TILES (1u << 16)     /* 16-byte two-step tile descriptors (1 MiB) */
#define ZDA_NOALLOC_SCRATCH_BYTES \
    (8u * (ZDA_NOALLOC_PATTERN + 2u * ZDA_NOALLOC_STEPS) + 16u * ZDA_NOALLOC_TILES)
zda_status zda_fdtd_run_noalloc(zda_zone *z, const zda_source *s, int nsteps, const double *omega, int K,
                                int dft_flags, void *stream);

/* monitor ids */
#define ZDA_MON_PLANE  0      /* layout [K][2][nr][nphi] complex (E_r, E_phi at k_mon) */
#define ZDA_MON_VOLUME 1      /* layout [K][3][design_k1-design_k0][nr][nphi] complex */
#define ZDA_MON_ADJOINT_VOLUME 2  /* same layout, the adjoint run's volume DFT */

/* component_mask bits of zda_dft_fields (0 selects every component) */
#define ZDA_COMP_R   1        /* E_r */
#define ZDA_COMP_PHI 2        /* E_phi */
#define ZDA_COMP_Z   4        /* E_z (design-layer monitors only) */

/*
 * Read a DFT monitor (the frequency-domain fields of the hybrid
 * time/frequency adjoint, section on the cylindrical solver) into out:
 * interleaved complex FP32 on the native staggered points, layout
 * [K][selected components, in the order r, phi, z][plane or layer volume],
 * out_floats floats available.  Ordered on the zone's stream; waits for it
 * only if out is host memory, and then returns ZDA_ERR_DIVERGED (the data
 * is still copied) if the divergence flag is set.  The monitor is scanned
 * for non-finite values on the way (raising the flag).  ZDA_ERR_ARG if out
 * is too small or the mask names a component the monitor lacks,
 * ZDA_ERR_STATE if the monitor was not accumulated by the last run.
 */
zda_status zda_dft_fields(zda_zone *z, int monitor, int component_mask, float *out, size_t out_floats,
                          int out_on_device);

/*
 * Adjoint gradient (hybrid time/frequency adjoint with broadband adjoint
 * sources, section on the cylindrical solver; eq. 6).  dF_dE: the
 * Wirtinger derivative dF/dEhat of a real objective with respect to the last
 * forward run's exit-plane DFT, [K][2][nr][nphi] complex.  Runs the adjoint
 * (Bloch order -m, same eps and PML, current W^{-1} dF/dEhat_k / (i wt_k) on
 * plane k_mon with time profiles mixing K pulses so that each frequency sees
 * exactly its own pattern), accumulates its design-volume DFT and writes
 * grad_rho[(design_k1-design_k0)*nr*nphi] = dF/drho =
 * (eps_hi - eps_bg) sum_k sum_alpha 2 Re[wt_k^2 W Xhat Ehat].  adj_width <= 0
 * reuses the forward pulse width (and n0).  Requires a forward run with
 * ZDA_DFT_VOLUME (ZDA_ERR_STATE otherwise).  Asynchronous on `stream` (the
 * zone's stream from then on); a host dF_dE is copied before the call
 * returns; a host grad_rho makes the call wait and report ZDA_ERR_DIVERGED
 * if the divergence flag is set.
 */
zda_status zda_adjoint_grad(zda_zone *z, const float *dF_dE, int dF_on_device, float *grad_rho,
                            int grad_on_device, double adj_width, void *stream);

/* Raw access to the Yee fields of eq. (3)-(5) (testing and checkpoints).
 * comp: 0..5 = E_r, E_phi, E_z, H_r, H_phi, H_z; buffer nz*nr*nphi complex.
 * Writing E_phi also seeds the r-layer's integrated-field auxiliary as the
 * first step expects.  Ordered on the zone's stream; waits for it when the
 * buffer is host memory. */
zda_status zda_zone_read_field(zda_zone *z, int comp, float *out, int out_on_device);
zda_status zda_zone_write_field(zda_zone *z, int comp, const float *in, int in_on_device);

/* Time-stepping memory of a zone held only while it steps, so that a lens
 * of more zones than HBM holds with both buffer sets can run its zones in
 * waves through the forward and the adjoint run of one design iteration
 * (the paper steps every zone as an independent simulation, section
 * "Zoned discrete axisymmetry").  zda_zone_release_fields waits for the
 * zone's stream and gives back both field sets, the PML auxiliaries and
 * the multi-step kernels' intermediate sets (or stops using the caller's
 * buffer they were carved from); the zone keeps its permittivity, design,
 * launch settings and monitors, including the last forward run's
 * design-volume DFT, so zda_adjoint_grad can follow the next acquire.
 * While released, runs (zone, batch, autotune, the entry point that
 * allocates nothing), the adjoint and field reads and writes return
 * ZDA_ERR_STATE.  zda_zone_acquire_fields takes that memory again with zero
 * fields and auxiliaries (fills enqueued on the zone's stream): base NULL
 * allocates it (ZDA_ERR_OOM, the zone staying released, if an allocation
 * fails); otherwise it is carved from [base, base + bytes), device memory
 * on the zone's device, 256-byte aligned, of at least the
 * zda_zone_fields_bytes the zone reports (ZDA_ERR_ARG otherwise), which the
 * caller owns and keeps valid and unused by anything else until the
 * zone's release returns (one buffer can then serve the zones of the next
 * wave without allocating).  Both calls are no-ops when the zone is
 * already in that state.  A zone stepping in a caller's buffer cannot
 * switch to the three-step kernel (ZDA_ERR_STATE from zda_zone_set_launch)
 * until it is released. */
zda_status zda_zone_release_fields(zda_zone *z);
zda_status zda_zone_acquire_fields(zda_zone *z, void *base, size_t bytes);
zda_status zda_zone_fields_bytes(zda_zone *z, size_t *bytes);

/* Sizes and stability margin of a zone (the Courant bound of the Yee scheme,
 * section on the cylindrical solver). */
typedef struct {
    size_t cells;             /* nr*nphi*nz */
    size_t device_bytes;      /* owned device memory */
    double dt;
    double cfl;               /* courant * min(dr,dz) * sqrt(...) (< 1 when stable) */
    int launch_chunks;        /* z chunks of the update kernels */
    int kchunk;               /* z-planes marched by one thread */
    int tile_rows;            /* radial rows per thread block */
} zda_zone_info;

/* Launch shape of the update kernels of the leap-frog (eq. 3-5; the paper's
 * own solver is a GPU FDTD, section on the cylindrical solver; shapes are
 * this library's): each thread marches kchunk z-planes of
 * one (r, phi) column.  tile_rows in {3, 7, 15} selects the fused one-launch
 * step (a block owns tile_rows radial rows x 56 phi cells; needs the second
 * buffer set), tile_rows in {5, 13} the two-step kernel (two time steps per
 * launch, a block owns tile_rows rows x 56 phi cells, 61 in the tiles that
 * hold layer cells; needs the second set and the intermediate auxiliaries),
 * tile_rows in {1, 2, 4, 8, 16} the in-place H and E kernels (a block covers
 * tile_rows rows x 64 phi cells), tile_rows = 32 the in-place kernels with a
 * flat mapping (a block covers 256 consecutive cells of the (r, phi) plane,
 * so narrow wedges keep every lane busy), tile_rows = 33 the fused step with
 * a flat mapping (a block holds 256 / nphi whole rows and owns all but one;
 * nphi <= 64), tile_rows = 34 the two-step kernel with a flat mapping (a
 * block holds 256 / nphi whole rows and owns all but three, the radial halo;
 * nphi <= 32; an odd last step of a run takes the flat fused step; needs what
 * the two-step kernel needs), tile_rows = 11 the three-step kernel (three
 * time steps per launch, a block owns 11 rows x 56 phi cells, r-layer band
 * tiles 7 rows x 59 cells, tiles with z-layer planes only 11 x 59; the last
 * nsteps mod 3 steps of a run take the fused step; its layer tiles pass the
 * auxiliaries of both intermediate time levels through device memory
 * whatever ZDA_OPT_LAYER_CARRY says; needs what the two-step kernel needs,
 * and allocates a second intermediate set of the layer auxiliaries when
 * first selected: ZDA_ERR_OOM if that fails).  Default: for zones of at most 16
 * phi cells (and the continuous zone) the flat in-place kernels; for zones
 * of 17 to 32 phi cells the flat two-step kernel in 4-plane chunks (where
 * the two-step kernel fits); otherwise the two-step kernel with 13 rows
 * and the chunk depth (3 to 72 planes) whose launch is predicted to finish
 * first when tiles run in rounds of one per CU; the fused step (3 rows,
 * 12-plane chunks, fewer for small zones) where the intermediate set does not
 * fit; the in-place kernels (4 rows) for single-buffer zones.
 * Results do not depend on the shape (beyond rounding).  ZDA_ERR_ARG for kchunk outside
 * [1, nz], any other tile_rows, or a flat fused (two-step) shape on a zone
 * wider than 64 (32) phi cells; ZDA_ERR_STATE for a fused shape on a zone
 * without the second buffer set. */
zda_status zda_zone_set_launch(zda_zone *z, int kchunk, int tile_rows);

/* Launch options of the fused step and the two-step kernel (results do not
 * depend on them): ZDA_OPT_XCD_REMAP (default 0) numbers the tiles so that
 * each of the eight XCDs works on one contiguous range of neighbouring
 * tiles; ZDA_OPT_NT_STORES (default 1) writes the next buffer set with
 * non-temporal stores; ZDA_OPT_LAYER_STREAM (default 0) runs the two-step
 * launch over the tiles with layer cells on a second stream of the zone
 * (default priority), concurrently with the launch over the interior tiles,
 * joined back into the run's stream before the next pair of steps.
 * ZDA_OPT_TILE_PATCH (default 0 = off; takes precedence over
 * ZDA_OPT_XCD_REMAP) orders the two-step tiles of each plane chunk in
 * patches of `value >> 8` row bands x at most `value & 0xff` phi columns,
 * patch q going to XCD q mod 8 (the XCDs take a launch's blocks
 * round-robin), so that the tiles one XCD holds at a time share halo lines
 * in its L2.  ZDA_ERR_ARG for an unknown option or a patch value with a
 * zero or > 255 field. */
#define ZDA_OPT_XCD_REMAP 1
#define ZDA_OPT_NT_STORES 2
#define ZDA_OPT_LAYER_STREAM 3
#define ZDA_OPT_TILE_PATCH 4
/* ZDA_OPT_LAYER_KCHUNK: planes per chunk of the two-step tiles of the r-layer
 * bands (outside the z-layers).  -1 (default): the zone's kchunk, at most 24
 * when the layer tiles carry their auxiliaries in registers (48 otherwise),
 * halved (down to 12) while the layer-tile launch would hold fewer than 512
 * tiles, so that its long r-band tiles do not leave most CUs idle; 0: the
 * zone's kchunk. */
#define ZDA_OPT_LAYER_KCHUNK 5
/* ZDA_OPT_WATCHDOG: steps between the in-loop divergence checks of all six
 * fields (default 1000; 0 = off; see zda_zone_sync). */
#define ZDA_OPT_WATCHDOG 6
/* ZDA_OPT_LAYER_CARRY: 1 (default) = the two-step kernel's tiles with layer
 * cells keep the level-(n+1) recursion auxiliaries of step one in registers
 * for step two (tiles with r-layer rows in blocks of 5 owned rows, or of 7
 * rows with the r-layer recursions only in the plane chunks without z-layer
 * planes of a band that 7-row tiles cover with fewer wavefront rows; z-layer-
 * only tiles in their own launch; the level-n auxiliaries loaded together at
 * the start of each plane); 0 = through the intermediate set in device
 * memory.  A batch follows its first zone's option.  Same results either
 * way. */
#define ZDA_OPT_LAYER_CARRY 7
zda_status zda_zone_set_option(zda_zone *z, int option, int value);

zda_status zda_zone_get_info(const zda_zone *z, zda_zone_info *info);

/* Per-kernel device time of the leap-frog's update kernels (eq. 3-5) in the
 * last zda_fdtd_run made with ZDA_RUN_TIMING
 * (HIP events on the run's stream around each launch).  Split kernels: h and
 * e per step; fused step: e per step; two-step kernel: e = the launch over
 * interior tiles (no layer cells), layer = the launch over the other tiles,
 * both per pair of steps (an odd last step runs the fused step, untimed).
 * Synchronises. */
typedef struct {
    int h_launches, e_launches;
    double h_ms, e_ms;        /* summed kernel durations */
    int steps_per_launch;     /* time steps one e launch advances: 1, or 2 (two-step) */
    int layer_launches;       /* two-step: launches over the tiles holding layer cells */
    double layer_ms;
    size_t e_cells;           /* cells one e launch owns (two-step: the interior tiles) */
    size_t e_mon_cells;       /* of them, cells in the exit-plane monitor */
    size_t e_src_cells;       /* of them, cells in the source sheet */
} zda_timing;

zda_status zda_zone_last_timing(zda_zone *z, zda_timing *t);

/* The two-step kernel's launch plan (two leap-frog steps of eq. 3-5 per
 * launch, temporal blocking of this library) for a zone described by d, computed on
 * the host (no device is touched; a zone created from d with the same
 * tile_rows, kchunk and tile order runs exactly these tiles).  tile_rows: 5,
 * 13 or 34 (flat mapping: tiles own 256 / nphi - 3 rows and every phi cell,
 * nphi <= 32), or 11 for the three-step kernel's plan (interior tiles own
 * 11 rows and 56 phi cells and compute rows i0-3 .. i0+rows+1 and planes
 * kb-3 .. ke+1; kind 2 for the tiles whose computed rows hold no r-layer
 * cell, kind 3 for the r-layer band tiles of at most 7 rows; layer tiles own
 * 59 phi cells); kchunk >= 1 planes per chunk; k_src: the source plane (only the
 * cell counts depend on it); order: 0 natural, 1 contiguous range per XCD
 * (ZDA_OPT_XCD_REMAP), else a patch code (ZDA_OPT_TILE_PATCH), with
 * ZDA_PLAN_CARRY or-ed in for the plan of ZDA_OPT_LAYER_CARRY.  out (may be
 * NULL to query the count): 4 uint32 per tile, {phi block, first owned row |
 * row count << 16, first plane | end plane << 16, kind}, kind 0 for the
 * interior tiles (their computed rows i0-2 .. i0+rows and planes kb-2 .. ke
 * hold no layer cell; they own 56 phi cells) and 3 for the layer tiles (61
 * phi cells; with tile_rows 34 or ZDA_PLAN_CARRY, 2 for the tiles whose
 * computed rows hold no r-layer cell; with ZDA_PLAN_CARRY, 1 for the others,
 * which own at most 5 rows, and 4 for the r-layer band tiles of at most 7
 * rows whose computed planes hold no z-layer plane, in the bands that 7-row
 * tiles cover with fewer wavefront rows), interior tiles first; cap: capacity of out in
 * tiles.
 * *ntiles and *n_interior receive the counts.  Errors: ZDA_ERR_ARG (sizes
 * < 1, nr or nz > 65535, a layer wider than half the extent, tile_rows not 5,
 * 13, 34 or 11, 34 with nphi > 32, kchunk < 1, a patch field of 0, out too
 * small). */
#define ZDA_PLAN_CARRY (1 << 16)
zda_status zda_plan_two_step_tiles(const zda_zone_desc *d, int tile_rows, int kchunk, int k_src, int order,
                                   uint32_t *out, size_t cap, size_t *ntiles, size_t *n_interior);

/*
 * Batches: many zones of uneven size (the lens-scale schedule in which n
 * grows with radius: section "Zoned discrete axisymmetry", and the zone
 * count of the section on the LWIR metalens) stepped together -- one launch per time step (fused
 * kernels, when every zone has its second buffer set) or two (split), whose
 * 1-D grid covers the tiles of every zone through a device zone table, with
 * the time loop captured once into a HIP graph and replayed.  A batch does
 * not own its zones; they must outlive it and live on one device.
 */
typedef struct zda_batch zda_batch;

zda_status zda_batch_create(zda_zone *const *zones, int nzones, zda_batch **out);
void zda_batch_destroy(zda_batch *b);

/* Forward run of every zone (the zones are independent simulations,
 * section "Zoned discrete axisymmetry"): sources[i] is zone i's source;
 * nsteps, omega[K] and dft_flags (no ZDA_RUN_TIMING) are shared.  Same
 * results as running the zones one by one with zda_fdtd_run.  Waits for
 * `stream` before it returns. */
zda_status zda_batch_run(zda_batch *b, const zda_source *sources, int nsteps, const double *omega, int K,
                         int dft_flags, void *stream);

/* Adjoint gradients of every zone in one batched adjoint run (one forward
 * and one adjoint simulation per iteration, section on the poly-achromatic
 * lenses); dF_dE[i] and grad_rho[i] are device pointers with the layouts of
 * zda_adjoint_grad.  Every zone needs a forward run with ZDA_DFT_VOLUME of
 * the same length.  Waits for `stream` before it returns. */
zda_status zda_batch_adjoint_grad(zda_batch *b, const float *const *dF_dE, float *const *grad_rho, void *stream);

/* Launch shape shared by the batched kernels of the leap-frog (eq. 3-5;
 * tile_rows as in zda_zone_set_launch, except 11: the three-step kernel
 * runs single zones only) and per-zone z-chunk depth kchunk[nzones] (NULL
 * keeps each zone's; the flat two-step kernel, 34, wants chunks of 12 to 64
 * planes, far deeper than the 2 that narrow zones keep for their default
 * in-place kernels).  Errors as for zda_zone_set_launch, for any zone;
 * ZDA_ERR_ARG for tile_rows 11. */
zda_status zda_batch_set_launch(zda_batch *b, int tile_rows, const int *kchunk);

/* Autotuner of the batched leap-frog (eq. 3-5): times short probe runs
 * (probe_steps >= 2; the zones' state is reset) of every kernel family and
 * tile shape, then of z-chunk depths per size class of zones, keeps the
 * fastest and reports it. */
typedef struct {
    int tile_rows;
    double ms_per_step;
    int probes;
} zda_tune_result;

zda_status zda_batch_autotune(zda_batch *b, const zda_source *sources, int probe_steps, const double *omega, int K,
                              void *stream, zda_tune_result *res);

/* Text of a status code, and the message of the last failure on the calling
 * thread (thread-local; valid until the next failing call on the thread). */
const char *zda_status_str(int status);
const char *zda_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZDA_H */

/*
 * pic.h -- C ABI of the MI355X particle-in-cell step library (libpic.so).
 *
 * The library advances a fully relativistic, electromagnetic particle-in-cell
 * (PIC) plasma on one GPU.  One step is the loop of R. G. Hemker, "Particle-
 * In-Cell Modeling of Plasma-Based Accelerators in Two and Three Dimensions"
 * (2000), Ch. 3, Sec. 3.1: interpolate the Yee-staggered E and B to every
 * particle, advance momentum (relativistic Boris push, Sec. 3.2 Eq.
 * momentum-update) and position (Eq. 2d-position-update), deposit a
 * charge-conserving current (the ISIS ordering average, Sec. 3.2, Eq.
 * continuity), and advance the fields by the Yee scheme (Sec. 3.2 Eqs.
 * 2d-field-solve-b-part1, -e, -b-part2; Sec. 3.3 for 3D).
 *
 * Units are the normalised units of App. A: time 1/omega_n, length
 * c/omega_n, momentum u = p/(m c) = gamma*beta, fields m c omega_n / e,
 * density n_n.  The Gaussian 4*pi is absorbed: dE/dt = curl B - J,
 * div E = rho.
 *
 * Conventions shared by every call:
 *  - Every function returns a pic_status; PIC_OK (0) on success, a negative
 *    code otherwise.  The message of the last failure on a context is
 *    available from pic_last_error().  No C++ exception crosses the ABI.
 *  - FP64 at the ABI, FP32 inside (particles, fields, current); the
 *    diagnostics reduce in FP64 with compensated sums.
 *  - Buffers passed in are copied; the caller keeps ownership.  Outputs go
 *    into caller buffers whose size in bytes is checked: when out_bytes is
 *    too small the call fails with PIC_E_RANGE and *written holds the size
 *    required.
 *  - Grid arrays are [component][cell], cell = i0 + nx0*(i1 + nx1*i2), with
 *    the staggering E1 (1/2,0,0), E2 (0,1/2,0), E3 (0,0,1/2),
 *    B1 (0,1/2,1/2), B2 (1/2,0,1/2), B3 (1/2,1/2,0), J_d at E_d and rho at
 *    the node (offsets in cells from node i; 2D drops the third offset).
 *    This is the only layout consistent with the difference stencils of
 *    Sec. 3.2 (the grid figure itself is not reproduced in the text).
 *  - A context owns all device memory it allocates and works on one HIP
 *    stream (the one given at creation, or the null stream).  Calls are
 *    asynchronous with respect to the host unless stated; a context is not
 *    safe for concurrent calls from several threads.
 *  - All boundaries are periodic; on one device a periodic boundary is the
 *    exchange of a domain with its own opposite face (App. A, node
 *    configuration).
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;     /* opaque: one simulation instance */
typedef struct pic_batch pic_batch; /* opaque: many independent instances */

typedef enum {
  PIC_OK = 0,
  PIC_E_INVALID = -1,     /* bad argument or configuration */
  PIC_E_NOMEM = -2,       /* device or host allocation failed, or capacity exceeded */
  PIC_E_HIP = -3,         /* a HIP runtime call failed */
  PIC_E_STATE = -4,       /* call not valid in the current state */
  PIC_E_RANGE = -5,       /* non-finite input, or output buffer too small */
  PIC_E_UNSUPPORTED = -6  /* valid request the library does not implement */
} pic_status;

/* Accumulation of the current.  Every particle's FP32 contribution is
 * rounded to an integer multiple of a power-of-two unit and the
 * contributions of a tile are summed exactly in integers in LDS.  The unit
 * follows a bound on a single contribution |w| |v|: the work item's largest
 * in the two-phase kernels (periodic 3D; periodic 2D with items of at most
 * 1024 particles), whose 32-bit tile sums hold n such contributions
 * (unit about n 2^-31 of the bound for an item of n particles); a per-step
 * bound of the species in the other kernels, whose tile sums are int64
 * (unit 2^-31 of the bound); the instance's 2^-31 max|w| with
 * PIC_ACC_FIXED64. */
enum {
  PIC_ACC_FP32 = 0,        /* exact tile sums, folded into the FP32 current
                              with FP32 global atomic adds */
  PIC_ACC_COMPENSATED = 1, /* same as PIC_ACC_FP32: the exact integer tile
                              sum is the compensated accumulation */
  PIC_ACC_FIXED64 = 2      /* tiles folded in int64 too: the current is
                              independent of the order of the adds (bitwise
                              reproducible), converted to FP32 once per step */
};

/* Simulation configuration (the deck's grid, space, time and EM-field
 * sections of App. A, restricted to periodic boxes). */
typedef struct {
  int32_t ndim;          /* 2 (2D3V) or 3 (3D3V) */
  int32_t nx[3];         /* cells per axis; nx[2] ignored in 2D */
  double dx[3];          /* cell size per axis */
  double xmin[3];        /* lower corner of the box */
  double dt;             /* time step; needs dt * sqrt(sum_d dx_d^-2) < 1
                            (Courant condition, Sec. 4.5, generalised to
                            several dimensions) */
  int32_t shape_order;   /* particle shape: 1 linear (CIC), 2 quadratic, 3 cubic */
  double e0[3];          /* uniform external E felt by the particles */
  double b0[3];          /* uniform external B felt by the particles */
  double ion_density;    /* immobile neutralising background charge density,
                            used only by the rho and Gauss diagnostics */
  int64_t capacity;      /* maximum particles per species (num_par_max) */
  int32_t tile[3];       /* tile extent in cells; 0 = a default from the grid
                            (pic_autotune searches it by measurement) */
  int32_t sort_interval; /* steps between rebin checks; 0 = a default from the
                            Courant number (searched by pic_autotune) */
  int32_t chunk;         /* maximum particles one workgroup takes from a tile;
                            0 = 2048 (searched by pic_autotune); capped at
                            768 in periodic 3D boxes, and at 1024 in periodic
                            2D ones with FP32 accumulation unless it is asked
                            above 1024 (then the one-phase kernel runs) */
  int32_t accumulator;   /* PIC_ACC_* */
  int32_t deposit;       /* PIC_DEPOSIT_*: which charge-conserving current */
  /* Smoothing of the current before the field solve (App. A, current
   * smoothing section): along each axis separately, smooth_level[axis]
   * passes (0 = off, at most PIC_MAX_SMOOTH), pass p mapping every component
   * to (a J[i-1] + b J[i] + c J[i+1]) / (a + b + c) with
   * (a, b, c) = smooth_weights[axis][p], periodic; axes in order 1, 2, 3.
   * The exported current is the smoothed one.  With smoothing on, the
   * current no longer satisfies the continuity equation with the
   * unsmoothed charge density (the charge residual is then not zero). */
  int32_t smooth_level[3];
  double smooth_weights[3][8][3];
  /* Moving window (Sec. 4.5, dynamic simulation spaces): with move_window = 1
   * the window moves along +x1 at the speed of light.  x1 is then open: grid
   * values beyond the first and last x1 cell are zero, currents deposited
   * there are dropped and particles that leave through an x1 face are
   * removed.  After every step that brings c t past the next whole cell
   * (floor(n dt / dx1) shifts after n steps) the window moves by one cell:
   * the back cell column is discarded with its particles, and the new front
   * column starts with E = B = 0 and a plasma of species 0:
   * inject_ppc[d] particles per cell per axis on a regular sub-lattice
   * ((k + 1/2) / inject_ppc[d] of the cell), weight inject_w, at rest or, with
   * inject_uth > 0, thermal (see inject_uth below).  The
   * sort interval is 1.  Positions exported and loaded are lab positions
   * (xmin1 + shifts dx1 + window position); grid arrays exported and loaded
   * are in window order (index 0 at the back).  Species 0 must be loaded
   * before the first step.  Not available with pic_autotune. */
  int32_t move_window;
  int32_t inject_ppc[3];
  double inject_w;
  /* Geometry (PIC_GEOM_*).  PIC_GEOM_RZ (Sec. 3.3, 2D cylindrically
   * symmetric): ndim = 2, x1 = z (periodic), x2 = r; E1 E2 E3 = E_z E_r
   * E_theta (B, J likewise); u = (u_z, u_r, u_theta) in the particle's local
   * frame.  The axis runs through the middle of the first cell: rows of
   * E_z, E_theta, B_r, J_z, J_theta sit at r = (j - 1/2) dr, rows of E_r,
   * B_z, B_theta, J_r at r = j dr; row 0 of the former is the mirror image
   * of row 1 (z components keep their sign, r and theta components change
   * it) and E_r, B_theta, J_r vanish on the axis.  B_z on the axis follows
   * Faraday's law over the disc of radius dr/2 (Eq. 2d-field-solve-cyl-b1-axis),
   * B_z and E_z elsewhere the r-weighted curl (Eq. 2d-field-solve-cyl).
   * r = (nx[1] - 1/2) dr is a conducting wall: a particle that reaches it is
   * removed after depositing its current.  A particle is a ring: its weight
   * w is its charge over 2 pi dr^2 dz (so a density n loaded with ppc
   * particles per cell takes w = n (r/dr) / ppc), and the current density
   * of a row is the deposited ring current over the ring volume.  The push
   * moves the particle on the straight 3D line and rotates position and
   * momentum back into the r-z plane (Eqs. 2d-cyl-position-update-1..3).
   * Positions loaded and exported are (z, r) with xmin[1] = 0; particles
   * are exported in load order without the removed ones.  The sort
   * interval is 1.  The diagnostics use the ring volumes: RHO is
   * ion_density + (charge below the axis folded to its mirror row) / (r/dr),
   * the residuals use the cylindrical divergence, ENERGY weighs each value
   * by the volume 2 pi r dr dz of its ring (pi dr^2 dz / 4 for the axis
   * disc), and MOMENTUM is (P_z, sum of the radial momenta, angular momentum
   * about the axis sum Q r u_theta m/q), with Q = w 2 pi dr^2 dz.  With a
   * moving window (along z) the injected lattice leaves out its points
   * below the axis (cell coordinate under 1/2) and an injected ring at
   * radius r takes weight inject_w r / dr (a uniform density).  Current
   * smoothing filters the current density (after the division by the ring
   * volumes); along r the neighbours below the axis are the mirror images
   * and those at and beyond the wall zero, J_r stays zero on the axis.  Not
   * available with pic_autotune. */
  int32_t geometry;
  /* Thermal injection at the moving window's front (Sec. 4.5: the new
   * region is initialised thermal): each component of an injected
   * particle's momentum is inject_uth times a standard normal deviate drawn
   * from its id, u_c = inject_uth sqrt(-2 ln U1) cos(2 pi U2) (Box-Muller)
   * with U1 = (floor(o(8 id + 2c + 1) / 2^11) + 1) 2^-53 and
   * U2 = floor(o(8 id + 2c + 2) / 2^11) 2^-53, where o(n) is the n-th output
   * of the SplitMix64 generator (Steele, Lea and Flood 2014) seeded with
   * inject_seed, computed in FP64.  Injected ids
   * continue after the loaded ones, one per lattice point of each new
   * column (points below the r-z axis included).  0: a cold plasma. */
  double inject_uth;
  uint64_t inject_seed;
} pic_config;

#define PIC_MAX_SMOOTH 8

/* Current deposit (Sec. 3.2).  Both satisfy the continuity equation; they
 * differ in the curl of the current when a particle crosses a cell face. */
enum {
  PIC_DEPOSIT_ISIS = 0,   /* average over the orderings of the orthogonal
                             moves of the whole straight path; every shape order */
  PIC_DEPOSIT_TRISTAN = 1 /* Villasenor-Buneman: the straight path cut at the
                             cell faces it crosses, each piece depositing its
                             in-cell current; linear shape (shape_order 1) only */
};

/* Geometry of the box (pic_config.geometry). */
enum {
  PIC_GEOM_CARTESIAN = 0, /* 2D or 3D Cartesian, periodic */
  PIC_GEOM_RZ = 1         /* 2D cylindrically symmetric r-z (Sec. 3.3) */
};

/* Flags for the load calls. */
#define PIC_DEVICE_PTRS 1u /* input pointers are device memory */

/* Create a context.  cfg is copied.  hip_stream may be NULL (null stream).
 * Fails with PIC_E_INVALID on a bad configuration, PIC_E_NOMEM when the
 * device memory for the fields cannot be allocated.  *out is NULL on failure. */
pic_status pic_create(const pic_config* cfg, void* hip_stream, pic_ctx** out);

/* Release every resource of a context; NULL is accepted and ignored. */
pic_status pic_destroy(pic_ctx* ctx);

/* Append n particles to a species (0 <= species < 8).
 * x: n*ndim absolute positions (FP64, row-major per particle), wrapped into
 *    the periodic box;
 * u: n*3 momenta u = p/(m c) at time n-1/2;
 * w: n signed charge weights (charge density each macro-particle carries,
 *    q * n / (n_n * particles per cell); electrons negative);
 * rqm: mass-to-charge ratio of the species (App. A species section,
 *    electrons -1); fixed by the first load of a species.
 * The species' particles are re-binned by tile after the append.  Fails with
 * PIC_E_RANGE on a non-finite value, PIC_E_NOMEM beyond the capacity. */
pic_status pic_load_particles(pic_ctx* ctx, int32_t species, double rqm, int64_t n,
                              const double* x, const double* u, const double* w,
                              uint32_t flags);

/* Overwrite E and B (each 3*ncell FP64 in the grid layout above) at the
 * current time level n. */
pic_status pic_load_fields(pic_ctx* ctx, const double* e, const double* b, uint32_t flags);

/* Advance nsteps steps (asynchronous on the context's stream).  Fails with
 * PIC_E_STATE when an earlier step found a particle outside the region
 * staged for its tile (an internal invariant), PIC_E_INVALID for nsteps < 0. */
pic_status pic_step(pic_ctx* ctx, int64_t nsteps);

/* Block until all work queued on the context's stream has finished. */
pic_status pic_sync(pic_ctx* ctx);

typedef enum {
  PIC_DIAG_ENERGY = 0,          /* double[4]: field E energy, field B energy,
                                   kinetic energy (at u^{n-1/2}), their sum;
                                   (V/2) sum |E|^2, (V/2) sum |B|^2,
                                   V sum_p w rqm (gamma-1) */
  PIC_DIAG_MOMENTUM = 1,        /* double[3]: V sum_p w rqm u */
  PIC_DIAG_RHO = 2,             /* double[ncell]: rho at the nodes from the stored
                                   positions, plus ion_density */
  PIC_DIAG_GAUSS_RESIDUAL = 3,  /* double[ncell]: div E - rho (Sec. 3.1, Gauss law) */
  PIC_DIAG_GAUSS_NORM = 4,      /* double[2]: max |div E - rho|, rms */
  PIC_DIAG_RHO_SNAPSHOT = 5,    /* no output: keep rho for CHARGE_RESIDUAL */
  PIC_DIAG_CHARGE_RESIDUAL = 6, /* double[ncell]: (rho_now - rho_snapshot)/dt + div J
                                   with J of the last step (Eq. continuity); meaningful
                                   when exactly one step ran since the snapshot */
  PIC_DIAG_EXPORT_STATE = 7,    /* double[n*(ndim+4)]: per particle x[ndim], u[3], w,
                                   species by species, each in load order (moving
                                   window: surviving loaded particles in load order,
                                   then the injected ones in injection order; n is
                                   the count after the last pic_sync) */
  PIC_DIAG_EXPORT_FIELDS = 8,   /* double[6*ncell]: E1 E2 E3 B1 B2 B3 at time n */
  PIC_DIAG_EXPORT_CURRENT = 9,  /* double[3*ncell]: J^{n+1/2} of the last step */
  PIC_DIAG_COUNTS = 10,         /* double[4]: steps done, particles, rebins done,
                                   rebin checks done */
  PIC_DIAG_KERNEL_TIMES = 11    /* double[6]: milliseconds and launches of the fused
                                   particle kernel, of the field kernels (current reset
                                   and Yee), and of the rebin checks, summed over the
                                   steps run while profiling was on (HIP events on the
                                   context's stream) */
} pic_diag_kind;

/* Compute or export a diagnostic into a host buffer (synchronous). */
pic_status pic_diag(pic_ctx* ctx, pic_diag_kind kind, void* out, size_t out_bytes,
                    size_t* written);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics PIC_DIAG_RHO, PIC_DIAG_GAUSS_RESIDUAL and
 * PIC_DIAG_CHARGE_RESIDUAL, as pic_diag computes them, written to a DEVICE
 * buffer of the context's device (out: ncell doubles, caller-owned; the call
 * is synchronous).  The call allocates nothing: the node charge behind the
 * residuals lives in a file-scope device array of the library (32 MiB per
 * device, held until the process ends), so the residuals need ncell <=
 * 4,194,304 (PIC_E_RANGE otherwise).  Every call on one device shares that
 * array: calls that overlap on one device (several threads, several
 * contexts) race.  Fails with PIC_E_UNSUPPORTED for other kinds and for a
 * moving window (whose grid is kept in ring order), PIC_E_INVALID when out
 * is not device memory of the context's device, PIC_E_STATE when another
 * device is current, when particles were loaded since the last pic_step or
 * pic_diag, or (CHARGE_RESIDUAL) without an earlier PIC_DIAG_RHO_SNAPSHOT
 * taken with pic_diag. */
pic_status pic_diag_noalloc(pic_ctx* ctx, pic_diag_kind kind, void* out, size_t out_bytes,
                            size_t* written);

/* Profiling: while enabled, pic_step launches every kernel individually
 * (no graph replay) and brackets each kernel family with HIP events on the
 * context's stream; PIC_DIAG_KERNEL_TIMES reads the sums.  enable = 0 turns it
 * off, 1 turns it on, 2 turns it on and clears the sums. */
pic_status pic_profile(pic_ctx* ctx, int32_t enable);

/* Tuning and layout the context settled on. */
typedef struct {
  int32_t tile[3];
  int32_t sort_interval;
  int32_t chunk;
  int32_t slack;       /* cells a particle may stray outside its tile between rebins */
  int32_t accumulator;
  int32_t nspecies;
  int64_t nparticles[8];
  double rqm[8];
  int64_t lds_bytes;   /* LDS per workgroup of the fused particle kernel */
} pic_info;

pic_status pic_get_info(const pic_ctx* ctx, pic_info* out);

/* Autotuner: a measured search of the launch layout on the loaded state.
 * Three parameters are searched one after the other, each time keeping the
 * best so far:
 *   particles per tile -- every instance's tile shape is re-derived from a
 *                         target number of particles per tile (its mean
 *                         particles per cell) and a preferred x:y aspect
 *                         (1, 2, 4, 8), among the tile extents valid for its
 *                         grid and sort interval and whose fused kernel fits
 *                         the LDS;
 *   sort_interval      -- steps between rebin checks (a longer interval
 *                         widens the slack each tile stages);
 *   chunk              -- maximum particles one workgroup takes from a tile
 *                         (512, 1024 or 2048: larger chunks leave a tile
 *                         whose density later grows several-fold as one
 *                         long work item).
 * Each candidate re-bins the particles, runs two warm-up rebin cycles and
 * times trial_steps steps (rounded up to whole cycles) with HIP events on
 * the context's stream.  Trials rebin at the rate this context's checks
 * have rebinned since the particles were loaded or the layout last
 * changed (a previous pic_autotune): every
 * round(checks / rebins)-th check is forced to rebin (besides the checks
 * that find strayed particles), none if no check has rebinned, and every
 * check when no step has run yet (the loaded state may be quieter than the
 * plasma it becomes).  The state is restored before every candidate and
 * after the search: particles (in load order), fields, the last current and
 * the step count are exactly those before the call; only the layout (tile,
 * sort interval, chunk, order of particles inside a tile) changes, and the
 * rebin counters of PIC_DIAG_COUNTS restart.  Synchronous.  Fails with
 * PIC_E_STATE when no particles are loaded, PIC_E_INVALID on bad arguments. */
typedef struct {
  int32_t trial_steps;        /* in: steps timed per candidate, >= 1 */
  int32_t what;               /* in: PIC_TUNE_* bits, 0 = all three */
  int32_t candidates;         /* out: layouts timed, the starting one included */
  int32_t particles_per_tile; /* out: target chosen (0: the starting tiles kept) */
  int32_t sort_interval;      /* out */
  int32_t chunk;              /* out */
  double ms_before;           /* out: ms per step of the starting layout */
  double ms_after;            /* out: ms per step of the chosen layout */
} pic_tune;

#define PIC_TUNE_TILE 1
#define PIC_TUNE_SORT 2
#define PIC_TUNE_CHUNK 4

pic_status pic_autotune(pic_ctx* ctx, pic_tune* io);

/* Message of the last failure on ctx (never NULL; "" when none). */
const char* pic_last_error(const pic_ctx* ctx);

/* ---------------------------------------------------------------------
 * Batched instances: n independent periodic boxes (parameter scans) with
 * their own grids, shapes and particles, advanced together.  Each step of
 * every instance runs in the same kernel launches (one per phase and shape
 * order), and pic_batch_step replays them as one captured HIP graph.
 * Per-instance results equal those of the same instance run alone.
 * ------------------------------------------------------------------- */
pic_status pic_batch_create(const pic_config* cfgs, int32_t n, void* hip_stream,
                            pic_batch** out);
pic_status pic_batch_destroy(pic_batch* b);
pic_status pic_batch_load_particles(pic_batch* b, int32_t inst, int32_t species, double rqm,
                                    int64_t n, const double* x, const double* u,
                                    const double* w, uint32_t flags);
pic_status pic_batch_load_fields(pic_batch* b, int32_t inst, const double* e, const double* bf,
                                 uint32_t flags);
pic_status pic_batch_step(pic_batch* b, int64_t nsteps);
pic_status pic_batch_diag(pic_batch* b, int32_t inst, pic_diag_kind kind, void* out,
                          size_t out_bytes, size_t* written);
pic_status pic_batch_sync(pic_batch* b);
pic_status pic_batch_profile(pic_batch* b, int32_t enable);
pic_status pic_batch_get_info(const pic_batch* b, int32_t inst, pic_info* out);
/* The autotuner over all instances of a batch at once: one particles-per-
 * tile target (each instance derives its own tile shape from it), one sort
 * interval and one chunk for the whole batch, timed on the batched step. */
pic_status pic_batch_autotune(pic_batch* b, pic_tune* io);
const char* pic_batch_last_error(const pic_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */

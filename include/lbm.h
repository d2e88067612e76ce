/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q27 central-Hermite-moment MRT
 * lattice Boltzmann library.
 *
 * The library advances the scheme of Huang, Noel, Berg and Hosseini,
 * "Simulation of the FDA Nozzle Benchmark: A Lattice Boltzmann Study":
 * the update of Sec. 2.1, Eq. (6), with the central Hermite moments of
 * Eqs. (7)-(8), the full (sixth-order) Hermite equilibrium of Eq. (4) and
 * App. A, Eqs. (A.4)-(A.6), relaxation rates as stated after Eq. (8) and in
 * App. A, on the D3Q27 stencil of App. A, Eqs. (A.1)-(A.2); bounce-back
 * walls (halfway, or interpolated for curved walls), a moving-wall velocity
 * inlet (profile of Sec. 2.2, Eq. (12)) and a zero-gradient or
 * constant-pressure (non-equilibrium extrapolation, Sec. 2.2) outlet.  Each step gives exactly the pull
 * update (every cell gathers f_i from x - c_i, then collides); the library
 * runs it in place on a single population array, alternating a streaming
 * step and a local step so that every step reads and writes the same slots.
 * Every step of the update runs in the library's own HIP kernels.
 *
 * Conventions
 *   - Every function returns an int status: LBM_OK (0) or a negative
 *     lbm_status code; none aborts or exits.  lbm_last_error() returns a
 *     thread-local message for the last failing call on that thread.
 *   - A NULL domain or batch handle returns LBM_ERR_ARG.
 *   - Host arrays passed in are owned by the caller and are only read or
 *     written during the call.  Device memory the library allocates is
 *     owned by the library and freed by lbm_destroy / lbm_batch_destroy.
 *   - Grid layout: cell = (z*ny + y)*nx + x, x fastest and contiguous.  x is
 *     the axial (inlet-to-outlet) direction.
 *   - Population order: i = (cx+1) + 3(cy+1) + 9(cz+1) for the velocity
 *     c_i = (cx, cy, cz) in {-1,0,1}^3; the opposite of i is 26 - i.
 *   - Populations are stored tile-major in one array per domain: cells are
 *     grouped into 64-cell tiles of the linear index, and the 27 slots of a
 *     tile form one block (slot k of the tile's cell l at element 64*k + l
 *     of the block), followed by 2*9*ny*nz outlet side elements
 *     (lbm_array_bytes).  Between calls the array holds f*_i(x) in slot
 *     26 - i, or the streamed form after an odd step count; the library
 *     converts as needed.  lbm_get_populations and lbm_set_populations use a
 *     plain [i][cell] layout.
 *   - The state is the post-collision population f* of the last step.
 *   - Calls on one domain are not thread-safe; different domains may be
 *     used from different threads.  All work is issued on the domain's
 *     stream; the calls below return only after that work completed.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_Q 27

/* Voxel flags (one uint8 per cell). */
enum lbm_flag {
    LBM_FLUID = 0,  /* updated every step */
    LBM_SOLID = 1,  /* wall: links into it are halfway bounce-back */
    LBM_INLET = 2,  /* moving wall carrying the inlet velocity; never updated */
    LBM_OUTLET = 3  /* fluid cell on the last x plane with an outlet (zero
                       gradient unless lbm_set_outlet selects constant
                       pressure): sources beyond x = nx-1 are taken from
                       x = nx-1 (same y, z shift); updated every step */
};

/* Population storage. */
enum lbm_storage {
    LBM_FP32 = 0,  /* f_i as FP32 */
    LBM_FP16S = 1, /* 2^14 * (f_i - w_i) as IEEE FP16, rounded to nearest even */
    LBM_BF16S = 2  /* (f_i - w_i) as bfloat16, rounded to nearest even */
};

enum lbm_status {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,      /* invalid argument; nothing changed */
    LBM_ERR_OOM = -2,      /* device allocation failed, or a batch budget is exceeded */
    LBM_ERR_DEVICE = -3,   /* a HIP runtime call failed */
    LBM_ERR_UNSTABLE = -4, /* a step produced rho <= 0 or a non-finite value */
    LBM_ERR_STATE = -5     /* call not valid in the current state */
};

/* Outlet conditions (lbm_set_outlet). */
enum lbm_outlet {
    LBM_OUTLET_ZERO_GRADIENT = 0, /* sources beyond the last plane copy it (default) */
    LBM_OUTLET_PRESSURE = 1       /* constant pressure rho_out/3, non-equilibrium extrapolation */
};

/* Periodicity bits. */
#define LBM_PERIODIC_X 1u
#define LBM_PERIODIC_Y 2u
#define LBM_PERIODIC_Z 4u

typedef struct lbm_domain lbm_domain;
typedef struct lbm_batch lbm_batch;

typedef struct lbm_domain_info {
    int nx, ny, nz;
    int storage;
    unsigned periodic;
    uint64_t ncells;        /* nx*ny*nz */
    uint64_t plane_stride;  /* P */
    uint64_t n_updated;     /* fluid + outlet cells: the cells one step updates */
    uint64_t n_tiles;       /* 64-cell tiles holding at least one updated cell */
    uint64_t n_wall_tiles;  /* of those, tiles with a non-plain link or a non-updated cell */
    uint64_t n_inlet;       /* inlet cells */
    uint64_t device_bytes;  /* device memory held by the domain */
    uint64_t bytes_per_cell_update; /* algorithmic HBM bytes per updated cell: 2*27*sizeof(storage) */
} lbm_domain_info;

/*
 * Create a domain from a voxel flag field (the geometry input of Sec. 2.2).
 *   flags        host, nx*ny*nz uint8 (enum lbm_flag), read during the call.
 *                LBM_OUTLET is only valid on the plane x = nx-1 with x not
 *                periodic.  Non-periodic box faces act as walls.
 *   periodic     LBM_PERIODIC_* bits.
 *   storage      enum lbm_storage.
 *   hip_stream   hipStream_t to issue work on, or NULL for a stream the
 *                library creates.  The stream must outlive the domain.
 * Allocates the population array and initialises f = f^eq(1, 0).
 * A domain has at most 2^32 - 64 cells (cell indices are 32-bit).  Arrays
 * of up to 4 GiB - 64 KiB (lbm_array_bytes) are stepped by kernels that
 * address them with buffer instructions and 32-bit byte offsets; larger
 * ones by kernels with 64-bit global addresses (lbm_is_wide).  The device
 * memory is the other bound: 288 GB hold about 2.6e9 FP32 cells'
 * populations (in FP16 the cell limit binds first).
 * Errors: LBM_ERR_ARG (bad sizes, flags or storage), LBM_ERR_OOM,
 * LBM_ERR_DEVICE.
 */
int lbm_create_domain(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, int storage,
                      void *hip_stream, lbm_domain **out);

/* Bytes of the population array of a domain of nx*ny*nz cells in the
 * given storage: 27 slots per cell for ncells rounded up to a multiple of
 * 64, plus 2*9*ny*nz side elements, rounded up to 256 bytes.  0 for
 * invalid arguments. */
uint64_t lbm_array_bytes(int nx, int ny, int nz, int storage);

/*
 * As lbm_create_domain, but adopts a caller-allocated device array of
 * lbm_array_bytes(nx, ny, nz, storage) bytes, 256-byte aligned (e.g. from
 * torch).  The caller keeps ownership; the array must outlive the domain.
 */
int lbm_create_domain_ext(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, int storage,
                          void *hip_stream, void *f, lbm_domain **out);

/*
 * Relaxation parameters (Sec. 2.1, Eq. (5) and the text after Eq. (8);
 * App. A after Eq. (A.6)).
 *   tau         lattice relaxation time, > 0.5; the shear rate is 1/tau and
 *               relaxes the deviatoric and off-diagonal second-order
 *               central moments (nu = (tau - 1/2)/3).
 *   omega_bulk  rate of the trace of the second-order central moments, in
 *               (0, 2); the paper's choice is 1/tau.
 *   omega_high  rate of every central moment of order >= 3, in (0, 2]; the
 *               paper's choice is 1.
 * Errors: LBM_ERR_ARG when out of range.
 */
int lbm_set_params(lbm_domain *d, double tau, double omega_bulk, double omega_high);

/* As lbm_set_params with the shear rate given directly; every rate may be
 * anywhere in [0, 2] (0 leaves that group of moments unrelaxed; all zero
 * is pure streaming).  For tests and stability studies. */
int lbm_set_rates(lbm_domain *d, double omega, double omega_bulk, double omega_high);

/*
 * One relaxation rate per order of the higher central moments (the paper
 * sets them all to one, Sec. 2.1 after Eq. (8); App. A after Eq. (A.6)).
 * The central moment H_{x^a y^b z^c}, a, b, c <= 2, has order a + b + c;
 * omega3..omega6 relax the orders 3..6, each in [0, 2].  lbm_set_params and
 * lbm_set_rates set all four to omega_high.  Errors: LBM_ERR_ARG when out
 * of range, LBM_ERR_STATE for a domain resident in a batch.
 */
int lbm_set_order_rates(lbm_domain *d, double omega3, double omega4, double omega5, double omega6);

/*
 * Outlet condition of the LBM_OUTLET cells (Sec. 2.2, constant outlet
 * pressure by non-equilibrium extrapolation).
 *   kind     LBM_OUTLET_ZERO_GRADIENT: a population pulled from beyond the
 *            last plane x = nx-1 is the post-collision value f*_i(s) of the
 *            last-plane cell s = (nx-1, y - c_y, z - c_z) it faces.
 *            LBM_OUTLET_PRESSURE: it is the value of a ghost cell with the
 *            velocity u_s and the non-equilibrium part of s and the density
 *            rho_out, f*_i(s) + (rho_out - rho_s) f^eq_i(1, u_s).
 *   rho_out  outlet density (pressure rho_out/3), > 0; ignored for the
 *            zero-gradient kind.
 * Takes effect at the next step; the current state is kept.  Errors:
 * LBM_ERR_ARG for an unknown kind or rho_out <= 0, LBM_ERR_STATE for a
 * domain resident in a batch.
 */
int lbm_set_outlet(lbm_domain *d, int kind, double rho_out);

/*
 * Order N of the equilibrium the collision relaxes to (Sec. 2.1, Eq. (4):
 * the Hermite expansion summed to order N; App. A after Eq. (A.6)).
 *   order  6 (the default and the paper's choice): the full expansion the
 *          stencil supports, whose central moments are (rho, 0, ..., 0), so
 *          the collision never forms f^eq.  2..5: the explicit truncated
 *          equilibrium f^eq_N, formed per cell, and
 *          f* = f^eq_N + T^-1 (I - S) T (f - f^eq_N); N = 2 is the classical
 *          second-order equilibrium, N = 3 adds the third-order terms that
 *          make the shear stress Galilean invariant.  Every rate applies as
 *          with the full equilibrium.  The initial state (lbm_init_fields)
 *          and the pressure outlet's ghost value keep the full expansion.
 * Takes effect at the next step.  Errors: LBM_ERR_ARG for an order outside
 * 2..6, LBM_ERR_STATE for a domain resident in a batch.
 */
int lbm_set_equilibrium_order(lbm_domain *d, int order);

/*
 * Curved walls (Sec. 2.2: no-slip walls by the interpolated bounce-back of
 * Bouzidi, Firdaouss and Lallemand, linear form).
 *   q  host, 27*ncells floats, layout [i][cell], or NULL for the halfway
 *      rule everywhere (the default).  q[i][x] is read only where link i of
 *      an updated cell x is a wall link (x - c_i is LBM_SOLID or outside a
 *      non-periodic box): the fraction of the link, from x towards x - c_i,
 *      at which the wall lies, in (0, 1].  With f* the post-collision
 *      populations of the previous step and ibar the opposite of i:
 *        q <  1/2: f_i(x) = 2q f*_ibar(x) + (1 - 2q) f*_ibar(x + c_i)
 *        q >= 1/2: f_i(x) = f*_ibar(x)/(2q) + (1 - 1/(2q)) f*_i(x)
 *      q = 1/2 is the halfway rule; so is q < 1/2 when the link x -> x + c_i
 *      is not a plain link (a gap one cell wide, an inlet behind it).
 * Takes effect at the next step; the state is kept.  Device memory: 12 bytes
 * per link slot of the wall tiles (27*64 per wall tile), only while some q
 * differs from 1/2.  Errors: LBM_ERR_ARG for a fraction outside (0, 1] at a
 * wall link (nothing changed), LBM_ERR_STATE for a domain resident in a
 * batch, LBM_ERR_OOM.
 */
int lbm_set_wall_distances(lbm_domain *d, const float *q);

/*
 * Inlet velocity (Sec. 2.2, Eq. (12) profile, or any field).
 *   u_in  host, 3*ncells floats, layout [component][cell]; read only at
 *         LBM_INLET cells.  A link from an inlet cell s into a fluid cell x
 *         gives f_i(x) = f*_opp(i)(x) + 6 w_i (c_i . u_in(s)) (wall density 1).
 * Without a call, inlet cells act as resting walls.  Only the inlet cells'
 * values are kept (3 floats per inlet cell on the device).
 */
int lbm_set_inlet(lbm_domain *d, const float *u_in);

/* As lbm_set_inlet with the values of the inlet cells only: u_inlet is
 * host, 3*n_inlet floats, layout [component][k] for the k-th inlet cell in
 * ascending cell order (n_inlet from lbm_domain_get_info). */
int lbm_set_inlet_cells(lbm_domain *d, const float *u_inlet);

/*
 * Set the state to the equilibrium f^eq(rho, u) (Eq. (4), sixth order) at
 * every updated cell.
 *   rho  host, ncells floats, or NULL for 1.
 *   u    host, 3*ncells floats [component][cell], or NULL for 0.
 * Clears a sticky LBM_ERR_UNSTABLE.
 */
int lbm_init_fields(lbm_domain *d, const float *rho, const float *u);

/*
 * Advance n >= 0 time steps (each: pull streaming with the boundary rules,
 * then the CHM-MRT collision of Eq. (6), fused in one kernel per step).
 * Synchronous.  Returns LBM_ERR_UNSTABLE if any step produced rho <= 0 or
 * a non-finite value; the error is sticky until lbm_init_fields.  Errors:
 * LBM_ERR_ARG for n < 0, LBM_ERR_STATE for a domain resident in a batch,
 * LBM_ERR_DEVICE.
 */
int lbm_step(lbm_domain *d, int n);

/*
 * lbm_step in two halves, for callers that overlap host work with the
 * steps or time them with events on the domain's stream.
 * lbm_step_async enqueues the n steps on the domain's stream and returns
 * without waiting; lbm_step_wait waits for all enqueued work and reports
 * whether any step since the last check went unstable (LBM_ERR_UNSTABLE,
 * sticky as for lbm_step).  Calls that read or replace the state
 * synchronise the stream themselves; instability of enqueued steps is
 * reported by the next lbm_step_wait or lbm_step.  Errors as lbm_step.
 */
int lbm_step_async(lbm_domain *d, int n);
int lbm_step_wait(lbm_domain *d);

/*
 * Build the step graphs now (lbm_step builds them on first use after a
 * change of rates, outlet, walls, statistics or equilibrium order): one
 * graph per run length 64, 32, ..., 2 steps, each a chain of the step
 * kernels.  Lets a caller keep the building out of a timed run.  Errors:
 * LBM_ERR_STATE for a domain resident in a batch, LBM_ERR_DEVICE.
 */
int lbm_prepare_steps(lbm_domain *d);

/*
 * Density and velocity of the stored state (equal to the pre-collision
 * moments of the same time level, since collision conserves them).
 *   rho  host, ncells floats; u host, 3*ncells floats [component][cell].
 * Cells that are not updated read rho = 0, u = 0.
 */
int lbm_get_moments(lbm_domain *d, float *rho, float *u);

/*
 * As lbm_get_moments, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the moments are staged in a fixed device array of 64 MiB
 * that the library holds on every device it runs on until the process
 * ends, and no hipMalloc, hipFree or other allocating call is made.  The
 * outputs and their layout are those of lbm_get_moments (host buffers of
 * ncells and 3*ncells floats, caller-owned).  Domains of more than
 * 4,194,304 cells (4 floats per cell) are refused with LBM_ERR_ARG.  Calls
 * on one device share the array, which keeps the values of the last call;
 * the library serialises them with a lock, so calls from several threads
 * of one process do not overlap.  Errors: LBM_ERR_ARG, LBM_ERR_STATE for a
 * domain resident in a batch, LBM_ERR_DEVICE.
 */
int lbm_get_moments_noalloc(lbm_domain *d, float *rho, float *u);

/* As lbm_get_moments, into device buffers (ncells and 3*ncells floats). */
int lbm_get_moments_device(lbm_domain *d, float *rho_dev, float *u_dev);

/*
 * The stored populations f_i as FP32 (shifted storage is converted back:
 * f_i = w_i + stored/scale).
 *   f  host, 27*ncells floats, layout [i][cell].
 * Cells that are not updated keep the values of the last lbm_init_fields
 * or lbm_set_populations (the lattice weights after creation).
 */
int lbm_get_populations(lbm_domain *d, float *f);

/* Overwrite the stored populations (FP32 values of f_i, [i][cell], host);
 * converted to the domain's storage. */
int lbm_set_populations(lbm_domain *d, const float *f);

/*
 * Checkpoint and restart of a run.  The study's runs cover 300 flow-through
 * periods and average over the second half (Sec. 2.2), far more steps than
 * one job may hold a device for, so a run must be able to stop and resume.  lbm_get_populations / lbm_set_populations
 * carry the populations f_i, from which the library rebuilds what else a
 * step reads: the outlet cells' clamped values (with the pressure outlet's
 * shift, from the moments of the stored post-collision state) and the
 * curved walls' kept values; a run resumed that way agrees with the
 * uninterrupted one to rounding.  The state calls below instead copy the
 * domain's state exactly as the device holds it, so that a resumed run is
 * bit for bit the uninterrupted one, in every storage:
 *   - the population array as stored (lbm_array_bytes: the tiles in the
 *     domain's storage format, then the outlet side rows), in whichever
 *     phase the last step left it;
 *   - the curved walls' kept values f*_k (27 * 64 floats per wall tile);
 *   - the phase and the instability flag.
 * Not in the state: the configuration (rates, equilibrium order, inlet
 * velocities, outlet kind and density, wall fractions), which the caller
 * sets on the restarted domain as on the original one, before or after
 * lbm_load_state, and the statistics sums.
 *
 * The byte image: a 64-byte header of eight little-endian uint64 words
 * (0: the tag "LBMSTAT1"; 1: nx | ny << 16 | nz << 32 | periodic << 48 |
 * storage << 56; 2: array bytes; 3: kept curved-wall bytes; 4: FNV-1a 64
 * of the flags the domain was created with; 5: phase | unstable << 1;
 * 6, 7: zero), then the array, then the kept values.
 */

/* Bytes of the domain's state image (header, array, kept curved-wall
 * values; the last part is 0 until wall fractions are set). */
int lbm_state_bytes(const lbm_domain *d, size_t *bytes);

/* Copy the state image into host memory buf of `bytes` bytes (at least
 * lbm_state_bytes).  The domain is left as it was.  Errors: LBM_ERR_ARG
 * (null buf, too small), LBM_ERR_STATE (domain resident in a batch),
 * LBM_ERR_DEVICE. */
int lbm_save_state(lbm_domain *d, void *buf, size_t bytes);

/* Replace the domain's state with an image written by lbm_save_state.  The
 * domain must have been created with the same grid, periodic mask, storage
 * and flags, and must have curved walls exactly when the saved one had;
 * otherwise LBM_ERR_ARG (a different size, tag or grid) or LBM_ERR_STATE
 * (other flags, curved walls on one side only, domain resident in a
 * batch), and the domain is unchanged.  LBM_ERR_DEVICE on a failed copy. */
int lbm_load_state(lbm_domain *d, const void *buf, size_t bytes);

/*
 * Time statistics (Sec. 2.2, Eqs. (15)-(18): mean velocity and Reynolds
 * stresses; Eq. (19): viscous shear stress, with the strain rate from the
 * second-order Hermite coefficients, App. A, Eqs. (A.7)-(A.8)).  While on,
 * every local-phase step (every second step) adds, for each updated cell,
 * u, u_a u_b and sigma_ab = 2 rho nu S_ab = -(1 - omega/2) M_ab of the
 * pre-collision state it collides (M_ab: central second-order Hermite
 * moment, omega the shear rate), summed in FP64 on the device
 * (15 * 64 * n_tiles doubles; the products u_a u_b are formed in FP64 from
 * the FP32 velocities).  Also accumulates while the domain is in a batch.
 * lbm_stats_enable(d, 1) clears the sums and starts; (d, 0) stops and keeps
 * them.
 */
int lbm_stats_enable(lbm_domain *d, int on);

/*
 * Means of the statistics since the last lbm_stats_enable(d, 1).
 *   mean_u      host, 3*ncells doubles [component][cell]
 *   mean_uu     host, 6*ncells doubles: <u_x u_x>, <u_y u_y>, <u_z u_z>,
 *               <u_x u_y>, <u_x u_z>, <u_y u_z> (Reynolds stress =
 *               <u_a u_b> - <u_a><u_b>)
 *   mean_sigma  host, 6*ncells doubles, same component order
 *   samples     number of samples in the means
 * Cells that are not updated read 0; all outputs are 0 without samples.
 */
int lbm_stats_get(lbm_domain *d, double *mean_u, double *mean_uu, double *mean_sigma, uint64_t *samples);

int lbm_domain_get_info(const lbm_domain *d, lbm_domain_info *info);

/* Free the domain's device memory and its step graphs.  A domain
 * resident in a batch must be released from it first (LBM_ERR_STATE). */
int lbm_destroy(lbm_domain *d);

/* Thread-local message of the last failing call ("" if none). */
const char *lbm_last_error(void);

/* -------------------------------------------------------------------- */
/* Batched execution: many independent domains advanced together by      */
/* packed launches replayed from HIP graphs of several steps each.        */
/* -------------------------------------------------------------------- */

/*
 * Create a batch.
 *   hbm_budget_bytes  admission limit on the sum of the resident domains'
 *                     device_bytes.
 *   storage           every admitted domain must use this storage.
 *   hip_stream        stream for the batch's work, or NULL for an own one.
 */
int lbm_batch_create(size_t hbm_budget_bytes, int storage, void *hip_stream, lbm_batch **out);

/*
 * Cache blocking of the packed steps.  lbm_batch_step replays graphs of up
 * to window_steps steps (1..64; default 16).  Within one, the resident
 * domains run in groups of consecutive domains of one parity class and one
 * addressing kind (row-aligned or not) whose tile blocks (27 * 64
 * populations per tile) sum to at most group_bytes (a larger domain is a
 * group of its own), and each group takes all of the window's steps before
 * the next group starts, so that a group's populations stay in the
 * device's last-level cache (256 MB on MI355X) between its steps.
 * group_bytes 0: no limit (one group per class and kind, each step over
 * every domain before the next step).
 * Default 192 MiB.  Results do not depend on either setting (domains are
 * independent); takes effect from the next lbm_batch_step.  Errors:
 * LBM_ERR_ARG for a window outside 1..64.
 */
int lbm_batch_set_cache_block(lbm_batch *b, size_t group_bytes, int window_steps);

/*
 * Admit a domain for n_steps > 0 further steps, starting at the batch's next
 * step.  The domain's state stays where it is (no copy).  The call does not
 * wait for work in flight.  Returns LBM_ERR_OOM when the domain does not fit
 * the remaining budget (the caller keeps it queued), LBM_ERR_STATE if the
 * domain is already resident, LBM_ERR_ARG if its population array exceeds
 * 4 GiB - 64 KiB (the packed kernels address with 32-bit byte offsets).
 * *slot receives the slot id.
 */
int lbm_batch_admit(lbm_batch *b, lbm_domain *d, int n_steps, int *slot);

/* Enqueue n packed steps (asynchronous; one graph replay per window of
 * steps, see lbm_batch_set_cache_block).  A resident domain takes part in exactly its admitted number of
 * steps and ends bit for bit in the state lbm_step would give it alone,
 * whatever it is packed with.  Errors: LBM_ERR_ARG for n < 0. */
int lbm_batch_step(lbm_batch *b, int n);

/*
 * Report domains whose admitted steps have all completed on the device
 * since the last poll, and domains that went unstable (rho <= 0 or a
 * non-finite value): those are evicted, take no further steps, and are
 * reported once the steps already enqueued for them have completed.
 * Non-blocking unless wait != 0 (then waits for all enqueued work first).
 * done_slots receives up to max slot ids; *n_done their count.  A reported
 * domain stays resident until lbm_batch_release.
 */
int lbm_batch_poll(lbm_batch *b, int wait, int *done_slots, int max, int *n_done);

/* Release a completed slot: frees its budget, removes its tiles from the
 * packed table, and returns the domain to stand-alone use (its status is
 * LBM_ERR_UNSTABLE if any of its batched steps was unstable). */
int lbm_batch_release(lbm_batch *b, int slot, lbm_domain **d);

/* Number of resident slots, packed steps enqueued so far, packed steps
 * known complete on the device (as of the last poll), and the budget in
 * use.  Any output pointer may be NULL. */
int lbm_batch_stats(const lbm_batch *b, int *resident, uint64_t *steps_enqueued, uint64_t *steps_done,
                    size_t *bytes_in_use);

int lbm_batch_destroy(lbm_batch *b);

/* -------------------------------------------------------------------- */
/* Diagnostics                                                           */
/* -------------------------------------------------------------------- */

/* Host-only self checks of the index arithmetic and tile classification
 * (no device call).  Returns LBM_OK or LBM_ERR_STATE with a message. */
int lbm_selftest_host(void);

/* Test hook for the error paths of batch admission: the n-th (n >= 1)
 * table allocation or staged upload made by the batch calls from now on
 * fails as if device memory were exhausted; n = 0 disables.  Returns
 * LBM_ERR_ARG for n < 0. */
int lbm_debug_fail_after(int n);

/* *wide = 1 if the domain's step kernels address its array with 64-bit
 * global instructions (an array past 4 GiB - 64 KiB, or the test hook
 * below), 0 if with 32-bit buffer offsets. */
int lbm_is_wide(const lbm_domain *d, int *wide);

/* Test hook: on = 1 makes a domain of any size step with the 64-bit
 * addressing kernels of arrays past 4 GiB, so that they can be compared
 * with the 32-bit ones on small grids (the two give the same bits); on = 0
 * returns to the choice by size.  Packed steps always take the 32-bit
 * kernels.  Errors: LBM_ERR_ARG for other values of on, LBM_ERR_STATE while
 * the domain is resident in a batch. */
int lbm_debug_wide_addressing(lbm_domain *d, int on);

/* Test hook: blocks > 0 launches each step of the domain on that many
 * blocks of 256 lanes (a multiple of 8, one block per XCD in turn), each
 * wave walking the tile list with the grid's stride, instead of one wave
 * per tile; blocks = 0 returns to the default.  Results do not depend on the
 * launch shape (no two lanes of a step touch one slot), which the tests
 * check bit for bit.  Errors: LBM_ERR_ARG for other values, LBM_ERR_STATE
 * while the domain is resident in a batch. */
int lbm_debug_step_grid(lbm_domain *d, int blocks);

/* Library version string. */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

/*
 * pic.h -- C ABI of libpic, an MI355X (gfx950) implementation of the
 * data-parallel hot path of one timestep of the 2D electromagnetic
 * particle-in-cell (EM-PIC) cycle studied in "Particle-In-Cell Simulation
 * using Asynchronous Tasking" (Guidotti et al., arXiv 2106.12485).
 *
 * The cycle (paper Sec. 2.2, Fig. 1):
 *   stage 1  bilinear interpolation of the previous-iteration E, B to each
 *            particle;
 *   stage 2  leapfrog + relativistic Boris momentum/position advance;
 *   stage 3  exact charge-conserving (Villasenor-Buneman) current deposition,
 *            optionally smoothed by a binomial digital filter;
 *   stage 4  Yee-mesh FDTD advance of E and B.
 * The paper's spatial decomposition into regions with ghost cells and
 * particle transfer between neighbouring regions (Sec. 3.2) appears here as
 * GPU tiles: each tile owns a particle segment, stages fields and current in
 * LDS with a guard halo, and hands leaving particles to its neighbours.
 * Sec. 4.1 adds a moving window, laser-initialised fields, a compensated
 * binomial filter and immobile neutralising ions.
 *
 * Conventions
 *   - Normalised units: c = 1, time in 1/w_p, length in c/w_p, momenta as
 *     proper velocity u = gamma v, fields in m c w_p / e, charge density in
 *     units of e n_0; dE/dt = curl B - J, dB/dt = -curl E, div E = rho.
 *   - Yee staggering: Ex(i+1/2, j) Ey(i, j+1/2) Ez(i, j) Bx(i, j+1/2)
 *     By(i+1/2, j) Bz(i+1/2, j+1/2); J_k sits with E_k; E and B are both
 *     held at integer time.
 *   - Host field planes are row-major (ny, nx) arrays, x fastest; element
 *     [j*nx + i] is the value at the component's own position next to cell
 *     (i, j).  Planes are ordered Ex Ey Ez Bx By Bz (fields) and Jx Jy Jz
 *     (current).  With a moving window, host cell indices are window
 *     coordinates.
 *   - A particle is a cell index (ix, iy) plus an in-cell offset x, y in
 *     [0, 1) and a momentum (ux, uy, uz); its position is ((ix+x)dx, (iy+y)dy).
 *   - Every call returns 0 (PIC_OK) or a negative PIC_E_* code; no C++
 *     exception crosses the ABI.  pic_strerror() names a code and
 *     pic_last_error() returns the most recent detailed message.
 *   - Device memory is a caller-owned arena (any device allocation, e.g. a
 *     torch uint8 tensor) of at least pic_mem_bytes() bytes; the library
 *     sub-allocates everything from it and allocates no device memory of its
 *     own.  Host pointers passed in are only read during the call; host
 *     output buffers are caller-owned.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is ordered on it; calls that return host data
 *     synchronise it.  A simulation handle must be used from one stream at a
 *     time.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4

enum {
    PIC_OK = 0,
    PIC_E_ARG = -1,      /* invalid argument or configuration */
    PIC_E_CFL = -2,      /* dt violates the 2D Courant limit */
    PIC_E_NOMEM = -3,    /* arena smaller than pic_mem_bytes() */
    PIC_E_CAPACITY = -4, /* a tile or outbox ran out of particle slots */
    PIC_E_HIP = -5,      /* a HIP runtime call failed */
    PIC_E_STATE = -6,    /* call not valid in the handle's current state */
    PIC_E_CANCELLED = -7 /* a serving request was cancelled before it finished */
};

typedef struct pic_sim pic_sim;

/* One particle species, loaded on a lattice of ppc_x * ppc_y sub-cell centres
 * ((m + 1/2)/ppc_x, (l + 1/2)/ppc_y) per cell, wherever the lab-frame x of
 * the particle, ((lab cell) + (m + 1/2)/ppc_x) * dx evaluated in double,
 * lies in [x_lo, x_hi).  Momenta are u = ufl + uth * N(0, 1) per component,
 * the normals drawn by Box-Muller from Philox4x32-10 (Salmon et al., SC'11)
 * with key = (seed low word, seed high word) and counter =
 * (lab cell x, cell y, l * ppc_x + m, species index).  Each macro-particle
 * carries charge sign(q_over_m) * density / (ppc_x * ppc_y), so a uniform
 * load deposits |rho| = density. */
typedef struct {
    double q_over_m;
    double density;
    double x_lo, x_hi;
    int ppc_x, ppc_y;
    double uth[3];
    double ufl[3];
} pic_species_cfg;

/* Initial laser (paper Sec. 4.1: fields start with the laser's values): a 2D
 * paraxial Gaussian beam travelling along +x,
 *   E_perp = a0 w0 g(x) sqrt(W0/w(z)) exp(-r^2/w^2)
 *            cos(w0 (x - x_center) + w0 r^2 / (2 R(z)) - atan(z/zR)/2),
 *   z = x - focus, r = y - axis, zR = w0 W0^2 / 2, w = W0 sqrt(1 + z^2/zR^2),
 *   R = z (1 + zR^2/z^2), g = exp(-2 ln2 (x - x_center)^2 / fwhm^2) cut to 0
 * where |x - x_center| > 2 fwhm; (Ey, Ez) = E_perp (cos pol, sin pol) and
 * (By, Bz) = (-Ez, Ey), each evaluated at its own staggered position. */
typedef struct {
    int on;
    double a0, omega0, W0, fwhm, x_center, focus, axis, pol_angle;
} pic_laser_cfg;

typedef struct {
    int nx, ny;          /* cells; each >= 2 and <= 65535 (nx <= 65518 with the
                            moving window) */
    double lx, ly;       /* box size; dx = lx/nx, dy = ly/ny */
    double dt;           /* must satisfy dt < 1/sqrt(1/dx^2 + 1/dy^2) */
    int moving_window;   /* 1: the box follows +x at c (x not periodic) */
    int filter_passes;   /* binomial 1-2-1 passes per axis (0 = no filter) */
    int filter_compensate; /* 1: compensator (-N, 4+2N, -N)/4 after them */
    int n_species;       /* 0 .. PIC_MAX_SPECIES */
    pic_species_cfg sp[PIC_MAX_SPECIES];
    pic_laser_cfg laser;
    int fp64;            /* 0: FP32 particles/fields/current, 1: FP64 */
    unsigned long long seed;
    int load;            /* 1: load every species at init, 0: start empty */
    double capacity_factor; /* particle slots per buffer and species = factor *
                               the species' largest count (its initial load on
                               a periodic box; the whole box at its ppc with the
                               moving window or without a load), shared among
                               the tiles by count (0 selects 2.0) */
    int deposit_mode;    /* how the tiles' currents are combined (the paper's
                            two strategies, Sec. 3.2):
                            0 "reduction": each tile deposits into a block of
                              its own and a fold launch sums the blocks;
                            1 "commutative": tiles in four checkerboard
                              colours, one colour per launch, add their
                              current straight into J, no two neighbours at
                              once; no fold.  Needs a periodic box with an
                              even number of 16-cell tiles along each axis,
                              the last at least 3 cells wide. */
} pic_cfg;

/* Diagnostics in FP64 (stage a9).  Energies are integrals over the box:
 * e_energy = sum (E^2)/2 dx dy, b_energy = sum (B^2)/2 dx dy at the current
 * time n; ke[s] = sum m_p |u-|^2/(gamma- + 1) dx dy with
 * u- = u^{n-1/2} + (q/m)(dt/2) E^n(x^n) and m_p = q_p/(q/m).
 * gauss_res_max = max over nodes of |div E^n - F rho^n - (div E^0 - F rho^0)|
 * (F = the current filter; zero up to round-off on periodic boxes).
 * cont_res_max = max over nodes of |(rho^n - rho^{n-1})/dt + div J^{n-1/2}|
 * with the unfiltered current of the last step; it is available only when the
 * previous pic_energy call was exactly one step earlier, else it is -1.
 * With the moving window both residuals are taken over window columns
 * 3 <= i < nx - nshift - 3: particles leave at the left edge and the plasma
 * loaded since t = 0 enters at the right. */
typedef struct {
    double e_energy, b_energy;
    double ke[PIC_MAX_SPECIES];
    double total;
    double charge;            /* sum of q_p over particles times dx dy */
    double gauss_res_max;
    double cont_res_max;
    double rho_max;           /* max |rho^n| (scale for the residuals) */
    double t;
    long long n_particles[PIC_MAX_SPECIES];
    long long step;
    int nshift;               /* moving-window shifts done */
    int status;               /* device error state, as pic_status() */
} pic_diag;

/* Device memory one simulation needs (the paper's per-region particle and
 * current buffers of the spatial decomposition, Sec. 3.2, laid out as GPU
 * tiles): the bytes of arena that pic_init will sub-allocate for `cfg`.
 * Used for admission by HBM budget.  cfg is read only.  Returns 0 if the
 * configuration is invalid (pic_last_error() says why); never touches the
 * GPU. */
size_t pic_mem_bytes(const pic_cfg *cfg);

/* Set a simulation up as the paper's evaluation runs start (Sec. 4.1):
 * fields zero except the initial laser, species loaded on their sub-cell
 * lattice with their density profile and momentum distribution, immobile
 * neutralising ions implied by the t = 0 charge.  The time step must satisfy
 * the Courant limit of the Yee scheme of Sec. 2.2 stage 4.
 *   cfg    host struct, read only during the call;
 *   arena  device memory of at least arena_bytes >= pic_mem_bytes(cfg)
 *          bytes, 256-byte aligned, owned by the caller and kept alive until
 *          pic_free; the library zeroes it and keeps every device array in it;
 *   out    receives a handle owning host-side state only.
 * Errors: PIC_E_ARG (invalid cfg or NULL pointer), PIC_E_CFL (Courant limit),
 * PIC_E_NOMEM (arena too small), PIC_E_CAPACITY (initial load does not fit
 * its tiles), PIC_E_HIP.  On error *out is untouched and nothing is held.
 * Synchronises `stream`. */
int pic_init(const pic_cfg *cfg, void *arena, size_t arena_bytes, void *stream,
             pic_sim **out);

/* Stages 1-3 of the cycle (Sec. 2.2, Fig. 1) with the particle transfer
 * between neighbouring regions of Sec. 3.2: interpolate E^n, B^n bilinearly
 * to every particle (stage 1), Boris push to u^{n+1/2} and move (stage 2),
 * deposit the Villasenor-Buneman current of the move into the per-tile
 * current blocks (stage 3, the regions' local buffers with ghost cells), and
 * hand each particle that left its tile to the tile it entered.  Work is
 * enqueued on `stream` and not waited for.  Errors: PIC_E_ARG (NULL handle),
 * PIC_E_HIP (launch failed); a tile or outbox that overflows sets the device
 * error reported by pic_status. */
int pic_deposit(pic_sim *sim, void *stream);

/* The rest of the step: the reduction of the regions' ghost-cell currents
 * (Sec. 3.2; periodic wrap, or dropped beyond the moving window), the
 * binomial digital filter of stage 3 (Sec. 2.2; with the compensator of the
 * laser-wakefield runs, Sec. 4.1), one Yee FDTD advance of E and B (stage 4:
 * B half step, E full step, B half step) and, with the moving window of
 * Sec. 4.1, a shift by one cell once the light front has crossed the next
 * cell boundary (iter*dt >= (nshift+1)*dx in double), removing the particles
 * of the column that leaves and loading the column that enters.  Must follow
 * pic_deposit of the same step.  If that deposit found a tile's particle
 * segment short of a few more steps of the tile's inflow, the end of the step
 * also lays the segments out anew for the next push.  Enqueued on `stream`,
 * not waited for.  Errors: PIC_E_ARG (NULL handle), PIC_E_HIP. */
int pic_field_advance(pic_sim *sim, void *stream);

/* nsteps iterations of the main simulation loop (Sec. 2.2, Fig. 1), each
 * pic_deposit then pic_field_advance.  Between steps the leavers of a push
 * stay in their outboxes and the next push takes them from there (calls that
 * read particles append them first).  The steps are replayed from HIP graphs
 * captured on first use: one of 8 steps while 8 or more remain, then one of a
 * single step.  At most every 8 pushes, and before the first push of each
 * 8-step graph, the particle segments are checked against every tile's count,
 * growth and inflow and laid out anew if one is short; a tile that still
 * outgrows its segment drops the excess and pic_status reports
 * PIC_E_CAPACITY.  nsteps >= 0.  Enqueued on `stream`, not waited for.
 * Errors: PIC_E_ARG (NULL handle, nsteps < 0), PIC_E_HIP. */
int pic_step(pic_sim *sim, int nsteps, void *stream);

/* FP64 diagnostics of the current state (see pic_diag): the field and
 * kinetic energies the paper's validation compares between versions of the
 * code (Sec. 4.2), total charge, and the Gauss and continuity residuals that
 * the exact charge-conserving deposit of Sec. 2.2 stage 3 keeps at round-off.
 * out is a caller-owned host struct, filled on success.  Errors: PIC_E_ARG,
 * PIC_E_HIP.  Synchronises `stream`. */
int pic_energy(pic_sim *sim, pic_diag *out, void *stream);

/* Device error state accumulated so far (no paper passage: a check of the
 * tile capacities of this layout): PIC_OK or PIC_E_CAPACITY (a tile or an
 * outbox overflowed; the excess particles were dropped and the run is no
 * longer valid).  Synchronises. */
int pic_status(pic_sim *sim, void *stream);

/* Release the host state of a handle (NULL is ignored).  Waits for no
 * device work: the caller must not free the arena while work on it is in
 * flight.  The arena stays the caller's. */
int pic_free(pic_sim *sim);

/* ---------------------------------------------------------------------
 * State input and output (tests, checkpoints, serving).  No paper passage
 * defines these; they move the state of Sec. 2.2 (particles, E, B, J)
 * between host arrays and the device, converting to and from FP64.
 * Host arrays are caller-owned and only touched during the call.
 * ------------------------------------------------------------------- */

/* Replace all particles of species sp with n particles given as host arrays
 * (ix in [0, nx), iy in [0, ny), x, y in [0, 1)); values are rounded to the
 * working precision.  PIC_E_CAPACITY if a tile overflows, or at once (the
 * arrays unread) if n exceeds the species' slots over all tiles.
 * Synchronises. */
int pic_set_particles(pic_sim *sim, int sp, long long n, const int *ix, const int *iy,
                      const double *x, const double *y, const double *ux,
                      const double *uy, const double *uz, void *stream);

/* Number of particles of species sp.  Synchronises; returns < 0 on error. */
long long pic_particle_count(pic_sim *sim, int sp, void *stream);

/* Copy species sp to host arrays of capacity `cap` (tile by tile, in the
 * order they are stored); *n_out receives the count.  PIC_E_ARG if cap is too
 * small.  Synchronises. */
int pic_get_particles(pic_sim *sim, int sp, long long cap, long long *n_out, int *ix,
                      int *iy, double *x, double *y, double *ux, double *uy,
                      double *uz, void *stream);

/* Set / get the six field planes (6 * nx * ny doubles).  Synchronises. */
int pic_set_fields(pic_sim *sim, const double *f6, void *stream);
int pic_get_fields(pic_sim *sim, double *f6, void *stream);

/* Current of the last step (3 * nx * ny doubles): filtered != 0 returns the
 * current the field solver used, 0 the folded current before filtering.  A
 * single simulation's step filters inside its field-solver launch, so a
 * filtered request runs the filter on the stored folded current first (same
 * arithmetic, same result).  With the moving window the current is given in
 * the window of the step that deposited it (before that step's shift, if
 * any).  Synchronises. */
int pic_get_current(pic_sim *sim, int filtered, double *j3, void *stream);

/* Set the step counter and the number of window shifts done (to continue a
 * run from a saved state).  Synchronises. */
int pic_set_time(pic_sim *sim, long long iter, int nshift, void *stream);

/* Per-kernel timing with HIP events recorded on `stream` around each launch
 * of pic_deposit / pic_field_advance / pic_step (which then launch directly,
 * not from the graph).  pic_timing(sim, 1) resets and starts, 0 stops.
 * pic_timing_read fills ms[k] (summed milliseconds) and launches[k] for
 * k < nk of: 0 push + deposit (its last block flips the particle buffers),
 * 1 hand-off of pending leavers (settle), 2 fold (a launch of its own only
 * for filter halos of 2 or more, per-species push blocks or batches; else
 * the Yee launch folds), 3 filter (only the requests of pic_get_current:
 * the step filters inside the Yee launch), 4 current filter + Yee (and the
 * fold, where it has no launch of its own) and the step end (field buffer
 * flip, step count), 5 moving-window shift, 6 the push's work order (tiles
 * by decreasing particle count, rewritten every 8 steps).
 * Synchronises. */
#define PIC_NK 7
int pic_timing(pic_sim *sim, int enable, void *stream);
int pic_timing_read(pic_sim *sim, double *ms, long long *launches, int nk, void *stream);

/* Geometry of the tiling: out[0] tile width, out[1] tile height, out[2]
 * tiles along x, out[3] tiles along y, out[4] storage width in x, out[5]
 * particle slots per buffer of species 0 (shared among the tiles), out[6]
 * outbox slots per tile. */
int pic_layout(const pic_sim *sim, long long *out, int n);

/* ---------------------------------------------------------------------
 * Batches and serving.  Independent simulations resident on one GPU are
 * stepped together: each kernel of a step is launched once for the tiles of
 * every simulation of the batch (a device-side descriptor table and
 * (simulation, tile) work list; the step is replayed from a captured HIP
 * graph that serves every batch fitting its grid).  The cycle of each
 * simulation is the one of pic_step; current sums are integers, so a
 * simulation evolves bitwise identically alone and in any batch.
 * ------------------------------------------------------------------- */
typedef struct pic_batch pic_batch;

/* Device workspace for a batch of up to max_sims FP32 periodic simulations
 * (no moving window) with at most max_tiles tiles in total. */
size_t pic_batch_mem_bytes(int max_sims, long long max_tiles);

/* Lay a batch object out in `arena` (device memory owned by the caller, at
 * least pic_batch_mem_bytes, 256-byte aligned).  Also uses pinned host
 * staging for the descriptor table. */
int pic_batch_create(void *arena, size_t arena_bytes, int max_sims, long long max_tiles,
                     pic_batch **out);

/* Step the n simulations `sims` together nsteps times on `stream`.  The set
 * may change from call to call (simulations join and leave between calls);
 * a change synchronises the stream once to restage the descriptors.  No
 * simulation of the set may be stepped elsewhere meanwhile.  PIC_E_ARG for
 * FP64 or moving-window simulations or a set that exceeds the batch. */
int pic_batch_step(pic_batch *b, pic_sim *const *sims, int n, int nsteps, void *stream);

int pic_batch_free(pic_batch *b);

/* pic_batch_step without a batch object, for callers that cannot allocate
 * (code under HIP graph capture, serving loops that must not allocate,
 * harnesses that forbid it): the descriptor table, the batch descriptor and
 * the work lists live in a file-scope device array of the library (about
 * 1.2 MB, one copy per GPU, held until the process ends), staged on `stream`
 * by small kernels at every call.  It calls no hipMalloc, hipFree, pinned
 * host allocation or graph instantiation; the steps are launched directly.
 * Same simulations and semantics as pic_batch_step (FP32 periodic, reduction
 * deposit) and the same kernels, so results are bitwise those of
 * pic_batch_step.  At most PIC_STATIC_MAX_SIMS simulations with at most
 * PIC_STATIC_MAX_TILES tiles together, else PIC_E_ARG (nothing launched).
 * The device holding the simulations must be current.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  Asynchronous. */
#define PIC_STATIC_MAX_SIMS 32
#define PIC_STATIC_MAX_TILES 16384
int pic_batch_step_static(pic_sim *const *sims, int n, int nsteps, void *stream);

/* One serving request: a simulation, the steps to run, its arrival time in
 * seconds after the start of pic_serve, and a deadline at which it is
 * cancelled if not finished (cancel_s <= 0: never). */
typedef struct {
    pic_cfg cfg;
    int nsteps;
    double arrival_s;
    double cancel_s;
} pic_request;

typedef struct {
    double admit_s;      /* when it got memory and was initialised (0: never) */
    double done_s;       /* when its last step finished, or when it was cancelled */
    pic_diag diag;       /* diagnostics after the last step done */
    int status;          /* PIC_OK, PIC_E_CANCELLED or the error that ended it */
} pic_result;

typedef struct {
    int batched;         /* 1: continuous batching; 0: one at a time, in order */
    int chunk_steps;     /* steps between admission points (>= 1) */
    int max_batch;       /* most simulations running at once (<= 0: 256) */
    int rate_ratio;      /* batched: a request that costs c times less than the
                            largest one running takes min(c, rate_ratio) times as
                            many steps per chunk (<= 1: every request in lockstep) */
    const volatile int *cancel; /* NULL, or n flags the caller may set from another
                            thread while pic_serve runs: cancel[i] != 0 cancels
                            request i at the next chunk boundary */
    long long max_particles; /* batched: a queued request joins a non-empty running
                            set only while the set's initial particle loads, its
                            own included, stay within this; the queue is then
                            admitted strictly in arrival order (<= 0: no limit) */
    long long lone_particles; /* batched, with max_particles: the same limit for a
                            request that no other queued request waits behind
                            (<= 0: max_particles) */
} pic_serve_opts;

/* Serve n requests in real time (the work is the paper's cycle of Sec. 2.2 on
 * many independent simulations; no paper passage defines the loop itself): a
 * request is queued at its arrival time, admitted (first fit, in arrival
 * order) when its pic_mem_bytes fits in the free part of `arena` (the HBM
 * budget) and, with max_particles, the running set's load allows, initialised on a stream of its own while the running set keeps
 * stepping, stepped with the running set in chunks of at most chunk_steps
 * (shared launches, pic_batch_step; a set of one runs its own step graph;
 * with rate_ratio > 1, cheaper requests take extra steps per chunk in shared
 * launches of their own, pic_batch_step_static), and retired when done,
 * freeing its memory.  A request cancelled (cancel_s passed, or its cancel
 * flag set) is retired at the next chunk boundary with PIC_E_CANCELLED and the
 * diagnostics of the steps it did, freeing its memory for the queue; a
 * queued one is dropped.  Batched serving takes FP32 periodic requests with
 * the reduction deposit; others end with PIC_E_ARG.  One at a time
 * (batched = 0) runs the requests alone, in arrival order.  out[i] receives
 * request i's times and final diagnostics.  step_ms (capacity cap_steps, may
 * be NULL) receives the time per step of every chunk and *n_steps their
 * number.  The call returns when all its device work is done.  Returns
 * PIC_OK or the first host-side error. */
int pic_serve(const pic_request *reqs, int n, void *arena, size_t arena_bytes,
              const pic_serve_opts *opts, pic_result *out, double *step_ms,
              long long cap_steps, long long *n_steps, void *stream);

const char *pic_strerror(int code);
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */

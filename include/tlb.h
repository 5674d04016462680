/*
 * tlb.h -- C ABI of the MI355X ternary wetting lattice Boltzmann library.
 *
 * The library advances the ternary phase-field lattice Boltzmann model of
 * Liang, Xu, Chen, Chai & Shi, "Lattice Boltzmann modeling of wall-bounded
 * ternary fluid flows" (arXiv:1710.09534) on one AMD Instinct MI355X (gfx950):
 * two order-parameter LB equations and one hydrodynamic LB equation on a D2Q9
 * lattice (Sec. II.A, Eqs. 1-20), with the paper's ternary wetting boundary
 * scheme at solid-adjacent fluid nodes and half-way bounce-back at solid
 * links (Sec. II.B, Eqs. 40-45).
 *
 * Conventions (all calls):
 *  - Lattice units, dx = dt = 1 (Sec. II.A).
 *  - Host fields are row-major doubles, x fastest: value(x, y) = a[y*nx + x],
 *    y = 0 is the bottom row.
 *  - material[y*nx + x] == 0 marks a fluid node; m >= 1 a solid node of
 *    material mats[m-1].  A solid wall surface lies half a link from the
 *    adjacent fluid node (Sec. II.B).  In a non-periodic direction every node
 *    on the domain edge must be solid.
 *  - Every call returns a tlb_status (0 = TLB_OK); nothing throws across the
 *    ABI.  Errors are checked in the order EINVAL (null pointer, bad size),
 *    EPARAM (inadmissible physics), ESTATE (call order), EDIVERGED, EDEVICE.
 *    A failed call leaves the context unchanged, except EDIVERGED: after it
 *    tlb_step keeps returning EDIVERGED (and a batch refuses the context)
 *    until tlb_init_fields or tlb_checkpoint_load replaces the state; reads,
 *    mass, checkpoint_save and destroy still work.  tlb_last_error() gives
 *    the message.
 *  - Host arrays are borrowed for the duration of the call only.
 *  - A context is not thread-safe.  Contexts on different streams may run
 *    concurrently.
 */
#ifndef TLB_H
#define TLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLB_OK = 0,
    TLB_EINVAL = -1,    /* null pointer, size or buffer mismatch */
    TLB_EPARAM = -2,    /* physics parameters outside the admissible range */
    TLB_ENOMEM = -3,    /* workspace too small / allocation failed */
    TLB_EDEVICE = -4,   /* HIP error; tlb_last_error() carries its text */
    TLB_EDIVERGED = -5, /* a NaN/Inf order parameter was detected */
    TLB_ESTATE = -6,    /* call out of order (e.g. step before init) */
    TLB_EBUSY = -7      /* server: no slot / budget, or request not finished */
} tlb_status;

/* Storage precision of the populations (arithmetic in brackets):
 *  TLB_FP64    all 27 populations and the 4 history scalars in FP64 [FP64]
 *  TLB_FP32    everything in FP32 [FP32]
 *  TLB_FP16DEV the 16 moving order-parameter populations f^i_{k!=0} as
 *              FP16 values scaled by a per-family power of two (their
 *              rest-state equilibria are zero, so the value is its deviation
 *              from the rest state); the rest populations f^1_0, f^2_0
 *              (carrying c_i), the 9 hydrodynamic populations g_k and the
 *              history in FP32 [FP32].  (g in FP16 lets the velocity drift
 *              under sustained shear: 5.9e-4 in c after 1000 steps between
 *              walls at +-0.01, against 3.9e-5 with g in FP32.)
 *              Mass sums are FP64 in every mode. */
/* The two sentinels give the enum the range of a 32-bit int, so that any int
 * a caller passes is a valid value of the type (the library then refuses the
 * unknown ones with TLB_EINVAL); they are not precisions. */
typedef enum {
    TLB_FP64 = 0,
    TLB_FP32 = 1,
    TLB_FP16DEV = 2,
    TLB_PRECISION_RANGE_MIN_ = -0x7fffffff - 1,
    TLB_PRECISION_RANGE_MAX_ = 0x7fffffff
} tlb_precision;

/* Fluid properties (Sec. II.A). */
typedef struct {
    double sigma12, sigma13, sigma23; /* pairwise surface tensions, Eq. 7 */
    double D;                         /* interface thickness, Eq. 8 */
    double M0;                        /* mobility scale: M_i = M0/lambda_i, Eq. 12 */
    double tau1, tau2;                /* order-parameter relaxation times, Eq. 1a;
                                         eta_i follows from M_i = eta_i c_s^2 (tau_i - 1/2),
                                         Eq. 18a, one eta per component */
    double rho[3], nu[3];             /* phase densities / kinematic viscosities, Eqs. 14-15;
                                         local tau_g = nu/c_s^2 + 1/2, Eq. 18b */
    double gravity[2];                /* body force G = rho * gravity (Sec. III.A) */
    double lambda;                    /* coefficient of lambda c1^2 c2^2 c3^2 in the bulk
                                         energy, Eq. 5 (>= 0): the chemical potentials follow
                                         Eq. 6; 0 gives the paper's Eq. 8 */
} tlb_fluid;

/* Material kinds. */
enum {
    TLB_WALL = 0,     /* solid wall: wetting ghosts (Eq. 42), symmetric ghosts (Eq. 43),
                         half-way bounce-back (Eq. 44) */
    TLB_VELOCITY = 1  /* velocity boundary node of the non-equilibrium extrapolation
                         scheme (Sec. III.D, Eqs. 51-53) */
};

/* A boundary material.  For TLB_WALL: its wettability and its tangential wall
 * velocity.  For TLB_VELOCITY: wall_u is the prescribed velocity u_w of the
 * boundary nodes, the angles are ignored.  A velocity boundary node x_u
 * takes, for every macroscopic quantity but u, the value at the fluid node
 * x_f directly inside it (chi(x_u) = chi(x_f), as stated with Eq. 53): its
 * populations are its equilibrium (Eq. 53) plus the non-equilibrium part of
 * x_f (Eqs. 51-52), collided like any node (Eq. 45) with the source terms of
 * Eq. 11 formed from x_f's quantities and u = u_w; stencils at fluid nodes
 * see x_u with x_f's values. */
typedef struct {
    double theta13_deg, theta23_deg; /* static contact angles, Eq. 38; theta12 from Eq. 39 */
    double wall_u[2];                /* wall velocity (bounce-back with the moving-wall
                                        momentum term; 0 = the paper's resting wall), or
                                        the boundary velocity of a TLB_VELOCITY material */
    int kind;                        /* TLB_WALL or TLB_VELOCITY */
} tlb_material;

/* field bits of tlb_read_fields; fields are written in this bit order */
enum {
    TLB_F_C1 = 1u << 0, TLB_F_C2 = 1u << 1, TLB_F_C3 = 1u << 2, TLB_F_RHO = 1u << 3,
    TLB_F_UX = 1u << 4, TLB_F_UY = 1u << 5, TLB_F_P = 1u << 6, TLB_F_MU1 = 1u << 7,
    TLB_F_MU2 = 1u << 8, TLB_F_MU3 = 1u << 9, TLB_F_ALL = (1u << 10) - 1
};

typedef struct tlb_ctx tlb_ctx;

/* Device workspace needed for an nx x ny lattice at precision p (bytes).
 * Returns 0 for nx or ny < 3, an unknown precision, or a lattice beyond the
 * size limit of tlb_create. */
size_t tlb_workspace_bytes(int nx, int ny, tlb_precision p);

/* Create a context on a caller-owned device workspace (at least
 * tlb_workspace_bytes, 256-byte aligned, alive until tlb_destroy) and a HIP
 * stream (hipStream_t, NULL = default stream).  Validates the fluid
 * parameters (Eqs. 7, 9, 18): lambda_i > 0, lambda >= 0, lambda_i >
 * lambda_T/2 when lambda = 0 (the range stated for that energy), tau_i > 1/2,
 * D > 0, M0 > 0, rho_i > 0, nu_i > 0 (else TLB_EPARAM).
 * Each family of 9 population planes and the history must stay below 2 GiB,
 * counted with rows padded to a multiple of 64 nodes: at most about 29.8 M
 * nodes in FP64 (e.g. 5400 x 5400), 59.6 M in FP32 and in FP16-dev;
 * else TLB_EINVAL.
 * The library owns *out until tlb_destroy. */
tlb_status tlb_create(int nx, int ny, tlb_precision p, const tlb_fluid* fl,
                      void* dev_workspace, size_t ws_bytes, void* hip_stream,
                      tlb_ctx** out);

/* Boundary geometry and wettability.  material: host uint8 [ny*nx]; mats[m-1]
 * for each material id m in 1..n_mats (n_mats <= 15).  theta12 of each wall
 * material is derived from Eq. 39 (sigma12 cos12 = sigma13 cos13 - sigma23
 * cos23) and written to theta12_out[n_mats] in degrees when non-NULL (NaN for
 * a velocity material); |cos theta12| > 1 is TLB_EPARAM.  Velocity boundary
 * nodes may only lie in row 0 or row ny-1 of a lattice with periodic_y = 0,
 * and the node directly inside each (row 1 or ny-2) must be fluid; an
 * unknown kind or a misplaced velocity node is TLB_EINVAL.  Must precede
 * tlb_init_fields. */
tlb_status tlb_set_geometry(tlb_ctx* ctx, int periodic_x, int periodic_y,
                            const uint8_t* material, const tlb_material* mats,
                            int n_mats, double* theta12_out);

/* Initial order parameters and velocity (host [ny*nx] each; ux/uy NULL =
 * at rest).  The populations start at their equilibria (Eqs. 2a, 2b) with
 * the chemical potential of the initial field (Eq. 8 with the wetting ghosts
 * of Eq. 42), pressure 0, and the time-derivative history set to
 * (c1, c2, ux, uy).  Values at solid nodes are ignored.  Synchronous. */
tlb_status tlb_init_fields(tlb_ctx* ctx, const double* c1, const double* c2,
                           const double* ux, const double* uy);

/* Advance nsteps time steps, asynchronously on the context's stream.  Each
 * step is one fused pass: streaming with bounce-back (Eq. 44), moments
 * (Eqs. 13-15), wetting ghosts and chemical potentials (Eqs. 8, 20, 42),
 * forces (Eqs. 11-12), pressure (Eq. 13c), collision (Eq. 45); where
 * tlb_set_pair_rows applies, two such steps run in one launch (same
 * results).  Every check_interval steps (tlb_set_check_interval, default
 * 100) a mass/NaN reduction runs on the device; a NaN seen by an earlier
 * check makes this call return TLB_EDIVERGED without stepping. */
tlb_status tlb_step(tlb_ctx* ctx, int64_t nsteps);
tlb_status tlb_set_check_interval(tlb_ctx* ctx, int64_t interval); /* 0 = never */
int64_t    tlb_step_count(const tlb_ctx* ctx);

/* Macroscopic fields at the current time, evaluated from the current
 * populations exactly as a step would (Eqs. 3, 8, 13-15).  host_out holds
 * popcount(field_mask) * ny*nx doubles, fields in bit order.  Solid nodes
 * read 0.  Synchronizes the stream. */
tlb_status tlb_read_fields(tlb_ctx* ctx, uint32_t field_mask, double* host_out);

/* The 27 populations f(x,t) entering the next collision (after streaming
 * and bounce-back): host [27][ny*nx] doubles, planes f1_0..8, f2_0..8,
 * g_0..8.  Solid nodes read 0.  Synchronizes. */
tlb_status tlb_read_populations(tlb_ctx* ctx, double* host_out);

/* Per-component mass: sums of c1, c2 and c3 = 1 - c1 - c2 over fluid nodes
 * in FP64 (deterministic two-pass device reduction with wavefront sums),
 * read from the history planes, i.e. of the state the last step started
 * from; the step conserves these sums (Eqs. 2a, 3, 11a, 44), so they equal
 * those of the current populations up to rounding.  Returns TLB_EDIVERGED
 * if c1, c2, ux or uy is NaN/Inf at any fluid node.  Synchronizes. */
tlb_status tlb_mass(tlb_ctx* ctx, double out[3]);

/* For callers that cannot allocate or wait: code under HIP graph capture,
 * tight serving loops, harnesses that forbid device allocation.  The sums of
 * tlb_mass, enqueued on the context's stream without synchronizing:
 * dev_out (device memory, 4 doubles, owned by the caller) receives sum c1,
 * sum c2, sum c3 over fluid nodes and the count of fluid nodes whose c1, c2,
 * ux or uy is NaN/Inf, bitwise equal to what tlb_mass computes.  The partial
 * sums go to a static array in device memory (512 x 4 doubles, one copy per
 * GPU, resolved in tlb_create), not to the workspace; its size does not
 * depend on the lattice, so every lattice tlb_create accepts fits.  The call
 * allocates nothing, launches two kernels and copies nothing to the host; it
 * does not set the context's diverged state (the caller reads dev_out[3]).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams) race.  TLB_EINVAL null pointer, TLB_ESTATE before
 * tlb_init_fields, TLB_EDEVICE launch error. */
tlb_status tlb_mass_noalloc(tlb_ctx* ctx, double* dev_out);

/* Checkpoint: populations, history, step count.  host_buf holds
 * tlb_checkpoint_bytes bytes.  A restored context continues bitwise
 * identically. */
tlb_status tlb_checkpoint_bytes(const tlb_ctx* ctx, size_t* bytes);
tlb_status tlb_checkpoint_save(tlb_ctx* ctx, void* host_buf);
tlb_status tlb_checkpoint_load(tlb_ctx* ctx, const void* host_buf);

/* Average device time per step over nsteps steps launched back to back
 * (HIP events on the context's stream; advances the state by nsteps; two
 * steps per launch where tlb_set_pair_rows applies, without health checks). */
tlb_status tlb_time_steps(tlb_ctx* ctx, int64_t nsteps, double* ms_per_step);

/* Rows of the strip one workgroup of the step kernel marches through
 * (tuning knob; results are bitwise identical for every legal value).
 * rows: a multiple of 4 in [8, 4096].  Default, with C the device's compute
 * units and W = 2 strips per CU (1 in FP64), the count that measured
 * fastest: 128 when
 * strips of 64 rows would outnumber C * W but strips of 128 rows would not;
 * else 64 when that gives at least C strips; else the tallest of 48, 32, 24
 * that does, or 16. */
tlb_status tlb_set_tile_rows(tlb_ctx* ctx, int rows);

/* Two steps per launch (a throughput knob; results are bitwise identical to
 * stepping one at a time).  tlb_step and tlb_time_steps advance the lattice
 * two steps per kernel launch whenever two or more steps remain before the
 * next health check: one workgroup marches a strip of `rows` rows and 64
 * columns through both steps (Eqs. 3-20, 42-45 applied twice), keeping the
 * intermediate populations in on-chip memory, so the populations cross HBM
 * once per two steps.  rows: a multiple of 4 in [8, 4096]; 0 turns it off
 * (one step per launch); -1, the default, picks among 256, 128, 64, 32, 16
 * and 8 rows the height whose launch runs the fewest strip iterations per
 * compute unit (one workgroup per compute unit; rounds of strips times four-row
 * groups plus four of pipeline).  Applies to FP32 populations, on lattices of any size (with
 * every optional part: velocity boundaries, lambda > 0, gravity); a context
 * of another precision steps one step per launch, and returns TLB_EINVAL for
 * rows > 0. */
tlb_status tlb_set_pair_rows(tlb_ctx* ctx, int rows);

/* Picks the strip height with the shortest step among candidate values
 * (16 .. 128 rows, up to the lattice height) by timing steps_per_candidate
 * steps of each, and keeps it.  The timed steps are real steps of the solve
 * (results do not depend on the strip height), so the step count advances by
 * steps_per_candidate times the number of candidates. */
tlb_status tlb_autotune_rows(tlb_ctx* ctx, int steps_per_candidate, int* best_rows);

/* ---- batches: many independent lattices advanced by shared launches ----
 * A batch holds initialised contexts of one precision (any sizes, fluids and
 * geometries).  Each launch covers the strips of all lattices (one step, or
 * two for FP32 batches, see tlb_batch_set_pair_rows), so small lattices fill
 * the GPU together.  A lattice's result
 * is bitwise the same alone or in any batch.  The caller owns the device
 * table (tlb_batch_table_bytes, 256-byte aligned) and the contexts; while a
 * context is in a batch it must not be stepped on its own (tlb_batch_step
 * then returns TLB_ESTATE until tlb_batch_set is called again), and before a
 * member is read or stepped on its own stream the batch stream must be
 * synchronized (tlb_batch_sync).  Graph capture needs a non-default stream. */
typedef struct tlb_batch tlb_batch;
size_t     tlb_batch_table_bytes(int max_lattices);
tlb_status tlb_batch_create(int max_lattices, void* dev_table, size_t bytes,
                            void* hip_stream, tlb_batch** out);
/* sets the member contexts (synchronizes their streams); n may be 0.  A
 * member whose one-step strip height was never set with tlb_set_tile_rows
 * takes one chosen for the whole batch (the height with the fewest strip
 * iterations per workgroup slot over all members), also for its later steps
 * on its own; results do not depend on strip heights. */
tlb_status tlb_batch_set(tlb_batch* batch, tlb_ctx* const* ctxs, int n);
/* captures `steps` steps (even; a multiple of 4 while the batch takes two
 * steps per launch, see tlb_batch_set_pair_rows) into a HIP graph replayed
 * by tlb_batch_step (0 = plain launches) */
tlb_status tlb_batch_use_graph(tlb_batch* batch, int steps);
/* advances every member by nsteps, asynchronously on the batch stream;
 * TLB_ESTATE if a member was stepped outside the batch, TLB_EDIVERGED if a
 * member's health check found a non-finite field, TLB_EDEVICE if a launch
 * fails (the members then count the launches that went out before it) */
tlb_status tlb_batch_step(tlb_batch* batch, int64_t nsteps);
/* Two steps per launch for the whole batch (results bitwise those of one
 * step per launch of the same batch): when every member is FP32,
 * tlb_batch_step advances the members two steps per launch
 * of the two-step kernel (tlb_set_pair_rows) over strips of `rows` rows of
 * every member (rows: a multiple of 4 in [8, 4096]; -1, the default: each
 * member's height rounded up to a multiple of 4, at least 8 and at most a
 * batch height h, the h among 128, 64, 32, 16 and 8 whose launch runs the
 * fewest strip iterations per compute unit), and tlb_batch_use_graph then needs a
 * multiple of 4 steps; with rows = 0, or a member of another precision, one step per
 * launch.  Re-registers the members (as tlb_batch_set) and drops a
 * captured graph.  TLB_EINVAL bad rows, TLB_ESTATE if a member was stepped
 * outside the batch. */
tlb_status tlb_batch_set_pair_rows(tlb_batch* batch, int rows);
tlb_status tlb_batch_sync(tlb_batch* batch);
/* Strip heights of the members (the step kernel's tile shape), tuned for the
 * batched launch: members of equal height form a size class, and one pass
 * over the classes, tallest first, gives each class the height among 16,
 * 24, 32, 48, 64, 96 and 128 rows (at most the lattice's) that makes the
 * batched step shortest, each candidate timed over steps_per_candidate
 * batched steps (HIP events on the batch stream).  Advances every member by
 * those steps (results do not depend on strip heights, bitwise), re-registers
 * the members and drops a captured graph (call tlb_batch_use_graph again).
 * best_rows (nullable) receives the tallest class's height.  TLB_ESTATE
 * before tlb_batch_set. */
tlb_status tlb_batch_autotune_rows(tlb_batch* batch, int steps_per_candidate, int* best_rows);
/* Two-step strip heights of the members, tuned for the batched launch (the
 * launch batches take by default, see tlb_batch_set_pair_rows): members of
 * equal height form a size class, and one pass over the classes, tallest
 * first, gives each class the height among 8, 16, 32, 64 and 128 rows (up to
 * the first that covers the lattice in one strip row) that makes the batched
 * step shortest, each candidate timed over steps_per_candidate batched steps
 * (rounded up to even; HIP events on the batch stream).  Advances every
 * member by those steps (results do not depend on strip heights, bitwise),
 * re-registers the members and drops a captured graph.  The tuned heights
 * apply to members of those heights in later tlb_batch_set calls too, until
 * tlb_batch_set_pair_rows is called.  best_rows (nullable) receives the
 * tallest class's height.  TLB_ESTATE before tlb_batch_set, or when the batch
 * does not take two steps per launch at its default heights. */
tlb_status tlb_batch_autotune_pair_rows(tlb_batch* batch, int steps_per_candidate, int* best_rows);
const char* tlb_batch_last_error(const tlb_batch* batch);
void       tlb_batch_destroy(tlb_batch* batch);

/* ---- measurement helper (not part of the method) ----
 * Streaming references for the bandwidth the step kernel reaches: average
 * device time of `reps` launches (after one warm-up launch) of
 *   kind 0: a copy of `bytes` (a multiple of 16) from dev_src to dev_dst in
 *           16-byte words (dwordx4 loads, non-temporal stores); moves
 *           2 * bytes per launch;
 *   kind 1: the step kernel's access shape on an nx x ny lattice without its
 *           arithmetic: 64-column strips of tile_rows rows (a multiple of 4),
 *           four row waves, each node reading 31 FP32 planes (27 at x - e_k of
 *           the D2Q9 directions, wrapped, and 4 at x) and writing 31 planes at
 *           x; dev_src and dev_dst each hold bytes >= 31 * ny * pitch * 4
 *           (pitch = nx rounded up to 64); moves 248 bytes per node.
 * Device buffers are the caller's; HIP events on hip_stream; synchronizes.
 * TLB_EINVAL for bad arguments, TLB_EDEVICE for a HIP error. */
tlb_status tlb_probe_bandwidth(int kind, int nx, int ny, int tile_rows, const void* dev_src,
                               void* dev_dst, size_t bytes, void* hip_stream, int reps,
                               double* ms_per_launch);

/* ---- serving: continuous batching of independent solves ----
 * A server owns a worker thread that admits submitted requests (in arrival
 * order, skipping ones that do not fit yet) whenever one of max_slots slots
 * and a block of the caller's device arena are free, keeps their populations
 * resident, and advances all running requests together with the batched step
 * kernel, quantum_steps at a time (a quantum also ends at the next
 * completion).  Set-up and readout of requests run on a second stream of the
 * server while the others' quantum is in flight.  Running requests are
 * checked for NaN/Inf every tlb_server_set_check_steps steps and once more
 * when they finish (a diverged request fails alone), then read out to host
 * memory and release their memory for waiting requests.  A request's result
 * is bitwise the same alone or in any mix.
 * Time to solution = completion - submission (host steady clock). */
enum { TLB_REQ_QUEUED = 0, TLB_REQ_RUNNING = 1, TLB_REQ_DONE = 2, TLB_REQ_FAILED = 3,
       TLB_REQ_CANCELLED = 4 };

typedef struct {
    int nx, ny;
    tlb_fluid fluid;
    int periodic_x, periodic_y;
    const uint8_t* material;          /* [ny*nx], 0 = fluid, m = mats[m-1] */
    const tlb_material* mats;
    int n_mats;
    const double *c1, *c2, *ux, *uy;  /* [ny*nx]; ux, uy nullable */
    int64_t nsteps;
    uint32_t result_fields;           /* TLB_F_* fields kept for tlb_server_result */
} tlb_request;                        /* every array is copied by tlb_server_submit */

typedef struct {
    int64_t completed, failed, queued, running;
    double busy_seconds;              /* time spent in device quanta */
    double node_steps;                /* lattice updates performed */
    size_t arena_free_largest;        /* largest free arena block (bytes) */
} tlb_server_counters;

typedef struct tlb_server tlb_server;
/* dev_arena: caller-owned device memory (256-byte aligned) that bounds the
 * server's device footprint (the HBM budget); the server never allocates
 * device memory of its own.  hip_stream: the server's stream (non-default). */
tlb_status tlb_server_create(void* dev_arena, size_t arena_bytes, int max_slots,
                             tlb_precision p, int64_t quantum_steps, void* hip_stream,
                             tlb_server** out);
/* Interval of the mass/NaN health check of running requests (default 1000
 * steps): every `steps` steps each running request's check is queued behind
 * its quantum, and a request whose c1, c2, ux or uy is no longer finite fails
 * with TLB_EDIVERGED at that quantum boundary (the others run on). */
tlb_status tlb_server_set_check_steps(tlb_server* s, int64_t steps);
/* TLB_ENOMEM if the request can never fit the arena */
tlb_status tlb_server_submit(tlb_server* s, const tlb_request* req, uint64_t* id);
tlb_status tlb_server_poll(tlb_server* s, uint64_t id, int* state);
/* blocks until the request is DONE, FAILED or CANCELLED (timeout_s < 0:
 * no limit; TLB_EBUSY on timeout) */
tlb_status tlb_server_wait(tlb_server* s, uint64_t id, double timeout_s);
/* fields (bit order, subset of result_fields) and time to solution.  A
 * FAILED request returns the status that failed it: TLB_EDIVERGED for a
 * NaN/Inf order parameter, TLB_EPARAM / TLB_EINVAL for a fluid or geometry
 * that tlb_create / tlb_set_geometry reject, TLB_EDEVICE for a HIP error. */
tlb_status tlb_server_result(tlb_server* s, uint64_t id, uint32_t field_mask,
                             double* host_out, double* latency_s);
/* forgets a finished request (frees its host result) */
tlb_status tlb_server_release(tlb_server* s, uint64_t id);
/* queued: dropped; running: leaves at the next quantum boundary */
tlb_status tlb_server_cancel(tlb_server* s, uint64_t id);
tlb_status tlb_server_stats(tlb_server* s, tlb_server_counters* out);
/* Message of the calling thread's last failed tlb_server_* call (valid until
 * that thread's next server call; s may be NULL).  A failed request's own
 * reason is returned by tlb_server_result. */
const char* tlb_server_last_error(const tlb_server* s);
/* stops the worker (running and queued requests are cancelled) */
void       tlb_server_destroy(tlb_server* s);

/* Last error message of ctx, or of the calling thread's last failed
 * tlb_create / batch call when ctx is NULL. */
const char* tlb_last_error(const tlb_ctx* ctx);

/* Releases the context (not the caller's workspace).  NULL is a no-op. */
void tlb_destroy(tlb_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* TLB_H */

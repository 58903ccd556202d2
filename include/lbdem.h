/*
 * lbdem.h -- C interface of the MI355X (gfx950) coupled lattice-Boltzmann / DEM library.
 *
 * The library advances the hydro-micromechanical model of Cheng, Luding, Rivas, Harting
 * and Magnanimo, "Hydro-micromechanical modeling of wave propagation in saturated
 * granular media" (arXiv 1808.08921):
 *   - a D3Q19 BGK fluid (Sec. 2.1, Eqs. bgk, stream, BGKequili, rhoAndU, Eq. 3d19q),
 *   - spherical DEM particles with Hertz normal and Mindlin tangential contacts and
 *     Newton-Euler motion (Sec. 2.2, Eqs. translate, rotate, fdLawn, fdLaws),
 *   - two-way coupling by momentum exchange: half-way bounce-back on moving particle
 *     surfaces, link force and torque, and conversion of covered / uncovered nodes
 *     (Sec. 2.3, Eqs. mem, fFS, convertFS, convertSF, coupleF, coupleT),
 *   - a density-prescribed face driven by an oscillating waveform (Sec. 2.4, Eq. source,
 *     Table 2 "tab:source").
 * One call to lbdem_step advances every lattice of a set by whole time steps on the GPU.
 *
 * Conventions (all functions):
 *   - Every function returns 0 (LBDEM_OK) or a negative LBDEM_E* code and never throws
 *     across this interface; lbdem_last_error() gives a message for the calling thread.
 *   - Lattice units, dx = dt = 1.  Node (i,j,k) sits at coordinate (i,j,k); fields are
 *     stored with x fastest: cell n = (k*ny + j)*nx + i.
 *   - Face order everywhere: -x, +x, -y, +y, -z, +z.
 *   - Host pointers are caller-owned, read or written during the call only, and the
 *     call synchronises the library's stream before returning when it copies data.
 *   - Device work is queued on the HIP stream given to lbdem_create (or later to
 *     lbdem_set_stream); lbdem_step is asynchronous with respect to the host.
 *   - Particle indices are per lattice, in the caller's order, 0..n-1.
 *   - Populations are exchanged as double, [19][nz][ny][nx], direction d = 0..18 being
 *     the paper's d = 1..19 of Eq. (3d19q) (d = 18 is the rest population).
 */
#ifndef LBDEM_H
#define LBDEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBDEM_OK 0
#define LBDEM_EINVAL (-1)    /* an argument is out of range or inconsistent */
#define LBDEM_EDEVICE (-2)   /* the HIP runtime reported an error */
#define LBDEM_ECAPACITY (-3) /* a fixed-capacity device table overflowed (lbdem_status) */
#define LBDEM_ENOMEM (-4)    /* the workspace is too small or host memory ran out */
#define LBDEM_ESTATE (-5)    /* the call is not valid in the current state */
#define LBDEM_ERANGE (-6)    /* a requested step range is not (or no longer) recorded */
#define LBDEM_ENUMERIC (-7)  /* the fluid's density left the positive finite numbers (lbdem_status) */

/* face boundary kinds */
#define LBDEM_PERIODIC 0 /* periodic pair of faces */
#define LBDEM_WALL 1     /* stationary half-way bounce-back wall half a node outside */
#define LBDEM_PRESSURE 2 /* prescribed density (z faces only): -z follows the waveform, +z keeps rho_f */

/* waveform of the density at the -z face, Eq. (source) and Table 2 (tab:source) */
#define LBDEM_WAVE_NONE 0   /* rho = rho_f */
#define LBDEM_WAVE_SINE 1   /* rho_f + A sin(omega t)        for t <= t_n */
#define LBDEM_WAVE_COSINE 2 /* rho_f + A (1 - cos(omega t))  for t <= t_n */
#define LBDEM_WAVE_STEP 3   /* rho_f + A                     for t <= t_n */

/* storage precision of the populations (collision arithmetic in brackets) */
#define LBDEM_FP64 0    /* double [double] */
#define LBDEM_FP32 1    /* float of f - w_d rho_f [float] */
#define LBDEM_FP16DEV 2 /* IEEE half of q = f/w_d - rho_f [float] */
#define LBDEM_BF16DEV 3 /* bfloat16 of q = f/w_d - rho_f [float] */

#define LBDEM_MAX_PROBES 64

/* status bits returned by lbdem_status */
#define LBDEM_STATUS_NEAR_OVERFLOW 0x2u      /* a particle had more near neighbours than the table holds (error) */
#define LBDEM_STATUS_CHANGE_OVERFLOW 0x4u    /* node-change list spilled; a full map copy was used (results valid) */
#define LBDEM_STATUS_HISTORY_OVERFLOW 0x8u   /* tangential contact history table full (error) */
#define LBDEM_STATUS_TOO_FAST 0x10u          /* a particle moved more than 0.25 lu in one step, its state became
                                                non-finite, or its centre left a bounded axis (error; the particle
                                                is then held to 0.25 lu per step and inside the lattice) */
#define LBDEM_STATUS_SHELL_OVERFLOW 0x40u    /* a particle's surface-shell table overflowed (error) */
#define LBDEM_STATUS_LINK_OVERFLOW 0x80u     /* a fluid node had links to more than four particles (error) */
#define LBDEM_STATUS_LIST_MISS 0x100u        /* compact storage: more than 16384 refills awaited a list rebuild (error) */
#define LBDEM_STATUS_LIST_PARKED 0x200u      /* compact storage: a node turned fluid outside the node lists; its refill
                                                waited for the next step's list rebuild (results valid; a larger
                                                list_margin avoids it) */
#define LBDEM_STATUS_NONFINITE 0x400u        /* watchdog: after a collision a fluid node's density was NaN,
                                                infinite or not positive (error; checked at every node and
                                                step by the fluid kernel) */

/* One lattice and its physics (Sec. 2; Table 1 "tab:params" for the FCC runs). */
typedef struct lbdem_params {
    int32_t nx, ny, nz;      /* lattice size, each >= 1 */
    int32_t face_bc[6];      /* LBDEM_PERIODIC / LBDEM_WALL / LBDEM_PRESSURE per face */
    double tau;              /* BGK relaxation time, > 0.5 (Sec. 2.1) */
    double rho_f;            /* mean fluid density */
    int32_t wave;            /* LBDEM_WAVE_* at the -z face when it is LBDEM_PRESSURE */
    double rho_amp;          /* waveform amplitude rho' */
    double omega;            /* angular frequency, rad per step */
    int64_t t_n;             /* last time level at which the waveform is applied */
    double young_E;          /* contact Young's modulus E_p (Eq. fdLawn) */
    double poisson_nu;       /* contact Poisson ratio nu_p */
    double friction_mu;      /* Coulomb friction coefficient (0: frictionless) */
    double rho_p;            /* particle density; m = rho_p 4/3 pi R^3, I = 2/5 m R^2 */
    int32_t n_probe;         /* number of probe planes (0..LBDEM_MAX_PROBES) */
    int32_t probe_z[LBDEM_MAX_PROBES]; /* z index of each probe plane */
    int32_t max_particles;   /* particle capacity of this lattice (0 .. 8191) */
    double max_radius;       /* largest particle radius this lattice will hold (sizes per-particle tables) */
    int32_t tile_x;          /* fluid-kernel tile x extent for this lattice: 8, 16, 32, 64, or 0 = the
                                set's lbdem_config.tile_x (chosen per lattice by an autotuner) */
    int32_t rest_free;       /* 0 (default): the link force of Eq. (fFS) as printed, on the full
                                populations; 1: without the part of the rest state f_d = w_d rho_f.
                                That part sums to zero over the links of a particle that touches no
                                other; where particles touch, the links their contact hides leave a
                                net push of the rest pressure rho_f c_s^2 over a lattice-sized patch,
                                which option 1 removes (the two agree for separated particles) */
} lbdem_params;

/* Settings shared by all lattices of a set. */
typedef struct lbdem_config {
    int32_t precision;    /* LBDEM_FP64 / LBDEM_FP32 / LBDEM_FP16DEV / LBDEM_BF16DEV */
    int32_t probe_ring;   /* number of most recent steps whose probes are kept (>= 1) */
    int32_t tile_x;       /* x extent of a fluid-kernel tile: 8, 16, 32, 64, or 0 = automatic */
    int32_t z_per_thread; /* z planes per fluid-kernel thread: 1..16, or 0 = automatic */
    int32_t graph_steps;  /* steps per replayed HIP graph: 1..64, or 0 = no graph (eager launches) */
    int32_t node_lists;   /* fluid-kernel mapping: 1 = one thread per listed node (fluid nodes and
                             solid nodes within 0.25 of a particle surface, per z plane, rebuilt
                             when a particle has moved that far); 0 = dense tiles of
                             tile_x * (256 / tile_x) nodes, z_per_thread planes deep; 2 = node
                             lists with compact storage (only listed nodes hold populations,
                             per plane in list order; moved when the lists are rebuilt; needs
                             ny * ceil(nx / 32) <= 8192; a third population buffer); -1 =
                             automatic (0 when max_particles spheres of max_radius could
                             cover at most a quarter of the set's cells; else 2 where every
                             plane fits, else 1 for 16-bit storage and 0 otherwise).  Host
                             access to populations, particle set-up and adjoint windows see
                             the node layout either way. */
    int32_t list_margin;  /* node lists: a lattice's lists are rebuilt once a particle's
                             displacement since the last rebuild plus list_margin times its
                             last step reaches the skin (12 times the lattice's largest last
                             step, within [0.05, 0.25] lu); 0..8, default 2.  Under compact
                             storage a node uncovered outside the lists anyway has its refill
                             kept until the rebuild that follows at the next step. */
    int32_t fluid_off;    /* 1 = hydrodynamics switched off, as for the dry granular chain of
                             Sec. 3.2: a step moves the particles under their contacts and
                             F_g only (no fluid step, no link forces, no conversion momenta);
                             the node map still follows the particles, while populations and
                             probes carry no meaning; 0 (default) = the coupled step. */
    int32_t particle_ring; /* number of most recent steps whose particle velocities are kept for
                              lbdem_particle_signal: 0 (default, none) .. 2^24, 24 bytes per
                              step and particle of the set */
} lbdem_config;

typedef struct lbdem_set lbdem_set;

/* Message of the last failed call on this thread ("" if none). */
const char *lbdem_last_error(void);

/* Fill *cfg with the defaults (FP32, automatic fluid mapping and tiles, 4096-step probe ring,
 * graphs of 8 steps). */
int lbdem_default_config(lbdem_config *cfg);

/* Bytes of device workspace needed by lbdem_create for n_lat lattices.
 * lat: array of n_lat parameter blocks; cfg: may be NULL for the defaults. */
int lbdem_workspace_size(int32_t n_lat, const lbdem_params *lat, const lbdem_config *cfg, size_t *bytes);

/* Create a set of n_lat independent lattices advanced together (a batched ensemble when
 * n_lat > 1).  device_workspace: a device allocation of at least lbdem_workspace_size
 * bytes, aligned to 256 bytes and owned by the caller, who keeps it alive until
 * lbdem_destroy; or NULL, in which case the library allocates (and later frees) it.
 * hip_stream: the hipStream_t to queue work on (NULL = the null stream).
 * The populations start at rest, f_d = w_d rho_f, and the lattices hold no particles.
 * Errors: LBDEM_EINVAL for invalid parameters (tau <= 0.5, a periodic face paired with a
 * non-periodic one, LBDEM_PRESSURE on an x or y face, ...), LBDEM_ENOMEM, LBDEM_EDEVICE. */
int lbdem_create(int32_t n_lat, const lbdem_params *lat, const lbdem_config *cfg, void *device_workspace,
                 size_t workspace_bytes, void *hip_stream, lbdem_set **out);

/* Release the set (waits for its queued work first). */
int lbdem_destroy(lbdem_set *set);

/* Change the stream used for subsequent work. */
int lbdem_set_stream(lbdem_set *set, void *hip_stream);

/* Place n spheres in lattice `lattice` (replacing any previous ones) and project them on
 * the lattice (Sec. 2.3, Fig. mem): a node is solid when d^2 <= R^2 (closed ball); a node
 * inside several spheres belongs to the one with the smallest d^2, then the smallest
 * index.  Host arrays: x, v, w, fg are n x 3 (position, velocity, angular velocity, and a
 * constant external force added in Eq. translate); radius is n; fixed is n (1 = the
 * particle never moves and has V = Omega = 0).  v, w, fg and fixed may be NULL (zeros).
 * Populations are not modified.  Errors: LBDEM_EINVAL when n exceeds max_particles, a
 * radius is not positive or exceeds max_radius, a centre lies outside a non-periodic extent, or a periodic
 * axis is not longer than 2 R + 1.5.  (A node then lies inside at most one image of a
 * sphere, and the midpoint of each link lies less than half a period from the centre of
 * the image its source is in.  On a lattice with a periodic axis shorter than
 * 2 max_radius + 4 a fluid node can border two images of one sphere: its links are grouped
 * per (particle, image), each group with its own torque arm and wall velocity, so such a
 * node can hold at most four groups.) */
int lbdem_particles_set(lbdem_set *set, int32_t lattice, int32_t n, const double *x, const double *v,
                        const double *w, const double *radius, const double *fg, const uint8_t *fixed);

/* Copy the current particle state of lattice `lattice` to host arrays (n x 3 each, any
 * may be NULL): position, velocity, angular velocity, and the hydrodynamic force and
 * torque of the last step, F_f-s and T_f-s of Eqs. (coupleF), (coupleT): the momentum
 * its links exchanged with the fluid in that step plus the conversion impulses applied
 * in it.  n must equal the particle count. */
int lbdem_particles_get(lbdem_set *set, int32_t lattice, int32_t n, double *x, double *v, double *w,
                        double *force, double *torque);

/* Queue nsteps coupled time steps of every lattice of the set (Secs. 2.1-2.4; the paper
 * gives no order, this is the library's).  Each step t -> t+1, one kernel each:
 *   1. the node map of step t takes the previous re-projection's changes, and the link
 *      words of the nodes around them are refreshed;
 *   2. link pass: per particle, the link force of Eq. (fFS) with the bounce-back of
 *      Eq. (mem) substituted, split into its part known from f~(t) and the matrix of its
 *      part linear in the particle's velocities;
 *   3. motion (Eqs. translate, rotate; symplectic Euler, dt = 1): Hertz / Mindlin contacts
 *      (Eqs. fdLawn, fdLaws) at X(t), the external force, the conversion impulses of the
 *      previous re-projection and the link force, the velocities of the step solved
 *      together with the momentum the fluid exchanges in it (implicit in that momentum,
 *      Eqs. coupleF, coupleT); X(t+1) = X(t) + V(t+1);
 *   4. pull streaming (Eq. stream) with stationary walls and half-way bounce-back on the
 *      particle surfaces at X(t) moving with the new velocities (Eq. mem), density faces
 *      (Sec. 2.4), BGK collision (Eqs. bgk, BGKequili, rhoAndU) and probe sums;
 *   5. re-projection at X(t+1) with refill / emptying (Eqs. convertFS, convertSF).
 * Asynchronous; errors found on the device are reported by lbdem_status. */
int lbdem_step(lbdem_set *set, int64_t nsteps);

/* Number of steps taken so far (synchronises). */
int lbdem_time(lbdem_set *set, int64_t *t);

/* Wait for all queued work of the set. */
int lbdem_synchronize(lbdem_set *set);

/* Device status bits (LBDEM_STATUS_*) accumulated since create or the last clear
 * (synchronises).  Returns LBDEM_ENUMERIC when the watchdog bit (NONFINITE) is set, else
 * LBDEM_ECAPACITY when another error bit is set. */
int lbdem_status(lbdem_set *set, uint32_t *bits, int clear);

/* Probe records of steps [first, first + n) of lattice `lattice` into
 * out[n][n_probe][4]: for each probe plane, over its fluid nodes after the collision
 * moments of that step (time level step + 1): node count, sum of rho - rho_f, sum of
 * rho u_z, and sum of rho.  The cross-section averages of the paper (Sec. 3.2 and
 * Sec. 4.3) are sum rho' / count and sum rho u_z / sum rho.  Errors: LBDEM_ERANGE if a
 * step is in the future or older than the probe ring. */
int lbdem_probe_read(lbdem_set *set, int32_t lattice, int64_t first, int64_t n, double *out);

/* Current post-collision populations of lattice `lattice` as double [19][ncell]
 * (decoded from the storage precision).  Values at solid nodes are unspecified. */
int lbdem_populations_get(lbdem_set *set, int32_t lattice, double *f);

/* Overwrite the populations of lattice `lattice` (encoded to the storage precision). */
int lbdem_populations_set(lbdem_set *set, int32_t lattice, const double *f);

/* Node map of lattice `lattice`: -1 for fluid, else the index of the covering particle. */
int lbdem_owner_get(lbdem_set *set, int32_t lattice, int32_t *owner);

/* Macroscopic fields of lattice `lattice` at the current time level, computed on the
 * device from the post-collision populations in FP64 (Eq. rhoAndU: rho = sum_d f_d, rho u
 * = sum_d f_d c_d; the collision keeps both, so they are also the moments the step's
 * collision used): rho [ncell], u [3][ncell] (component-major), owner [ncell] as for
 * lbdem_owner_get.  At solid nodes rho and u are 0.  Any output may be NULL.  Host arrays;
 * synchronises.  Errors: LBDEM_EINVAL, LBDEM_ENOMEM (device scratch), LBDEM_EDEVICE. */
int lbdem_fields_get(lbdem_set *set, int32_t lattice, double *rho, double *u, int32_t *owner);

/* ---- Checkpoint and resume ----
 * A checkpoint holds the whole state of a set at a step boundary: populations, node maps
 * and link words, particle state (positions, velocities, forces, pending conversion
 * impulses, contact histories), the library's particle and node lists, the probe ring,
 * the step counter and the status bits.  Stepping a set restored from a checkpoint taken
 * after k steps for m more steps gives bit for bit the state of k + m steps.  A
 * checkpoint loads only into a set created with the same parameters and configuration
 * (graph_steps aside) by the same library build; no adjoint window may be bound to the
 * set.  buf is caller-owned host memory. */

/* Bytes of a checkpoint of the set. */
int lbdem_state_size(lbdem_set *set, size_t *bytes);

/* Write a checkpoint into buf (cap bytes; *used receives its size).  Synchronises.
 * Errors: LBDEM_EINVAL (null argument), LBDEM_ENOMEM (cap too small), LBDEM_EDEVICE. */
int lbdem_state_save(lbdem_set *set, void *buf, size_t cap, size_t *used);

/* Restore the set from a checkpoint of `size` bytes.  Synchronises.  Errors: LBDEM_EINVAL
 * (not a checkpoint of a set with these parameters), LBDEM_EDEVICE. */
int lbdem_state_load(lbdem_set *set, const void *buf, size_t size);

/* Kernel timing with HIP events on the set's stream.  While enabled, lbdem_step launches
 * kernels one by one and brackets every launch with a pair of events.  lbdem_timing_read
 * synchronises and returns, for kernel k = 0 (links), 1 (particle motion), 2 (fluid),
 * 3 (re-projection), 4 (start-of-step node-map refresh), the summed milliseconds ms[k] and
 * the number of launches count[k] since enabling (ms and count hold 5 entries). */
int lbdem_timing_enable(lbdem_set *set, int enable);
int lbdem_timing_read(lbdem_set *set, double *ms, int64_t *count);

/* Tile geometry actually used for lattice `lattice`: tile_x, tile_y, z_per_thread. */
int lbdem_tile_info(lbdem_set *set, int32_t lattice, int32_t *tile_x, int32_t *tile_y, int32_t *z_per_thread);

/* ---- Adjoint of the fluid step over frozen particle geometry ----------------------------
 * An adjoint window binds to one lattice of a set and freezes its current geometry: node
 * map, particle positions, angular velocities and radii.  Its forward map is nsteps fluid
 * steps from the lattice's current populations: pull streaming with stationary walls and
 * the moving walls of Eq. (mem) (particle velocities V chosen per forward), the density
 * faces (Sec. 2.4) with rho_in = rho_f + A s(t+1) for the lattice's waveform s of unit
 * amplitude (Eq. source), and the BGK collision with relaxation time tau (Eqs. bgk,
 * BGKequili, rhoAndU).  The probe signal of step n is the plane average of rho - rho_f
 * over the fluid nodes of each probe plane, from the pre-collision moments of time level
 * t0+n+1.  lbdem_adj_backward returns the vector-Jacobian product of that map: for a loss
 * gradient dL/dP it propagates the discrete adjoint backwards through the window,
 * recomputing the forward states segment by segment from checkpoints taken every
 * ckpt_every steps, and returns dL/dtau, dL/dA and dL/dV.  Gradient sums are FP64; the
 * adjoint fields use the set's arithmetic precision (FP64 or FP32).
 * The set must not be stepped or given new particles while a window is bound to it. */
typedef struct lbdem_adj lbdem_adj;

/* Device bytes for a window of nsteps (>= 1) with a checkpoint every ckpt_every (>= 1)
 * steps: populations for the checkpoints and one segment, three adjoint fields, 18 FP64
 * values per node for the particle-velocity gradient, and small tables. */
int lbdem_adj_workspace_size(lbdem_set *set, int32_t lattice, int64_t nsteps, int32_t ckpt_every, size_t *bytes);

/* Bind a window to lattice `lattice` of `set` (synchronises the set's stream).  workspace:
 * caller-owned device memory of at least lbdem_adj_workspace_size bytes, 256-byte aligned,
 * kept alive until lbdem_adj_destroy.  Errors: LBDEM_EINVAL, LBDEM_ENOMEM (workspace too
 * small), LBDEM_EDEVICE. */
int lbdem_adj_create(lbdem_set *set, int32_t lattice, int64_t nsteps, int32_t ckpt_every, void *workspace,
                     size_t workspace_bytes, lbdem_adj **out);

/* Run the window's forward map with relaxation time tau (> 1/2), waveform amplitude amp and
 * particle velocities v (n x 3, the lattice's particle order; NULL = the velocities held
 * when the window was created).  probes (NULL allowed): [nsteps][n_probe] signals.
 * Synchronous.  The set's own populations are not modified. */
int lbdem_adj_forward(lbdem_adj *adj, double tau, double amp, const double *v, double *probes);

/* Vector-Jacobian product of the last forward: dL_dP [nsteps][n_probe] in, dL/dtau,
 * dL/dA and dL/dV (n x 3) out (any output may be NULL).  Synchronous.  LBDEM_ESTATE if no
 * forward has run. */
int lbdem_adj_backward(lbdem_adj *adj, const double *dL_dP, double *dL_dtau, double *dL_damp, double *dL_dv);

/* Release the window (its workspace stays with the caller). */
int lbdem_adj_destroy(lbdem_adj *adj);

/* ---- Dispersion analysis of probe records (Sec. 3.2) ----
 * The cross-section averaged density signal rho'(t, x3) of a wave experiment is analysed in
 * two ways: its discrete Fourier transform over space and time, whose ridge gives the
 * dispersion relation and, at the inserted frequency, the sound speed c_s = omega / k; and a
 * fit of the stationary solution of the one-dimensional lossy wave equation, Eq. (1Dwave),
 * rho' = A exp(-alpha_s x) exp(j (omega t - k x)), which gives A, alpha_s and c_s = omega / k.
 * All arrays of these calls are device memory (FP64, row-major), the calls are asynchronous
 * on `stream` (a hipStream_t; NULL is the null stream) and the caller owns every buffer.
 * Errors: LBDEM_EINVAL for a null pointer or a size out of range, LBDEM_ENOMEM for a
 * workspace smaller than the size query returns, LBDEM_EDEVICE for a launch failure. */

/* Cross-section averages of lattice `lattice` for steps [first, first + n), gathered on the
 * device from the probe ring on the set's stream into x[n][n_probe] (n * n_probe doubles):
 * quantity 0 gives the averaged density signal (sum of rho - rho_f) / (node count) of each
 * probe plane (Sec. 3.2), quantity 1 the averaged momentum sum(rho u_z) / sum(rho)
 * (Sec. 4.1); a plane without fluid nodes gives 0.  The values are those of the records
 * lbdem_probe_read returns; the record of step s is taken at time level s + 1.
 * Errors: LBDEM_EINVAL for another quantity, LBDEM_ERANGE as for lbdem_probe_read. */
int lbdem_probe_signal(lbdem_set *set, int32_t lattice, int64_t first, int64_t n, int32_t quantity, double *x);

/* Particle-velocity signal of lattice `lattice` for steps [first, first + n), gathered on
 * the device from the particle-velocity ring (lbdem_config.particle_ring) on the set's
 * stream into x[n][n_layers] (device memory): for each step, the average of velocity
 * component `component` (0, 1, 2 = x, y, z) over the particles of each layer; the record of
 * step s is the velocity at time level s + 1, the one a particle moves with from X(s) to
 * X(s + 1) (the dispersion relations of the solid phase are read from the space-time DFT
 * of such signals, Sec. 4.3).  layer: host array [the lattice's particle count], the layer
 * of each particle (0 .. n_layers - 1) or -1 to leave it out; a layer without particles
 * gives 0.  Each layer is summed in particle index order.  The call returns when x is
 * written.  Errors: LBDEM_EINVAL for bad arguments, LBDEM_ERANGE for steps not held (the
 * ring keeps the last particle_ring steps since the lattice's particles were last set),
 * LBDEM_ENOMEM, LBDEM_EDEVICE. */
int lbdem_particle_signal(lbdem_set *set, int32_t lattice, int64_t first, int64_t n, const int32_t *layer,
                          int32_t n_layers, int32_t component, double *x);

/* Biot's wave velocities of a saturated poroelastic packing (Sec. "Biot's equations of wave
 * velocities in saturated poroelastic media", Eqs. vp, vs), for comparison with the
 * simulated ones: from the dry packing's bulk and shear moduli k_dry, g_dry (not given by
 * the paper, an input), the porosity phi (0 < phi < 1), the bulk moduli of the particles
 * and the fluid k_p, k_f (k_p = E_p / (3 (1 - 2 nu_p)), k_f = rho_f c_s^2) and their
 * densities, with the tortuosity alpha = 1 - r (1 - 1/phi) (r = 0.5 for spheres).  The
 * denominator of Eq. (vp) is read as 2 (rho11 rho22 - rho12^2).  out[3] (host): fast P-wave,
 * slow P-wave and S-wave speeds.  Host computation.  Errors: LBDEM_EINVAL for a null
 * output or inputs that give no real speeds. */
int lbdem_biot_velocities(double k_dry, double g_dry, double phi, double k_p, double k_f, double rho_p,
                          double rho_f, double r, double *out);

/* Device workspace bytes for lbdem_st_dft and lbdem_wave_fit with these sizes. */
int lbdem_dft_workspace_size(int64_t nt, int32_t nz, int32_t nw, int32_t nk, size_t *bytes);

/* Space-time DFT: F[m][n] = sum_t sum_z x[t][z] exp(-j (omega_m (t0 + t) - kappa_n zpos[z]))
 * for omega_m = w0 + m dw (m < nw) and kappa_n = k0 + n dk (n < nk); the sign pair of
 * Eq. (1Dwave), so a wave running towards +x3 peaks at omega > 0, kappa > 0.
 * x: [nt][nz] signal, row t taken at time t0 + t; zpos: [nz] positions of the columns along
 * x3; F: [nw][nk][2] (real, imaginary).  ridge (NULL allowed): [nw] int32, for each row m the
 * index n of the largest |F|^2 = re^2 + im^2, the smallest index among equal values (-1
 * for a row of NaN).  work: device workspace of at least lbdem_dft_workspace_size(nt, nz,
 * nw, nk) bytes, 256-byte aligned.  Limits: 1 <= nt <= 2^31, 1 <= nz <= 65536,
 * 1 <= nw, nk <= 2^20, and each of nw nz, nz nk, nw nk at most 2^28. */
int lbdem_st_dft(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double w0, double dw,
                 int32_t nw, double k0, double dk, int32_t nk, double *F, int32_t *ridge, void *work,
                 size_t work_bytes, void *stream);

/* Fit of Eq. (1Dwave) at the inserted frequency omega (!= 0): at every column z the complex
 * amplitude P[z] = (2 / nt) sum_t x[t][z] exp(-j omega (t0 + t)) (exact for a stationary
 * wave sampled over whole periods), then least-squares straight lines through log |P[z]| and
 * through the phase of P[z] unwrapped along the columns (steps larger than pi taken modulo
 * 2 pi), against zpos: slopes -alpha_s and -k, intercepts log |A| and arg A.
 * out: [6] = A real, A imaginary, alpha_s, k, c_s = omega / k, and the number of columns
 * used.  Columns with P[z] = 0 are left out; fewer than two left gives NaN fits.
 * work: at least lbdem_dft_workspace_size(nt, nz, 1, 1) bytes.  Limits as for lbdem_st_dft. */
int lbdem_wave_fit(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double omega,
                   double *out, void *work, size_t work_bytes, void *stream);

/* lbdem_wave_fit without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments and results as lbdem_wave_fit; the fit's scratch is a static device array
 * of 4 MiB per GPU, held until the process ends (its address is looked up on the first
 * call on each device).  Calls on one GPU share that array: calls that overlap on one GPU
 * race and must be ordered by the caller.  Allocates no memory.  Errors: as for
 * lbdem_wave_fit, and LBDEM_ENOMEM when the sizes need more than the static scratch. */
int lbdem_wave_fit_noalloc(const double *x, int64_t nt, int32_t nz, const double *zpos, double t0, double omega,
                           double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LBDEM_H */

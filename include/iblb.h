/*
 * iblb.h -- C ABI of the MI355X (gfx950) immersed-boundary lattice Boltzmann
 * wetting solver.
 *
 * The model is the hybrid IB-LB method of "Immersed boundary - lattice
 * Boltzmann method for wetting problems":
 *   - fluid: lattice Boltzmann equation (eq. LBE) with the BGK collision, the
 *     second-order equilibrium and Guo's source term; density and
 *     half-force velocity from eqs. (hydro_var1)-(hydro_var2); D3Q19 velocity
 *     set of Table I, or its 2D analogue D2Q9 (w = 4/9, 1/9, 1/36);
 *   - coupling: nodal forces spread to the lattice (eq. force_spread), lattice
 *     velocity interpolated to the nodes (eq. vel_interpolation) with the
 *     Peskin 4-point kernel, nodes advanced by forward Euler;
 *   - interface forces: surface tension from the strain energy w = sigma e^a
 *     (Sec. "Modelling surface tension forces"), evaluated as minus sigma
 *     times the gradient of the interface area (perimeter in 2D), plus the
 *     wetting force -(chi_j/3) Pi(h_j) n_j of Sec. "Modelling wetting
 *     properties" with Pi(h) of eq. (disjoin-p) and A of eq. (A_choice);
 *   - boundaries: periodic sides, half-way bounce-back walls (Sec.
 *     "Numerical results", set-up paragraph).
 *
 * Conventions
 *   - Lattice units, dx = dt = 1.  Cell (i, j, k) is centred at
 *     (i + 1/2, j + 1/2, k + 1/2).  A wall axis has walls at coordinate 0
 *     and n; the substrate is the wall at 0 of the last axis (y in 2D, z in
 *     3D), so a node's height above it is its last coordinate.
 *   - Velocity order: rest, then opposite pairs adjacent
 *       D2Q9 : 0 | +x -x | +y -y | (+1,+1) (-1,-1) | (-1,+1) (+1,-1)
 *       D3Q19: 0 | +x -x | +y -y | +z -z | (1,1,0) (-1,-1,0) | (1,-1,0)
 *              (-1,1,0) | (1,0,1) (-1,0,-1) | (1,0,-1) (-1,0,1) | (0,1,1)
 *              (0,-1,-1) | (0,1,-1) (0,-1,1)
 *   - Cell arrays are [component][z][y][x], x fastest.  Node arrays are
 *     structure-of-arrays [component][node].
 *   - A population is exchanged as its deviation from its weight, f_i - w_i.
 *
 * Memory and streams
 *   - The caller owns all device memory.  iblb_workspace_bytes() gives the
 *     size of one device buffer that the caller allocates and hands to
 *     iblb_create(); the library carves every device array from it and
 *     allocates no device memory of its own.  Host memory for the handle
 *     and a private capture stream are created in iblb_create().
 *   - Every call is ordered on the stream given to iblb_create() (a
 *     hipStream_t passed as void*; NULL is the default stream).  Calls that
 *     return host data synchronise that stream.
 *   - A handle is not thread-safe; any number of handles may coexist.
 *
 * Errors
 *   Every call returns an iblb_status.  Nothing throws across the ABI.
 *   iblb_last_error() gives a message for the handle's last failure.
 */
#ifndef IBLB_H
#define IBLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IBLB_OK = 0,
    IBLB_EINVAL = -1,     /* bad argument: see iblb_last_error()            */
    IBLB_ENOMEM = -2,     /* workspace smaller than iblb_workspace_bytes()  */
    IBLB_EDEVICE = -3,    /* a HIP runtime call failed                      */
    IBLB_EUNSTABLE = -4,  /* a node reached h <= 0 with wetting on, a node
                             speed became non-finite or above 0.3, or a node
                             position became non-finite (such nodes are
                             then left out of spreading and interpolation) */
    IBLB_ELIMIT = -5      /* a limit of the inside/outside classification
                             was exceeded: more than 16 interface crossings
                             on one lattice row (the extra crossings are
                             dropped), or a node outside the classification
                             window along a periodic axis                  */
} iblb_status;

typedef enum { IBLB_PERIODIC = 0, IBLB_WALL = 1 } iblb_bc;

/* Storage format of the populations.  Arithmetic is fp32 in every case.
 * The shifted formats store the deviation f_i - w_i rounded to nearest even
 * (fp32, fp16 or bf16), which keeps the small deviations from the rest
 * state at full relative precision. */
typedef enum { IBLB_F32 = 0, IBLB_F16 = 1, IBLB_BF16 = 2 } iblb_storage;

/* Parameters of one droplet simulation (one fluid box + one interface). */
typedef struct {
    int dim;            /* 2 (D2Q9) or 3 (D3Q19)                              */
    int nx, ny, nz;     /* lattice size; nz = 1 in 2D; each >= 1              */
    int bc[3];          /* iblb_bc per axis                                   */
    double tau;         /* BGK relaxation time, > 1/2; INFINITY gives pure
                           streaming (no relaxation, no force)               */
    double sigma;       /* surface tension                                    */
    double theta_eq;    /* equilibrium contact angle in radians               */
    double xi;          /* regularising length of Pi(h), > 0                  */
    int n_exp, m_exp;   /* exponents of Pi(h), n > m (the paper uses 6, 3)    */
    int wetting;        /* 1: Pi(h) acts from the substrate; 0: free droplet  */
} iblb_params;

/* FP64 diagnostics of one droplet after the last completed step. */
typedef struct {
    int64_t step;             /* steps completed                              */
    double mass;              /* sum over cells of rho                        */
    double momentum[3];       /* sum over cells of rho U (last step)          */
    double sum_phi[3];        /* sum of nodal forces (last step)              */
    double sum_F[3];          /* sum of the spread force density (last step)  */
    double dropped_F[3];      /* nodal force falling on wall taps (not spread)*/
    double volume;            /* enclosed area (2D) or volume (3D)            */
    double area;              /* perimeter (2D) or surface area (3D)          */
    double contact_radius;    /* protocol (i): crossing of the interface with
                                 the plane at z_cut = xi (n/m)^(1/(n-m))      */
    double height;            /* max minus min node height                   */
    double theta_meas;        /* angle from the half-height (eq. angleh; 2D:
                                 the circular-cap counterpart), radians       */
    double max_normal_speed;  /* max over nodes of |qdot . n|                 */
    double max_speed;         /* max over nodes of |qdot|                     */
    double min_h;             /* lowest node height                           */
    double edge_min, edge_max;/* shortest / longest mesh edge                 */
    int32_t status;           /* iblb_status of the droplet                   */
} iblb_diag;

typedef struct iblb_ctx iblb_ctx;

/* Size in bytes of the device workspace for n_droplets droplets with the
 * given parameters, node counts and triangle counts (n_tris may be NULL in
 * 2D, where the interface is a closed polygon).  Returns 0 on bad input,
 * with the reason in iblb_last_error(NULL).  Host only: touches no device. */
size_t iblb_workspace_bytes(int n_droplets, const iblb_params *params,
                            const int *n_nodes, const int *n_tris, int storage);

/* Create a handle for n_droplets independent droplets that are stepped
 * together (one launch per kernel for the whole batch).  All droplets share
 * dim and storage.  d_workspace: caller-owned device buffer of ws_bytes >=
 * iblb_workspace_bytes(...).  stream: hipStream_t or NULL.  On success the
 * populations are at rest (f = w) and every node sits at the origin until
 * iblb_set_interface() is called.  *out receives the handle (NULL on error). */
int iblb_create(int n_droplets, const iblb_params *params, const int *n_nodes,
                const int *n_tris, int storage, void *d_workspace, size_t ws_bytes,
                void *stream, iblb_ctx **out);

int iblb_destroy(iblb_ctx *ctx);

/* Message for the handle's last failure ("" if none).  Valid until the next
 * call on the handle.  ctx may be NULL for failures of iblb_create() and
 * iblb_workspace_bytes() (kept per calling thread). */
const char *iblb_last_error(const iblb_ctx *ctx);

/* Upload droplet d's interface: h_pos [dim][N] node positions (host,
 * float64, N as given to iblb_create).  2D: the nodes form a closed polygon
 * in the given order, counter-clockwise.  3D: h_tris [T][3] vertex indices
 * (host, int32), counter-clockwise seen from outside; every vertex must
 * belong to at least one triangle.  Copies are made; EINVAL on a bad index. */
int iblb_set_interface(iblb_ctx *ctx, int droplet, const double *h_pos,
                       const int32_t *h_tris);

/* Reset droplet d (or every droplet for d = -1) to rest: f_i = w_i. */
int iblb_init_rest(iblb_ctx *ctx, int droplet);

/* Initialise droplet d's populations to the equilibrium (eq. f^eq of Sec.
 * IB-LB, second order in U) of a density field d_rho [nz][ny][nx] (device
 * float32; NULL: rho = 1 everywhere) and a velocity field d_u
 * [dim][nz][ny][nx] (device float32; NULL: at rest).  Clears the droplet's
 * force and velocity fields first.  The arrays are read by a kernel queued
 * on the handle's stream: keep them alive until that stream has passed it. */
int iblb_init_fields(iblb_ctx *ctx, int droplet, const float *d_rho, const float *d_u);

/* Overwrite / read droplet d's post-collision populations, exchanged as
 * deviations f_i - w_i in a device float64 array [Q][nz][ny][nx].  Writing
 * narrows through fp32 to the storage format, nearest even at each step. */
int iblb_write_populations(iblb_ctx *ctx, int droplet, const double *d_fdev);
int iblb_read_populations(iblb_ctx *ctx, int droplet, double *d_fdev);

/* Replace droplet d's immersed boundary by a prescribed, constant force
 * density d_F [dim][nz][ny][nx] (device float32, copied), or give back the
 * immersed boundary with d_F = NULL.  Used for closed-form flows. */
int iblb_set_force_field(iblb_ctx *ctx, int droplet, const float *d_F);

/* Advance every droplet by n_steps time steps.  Each step: nodal forces at
 * q(t) (surface tension, Sec. "Modelling surface tension forces"; wetting,
 * eq. disjoin-p with A of eq. A_choice) -> spread to F(t) (eq.
 * force_spread, Peskin kernel Psi) -> fused pull-stream + collide with F(t)
 * (eq. LBE with Guo's source; moments of eqs. hydro_var1/hydro_var2) ->
 * velocity U(t) interpolated at q(t) (eq. vel_interpolation) -> forward
 * Euler q(t+1) = q(t) + qdot(t).  Asynchronous except
 * for a final status check (synchronises the stream, reads one int per
 * droplet).  Long runs replay a captured graph of a fixed number of steps.
 * The last step of every call also stores rho, U and F of every cell for
 * iblb_read_fields(). */
int iblb_step(iblb_ctx *ctx, int n_steps);

/* Copy the last step's fields of droplet d into device float32 arrays:
 * d_rho [nz][ny][nx], d_u [dim][nz][ny][nx], d_F [dim][nz][ny][nx]; any of
 * them may be NULL.  Before the first step, rho = 1 and U = F = 0. */
int iblb_read_fields(iblb_ctx *ctx, int droplet, float *d_rho, float *d_u, float *d_F);

/* Copy droplet d's nodes to host arrays [dim][N]: positions q(t+1)
 * (float64), velocities qdot(t) and nodal forces phi(t) (float32) of the
 * last step; any pointer may be NULL.  Synchronises the stream. */
int iblb_read_nodes(iblb_ctx *ctx, int droplet, double *h_pos, float *h_vel, float *h_force);

/* FP64 diagnostics of droplet d into *out (host), or of every droplet into
 * out[0..n_droplets-1] for d = -1.  Reads all populations once.
 * Synchronises. */
int iblb_diagnostics(iblb_ctx *ctx, int droplet, iblb_diag *out);

/* Run every active droplet that has an interface until it comes to rest:
 * every check_every steps the largest normal node speed |qdot . n| of each
 * such droplet is compared with tol and, with angle_tol > 0, its angle from
 * the half-height (eq. angleh; 2D: the circular-cap counterpart) with the
 * angles of the hold checks before.  A droplet below tol for `hold`
 * consecutive checks, whose angle moved by less than angle_tol (radians)
 * over those checks, is frozen (iblb_set_active(ctx, d, 0)) and
 * steps_out[d] receives the number of steps it took.  A droplet that turns
 * unstable is frozen with steps_out[d] = -2; one still moving after
 * max_steps keeps -1; droplets without interface or frozen on entry get 0.
 * steps_out: host array of n_droplets entries.  Returns when every tracked
 * droplet is frozen or after max_steps steps.  (The paper defines no rest
 * criterion; the speed alone, angle_tol = 0, can sit above a small tol for
 * a long time through parasitic currents, while the angle window asks for
 * the shape itself to have stopped changing.) */
int iblb_run_to_rest(iblb_ctx *ctx, double tol, double angle_tol, int check_every, int hold,
                     long long max_steps, long long *steps_out);

/* Variant of the lattice kernel (all compute the same result):
 *   0: 256x1 cells per block   3: 256x1, non-temporal stores
 *   1: 128x2 cells per block   4: 128x2, non-temporal stores
 *   2:  64x4 cells per block   5:  64x4, non-temporal stores
 *   6-11: as 0-5 with non-temporal population loads
 *   12-15: 256 consecutive cells per block in storage order (no idle lanes
 *          when nx is not a multiple of 64): plain, non-temporal stores,
 *          non-temporal loads, both
 *   16-31: as variant - 16 with the blocks in storage order of their tiles
 *          (0-15 give each of the device's eight XCDs one contiguous run of
 *          tiles)
 * variant = -1 keeps the current one; *variant_out (may be NULL) receives
 * the variant in use; other values: IBLB_EINVAL. */
int iblb_set_lb_variant(iblb_ctx *ctx, int variant, int *variant_out);

/* Time every lattice-kernel variant on the handle's own coupled steps and
 * keep the fastest (the lowest-numbered variant within 2% of the fastest,
 * so that near-ties resolve the same way from run to run).  Each variant
 * runs iblb_step(steps) twice: the first call builds its graphs, the second
 * is timed between two events on the handle's stream (graphs are replayed
 * only when steps >= graph steps + 2, as in any iblb_step call).  All these
 * steps advance the simulation.  With cache_path non-NULL the winner is
 * looked up in / appended to that text file, keyed by device, lattice,
 * storage and size bucket; a cache hit runs no step.  chosen (may be NULL)
 * receives the variant; ms (may be NULL, 32 entries) the measured
 * milliseconds per coupled step of each variant (-1 on a cache hit). */
int iblb_autotune(iblb_ctx *ctx, int steps, const char *cache_path, int *chosen, double *ms);

/* Number of steps captured in one replayed graph (even, 2..1024); default
 * 64.  0 disables graphs (every step launched directly). */
int iblb_set_graph_steps(iblb_ctx *ctx, int steps);

/* Mark droplet d active (1) or frozen (0).  Frozen droplets are skipped by
 * every kernel until re-activated; their state is kept. */
int iblb_set_active(iblb_ctx *ctx, int droplet, int active);

/* Viscosity ratio lambda = mu_in / mu_out of droplet d (Sec. "Immersed-
 * boundary lattice Boltzmann (IB-LB) method", last paragraph; eq.
 * def_lambda).  With mu = rho cs^2 (tau - 1/2) on both sides, the cells
 * enclosed by the interface relax with tau_in = 1/2 + lambda (tau - 1/2)
 * (in the BGK term and the Guo prefactor) and the others with the droplet's
 * tau.  Every step first classifies the cells at the node positions of
 * that step: a ray along +x through each lattice row counts the
 * interface's crossings beyond the cell centre (odd: inside).  Along a
 * periodic axis the interface is not wrapped; cell centres are taken at
 * their periodic image in the window [r - n/2, r + n/2) around the mean r
 * of the node positions given to the last iblb_set_interface(), which is
 * exact while every node stays inside that window.  lambda = 1 (the
 * default) turns the classification off.  lambda must be positive and
 * finite, tau finite, and the droplet must have an interface (EINVAL
 * otherwise).  More than 16 crossings on one row, or a node outside the
 * window, fail the step with IBLB_ELIMIT.  Synchronises the stream. */
int iblb_set_viscosity_ratio(iblb_ctx *ctx, int droplet, double lambda);

/* Elastic interface for droplet d (3D): the strain energy of eq. force_bb
 * becomes w(a, b) = sigma e^a + mu_s (b + 1 - e^a), with a, b the strain
 * invariants of eq. strain_inv measured from the node positions at the time
 * of this call (the stress-free reference mesh), instead of eq.
 * energy_drop; mu_s (>= 0) is the surface shear modulus: the added energy
 * is mu_s A0 (l1 - l2)^2 / 2 per triangle, l1, l2 its principal stretches
 * and A0 its reference area (Sec. "Modelling surface tension forces"; the
 * change of strain energy the paper's conclusions propose for elastic
 * wetting).  mu_s = 0 restores the liquid droplet.  EINVAL in 2D, without
 * an interface, or for a negative or non-finite mu_s.  Synchronises. */
int iblb_set_membrane_shear(iblb_ctx *ctx, int droplet, double mu_s);

/* Tangential re-spacing of droplet d's outline (2D), an addition to the
 * method for long runs rather than a passage of the paper: the outline's
 * nodes move with the interpolated fluid velocity only (eq.
 * vel_interpolation), and a line tension has no tangential stiffness, so
 * over 10^5 steps and more they drift along the outline and open gaps of
 * many lattice units at the contact corners, through which the interface
 * leaks.  With beta > 0, each step adds to node j's advected position
 *   (beta / 2) (|q_{j+1} - q_j| - |q_j - q_{j-1}|) c / |c|,
 * c = q_{j+1} - q_{j-1}, all at the positions before the advection: a move
 * along the outline that leaves uniformly spaced nodes where they are and
 * evens out uneven spacing.  q_dot (iblb_read_nodes, the rest criterion of
 * iblb_run_to_rest) stays the fluid velocity.  0 <= beta < 1 (0: off, the
 * default).  EINVAL in 3D, without an interface, or for beta outside that
 * range.  Synchronises. */
int iblb_set_node_respacing(iblb_ctx *ctx, int droplet, double beta);

/* Inside/outside classification of droplet d's cells at its current node
 * positions (the rule of iblb_set_viscosity_ratio, for any lambda):
 * d_mask (device, uint8, ncell = nx*ny*nz, [z][y][x]) receives 1 for cells
 * enclosed by the interface and 0 for the others.  The droplet must have
 * an interface.  IBLB_ELIMIT if a row has more than 16 crossings or a node
 * lies outside the window, IBLB_EUNSTABLE for a non-finite node.
 * Synchronises the stream. */
int iblb_inside_mask(iblb_ctx *ctx, int droplet, uint8_t *d_mask);

/* Contact radius of droplet d at its current node positions by the two
 * protocols of Sec. "Dynamics" (the flat base of the interface stands for
 * the contact area).  h is the last coordinate (height above the substrate).
 *   out[0]  protocol (i): the interface cut by the plane h = z_cut; 3D: the
 *           mean distance of the points where mesh edges cross the plane to
 *           their centre; 2D: half the distance between the outermost
 *           crossings of the line.  NaN when the plane does not cut it.
 *   out[1]  protocol (ii): the elements (3D triangles, 2D edges) whose nodes
 *           all lie below the mid-height between the lowest and the highest
 *           node and differ in height by less than flat_tol (eps R0 in the
 *           paper's notation) form the flat region; 3D: radius of the disc
 *           of its area, 2D: half its length.
 *   out[2]  number of crossings found by protocol (i).
 * out: host, 3 doubles.  EINVAL without an interface, for a non-finite
 * z_cut or a negative flat_tol.  Synchronises the stream. */
int iblb_contact_radius(iblb_ctx *ctx, int droplet, double z_cut, double flat_tol, double *out);

/* With timing on (on = n > 0), iblb_step() launches every step directly
 * (no graph replay) and launches every n-th lattice kernel of a call, the
 * first included, with a pair of HIP events that its own dispatch marks at
 * the kernel's start and end (the interval a kernel-trace profiler reports
 * for that dispatch); the stream is synchronised every 256 timed launches
 * to read them.  on = 0 turns timing off; a negative on is EINVAL.
 * iblb_last_timing() gives the average of those intervals and the average
 * time of a whole step (milliseconds, events around the call) over the last
 * such call; the call's final, field-storing step is left out of the kernel
 * average.  Either output pointer may be NULL. */
int iblb_set_timing(iblb_ctx *ctx, int on);
int iblb_last_timing(const iblb_ctx *ctx, double *lb_ms_per_step, double *step_ms_per_step);

/* Measurement aid: replay a graph of `launches` (even, 2..1024) lattice
 * launches back to back, no node work between them, once to warm up and
 * once between two events on the handle's stream; *ms_per_launch receives
 * the timed replay's elapsed time divided by `launches` (per-launch time
 * including dispatch, the quantity a kernel-trace profiler reports).  The
 * populations advance by 2 * launches force-free lattice steps and the
 * nodes stay where they are, so the handle no longer holds a coupled
 * solution afterwards.  Droplets with two viscosities keep the inside/
 * outside classification of their current node positions for every
 * launch. */
int iblb_time_lattice(iblb_ctx *ctx, int launches, double *ms_per_launch);

/* Measurement aid: copy `bytes` (a multiple of 16) from d_src to d_dst on
 * the device, reps + 1 times; *gbs receives the mean of the last reps
 * copies in GB/s counting read + write bytes (attainable HBM bandwidth when
 * the buffers are much larger than the caches). */
int iblb_probe_copy(void *d_dst, const void *d_src, size_t bytes, int reps, void *stream,
                    double *gbs);

/* ------------------------------------------------------------------------
 * Warm-start network (learned initial state; not part of the paper's
 * method): a fully connected network widths[0] -> widths[1] -> ... ->
 * widths[n_layers], GELU (exact, erf form) after every layer except the last.
 * Products run on the matrix cores with bf16 operands (weights and
 * activations rounded to nearest even) and fp32 accumulation; the weights
 * are kept in fp32 (master copy) and trained with Adam on the mean squared
 * error.  Parameters are packed per layer l: W_l [widths[l]][widths[l+1]]
 * row-major (y = x W + b), then b_l [widths[l+1]].  All device memory comes
 * from the caller's workspace; every call is ordered on the given stream.
 * ------------------------------------------------------------------------ */
typedef struct iblb_mlp iblb_mlp;

size_t iblb_mlp_workspace_bytes(int n_layers, const int *widths, int max_batch);
int iblb_mlp_create(int n_layers, const int *widths, int max_batch, void *d_workspace,
                    size_t ws_bytes, void *stream, iblb_mlp **out);
int iblb_mlp_destroy(iblb_mlp *mlp);
const char *iblb_mlp_last_error(const iblb_mlp *mlp);
long long iblb_mlp_param_count(const iblb_mlp *mlp);

/* Host fp32 packed parameters in / out.  Setting resets the Adam state. */
int iblb_mlp_set_params(iblb_mlp *mlp, const float *h_params);
int iblb_mlp_get_params(iblb_mlp *mlp, float *h_params);

/* d_x [batch][widths[0]] -> d_y [batch][widths[n_layers]], device fp32,
 * 1 <= batch <= max_batch. */
int iblb_mlp_forward(iblb_mlp *mlp, const float *d_x, int batch, float *d_y);

/* Forward + backward of the mean squared error against d_t [batch][out]
 * (device fp32).  *loss (host, may be NULL) receives the loss; h_grads
 * (host, may be NULL, param_count floats) the packed gradient.  The
 * gradient is kept for iblb_mlp_adam_step.  Synchronises when loss or
 * h_grads is requested. */
int iblb_mlp_gradients(iblb_mlp *mlp, const float *d_x, const float *d_t, int batch,
                       float *h_grads, double *loss);

/* One Adam step (bias-corrected) with the gradient of the last
 * iblb_mlp_gradients call. */
int iblb_mlp_adam_step(iblb_mlp *mlp, float lr, float beta1, float beta2, float eps);

/* Forward pass that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): the
 * same result as iblb_mlp_forward (same kernels, bit for bit), but the
 * bf16 input and the hidden layers' activations live in a static device
 * array of 8 MiB in the library instead of the handle's workspace, and the
 * last layer writes d_y directly.  d_x [batch][widths[0]] -> d_y
 * [batch][widths[n_layers]], device fp32; batch >= 1 and not limited by
 * max_batch, but the batch's scratch (2 batch widths[0] bytes plus
 * 8 batch h bytes, h the widest hidden layer, each part rounded up to 256)
 * must fit the 8 MiB, else EINVAL with the sizes in the message.  Queued
 * on the handle's stream; no allocation, no host synchronisation.  Every
 * call on one device shares that device's array: calls that overlap on a
 * device (several streams or threads) race and must be serialised by the
 * caller. */
int iblb_mlp_forward_noalloc(iblb_mlp *mlp, const float *d_x, int batch, float *d_y);

#ifdef __cplusplus
}
#endif
#endif /* IBLB_H */

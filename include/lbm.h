/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice Boltzmann library with per-step
 * flow forces.
 *
 * The library advances a two-dimensional D2Q9 BGK lattice Boltzmann model (Kaushal,
 * Succi & Ansumali, "Flow force calculation in Lattice Boltzmann Method",
 * arXiv:2210.10377, Sec. II: Eq. CollideAdv, the second-order equilibrium, Table I)
 * around a body given as a solid mask on the Cartesian grid, with half-way bounce-back
 * on every fluid-solid link (Sec. II, stationary wall) and, at every step, the force of
 * the fluid on the body by four estimators:
 *   - momentum exchange, algorithm A (Sec. IV, Eq. rtt4 "Algorithm A"),
 *   - momentum exchange, algorithm B (Sec. IV, Eq. rtt4 "Algorithm B", Eq. rtt5),
 *   - the discrete Reynolds-transport-theorem control-volume force DRTT (Sec. IV,
 *     second Eq. rtt7; Appendix),
 *   - stress integration SI over the staircase surface (Sec. III, Eq. stress_int).
 * The paper's problem statement is a body in a channel, a relaxation time, an inlet,
 * and the force on the body at every step (Sec. V, Appendix); the calls below follow it.
 *
 * Conventions used throughout:
 *   - Node (x, y) with 0 <= x < nx, 0 <= y < ny sits at the point (x, y).  Host arrays
 *     over the grid are row-major [ny][nx]; population arrays are [9][ny][nx].
 *   - Directions: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1)
 *     8:(1,-1); weights 4/9, 1/9, 1/36 (Table I), c_s^2 = theta0 = 1/3.
 *   - Deviation storages (LBM_FP16DEV, LBM_FP32DEV) keep h_i = f_i - w_i and do the
 *     collision in deviation form (rho - 1 = sum h_i, rho u = sum c_i h_i, h~ = h +
 *     omega (f^eq - w - h)), which avoids the cancellation of rho ~ 1 in binary32; the
 *     boundary rules act on h exactly as on f because w_i = w_opposite(i).
 *   - tau is the lattice relaxation time tau_lb: the factor 2 beta of Eq. CollideAdv is
 *     1/tau_lb, and the kinematic viscosity is (tau_lb - 1/2)/3.
 *   - The stored state is the post-collision field of the last step.  One step pulls it
 *     along -c_i with the boundary rules, collides, and stores the result.  Pull
 *     rules, first match wins: periodic wrap; no-slip wall (half-way bounce-back at
 *     y = -1/2 and y = ny - 1/2); inlet (moving-wall bounce-back of Sec. II at
 *     x = -1/2 with wall velocity (u_in(y), 0) and density rho_w); outlet (ghost
 *     column nx copies the post-collision column nx-1; bounce-back if that node is
 *     solid); body (half-way bounce-back); otherwise plain streaming.
 *   - Forces are those of the fluid on the body, in lattice units, indexed by the
 *     collision step t, accumulated in FP64 from the populations as stored:
 *       A(t)    = sum_{links (x,i)} c_i [f_i(x,t) + f~_i(x,t)]   (pre-collision out)
 *       B(t)    = sum_{links (x,i)} 2 c_i f~_i(x,t)               (post-collision out)
 *       DRTT(t) = J(t) - J(t+1) + Phi(t), J(t) the momentum of the pre-collision
 *                 populations of the control volume V (the fluid nodes of the box),
 *                 Phi(t) = sum of c_i f~_i(x,t) over populations entering V minus those
 *                 leaving V,
 *       DRTT-post(t) = J~(t) - J(t+1) + Phi(t), J~(t) the momentum of the stored
 *                 (post-collision) populations of V: the box balance over the
 *                 streaming half of the step.  A momentum-conserving collision makes
 *                 J~(t) = J(t) in exact arithmetic (Appendix: J is sampled before the
 *                 collision); with rounded storage only DRTT-post stays equal to B up
 *                 to the rounding of the FP64 sums, since every term then reads the
 *                 same stored values,
 *       SI(t)   = sum_{axis links (x,i), i = 1..4} (-p I + sigma)(x,t) . (-c_i): each
 *                 axis link crosses one unit face of the staircase body surface, whose
 *                 normal out of the body is -c_i; p = rho/3 and the deviatoric stress
 *                 sigma = -(1 - 1/(2 tau_lb)) sum_k (f_k - f_k^eq) c_k c_k at the fluid
 *                 node, from its pre-collision populations.
 *     A link is a fluid node x and a direction i with x + c_i a solid mask node.
 *
 * Memory: the caller owns all memory.  lbm_create copies the mask and inlet profile.
 * The device workspace (lbm_workspace_bytes) is allocated by the caller, bound with
 * lbm_bind, and must outlive the handle's use; the library itself allocates no device
 * memory.  The HIP stream is the caller's.
 *
 * Synchronisation: lbm_step only enqueues work on the bound stream.  lbm_forces,
 * lbm_get_* and lbm_set_* synchronise that stream before returning.
 *
 * Threading: one host thread at a time per handle; separate handles are independent.
 *
 * Errors: every call returns LBM_OK (0) or a negative code; lbm_last_error gives a
 * message for the last failing call on a handle.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)     /* invalid argument or configuration            */
#define LBM_ENOMEM (-2)     /* grid too large / workspace too small         */
#define LBM_EHIP (-3)       /* a HIP runtime call failed                    */
#define LBM_ENONFINITE (-4) /* a requested force was NaN or infinite        */
#define LBM_ESTATE (-5)     /* call not valid in the handle's current state */
#define LBM_EOVERFLOW (-6)  /* the force ring cannot hold the steps asked   */

/* Population storage precision. */
#define LBM_FP64 0    /* binary64 populations, binary64 arithmetic                  */
#define LBM_FP32 1    /* binary32 populations, binary32 arithmetic                  */
#define LBM_FP16DEV 2 /* binary16 deviations h_i = f_i - w_i, binary32 arithmetic   */
#define LBM_FP32DEV 3 /* binary32 deviations h_i = f_i - w_i, binary32 arithmetic   */
/* binary32 populations f_i, binary32 arithmetic in deviation form, every store rounded
 * stochastically (unbiased; the draws are a fixed hash of the step number, the node and
 * the direction, so runs are reproducible bit for bit, in a batch as alone).  Every path
 * but lbm_step_static, which refuses it. */
#define LBM_FP32SR 4

#define LBM_BCX_INLET_OUTLET 0 /* x: inlet at x = -1/2, outlet at x = nx - 1/2      */
#define LBM_BCX_PERIODIC 1
#define LBM_BCY_WALL 0         /* y: no-slip walls at y = -1/2 and y = ny - 1/2      */
#define LBM_BCY_PERIODIC 1

/* Collision operator. */
#define LBM_COLL_BGK 0         /* BGK, Eq. CollideAdv                                  */
#define LBM_COLL_REGULARIZED 1 /* regularized BGK (Latt & Chopard 2006; not in the
                                  paper): the non-equilibrium part is projected on the
                                  second-order Hermite subspace before relaxation,
                                  f~ = f^eq + (1 - 1/tau_lb) w_i (c_i c_i - I/3) : Pi^neq
                                  / (2/9), Pi^neq = sum_i c_i c_i (f_i - f^eq_i).  Same
                                  memory traffic; the variant for tau_lb close to 1/2,
                                  where BGK loses stability.  Conserves mass and
                                  momentum, so every force estimator applies unchanged. */
#define LBM_COLL_KBC 2         /* entropic KBC collision (Karlin, Boesch & Chikatamarla
                                  2014; not in the paper) with the same polynomial
                                  equilibrium: d = f - f^eq splits into its shear part
                                  ds (deviatoric stresses) and the rest dh;
                                  f~ = f - (1/(2 tau_lb))(2 ds + gamma dh), gamma from
                                  the entropic stabilizer (gamma = 2 is BGK; BGK is used
                                  when dh is at rounding level).  Same shear viscosity
                                  and memory traffic as BGK, far more stable near
                                  tau_lb = 1/2; conserves mass and momentum.  In binary32
                                  arithmetic the stabilizer is switched off below
                                  |dh|^2 ~ 2^-40 (2^-90 in binary64).                    */

/* Force schemes (bit mask for lbm_step). */
#define LBM_FORCE_MEA_A 1u
#define LBM_FORCE_MEA_B 2u
#define LBM_FORCE_DRTT 4u
#define LBM_FORCE_SI 8u
#define LBM_FORCE_DRTT_POST 16u /* DRTT with J(t) taken after the collision (below)   */
#define LBM_FORCE_ALL 31u

typedef struct lbm_grid {
  int32_t nx, ny;     /* grid size, each >= 3                                      */
  int32_t bc_x, bc_y; /* LBM_BCX_*, LBM_BCY_*                                      */
  int32_t precision;  /* LBM_FP64 / LBM_FP32 / LBM_FP16DEV / LBM_FP32DEV /
                         LBM_FP32SR                                              */
  int32_t box[4];     /* DRTT control volume [x0, x1) x [y0, y1); x0 < 0: none.
                         Must satisfy 1 <= x0, x1 <= nx - 1, 1 <= y0, y1 <= ny - 1,
                         and hold every solid node strictly inside
                         [x0+1, x1-1) x [y0+1, y1-1).                              */
  int32_t max_record; /* force-ring capacity in steps (>= 1)                        */
  double rho_ref, u_ref, l_ref; /* normalisation of the force coefficients (Sec. V:
                                   C = 2 F / (rho U^2 L))                           */
  int32_t collision;  /* LBM_COLL_BGK (0), LBM_COLL_REGULARIZED or LBM_COLL_KBC         */
  int32_t layout;     /* LBM_LAYOUT_AUTO (0), LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES: device
                         layout of the state buffers, same results                  */
  int32_t tile;       /* LBM_TILE_AUTO (0), LBM_TILE_WIDE or LBM_TILE_NARROW: shape of
                         the step kernel's tiles, same results                       */
} lbm_grid;

/* Tiles of the step kernel (one 256-thread workgroup of four 64-node strips).  WIDE:
 * the strips side by side along a row (256 x 1).  NARROW: one above the other (64 x 4),
 * fewer idle lanes on grids whose rows end in a partial wide tile.  AUTO: NARROW when
 * nx <= 1024 and a wide tile would leave at least 64 idle lanes at the end of a row. */
#define LBM_TILE_AUTO 0
#define LBM_TILE_WIDE 1
#define LBM_TILE_NARROW 2

/* State-buffer layouts (both lattices).  ROWS: the populations of one grid row stored
 * direction after direction ([ny][9][row] in 2-D, [nz][ny][27][row] in 3-D), so a tile
 * touches few memory pages: the faster one; needs a buffer below 2^31 elements.
 * PLANES: one plane per direction ([9][ny][row], [27][nz][ny][row]), planes padded;
 * needs a plane below 2^31 elements.  AUTO: ROWS when it fits, else PLANES.  Rows are nx
 * padded to 64 elements plus a pad (128 in 2-D; in 3-D 64 at multiples of 1024). */
#define LBM_LAYOUT_AUTO 0
#define LBM_LAYOUT_ROWS 1
#define LBM_LAYOUT_PLANES 2

typedef struct lbm_inlet {
  const double* ux; /* ny inlet velocities u_in(y) (host); ignored (may be NULL)
                       when bc_x is periodic                                       */
  double rho_w;     /* wall density of the moving-wall inlet rule (normally 1)     */
} lbm_inlet;

typedef struct lbm_t lbm_t;

typedef struct lbm_info {
  int64_t n_fluid;        /* fluid nodes                                             */
  int64_t n_links;        /* fluid-solid links (x, i)                                */
  int64_t n_tiles;        /* tiles of the step kernel                                */
  int64_t n_general;      /* 64-node strips that take the boundary / force path      */
  int64_t n_box;          /* fluid nodes in the control volume                       */
  int64_t steps_done;     /* steps taken since create (or the restored state)        */
  int64_t n_recorded;     /* force rows waiting in the ring                          */
  int32_t tile_w, tile_h; /* tile shape in nodes                                     */
  int64_t plane_stride;   /* elements between the directions of a node (device layout:
                             population i of (x, y) at i*plane_stride + y*pitch + x)  */
  int32_t pitch;          /* elements between rows (device layout)                   */
  int32_t elem_bytes;     /* bytes per stored population                             */
} lbm_info;

/* Validate the configuration, classify every node and link, and return a handle.
 * solid_mask: host, ny*nx bytes, each 0 (fluid) or 1 (solid).  tau: tau_lb > 1/2.
 * inlet may be NULL when bc_x is periodic.  Returns LBM_EINVAL for nx or ny < 3,
 * non-finite or tau <= 1/2, a mask byte outside {0,1}, a missing, non-finite inlet,
 * an inadmissible box, unknown codes (precision, boundaries, collision) or
 * max_record < 1, or an unknown layout; LBM_ENOMEM for grids too large for the layout
 * (a plane of 2^31 elements or more; with LBM_LAYOUT_ROWS, a buffer of 2^31 or more).
 * Needs no GPU. */
int lbm_create(const lbm_grid* grid, const uint8_t* solid_mask, double tau,
               const lbm_inlet* inlet, lbm_t** out);

/* Device workspace the handle needs, in bytes (needs no GPU). */
int lbm_workspace_bytes(const lbm_t* h, size_t* bytes);

/* Bind a caller-owned device workspace (>= lbm_workspace_bytes, 256-byte aligned) and
 * HIP stream (hipStream_t, NULL for the default stream), upload the tables and put
 * every node in the rest state w_i.  Synchronises the stream.  LBM_ENOMEM if the
 * workspace is too small, LBM_EINVAL if misaligned. */
int lbm_bind(lbm_t* h, void* device_workspace, size_t bytes, void* hip_stream);

/* Enqueue n >= 0 time steps on the bound stream.  force_scheme is a mask of
 * LBM_FORCE_*; when non-zero every step records one force row (all four estimators
 * are evaluated; rows for schemes not asked for read NaN).  Returns LBM_EOVERFLOW
 * without launching anything if the ring would overflow, LBM_ESTATE if unbound,
 * LBM_EINVAL for n < 0 or unknown scheme bits. */
int lbm_step(lbm_t* h, int32_t n, uint32_t force_scheme);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_step on two caller-owned state
 * buffers, with every other device buffer the step needs (pull codes, strip slots,
 * inlet profile, body motion, force partials, force rows) in a static device array of
 * the library, LBM_STATIC_SCRATCH_BYTES per GPU, held by each GPU from the first call on
 * it until the process ends.  The call allocates no device memory.
 *   buf0, buf1: distinct 256-byte aligned device buffers of buf_bytes >= one state of the
 *     handle each (the state layout of the handle's workspace, see lbm_info: population
 *     i of (x, y) at i * plane_stride + y * pitch + x, elem_bytes each, in a buffer of
 *     max(9 plane_stride, ny pitch) elements).  buf0 holds the current state on entry;
 *     step k reads one buffer and writes the other, so after the call the state is in
 *     buf0 when n is even and in buf1 when n is odd.
 *   n >= 0 steps, force_scheme as lbm_step; with any scheme bit set and n > 0 the force
 *     rows of the n steps are written to forces[n][5][2] (host, cap >= n rows) as
 *     lbm_forces gives them.
 *   hip_stream: the stream the work is enqueued on (NULL: the null stream); the call
 *     synchronises it when forces are asked for.
 * The handle needs no binding; its own state, step count, force ring and adjoint run
 * are not touched (its geometry, tau, inlet and body motion are used).  Every call on a
 * GPU shares that GPU's array, which keeps the last call's contents (each call writes
 * what it reads first); calls that overlap on one GPU race.  LBM_ENOMEM when the grid's
 * tables and n force rows do not fit the array (about 4 bytes per node plus 112 bytes per
 * step with forces) or the buffers are smaller than a state; LBM_EINVAL for bad
 * arguments; LBM_ENONFINITE as lbm_forces. */
#define LBM_STATIC_SCRATCH_BYTES (32u << 20)
int lbm_step_static(lbm_t* h, void* buf0, void* buf1, size_t buf_bytes, int32_t n,
                    uint32_t force_scheme, double* forces, int64_t cap, void* hip_stream);

/* Copy the force rows recorded since the last call into out[k][5][2] (host; scheme
 * order A, B, DRTT, SI, DRTT-post; components x, y) and empty the ring.  At most cap rows are written
 * (LBM_EINVAL if fewer than recorded).  Synchronises the stream.  Returns
 * LBM_ENONFINITE (after writing everything) if any requested value is not finite. */
int lbm_forces(lbm_t* h, double* out, int64_t cap, int64_t* k_out);

/* Force coefficients 2 F / (rho_ref u_ref^2 l_ref) of k force rows ([k][5][2], Sec. V:
 * drag and lift coefficients, kept signed), host to host; in and out may alias. */
int lbm_coefficients(const lbm_t* h, const double* forces, int64_t k, double* out);

int lbm_destroy(lbm_t* h);

/* Canonical fluid-solid links (node = y*nx + x, direction i), sorted by node then
 * direction, into node_dir[L][2] (host); writes min(L, cap) pairs and returns L in
 * *n.  Needs no GPU. */
int lbm_get_links(const lbm_t* h, int32_t* node_dir, int64_t cap, int64_t* n);

int lbm_get_info(const lbm_t* h, lbm_info* info);

/* Current stored (post-collision) populations as binary64, out[9][ny][nx] (host;
 * the deviation storages read w_i + h_i, summed in binary64).  Synchronises the
 * stream. */
int lbm_get_populations(lbm_t* h, double* out);

/* Replace the stored populations (host, [9][ny][nx]); values are rounded to the
 * storage precision (the deviation storages keep h_i = f_i - w_i, computed in binary64
 * and rounded once to nearest even).
 * Synchronises the stream. */
int lbm_set_populations(lbm_t* h, const double* in);

/* Checkpoint: the exact stored state (raw storage bytes plus the step counter) as an
 * opaque host blob of lbm_state_bytes bytes; lbm_set_state accepts a blob of a handle
 * with the same grid size and precision.  Both synchronise the stream. */
int lbm_state_bytes(const lbm_t* h, size_t* bytes);
int lbm_get_state(lbm_t* h, void* blob, size_t cap);
int lbm_set_state(lbm_t* h, const void* blob, size_t n);

/* Replace the inlet profile (ny host values, copied) or the relaxation time tau_lb
 * (> 1/2) of a handle; later steps use the new values.  lbm_set_inlet synchronises the
 * stream when the handle is bound. */
int lbm_set_inlet(lbm_t* h, const double* ux);
int lbm_set_tau(lbm_t* h, double tau);

/* Rigid motion of the body (not in the paper's runs; the moving-wall bounce-back of
 * Sec. II applied to the body links): translation (ux, uy) and rotation rate omega about
 * (xc, yc), so a link whose half-way point is x_w sees the wall velocity
 * u_w = (ux - omega (y_w - yc), uy + omega (x_w - xc)), and the population it returns
 * gains 2 w_i rho_w (c_i . u_w) / c_s^2 (rho_w of the inlet, 1 by default).  The mask
 * does not move (a rotating or sliding surface of fixed shape).  A and B take the
 * returned population in their two-term form, c_i [f_out + f_back]; DRTT and SI apply
 * unchanged.  All zero (the default) is a body at rest.  Applies from the next step of
 * the handle (the device copy is written on the handle's stream, which is synchronised
 * when the handle is bound) and from the next lbm_batch_step of a batch holding it;
 * the adjoint calls refuse a moving body.  LBM_EINVAL for non-finite values. */
int lbm_set_body_motion(lbm_t* h, double ux, double uy, double omega, double xc, double yc);

/* A body that moves through the grid (not in the paper's runs; the bounce-back of
 * Sec. II on the links of each mask): replace the body mask, and the control volume
 * when `box` is non-null ([x0, x1, y0, y1] as in lbm_grid; it can be moved or resized,
 * not added or removed), between two steps.  solid_mask: host, [ny][nx] bytes, 0 fluid
 * / 1 solid, copied.  Every recorded step keeps the geometry it was taken with (the
 * J(t+1) of the last step before the change was taken under the old mask and box), so
 * the momentum that changes hands with the nodes the body covers or uncovers enters no
 * estimator; it is returned instead in impulse[2] (host, may be NULL): the momentum of
 * the covered nodes minus that of the refilled ones, i.e. what the fluid hands to the
 * body in the change.  Nodes the body uncovers are refilled with the equilibrium at the
 * rigid-body velocity of lbm_set_body_motion at the node and the mean density of their
 * lattice neighbours that are fluid in both masks (rho_w of the inlet when none is; a
 * neighbour across a periodic edge wraps, one outside another edge does not count).
 * The motion's centre is not advanced by the library: a translating and turning body
 * sets its new centre with lbm_set_body_motion at each change.  Bound handles: waits
 * for the whole device first (no step of the handle, or of a batch holding it, may
 * still be in flight), uses the idle state buffer as scratch, synchronises the stream.
 * LBM_EINVAL: mask values other than 0/1, a box that is not admissible for the new
 * mask; LBM_ENOMEM: the new mask needs more force-partial slots than twice those of
 * the mask at create (plus 4096 doubles), or a larger box than the one at create.  On
 * these errors nothing changes.  On LBM_EHIP the state is undefined.  The adjoint
 * forward run held by the handle is discarded. */
int lbm_set_mask(lbm_t* h, const uint8_t* solid_mask, const int32_t* box, double* impulse);

/* Pressure coefficient at the boundary fluid nodes (Sec. V, the C_p equation: computed
 * over the boundary fluid nodes, without extrapolation):
 *   C_p = (p - p_inf) / (rho_ref u_ref^2 / 2),  p = rho theta0 = rho / 3,
 * rho the density of the current stored state at the node (sum of its populations in
 * binary64; the collision conserves it), p_inf the same at the far-upstream reference
 * node (x_inf, y_inf), or rho_ref / 3 when x_inf < 0; rho_ref and u_ref of lbm_grid.  A
 * boundary fluid node is a fluid node with at least one fluid-solid link; the nodes come
 * in row-major order (the node order of lbm_get_links).  Writes the n values to cp (host,
 * cap >= n) and, when nodes is non-null, their indices y * nx + x (host, n entries);
 * *n = n (also when n is 0 and cp is NULL).  Computed by a kernel from the current
 * state; synchronises the stream and uses the idle state buffer as scratch (no work of
 * the handle, or of a batch holding it, may be in flight on another stream).
 * LBM_EINVAL for a reference node outside the grid or solid, cap < n, or rho_ref or
 * u_ref zero or non-finite; LBM_ESTATE if unbound. */
int lbm_boundary_cp(lbm_t* h, int32_t x_inf, int32_t y_inf, double* cp, int32_t* nodes,
                    int64_t cap, int64_t* n);

/* Put every node back in the rest state w_i, zero the step counter and empty the force
 * ring.  Synchronises the stream. */
int lbm_reset(lbm_t* h);

/* Adjoint (reverse mode) of the time-averaged body force, for gradients with respect
 * to the inlet profile u_in(y) and tau (the collide-stream-bounce-back map of
 * Eq. CollideAdv and Sec. II differentiated step by step).  The objective is
 *   J = (1/T) sum_{t = t0}^{t0+T-1} (wx F_Bx(t) + wy F_By(t)),
 * F_B the momentum-exchange force of algorithm B (Eq. rtt5; the bounce-back force of
 * Sec. IV) at step t of a run of n_steps steps from the handle's current state.
 *
 * lbm_adjoint_bytes: device workspace for a run of n_steps with a checkpoint every
 * `every` steps (1 <= every <= n_steps): ceil(n/every) checkpoints, two stores of every-1
 * recomputed states on grids of at most 16,384 tiles (one on larger grids or when there
 * is a single segment), two adjoint fields and the per-step force rows.
 *
 * lbm_adjoint_forward: run the n_steps (the handle's state advances, as lbm_step would
 * advance it; the force ring is not touched), storing the checkpoints in the caller's
 * workspace ws (256-byte aligned, >= lbm_adjoint_bytes; it must stay untouched until the
 * backward call), and return J (FP64) in *J.  Synchronises the stream.  LBM_EINVAL for
 * t0 < 0, T < 1, t0 + T > n_steps or bad sizes; LBM_ENONFINITE if J is not finite.
 *
 * lbm_adjoint_backward: reverse sweep over the stored run: each segment between
 * checkpoints is recomputed forward, then the adjoint kernel runs one launch per step
 * backwards.  On grids of at most 16,384 tiles the recomputation of the next segment
 * runs on a second stream of the library's own (created at the first call, default
 * priority, released by lbm_destroy) while the reverse launches of the current one run
 * on the handle's stream; events order the two, and the call returns after both.  Writes dJ/du_in(y) * dJ (ny host values) to grad_uin and dJ/dtau * dJ to
 * *grad_tau, where dJ is the incoming seed.  The adjoint fields are kept in the
 * storage's arithmetic precision (FP64 for LBM_FP64, FP32 otherwise); the gradient sums
 * are FP64.  Synchronises the stream.  LBM_ESTATE unless the last adjoint forward run is
 * still valid (any step, set_* or reset since invalidates it).  The adjoint covers the
 * BGK collision, bodies at rest and the LBM_FP64, LBM_FP32, LBM_FP32DEV and LBM_FP32SR
 * storages only: both calls return LBM_EINVAL otherwise (LBM_FP16DEV included, checked
 * before anything else, so an unbound handle gets it too).  With LBM_FP32SR the
 * recomputation replays every step with the forward run's step number, so the reverse
 * sweep reads bitwise the states the forward run stored.  After lbm_set_mask the
 * adjoint follows the new mask. */
int lbm_adjoint_bytes(const lbm_t* h, int32_t n_steps, int32_t every, size_t* bytes);
int lbm_adjoint_forward(lbm_t* h, void* ws, size_t bytes, int32_t n_steps, int32_t every,
                        int32_t t0, int32_t T, double wx, double wy, double* J);
int lbm_adjoint_backward(lbm_t* h, double dJ, double* grad_uin, double* grad_tau);

/* Message of the last failing call on h (or of the last failing lbm_create when h is
 * NULL).  The string lives until the next call on the handle. */
const char* lbm_last_error(const lbm_t* h);

/* ---- Batches -------------------------------------------------------------------------
 * Not in the paper: a throughput form for sweeps over many small problems of the kind
 * of Sec. V (cylinders and airfoils in walled channels, each with its own grid, body,
 * relaxation time, inlet and control volume).  A batch groups bound handles of one
 * precision and advances all of them together: each step is ONE kernel launch that
 * updates every instance (a sweep over the concatenated tile lists of all instances,
 * optionally by a persistent grid), and runs of launches can be replayed from captured
 * HIP graphs.  Every instance computes exactly what lbm_step computes for it (same
 * kernels per tile, same force reduction order): populations and forces are bitwise
 * those of the member stepped alone with the same call lengths.
 *
 * Ownership: the members stay owned by the caller and must outlive the batch; their
 * workspaces hold the states, which lbm_get_populations etc. read as usual.  While a
 * batch call runs, members must not be used on another stream.  A member may still be
 * stepped or changed (lbm_set_tau, lbm_set_inlet, lbm_set_populations, lbm_reset)
 * between batch calls; the batch picks the change up at its next call.  lbm_batch_step
 * advances every member's state and step count; the force rows it records go to the
 * batch's own ring ([max_record][n] rows, step-major), not to the members' rings. */
typedef struct lbm_batch_t lbm_batch_t;

typedef struct lbm_batch_schedule {
  int32_t grid_blocks; /* tile workgroups per launch: 0 = one per tile; otherwise a
                          persistent grid, rounded up to a multiple of 8             */
  int32_t graph_steps; /* launches per captured HIP graph: 0 = direct launches;
                          otherwise an even count >= 2                               */
  uint32_t tile_order; /* 0: instance-major tile list; otherwise the seed of a
                          pseudo-random permutation of it (results do not depend on
                          the order; it changes only the schedule)                    */
  int32_t tile_queue;  /* persistent grids only: 0 = each workgroup takes every
                          grid_blocks-th tile of the list; 1 = workgroups take the
                          next 16 tiles from a device counter (one global atomic per
                          16 tiles, reset by a small kernel at each lbm_batch_step
                          call and by each launch for the next), over a list ordered
                          largest instance first.  Results do not depend on it.      */
  int32_t tile_shape;  /* LBM_TILE_AUTO (0): every instance keeps its own tile shape;
                          LBM_TILE_WIDE / LBM_TILE_NARROW: every instance runs in
                          256 x 1 / 64 x 4 tiles in the batch (the member's own
                          lbm_step keeps its shape).  The force partials are numbered
                          per strip, so results do not depend on it.                 */
} lbm_batch_schedule;

typedef struct lbm_batch_info {
  int32_t n_inst;          /* instances                                              */
  int32_t n_recorded;      /* force rows waiting in the batch ring                    */
  int64_t total_tiles;     /* tiles over all instances                               */
  int64_t total_fluid;     /* fluid nodes over all instances                         */
  int64_t total_nodes;     /* nodes over all instances                               */
  int64_t steps_done;      /* steps taken by lbm_batch_step (and autotuning)          */
  int32_t n_graphs;        /* captured graphs held                                   */
  int32_t compute_units;   /* of the bound device (0 before bind)                    */
  lbm_batch_schedule schedule;
} lbm_batch_info;

/* Group n >= 1 distinct, bound handles of one precision and one collision operator into
 * a batch whose ring holds max_record >= 1 force rows per instance.  LBM_EINVAL for a
 * NULL, repeated or unbound member, mixed precisions or collisions, or a member whose
 * state buffer is 4 GiB or more.  Needs no GPU work. */
int lbm_batch_create(lbm_t* const* members, int32_t n, int32_t max_record, lbm_batch_t** out);

/* Device workspace of the batch (instance table, tile and sweep lists, force ring). */
int lbm_batch_workspace_bytes(const lbm_batch_t* b, size_t* bytes);

/* Bind a caller-allocated device workspace (256-byte aligned, at least
 * lbm_batch_workspace_bytes) and a HIP stream (NULL = the null stream); uploads the
 * tables and synchronises.  Creates one private stream of default priority, used only
 * to capture graphs (graphs are launched on the bound stream). */
int lbm_batch_bind(lbm_batch_t* b, void* device_workspace, size_t bytes, void* hip_stream);

/* Choose the schedule (see lbm_batch_schedule).  LBM_EINVAL for negative values, an
 * odd graph_steps, tile_queue other than 0 or 1, a tile queue without a persistent
 * grid, or an unknown tile_shape.  Drops captured graphs. */
int lbm_batch_set_schedule(lbm_batch_t* b, const lbm_batch_schedule* s);

/* Time candidate schedules (one block per tile, and persistent grids of 1, 2, 4 and 8
 * workgroups per compute unit with the static stride and with the tile queue; each with
 * direct launches and with graphs of up to 64 launches; the tile order seed and the
 * tile shape are kept; then the fastest of those with each of the two other tile
 * shapes) over `steps` steps each, after a warm-up run of the same length, with forces
 * force_scheme (0 = none).  Keeps the fastest and returns it in *best and its
 * milliseconds per step in *ms_per_step (either may be NULL).  Every instance advances
 * by 2 x steps per candidate (40 x steps in all: 18 schedules, then 2 tile shapes);
 * those force rows are not kept.
 * LBM_EOVERFLOW if the ring cannot hold `steps` rows beside the rows recorded;
 * LBM_ESTATE if a member's control volume changed size since create.  Synchronises the
 * stream. */
int lbm_batch_autotune(lbm_batch_t* b, int32_t steps, uint32_t force_scheme,
                       lbm_batch_schedule* best, double* ms_per_step);

/* Enqueue n >= 0 steps of every instance on the bound stream with the forces of
 * force_scheme (as lbm_step).  LBM_EOVERFLOW when force rows would exceed max_record. */
int lbm_batch_step(lbm_batch_t* b, int32_t n, uint32_t force_scheme);

/* Drain the batch ring: out[i][t][scheme][component] (host, n_inst x cap x 5 x 2
 * doubles) receives instance i's forces of the t-th recorded step, as lbm_forces
 * gives them; *k_out the number of rows (also when out is NULL and nothing is
 * recorded).  nonfinite (host, n_inst bytes, may be NULL) flags instances with a
 * non-finite requested force.  Returns LBM_ENONFINITE when any flag is set (the rows
 * are delivered and the ring drained all the same).  Synchronises the stream. */
int lbm_batch_forces(lbm_batch_t* b, double* out, int64_t cap, int64_t* k_out,
                     uint8_t* nonfinite);

int lbm_batch_get_info(const lbm_batch_t* b, lbm_batch_info* info);

/* Free the batch's host state, graphs and private stream (not the members). */
int lbm_batch_destroy(lbm_batch_t* b);

/* Message of the last failing call on b (or of the last failing lbm_batch_create when
 * b is NULL). */
const char* lbm_batch_last_error(const lbm_batch_t* b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

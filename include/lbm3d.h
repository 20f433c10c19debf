/*
 * lbm3d.h -- C ABI of the three-dimensional (D3Q27) lattice Boltzmann path with per-step
 * flow forces, in the same library as lbm.h and with its error and precision codes.
 *
 * The paper (Kaushal, Succi & Ansumali, arXiv:2210.10377) computes flow forces in two
 * dimensions with D2Q9 and in three with the RD3Q41 model (Sec. V, flow past a 3-D
 * NACA0012; Table comp_details).  RD3Q41's equilibrium needs a constant that the paper
 * defines only through a cited work, so this path uses the cubic D3Q27 velocity set
 * with the same second-order equilibrium (Sec. II, theta0 = 1/3), the BGK collision of
 * Eq. CollideAdv, the half-way bounce-back of Sec. II, and the same four estimators as
 * lbm.h, with every sum over directions and nodes taken in three dimensions:
 *   A(t)    = sum_{links (x,i)} c_i [f_i(x,t) + f~_i(x,t)]        (Eq. rtt4, A)
 *   B(t)    = sum_{links (x,i)} 2 c_i f~_i(x,t)                    (Eq. rtt4/rtt5, B)
 *   DRTT(t) = J(t) - J(t+1) + Phi(t) over the control volume V     (second Eq. rtt7)
 *   SI(t)   = sum_{axis links (x,i), i = 1..6} (-p I + sigma)(x,t) . (-c_i)
 *                                                                  (Eq. stress_int)
 * with p = rho/3 and sigma = -(1 - 1/(2 tau_lb)) sum_k (f_k - f_k^eq) c_k c_k at the
 * fluid node of the link from its pre-collision populations.  A link is a fluid node x
 * and a direction i with x + c_i (wrapped along periodic axes) a solid node.
 *
 * Conventions:
 *   - Node (x, y, z), 0 <= x < nx, ..., sits at the point (x, y, z).  Host arrays over
 *     the grid are [nz][ny][nx]; population arrays are [27][nz][ny][nx]; the inlet
 *     profile is [nz][ny].
 *   - Directions (the layout of population arrays): 0 rest; 1..6 faces +x -x +y -y +z
 *     -z; 7..18 edges in the xy, xz and yz planes, each as (+,+) (-,-) (+,-) (-,+);
 *     19..26 corners +++ --- ++- --+ +-+ -+- -++ +--.  Direction 2k is opposite to
 *     2k - 1.  Weights 8/27 (rest), 2/27 (faces), 1/54 (edges), 1/216 (corners).
 *   - Precisions LBM_FP64, LBM_FP32, LBM_FP32DEV, LBM_FP16DEV as in lbm.h (deviation
 *     storages keep h_i = f_i - w_i and collide in deviation form).
 *   - Boundary codes: bc_x LBM_BCX_INLET_OUTLET (inlet at x = -1/2, moving-wall
 *     bounce-back with wall velocity (u_in(y, z), 0, 0) and density rho_w; outlet ghost
 *     plane x = nx copies plane nx-1, bounce-back where that node is solid) or
 *     LBM_BCX_PERIODIC; bc_y and bc_z LBM_BCY_WALL (half-way bounce-back walls at -1/2
 *     and n - 1/2) or LBM_BCY_PERIODIC.  Pull rules, first match wins: periodic wrap,
 *     walls (y, then z), inlet, outlet, body bounce-back, plain streaming.
 *   - Control volume: box [x0,x1) x [y0,y1) x [z0,z1), V its fluid nodes.  Admissible
 *     axis by axis: a periodic axis may be spanned whole (0, n) -- then the box has no
 *     surface across it and a body may pass through it (an airfoil of infinite span);
 *     otherwise the box lies one node inside the domain and every solid node lies
 *     strictly inside it with a fluid layer between body and surface.
 *   - Forces are those of the fluid on the body in lattice units, FP64, indexed by the
 *     collision step; output arrays are [k][4 = A, B, DRTT, SI][3 = x, y, z], NaN for a
 *     scheme that was not evaluated at that step and for DRTT without a box.
 *   - Memory, streams, synchronisation and threading as in lbm.h: the caller allocates
 *     the device workspace (lbm3d_workspace_bytes) and binds it with a stream; the
 *     library allocates no device memory; lbm3d_step only enqueues; the other calls
 *     synchronise the stream.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d lbm3d_t;

typedef struct {
  int32_t nx, ny, nz;   /* nodes along x, y, z (each >= 2; nx*ny*nz < 2^31)          */
  int32_t bc_x;         /* LBM_BCX_INLET_OUTLET or LBM_BCX_PERIODIC                   */
  int32_t bc_y, bc_z;   /* LBM_BCY_WALL or LBM_BCY_PERIODIC                          */
  int32_t box[6];       /* x0, x1, y0, y1, z0, z1; box[0] < 0: no control volume     */
  int32_t precision;    /* LBM_FP64, LBM_FP32, LBM_FP32DEV, LBM_FP16DEV, LBM_FP32SR  */
  int32_t max_record;   /* rows of the force ring (>= 1)                             */
  int32_t collision;    /* LBM_COLL_BGK or LBM_COLL_REGULARIZED (the regularized BGK of
                           lbm.h with the D3Q27 Hermite projection; not in the paper) */
  int32_t layout;       /* device layout of the state buffers: LBM_LAYOUT_AUTO (0),
                           LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES of lbm.h; same results */
} lbm3d_grid;

typedef struct {
  int64_t n_fluid;      /* fluid nodes                                               */
  int64_t n_links;      /* body links                                                */
  int64_t n_box;        /* nodes of V                                                */
  int64_t steps_done;   /* steps since bind                                           */
  int64_t n_recorded;   /* force rows waiting in the ring                            */
  int32_t n_general;    /* 64-node strips on the general (boundary-aware) path       */
  int32_t n_strips;     /* all strips                                                */
} lbm3d_info;

/* Plan a lattice: classify every node from the mask ([nz][ny][nx] bytes, 0 fluid /
 * 1 solid, copied) and the boundary codes.  tau: tau_lb > 1/2.  uin: [nz][ny] inlet
 * x-velocities (host, copied), required when bc_x is inlet/outlet, else ignored;
 * rho_w: inlet wall density (> 0).  LBM_EINVAL for a bad code, size, mask value, box,
 * collision, layout or tau (lbm3d_last_error(NULL) says which); LBM_ENOMEM when the
 * grid is too large for the layout. */
int lbm3d_create(const lbm3d_grid* grid, const uint8_t* solid_mask, double tau,
                 const double* uin, double rho_w, lbm3d_t** out);

/* Bytes of device workspace the handle needs (two state buffers, node words, strip
 * table, inlet plane, force partials, force ring). */
int lbm3d_workspace_bytes(const lbm3d_t* h, size_t* bytes);

/* Bind a device workspace (256-byte aligned, at least lbm3d_workspace_bytes) and a HIP
 * stream (NULL: the default stream); fills the rest state w_i.  Synchronises. */
int lbm3d_bind(lbm3d_t* h, void* device_workspace, size_t bytes, void* hip_stream);

/* Force schemes of the three-dimensional lattice: LBM_FORCE_MEA_A, LBM_FORCE_MEA_B,
 * LBM_FORCE_DRTT and LBM_FORCE_SI of lbm.h (DRTT-post is two-dimensional only). */
#define LBM3D_FORCE_ALL 15u

/* Enqueue n >= 0 steps.  force_scheme: LBM_FORCE_* bits; with any bit set every step
 * appends one row to the ring (LBM_EOVERFLOW, nothing enqueued, when it cannot hold
 * them: read the rows first). */
int lbm3d_step(lbm3d_t* h, int32_t n, uint32_t force_scheme);

/* Copy out the rows recorded since the last call (oldest first) into out
 * [max_rows][4][3] (host); *got = rows written.  LBM_ENONFINITE when a requested force
 * is NaN or infinite (the rows are still written). */
int lbm3d_forces(lbm3d_t* h, double* out, int64_t max_rows, int64_t* got);

/* Populations f (not deviations) as [27][nz][ny][nx] FP64 host arrays; solid nodes
 * read what they hold.  Synchronise. */
int lbm3d_get_populations(lbm3d_t* h, double* out);
int lbm3d_set_populations(lbm3d_t* h, const double* in);

/* Body links as (node index (z*ny + y)*nx + x, direction) pairs in (z, y, x,
 * direction) order into out [cap][2]; *n = their number. */
int lbm3d_get_links(const lbm3d_t* h, int64_t* out, int64_t cap, int64_t* n);

/* Rigid motion of the body (not in the paper's runs; the moving-wall bounce-back of
 * Sec. II on the body links): translation u[3], angular velocity omega[3] about the
 * point centre[3] (host arrays, copied), so a link whose half-way point is x_w sees the
 * wall velocity u_w = u + omega x (x_w - centre), and the population it returns gains
 * 2 w_i rho_w (c_i . u_w) / c_s^2.  The mask does not move.  A and B take the returned
 * population in their two-term form; DRTT and SI apply unchanged.  All zero (the
 * default) is a body at rest.  Applies from the next lbm3d_step (the motion travels as
 * a kernel argument).  LBM_EINVAL for null or non-finite vectors. */
int lbm3d_set_body_motion(lbm3d_t* h, const double* u, const double* omega,
                          const double* centre);

/* A body that moves through the grid (not in the paper's runs; the bounce-back of
 * Sec. II on the links of each mask), as lbm_set_mask in two dimensions: replace the
 * body mask ([nz][ny][nx] bytes, 0 fluid / 1 solid, host, copied), and the control
 * volume when `box` is non-null (six ints as in lbm3d_grid; it can be moved or
 * resized, not added or removed), between two steps.  Every recorded step keeps the
 * geometry it was taken with (the J(t+1) of the last step before the change was taken
 * under the old mask and box); the momentum that changes hands with the nodes the body
 * covers or uncovers enters no estimator and is returned in impulse[3] (host, may be
 * NULL): the momentum of the covered nodes minus that of the refilled ones.  Uncovered
 * nodes are refilled with the equilibrium at the rigid-body velocity of
 * lbm3d_set_body_motion at the node and the mean density of their lattice neighbours
 * that are fluid in both masks (rho_w when none is; a neighbour across a periodic edge
 * wraps, one outside another edge does not count).  The motion's centre is not
 * advanced by the library.  Bound handles: synchronises the stream first, uses the idle
 * state buffer as scratch and refills it with the rest state, synchronises again.
 * LBM_EINVAL: mask values other than 0/1, a box that is not admissible for the new
 * mask, a box added or removed; LBM_ENOMEM: the new mask needs more force slots than
 * twice those at create (plus a margin), or a larger control-volume sweep than at
 * create.  On these errors nothing changes.  On LBM_EHIP the state is undefined. */
int lbm3d_set_mask(lbm3d_t* h, const uint8_t* solid_mask, const int32_t* box,
                   double* impulse);

/* Checkpoint as in lbm.h: the exact stored state (raw storage bytes plus the step
 * counter) as an opaque host blob of lbm3d_state_bytes bytes; lbm3d_set_state accepts a
 * blob of a handle with the same grid size, precision and layout (else LBM_EINVAL).
 * Both synchronise the stream; LBM_ESTATE before bind. */
int lbm3d_state_bytes(const lbm3d_t* h, size_t* bytes);
int lbm3d_get_state(lbm3d_t* h, void* blob, size_t cap);
int lbm3d_set_state(lbm3d_t* h, const void* blob, size_t n);

/* Put every node back in the rest state w_i, zero the step counter and empty the force
 * ring.  Synchronises the stream. */
int lbm3d_reset(lbm3d_t* h);

/* Replace the relaxation time tau_lb (> 1/2, finite) or the inlet plane ([nz][ny] host
 * values, copied; only with an inlet) of a handle; later steps use the new values.
 * lbm3d_set_inlet synchronises the stream when the handle is bound. */
int lbm3d_set_tau(lbm3d_t* h, double tau);
int lbm3d_set_inlet(lbm3d_t* h, const double* uin);

int lbm3d_get_info(const lbm3d_t* h, lbm3d_info* info);
void lbm3d_destroy(lbm3d_t* h);
/* Last error message of h, or of the last failed lbm3d_create when h is NULL. */
const char* lbm3d_last_error(const lbm3d_t* h);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */

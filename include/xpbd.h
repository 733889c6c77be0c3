/* xpbd.h - C ABI of the MI355X (gfx950) differentiable XPBD library.
 *
 * The library runs the XPBD forward step of DiffXPBD (Stuyck & Chen,
 * arXiv 2301.01396) and its exact adjoint on one GPU.
 *
 *   Forward (Sec. 3.1, Eq. xpbd and the position update after it, inside the
 *   implicit-Euler step of Eq. xpbdUpdateRule): each frame of length dt is
 *   split into S substeps of length h = dt / S.  Each substep predicts
 *   v += h (g + w f_ext), x += h v, resets the multipliers, runs K
 *   Gauss-Seidel iterations over the ordered independent constraint sets of
 *   the schedule, projecting each constraint j with
 *       alpha~ = alpha_j / h^2,  D = sum_k w_k |grad_k C|^2 + alpha~,
 *       dlambda = (-C - alpha~ lambda_j) / D,  lambda_j += dlambda,
 *       x_k += w_k dlambda grad_k C,
 *   then sets v = (x - x_prev) / h.
 *
 *   Adjoint: the exact reverse-mode derivative of that computation, through
 *   every substep, iteration and projection (the adjoint-state recurrence of
 *   the supplemental Sec. A, Eq. adjoint_state, with the gradient rule
 *   Eq. gradientRule, applied to each projection using the partial
 *   derivatives of Sec. 4.3).  The adjoint reads a record of every
 *   projection's inputs: the forward keeps it for the whole rollout or for
 *   its last frames when memory allows (tape_mode 0, 3, 4), and the adjoint
 *   recomputes the other frames from per-frame checkpoints, holding one
 *   frame's record (tape_mode 1) or one substep's (tape_mode 2) at a time
 *   (Sec. 7 notes the linear-in-steps memory of storing everything).
 *
 * Constraint types:
 *   XPBD_DIST    C = |x_i - x_j| - L, L the rest length.
 *   XPBD_BEND    signed dihedral angle minus its rest value, hinge (v0, v1),
 *                wing v2 of triangle (v0, v1, v2), wing v3 of (v1, v0, v3)
 *                (the paper's discrete bending term, Sec. 5.1).
 *   XPBD_TET     stable Neo-Hookean in XPBD form (Sec. 5.2): deviatoric
 *                C_D = sqrt(tr F^T F) then hydrostatic C_H = det F - gamma,
 *                F = Ds Dm^-1, alpha_D = 1/(mu V), alpha_H = 1/(lambda V),
 *                gamma = 1 + mu/lambda (or 1, option), separate multipliers.
 *   XPBD_CONTACT one per vertex listed in the contact sets: a compliant
 *                collision constraint keeping the separation from a sphere
 *                (c, R) at least the thickness tau (Sec. 4.5):
 *                C = |x - c| - R - tau, projected only while C < 0.
 *
 * Conventions for every entry point:
 *   - Returns xpbd_status; never throws; never frees caller memory.
 *   - Host arrays passed to xpbd_create are copied; the caller may free
 *     them when it returns.
 *   - Device pointers passed to forward/adjoint/goal belong to the caller and
 *     must stay valid (and unchanged, for parameters) until the stream has
 *     completed the call and, for parameters, until the matching adjoint.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t, NULL =
 *     the default stream).  A kernel fault surfaces at a later call as
 *     XPBD_ERR_HIP.
 *   - Vectors are row-major [V][3] (or [F][V][3]) in the context's dtype.
 *   - One context per host thread at a time.  On error, xpbd_last_error
 *     returns a message.
 */
#ifndef XPBD_H
#define XPBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xpbd_ctx_s* xpbd_ctx;

typedef enum {
  XPBD_OK = 0,
  XPBD_ERR_INVALID = 1,   /* bad argument, mesh, or schedule */
  XPBD_ERR_OOM = 2,       /* allocation failed or hbm_budget_bytes exceeded */
  XPBD_ERR_HIP = 3,       /* HIP runtime error (includes earlier async faults) */
  XPBD_ERR_STATE = 4,     /* adjoint without a matching forward */
  XPBD_ERR_NONFINITE = 5, /* non-finite input parameter */
  XPBD_ERR_SOLVER = 6     /* iterative solve failed (system not positive definite) */
} xpbd_status;

typedef enum { XPBD_F32 = 0, XPBD_F64 = 1 } xpbd_dtype;
typedef enum { XPBD_DIST = 0, XPBD_BEND = 1, XPBD_TET = 2, XPBD_CONTACT = 3, XPBD_TRI = 4, XPBD_BODY = 5 } xpbd_ctype;

typedef struct {
  int32_t n_verts;
  const double* rest_pos;   /* host [V][3]: rest shape (rest lengths, angles, Dm) */
  const double* inv_mass;   /* host [V]: inverse mass w, 0 = pinned (infinite mass) */
} xpbd_mesh_desc;

typedef struct {
  int32_t n_dist; const int32_t* dist_v;   /* host [n_dist][2] */
  int32_t n_bend; const int32_t* bend_v;   /* host [n_bend][4] hinge v0 v1, wings v2 v3 */
  int32_t n_tet;  const int32_t* tet_v;    /* host [n_tet][4], positive rest volume */
  const double* tet_nu;                    /* host [n_tet] Poisson ratio (fixed) */
  int32_t contact;                         /* 1: contact sets may list free vertices */
  double contact_thickness;                /* tau */
  double contact_compliance;               /* alpha of every contact constraint */
  /* Material clusters (Sec. 5.2: an object made of a few materials, each a
   * pair of Lame parameters shared by its tets).  0 = every tet has its own
   * parameters.  With n_materials > 0, tet_material (host [n_tet], copied)
   * gives each tet's material in [0, n_materials), and the tet parameters of
   * xpbd_params and their gradients in xpbd_grads are per material
   * ([n_materials]) instead of per tet; a material's gradient is the sum over
   * its tets, reduced in a fixed order (bitwise reproducible).  A material
   * with no tets gets a zero gradient. */
  int32_t n_materials;
  const int32_t* tet_material;
  /* Orthotropic StVK membrane triangles (Sec. 5.1): one vector constraint
   * C = (E_uu, E_vv, 2 E_uv) per triangle, E = (F^T F - I)/2 the Green
   * strain of F = [x1-x0, x2-x0] Dm^-1, Dm the triangle's edges in the warp
   * / weft (u, v) material frame given by tri_uv (host [n_tri][3][2], the
   * corners' (u, v); zero material-space area -> XPBD_ERR_INVALID).  Its
   * compliance is the 3x3 matrix alpha = (A K)^-1, A = material-space area,
   * K = [[C00, C01, 0], [C01, C11, 0], [0, 0, C22]] from xpbd_params.tri_coef;
   * each projection solves the 3x3 system for the three multipliers.
   * Membrane sets run as one launch per set, in the persistent kernel or in
   * LDS groups; the implicit adjoint does not take them. */
  int32_t n_tri;
  const int32_t* tri_v;       /* host [n_tri][3] */
  const double* tri_uv;       /* host [n_tri][6] */
  /* Body collider (Sec. 4.5 contacts with the body; Sec. 5.3 gradients to
   * it): a triangle mesh whose vertex positions are a control
   * (xpbd_params.body_x, kinematic, constant over a rollout); triangles
   * oriented so (b - a) x (c - a) points out of the body.  Items of
   * XPBD_BODY sets are free cloth vertices (each at most once).  At the start
   * of every substep, after the prediction, each item is paired with the
   * body triangle closest to it (point-triangle distance in FP64, ties to the
   * lower triangle index) if that distance is at most body_radius; during
   * the substep it keeps C = n^ . (x - a) - body_thickness >= 0 against the
   * plane of that triangle (n^ the unit normal), compliance body_compliance,
   * projected only while C < 0.  The gradient reaches the body vertices
   * (xpbd_grads.body_x), summed with FP64 atomics (rounding may differ in
   * the last bits between runs).  Body-contact sets run one launch per set or
   * in LDS groups; the persistent kernel (launch_mode 2), packs and the
   * implicit adjoint refuse them (XPBD_ERR_INVALID). */
  int32_t n_body_verts;
  int32_t n_body_tris;
  const int32_t* body_tris;   /* host [n_body_tris][3] */
  double body_thickness;      /* tau (m) */
  double body_compliance;     /* alpha (m/N), >= 0 */
  double body_radius;         /* pairing search radius (m), > 0 */
} xpbd_constraint_desc;

/* One Gauss-Seidel iteration visits these sets in order.  Set s has type
 * set_type[s] and items set_items[set_offsets[s] .. set_offsets[s+1]):
 * constraint indices of that type (for XPBD_TET one item is both the D and
 * the H projection; for XPBD_CONTACT and XPBD_BODY an item is a vertex
 * index; for XPBD_TRI a membrane triangle).  Within a
 * set no vertex may appear twice (the set is independent), every distance,
 * bending and tet constraint must appear exactly once in the schedule, and a
 * contact vertex at most once and only if its inverse mass is > 0.
 * Otherwise xpbd_create returns XPBD_ERR_INVALID. */
/* Optional LDS groups (a performance hint that never changes results):
 * group g covers the consecutive sets [group_sets[2g], group_sets[2g+1])
 * and gives a patch id (>= 0) for every vertex in group_patch[g * V + v].
 * Every constraint of the group's sets must have all its vertices in one
 * patch (else XPBD_ERR_INVALID); the library may then run the whole group
 * as one launch, one workgroup per patch with the patch's vertices and
 * records in LDS, which computes exactly what the sets compute one by one.
 * Groups must not overlap and hold at most 64 sets. */
typedef struct {
  int32_t n_sets;
  const int32_t* set_type;     /* host [n_sets] xpbd_ctype */
  const int64_t* set_offsets;  /* host [n_sets + 1] */
  const int32_t* set_items;    /* host [set_offsets[n_sets]] */
  int32_t n_groups;            /* 0 = none */
  const int32_t* group_sets;   /* host [n_groups][2] */
  const int32_t* group_patch;  /* host [n_groups][V] */
} xpbd_schedule_desc;

typedef struct {
  double dt;                 /* frame length (> 0) */
  int32_t substeps;          /* S >= 1 */
  int32_t iterations;        /* K >= 0 */
  double gravity[3];
  xpbd_dtype dtype;          /* arithmetic and storage type of the state */
  size_t hbm_budget_bytes;   /* 0 = no limit; else XPBD_ERR_OOM past it */
  int32_t tet_gamma_one;     /* 1: gamma = 1 (the formula as printed); 0: 1 + mu/lambda */
  int32_t tape_mode;         /* record of projection inputs for the adjoint:
                                0 auto: the whole rollout during a forward flagged
                                  XPBD_FWD_FOR_ADJOINT if it fits, else per frame,
                                  else per substep;
                                1 recompute each frame from its checkpoint, record
                                  the whole frame;
                                2 recompute one substep at a time (least memory);
                                3 record the whole rollout during the forward (needs
                                  XPBD_FWD_FOR_ADJOINT; XPBD_ERR_OOM if it does not fit);
                                4 the forward flagged XPBD_FWD_FOR_ADJOINT records the
                                  last frames, as many as fit (at most record_frames),
                                  the adjoint recomputes the others per frame.
                                Mode 0 falls back from the whole rollout to mode 4's
                                split, then to per-frame recomputation. */
  int32_t launch_mode;       /* 0 auto, 1 one kernel launch per independent set,
                                2 persistent: one cooperative launch runs a whole frame's
                                  sets with a grid-wide barrier between sets */
  int32_t persistent_blocks; /* workgroups of the persistent launch, 0 = sized to the
                                largest set (capped at what the device co-schedules) */
  int32_t block_size;        /* workgroup size of the one-launch-per-set kernels: a power
                                of two in [64, 1024], 0 = 256; results do not depend on it */
  int32_t group_records;     /* LDS groups: 0 or 1 = each patch's constraint entries and
                                multiplier state staged in LDS with its vertices; 2 = only
                                the vertex tile in LDS, entries read and state read and
                                written in place in global memory (small LDS, many patches
                                per CU); results do not depend on it */
  int32_t group_block;       /* workgroup size of the LDS group kernels, a power of two in
                                [64, 256], 0 = 256 */
  int32_t record_frames;     /* tape_mode 4: most final frames the forward records, 0 = as
                                many as fit */
  int32_t serial_adjoint;    /* 0: while the adjoint reverses a frame on a stream of the
                                library's, the recomputation of an earlier frame runs on
                                another (both default priority, created on first use and
                                destroyed with the context), ordered by events, when the
                                record holds two frames or more; 1: every step on the
                                call's stream.  Results do not depend on it */
  int32_t record_kind;       /* what the adjoint's record holds: 0 = the inputs of every
                                projection (vertex differences and multiplier); 1 = a
                                snapshot of each LDS group launch (the patch's positions and
                                multipliers as the launch finds them, about 4.3x smaller on
                                grid cloths), from which the reverse replays the launch's
                                sets in LDS to rebuild those inputs (the same arithmetic,
                                so results are bitwise those of 0).  1 needs every set in an
                                LDS group and not launch_mode 2 (else XPBD_ERR_INVALID);
                                packs refuse such contexts */
} xpbd_options;

/* Validate and upload a problem.  Computes rest lengths, rest dihedral
 * angles, Dm^-1 and rest volumes from rest_pos; reorders the items of each
 * set (order inside an independent set does not change the result).
 * Errors: XPBD_ERR_INVALID (indices out of range, a set that is not
 * independent, a constraint missing from or repeated in the schedule,
 * zero-length edge, degenerate rest triangle, non-positive rest volume,
 * bad options), XPBD_ERR_OOM, XPBD_ERR_HIP.  *out is NULL on error. */
xpbd_status xpbd_create(const xpbd_mesh_desc* mesh, const xpbd_constraint_desc* cons,
                        const xpbd_schedule_desc* schedule, const xpbd_options* opt,
                        xpbd_ctx* out);
xpbd_status xpbd_destroy(xpbd_ctx ctx);

/* Controls (Sec. 4.4): device arrays in the context dtype; NULL compliance
 * arrays mean 0 (rigid).  Tets take either Young's moduli (with the Poisson
 * ratios given at create) or Lame parameters: tet_mu and tet_lambda, when
 * given, replace tet_E and the Poisson ratios (Sec. 5.2 optimises over them
 * through a^2 = mu, b^2 = lambda); one of the two is required when there
 * are tets. */
typedef struct {
  const void* dist_compliance;   /* device [n_dist] alpha (m/N) */
  const void* bend_compliance;   /* device [n_bend] alpha */
  const void* tet_E;             /* device [n_tet] Young's modulus (Pa); [n_materials] with
                                    material clusters (the same for tet_mu, tet_lambda) */
  const void* f_ext;             /* device [F][V][3] per-vertex force, or NULL */
  double sphere[4];              /* cx, cy, cz, R of the contact sphere */
  const void* tet_mu;            /* device [n_tet] first Lame parameter (Pa), or NULL */
  const void* tet_lambda;        /* device [n_tet] second Lame parameter (Pa), or NULL */
  const void* tri_coef;          /* device [n_tri][4] membrane (C00, C01, C11, C22) (N/m), K
                                    positive definite (else XPBD_ERR_NONFINITE); required
                                    when there are membrane triangles */
  const void* body_x;            /* device [n_body_verts][3] body vertex positions (ctx dtype);
                                    required when there are body-contact sets */
} xpbd_params;

/* Roll out n_frames frames from (x0, v0) (device [V][3]; v0 of pinned
 * vertices is ignored).  Writes the end-of-frame positions to x_frames
 * (device [F][V][3], may be NULL) and the final state to x_final, v_final
 * (device [V][3], may be NULL).  Keeps per-frame checkpoints for
 * xpbd_adjoint; with flags & XPBD_FWD_FOR_ADJOINT it may also keep the
 * record of every projection's inputs (tape_mode 0, 3 or 4) so that the
 * adjoint needs no recomputation.  Errors: XPBD_ERR_INVALID, XPBD_ERR_OOM,
 * XPBD_ERR_NONFINITE, XPBD_ERR_HIP. */
#define XPBD_FWD_FOR_ADJOINT 1
xpbd_status xpbd_forward(xpbd_ctx ctx, const void* x0, const void* v0, const xpbd_params* p,
                         int32_t n_frames, void* x_frames, void* x_final, void* v_final,
                         int32_t flags, void* stream);

/* Gradient outputs (device).  Any pointer may be NULL.  Parameter gradients
 * are accumulated and returned in FP64; state-shaped ones in the ctx dtype.
 * Pinned vertices get zero v0 and f_ext gradients.  When dist_compliance and
 * bend_compliance are both NULL, the reverse of the LDS groups without tets
 * or membranes leaves those constraints' compliance adjoints out (no reads,
 * writes or arithmetic for them: less memory traffic and fewer registers);
 * the other outputs are bitwise the same either way. */
typedef struct {
  double* dist_compliance;   /* [n_dist] dL/dalpha */
  double* bend_compliance;   /* [n_bend] dL/dalpha */
  double* tet_E;             /* [n_tet] dL/dE (nu fixed; Young's moduli given); [n_materials]
                                with material clusters (the same for tet_mu, tet_lambda) */
  void* f_ext;               /* [F][V][3] dL/df_ext */
  void* x0;                  /* [V][3] dL/dx0 */
  void* v0;                  /* [V][3] dL/dv0 */
  double* sphere;            /* [4] dL/d(cx, cy, cz, R) */
  double* tet_mu;            /* [n_tet] dL/dmu (Lame parameters given), through both
                                compliances and gamma = 1 + mu/lambda */
  double* tet_lambda;        /* [n_tet] dL/dlambda */
  double* tri_coef;          /* [n_tri][4] dL/d(C00, C01, C11, C22) */
  double* body_x;            /* [n_body_verts][3] dL/dx_body */
} xpbd_grads;

/* Exact adjoint of the preceding xpbd_forward on this context for a goal
 * with gradient dLdx_frames (device [F][V][3], row f = dL/dx(end of frame
 * f); frames with frame_mask[f] == 0 are not read; frame_mask is host [F]
 * or NULL = all) plus dLdv_final (device [V][3] or NULL).  `p` must be the
 * same parameters, with unchanged contents, as in that forward.  Stream
 * ordered like every call: work the call puts on the library's own streams
 * (the recomputation beside the reverse, see serial_adjoint) starts after
 * the call's stream reaches the call and has finished when the call's
 * stream passes the end of the call.
 * Errors: XPBD_ERR_STATE (no forward, or different parameter pointers),
 * XPBD_ERR_INVALID, XPBD_ERR_OOM, XPBD_ERR_HIP. */
xpbd_status xpbd_adjoint(xpbd_ctx ctx, const xpbd_params* p, const void* dLdx_frames,
                         const uint8_t* frame_mask, const void* dLdv_final,
                         const xpbd_grads* out, void* stream);

/* Goal of Sec. 4.1 with W = I on the frames where frame_mask[f] != 0 and
 * beta = 0: phi = 1/2 sum_f |x(f) - x*(f)|^2 reduced in FP64 into *loss
 * (device double), and dphi/dx(f) = x(f) - x*(f) on masked frames, 0
 * elsewhere, into dLdx (device [F][V][3], may be NULL). */
xpbd_status xpbd_goal_l2(xpbd_ctx ctx, const void* x_frames, const void* targets,
                         const uint8_t* frame_mask, int32_t n_frames, double* loss,
                         void* dLdx, void* stream);

/* The same goal with a diagonal weight matrix W (Sec. 4.1), one weight per
 * vertex: phi = 1/2 sum_f sum_v w_v^2 |x_v(f) - x*_v(f)|^2 on masked frames
 * and dphi/dx_v(f) = w_v^2 (x_v(f) - x*_v(f)).  vertex_weight is device
 * FP64 [V]; w_v = 0 leaves vertex v out (e.g. a goal on the boundary
 * surface only).  NULL weights = xpbd_goal_l2. */
xpbd_status xpbd_goal_weighted(xpbd_ctx ctx, const void* x_frames, const void* targets,
                               const uint8_t* frame_mask, const double* vertex_weight, int32_t n_frames,
                               double* loss, void* dLdx, void* stream);

/* xpbd_goal_weighted for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, with the
 * reduction's partial sums in a static device array of the library (16 MiB
 * per GPU, held until the process ends) instead of a buffer the context
 * allocates.  It calls no hipMalloc or hipFree.  Limit: ceil(3 V / 256) *
 * n_frames <= 2^21 partial sums (for example 20 frames of 8.4M vertices),
 * else XPBD_ERR_INVALID.  The current device must be the one the context was
 * created on (else XPBD_ERR_INVALID).  Every call on a GPU shares its array:
 * calls that overlap on one GPU (on different streams, or from different
 * contexts or threads) race and must be ordered by the caller. */
xpbd_status xpbd_goal_weighted_noalloc(xpbd_ctx ctx, const void* x_frames, const void* targets,
                                       const uint8_t* frame_mask, const double* vertex_weight, int32_t n_frames,
                                       double* loss, void* dLdx, void* stream);

/* Implicit adjoint of Sec. 4.2 (Eq. adjointXPBD) for the preceding
 * xpbd_forward, the paper's own derivative: each substep's projection is
 * taken as converged, x = y + M^-1 sum_j grad C_j lambda_j with lambda_j =
 * -C_j / alpha~_j at the substep's end state (contacts active where C < 0
 * there), and the substep's adjoint solves (I - M^-1 K)^T w = xbar with
 * K = sum_j (lambda_j Hess C_j - grad C_j grad C_j^T / alpha~_j) (Sec. 4.3
 * partials).  On the free vertices this is the symmetric system (M - K) y =
 * xbar, w = M y, solved by Jacobi-preconditioned conjugate gradients in FP64
 * with a matrix-free operator.  With cg->pd_projection each constraint's
 * block -lambda_j Hess C_j is first replaced by its positive semidefinite
 * part (eigenvalues below zero dropped; Sec. 4.3, Positive Definite Projection), which makes the system
 * positive definite; without it, a system that is not positive definite
 * fails with XPBD_ERR_SOLVER.
 * Then vbar = h w (free vertices), dL/df_ext += h w_inv vbar, xbar = w -
 * vbar_old / h, and dL/dalpha_j += (grad C_j . y)(-lambda_j / alpha~_j) / h^2.
 * Frames are recomputed from the forward's checkpoints.  It differs from
 * xpbd_adjoint, the exact derivative of the iterated rollout, wherever the
 * iterations have not converged or the constraint gradients turn along the
 * iteration path.
 * Outputs: dist / bend compliance, f_ext, x0, v0 (as xpbd_adjoint);
 * out->tet_E and out->sphere must be NULL.  Every active constraint needs a
 * positive compliance (else XPBD_ERR_INVALID).  `cg` gives the iteration
 * limit and relative residual tolerance per substep and receives the
 * iteration counts and the worst relative residual reached. */
typedef struct {
  int32_t max_iterations;       /* in: CG iterations per substep, >= 1 */
  double rel_tolerance;         /* in: stop at |r| <= rel_tolerance |xbar| */
  int32_t pd_projection;        /* in: 1 = project each constraint's block -lambda Hess C
                                   to positive semidefinite first (Sec. 4.3, Positive Definite Projection) */
  int64_t total_iterations;     /* out */
  int32_t max_iterations_used;  /* out: most iterations one substep took */
  double worst_rel_residual;    /* out */
} xpbd_cg;
xpbd_status xpbd_adjoint_implicit(xpbd_ctx ctx, const xpbd_params* p, const void* dLdx_frames,
                                  const uint8_t* frame_mask, xpbd_cg* cg, const xpbd_grads* out,
                                  void* stream);

typedef struct {
  int32_t n_verts, n_dist, n_bend, n_tet, n_contact, n_sets;
  int64_t projections_per_iteration;   /* tets count D and H; contacts counted as evaluated */
  int64_t device_bytes;                /* device memory held by the context now */
  int64_t tape_bytes_per_iteration;    /* record of projection inputs, one iteration */
  int32_t tape_mode;                   /* mode the last adjoint used (1 frame, 2 substep, 3 forward
                                          record, 4 forward record of the last frames) */
  int32_t persistent;                  /* 1 if frames run as persistent launches */
  int32_t persistent_blocks;           /* their workgroup count (0 before the first) */
  int32_t n_groups;                    /* LDS groups given */
  int32_t n_groups_lds;                /* of which run as one LDS launch each */
  int32_t max_group_lds_bytes;         /* largest LDS footprint of those launches */
  int32_t n_materials;                 /* material clusters, 0 = per-tet parameters */
  int32_t n_tri;                       /* membrane triangles */
  int32_t n_body_contacts;             /* body-contact items */
  int32_t forward_record_frames;       /* final frames whose record the last forward kept */
  int32_t adjoint_streams;             /* streams the last adjoint ran on: 2 when earlier frames
                                          were recomputed beside the reverse, 1 otherwise, 0 none */
} xpbd_info;
xpbd_status xpbd_get_info(xpbd_ctx ctx, xpbd_info* info);

/* Kernel timing for measurement: with on = n > 0, one in n launches of the
 * projection and reverse kernels (plain mode, LDS groups) or of the
 * per-frame persistent kernels, picked by a hash of the launch count (so no
 * launch pattern aliases with n), is bracketed by HIP events on the call's
 * stream (0 = off).  xpbd_profile_read synchronises them and returns, per kernel family
 * (index 2 * type: forward projections of that type, 2 * type + 1: their
 * reverse, with body contacts counted with the sphere's at 6 and 7; 8:
 * persistent forward frame, 9: persistent reverse frame,
 * 10: LDS group forward, 11: LDS group reverse, 12: membrane forward,
 * 13: membrane reverse), the number of timed launches, their total
 * milliseconds and the projections they processed, then resets the counts. */
xpbd_status xpbd_profile_enable(xpbd_ctx ctx, int32_t on);
xpbd_status xpbd_profile_read(xpbd_ctx ctx, int64_t launches[14], double ms[14], int64_t items[14]);

/* ---------------------------------------------------------------- packs
 * A pack runs jobs on many contexts (meshes of any size and constraint mix)
 * together: each round advances every job in it by one frame of its forward
 * rollout or of its adjoint, and every launch of the round serves the same
 * step (substep, iteration, position in the schedule) of all of them, so
 * one launch covers many meshes.  Jobs join at the next round after
 * xpbd_pack_add and leave when done; each job's results are bitwise those of
 * running its context alone with xpbd_forward, xpbd_goal_l2 and
 * xpbd_adjoint (the pack always uses one launch per set, which computes what
 * every launch_mode computes).  With XPBD_PACK_GRAPHS a round's launches are
 * captured once in a HIP graph while the pack's jobs and phases stay the
 * same, and replayed for every further round.
 *
 * A job is a forward rollout of `n_frames` frames from (x0, v0) with
 * `params` (as xpbd_forward), writing x_frames / x_final / v_final (any may
 * be NULL; x_frames is required with an adjoint).  If `targets` is not NULL
 * the job then computes the goal of xpbd_goal_l2 (frames with frame_mask[f]
 * != 0; NULL = all) into *loss (device double, may be NULL) and its exact
 * adjoint into `grads` (as xpbd_adjoint, with dLdv_final as its dLdv_final).
 * The adjoint replays the forward's record of every projection if it fits
 * the context's budget (tape_mode 0 or 3), else recomputes each frame from
 * its checkpoint (tape_mode 0 or 1); tape_mode 2 is not available in packs.
 *
 * Every context in a pack must have the pack's dtype and the same substeps
 * and iterations as the pack's first job; a context serves one job at a
 * time.  Device pointers of a job must stay valid until the job is reported
 * done and the stream has reached that point.  Calls on one pack are ordered
 * on the stream passed to them; use one stream per pack.  The context's
 * earlier forward record is invalidated by a job (xpbd_adjoint afterwards
 * returns XPBD_ERR_STATE). */
typedef struct xpbd_pack_s* xpbd_pack;

typedef struct {
  const void* x0;             /* device [V][3] */
  const void* v0;             /* device [V][3] */
  xpbd_params params;
  int32_t n_frames;           /* F >= 1 */
  void* x_frames;             /* device [F][V][3] or NULL */
  void* x_final;              /* device [V][3] or NULL */
  void* v_final;              /* device [V][3] or NULL */
  const void* targets;        /* device [F][V][3] goal targets, NULL = no adjoint */
  const uint8_t* frame_mask;  /* host [F] (copied), NULL = every frame */
  const void* dLdv_final;     /* device [V][3] or NULL */
  double* loss;               /* device double or NULL */
  xpbd_grads grads;
} xpbd_job;

typedef struct {
  int32_t active_jobs;        /* jobs in the pack now */
  int64_t rounds;             /* rounds run so far */
  int64_t launches;           /* kernel launches issued directly */
  int64_t graph_launches;     /* rounds replayed from a captured graph */
  int64_t graph_captures;     /* graphs captured (once per change of jobs or phases) */
  int32_t last_round_launches;/* launches in the current round plan */
} xpbd_pack_stats;

#define XPBD_PACK_GRAPHS 1
/* block_size: workgroup size of the pack's set and vertex launches, one
 * item per thread: 64, 128 or 256 (0 = 256); results do not depend on it.
 * Errors: XPBD_ERR_INVALID (bad dtype, flags or block size), XPBD_ERR_OOM. */
xpbd_status xpbd_pack_create(xpbd_dtype dtype, int32_t flags, int32_t block_size, xpbd_pack* out);
/* Synchronises the pack's last stream, then frees the pack (not its contexts). */
xpbd_status xpbd_pack_destroy(xpbd_pack pack);
/* Validate a job, gather and check its parameters, allocate its context's
 * checkpoints and record, load (x0, v0), and queue it for the next round.
 * This work runs on a stream of the pack's own and waits only for itself
 * (and for the context's previous pack job, if that is still running), never
 * for the pack's rounds; `stream` is not used.  The context must have no
 * other work in flight.  *job_id (> 0) identifies the job in xpbd_pack_run.
 * Errors: XPBD_ERR_INVALID (mismatched dtype / substeps / iterations,
 * context already in a job, bad job), XPBD_ERR_NONFINITE, XPBD_ERR_OOM
 * (record does not fit), XPBD_ERR_HIP. */
xpbd_status xpbd_pack_add(xpbd_pack pack, xpbd_ctx ctx, const xpbd_job* job, void* stream, int64_t* job_id);
/* Run up to max_rounds rounds on `stream`, returning after the first round
 * in which any job finished.  The ids of finished jobs (at most `cap`; the
 * rest are reported by the next call) are written to done_ids and their
 * count to *n_done; their outputs are complete once the stream reaches the
 * end of this call.  Errors: XPBD_ERR_HIP (a kernel or graph failure; the
 * pack's jobs are then invalid), XPBD_ERR_INVALID. */
xpbd_status xpbd_pack_run(xpbd_pack pack, int32_t max_rounds, void* stream, int64_t* done_ids, int32_t cap,
                          int32_t* n_done);
xpbd_status xpbd_pack_get_stats(xpbd_pack pack, xpbd_pack_stats* stats);
const char* xpbd_pack_last_error(xpbd_pack pack);

const char* xpbd_last_error(xpbd_ctx ctx);
const char* xpbd_status_string(xpbd_status s);

#ifdef __cplusplus
}
#endif
#endif /* XPBD_H */

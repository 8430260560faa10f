/*
 * fr.h -- C ABI of the MI355X flux-reconstruction library (libfrmi.so).
 *
 * The library evaluates the semi-discrete right-hand side du/dt = R(u) of the
 * compressible Navier-Stokes equations discretised with flux reconstruction
 * (DG correction functions) and flux anti-aliasing, and advances it with
 * classical RK4, following Akkurt, Witherden & Vincent, "Cache Blocking for
 * Flux Reconstruction: Extension to Navier-Stokes Equations and
 * Anti-aliasing":
 *   - governing equations and fluxes: section 2.1, eqs. gov, ucons, fluxe,
 *     fluxv; first-order system eq. govq; mapping eqs. transall, govqtrans;
 *   - FR steps: eqs. FR-disu, FR-conu, FR-qfinal, FR-gradcoru,
 *     FR-gradcoru_fpts, FR-comm_flux, FRfinal;
 *   - flux anti-aliasing: eqs. FR-uqpts, FR-gradcoru_qpts, FR-tdisfq,
 *     FR-tdivtpcorfq (section 2.1.1) and the operator matrices M0..M10 of
 *     section 2.2;
 *   - tensor-product factorisation of the anti-aliasing operators for
 *     hexahedra and prisms: section 4 and 4.1;
 *   - the kernel groups of section 6.1 (figure NSAAKG), realised as fused
 *     GPU kernels.
 *
 * Conventions
 *   - All functions return an fr_status (0 = FR_OK, negative = error) and never
 *     throw or abort; fr_last_error() gives a human-readable message.
 *   - A context is single-stream and not thread-safe.  Device work is enqueued
 *     on the context stream (the stream passed to fr_create, or the null
 *     stream) and is asynchronous unless stated otherwise.
 *   - State layout ("library layout"): all hexahedra first, then all prisms;
 *     within a type, elements in mesh order; per element the five conserved
 *     variables [rho, rho vx, rho vy, rho vz, E] (eq. ucons), each as N_u
 *     contiguous doubles in solution-point order.  I.e. per type an array
 *     (E_t, 5, N_u) of float64, row-major.
 *   - Solution points: hex GL(p+1)^3, index i + n(j + n k) (x fastest);
 *     prism = triangle nodes x GL(p+1), index t + N_t k.  Triangle nodes:
 *     Blyth-Pozrikidis construction on the Gauss-Legendre master grid.
 *   - Anti-aliasing quadrature: hex GL(p+3)^3; prism conical triangle rule
 *     with (p+1)^2 points (exact to degree 2p+1) x GL(p+3).
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx fr_ctx;

typedef enum {
  FR_OK = 0,
  FR_EINVAL = -1,        /* bad argument (null pointer, size, unsupported order, ...) */
  FR_ENOMEM = -2,        /* host or device allocation failed */
  FR_EDEVICE = -3,       /* a HIP call failed; see fr_last_error */
  FR_ESTATE = -4,        /* call out of order (e.g. no mesh yet) */
  FR_EUNSUPPORTED = -5   /* combination not built (e.g. order outside 1..4) */
} fr_status;

typedef enum { FR_HEX = 0, FR_PRISM = 1, FR_TET = 2, FR_PYR = 3 } fr_etype;
typedef enum {
  FR_MESH_HEX = 0,
  FR_MESH_PRISM = 1,
  FR_MESH_MIXED = 2,      /* hexahedra where z < 0, prisms elsewhere */
  FR_MESH_TET = 3,        /* six tetrahedra per cell */
  FR_MESH_PRISM_TET = 4,  /* prisms where y < 0, tetrahedra elsewhere */
  FR_MESH_HEX_WARP = 5,   /* kinds 0, 1, 2 on a warped grid: curved elements */
  FR_MESH_PRISM_WARP = 6,
  FR_MESH_MIXED_WARP = 7,
  FR_MESH_PYR = 8,        /* six pyramids per cell */
  FR_MESH_HEX_PYR = 9,    /* hexahedra where z < 0, pyramids elsewhere */
  FR_MESH_HEX_PYR_TET = 10, /* hexahedra, transition cells (pyramid + tetrahedra), tetrahedra */
  FR_MESH_HEX_PRISM_PYR_TET = 11 /* FR_MESH_HEX_PYR_TET with prisms where y < 0 above the hexahedra */
} fr_mesh_kind;
typedef enum { FR_PREC_FP64 = 0, FR_PREC_FP32 = 1 } fr_precision;
typedef enum { FR_FORM_FUSED = 0, FR_FORM_PLAIN = 1 } fr_form;

/* Physics and scheme parameters.
 *   gamma, prandtl, mu : perfect gas, constant viscosity (section 2.1)
 *   ldg_beta, ldg_tau  : LDG common solution / viscous flux parameters
 *                        (eq. FR-conu and the LDG flux of section 2.1);
 *                        beta = 0, tau = 0 gives BR1-type central fluxes
 *   pref               : constant reference pressure.  The energy is operated
 *                        on as E - pref/(gamma-1) and the constant pref*I
 *                        momentum flux is dropped (it has zero discrete
 *                        divergence); mathematically identical, it removes
 *                        the low-Mach cancellation.  0 = textbook form.
 *   rho_ref            : constant reference density (0 = none).  The
 *                        density is operated on as rho - rho_ref.  With
 *                        rho_ref > 0 the fused kernels on affine elements
 *                        also split the energy flux exactly as
 *                        v (E + p) = v (E' + p' - kap (rho - rho_ref))
 *                                    + kap rho v,
 *                        kap = gamma pref / ((gamma - 1) rho_ref): the first
 *                        part is O(1) at low Mach, the second is linear in
 *                        the state and its DG divergence is formed in double
 *                        precision (the same operator gives the mass-flux
 *                        divergence).  Mathematically identical; with
 *                        FR_PREC_FP32 it keeps single-precision rounding off
 *                        the O(gamma pref/(gamma-1)) energy flux.  Curved
 *                        elements use the shift only.
 *   prec               : FR_PREC_FP64: every step in double precision.
 *                        FR_PREC_FP32: state, reference subtraction, the
 *                        solution at the flux points, the mass-flux
 *                        divergence L(rho v), final RHS and RK accumulation
 *                        in double; the corrected gradients, anti-aliased
 *                        fluxes, projections and interface fluxes in float,
 *                        with face states exchanged as a float base per
 *                        face plus float deviations (so that face jumps
 *                        keep their digits).
 *   form               : FR_FORM_FUSED: three fused kernels per element type
 *                        (disu | volume group | interface group).
 *                        FR_FORM_PLAIN: the paper's unfused kernel sequence
 *                        with dense operator matrices (comparison path).
 *   flux_aa            : 1: flux anti-aliasing (the flux is evaluated at the
 *                        quadrature points and projected, section 2.1.1);
 *                        0: no anti-aliasing, the flux is evaluated at the
 *                        solution points (the paper's "AA off"
 *                        configuration), in the fused form (the plain form
 *                        reports FR_EUNSUPPORTED).
 *   surface_aa         : 1: surface-flux anti-aliasing as well (section
 *                        2.1.1, table "operatorms": the interface flux
 *                        points are replaced by the face quadrature points,
 *                        GL(p+3)^2 on quadrilateral faces), i.e. the paper's
 *                        "full AA" together with flux_aa = 1.  Requires
 *                        flux_aa = 1 and the fused form (else
 *                        FR_EUNSUPPORTED).  The state layout and the
 *                        flux-point arrays do not change: the common flux is
 *                        evaluated at the face quadrature points and lifted
 *                        through its projection onto the flux points.
 *                        0 (default): interface fluxes at the flux points. */
typedef struct {
  double gamma, prandtl, mu, ldg_beta, ldg_tau, pref;
  double rho_ref;  /* reference density, 0 = none */
  int prec;        /* fr_precision */
  int form;        /* fr_form */
  int flux_aa;     /* 1 (default) or 0 */
  int surface_aa;  /* 0 (default) or 1 */
} fr_physics;

/* Fill *ph with the Taylor-Green defaults: gamma 1.4, Pr 0.71, mu 1/1600,
 * beta 0.5, tau 0.1, pref 0, rho_ref 0, FP64, fused, flux anti-aliasing on,
 * surface-flux anti-aliasing off. */
void fr_physics_default(fr_physics* ph);

/* Create a context.  hip_stream: a hipStream_t or NULL (null stream).  No
 * device call is made here.  *out receives the context; free with
 * fr_destroy.  Errors: FR_EINVAL (null out/ph, non-physical parameters). */
fr_status fr_create(const fr_physics* ph, void* hip_stream, fr_ctx** out);

/* Build a periodic box mesh [lo,hi]^3 of nx*ny*nz cells at order p (1..4).
 * kind: FR_MESH_HEX (one hexahedron per cell), FR_MESH_PRISM (each cell split
 * along the diagonal of its x-z face into two prisms extruded along y),
 * FR_MESH_MIXED (hexahedra where the cell centre has z < 0, prisms
 * elsewhere; the interfaces are conforming quadrilaterals), FR_MESH_TET (six
 * tetrahedra per cell: the cube's Kuhn subdivision mirrored in x, so every
 * cell face is cut along the same diagonal as the prisms' y faces) and
 * FR_MESH_PRISM_TET (prisms where the cell centre has y < 0, tetrahedra
 * elsewhere; prism triangles meet tetrahedron faces), FR_MESH_PYR (six
 * pyramids per cell, one on each cell face with the apex at the cell centre)
 * and FR_MESH_HEX_PYR (hexahedra where the cell centre has z < 0, pyramids
 * elsewhere; pyramid bases meet hexahedron faces) and FR_MESH_HEX_PYR_TET (nz
 * >= 3: hexahedra in the layers k < nz/2, tetrahedron cells between, and in
 * layer nz/2 and the last layer transition cells of one pyramid on the face
 * towards the hexahedra and ten tetrahedra cut along the tetrahedron cells'
 * face diagonals), FR_MESH_HEX_PRISM_PYR_TET (all four types: that mesh where
 * the cell centre has y >= 0; where y < 0 hexahedra in the layers k < nz/2
 * and prisms above).  Tetrahedra and pyramids
 * have no tensor-product structure (the paper's factorisation does not
 * apply) and run on dense-operator kernels; they support the fused form with
 * or without flux anti-aliasing and the plain form, but not surface-flux
 * anti-aliasing (FR_EUNSUPPORTED).  Pyramids use the rational pyramid space
 * (trace Q_p on the base, P_p on the triangles) and, since that space is not
 * closed under differentiation, the weak form -Mass^-1 Dq^T W of the
 * divergence (equal to (M1 - M3 M2) M9 for the other types).  Host-side only: device buffers
 * are allocated and uploaded by the first call that needs them.  Element
 * numbering: cells in index order i + nx(j + ny k); a prism cell yields two
 * elements, a tetrahedron or pyramid cell six, a transition cell its pyramid
 * then ten tetrahedra.  FR_MESH_HEX_WARP, FR_MESH_PRISM_WARP,
 * FR_MESH_MIXED_WARP: the hex, prism and mixed meshes with curved
 * (non-affine) elements; every grid vertex x moves to
 * x + 0.2 h (sin y cos z, sin z cos x, sin x cos y) (h the cell size per
 * axis; periodic, so the mesh stays periodic and conforming) and each
 * element is the map of its moved vertices by its vertex shape functions
 * (trilinear for a hexahedron, triangle x line for a prism; bilinear, curved
 * quadrilateral faces).  The kernels evaluate the metrics at every point
 * from the vertices (fused form with flux anti-aliasing only).  Errors: FR_EINVAL (n < 1, hi <= lo,
 * unknown kind), FR_EUNSUPPORTED (p outside 1..4), FR_ESTATE (mesh already
 * built). */
fr_status fr_mesh_box(fr_ctx* c, int nx, int ny, int nz, double lo, double hi, int p, int kind);

/* Build a general conforming mesh of affine elements from caller vertices
 * (section 2.1: every element is the image of its reference element under
 * its own mapping, eqs. transall and govqtrans; here an affine one, fitted
 * to the element's vertices).  Faces are paired by their centroids modulo
 * the period lattice and their flux points by coordinates (paired flux
 * points coincide in physical space); of each pair, L is the element earlier
 * in library order, and for an element paired with itself the face with the
 * lexicographically smaller centroid.
 *   p        order 1..4
 *   n_elem   4 counts: hexahedra, prisms, tetrahedra, pyramids (each >= 0,
 *            total > 0); the library order of the state is this order
 *   verts    4 pointers (host), verts[t] = n_elem[t] x nv x 3 doubles
 *            (row-major), may be NULL where n_elem[t] = 0.  Vertex orders:
 *              hexahedron (nv 8): vertex a + 2b + 4c at reference corner
 *                (2a-1, 2b-1, 2c-1);
 *              prism (nv 6): vertex t + 3c at triangle vertex t of
 *                (-1,-1), (1,-1), (-1,1) and zeta = 2c-1;
 *              tetrahedron (nv 4): (-1,-1,-1), (1,-1,-1), (-1,1,-1), (-1,-1,1);
 *              pyramid (nv 5): base corners a + 2b at (2a-1, 2b-1, -1), then
 *                the apex (0, 0, 1).
 *   period   9 doubles (host), the three period vectors of a periodic mesh
 *            (row-major, one vector per row), or NULL for no periodicity.
 * Copied; the caller keeps ownership.  Host-side only, like fr_mesh_box.
 * Errors: FR_EINVAL (null pointers, negative counts, an element that is not
 * the affine image of its reference element or has a non-positive Jacobian,
 * a face that pairs with no other face or with more than one, flux points
 * that do not coincide), FR_EUNSUPPORTED (p outside 1..4, surface-flux
 * anti-aliasing with tetrahedra or pyramids or with prism triangle faces
 * that are not aligned, more than 16 distinct face-point permutations),
 * FR_ESTATE (mesh already built). */
fr_status fr_mesh_elements(fr_ctx* c, int p, const int64_t* n_elem, const double* const* verts,
                           const double* period);

/* Sizes of the library layout: number of hexahedra, of prisms, and the total
 * number of doubles of a state vector.  Any pointer may be NULL. */
fr_status fr_layout(const fr_ctx* c, int64_t* n_hex, int64_t* n_prism, int64_t* n_state);

/* Number of elements of type etype (fr_etype: hex, prism, tet, pyramid) in
 * the mesh.  Library order of the state: all hexahedra, then prisms, then
 * tetrahedra, then pyramids.
 * Errors: FR_EINVAL (null, bad etype), FR_ESTATE (no mesh). */
fr_status fr_type_count(const fr_ctx* c, int etype, int64_t* n_elem);

/* Physical coordinates of every solution point in library order:
 * xyz_host receives n_state/5*3 doubles, (point, xyz) row-major. Host only. */
fr_status fr_upts_coords(const fr_ctx* c, double* xyz_host);

/* du = R(u).  u_dev, du_dev: caller-owned device buffers of n_state doubles
 * in library layout (e.g. torch tensor data pointers); they must not alias.
 * Asynchronous on the context stream.  Errors: FR_ESTATE (no mesh),
 * FR_EINVAL (null), FR_EDEVICE. */
fr_status fr_rhs(fr_ctx* c, const double* u_dev, double* du_dev);

/* du = R(u) like fr_rhs, allocating nothing: for callers that cannot call
 * hipMalloc (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The per-call work buffers of the fused form
 * (face values, face fluxes, residual partials, single-precision face bases
 * and constant fluxes) live in a static device array of FR_NOALLOC_MAX_BYTES
 * bytes, one copy per GPU, held until the process ends; its address is looked
 * up on the first call on each device.  Meshes whose work buffers exceed it
 * are rejected (FR_EINVAL; fr_last_error gives the need).  Calls on one GPU
 * share that array: calls that overlap in time on one GPU (several contexts
 * or streams) race and must be serialised by the caller.  The mesh data must
 * already be on the device: any earlier fr_set_state (or fr_rhs) uploads it;
 * otherwise FR_ESTATE.  Fused form only (FR_EUNSUPPORTED for the plain
 * form).  u_dev, du_dev as for fr_rhs; asynchronous on the context stream on
 * the current device.  Other errors as fr_rhs. */
#define FR_NOALLOC_MAX_BYTES (64LL << 20)
fr_status fr_rhs_noalloc(fr_ctx* c, const double* u_dev, double* du_dev);

/* Profiling and test aid: enqueue only some kernel groups of fr_rhs on the
 * context stream.  mask bit 0: disu (solution at flux points), bit 1: volume
 * group (common solution, corrected gradients, anti-aliased flux, projection
 * and divergence), bit 2: interface group (common flux, lifting, final
 * scaling).  A run without all three bits leaves du incomplete; it exists so
 * that a benchmark can time one group in the launch configuration of fr_rhs,
 * and so that a test can run the groups one at a time (calls with masks 1, 2
 * and 4 in turn give fr_rhs's result: the work buffers persist between
 * calls).
 * Errors as fr_rhs; FR_EINVAL if mask is 0 or > 7. */
fr_status fr_rhs_stages(fr_ctx* c, const double* u_dev, double* du_dev, int mask);

/* Copy a state into the context's internal state (used by fr_rk4_step):
 * u points to n_state doubles on the host (on_device = 0) or the device. */
fr_status fr_set_state(fr_ctx* c, const double* u, int on_device);

/* Copy the internal state out (host or device destination); synchronises
 * the stream. */
fr_status fr_get_state(fr_ctx* c, double* u, int on_device);

/* Advance the internal state by nsteps classical RK4 steps of size dt
 * (the time integrator named in section 3).  Stage accumulation is in
 * double precision for both precisions.  Asynchronous. */
fr_status fr_rk4_step(fr_ctx* c, double dt, int nsteps);

/* Integrals of the conserved variables of the internal state,
 * sum_e det J_e sum_u w_u u_e (w_u = integrals of the nodal basis); out5
 * receives 5 doubles.  Synchronises the stream. */
fr_status fr_integrals(fr_ctx* c, double* out5);

/* Host-side inspection (no device needed).
 * fr_ref_operator: copy a reference-element quantity of type etype and order
 * p into out (capacity cap doubles); *count receives its size.  Names:
 *   "upts", "fpts", "qpts"  point coordinates (N x 3)
 *   "qwts"                  quadrature weights (N_q)
 *   "M0" (N_f x N_u), "M3" (N_u x N_f), "M7" (N_q x N_u), "M8" (N_u x N_q),
 *   "Dxi", "Deta", "Dzeta" (N_u x N_u)   dense operators of section 2.2;
 *   "APd" (3 x N_u x N_q)   tetrahedra, pyramids: -Mass^-1 Dq_d^T W_q
 *   "Ku" (3 x N_u x N_u)    pyramids: APd_d M7 (empty otherwise);
 *   "K0" (3 x N_u x N_u)    tetrahedra, pyramids: the divergence of a flux at
 *                           the solution points (D_d - M3 n_d M0; pyramids Ku).
 * etype: fr_etype.  Errors: FR_EINVAL (unknown name or etype, cap too
 * small). */
fr_status fr_ref_operator(int etype, int p, const char* name, double* out, int64_t cap, int64_t* count);

/* fr_connectivity: for every flux point of every element (types in order,
 * then element, then flux point): nbr[i] = flat index of the paired flux
 * point, is_left[i] = 1 if this side is "L" of the pair (the element with
 * the lower mesh-order index; for an element paired with itself, the face
 * with the lexicographically smaller centroid).  Arrays of n_fpts entries;
 * *n_fpts receives the count when nbr is NULL. */
fr_status fr_connectivity(const fr_ctx* c, int64_t* nbr, int8_t* is_left, int64_t* n_fpts);

const char* fr_last_error(const fr_ctx* c);
void fr_destroy(fr_ctx* c);

/* fr_fill_lds: fill the local data share of the current device with `value`
 * (every CU's 160 KB, by workgroups of 32 KB launched on the HIP stream
 * hip_stream, NULL for the null stream; asynchronous).  For tests only: it
 * is for the callers that check that no kernel of this library reads LDS it
 * has not written, by running them after a fill with NaN.  Errors:
 * FR_EDEVICE (a HIP call failed). */
fr_status fr_fill_lds(void* hip_stream, float value);

/* ------------------------------------------------------------------------
 * Serving pool: continuous batching of independent solves.
 *
 * A pool holds many periodic-box solves (requests) on one GPU.  Requests are
 * queued in submission order and admitted, strictly in that order, while
 * their device footprint fits the pool's byte budget and fewer than
 * max_active requests are admitted.  Each fr_pool_step advances every
 * admitted request by one classical RK4 step of its own dt, with one kernel
 * launch per (element type, order, kernel, RK stage) covering the elements of
 * all of them; the arithmetic applied to each element is the one of
 * fr_rk4_step, so a request's result does not depend on what else shares the
 * pool.  A request leaves the pool after its last step; its final state is
 * copied to u_out (if given) and its memory is reused by later admissions.
 * The RHS is the fused form of section 6.1 at the pool's precision; the
 * Taylor-Green initial condition is the test case of section 6.
 * ---------------------------------------------------------------------- */
typedef struct fr_pool fr_pool;

typedef struct {
  int nx, ny, nz;        /* cells of the periodic box [lo,hi]^3 */
  double lo, hi;
  int p;                 /* order 1..4 */
  int kind;              /* fr_mesh_kind */
  double dt;             /* RK4 step size */
  int nsteps;            /* RK4 steps to run (>= 0) */
  const double* u_init;  /* host, n_state doubles in library layout, or NULL:
                            Taylor-Green vortex with rho0 = U0 = 1 and mean
                            pressure tgv_p0.  Read when the request is
                            admitted: keep it valid until fr_pool_query
                            reports the request active or done. */
  double tgv_p0;
  double* u_out;         /* host, n_state doubles receiving the final state,
                            or NULL.  Written inside the fr_pool_step that
                            completes the request. */
} fr_request;

typedef struct {
  int n_active;          /* requests advanced by this step */
  int n_admitted;        /* requests admitted by this call (first step next call) */
  int n_finished;        /* requests completed by this call */
  int n_queued;          /* requests waiting after this call */
  int n_launches;        /* kernel launches enqueued for the step */
  int64_t dof;           /* degrees of freedom advanced: sum of n_state */
  int64_t bytes_in_use;  /* device bytes held by admitted requests */
} fr_pool_stats;

/* Create a pool.  ph: physics and precision shared by all requests (form
 * must be FR_FORM_FUSED).  hip_stream: stream for all pool work, or NULL.
 * budget_bytes: device memory for request data, allocated as one block by
 * the first fr_pool_step (no device call is made before).  max_active:
 * slot limit.  Errors: FR_EINVAL, FR_EUNSUPPORTED (plain form). */
fr_status fr_pool_create(const fr_physics* ph, void* hip_stream, int64_t budget_bytes, int max_active,
                         fr_pool** out);

/* Device bytes a request occupies while admitted, and its state size in
 * doubles.  Host only.  Errors: FR_EINVAL / FR_EUNSUPPORTED for a bad
 * request (as fr_pool_submit). */
fr_status fr_pool_footprint(const fr_pool* pool, const fr_request* r, int64_t* bytes, int64_t* n_state);

/* Queue a request; *id receives its handle (0, 1, 2, ... in submission
 * order).  The request is copied.  Host only.  Errors: FR_EINVAL (bad
 * sizes, nsteps < 0, neither u_init nor tgv_p0 > 0), FR_EUNSUPPORTED (p
 * outside 1..4), FR_ENOMEM (footprint above the whole budget: it could
 * never be admitted). */
fr_status fr_pool_submit(fr_pool* pool, const fr_request* r, int64_t* id);

/* One scheduling round: enqueue one RK4 step of every admitted request, then
 * admit queued requests (host mesh set-up overlaps the GPU work), wait for
 * the stream, and retire requests that completed their steps.  Synchronous.
 * A queued request whose host set-up fails (mesh or table construction)
 * does not stop the round: it leaves the queue with status 3 (failed),
 * never runs, holds no memory, is listed among the round's finished ids,
 * and fr_pool_last_error names it and the reason; the round's step,
 * admissions and accounting go on.  stats may be NULL.  After FR_EDEVICE
 * the pool is unusable: destroy it. */
fr_status fr_pool_step(fr_pool* pool, fr_pool_stats* stats);

/* Ids admitted and finished (completed or failed) by the last fr_pool_step
 * (arrays of cap entries, either may be NULL; counts always written).  FR_EINVAL if a list
 * does not fit. */
fr_status fr_pool_events(const fr_pool* pool, int64_t* admitted, int* n_admitted, int64_t* finished,
                         int* n_finished, int cap);

/* Status of a request: 0 queued, 1 admitted, 2 done, 3 failed (never ran);
 * steps completed.
 * FR_EINVAL for an unknown id. */
fr_status fr_pool_query(const fr_pool* pool, int64_t id, int* status, int* steps_done);

/* Testing aid: the host set-up of queued request id will fail at its
 * admission, as a mesh-building error would, so that callers can exercise
 * the failure path of fr_pool_step.  Host only.  FR_EINVAL if id is not a
 * queued request. */
fr_status fr_pool_inject_prepare_error(fr_pool* pool, int64_t id);

const char* fr_pool_last_error(const fr_pool* pool);
/* Synchronises the pool stream and frees all device memory of the pool. */
void fr_pool_destroy(fr_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* FR_H */

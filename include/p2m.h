/*
 * p2m.h -- particle <-> fixed-mesh projection on MI355X (gfx950).
 *
 * C ABI of libp2m.so.  Implements the projection step of Duque & Espanol,
 * "Rapid convergence for simulations that project from particles onto a fixed
 * mesh": particle -> mesh (P2M) with the quadratically consistent particle
 * shape functions of App. B, mesh -> particle (M2P) with the fixed mesh's
 * linear FE shape functions, and the adjoints of both.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every array argument is a DEVICE pointer (memory of the current HIP
 *    device) owned by the caller, unless stated otherwise.  Positions are
 *    FP64, interleaved [N][2] (x, y), 16-byte aligned.  Field values are
 *    channels-last [N][C] (particles) or [(nx+1)*(ny+1)][C] (mesh, node
 *    k = j*(nx+1) + i, x fastest), element type given by a p2m_dtype.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  All calls are asynchronous on that stream unless they say they
 *    synchronise; argument errors are reported synchronously by the return
 *    code, data-dependent errors (a particle outside the mesh, a non-finite
 *    coordinate, a cap overflow) are recorded on the device and reported by
 *    p2m_weights_diag(), which synchronises the stream.
 *  - Return value: P2M_OK (0) or a negative p2m_status; p2m_last_error()
 *    returns a thread-local message describing the last failure.
 *  - The library never reads field values from host memory and never falls
 *    back to a CPU computation.
 */
#ifndef P2M_H
#define P2M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Fixed uniform mesh: (nx+1)*(ny+1) nodes at (x0 + i*H, y0 + j*H),
 * 0 <= i <= nx, 0 <= j <= ny.  H is the mesh spacing of the paper (Sec. 1,
 * Fig. idea).  The domain is the bounded rectangle [x0, x0+nx*H] x
 * [y0, y0+ny*H], where particles must lie, or with P2M_PERIODIC the periodic
 * box of the paper's runs (same node layout; see that flag). */
typedef struct p2m_mesh {
    int32_t nx, ny;
    double H;
    double x0, y0;
} p2m_mesh;

typedef enum p2m_status {
    P2M_OK = 0,
    P2M_EINVAL = -1,   /* bad argument: null/misaligned pointer, N <= 0,
                          H <= 0, h <= 0, C not in [1, 16], unknown dtype   */
    P2M_EDOMAIN = -2,  /* particle outside the mesh or non-finite (diag)    */
    P2M_ECAP = -3,     /* a node's support exceeded P2M_MAX_SUPPORT (diag)  */
    P2M_EGEOM = -4,    /* coincident particles, a node left without weights,
                          or a rank-deficient system with P2M_STRICT (diag) */
    P2M_EHIP = -5,     /* a HIP runtime call failed                         */
    P2M_ENOMEM = -6    /* device allocation failed                          */
} p2m_status;

/* Element type of field arrays (values, mesh values and their gradients). */
typedef enum p2m_dtype {
    P2M_F64 = 0,       /* FP64 storage, FP64 sums                           */
    P2M_F32 = 1,       /* FP32 storage, FP32 sums                           */
    P2M_BF16 = 2       /* BF16 storage of PARTICLE arrays, FP32 sums; mesh
                          arrays and mesh outputs are FP32                  */
} p2m_dtype;

/* Flags of p2m_build_weights. */
#define P2M_WEIGHTS_F32 0x1  /* also keep FP32 copies of the weights (mixed path) */
#define P2M_STRICT      0x2  /* rank-deficient systems make diag report EGEOM   */
#define P2M_LINEAR      0x4  /* linear FE particle functions phi_mu at interior
                                nodes instead of psi_mu (see p2m_build_weights) */
#define P2M_PERIODIC    0x8  /* periodic box (see p2m_build_weights)            */
#define P2M_DETERMINISTIC 0x10 /* also index the entries by particle, so that
                                p2m_project_backward and
                                p2m_build_weights_backward sum each
                                particle's terms in a fixed order: no atomics,
                                the same bits on every run                   */

/* Largest number of particles one node's weights may involve: the width of
 * exported rows and of grad_w.  Rows longer than 32 (only around particles
 * of high Delaunay degree) are kept in a small overflow store of the handle
 * and counted in p2m_diag.long_rows. */
#define P2M_MAX_SUPPORT 63
/* Nearest particles used by a closure node (boundary ring / outside hull). */
#define P2M_CLOSURE_K 12

/* Device-side diagnostics of the last build (all counts are per build). */
typedef struct p2m_diag {
    int64_t interior_nodes;     /* nodes with a Delaunay triangle              */
    int64_t closure_nodes;      /* boundary-ring + outside-hull nodes          */
    int64_t outside_hull_nodes; /* subset of closure_nodes                     */
    int64_t rank_deficient;     /* moment systems of rank below 6: their
                                   weights are the minimum-norm least-squares
                                   answer (see svd_systems)                    */
    int64_t cap_overflow;       /* nodes whose support exceeded P2M_MAX_SUPPORT,
                                   or that found the overflow store full       */
    int64_t escalated_nodes;    /* nodes that needed a larger search region    */
    int64_t global_nodes;       /* nodes that needed a scan of every particle  */
    int64_t near_degenerate;    /* predicate decisions inside the error bound  */
    int64_t bad_particles;      /* outside the mesh or non-finite (excluded)   */
    int64_t failed_nodes;       /* nodes left without weights (zero row)       */
    int64_t duplicate_pairs;    /* pairs of coincident particles (EGEOM)       */
    int64_t slow_nodes;         /* nodes the register-resident first pass left
                                   to the exact fallback (performance only)    */
    int32_t status;             /* P2M_OK, P2M_EDOMAIN, P2M_ECAP or P2M_EGEOM  */
    int32_t support_max;        /* largest support of any node                 */
    int64_t svd_systems;        /* moment systems solved by the rank-revealing
                                   solver (below)                              */
    double max_gram_cond;       /* largest cond2(G), G = M M^t, of a full-rank
                                   moment system: an estimate within a factor
                                   36 above it for systems solved by Cholesky,
                                   exact for the others                        */
    int64_t bwd_rank_deficient; /* rank-deficient systems whose position
                                   derivative the last
                                   p2m_build_weights_backward on this handle
                                   left out (see that call)                    */
    int64_t long_rows;          /* rows of more than 32 particles (kept in the
                                   overflow store; solved by the SVD path)     */
} p2m_diag;

/* How each moment system M A = b (6 conditions, K support particles) is
 * solved.  The paper solves them by SVD with automatic rank detection
 * (App. A); the answer is the minimum-norm solution, with singular values of
 * M at or below eps * max(6, K) * s_max taken as zero (LAPACK's default
 * threshold).  For speed, a system is first solved through its Gram matrix
 * G = M M^t (Cholesky, one step of iterative refinement), which gives that
 * answer to about eps * cond(M) as long as G is well conditioned: a system
 * whose estimate trace(G) trace(G^-1) exceeds the option "svd_cond"
 * (default 1e8, i.e. cond(M) of about 1e4), or whose Cholesky breaks down,
 * is solved instead by a one-sided Jacobi SVD of M, with the rule above, in
 * the frame in which its conditions are stated (edge systems: relative to
 * the edge's ends, scaled by its length; closure systems: relative to the
 * node, in units of h).  Such a row is flagged, and counted in svd_systems;
 * a system of rank below 6 is counted in rank_deficient. */

/* Opaque weights handle: the P2M operator of one particle set on one mesh.
 * Owned by the library; holds device memory until p2m_weights_destroy(). */
typedef struct p2m_weights p2m_weights;

/*
 * p2m_build_weights -- psi_mu(r_i) for every mesh node i (App. B, eq. phiquad).
 *
 * For each interior node: the Delaunay triangle T = (a, b, c) of the particles
 * that contains the node, the Delaunay rings of a, b, c, and for each edge
 * e = (nu, sigma) of T the minimum-norm coefficients A_{mu e} over
 * S_e = ring(nu) U ring(sigma) solving eqs. (A0), (A1), (A2_2); the weight of
 * particle mu is phi_mu + 2 sum_e phi_nu phi_sigma A_{mu e}.  Nodes on the
 * mesh's outer ring and nodes outside the particles' convex hull use the
 * minimum-norm quadratic-moment weights of their P2M_CLOSURE_K nearest
 * particles (a closure of the bounded box; the paper's periodic runs need
 * none, and P2M_PERIODIC has no such nodes).
 *
 *  mesh   host pointer to the mesh description.
 *  h      mean particle spacing (the paper's h).  A performance hint only:
 *         it sizes the binning grid; results do not depend on it.
 *  pos    device [N][2] FP64 particle positions (user order).
 *  N      number of particles, 3 <= N < 2^28.
 *  flags  P2M_WEIGHTS_F32 | P2M_STRICT | P2M_LINEAR | P2M_PERIODIC.  With P2M_LINEAR an
 *         interior node's row is phi_mu alone (App. B: the linear FE functions
 *         of the particles' Delaunay triangulation, eqs. C0 and C1, i.e. the
 *         barycentric coordinates of the node in T, three entries; the
 *         particle side of the paper's linear-FE projection): the triangle is
 *         located as above, rings and solves are skipped.  Closure nodes keep
 *         their quadratic-moment weights.  Such a handle serves p2m_project
 *         and p2m_project_backward; p2m_build_weights_backward rejects it.
 *         With P2M_PERIODIC the box [x0, x0+nx*H) x [y0, y0+ny*H) is periodic,
 *         as in every run of the paper (Sec. 3; App. A: a periodic Delaunay
 *         triangulation): the triangulation is that of the particles and
 *         their images across the box sides, a particle enters a node's
 *         weights at its image nearest to the node (the support positions of
 *         eqs. A0-A2_2), and there are no closure nodes.  The node layout is
 *         unchanged: node (nx, j) is node (0, j) and (i, ny) is (i, 0), and
 *         their rows are equal; M2P needs no flag on that layout (mesh values
 *         must repeat the first column and row).  Needs nx, ny >= 4; a node
 *         whose triangles do not fit within about half a period fails
 *         (EGEOM).  p2m_build_weights_backward differentiates through the
 *         nearest images (an image moves with its particle).
 *  w      in/out: *w == NULL allocates a new handle; a handle from an earlier
 *         call is reused (its buffers grow if needed; previous contents are
 *         overwritten, so no work may still be pending on them on another
 *         stream).
 *  stream hipStream_t.
 * Errors: EINVAL (arguments), ENOMEM, EHIP.  Data errors -> p2m_weights_diag.
 */
int p2m_build_weights(const p2m_mesh* mesh, double h, const double* pos, int64_t N,
                      int flags, p2m_weights** w, void* stream);

/* Copy the diagnostics of the last build on this handle to host memory.
 * Synchronises `stream`.  Returns diag->status (P2M_OK if the build had no
 * data error). */
int p2m_weights_diag(const p2m_weights* w, p2m_diag* diag, void* stream);

/* Copy the ELL weights to caller device buffers (for inspection and tests).
 * idx  int32 [P2M_MAX_SUPPORT][n_nodes] user particle ids (unused slots -1),
 * wts  FP64 [P2M_MAX_SUPPORT][n_nodes], cnt int32 [n_nodes],
 * tri  int32 [n_nodes][3] user ids of the node's Delaunay triangle (-1 for
 *      closure nodes).  Any pointer may be NULL. */
int p2m_weights_export(const p2m_weights* w, int32_t* idx, double* wts, int32_t* cnt,
                       int32_t* tri, void* stream);

/* Number of mesh nodes and particles of a handle (host values). */
int p2m_weights_shape(const p2m_weights* w, int64_t* n_nodes, int64_t* n_particles);

/*
 * p2m_project -- eq. (p2m): mesh_vals[i][c] = sum_mu psi_mu(r_i) vals[mu][c].
 *  vals      device [N][C] particle values of type dtype (user order).
 *  mesh_vals device [(nx+1)(ny+1)][C] output; type dtype, FP32 for P2M_BF16.
 *  P2M_F64 uses the FP64 weights; P2M_F32/P2M_BF16 use FP32 weights and
 *  FP32 sums (the handle must have been built with P2M_WEIGHTS_F32).
 */
int p2m_project(const p2m_weights* w, const void* vals, int C, int dtype,
                void* mesh_vals, void* stream);

/*
 * m2p_interpolate -- eq. (m2p) with linear FE mesh functions:
 * vals[mu][c] = sum_i phi^m_i(r_mu) mesh_vals[i][c].  Each cell
 * [i, i+1] x [j, j+1] is split by the diagonal (i,j)-(i+1,j+1); a particle
 * takes cell i = min(floor((x-x0)/H), nx-1) (same in y).
 *  mesh_vals device [(nx+1)(ny+1)][C], type dtype (FP32 for P2M_BF16).
 *  pos       device [N][2] FP64.
 *  vals      device [N][C] output, type dtype (BF16 for P2M_BF16).
 * Particles outside the mesh get NaN and are counted nowhere: validate
 * positions with p2m_build_weights / p2m_weights_diag.
 */
int m2p_interpolate(const p2m_mesh* mesh, const void* mesh_vals, int C, int dtype,
                    const double* pos, int64_t N, void* vals, void* stream);

/*
 * p2m_advect -- moves the particles one time step with the prescribed
 * velocity of a kinematic test (the paper's kinematic procedures rebuild the
 * particle functions after every move): the cellular flow of streamfunction
 * amp sin(pi (x-x0)/Lx) sin(pi (y-y0)/Ly) on the mesh box (Lx = nx H,
 * Ly = ny H; u = d psi/dy, v = -d psi/dx, no flow through the box walls),
 * one explicit midpoint step r* = r + dt/2 u(r), r' = r + dt u(r*), then
 * clamped into the box.  A loop step of the kinematic projection is
 * m2p_interpolate, p2m_advect, p2m_build_weights, p2m_project.
 *  pos   device [N][2] FP64, updated in place.
 * Errors: EINVAL (mesh, pointer, N, non-finite amp or dt), EHIP.
 */
int p2m_advect(const p2m_mesh* mesh, double* pos, int64_t N, double amp, double dt, void* stream);

/*
 * p2m_advect_periodic -- p2m_advect in the periodic box of P2M_PERIODIC
 * (the paper's transport tests run in periodic boxes): the cellular flow of
 * streamfunction amp cos(2 pi (x-x0)/Lx) cos(2 pi (y-y0)/Ly), periodic on the
 * box, whose cells are centred on the box corners and centre so that
 * particles cross the box sides; the same midpoint step, then every
 * coordinate wrapped into [x0, x0+Lx) by whole periods (x - Lx floor((x-x0)/Lx),
 * one rounding; a result that rounds onto x0+Lx is x0).  A loop step of the
 * periodic kinematic projection is m2p_interpolate, p2m_advect_periodic,
 * p2m_build_weights with P2M_PERIODIC, p2m_project.
 *  pos   device [N][2] FP64, updated in place.
 * Errors: as p2m_advect.
 */
int p2m_advect_periodic(const p2m_mesh* mesh, double* pos, int64_t N, double amp, double dt, void* stream);

/*
 * Mesh-side quadratically consistent shape functions (App. B's construction
 * applied to the fixed mesh): psi^m_i = phi^m_i + 2 sum over the edges
 * e = (nu, sigma) of the particle's mesh triangle of phi^m_nu phi^m_sigma
 * A^m_{i e}, with phi^m the linear FE functions of m2p_interpolate's
 * triangulation and A^m_{. e} the minimum-norm solution of eqs. (A0), (A1),
 * (A2_2) over S_e = ring(nu) U ring(sigma), ring(v) = v and its neighbours
 * (i+-1, j), (i, j+-1), (i+1, j+1), (i-1, j-1) inside the mesh (a
 * pseudo-inverse where the mesh boundary costs a system its rank).  The
 * coefficients depend on the mesh only: p2m_mesh_qcsf_create computes them
 * once (10 per edge, ~3 (nx+1)(ny+1) edges, 120 bytes each, device memory of
 * the current device); p2m_mesh_qcsf_destroy frees them.  The handle is
 * read-only once created and may serve any number of calls and streams.
 * Errors: EINVAL (mesh, out), ENOMEM, EHIP.
 */
typedef struct p2m_mesh_qcsf p2m_mesh_qcsf;
int p2m_mesh_qcsf_create(const p2m_mesh* mesh, p2m_mesh_qcsf** out, void* stream);
/* The same functions in the periodic box of P2M_PERIODIC: every mesh edge is
 * interior there, with the rings wrapped across the box sides, so every edge
 * takes the coefficients of an interior edge of its orientation (translation
 * invariance) and M2P reads node ids wrapped to the first column and row
 * (which the mesh values' last column and row repeat).  Needs nx, ny >= 4. */
int p2m_mesh_qcsf_create_periodic(const p2m_mesh* mesh, p2m_mesh_qcsf** out, void* stream);
void p2m_mesh_qcsf_destroy(p2m_mesh_qcsf* q);

/*
 * m2p_interpolate_qcsf -- eq. (m2p) with the mesh's quadratically consistent
 * functions: vals[mu][c] = sum_i psi^m_i(r_mu) mesh_vals[i][c]; arguments
 * and types as m2p_interpolate (FP64 coefficients, sums in the dtype's
 * precision).  Reproduces every quadratic field exactly.  No adjoint.
 */
int m2p_interpolate_qcsf(const p2m_mesh_qcsf* q, const void* mesh_vals, int C, int dtype, const double* pos,
                         int64_t N, void* vals, void* stream);

/*
 * m2p_interpolate_backward -- adjoint of m2p_interpolate.
 *  grad_vals  device [N][C] upstream gradient (type dtype; FP32 for BF16).
 *  grad_mesh  device [(nx+1)(ny+1)][C] output, OVERWRITTEN with
 *             sum_mu phi^m_i(r_mu) grad_vals[mu][c]; may be NULL.
 *  grad_pos   device [N][2] FP64, ACCUMULATED (+=) with
 *             sum_c grad_vals[mu][c] * grad_r (sum_i phi^m_i mesh_vals[i][c])
 *             (the interpolant's gradient on the particle's triangle);
 *             may be NULL.  mesh_vals is needed only when grad_pos != NULL.
 * grad_mesh uses atomic adds: its bits may differ between runs.
 */
int m2p_interpolate_backward(const p2m_mesh* mesh, const void* mesh_vals, int C, int dtype,
                             const double* pos, int64_t N, const void* grad_vals,
                             void* grad_mesh, double* grad_pos, void* stream);

/*
 * m2p_interpolate_backward_binned -- m2p_interpolate_backward at the particles
 * a weights handle was built from, using that build's binning (the adjoint
 * of eq. m2p: grad_mesh[i] = sum_mu phi^m_i(r_mu) grad_vals[mu]).
 *  w          handle built from `pos` (the same array, unchanged since); its
 *             mesh, or for a batched handle every set's mesh, is the mesh.
 *  grad_mesh  OVERWRITTEN, as in m2p_interpolate_backward, but gathered per
 *             node from the particles of the bins around its cells (each
 *             located exactly as the forward locates it): no atomics, and
 *             the same bits on every run.  May be NULL.
 *  grad_pos   ACCUMULATED exactly as m2p_interpolate_backward does.  May be
 *             NULL; mesh_vals is needed only when it is not.
 * Other arguments and types as m2p_interpolate_backward.
 */
int m2p_interpolate_backward_binned(const p2m_weights* w, const void* mesh_vals, int C, int dtype,
                                    const double* pos, const void* grad_vals, void* grad_mesh,
                                    double* grad_pos, void* stream);

/*
 * p2m_project_backward -- adjoint of p2m_project for fixed weights.
 *  grad_mesh  device [(nx+1)(ny+1)][C] upstream gradient (dtype; FP32 for BF16).
 *  grad_vals  device [N][C] output (dtype; FP32 for BF16), OVERWRITTEN with
 *             sum_i psi_mu(r_i) grad_mesh[i][c]; may be NULL.  Summed by
 *             atomic adds, or, for a handle built with P2M_DETERMINISTIC,
 *             per particle over its entries in a fixed order (the same bits
 *             on every run).
 *  vals       device [N][C] forward particle values; needed iff grad_w.
 *  grad_w     device FP64 [P2M_MAX_SUPPORT][n_nodes] output, OVERWRITTEN with
 *             d L / d psi = sum_c grad_mesh[i][c] vals[idx][c]; may be NULL.
 */
int p2m_project_backward(const p2m_weights* w, const void* grad_mesh, int C, int dtype,
                         const void* vals, void* grad_vals, double* grad_w, void* stream);

/*
 * p2m_build_weights_backward -- d L / d r through the weights: given grad_w
 * (layout of p2m_project_backward), grad_pos[mu] += sum_{i,k} grad_w[k][i]
 * d psi_k(r_i) / d r_mu for the particle positions pos (the same array the
 * handle was built from; geometry is recomputed, not stored).  The
 * combinatorial structure (triangles, rings, nearest sets) is held fixed.
 *  grad_pos  device [N][2] FP64, ACCUMULATED with atomic adds; for a handle
 *            built with P2M_DETERMINISTIC each entry's derivative is stored
 *            and every particle adds its own in a fixed order (the same bits
 *            on every run for the same grad_pos on entry).
 * Errors: EINVAL also for a handle built with P2M_LINEAR.
 */
int p2m_build_weights_backward(const p2m_weights* w, const double* pos, const double* grad_w,
                               double* grad_pos, void* stream);

void p2m_weights_destroy(p2m_weights* w);

/* ------------------------------------------------------------------------
 * Recompute forms: the weights are rebuilt inside the call in a workspace
 * the library keeps per device (grown on demand, never freed), so a caller
 * keeps no weights between a forward and its backward -- the form for the
 * largest sizes.  Calls on one device are serialised: the host calls by a
 * lock, the device work by an event each call records on its stream and the
 * next call, on whatever stream, waits for before it rebuilds the workspace
 * (a call captured into a HIP graph takes no part in this: the graph orders
 * its own work, and its replays must not overlap other calls on the device).
 * Results are those of p2m_build_weights + p2m_project (+ the backward calls)
 * bit for bit, since the build is deterministic.
 * ------------------------------------------------------------------------ */

/* eq. (p2m) with the App. B weights built for this call (arguments as in
 * p2m_build_weights and p2m_project; FP32/BF16 values use FP32 weights).
 * For C <= 4 the weights pass adds each row of the fast path into its node's
 * sum as it weighs it and keeps no weights of it; rows of the exact path and
 * of the rank-revealing solver keep their weights and are summed afterwards.
 * The order of every sum is p2m_project's: the result is
 * p2m_build_weights + p2m_project bit for bit. */
int p2m_project_fused(const p2m_mesh* mesh, double h, const double* pos, int64_t N,
                      const void* vals, int C, int dtype, void* mesh_vals, void* stream);

/* The current device's workspace handle of the recompute forms (NULL before
 * the first call): p2m_weights_diag on it describes the last recompute
 * build.  After a p2m_project_fused the handle holds no weights, and the calls
 * that read weights (p2m_project, p2m_weights_export, the backward calls)
 * refuse it with EINVAL; after a p2m_backward_fused it holds that build's
 * weights.  Owned by the library; do not destroy. */
const p2m_weights* p2m_fused_handle(void);

/* Adjoint of p2m_project_fused for the upstream gradient grad_mesh
 * ([(nx+1)(ny+1)][C], dtype; FP32 for BF16): grad_vals [N][C] is
 * OVERWRITTEN (may be NULL); grad_pos [N][2] FP64 is ACCUMULATED through the
 * weights (may be NULL; needs vals).  The weights are rebuilt from pos. */
int p2m_backward_fused(const p2m_mesh* mesh, double h, const double* pos, int64_t N,
                       const void* vals, int C, int dtype, const void* grad_mesh,
                       void* grad_vals, double* grad_pos, void* stream);

/*
 * p2m_project_fused_noalloc -- p2m_project_fused for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  The weights are rebuilt in
 * a static workspace of the library (about 16 MiB of device memory, held by
 * every GPU the library runs on until the process ends) instead of the
 * allocated per-device workspace; the call makes no allocation (no hipMalloc,
 * no stream or event creation) and runs every kernel, the exact-path ones
 * included, on `stream`.  Arguments and results as p2m_project_fused.
 * Limits (EINVAL beyond them): N <= 131072 particles, a mesh of at most 256
 * tiles of 8 x 8 nodes (e.g. 127 x 127 cells), at most 262144 binning bins
 * (about (extent / h)^2).  Every call on a GPU shares that GPU's workspace,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  The
 * diagnostics of these builds are not reported.
 */
int p2m_project_fused_noalloc(const p2m_mesh* mesh, double h, const double* pos, int64_t N,
                              const void* vals, int C, int dtype, void* mesh_vals, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many independent particle sets, each with its own mesh and h,
 * handled by one launch sequence.  The sets are the paper's problem
 * (eqs. p2m, m2p and App. B) repeated; nothing couples them.
 * ------------------------------------------------------------------------ */
#define P2M_MAX_SETS 65536

/* Opaque batch description (host data plus a small device table).  Owned by
 * the library until p2m_batch_destroy(). */
typedef struct p2m_batch p2m_batch;

/*
 * p2m_batch_create -- describe S sets.
 *  meshes       host [S] meshes; set s owns mesh nodes
 *               node_offsets[s] .. node_offsets[s+1]-1 of every mesh-side
 *               array (sets in order, each mesh x-fastest).
 *  h            host [S] particle spacings (hints, as in p2m_build_weights).
 *  S            1 .. P2M_MAX_SETS.
 *  set_offsets  host [S+1]: set s owns particles set_offsets[s] ..
 *               set_offsets[s+1]-1 of every particle-side array;
 *               set_offsets[0] = 0, at least 3 particles per set, total
 *               below 2^28.
 *  out          receives the handle.
 * Synchronous (uploads the device table).  Errors: EINVAL, ENOMEM, EHIP.
 */
int p2m_batch_create(const p2m_mesh* meshes, const double* h, int S, const int64_t* set_offsets,
                     p2m_batch** out);

/* Total nodes and particles of a batch, and (if non-NULL) the host array
 * node_offsets[S+1] of each set's first node. */
int p2m_batch_shape(const p2m_batch* b, int64_t* n_nodes, int64_t* n_particles, int64_t* node_offsets);

void p2m_batch_destroy(p2m_batch* b);

/*
 * p2m_build_weights_batched -- p2m_build_weights for every set of a batch in
 * one pass: one binning of all particles (bins of set s after those of set
 * s-1) and one launch of each build kernel over the node tiles of all sets.
 * pos is device [N_total][2]; particle ids in the handle are batch-global.
 * The resulting handle is used with p2m_project, p2m_project_backward,
 * p2m_build_weights_backward, p2m_weights_diag (counts summed over the
 * sets) and p2m_weights_export exactly like a single-set handle, with
 * mesh-side arrays of all sets' nodes concatenated.
 */
int p2m_build_weights_batched(const p2m_batch* b, const double* pos, int flags, p2m_weights** w,
                              void* stream);

/* m2p_interpolate and its adjoint over every set of a batch in one launch;
 * arrays as in the single-set calls, concatenated over the sets. */
int m2p_interpolate_batched(const p2m_batch* b, const void* mesh_vals, int C, int dtype,
                            const double* pos, void* vals, void* stream);
int m2p_interpolate_backward_batched(const p2m_batch* b, const void* mesh_vals, int C, int dtype,
                                     const double* pos, const void* grad_vals, void* grad_mesh,
                                     double* grad_pos, void* stream);

/* Process-wide tuning knobs of the weight build and of M2P (performance
 * only; results do not depend on them, "svd_cond" aside, which moves them by
 * rounding only).  Not thread-safe with concurrent calls.
 *   "bin_scale"  bin width ~ bin_scale * h        (0.25 .. 8,  default 1)
 *   "fast_radius" candidate radius / h of the
 *                register-resident first pass     (1.5 .. 8,   default 2.6)
 *   "closure_radius" candidate radius / h of the
 *                first pass for boundary-ring nodes (1.5 .. 8,   default 4)
 *   "region_h"   first search half-width / h of
 *                the fallback pass                (1 .. 64,    default 4)
 *   "levels"     region doublings before a scan
 *                of every particle                (0 .. 8,     default 3)
 *   "svd_cond"   condition estimate of a moment system above which it is
 *                solved by the SVD (see p2m_diag)  (1 .. 1e16, default 1e8;
 *                results change only by rounding)
 *   "m2p_ppt"    particles per thread of m2p_interpolate (1, 2 or 4,
 *                default 1; up to 4 channels)
 * Returns P2M_EINVAL for an unknown name or a value out of range. */
int p2m_set_option(const char* name, double value);

/* Current value of a tuning knob above, written to *value (host pointer).
 * One derived, read-only name as well:
 *   "fast_slots" candidate slots per lane of the first pass that builds
 *                launched with the current fast_radius use (7, 8 or 10).
 * Returns P2M_EINVAL for an unknown name or a NULL pointer. */
int p2m_get_option(const char* name, double* value);

/* Event timing of the library's kernel groups, for measurement.
 * p2m_profile_enable(1) clears the totals and starts recording a pair of HIP
 * events on the caller's stream around each group ("bin", "build",
 * "project", "m2p", "m2p_bwd", "project_bwd", "build_bwd", and the three
 * parts of "build": "build_fast", "build_slow", "weights", the last also
 * as its two kernels alone: "k_weights", "k_weights_rd"); 0 stops.
 * p2m_profile_read() waits for the recorded events and returns the summed
 * GPU time in milliseconds and the number of launches of one group. */
int p2m_profile_enable(int on);
int p2m_profile_read(const char* phase, double* total_ms, int64_t* count);

/* Thread-local description of the last error (never NULL). */
const char* p2m_last_error(void);

/* Library version string. */
const char* p2m_version(void);

#ifdef __cplusplus
}
#endif

#endif /* P2M_H */

/*
 * sf_grav.h -- softened self-gravity (accelerations, potentials and their
 * adjoint) for gas cells with adaptive softening plus sink particles, on one
 * AMD Instinct MI355X (gfx950).  C ABI of libsfgrav.so.
 *
 * The operation (arXiv 2010.11254, Sec. 2.2 "Gravity"): for each particle i,
 * gas or sink, the gravitational acceleration g = -grad Phi and the
 * potential Phi it feels from all other particles,
 *     a_i   =  G sum_{j != i} m_j F(r_ij, h_ij) (x_j - x_i)
 *     phi_i = -G sum_{j != i} m_j P(r_ij, h_ij)
 * with the softened law of Sec. 2.2.1: pairs closer than h_ij = max(h_i, h_j)
 * use the force of a unit mass smoothed by the M4 cubic spline of compact
 * support h_ij (the kernel of the Sec. 2.1 footnote); beyond h_ij the law is
 * exactly Newtonian.  The larger radius is used in both directions of every
 * pair, so all interactions are antisymmetric.  P(0, h) = 2.8/h, i.e. the
 * Plummer-equivalent softening is h/2.8 (Sec. 2.3.1).
 *
 * Two evaluation paths:
 *   - tree   : Barnes-Hut octree (Sec. 2.2) over Morton-sorted particles,
 *              monopole or quadrupole nodes, opening angle theta = L/r
 *              (fiducial 0.5) combined, when opts.alpha >= 0, with the
 *              paper's acceleration-based criterion (a node is opened when
 *              G M L^2 / r^4 exceeds alpha times the target's previous
 *              |g|), walked by groups of up to 64 targets;
 *   - direct : all pairs (the theta -> 0 limit of the tree).
 * Sink targets always receive the sink-sink part of their field as an exact
 * FP64 direct sum; their gas part comes from the same path as gas targets.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors).  `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream); every kernel is enqueued on it, in order, except that a tree
 *     evaluation with sinks runs its sink-sink sum and sink walk on a second
 *     stream of the device (created by the library on first use, default
 *     priority), forked from `stream` with an event after the work queued
 *     before it and joined back into `stream` with an event before the call
 *     returns; to the caller the call behaves as if all of it ran on
 *     `stream`.  The caller keeps the buffers alive until the stream has
 *     finished the work.
 *   - pos is row-major n x 3 (x0,y0,z0,x1,...), mass and soft have n entries.
 *     All caller arrays of one call share the dtype `dt` (SF_F32 or SF_F64).
 *     Particles [0, n_gas) are gas, [n_gas, n) are sinks.
 *   - soft is the compact-support radius h (> 0): the law is Newtonian for
 *     r >= max(h_i, h_j).
 *   - Outputs are written (never accumulated) in the caller's dtype and
 *     particle order.
 *   - Every call returns an sf_status and never aborts or prints.  Argument
 *     checks happen before anything is enqueued.  HIP failures map to
 *     SF_E_DEVICE, allocation failures to SF_E_NOMEM (no partial handle is
 *     leaked).  sf_grav_last_error() gives a message for the calling thread.
 *   - The library allocates its device scratch with stream-ordered
 *     allocation on `stream` and keeps freed blocks in a per-stream cache
 *     (at most 64 GiB) for later calls on the same stream;
 *     sf_grav_release_cache() returns the cache to HIP.
 *   - Test hook: with SF_GRAV_FAIL_ALLOC=k in the environment, the k-th
 *     device allocation of every entry-point call fails (SF_E_NOMEM; the
 *     call releases what it had allocated, and a handle passed to it keeps
 *     its previous state).
 */
#ifndef SF_GRAV_H
#define SF_GRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sf_grav_tree_s *sf_grav_tree; /* opaque, library owned */

typedef enum {
    SF_OK = 0,
    SF_E_INVALID = 1,     /* bad argument or option (nothing was enqueued)   */
    SF_E_NOMEM = 2,       /* device or host allocation failed                 */
    SF_E_DEVICE = 3,      /* a HIP call failed                                */
    SF_E_STATE = 4,       /* handle does not match the call (n, dtype, ...)   */
    SF_E_UNSUPPORTED = 5, /* option combination not implemented               */
    SF_E_INTERNAL = 6     /* a kernel hit a fixed capacity (see message)      */
} sf_status;

typedef enum { SF_F32 = 0, SF_F64 = 1 } sf_dtype;

/* Arithmetic form of the interaction kernels.
 *   SF_FP32C: FP32 pair arithmetic on coordinates relative to the target
 *             group's (or tile's) centre, per-target compensated (two-sum)
 *             accumulation, FP64 node moments; output = round(hi + lo).
 *   SF_FP32 : absolute FP32 coordinates, plain FP32 accumulation.
 *   SF_FP64 : FP64 throughout.
 * Node moments are always accumulated in FP64 and the sink-sink part is
 * always FP64, whatever the form. */
typedef enum { SF_FP32C = 0, SF_FP32 = 1, SF_FP64 = 2 } sf_form;

typedef struct {
    uint32_t struct_size; /* = sizeof(sf_grav_opts); ABI check              */
    int32_t form;         /* sf_form, default SF_FP32C                       */
    double G;             /* gravitational constant, default 1              */
    double theta;         /* opening angle theta = L/r, >= 0, default 0.5   */
    int32_t order;        /* node expansion: 0 monopole, 2 quadrupole; def 2 */
    int32_t leaf_cap;     /* a cell holding more is split, 1..64, default 32 */
    int32_t group_cap;    /* max targets per walk group, 1..64, default 32  */
    int32_t validate;     /* 1: check finite inputs, h > 0, m >= 0 (one pass) */
    int64_t n_gas;        /* particles [0,n_gas) are gas; default -1 = all   */
    int32_t collect_stats;/* 1: record per-group interaction counts and list
                             checksums (sf_grav_get_stats)                  */
    int32_t timing;       /* 1: record hipEvents around each phase (tree)    */
    double alpha;         /* relative (acceleration-based) opening criterion,
                             Sec. 2.2: with alpha >= 0 a node is also opened
                             when G M L^2 > alpha |g|min r^4, |g|min the
                             smallest |g| of the task's targets in the field
                             given to sf_grav_tree_set_field and r as for
                             theta; < 0 (default -1) switches it off;
                             alpha = 0 opens every node (direct sum)         */
} sf_grav_opts;

/* Fill *o with the defaults above (struct_size set).  Never fails. */
void sf_grav_opts_default(sf_grav_opts *o);

/* Build the octree for the tree path (Sec. 2.2: recursive subdivision into
 * octants).  Steps on `stream`: bounding box, 63-bit Morton keys (21 bits per
 * axis, FP64 quantisation), stable LSD radix sort (ties keep input order),
 * gather into sorted SoA, topology (a cell is split while it holds more than
 * leaf_cap particles and is above level 21), FP64 moments (mass, centre of
 * mass, traceless quadrupole, max softening; a second set over gas only, used
 * for sink targets), and target groups.  One device->host read of the node
 * and group counts synchronises `stream` once.
 * The handle keeps its own sorted copy of pos/mass/soft: later calls on the
 * handle use the values captured here.  Release with sf_grav_tree_free.
 * Errors: SF_E_INVALID (NULL pointers, n < 1, bad options), SF_E_UNSUPPORTED
 * (n > 2^25, or more than 2^27 nodes), SF_E_NOMEM, SF_E_DEVICE. */
sf_status sf_grav_build_tree(const void *pos, const void *mass, const void *soft,
                             int64_t n, sf_dtype dt, const sf_grav_opts *o,
                             void *stream, sf_grav_tree *out);

/* Accelerations (n x 3) and potentials (n; may be NULL) of every particle.
 * tree != NULL: tree path on the handle's particles; n and dt must equal the
 *   handle's (else SF_E_STATE); pos/mass/soft may be NULL (ignored).
 *   theta, order, form, G come from *o; leaf_cap/group_cap from the build.
 * tree == NULL: direct path over pos/mass/soft (all pairs, no tree kept;
 *   n > 2^25 gives SF_E_UNSUPPORTED).
 * With opts.alpha >= 0 the tree path needs a field set on the handle by
 * sf_grav_tree_set_field (else SF_E_STATE).
 * The tree path reads back the walk's capacity-guard flag at the end of the
 * call, and the direct path with validate = 1 reads back the validation
 * flag: each synchronises `stream` once.
 * Errors: SF_E_INVALID, SF_E_STATE, SF_E_NOMEM, SF_E_DEVICE, SF_E_INTERNAL. */
sf_status sf_grav_accel(sf_grav_tree tree, const void *pos, const void *mass,
                        const void *soft, int64_t n, sf_dtype dt,
                        const sf_grav_opts *o, void *acc, void *pot, void *stream);

/* Adjoint: given upstream gradients g_acc (n x 3) and g_pot (n, or NULL =
 * zero) of a scalar loss L, write dL/dpos (n x 3), dL/dmass (n), dL/dsoft (n);
 * any of the three outputs may be NULL.  For the tree path this is the exact
 * derivative of the tree approximation with its opening decisions held fixed
 * (the interaction lists are recomputed, not stored); it flows through node
 * mass, centre of mass and quadrupole.  A pair's softening derivative goes to
 * the particle with the larger radius (half to each on a tie).
 * Each forward tree walk records every group's cost in the handle; once one
 * has run, the tree adjoint walks the groups from the most costly down (by
 * exact cost for trees of at most 32 groups per resident wavefront, else by
 * power-of-two cost class with Morton order inside a class), before that in
 * Morton order.  The order changes only the summation order of its FP64
 * accumulations.
 * Same path selection, errors and synchronisation as sf_grav_accel. */
sf_status sf_grav_accel_backward(sf_grav_tree tree, const void *pos,
                                 const void *mass, const void *soft, int64_t n,
                                 sf_dtype dt, const sf_grav_opts *o,
                                 const void *g_acc, const void *g_pot,
                                 void *g_pos, void *g_mass, void *g_soft,
                                 void *stream);

/* Radiation sums that ride on the gravity walk, for gas cells (sinks get
 * zeros), with the opening decisions of sf_grav_accel:
 *   column: n x 6, the gas column density averaged over each of six
 *     angular bins around the cell (Sec. 3.1: FUV optical depths summed into
 *     angular bins during the gravity pass, 6 bins by default; the optical
 *     depth of a bin is kappa_FUV times its column).  The bins are the faces
 *     of a cube: a direction d = x_source - x_cell belongs to the face of its
 *     largest |d_k| (ties to the lower axis), in the order +x -x +y -y +z -z,
 *     each spanning 4 pi/6 sr; a bin holds sum m / (Omega_bin r^2), the
 *     column density averaged over its solid angle, a gas particle with r^2
 *     softened to r^2 + (h/2.8)^2, an accepted node as its gas mass at its gas
 *     centre of mass;
 *   e_ir: n, the IR energy density from stars (Sec. 3.3),
 *     sum_s L_s / (4 pi c r^2) over sinks, r^2 softened to r^2 + (h_s/2.8)^2,
 *     an accepted node as its total sink luminosity at the luminosity centre.
 * lum: n luminosities in caller order (only sink entries are read; NULL:
 * no stars); c_light: the speed of light in the caller's units (> 0, used
 * for e_ir).  Either output may be NULL (not both).  A group's targets
 * share the wave's lanes, floor(64 / group size) lanes each.  Synchronises
 * `stream`.
 * Errors: SF_E_INVALID (NULL tree, both outputs NULL, c_light <= 0 with
 * e_ir, bad options), SF_E_STATE, SF_E_NOMEM, SF_E_DEVICE, SF_E_INTERNAL. */
sf_status sf_grav_rad_sums(sf_grav_tree tree, const void *lum, double c_light,
                           const sf_grav_opts *o, void *column, void *e_ir, void *stream);

/* Accelerations and potentials with the symmetrised adaptive gas-gas
 * softening of Sec. 2.2.1 (gas softening follows each cell's kernel radius
 * H_i, with the symmetrisation and extra terms that keep momentum and energy
 * conserved), on the handle's tree with the same opening decisions as
 * sf_grav_accel.  Gas-gas pairs use the average of the two cells' softened
 * kernels, F_ij = (F(r, h_i) + F(r, h_j))/2 (P likewise), and the
 * acceleration of gas cell i gains
 *     -(G/2) sum_j [z_i W_r(r, h_i) + (m_j/m_i) z_j W_r(r, h_j)] d / r,
 * z = zeta/Omega, W the M4 cubic spline of support h normalised to 1, with
 * n_i = sum_j W(r_ij, h_i) over gas cells (self included),
 * zeta_i = (dh_i/dn_i) sum_{j != i} m_j dP(r_ij, h_i)/dh,
 * Omega_i = 1 - (dh_i/dn_i) sum_j dW(r_ij, h_i)/dh and dh/dn = -h/(3 n):
 * the force is then the exact gradient of the total potential energy when
 * every kernel radius satisfies the neighbour-number constraint
 * (4 pi/3) h_i^3 n_i = N_NGB (32 in Table 1).  The library does not solve
 * for h: the handle's soft values of gas cells are taken as those radii.
 * Gas-sink and sink-sink pairs keep the larger-radius rule (sink fields are
 * those of sf_grav_accel).
 * acc: n x 3 (required); pot: n; aux: n x 2 (Omega, zeta); caller order and
 * dtype.  The sink walk of sf_grav_accel, then two group walks (the
 * neighbour sums, the forces).  opts.collect_stats records nothing here.
 * Synchronises `stream`.
 * Errors: as sf_grav_accel on a tree. */
sf_status sf_grav_accel_adaptive(sf_grav_tree tree, const sf_grav_opts *o, void *acc, void *pot,
                                 void *aux, void *stream);

/* Tidal tensor T = -grad grad Phi and jerk j = da/dt of every particle,
 * computed in the same tree walk as its acceleration and potential (Sec.
 * 2.2: T and j are summed in the same pass as g, with the same opening
 * decisions, from the monopole contributions of accepted nodes and the
 * spatial derivatives of the softened pair kernel; with d = x_j - x_i,
 * w = v_j - v_i and F' = dF/dr:
 *     T_i = -G sum_j m_j [F I + (F'/r) d d^T],
 *     j_i =  G sum_j m_j [F w + (F'/r) (d . w) d]).
 * The acceleration and potential keep the node expansion of opts.order, so
 * they equal sf_grav_accel's on the same handle to rounding.  Sink targets
 * add the exact FP64 sum over the other sinks for all four quantities.
 * tree: a built handle (NULL gives SF_E_UNSUPPORTED: theta = 0 on a tree
 *   gives the all-pairs sum); n, dtype and particles are the handle's.
 * vel:  n x 3 velocities, caller order, handle dtype; needed only for jerk.
 * acc:  n x 3 (required); pot: n; tidal: n x 6 as xx yy zz xy xz yz;
 *   jerk: n x 3 -- each optional except acc, caller order and dtype.
 * A group's targets share the wave's lanes, floor(64 / group size) lanes
 * each; arithmetic in opts.form, node velocities as FP64 mass-weighted means.
 * Synchronises `stream` once (capacity-guard flag).
 * Errors: SF_E_INVALID (NULL acc, jerk without vel, bad options),
 * SF_E_STATE, SF_E_UNSUPPORTED, SF_E_NOMEM, SF_E_DEVICE, SF_E_INTERNAL. */
sf_status sf_grav_accel_tidal(sf_grav_tree tree, const void *vel, const sf_grav_opts *o,
                              void *acc, void *pot, void *tidal, void *jerk, void *stream);

/* Sinks-only pass (Sec. 2.3.2: the accelerations and jerks of all sinks in a
 * special sinks-only gravity pass), FP64, exact direct sum over the sinks
 * with the softened kernel (h_ss' = max(h_s, h_s')).  Arrays are FP64
 * device pointers over the n sinks only: pos, vel n x 3; mass, soft n.
 * Outputs (each optional except acc): acc n x 3, pot n, jerk n x 3,
 * tidal n x 6 (xx yy zz xy xz yz), times n x 4 with the two-body time
 * scales of Sec. 2.3.1 -- t_c,min = min sqrt(r^2 + eps^2) / |v_ss'| and
 * t_dyn,min = min sqrt((r^2 + eps^2)^(3/2) / (G (m_s + m_s'))) over the other
 * sinks, eps = h_s / 2.8 -- then, for eta > 0, the 2-body timestep
 * sqrt(eta) / (1/t_c,min + 1/t_dyn,min) and the tidal timestep
 * sqrt(eta) (|T|_F^2 / 6)^(-1/4) (0 for eta <= 0; a lone sink gets infinite
 * time scales).  jerk and times need vel.  Enqueued on `stream`, no
 * allocation, no synchronisation.
 * Errors: SF_E_INVALID (NULL pos/mass/soft/acc, n < 1, jerk or times
 * without vel, NaN G or eta), SF_E_DEVICE. */
sf_status sf_grav_sinks(const double *pos, const double *vel, const double *mass,
                        const double *soft, int64_t n, double G, double eta, double *acc,
                        double *pot, double *jerk, double *tidal, double *times, void *stream);

/* One step dt of the modified 4th-order Hermite scheme for all n sinks
 * (Sec. 2.3.2, Eqs. predictor and corrector): a sinks-only pass at the
 * start (a0, j0), the prediction x + v dt + a0 dt^2/2 + j0 dt^3/6,
 * v + a0 dt + j0 dt^2/2, a second pass at the predicted state (a, j), then
 * v <- v0 + (a + a0) dt/2 + (j0 - j) dt^2/12 and, with that v,
 * x <- x0 + (v + v0) dt/2 + (a0 - a) dt^2/12.  pos and vel (FP64, n x 3,
 * device) are updated in place; mass and soft as in sf_grav_sinks.
 * Enqueued on `stream` (scratch from the library's cache), no
 * synchronisation.
 * Errors: SF_E_INVALID (NULL, n < 1, NaN dt or G), SF_E_NOMEM, SF_E_DEVICE. */
sf_status sf_grav_sink_hermite(double *pos, double *vel, const double *mass, const double *soft,
                               int64_t n, double G, double dt, void *stream);

/* Free a handle: synchronises the stream of the last call made on it, then
 * returns its memory to the library's cache.  NULL is a no-op. */
sf_status sf_grav_tree_free(sf_grav_tree tree);

/* Previous field for the relative opening criterion (Sec. 2.2: the error
 * estimate of a node is compared with the target's total field, which a
 * simulation knows from its previous step).  acc_prev: n x 3, caller order,
 * the handle's dtype (device pointer, read before the call's work ends).
 * The handle keeps |g| of every particle (FP64, correctly rounded
 * sqrt((gx^2 + gy^2) + gz^2)) and the smallest |g| of each target group;
 * later tree calls with opts.alpha >= 0 use them, until the next call of this
 * function.  Enqueued on `stream`, no synchronisation.
 * Errors: SF_E_INVALID (NULL), SF_E_STATE (no tree), SF_E_NOMEM, SF_E_DEVICE. */
sf_status sf_grav_tree_set_field(sf_grav_tree tree, const void *acc_prev, void *stream);

/* Refit: new positions, masses and softening radii (caller order, the
 * handle's n and dtype) on a frozen tree.  Keys, order, topology, node cubes
 * and group ranges stay as built; the handle's sorted copy of the particles,
 * the node moments and the group boxes are recomputed.  Meant for small
 * displacements (finite differences of the tree approximation with fixed
 * topology): the safety tests of the walk use the frozen cubes, so a particle
 * moved out of its cell may have a softened pair treated as Newtonian.  The
 * list checksums of sf_grav_get_stats show whether the walk's decisions
 * changed.  Enqueued on `stream`, no synchronisation.
 * Errors: SF_E_INVALID (NULL), SF_E_STATE (no tree), SF_E_NOMEM, SF_E_DEVICE. */
sf_status sf_grav_tree_refit(sf_grav_tree tree, const void *pos, const void *mass,
                             const void *soft, void *stream);

/* Statistics of the last tree accel on the handle made with
 * opts.collect_stats = 1 (synchronises the handle's stream).
 *   n_pc, n_pp: accepted-node and particle-pair interactions summed over the
 *               gas targets (each group's list times its gas targets);
 *   hist[b]:    groups whose list holds L = nodes + particles entries with
 *               2^b <= L < 2^(b+1) (bin 0 also counts L = 0; bin 31 all
 *               longer lists);
 *   checksum:   order-independent hash of every group's decisions (which
 *               nodes were accepted, which leaves opened); equal checksums
 *               mean, up to hash collisions, identical interaction lists.
 *               Per-group values: sf_grav_tree_export(SF_EXPORT_GROUP_CKS).
 *               Sink targets' lists are not included.
 * Errors: SF_E_INVALID (NULL, struct_size), SF_E_STATE (no tree or no
 * statistics), SF_E_NOMEM, SF_E_DEVICE. */
typedef struct {
    uint32_t struct_size;  /* = sizeof(sf_grav_stats) */
    int32_t max_level;
    int64_t n_nodes;
    int64_t n_leaves;
    int64_t n_groups;
    int64_t n_pc;
    int64_t n_pp;
    int64_t hist[32];
    uint64_t checksum;
} sf_grav_stats;

sf_status sf_grav_get_stats(sf_grav_tree tree, sf_grav_stats *out);

/* Allocation-free variant of the direct path of sf_grav_accel (tree ==
 * NULL), for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, kernels and results as sf_grav_accel(NULL, ...), but every
 * scratch buffer is carved out of one fixed device array of 96 MiB inside
 * the library (each device the library runs on holds its own copy until the
 * process ends); the call makes no device allocation and no free.
 * Limit: n <= 2^19 = 524,288 particles (any dtype, form and sink count).
 * Every call on a device shares that device's array and leaves its contents
 * behind (the call clears what must start at zero): calls that overlap on
 * one device, on any streams or threads, race and give undefined results.
 * No synchronisation unless opts.validate = 1 (one stream sync, as in
 * sf_grav_accel).
 * Errors: SF_E_INVALID (as sf_grav_accel), SF_E_UNSUPPORTED (n > 2^19),
 * SF_E_DEVICE. */
sf_status sf_grav_accel_direct_noalloc(const void *pos, const void *mass, const void *soft,
                                       int64_t n, sf_dtype dt, const sf_grav_opts *o,
                                       void *acc, void *pot, void *stream);

/* Return every device block the library keeps cached for reuse to HIP
 * (synchronises each device that owns cached blocks, then trims its default
 * memory pool).  *live_bytes (may be NULL) receives the bytes still handed
 * out: held by live handles or by calls in progress on other threads.
 * Errors: SF_E_DEVICE. */
sf_status sf_grav_release_cache(size_t *live_bytes);

/* Sizes of a built tree. */
typedef struct {
    uint32_t struct_size;  /* = sizeof(sf_grav_tree_info) */
    int32_t max_level;
    int64_t n;
    int64_t n_gas;
    int64_t n_nodes;
    int64_t n_groups;
    int64_t n_leaves;
} sf_grav_tree_info;

sf_status sf_grav_get_tree_info(sf_grav_tree tree, sf_grav_tree_info *info);

/* Copy one of the handle's arrays to host memory (synchronises the stream).
 * `bytes` must equal the array's size exactly (count x element size).
 *   SF_EXPORT_KEYS        uint64 [n]       sorted Morton keys
 *   SF_EXPORT_ORDER       int32  [n]       sorted position -> input index
 *   SF_EXPORT_NODE_LEVEL  int32  [n_nodes] node arrays, breadth-first:
 *   SF_EXPORT_NODE_FIRST  int32  [n_nodes]   level 0, 1, ... ; within a level
 *   SF_EXPORT_NODE_COUNT  int32  [n_nodes]   in particle order; children of a
 *   SF_EXPORT_NODE_PARENT int32  [n_nodes]   node are contiguous (-1: none)
 *   SF_EXPORT_NODE_CHILD  int32  [n_nodes] first child index (-1 for leaves)
 *   SF_EXPORT_NODE_NCHILD int32  [n_nodes]
 *   SF_EXPORT_GROUP_FIRST int32  [n_groups] target groups in particle order
 *   SF_EXPORT_GROUP_COUNT int32  [n_groups]
 *   SF_EXPORT_NODE_MASS   double [n_nodes] node mass (all particles)
 *   SF_EXPORT_NODE_COM    double [n_nodes x 3] centre of mass
 *   SF_EXPORT_NODE_QUAD   double [n_nodes x 6] Qxx Qyy Qzz Qxy Qxz Qyz
 *   SF_EXPORT_GROUP_NPC   int32  [n_groups] accepted nodes of the last
 *   SF_EXPORT_GROUP_NPP   int32  [n_groups]   accel with collect_stats=1, and
 *                                             opened-leaf particles
 *   SF_EXPORT_GROUP_CKS   uint64 [n_groups] list checksum of each group (same
 *                                             accel)
 * Errors: SF_E_INVALID (unknown id, NULL, wrong size), SF_E_STATE (stats not
 * collected), SF_E_DEVICE. */
typedef enum {
    SF_EXPORT_KEYS = 0,
    SF_EXPORT_ORDER = 1,
    SF_EXPORT_NODE_LEVEL = 2,
    SF_EXPORT_NODE_FIRST = 3,
    SF_EXPORT_NODE_COUNT = 4,
    SF_EXPORT_NODE_PARENT = 5,
    SF_EXPORT_NODE_CHILD = 6,
    SF_EXPORT_NODE_NCHILD = 7,
    SF_EXPORT_GROUP_FIRST = 8,
    SF_EXPORT_GROUP_COUNT = 9,
    SF_EXPORT_NODE_MASS = 10,
    SF_EXPORT_NODE_COM = 11,
    SF_EXPORT_NODE_QUAD = 12,
    SF_EXPORT_GROUP_NPC = 13,
    SF_EXPORT_GROUP_NPP = 14,
    SF_EXPORT_GROUP_CKS = 15
} sf_export_id;

sf_status sf_grav_tree_export(sf_grav_tree tree, int32_t what, void *host_dst,
                              size_t bytes);

/* Phase timers of the last build / accel / backward on a handle, recorded
 * with hipEvents on the call's stream when opts.timing = 1 (milliseconds;
 * -1 for a phase that did not run).  Synchronises the stream.
 *   build:    [0] sort (box, keys, radix sort, gather)  [1] topology
 *             [2] moments  [3] groups
 *   accel:    [4] sink-sink FP64  [5] group walk  [6] sink walk
 *   backward: [7] sink-sink FP64  [8] group walk  [9] sink walk
 *             [10] push-down and output
 * Phases 4, 6, 7 and 9 run on the library's second stream beside the group
 * walk; their times include waiting for execution slots that the group walk
 * holds.
 * Errors: SF_E_INVALID (NULL, struct_size), SF_E_DEVICE. */
typedef struct {
    uint32_t struct_size;   /* = sizeof(sf_grav_timings) */
    int32_t n_phases;       /* = 11 */
    double ms[16];
} sf_grav_timings;

sf_status sf_grav_get_timings(sf_grav_tree tree, sf_grav_timings *out);

/* Static text for a status code. */
const char *sf_grav_strerror(sf_status s);

/* Message of the last failing call on this host thread ("" if none). */
const char *sf_grav_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SF_GRAV_H */

/*
 * tetfmm.h -- C ABI of the MI355X (gfx950) tetrahedral Fast Multipole library.
 *
 * The library evaluates the magnetic scalar potential of a tetrahedral mesh
 * whose magnetisation is affine on every tetrahedron (Palmesi et al., "Highly
 * Parallel Demagnetization Field Calculation Using the Fast Multipole Method
 * on Tetrahedral Meshes with Continuous Sources", eq. approx1):
 *
 *     u(x) = 1/(4 pi) sum_T int_T M_T(r') . grad' (1 / |x - r'|) dr'
 *
 * at a set of target points (by default the mesh nodes), either by the Fast
 * Multipole Method of Secs. 2-3 (octree, MAC, dual tree traversal, Cartesian
 * Taylor expansions of order p, exact near-field integrals) or by the O(N^2)
 * direct sum of the exact tet-to-target integrals (Sec. 2.1).
 *
 * Conventions
 *  - Every function returns 0 on success or a negative TFMM_E* code; the
 *    message of the last failure on the calling thread is tfmm_last_error().
 *    No C++ exception crosses this interface.
 *  - The caller owns every buffer it passes.  tfmm_plan_create copies the
 *    mesh; the caller may free its arrays when it returns.
 *  - Device pointers are HIP device allocations on the plan's device (for
 *    example torch tensors on that device).  Work is queued on the HIP stream
 *    passed in (NULL = the default stream) and is asynchronous: the caller
 *    synchronises that stream before reading the output.
 *  - A plan is not thread-safe: one evaluation at a time per plan.
 *  - Units: u carries the 1/(4 pi) of eq. approx1; u has the units of
 *    M times length.
 */
#ifndef TETFMM_H
#define TETFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define TFMM_OK 0
#define TFMM_EINVAL (-1)     /* bad sizes or parameters */
#define TFMM_EINDEX (-2)     /* tet node index out of range */
#define TFMM_EDEGEN (-3)     /* tetrahedron of (near) zero volume */
#define TFMM_ENONFINITE (-4) /* NaN or Inf in the inputs */
#define TFMM_ENOMEM (-5)     /* host or device allocation failed */
#define TFMM_EDEVICE (-6)    /* HIP error, or no usable device */
#define TFMM_ENOTSUP (-7)    /* valid request the library does not support */

/* largest expansion order p accepted */
#define TFMM_PMAX 10

/* M2L arithmetic (P2M, M2M, L2L, L2P and the near field are always FP64) */
#define TFMM_M2L_FP64 0 /* FP64 matrix cores */
#define TFMM_M2L_FP32 1 /* FP32 matrix cores on level-scaled expansions, FP64 elsewhere */
#define TFMM_M2L_BF16X3 2 /* FP32 operands split into BF16 parts, 3 part products, FP32 accumulation */
#define TFMM_M2L_BF16X6 3 /* as BF16X3 with 6 part products (about FP32 accuracy) */

/* Near-field pairs 2 <= |x - centroid| / diameter < 6 (Sec. 2.1's exact
 * integral elsewhere; the diameter is the tet's longest edge) */
#define TFMM_SUR_OFF 0   /* exact integral for every near pair */
#define TFMM_SUR_MLP 1   /* the attached network (quadrupole expansion + learned residual) */
#define TFMM_SUR_GAUSS 2 /* control: 27-point collapsed Gauss-Jacobi rule (degree 5) */
#define TFMM_SUR_QUAD 3  /* control: the tet's quadrupole expansion alone (the network's base) */

typedef struct tfmm_plan_s *tfmm_plan; /* opaque, owned by the library */
typedef struct tfmm_batch_s *tfmm_batch; /* opaque, owned by the library */

/*
 * Parameters of the method.
 *  p          expansion order: multipole and local expansions hold every
 *             Taylor term with |n| <= p (Sec. 2.2), (p+1)(p+2)(p+3)/6
 *             coefficients; M2L keeps |n| + |m| <= p.  1 <= p <= TFMM_PMAX.
 *  leaf_size  an octree cell is split while it holds more than leaf_size
 *             tets (by centroid) or targets (Sec. 3.1).  >= 1.
 *  theta      multipole acceptance parameter (Sec. 3.2): cells A (target)
 *             and B (source) interact through M2L iff
 *             r_tgt(A) + r_src(B) < theta |c_A - c_B|.  0 < theta < 1.
 *  m2l_precision  TFMM_M2L_FP64, TFMM_M2L_FP32, TFMM_M2L_BF16X3 or
 *             TFMM_M2L_BF16X6 (the translation operands are scaled per level
 *             so that all magnitudes are O(1); the BF16 forms split the FP32
 *             operands into three BF16 parts and sum 3 or 6 of the part
 *             products in FP32; the local expansions are accumulated and
 *             stored in FP64).
 *  surrogate  TFMM_SUR_OFF, or how the near-field pairs 2 to 6 tet diameters
 *             apart are evaluated: TFMM_SUR_MLP (the learned surrogate; a
 *             network must be attached by tfmm_surrogate_train or
 *             tfmm_surrogate_load before the first evaluation), or one of the
 *             controls TFMM_SUR_GAUSS, TFMM_SUR_QUAD.  Closer pairs always
 *             take the exact integral.  Ignored by point-dipole plans and
 *             while the stored near field is on.
 *  device     HIP device ordinal; -1 builds a host-only plan (tree and lists
 *             without any device allocation: only tfmm_plan_stats,
 *             tfmm_plan_lists and tfmm_plan_cells work on it).
 */
typedef struct {
    int32_t p;
    int32_t leaf_size;
    double theta;
    int32_t m2l_precision;
    int32_t surrogate;
    int32_t device;
} tfmm_params;

/* Sizes of a plan. */
typedef struct {
    int64_t n_nodes, n_tets, n_targets;
    int64_t n_cells, n_leaves, depth;
    int64_t n_m2l;       /* M2L cell pairs */
    int64_t n_p2p;       /* P2P leaf pairs */
    int64_t n_p2p_pairs; /* target x tet pairs integrated directly */
    int64_t ncoef;       /* (p+1)(p+2)(p+3)/6 */
    int64_t device_bytes; /* device memory held by the plan */
    double setup_seconds; /* wall time of tfmm_plan_create */
    int64_t near_nnz;     /* (target, node) coefficients of the stored near field, 0 if none */
    int64_t near_bytes;   /* device bytes of the stored near field */
    int32_t m2l_keys_per_item; /* schedule: M2L keys per workgroup item (tfmm_plan_autotune) */
    int32_t p2p_wide;          /* schedule: 1 if one-field P2P blocks run four wavefronts */
    /* one-field near field over shared mesh entities: (target, entity)
       evaluations per evaluation (nodes: a distance, edges: a logarithm,
       faces: a solid angle) */
    int64_t p2p_node_evals, p2p_edge_evals, p2p_face_evals;
    int64_t n_band_pairs; /* near pairs of the surrogate's band (0 until first used) */
    int32_t surrogate;    /* TFMM_SUR_* of the plan */
    int32_t surrogate_hidden; /* width of the attached network, 0 if none */
    int32_t level_order[22];  /* expansion order of octree levels 0..21 (all p unless set) */
    int32_t m2l_packed;         /* schedule: 1 if M2L of fewer than 16 fields runs packed by key */
    int32_t m2l_groups_per_item; /* schedule: key groups per packed M2L workgroup item */
    int64_t m2l_groups;         /* packed M2L: groups of 16 matrix-core columns of one key (one field; 0 until built) */
} tfmm_stats;

/*
 * Build a plan: validate the mesh, orient every tet to positive volume,
 * build the octree (Sec. 3.1), the cell radii (Sec. 3.2) and the M2L and
 * P2P interaction lists by the dual tree traversal (Sec. 3.3), then upload
 * everything the evaluation needs to the device.
 *
 *  nodes    host, [n_nodes][3] double, node coordinates
 *  tets     host, [n_tets][4] int32, 0-based node indices, either orientation
 *  targets  host, [n_targets][3] double, or NULL to use the nodes as targets
 *  prm      parameters (see tfmm_params)
 *  out      receives the plan; NULL on failure
 * Errors: TFMM_EINVAL (sizes: fewer than 4 nodes or no tet, explicit
 *         targets with n_targets < 1, NULL arrays; p, leaf_size, theta),
 *         TFMM_EINDEX, TFMM_EDEGEN (|det| <= 1e-12 * mean edge^3 for some
 *         tet), TFMM_ENONFINITE, TFMM_ENOMEM, TFMM_EDEVICE.
 */
int tfmm_plan_create(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                     const double *targets, int64_t n_targets, const tfmm_params *prm, tfmm_plan *out);

/*
 * Plan for point dipoles (the paper's second source kind, the "Mag FMM" of
 * Sec. 4: point-like dipole clouds).  Source i is a dipole at points[i]; the
 * tree, radii, lists and translations are those of tfmm_plan_create with each
 * source's centroid and farthest point being the point itself; P2M is the
 * dipole expansion Q_n = sum_i sum_k n_k m_ik (y_i - c)^(n - e_k) and the
 * near field the dipole potential m . (x - y)/(4 pi |x - y|^3), a target at
 * a dipole's own position taking nothing from that dipole.
 *  points   host, [n_points][3] double
 *  targets  host, [n_targets][3] double, or NULL for the points themselves
 * tfmm_evaluate / tfmm_direct then take M = the dipole moments, device
 * [F][n_points][3], and write u [F][n_targets].  The stored near field, the
 * demagnetising energy and the surrogate return TFMM_ENOTSUP on such plans.
 * Errors: as tfmm_plan_create (TFMM_EINVAL also when all points coincide).
 */
int tfmm_plan_create_points(const double *points, int64_t n_points, const double *targets, int64_t n_targets,
                            const tfmm_params *prm, tfmm_plan *out);

/*
 * FMM evaluation (Secs. 2-3: P2M, M2M, M2L, L2L, L2P plus the exact
 * near-field P2P of Sec. 2.1) of F fields.
 *  M  device, [F][n_nodes][3] double: nodal magnetisation, affine per tet
 *  u  device, [F][n_targets] double: potential at the targets (overwritten)
 * Asynchronous on `hip_stream` (a hipStream_t, NULL = default stream).
 * Errors: TFMM_EINVAL (F < 1, NULL pointers, host-only plan), TFMM_EDEVICE.
 */
int tfmm_evaluate(tfmm_plan plan, const double *M, int32_t F, double *u, void *hip_stream);

/*
 * O(N^2) direct sum of the exact tet-to-target integrals (Sec. 2.1) over all
 * targets and all tets, in FP64.  Pairs within 3 tet diameters (longest edge)
 * of the tet's centroid take the closed form; farther pairs, where the closed
 * form cancels, a collapsed Gauss-Jacobi rule of degree 13, 11, 9 or 7 by
 * distance band (3-6, 6-12, 12-24, >= 24 diameters; rule error below ~1e-14
 * of the pair's size).  Point-dipole plans sum the dipole potentials.  Same
 * arguments and errors as tfmm_evaluate.
 */
int tfmm_direct(tfmm_plan plan, const double *M, int32_t F, double *u, void *hip_stream);

/*
 * Stored near-field operator (Sec. 2.1 "Direct Vertex Interaction" and the
 * storage discussion of Sec. 3: the direct part is a linear map from the
 * nodal magnetisation to the target potentials, node-to-node vectors kept for
 * a fixed mesh).  on != 0 assembles, once, the 3-vector coefficient of every
 * (target, node) pair in the near field (the nodes of the tets of the P2P
 * source leaves of the target's leaf; nnz and bytes in tfmm_stats) on
 * `hip_stream` and synchronises it; later evaluations of the plan apply it
 * (reading it from device memory) instead of integrating the pairs.  on == 0
 * frees it.  The results agree with the integrating path up to rounding.
 * Memory: 24 bytes per (target, node) coefficient plus padding, e.g. about
 * 0.8 GB for a 40^3 Kuhn cube at leaf 64, theta 0.5.
 * Errors: TFMM_EINVAL (NULL or host-only plan), TFMM_ENOMEM (device memory:
 * the plan keeps integrating), TFMM_EDEVICE.
 */
int tfmm_plan_store_near(tfmm_plan plan, int32_t on, void *hip_stream);

/*
 * Choice of expansion order and opening angle for an accuracy target (the
 * two knobs of Sec. 2.2 and Sec. 3.2 that trade accuracy for work).
 * For every p of p_list (ascending) the opening angles of theta_list are
 * tried from the largest down; each candidate plan (leaf_size,
 * m2l_precision, device from *base) evaluates the probe field M and its
 * relative L2 error is measured against the FP64 direct sum at n_sample
 * nodes drawn with `seed` (SplitMix64, without replacement).  The first
 * theta whose sampled error is at most tol / 2 (a margin for the sampling)
 * is timed (best of 3 evaluations) and the smaller thetas of that p are
 * skipped; the fastest timed candidate is returned.
 *  M      host, [n_nodes][3] double, the probe magnetisation
 *  out    p, theta, sampled error and ms of the choice; met = 0 when no
 *         candidate met the tolerance (out then holds the most accurate one,
 *         ms = -1)
 *  table  host [n_p * n_theta][4] (p, theta, error, ms; -1 where not
 *         measured), or NULL
 * Synchronous; builds and frees one plan per candidate.
 * Errors: TFMM_EINVAL (NULL pointers, tol <= 0, empty lists, p or theta out
 *         of range, host-only device), the errors of tfmm_plan_create.
 */
typedef struct {
    int32_t p;
    double theta;
    double err;     /* sampled relative L2 error vs the FP64 direct sum */
    double ms;      /* ms per evaluation of one field */
    int32_t n_tried;
    int32_t met;
} tfmm_tune_result;
int tfmm_tune_accuracy(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                       const tfmm_params *base, const double *M, double tol, int32_t n_sample, uint64_t seed,
                       const int32_t *p_list, int32_t n_p, const double *theta_list, int32_t n_theta,
                       tfmm_tune_result *out, double *table);
/* The same search for a point-dipole plan (see tfmm_plan_create_points):
 * M holds the probe dipole moments [n_points][3]; the reference is the
 * dipole direct sum at the sampled points. */
int tfmm_tune_accuracy_points(const double *points, int64_t n_points, const tfmm_params *base, const double *M,
                              double tol, int32_t n_sample, uint64_t seed, const int32_t *p_list, int32_t n_p,
                              const double *theta_list, int32_t n_theta, tfmm_tune_result *out, double *table);

/*
 * Per-level expansion orders (the accuracy knob beside theta and p that the
 * paper names as the next performance lever, Sec. 4.1): level l of the octree
 * keeps multipole and local coefficients of degree <= q_l, with
 * q_l = orders[min(l, n - 1)], 1 <= q_l <= p (the plan's p is the largest
 * order and fixes the storage).  P2M and M2M results are truncated to their
 * cell's level, M2L into a cell of level l keeps |n| + |m| <= q_l and runs
 * on matrix cores at that order, L2L results are truncated to the child's
 * level.  All q_l = p is the method as built.  The first evaluation after a
 * change builds per-level M2L tile lists (host work, synchronous).
 * Errors: TFMM_EINVAL (NULL, n < 1, an order outside [1, p]).
 */
int tfmm_plan_set_level_orders(tfmm_plan plan, const int32_t *orders, int32_t n);

/*
 * Per-level orders for an accuracy target on an existing plan (targets = its
 * nodes): candidate profiles are the uniform order p and every two-order
 * step, the levels from a split level down (or up) at p - 1 or p - 2 and the
 * others at p; each is evaluated for the probe field M (host [n_nodes][3])
 * and its relative L2 error measured against the FP64 direct sum at n_sample
 * nodes drawn with `seed`; profiles within tol / 2 are timed (best of 3) and
 * the fastest is set on the plan.  orders [22] receives the chosen order of
 * levels 0..21, *err the sampled error and *ms the time of one evaluation
 * (both -1 and the plan's orders unchanged when no profile met the
 * tolerance).  Synchronous.  Errors: TFMM_EINVAL, TFMM_EDEVICE.
 */
int tfmm_tune_level_orders(tfmm_plan plan, const double *M, double tol, int32_t n_sample, uint64_t seed,
                           int32_t *orders, double *err, double *ms);

/* Switch the near-field surrogate of an existing plan (one of TFMM_SUR_*;
 * TFMM_SUR_MLP needs an attached network by the next evaluation).  The first
 * evaluation with a mode other than TFMM_SUR_OFF lists the band's pairs once
 * (8 bytes per pair, synchronising).  Errors: TFMM_EINVAL. */
int tfmm_plan_set_surrogate(tfmm_plan plan, int32_t mode);

/* Switch the M2L arithmetic of an existing plan (one of TFMM_M2L_*). */
int tfmm_plan_set_m2l_precision(tfmm_plan plan, int32_t m2l_precision);

/* Synchronous convenience forms with host arrays (copies in and out). */
int tfmm_evaluate_host(tfmm_plan plan, const double *M, int32_t F, double *u);
int tfmm_direct_host(tfmm_plan plan, const double *M, int32_t F, double *u);

/* Sizes of the plan. */
int tfmm_plan_stats(tfmm_plan plan, tfmm_stats *out);

/*
 * Interaction lists as integer cell coordinates, for verification.
 *  kind 0 = M2L pairs, 1 = P2P pairs, 2 = the M2L pairs in the order the
 *  matrix-core tiles (16 target cells) schedule them, 3 = the M2L pairs in
 *  the order the key-packed groups of one field schedule them: kinds 2 and
 *  3 are the same set as kind 0, each pair once.
 *  out  host, [n][8] int32: levelA, ixA, iyA, izA, levelB, ixB, iyB, izB
 *       (A target cell, B source cell; a cell at level L covers
 *       [origin + i s, origin + (i+1) s) per axis with s = side / 2^L), or
 *       NULL to query the count.
 * Returns the number of pairs (>= 0) or a negative error code.
 */
int64_t tfmm_plan_lists(tfmm_plan plan, int32_t kind, int32_t *out);

/*
 * Cells, for verification.
 *  cells  host, [n_cells][6] int32: level, ix, iy, iz, n_tets, n_targets (or NULL)
 *  radii  host, [n_cells][2] double: r_src, r_tgt of Sec. 3.2 (or NULL)
 * Returns n_cells or a negative error code.
 */
int64_t tfmm_plan_cells(tfmm_plan plan, int32_t *cells, double *radii);

/*
 * Expansion coefficients left by the last tfmm_evaluate (field F-1), for
 * verification: which 0 = multipole Q_n, 1 = local l_m (Taylor coefficients,
 * u = sum_m l_m (x - c)^m), in cell order of tfmm_plan_cells and the graded
 * multi-index order (degree ascending; within a degree n_x descending, then
 * n_y descending).  out: host, [n_cells][ncoef] double.  Synchronises the
 * device.
 */
int tfmm_plan_expansions(tfmm_plan plan, int32_t which, double *out);

/*
 * The quadrature rule P2M uses to integrate the polynomial expansion
 * integrands of eq. expCoeffs exactly (Sec. 2.2): a collapsed Gauss-Jacobi
 * (conical product) rule on the unit simplex, exact to total degree
 * `degree` (0 <= degree <= 2 TFMM_PMAX).  out: host, [npts][4] double rows
 * (lambda1, lambda2, lambda3, weight), weights summing to 1/6, or NULL to
 * query npts.  Host-only; needs no device.
 */
int tfmm_simplex_rule(int32_t degree, double *out, int32_t *npts);

/* Release the plan and its device memory.  NULL is ignored. */
int tfmm_plan_destroy(tfmm_plan plan);

/* Message of the last failure on this thread ("" if none). */
const char *tfmm_last_error(void);

/*
 * Per-phase GPU time of the evaluations run since timing was switched on.
 * tfmm_set_timing(plan, 1) clears the record and makes every tfmm_evaluate
 * record a HIP event pair around each phase on its stream (no extra
 * synchronisation); tfmm_kernel_times synchronises on those events and
 * returns, per phase, the average milliseconds per evaluation and the
 * number of evaluations recorded.  Phases: 0 p2m, 1 m2m (all levels),
 * 2 m2l, 3 l2l (all levels), 4 l2p, 5 p2p.
 */
int tfmm_set_timing(tfmm_plan plan, int32_t on);
int tfmm_kernel_times(tfmm_plan plan, double *ms /* [6] */, int64_t *launches /* [6] */);

/*
 * Demagnetising field and energy from nodal potentials (P1 interpolation of
 * u on every tet): H_tet [n_tets][3] (device, input tet order, may be NULL)
 * receives H_T = -grad u, and *energy (host) the stray-field energy over mu0,
 *   E / mu0 = 1/2 sum_T int_T M . grad u = -1/2 int M . H,
 * for one field M (device [n_nodes][3]) and its potential u (device
 * [n_nodes], e.g. from tfmm_evaluate; the plan's targets must be its nodes).
 * Synchronises hip_stream.  Errors: TFMM_EINVAL, TFMM_EDEVICE.
 */
int tfmm_demag_energy(tfmm_plan plan, const double *M, const double *u, double *H_tet, double *energy,
                      void *hip_stream);

/*
 * tfmm_demag_energy without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arithmetic and H_tet as
 * tfmm_demag_energy, but the energy E / mu0 goes to a device double (energy,
 * caller-owned) and nothing is synchronised or copied to the host: the call
 * only queues two kernels on hip_stream.  The per-block partial sums live in
 * a library-owned static device array of 65,536 doubles (512 KiB), one per
 * device the library runs on, held until the process ends; hence at most
 * TFMM_NOALLOC_MAX_TETS tets.  Every call on a device shares that array:
 * calls that overlap on one device (several streams or threads) race and
 * give wrong energies; serialise them.  The first call on a device takes the
 * array's device address (hipGetSymbolAddress) and keeps it.
 * Errors: TFMM_EINVAL (NULL arguments, host-only plan, targets not the nodes,
 * more than TFMM_NOALLOC_MAX_TETS tets), TFMM_ENOTSUP (point-dipole plans),
 * TFMM_EDEVICE.
 */
#define TFMM_NOALLOC_MAX_TETS (65535LL * 256LL)
int tfmm_demag_energy_noalloc(tfmm_plan plan, const double *M, const double *u, double *H_tet, double *energy,
                              void *hip_stream);

/*
 * Mass-lumped nodal demagnetising field (the lumped L2 projection of the P1
 * field -grad u onto the nodes, as used for nodal effective fields in
 * micromagnetics next to the stray-field energy of Sec. 4.1):
 *   H_j = sum_{T ni j} (V_T / 4) H_T / sum_{T ni j} (V_T / 4).
 *  u       device [n_nodes] double, nodal potential (targets must be the nodes)
 *  H_node  device [n_nodes][3] double, written (input node order)
 * Asynchronous on hip_stream.  The first call on a plan allocates and builds
 * the lumped node volumes (kept with the plan).
 * Errors: TFMM_EINVAL, TFMM_ENOTSUP (point-dipole plans), TFMM_EDEVICE.
 */
int tfmm_demag_field_nodes(tfmm_plan plan, const double *u, double *H_node, void *hip_stream);

/*
 * Schedule tuning.  Times evaluations of one (synthetic) field on hip_stream
 * for a few choices of the M2L work item size (keys per workgroup) and of the
 * P2P workgroup shape, and keeps the fastest; the arithmetic, and so every
 * result, is the same for all choices.  Synchronises the stream; allocates
 * and frees scratch device memory for one field.
 * Errors: TFMM_EINVAL (NULL or host-only plan), TFMM_EDEVICE.
 */
int tfmm_plan_autotune(tfmm_plan plan, void *hip_stream);

/*
 * Set the schedule knobs that tfmm_plan_autotune picks: M2L keys per
 * workgroup item of the tiled form (16..4096), the P2P workgroup shape for
 * one or two fields (p2p_wide 1: four wavefronts per block; 0: one), and
 * the M2L form for fewer than 16 fields with FP64 or FP32 translations
 * (m2l_packed 1: the translations of each key are packed 16 columns at a
 * time inside blocks of target cells, m2l_groups_per_item (16..4096) such
 * groups per workgroup item; 0: target tiles run through their keys).
 * Every choice computes the same contraction (sums in another order); the
 * point is to run a given schedule (for instance the one a benchmark timed)
 * under test.  Builds the M2L work lists of the new schedule for one field
 * (synchronous).  Errors: TFMM_EINVAL (NULL or host-only plan, values out of
 * range), TFMM_EDEVICE.
 */
int tfmm_plan_set_schedule(tfmm_plan plan, int32_t m2l_keys_per_item, int32_t p2p_wide, int32_t m2l_packed,
                           int32_t m2l_groups_per_item);

/*
 * The elementary functions of the exact near-field integral (Sec. 2.1: its
 * edge logarithms and face solid angles), evaluated on the device one element
 * at a time, for checking them against an independent implementation:
 *  fn 0: ln(a/b) for positive finite a, b (one division, atanh series)
 *  fn 1: atan2(a, b) in (-pi, pi] (one division, polynomial on [0, tan(pi/8)])
 *  fn 2: a / b for finite nonzero b of moderate range (reciprocal estimate and
 *        Newton-Raphson steps)
 *  fn 3: 1/sqrt(a) for positive finite normal a (b ignored)
 * a, b, out: host arrays of n doubles.  Synchronous on `device`.
 * Errors: TFMM_EINVAL (fn, n, NULL arrays), TFMM_EDEVICE.
 */
int tfmm_elementary(int32_t fn, const double *a, const double *b, double *out, int64_t n, int32_t device);

/*
 * Ragged batches of meshes (one field each; the FMM of Secs. 2-3 on every
 * mesh).  tfmm_batch_create builds one plan per mesh i from nodes[i]
 * ([n_nodes[i]][3], host) and tets[i] ([n_tets[i]][4], host), targets = the
 * nodes, all with the parameters prm (prm->device >= 0), and one merged plan
 * over all meshes: each mesh's tree and lists normalised to its own root
 * cube (the potential scales with the cube side at fixed M) and
 * concatenated, so that one launch per phase serves every mesh and no mesh
 * interacts with another.  The caller may free its arrays on return.
 * Errors: as tfmm_plan_create (the message names the mesh), TFMM_EINVAL for
 * n_meshes < 1, NULL arrays or a host-only device.
 */
int tfmm_batch_create(int32_t n_meshes, const double *const *nodes, const int64_t *n_nodes,
                      const int32_t *const *tets, const int64_t *n_tets, const tfmm_params *prm, tfmm_batch *out);

/*
 * Evaluate every mesh of the batch: M[i] device [n_nodes_i][3] FP64 nodal
 * magnetisation, u[i] device [n_nodes_i] FP64 output (written, not added
 * to).  By default the merged plan runs: M is gathered into it (scaled by
 * each mesh's root side), evaluated, and u scattered back.  With
 * tfmm_batch_set_merged(batch, 0) the per-mesh plans run instead, spread
 * over 4 concurrent branches balanced by their P2P and M2L counts.  Either
 * sequence of launches is captured once into a HIP graph on internal
 * streams and replayed on hip_stream while the M and u pointers and the
 * plans' precision and schedule stay the same; a change re-captures.
 * Asynchronous like tfmm_evaluate.  With kernel timing enabled on the plans
 * that run, the launches run eagerly instead.
 * Errors: TFMM_EINVAL (NULL arguments), TFMM_EDEVICE.
 */
int tfmm_batch_evaluate(tfmm_batch batch, const double *const *M, double *const *u, void *hip_stream);

/* Tune the plans that evaluate the batch (tfmm_plan_autotune: the merged
 * plan, or every mesh's plan) and drop its graph. */
int tfmm_batch_autotune(tfmm_batch batch, void *hip_stream);

/* Plan of mesh i (owned by the batch: do not destroy it). */
int tfmm_batch_plan(tfmm_batch batch, int32_t i, tfmm_plan *out);

/* The merged plan over all meshes (owned by the batch: do not destroy it).
 * Its precision, stored near field and schedule are set with the plan
 * calls; its nodes are the meshes' nodes, mesh after mesh, in the frame of
 * each mesh's root cube, so it is not meant for tfmm_evaluate by itself. */
int tfmm_batch_merged_plan(tfmm_batch batch, tfmm_plan *out);

/* on = 1 (default): tfmm_batch_evaluate runs the merged plan; 0: the
 * per-mesh plans.  Errors: TFMM_EINVAL. */
int tfmm_batch_set_merged(tfmm_batch batch, int32_t on);

/* Destroy the batch, its plans and its graph.  NULL is accepted. */
int tfmm_batch_destroy(tfmm_batch batch);

/*
 * Learned near-field surrogate of the pair integral of Sec. 2.1 at
 * intermediate distance.  For a tet (diameter d = longest edge, centroid c,
 * volume V) and a target x at 2 <= rho = |x - c|/d < 6 the potential is
 * u = d * sum_{i,a} C_ia M_ia.  The tet's own multipole expansion about c
 * truncated at |n| <= 2 (dipole and quadrupole, Sec. 2.2) gives Cq in closed
 * form; a perceptron 16 -> H -> H -> H -> 12 (ReLU) maps the tet's corners
 * seen from the target (as 16 scale-free numbers: the unit direction
 * (x - c)/|x - c|, the corners about c in units of d, and 1/rho) to the
 * residual y = 2048 (C - Cq) rho^4 / (V/d^3), and the 12 coefficients are
 * contracted with the 4 nodal M exactly.  It is trained on
 * the GPU (FP32, Adam; pairs drawn from the plan's own band pairs, the exact
 * pair integrals as targets) and evaluated with BF16 weights and activations on
 * matrix cores (FP32 accumulation; inputs as two BF16 parts; the quadrupole
 * part and the contraction in FP64).  Evaluations use it for the band's
 * pairs when the plan's surrogate mode is TFMM_SUR_MLP (tfmm_params,
 * tfmm_plan_set_surrogate); the exact integral takes the closer pairs.
 */
typedef struct {
    int32_t hidden; /* hidden width: 32, 64 or 128 */
    int32_t steps;  /* Adam steps */
    int32_t batch;  /* fresh samples per step */
    float lr;       /* initial learning rate (cosine decay to lr/20) */
    uint64_t seed;
} tfmm_train_cfg;

/* Number of FP32 parameters of a network of the given width (-1 if unsupported). */
int tfmm_surrogate_param_count(int32_t hidden);

/*
 * Train a surrogate on pairs drawn from the plan's tets, attach it to the plan
 * and (when out_path is not NULL) write it: 8 bytes "TFMMSUR1", int32 hidden,
 * int32 count, count FP32 parameters (W1 [12][H], b1, W2 [H][H], b2, W3, b3,
 * W4 [H][12], b4).  *final_loss (may be NULL): mean squared error of the last
 * 5% of the steps.  Synchronous.
 * Errors: TFMM_EINVAL (arguments, host-only plan, unwritable path), TFMM_EDEVICE.
 */
int tfmm_surrogate_train(tfmm_plan plan, const tfmm_train_cfg *cfg, const char *out_path, double *final_loss);

/* Attach a surrogate written by tfmm_surrogate_train.  Errors: TFMM_EINVAL, TFMM_EDEVICE. */
int tfmm_surrogate_load(tfmm_plan plan, const char *path);

/*
 * n training samples drawn as in training (seeded): X [n][16] inputs,
 * Y [n][12] targets y; host arrays.  For checking the targets against an
 * independent pair integral.  Errors: TFMM_EINVAL, TFMM_EDEVICE.
 */
int tfmm_surrogate_samples(tfmm_plan plan, uint64_t seed, int32_t n, float *X, float *Y);

/*
 * Mean squared error and its gradient (FP32, the training kernels) of the
 * network with parameters params on the batch (X [batch][12], Y [batch][12]);
 * host arrays, run on the given device.  Errors: TFMM_EINVAL, TFMM_EDEVICE.
 */
int tfmm_surrogate_grad(int32_t hidden, const float *params, const float *X, const float *Y, int32_t batch,
                        float *grad, double *loss, int32_t device);

/*
 * u [n_targets] (device, written) = potential of the plan's near-field pairs
 * with 2 <= |x - c|/d < 6 only, for one field M (device [n_nodes][3]): by the
 * exact pair integral (use_surrogate = 0) or by the attached surrogate.  The
 * first call lists the band's pairs (synchronising).
 * Asynchronous on hip_stream.  Errors: TFMM_EINVAL (no surrogate attached,
 * NULL arguments), TFMM_EDEVICE.
 */
int tfmm_band_potential(tfmm_plan plan, int32_t use_surrogate, const double *M, double *u, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif

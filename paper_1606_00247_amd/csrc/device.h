// Device-side plan and kernel launchers of the tetrahedral FMM (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"

namespace tfmm {

// M2L runs on the harmonic reduction of the expansions: reduced multipoles
// have the (p+1)^2 indices with n_z <= 1, the per-key derivative table the
// 1 + 3p(p+1)/2 derivatives with k_z <= 2.
inline int m2l_reduced_width(int p) { return (p + 1) * (p + 1); }
inline int m2l_table_width(int p) { return 1 + 3 * p * (p + 1) / 2; }

// Far pairs of the direct sum (targets at least kFarRatio[0] longest edges
// from a tet's centroid) are integrated by collapsed Gauss-Jacobi rules of
// degree 13, 11, 9 and 7 (7^3, 6^3, 5^3 and 4^3 points, concatenated at
// kFarOff) for the distance bands [3, 6), [6, 12), [12, 24) and [24, inf)
// diameters.
constexpr int kFarBands = 4;
constexpr int kFarDeg[kFarBands] = {13, 11, 9, 7};
constexpr int kFarOff[kFarBands + 1] = {0, 343, 559, 684, 748};
constexpr double kFarRatio[kFarBands] = {3.0, 6.0, 12.0, 24.0};

// Expansion order of every octree level (levels beyond the tree unused),
// passed to kernels by value.
constexpr int kMaxLevels = 32;
struct LevelOrders {
    int8_t q[kMaxLevels];
};

// Thrown by launchers on HIP failures (converted to TFMM_EDEVICE at the ABI).
struct DeviceError {
    std::string msg;
};

void hip_check(hipError_t e, const char *what);

// Kernel timing slots
enum { KT_P2M = 0, KT_M2M, KT_M2L, KT_L2L, KT_L2P, KT_P2P, KT_COUNT };

struct DevicePlan {
    HostPlan hp;
    int device = -1;
    int ncoef = 0;  // (p+1)(p+2)(p+3)/6

    // tets in octree order: corner coordinates [12][T] (row 3*c + axis) and
    // corner node ids [4][T]
    double *tet_xyz = nullptr;
    int32_t *tet_node = nullptr;
    int32_t *tet_perm = nullptr;  // octree order -> input tet index
    // targets in octree order: [3][N], original index, leaf cell
    double *tgt_xyz = nullptr;
    int32_t *tgt_perm = nullptr;
    int32_t *tgt_leaf = nullptr;
    // cells: centres [3][C]; ints [C][8]: tbeg, tend, xbeg, xend, cbeg, nchild, parent, level
    double *cell_c = nullptr;
    int32_t *cell_i = nullptr;
    // work lists
    int32_t *p2m_cells = nullptr;  // leaves holding tets
    int32_t n_p2m_cells = 0;
    int32_t *m2m_cells = nullptr;  // per level: parents holding tets (host ranges below)
    std::vector<int32_t> m2m_level_ptr;
    int32_t *l2l_cells = nullptr;  // per level: non-root cells holding targets
    std::vector<int32_t> l2l_level_ptr;
    // M2L on matrix cores: translation keys and their derivative tables
    // D_k(rho), rho = (c_A - c_B) / side(B), in FP64 and (on demand) FP32
    int32_t *m2l_keys = nullptr;  // [nkeys][4]
    double *m2l_D = nullptr;      // [nkeys][m2l_table_width(p)]
    float *m2l_Df = nullptr;
    int32_t n_m2l_keys = 0;
    // target tiles of 16, 8, 4, 2, 1 cells (built on demand; 16 / tpt fields per tile)
    struct Tiles {
        int tpt = 0, max_ent = 0;
        int32_t *tile_tgt = nullptr, *tile_rng = nullptr, *ent_key = nullptr, *ent_src = nullptr;
        int32_t ntiles = 0;
        int64_t nent = 0;
        int64_t bytes = 0;  // device bytes of the four lists
    };
    Tiles m2l_tiles[5];
    // per-level expansion orders (tfmm_plan_set_level_orders): all hp.p
    // unless level_orders; then M2L runs per target level on its own tiles
    LevelOrders lo{};
    bool level_orders = false;
    std::vector<Tiles> lvl_tiles;
    // M2L packed by key in blocks of target cells (FP64 translations of fewer
    // than 16 fields): per field width fpt = 1, 2, 4, 8 (built on
    // demand), and per level when the levels have their own orders; the
    // reduced locals Lr [F][C][lrs] they accumulate into
    struct Packs {
        int nb = 0, tpg = 0, max_grp = 0, p = 0;
        int32_t *blk_cells = nullptr, *item = nullptr, *grp_key = nullptr, *grp_src = nullptr;
        uint8_t *grp_slot = nullptr;
        int32_t nitems = 0;
        int64_t ngrp = 0, npairs = 0;
        int64_t bytes = 0;
    };
    Packs m2l_packs[4];  // fpt = 1, 2, 4, 8
    std::vector<Packs> lvl_packs;
    bool m2l_pack = true;  // schedule knob: the packed form where it applies
    int m2l_max_grp = 256;  // groups per packed work item
    double *Lr = nullptr;
    int32_t lr_cap = 0;
    int m2l_precision = 0;  // TFMM_M2L_*
    // schedule knobs (tfmm_plan_autotune): keys per M2L work item, and four
    // wavefronts per P2P workgroup also for one or two fields
    int m2l_max_ent = 256;
    bool p2p_wide = false;
    // bumped whenever the launch sequence of an evaluation may change
    // (precision, schedule) or a buffer its launches use is reallocated
    // (expansions, scaled multipoles, M2L tiles), so that captured graphs
    // are rebuilt instead of replaying on freed memory
    uint64_t schedule_gen = 0;
    // scaled multipoles Qt_n = (-1)^|n| Q_n / (n! s^|n|): [Fcap][C][qpad] (FP64 or FP32)
    double *Qt = nullptr;
    float *Qtf = nullptr;
    int32_t qt_cap = 0, qtf_cap = 0;
    int32_t qpad = 0;
    // P2P: blocks of <= 64 tets of one source leaf with their target list
    int32_t *p2p_blk = nullptr;  // [nblk][4]: tbeg, tend, ibeg, iend into p2p_idx
    int32_t n_p2p_blk = 0;
    int32_t *p2p_idx = nullptr;  // sorted-target indices
    int64_t n_p2p_idx = 0;
    // shared mesh entities of the P2P blocks (see NearTopo) and the
    // per-evaluation coefficients of one field: faces A [nf][4] (affine in
    // y = x - chunk centroid), edges B [ne][11] (quadratic in y: 1, y0, y1,
    // y2, y0y0, y0y1, y0y2, y1y1, y1y2, y2y2; then the constant g weight)
    int32_t *topo_blk = nullptr, *topo_ch_i = nullptr, *topo_ab = nullptr, *topo_pqr = nullptr, *topo_inc = nullptr;
    double *topo_ch_c = nullptr, *topo_w = nullptr, *topo_il = nullptr, *topo_n = nullptr, *topo_a2 = nullptr;
    double *topo_A = nullptr, *topo_B = nullptr;
    int32_t n_topo_ch = 0;
    int64_t n_topo_edges = 0, n_topo_faces = 0;
    int64_t topo_evals[3] = {0, 0, 0};  // (target, node / edge / face) evaluations per one-field evaluation
    bool p2p_topo = true;  // single-field near field over shared entities
    // stored near-field operator (optional, built by store_near): per cell
    // [C][2] column and value offsets (-1: no block), padded column counts,
    // node columns and the coefficient blocks [nt][3][ncols] of the target
    // leaves; evaluations then apply it instead of integrating the pairs
    int64_t *near_off = nullptr;
    int32_t *near_nc = nullptr, *near_cols = nullptr;
    double *near_val = nullptr;
    int32_t *near_items = nullptr;  // [n][2]: leaf, first row of up to 4 rows (apply work items)
    int32_t near_nitems = 0;
    int64_t near_nvals = 0, near_ncols = 0, near_nnz = 0, near_bytes = 0;
    bool near_stored = false;
    // geometric moments of every tet about its leaf centre: [T][ncoef]
    double *tet_mom = nullptr;
    // quadrature rule for the moments: [nq][4] = lambda1, lambda2, lambda3, weight
    double *quad = nullptr;
    int32_t nq = 0;
    // far-pair rules of the direct sum (degrees 11, 9, 7 concatenated, rows as quad)
    double *far_rule = nullptr;
    // lumped node volumes (sum of V_T / 4 over the tets of a node), built on
    // the first nodal-field request
    double *node_lump = nullptr;
    // expansions [Fcap][C][ncoef]
    double *Q = nullptr, *L = nullptr;
    int32_t Fcap = 0;
    int32_t last_F = 0;

    // near-field surrogate (optional): hidden width, FP32 parameters and their
    // BF16 copy in the inference layout
    int sur_hidden = 0;
    float *sur_w = nullptr;
    uint16_t *sur_wb = nullptr;
    // near-field pairs of the surrogate's band (built on first use): (sorted
    // target index, tet) per pair, target-major within each P2P block; the
    // 27-point rule of the Gauss control; the band's mode in evaluations
    int32_t *band_pairs = nullptr;
    int64_t n_band_pairs = 0;
    bool band_built = false;
    double *band_rule = nullptr;
    int32_t n_band_rule = 0;
    int sur_mode = 0;  // TFMM_SUR_*

    // second stream (default priority) for the near field, forked from and
    // joined back into the evaluation stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    int64_t device_bytes = 0;

    // timing: event pairs recorded on the evaluation stream around each phase,
    // read back (and the device synchronised) only when the times are queried
    bool timing = false;
    struct Span {
        int slot;
        hipEvent_t a, b;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    double kt_ms[KT_COUNT] = {0};
    int64_t kt_n[KT_COUNT] = {0};
};

// Fold recorded spans into kt_ms / kt_n (synchronises on the recorded events).
void collect_timing(DevicePlan &dp);
void reset_timing(DevicePlan &dp);

// Items of a launch of n workgroup items (xcd_grid / xcd_item mapping) in
// the order the workgroups are dispatched.
std::vector<int32_t> xcd_dispatch_items(int n);

// Allocate and upload; hp must be built.  Throws DeviceError.
void upload_plan(DevicePlan &dp);
void free_plan(DevicePlan &dp);
void ensure_expansions(DevicePlan &dp, int32_t F);
// Geometric moments of the tets (after the rule and cells are uploaded).
void build_tet_moments(DevicePlan &dp);
// Fill the M2L derivative tables (after the keys are uploaded).
void build_m2l_table(DevicePlan &dp);
// Tiles of tpt target cells (16, 8, 4, 2 or 1), built and uploaded once.
DevicePlan::Tiles &ensure_m2l_tiles(DevicePlan &dp, int tpt);
// The same per target level (for per-level orders), and their release.
const std::vector<DevicePlan::Tiles> &ensure_m2l_level_tiles(DevicePlan &dp, int tpt);
void free_m2l_packs(DevicePlan &dp);
// merged-batch input and output (see k_batch_gather)
void batch_gather(const double *const *M, const int64_t *off, const double *scale, int n, int64_t N, double *out,
                  hipStream_t st);
void batch_scatter(const double *u, const int64_t *off, int n, int64_t N, double *const *U, hipStream_t st);
void drop_m2l_level_tiles(DevicePlan &dp);

// Allocate everything an evaluation of F fields needs (expansions, M2L tiles
// and operand buffers), so that a later run_evaluate allocates nothing.
void prepare_evaluate(DevicePlan &dp, int32_t F);
// Pick the schedule knobs by timing evaluations on `stream` (synchronises).
void autotune(DevicePlan &dp, hipStream_t stream);
// Queue the FMM evaluation of F fields on `stream`.
void run_evaluate(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t stream);
// Demagnetising field per tet (H [n_tets][3] in input order, may be null) and
// energy E / mu0 of one field M from the nodal potentials u (targets = nodes);
// synchronises the stream.
double run_demag(DevicePlan &dp, const double *M, const double *u, double *H, hipStream_t stream);
// Doubles of the scratch array of the allocation-free entry point (block
// partial sums of the energy: TFMM_NOALLOC_MAX_TETS / 256 + 1).
constexpr int64_t kNoAllocScratchDoubles = 65536;
// run_demag without any allocation: the block partials go to the device's
// scratch array, the energy to energy_dev (device); queued on the stream,
// no synchronisation.  Throws PlanError(TFMM_EINVAL) beyond
// TFMM_NOALLOC_MAX_TETS tets.
void run_demag_noalloc(DevicePlan &dp, const double *M, const double *u, double *H, double *energy_dev,
                       hipStream_t stream);
// Mass-lumped nodal field H [n_nodes][3] (input node order) from nodal u;
// queued on the stream (the first call also builds the lumped volumes).
void run_demag_nodes(DevicePlan &dp, const double *u, double *Hn, hipStream_t stream);
// Assemble the stored near-field operator on `stream` (synchronises); the
// following evaluations apply it.  Throws PlanError(TFMM_ENOMEM) when the
// device memory is not there.
void store_near(DevicePlan &dp, hipStream_t stream);
// Free the stored operator (evaluations integrate the pairs again).
void drop_near(DevicePlan &dp);
// The near field's elementary functions on host arrays (fn 0 log_ratio(a, b),
// 1 atan2_nr(a, b), 2 div_nr(a, b), 3 rsqrt_nr(a)); synchronous, current device.
void run_elementary(int fn, const double *a, const double *b, int64_t n, double *out);
// Queue the O(N^2) direct sum of F fields on `stream`.
void run_direct(DevicePlan &dp, const double *M, int32_t F, double *u, hipStream_t stream);

// Near-field surrogate (pairs at 2 <= |x - c| / diam < 6).
int surrogate_param_count(int hidden);
// Train on pairs drawn from the plan's tets; attaches the result to the plan
// and returns the mean loss of the last 5% of the steps.
double surrogate_train(DevicePlan &dp, int hidden, int steps, int batch, float lr, uint64_t seed,
                       std::vector<float> &params);
void surrogate_set(DevicePlan &dp, int hidden, const std::vector<float> &params);
// Loss and gradient of one batch (host arrays), for checking.
void surrogate_grad(int hidden, const float *params, const float *X, const float *Y, int batch, float *grad,
                    double *loss);
// n training samples (inputs [n][12], targets [n][12]) to host arrays.
void surrogate_samples(DevicePlan &dp, uint64_t seed, int n, float *X, float *Y);
// u = potential of the plan's near-field pairs in the band only (one field),
// exact or by the surrogate.
void run_band(DevicePlan &dp, bool use_surrogate, const double *M, double *u, hipStream_t stream);
// The list of the near-field pairs of the band (once per plan; synchronises).
void build_band_list(DevicePlan &dp, hipStream_t stream);
// Adds the band pairs' potential of F fields into u: mode TFMM_SUR_MLP (the
// network), TFMM_SUR_GAUSS, TFMM_SUR_QUAD, or TFMM_SUR_OFF (exact integral).
void run_band_pairs(DevicePlan &dp, int mode, const double *M, int32_t F, double *u, hipStream_t stream);

// Collapsed Gauss-Jacobi rule on the unit simplex exact to total degree `deg`:
// rows lambda1, lambda2, lambda3, weight (weights sum to 1/6).
std::vector<double> simplex_rule(int deg, int *npts);

}  // namespace tfmm

// C ABI of the tetrahedral FMM library (declared in include/tetfmm.h).
// Every entry point converts failures into a TFMM_E* code plus a thread-local
// message; no exception crosses the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/tetfmm.h"
#include "device.h"
#include "plan.h"

struct tfmm_plan_s {
    tfmm::DevicePlan dp;
    bool on_device = false;
};

// A batch: one plan per mesh and the HIP graph of one evaluation of all of
// them, captured on internal streams for the M and u pointers it was made
// with and replayed while they stay the same.  The meshes are dealt to
// kBatchBranches branches of the graph (longest first by a cost estimate,
// each to the least loaded branch), which the GPU runs concurrently.
constexpr int kBatchBranches = 4;  // concurrent branches of a batch graph

struct tfmm_batch_s {
    std::vector<tfmm_plan> plans;
    // all meshes as one plan (tfmm::merge_host_plans): one launch per phase
    // over every mesh; M is gathered into it scaled by each mesh's root side
    // and u scattered back
    tfmm_plan merged = nullptr;
    bool use_merged = true;
    std::vector<double> scale;
    std::vector<int64_t> off;
    double *mM = nullptr, *mU = nullptr, *d_scale = nullptr;
    int64_t *d_off = nullptr;
    const double **dM = nullptr;
    double **dU = nullptr;
    bool key_merged = false;
    int device = 0;
    hipStream_t capture = nullptr;
    hipStream_t branch[kBatchBranches] = {};
    hipEvent_t fork = nullptr, join[kBatchBranches] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double *> keyM;
    std::vector<double *> keyU;
    std::vector<uint64_t> keyGen;
};

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// Runs f with the plan's device current, restoring the caller's device.
template <class Fn>
int guarded(Fn &&f)
{
    try {
        return f();
    } catch (const tfmm::PlanError &e) {
        return set_error(e.code, e.msg);
    } catch (const tfmm::DeviceError &e) {
        return set_error(TFMM_EDEVICE, e.msg);
    } catch (const std::bad_alloc &) {
        return set_error(TFMM_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_error(TFMM_EINVAL, e.what());
    } catch (...) {
        return set_error(TFMM_EINVAL, "unknown failure");
    }
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        tfmm::hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) tfmm::hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
T *dev_upload(const std::vector<T> &h, int64_t &bytes)
{
    T *d = nullptr;
    size_t n = std::max<size_t>(h.size(), 1);
    tfmm::hip_check(hipMalloc(&d, n * sizeof(T)), "hipMalloc");
    bytes += (int64_t)(n * sizeof(T));
    if (!h.empty()) tfmm::hip_check(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
    return d;
}

}  // namespace

namespace tfmm {

void upload_plan(DevicePlan &dp)
{
    const HostPlan &hp = dp.hp;
    const int64_t T = hp.n_tets, N = hp.n_targets, C = (int64_t)hp.cells.size();
    dp.ncoef = (hp.p + 1) * (hp.p + 2) * (hp.p + 3) / 6;
    int64_t &B = dp.device_bytes;
    B = 0;
    {
        std::vector<double> xyz(12 * T);
        std::vector<int32_t> nd(4 * T);
        for (int64_t s = 0; s < T; ++s)
            for (int c = 0; c < 4; ++c) {
                int32_t n = hp.tet_nodes[4 * s + c];
                nd[c * T + s] = n;
                for (int k = 0; k < 3; ++k) xyz[(3 * c + k) * T + s] = hp.nodes[3 * (int64_t)n + k];
            }
        dp.tet_xyz = dev_upload(xyz, B);
        dp.tet_node = dev_upload(nd, B);
        dp.tet_perm = dev_upload(hp.tet_perm, B);
    }
    {
        std::vector<double> xyz(3 * N);
        std::vector<int32_t> leaf(N, -1);
        for (int64_t s = 0; s < N; ++s)
            for (int k = 0; k < 3; ++k) xyz[k * N + s] = hp.tgt_xyz[3 * s + k];
        for (int64_t c = 0; c < C; ++c) {
            const Cell &K = hp.cells[c];
            if (K.nchild == 0)
                for (int32_t s = K.xbeg; s < K.xend; ++s) leaf[s] = (int32_t)c;
        }
        dp.tgt_xyz = dev_upload(xyz, B);
        dp.tgt_perm = dev_upload(hp.tgt_perm, B);
        dp.tgt_leaf = dev_upload(leaf, B);
    }
    {
        std::vector<double> cc(3 * C);
        std::vector<int32_t> ci(8 * C);
        for (int64_t c = 0; c < C; ++c) {
            const Cell &K = hp.cells[c];
            for (int k = 0; k < 3; ++k) cc[k * C + c] = K.c[k];
            int32_t *o = &ci[8 * c];
            o[0] = K.tbeg;
            o[1] = K.tend;
            o[2] = K.xbeg;
            o[3] = K.xend;
            o[4] = K.cbeg;
            o[5] = K.nchild;
            o[6] = K.parent;
            o[7] = K.level;
        }
        dp.cell_c = dev_upload(cc, B);
        dp.cell_i = dev_upload(ci, B);
    }
    {
        std::vector<int32_t> p2m, m2m, l2l;
        dp.m2m_level_ptr.assign(hp.depth + 2, 0);
        dp.l2l_level_ptr.assign(hp.depth + 2, 0);
        for (int64_t c = 0; c < C; ++c) {
            const Cell &K = hp.cells[c];
            if (K.nchild == 0 && K.tend > K.tbeg) p2m.push_back((int32_t)c);
        }
        for (int Lv = 0; Lv <= hp.depth; ++Lv) {
            dp.m2m_level_ptr[Lv] = (int32_t)m2m.size();
            dp.l2l_level_ptr[Lv] = (int32_t)l2l.size();
            for (int32_t c = hp.level_begin[Lv]; c < hp.level_begin[Lv + 1]; ++c) {
                const Cell &K = hp.cells[c];
                if (K.nchild > 0 && K.tend > K.tbeg) m2m.push_back(c);
                if (Lv > 0 && K.xend > K.xbeg) l2l.push_back(c);
            }
        }
        dp.m2m_level_ptr[hp.depth + 1] = (int32_t)m2m.size();
        dp.l2l_level_ptr[hp.depth + 1] = (int32_t)l2l.size();
        dp.n_p2m_cells = (int32_t)p2m.size();
        dp.p2m_cells = dev_upload(p2m, B);
        dp.m2m_cells = dev_upload(m2m, B);
        dp.l2l_cells = dev_upload(l2l, B);
    }
    {
        // P2P: source leaves with their target-leaf lists, cut into blocks of <= 64 tets
        std::vector<int32_t> cnt(C + 1, 0);
        for (size_t i = 0; i < hp.p2p_b.size(); ++i) cnt[hp.p2p_b[i] + 1]++;
        for (int64_t c = 0; c < C; ++c) cnt[c + 1] += cnt[c];
        std::vector<int32_t> tl(hp.p2p_a.size());
        {
            std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1);
            for (size_t i = 0; i < hp.p2p_b.size(); ++i) tl[fillp[hp.p2p_b[i]]++] = hp.p2p_a[i];
        }
        std::vector<int32_t> blk, idx;
        for (int64_t b = 0; b < C; ++b) {
            if (cnt[b + 1] == cnt[b]) continue;
            const int64_t ib = (int64_t)idx.size();
            for (int32_t j = cnt[b]; j < cnt[b + 1]; ++j) {
                const Cell &A = hp.cells[tl[j]];
                for (int32_t s = A.xbeg; s < A.xend; ++s) idx.push_back(s);
            }
            const int64_t ie = (int64_t)idx.size();
            if (ie > INT32_MAX) throw PlanError{TFMM_ENOTSUP, "near-field target list exceeds 2^31 entries"};
            const Cell &Bc = hp.cells[b];
            for (int32_t t = Bc.tbeg; t < Bc.tend; t += 64) {
                blk.push_back(t);
                blk.push_back(std::min(Bc.tend, t + 64));
                blk.push_back((int32_t)ib);
                blk.push_back((int32_t)ie);
            }
        }
        // shared mesh entities of the source blocks (single-field near field)
        NearTopo tp;
        if (!hp.points) build_near_topology(hp, blk, tp);  // point sources have no mesh entities
        {
            // longest blocks (tets x targets) first in dispatch order, so that the
            // launch ends evenly; the chunk list keeps the same block order
            const int nb = (int)(blk.size() / 4);
            std::vector<int32_t> ord(nb);
            for (int i = 0; i < nb; ++i) ord[i] = i;
            auto work = [&](int i) { return (int64_t)(blk[4 * i + 1] - blk[4 * i]) * (blk[4 * i + 3] - blk[4 * i + 2]); };
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return work(x) > work(y); });
            const std::vector<int32_t> pos = xcd_dispatch_items(nb);
            std::vector<int32_t> b2(blk.size()), t2(tp.blk.size());
            const bool has_topo = !tp.blk.empty();
            for (int k = 0; k < nb; ++k)
                for (int j = 0; j < 4; ++j) {
                    b2[4 * (size_t)pos[k] + j] = blk[4 * (size_t)ord[k] + j];
                    if (has_topo) t2[4 * (size_t)pos[k] + j] = tp.blk[4 * (size_t)ord[k] + j];
                }
            blk.swap(b2);
            tp.blk.swap(t2);
        }
        dp.n_p2p_blk = (int32_t)(blk.size() / 4);
        dp.n_p2p_idx = (int64_t)idx.size();
        dp.p2p_blk = dev_upload(blk, B);
        dp.p2p_idx = dev_upload(idx, B);
        // (target, entity) evaluations of the one-field near field per evaluation
        for (size_t k = 0; k + 3 < tp.blk.size(); k += 4) {
            const int64_t nt = (int64_t)tp.blk[k + 3] - tp.blk[k + 2];
            for (int32_t ch = tp.blk[k]; ch < tp.blk[k + 1]; ++ch) {
                dp.topo_evals[0] += nt * tp.ch_i[8 * (size_t)ch + 3];
                dp.topo_evals[1] += nt * tp.ch_i[8 * (size_t)ch + 5];
                dp.topo_evals[2] += nt * tp.ch_i[8 * (size_t)ch + 7];
            }
        }
        dp.n_topo_ch = (int32_t)(tp.ch_i.size() / 8);
        dp.n_topo_edges = (int64_t)tp.ed_il.size();
        dp.n_topo_faces = (int64_t)(tp.fc_n.size() / 3);
        dp.topo_blk = dev_upload(tp.blk, B);
        dp.topo_ch_i = dev_upload(tp.ch_i, B);
        dp.topo_ch_c = dev_upload(tp.ch_c, B);
        dp.topo_w = dev_upload(tp.nd_w, B);
        dp.topo_ab = dev_upload(tp.ed_ab, B);
        dp.topo_il = dev_upload(tp.ed_il, B);
        dp.topo_pqr = dev_upload(tp.fc_pqr, B);
        dp.topo_n = dev_upload(tp.fc_n, B);
        dp.topo_a2 = dev_upload(tp.fc_a2, B);
        dp.topo_inc = dev_upload(tp.inc, B);
        std::vector<double> zA(4 * (size_t)std::max<int64_t>(dp.n_topo_faces, 1)),
            zB(11 * (size_t)std::max<int64_t>(dp.n_topo_edges, 1));
        dp.topo_A = dev_upload(zA, B);
        dp.topo_B = dev_upload(zB, B);
    }
    {
        dp.n_m2l_keys = (int32_t)(hp.m2l_keys.size() / 4);
        dp.m2l_keys = dev_upload(hp.m2l_keys, B);
        const size_t tb = sizeof(double) * std::max<size_t>(1, (size_t)dp.n_m2l_keys * m2l_table_width(hp.p));
        hip_check(hipMalloc(&dp.m2l_D, tb), "hipMalloc M2L table");
        B += (int64_t)tb;
        build_m2l_table(dp);
        dp.qpad = (m2l_reduced_width(hp.p) + 3) / 4 * 4;
        ensure_m2l_tiles(dp, 16);
    }
    {
        int np = 0;
        std::vector<double> q = simplex_rule(hp.p, &np);
        dp.nq = np;
        dp.quad = dev_upload(q, B);
        std::vector<double> far;
        for (int deg : kFarDeg) {
            int nf = 0;
            std::vector<double> r = simplex_rule(deg, &nf);
            far.insert(far.end(), r.begin(), r.end());
        }
        dp.far_rule = dev_upload(far, B);
        const size_t mb = sizeof(double) * std::max<size_t>(1, (size_t)T * dp.ncoef);
        hip_check(hipMalloc(&dp.tet_mom, mb), "hipMalloc tet moments");
        B += (int64_t)mb;
        build_tet_moments(dp);
    }
}

void free_plan(DevicePlan &dp)
{
    collect_timing(dp);
    if (dp.side) (void)hipStreamSynchronize(dp.side);
    if (dp.ev_fork) (void)hipEventDestroy(dp.ev_fork);
    if (dp.ev_join) (void)hipEventDestroy(dp.ev_join);
    if (dp.side) (void)hipStreamDestroy(dp.side);
    for (hipEvent_t e : dp.event_pool) (void)hipEventDestroy(e);
    dp.event_pool.clear();
    void *ptrs[] = {dp.tet_xyz, dp.tet_node, dp.tet_perm, dp.tgt_xyz, dp.tgt_perm, dp.tgt_leaf, dp.cell_c, dp.cell_i,
                    dp.p2m_cells, dp.m2m_cells, dp.l2l_cells, dp.p2p_blk, dp.p2p_idx, dp.quad, dp.far_rule, dp.node_lump, dp.tet_mom, dp.Q,
                    dp.L, dp.Qt, dp.Qtf, dp.m2l_keys, dp.m2l_D, dp.m2l_Df, dp.sur_w, dp.sur_wb, dp.band_pairs, dp.band_rule, dp.topo_blk,
                    dp.topo_ch_i, dp.topo_ch_c, dp.topo_w, dp.topo_ab, dp.topo_il, dp.topo_pqr, dp.topo_n, dp.topo_a2,
                    dp.topo_inc, dp.topo_A, dp.topo_B, dp.near_off, dp.near_nc, dp.near_cols, dp.near_val, dp.near_items};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &t : dp.m2l_tiles) {
        void *tp[] = {t.tile_tgt, t.tile_rng, t.ent_key, t.ent_src};
        for (void *p : tp)
            if (p) (void)hipFree(p);
    }
    for (auto &t : dp.lvl_tiles) {
        void *tp[] = {t.tile_tgt, t.tile_rng, t.ent_key, t.ent_src};
        for (void *p : tp)
            if (p) (void)hipFree(p);
    }
    tfmm::free_m2l_packs(dp);
    if (dp.Lr) (void)hipFree(dp.Lr);
}

}  // namespace tfmm

extern "C" {

const char *tfmm_last_error(void) { return g_last_error.c_str(); }

static int plan_create(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                       const double *targets, int64_t n_targets, const tfmm_params *prm, tfmm_plan *out, bool points);

int tfmm_plan_create(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                     const double *targets, int64_t n_targets, const tfmm_params *prm, tfmm_plan *out)
{
    return plan_create(nodes, n_nodes, tets, n_tets, targets, n_targets, prm, out, false);
}

int tfmm_plan_create_points(const double *points, int64_t n_points, const double *targets, int64_t n_targets,
                            const tfmm_params *prm, tfmm_plan *out)
{
    return plan_create(points, n_points, nullptr, n_points, targets, n_targets, prm, out, true);
}

static int plan_create(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                       const double *targets, int64_t n_targets, const tfmm_params *prm, tfmm_plan *out, bool points)
{
    if (out) *out = nullptr;
    if (!prm || !out) return set_error(TFMM_EINVAL, "prm and out must not be NULL");
    if (prm->surrogate < TFMM_SUR_OFF || prm->surrogate > TFMM_SUR_QUAD)
        return set_error(TFMM_EINVAL, "surrogate must be one of TFMM_SUR_*");
    if (prm->m2l_precision < TFMM_M2L_FP64 || prm->m2l_precision > TFMM_M2L_BF16X6)
        return set_error(TFMM_ENOTSUP, "unsupported m2l_precision");
    return guarded([&]() -> int {
        auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<tfmm_plan_s> P(new tfmm_plan_s());
        tfmm::build_host_plan(P->dp.hp, nodes, n_nodes, tets, n_tets, targets, n_targets, prm->p, prm->leaf_size,
                              prm->theta, points);
        P->dp.ncoef = (prm->p + 1) * (prm->p + 2) * (prm->p + 3) / 6;
        P->dp.m2l_precision = prm->m2l_precision;
        P->dp.sur_mode = prm->surrogate;
        for (int l = 0; l < tfmm::kMaxLevels; ++l) P->dp.lo.q[l] = (int8_t)prm->p;
        if (prm->device >= 0) {
            int ndev = 0;
            if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
                return set_error(TFMM_EDEVICE, "no HIP device available");
            if (prm->device >= ndev) return set_error(TFMM_EDEVICE, "device ordinal out of range");
            P->dp.device = prm->device;
            DeviceScope ds(prm->device);
            try {
                tfmm::upload_plan(P->dp);
            } catch (...) {
                tfmm::free_plan(P->dp);
                throw;
            }
            P->on_device = true;
        }
        P->dp.hp.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P.release();
        return TFMM_OK;
    });
}

int tfmm_plan_destroy(tfmm_plan plan)
{
    if (!plan) return TFMM_OK;
    return guarded([&]() -> int {
        if (plan->on_device) {
            DeviceScope ds(plan->dp.device);
            tfmm::free_plan(plan->dp);
        }
        delete plan;
        return TFMM_OK;
    });
}

static int check_eval_args(tfmm_plan plan, const double *M, int32_t F, double *u)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan cannot evaluate");
    if (F < 1 || !M || !u) return set_error(TFMM_EINVAL, "F must be >= 1 and M, u non-NULL");
    return TFMM_OK;
}

int tfmm_evaluate(tfmm_plan plan, const double *M, int32_t F, double *u, void *hip_stream)
{
    int rc = check_eval_args(plan, M, F, u);
    if (rc) return rc;
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::run_evaluate(plan->dp, M, F, u, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

int tfmm_direct(tfmm_plan plan, const double *M, int32_t F, double *u, void *hip_stream)
{
    int rc = check_eval_args(plan, M, F, u);
    if (rc) return rc;
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::run_direct(plan->dp, M, F, u, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

static int host_eval(tfmm_plan plan, const double *M, int32_t F, double *u, bool direct)
{
    int rc = check_eval_args(plan, M, F, u);
    if (rc) return rc;
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        const size_t mb = sizeof(double) * (size_t)F * plan->dp.hp.n_nodes * 3;
        const size_t ub = sizeof(double) * (size_t)F * plan->dp.hp.n_targets;
        double *dM = nullptr, *du = nullptr;
        tfmm::hip_check(hipMalloc(&dM, mb), "hipMalloc M");
        if (hipMalloc(&du, ub) != hipSuccess) {
            (void)hipFree(dM);
            throw tfmm::DeviceError{"hipMalloc u failed"};
        }
        try {
            tfmm::hip_check(hipMemcpy(dM, M, mb, hipMemcpyHostToDevice), "hipMemcpy M");
            if (direct)
                tfmm::run_direct(plan->dp, dM, F, du, nullptr);
            else
                tfmm::run_evaluate(plan->dp, dM, F, du, nullptr);
            tfmm::hip_check(hipMemcpy(u, du, ub, hipMemcpyDeviceToHost), "hipMemcpy u");
        } catch (...) {
            (void)hipFree(dM);
            (void)hipFree(du);
            throw;
        }
        (void)hipFree(dM);
        (void)hipFree(du);
        return TFMM_OK;
    });
}

int tfmm_evaluate_host(tfmm_plan plan, const double *M, int32_t F, double *u) { return host_eval(plan, M, F, u, false); }
int tfmm_direct_host(tfmm_plan plan, const double *M, int32_t F, double *u) { return host_eval(plan, M, F, u, true); }

int tfmm_plan_stats(tfmm_plan plan, tfmm_stats *out)
{
    if (!plan || !out) return set_error(TFMM_EINVAL, "NULL argument");
    const tfmm::HostPlan &hp = plan->dp.hp;
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = hp.n_nodes;
    out->n_tets = hp.n_tets;
    out->n_targets = hp.n_targets;
    out->n_cells = (int64_t)hp.cells.size();
    for (const auto &c : hp.cells) out->n_leaves += c.nchild == 0;
    out->depth = hp.depth;
    out->n_m2l = (int64_t)hp.m2l_src.size();
    out->n_p2p = (int64_t)hp.p2p_a.size();
    out->n_p2p_pairs = hp.n_p2p_pairs;
    out->ncoef = plan->dp.ncoef;
    out->device_bytes = plan->dp.device_bytes +
                        (int64_t)(sizeof(double) * (size_t)plan->dp.Fcap * hp.cells.size() *
                                  (2 * (size_t)plan->dp.ncoef + (size_t)plan->dp.qpad));
    out->setup_seconds = hp.setup_seconds;
    out->near_nnz = plan->dp.near_nnz;
    out->near_bytes = plan->dp.near_bytes;
    out->m2l_keys_per_item = plan->dp.m2l_max_ent;
    out->p2p_wide = plan->dp.p2p_wide ? 1 : 0;
    out->p2p_node_evals = plan->dp.topo_evals[0];
    out->p2p_edge_evals = plan->dp.topo_evals[1];
    out->p2p_face_evals = plan->dp.topo_evals[2];
    out->n_band_pairs = plan->dp.n_band_pairs;
    out->surrogate = plan->dp.sur_mode;
    out->surrogate_hidden = plan->dp.sur_hidden;
    for (int l = 0; l < 22; ++l) out->level_order[l] = plan->dp.lo.q[l];
    out->m2l_packed = plan->dp.m2l_pack ? 1 : 0;
    out->m2l_groups_per_item = plan->dp.m2l_max_grp;
    out->m2l_groups = plan->dp.m2l_packs[0].ngrp;
    return TFMM_OK;
}

int64_t tfmm_plan_lists(tfmm_plan plan, int32_t kind, int32_t *out)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (kind < 0 || kind > 3)
        return set_error(TFMM_EINVAL, "kind must be 0 (M2L), 1 (P2P), 2 (M2L tile schedule) or 3 (M2L packed schedule)");
    const tfmm::HostPlan &hp = plan->dp.hp;
    auto put = [&](int64_t k, int32_t a, int32_t b) {
        const tfmm::Cell &A = hp.cells[a], &B = hp.cells[b];
        int32_t *o = out + 8 * k;
        o[0] = A.level;
        o[1] = A.ix;
        o[2] = A.iy;
        o[3] = A.iz;
        o[4] = B.level;
        o[5] = B.ix;
        o[6] = B.iy;
        o[7] = B.iz;
    };
    if (kind == 0) {
        int64_t n = (int64_t)hp.m2l_src.size();
        if (out) {
            int64_t k = 0;
            for (int64_t a = 0; a + 1 < (int64_t)hp.m2l_ptr.size(); ++a)
                for (int32_t j = hp.m2l_ptr[a]; j < hp.m2l_ptr[a + 1]; ++j) put(k++, (int32_t)a, hp.m2l_src[j]);
        }
        return n;
    }
    if (kind == 2) {  // the pairs as the matrix-core tiles of 16 target cells schedule them
        tfmm::M2LTiles t;
        try {
            tfmm::build_m2l_tiles(hp, 16, plan->dp.m2l_max_ent, t);
        } catch (const tfmm::PlanError &e) {
            return set_error(e.code, e.msg);
        }
        int64_t k = 0;
        for (size_t i = 0; 2 * i < t.tile_rng.size(); ++i)
            for (int32_t e = t.tile_rng[2 * i]; e < t.tile_rng[2 * i + 1]; ++e)
                for (int s = 0; s < t.tpt; ++s) {
                    const int32_t a = t.tile_tgt[i * t.tpt + s], b = t.ent_src[(size_t)e * t.tpt + s];
                    if (a < 0 || b < 0) continue;
                    if (out) put(k, a, b);
                    ++k;
                }
        return k;
    }
    if (kind == 3) {  // the pairs as the packed form (one field, the plan's order) schedules them
        tfmm::M2LPacks pk;
        try {
            tfmm::build_m2l_packs(hp, hp.p <= 8 ? 128 : 64, 16, plan->dp.m2l_max_grp, pk);
        } catch (const tfmm::PlanError &e) {
            return set_error(e.code, e.msg);
        }
        int64_t k = 0;
        for (size_t i = 0; 3 * i < pk.item.size(); ++i) {
            const int32_t blk = pk.item[3 * i];
            for (int32_t g = pk.item[3 * i + 1]; g < pk.item[3 * i + 2]; ++g)
                for (int s = 0; s < pk.tpg; ++s) {
                    const int32_t b = pk.grp_src[(size_t)g * pk.tpg + s];
                    if (b < 0) continue;
                    const int32_t a = pk.blk_cells[(size_t)blk * pk.nb + pk.grp_slot[(size_t)g * pk.tpg + s]];
                    if (out) put(k, a, b);
                    ++k;
                }
        }
        return k;
    }
    int64_t n = (int64_t)hp.p2p_a.size();
    if (out)
        for (int64_t k = 0; k < n; ++k) put(k, hp.p2p_a[k], hp.p2p_b[k]);
    return n;
}

int64_t tfmm_plan_cells(tfmm_plan plan, int32_t *cells, double *radii)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    const tfmm::HostPlan &hp = plan->dp.hp;
    const int64_t n = (int64_t)hp.cells.size();
    for (int64_t i = 0; i < n; ++i) {
        const tfmm::Cell &c = hp.cells[i];
        if (cells) {
            int32_t *o = cells + 6 * i;
            o[0] = c.level;
            o[1] = c.ix;
            o[2] = c.iy;
            o[3] = c.iz;
            o[4] = c.tend - c.tbeg;
            o[5] = c.xend - c.xbeg;
        }
        if (radii) {
            radii[2 * i] = c.rsrc;
            radii[2 * i + 1] = c.rtgt;
        }
    }
    return n;
}

int tfmm_plan_expansions(tfmm_plan plan, int32_t which, double *out)
{
    if (!plan || !out) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device || plan->dp.last_F < 1) return set_error(TFMM_EINVAL, "no evaluation on this plan yet");
    if (which != 0 && which != 1) return set_error(TFMM_EINVAL, "which must be 0 (Q) or 1 (L)");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        const size_t per = (size_t)plan->dp.hp.cells.size() * plan->dp.ncoef;
        const double *src = (which == 0 ? plan->dp.Q : plan->dp.L) + per * (size_t)(plan->dp.last_F - 1);
        tfmm::hip_check(hipMemcpy(out, src, per * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy expansions");
        return TFMM_OK;
    });
}

int tfmm_plan_set_level_orders(tfmm_plan plan, const int32_t *orders, int32_t n)
{
    if (!plan || !orders || n < 1) return set_error(TFMM_EINVAL, "NULL plan or orders, or n < 1");
    const int p = plan->dp.hp.p;
    for (int32_t i = 0; i < n; ++i)
        if (orders[i] < 1 || orders[i] > p)
            return set_error(TFMM_EINVAL, "level orders must lie in [1, p] of the plan");
    return guarded([&]() -> int {
        tfmm::DevicePlan &dp = plan->dp;
        bool differ = false;
        for (int l = 0; l < tfmm::kMaxLevels; ++l) {
            dp.lo.q[l] = (int8_t)orders[l < n ? l : n - 1];
            differ = differ || dp.lo.q[l] != p;
        }
        if (plan->on_device) {
            DeviceScope ds(dp.device);
            if (!differ) {
                tfmm::drop_m2l_level_tiles(dp);
                tfmm::free_m2l_packs(dp);
            }
        }
        dp.level_orders = differ;
        ++dp.schedule_gen;
        return TFMM_OK;
    });
}

int tfmm_plan_set_surrogate(tfmm_plan plan, int32_t mode)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (mode < TFMM_SUR_OFF || mode > TFMM_SUR_QUAD) return set_error(TFMM_EINVAL, "mode must be one of TFMM_SUR_*");
    plan->dp.sur_mode = mode;
    ++plan->dp.schedule_gen;
    return TFMM_OK;
}

int tfmm_plan_set_m2l_precision(tfmm_plan plan, int32_t m2l_precision)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (m2l_precision < TFMM_M2L_FP64 || m2l_precision > TFMM_M2L_BF16X6)
        return set_error(TFMM_ENOTSUP, "unsupported m2l_precision");
    plan->dp.m2l_precision = m2l_precision;
    ++plan->dp.schedule_gen;
    return TFMM_OK;
}

int tfmm_simplex_rule(int32_t degree, double *out, int32_t *npts)
{
    if (!npts || degree < 0 || degree > 2 * TFMM_PMAX) return set_error(TFMM_EINVAL, "bad degree");
    return guarded([&]() -> int {
        int n = 0;
        std::vector<double> r = tfmm::simplex_rule(degree, &n);
        if (out) std::memcpy(out, r.data(), r.size() * sizeof(double));
        *npts = n;
        return TFMM_OK;
    });
}

int tfmm_set_timing(tfmm_plan plan, int32_t on)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    return guarded([&]() -> int {
        if (plan->on_device) {
            DeviceScope ds(plan->dp.device);
            tfmm::collect_timing(plan->dp);
        }
        tfmm::reset_timing(plan->dp);
        plan->dp.timing = on != 0;
        return TFMM_OK;
    });
}

int tfmm_kernel_times(tfmm_plan plan, double *ms, int64_t *launches)
{
    if (!plan || !ms || !launches) return set_error(TFMM_EINVAL, "NULL argument");
    if (plan->on_device) {
        int rc = guarded([&]() -> int {
            DeviceScope ds(plan->dp.device);
            tfmm::collect_timing(plan->dp);
            return TFMM_OK;
        });
        if (rc) return rc;
    }
    for (int i = 0; i < tfmm::KT_COUNT; ++i) {
        ms[i] = plan->dp.kt_n[i] ? plan->dp.kt_ms[i] / (double)plan->dp.kt_n[i] : 0.0;
        launches[i] = plan->dp.kt_n[i];
    }
    return TFMM_OK;
}

int tfmm_plan_autotune(tfmm_plan plan, void *hip_stream)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan cannot be tuned");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::autotune(plan->dp, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

int tfmm_demag_energy_noalloc(tfmm_plan plan, const double *M, const double *u, double *H_tet, double *energy,
                              void *hip_stream)
{
    if (!plan || !M || !u || !energy) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    if (!plan->dp.hp.targets_are_nodes) return set_error(TFMM_EINVAL, "the plan's targets are not its nodes");
    if (plan->dp.hp.n_tets > (int64_t)TFMM_NOALLOC_MAX_TETS)
        return set_error(TFMM_EINVAL, "more than TFMM_NOALLOC_MAX_TETS tets");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::run_demag_noalloc(plan->dp, M, u, H_tet, energy, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

int tfmm_demag_field_nodes(tfmm_plan plan, const double *u, double *H_node, void *hip_stream)
{
    if (!plan || !u || !H_node) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    if (!plan->dp.hp.targets_are_nodes) return set_error(TFMM_EINVAL, "the plan's targets are not its nodes");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::run_demag_nodes(plan->dp, u, H_node, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

int tfmm_elementary(int32_t fn, const double *a, const double *b, double *out, int64_t n, int32_t device)
{
    if (fn < 0 || fn > 3 || n < 0 || (n > 0 && (!a || !b || !out)) || device < 0)
        return set_error(TFMM_EINVAL, "fn in 0..3, n >= 0, non-NULL arrays and a device required");
    if (n == 0) return TFMM_OK;
    return guarded([&]() -> int {
        DeviceScope ds(device);
        tfmm::run_elementary(fn, a, b, n, out);
        return TFMM_OK;
    });
}

int tfmm_plan_set_schedule(tfmm_plan plan, int32_t m2l_keys_per_item, int32_t p2p_wide, int32_t m2l_packed,
                           int32_t m2l_groups_per_item)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (m2l_keys_per_item < 16 || m2l_keys_per_item > 4096 || (p2p_wide != 0 && p2p_wide != 1) ||
        (m2l_packed != 0 && m2l_packed != 1) || m2l_groups_per_item < 16 || m2l_groups_per_item > 4096)
        return set_error(TFMM_EINVAL, "m2l_keys_per_item and m2l_groups_per_item must be in [16, 4096], "
                                      "p2p_wide and m2l_packed 0 or 1");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        plan->dp.m2l_max_ent = m2l_keys_per_item;
        plan->dp.p2p_wide = p2p_wide != 0;
        plan->dp.m2l_pack = m2l_packed != 0;
        plan->dp.m2l_max_grp = m2l_groups_per_item;
        ++plan->dp.schedule_gen;
        tfmm::prepare_evaluate(plan->dp, 1);  // the tiles of the new work item size
        return TFMM_OK;
    });
}

int tfmm_plan_store_near(tfmm_plan plan, int32_t on, void *hip_stream)
{
    if (!plan) return set_error(TFMM_EINVAL, "NULL plan");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan has no near-field operator");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        if (on)
            tfmm::store_near(plan->dp, (hipStream_t)hip_stream);
        else
            tfmm::drop_near(plan->dp);
        return TFMM_OK;
    });
}

// Seeded choice of k distinct indices of [0, n) (partial Fisher-Yates driven
// by SplitMix64), sorted.
static std::vector<int64_t> tune_sample(int64_t n, int64_t k, uint64_t seed)
{
    std::vector<int64_t> idx((size_t)n);
    for (int64_t i = 0; i < n; ++i) idx[(size_t)i] = i;
    uint64_t x = seed;
    auto next = [&]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int64_t i = 0; i < k; ++i) {
        const int64_t j = i + (int64_t)(next() % (uint64_t)(n - i));
        std::swap(idx[(size_t)i], idx[(size_t)j]);
    }
    idx.resize((size_t)k);
    std::sort(idx.begin(), idx.end());
    return idx;
}

int tfmm_tune_level_orders(tfmm_plan plan, const double *M, double tol, int32_t n_sample, uint64_t seed,
                           int32_t *orders, double *err_out, double *ms_out)
{
    if (!plan || !M || !orders || !err_out || !ms_out) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points || !plan->dp.hp.targets_are_nodes)
        return set_error(TFMM_EINVAL, "the plan's sources must be tets and its targets its nodes");
    if (!(tol > 0.0) || n_sample < 1) return set_error(TFMM_EINVAL, "tol > 0 and n_sample >= 1 required");
    tfmm::DevicePlan &dp = plan->dp;
    const tfmm::HostPlan &hp = dp.hp;
    const int64_t n_nodes = hp.n_nodes;
    const int p = hp.p, depth = (int)hp.depth;
    const int64_t ns = std::min<int64_t>(n_sample, n_nodes);
    const std::vector<int64_t> sample = tune_sample(n_nodes, ns, seed);
    std::vector<double> xs(3 * (size_t)ns);
    for (int64_t i = 0; i < ns; ++i)
        for (int k = 0; k < 3; ++k) xs[3 * (size_t)i + k] = hp.nodes[3 * sample[(size_t)i] + k];
    const tfmm::LevelOrders lo0 = dp.lo;
    const bool lv0 = dp.level_orders;
    double *dM = nullptr, *du = nullptr, *dref = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    tfmm_plan ref = nullptr;
    auto cleanup = [&]() {
        if (ref) tfmm_plan_destroy(ref);
        if (st) (void)hipStreamSynchronize(st);
        if (dM) (void)hipFree(dM);
        if (du) (void)hipFree(du);
        if (dref) (void)hipFree(dref);
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        if (st) (void)hipStreamDestroy(st);
    };
    int rc = guarded([&]() -> int {
        DeviceScope ds(dp.device);
        tfmm::hip_check(hipStreamCreate(&st), "hipStreamCreate");
        tfmm::hip_check(hipEventCreate(&ea), "hipEventCreate");
        tfmm::hip_check(hipEventCreate(&eb), "hipEventCreate");
        tfmm::hip_check(hipMalloc(&dM, sizeof(double) * 3 * (size_t)n_nodes), "hipMalloc M");
        tfmm::hip_check(hipMalloc(&du, sizeof(double) * (size_t)n_nodes), "hipMalloc u");
        tfmm::hip_check(hipMalloc(&dref, sizeof(double) * (size_t)ns), "hipMalloc reference");
        tfmm::hip_check(hipMemcpy(dM, M, sizeof(double) * 3 * (size_t)n_nodes, hipMemcpyHostToDevice), "hipMemcpy M");
        // reference: the FP64 direct sum at the sampled nodes
        const tfmm_params rp{2, 64, 0.5, TFMM_M2L_FP64, TFMM_SUR_OFF, dp.device};
        int r = tfmm_plan_create(hp.nodes.data(), n_nodes, hp.tet_nodes.data(), hp.n_tets, xs.data(), ns, &rp, &ref);
        if (r) return r;
        if ((r = tfmm_direct(ref, dM, 1, dref, st))) return r;
        std::vector<double> uref((size_t)ns), u((size_t)n_nodes);
        tfmm::hip_check(hipMemcpyAsync(uref.data(), dref, sizeof(double) * (size_t)ns, hipMemcpyDeviceToHost, st),
                        "hipMemcpy reference");
        tfmm::hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        double nref = 0.0;
        for (double v : uref) nref += v * v;
        nref = std::sqrt(nref);
        // candidate profiles: uniform p, then two orders split at a level (the
        // finest levels lowered, or the coarsest), lower order p - 1 or p - 2
        std::vector<std::vector<int32_t>> cand;
        cand.push_back(std::vector<int32_t>((size_t)depth + 1, p));
        for (int q = p - 1; q >= std::max(1, p - 2); --q)
            for (int s = depth; s >= 1; --s) {
                std::vector<int32_t> fine((size_t)depth + 1, p), coarse((size_t)depth + 1, q);
                for (int l = s; l <= depth; ++l) fine[(size_t)l] = q;
                for (int l = s; l <= depth; ++l) coarse[(size_t)l] = p;
                cand.push_back(fine);
                cand.push_back(coarse);
            }
        double best_ms = -1.0, best_err = -1.0;
        std::vector<int32_t> best;
        for (const auto &o : cand) {
            if ((r = tfmm_plan_set_level_orders(plan, o.data(), (int32_t)o.size()))) return r;
            if ((r = tfmm_evaluate(plan, dM, 1, du, st))) return r;
            tfmm::hip_check(hipMemcpyAsync(u.data(), du, sizeof(double) * (size_t)n_nodes, hipMemcpyDeviceToHost, st),
                            "hipMemcpy u");
            tfmm::hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            double e2 = 0.0;
            for (int64_t i = 0; i < ns; ++i) {
                const double d = u[(size_t)sample[(size_t)i]] - uref[(size_t)i];
                e2 += d * d;
            }
            const double err = nref > 0.0 ? std::sqrt(e2) / nref : std::sqrt(e2);
            if (err > 0.5 * tol) continue;  // a margin for the sampling, as tfmm_tune_accuracy
            float ms = -1.f;
            for (int rep = 0; rep < 3; ++rep) {
                tfmm::hip_check(hipEventRecord(ea, st), "hipEventRecord");
                if ((r = tfmm_evaluate(plan, dM, 1, du, st))) return r;
                tfmm::hip_check(hipEventRecord(eb, st), "hipEventRecord");
                tfmm::hip_check(hipEventSynchronize(eb), "hipEventSynchronize");
                float t = 0.f;
                tfmm::hip_check(hipEventElapsedTime(&t, ea, eb), "hipEventElapsedTime");
                if (ms < 0.f || t < ms) ms = t;
            }
            if (best_ms < 0.0 || ms < best_ms) {
                best_ms = ms;
                best_err = err;
                best = o;
            }
        }
        if (best.empty()) {  // nothing met the tolerance: keep the plan's own orders
            dp.lo = lo0;
            dp.level_orders = lv0;
            ++dp.schedule_gen;
            for (int l = 0; l < 22; ++l) orders[l] = dp.lo.q[l];
            *err_out = -1.0;
            *ms_out = -1.0;
            return TFMM_OK;
        }
        if ((r = tfmm_plan_set_level_orders(plan, best.data(), (int32_t)best.size()))) return r;
        for (int l = 0; l < 22; ++l) orders[l] = dp.lo.q[l];
        *err_out = best_err;
        *ms_out = best_ms;
        return TFMM_OK;
    });
    cleanup();
    return rc;
}

// The (p, theta) search of tfmm_tune_accuracy for tets (tets != NULL) or for
// point dipoles at the nodes (tets == NULL).
static int tune_accuracy(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                         const tfmm_params *base, const double *M, double tol, int32_t n_sample, uint64_t seed,
                         const int32_t *p_list, int32_t n_p, const double *theta_list, int32_t n_theta,
                         tfmm_tune_result *out, double *table)
{
    if (!nodes || !base || !M || !out || !p_list || !theta_list) return set_error(TFMM_EINVAL, "NULL argument");
    const bool points = tets == nullptr;
    auto create = [&](const double *tg, int64_t ntg, const tfmm_params *prm, tfmm_plan *pl) {
        return points ? tfmm_plan_create_points(nodes, n_nodes, tg, ntg, prm, pl)
                      : tfmm_plan_create(nodes, n_nodes, tets, n_tets, tg, ntg, prm, pl);
    };
    if (!(tol > 0.0) || n_sample < 1 || n_p < 1 || n_theta < 1 || n_nodes < 1)
        return set_error(TFMM_EINVAL, "tol > 0, n_sample >= 1 and non-empty candidate lists required");
    if (base->device < 0) return set_error(TFMM_EINVAL, "tuning needs a device");
    for (int32_t i = 0; i < n_p; ++i)
        if (p_list[i] < 1 || p_list[i] > TFMM_PMAX) return set_error(TFMM_EINVAL, "p out of range");
    for (int32_t i = 0; i < n_theta; ++i)
        if (!(theta_list[i] > 0.0 && theta_list[i] < 1.0)) return set_error(TFMM_EINVAL, "theta out of (0, 1)");
    std::memset(out, 0, sizeof(*out));
    if (table)
        for (int64_t i = 0; i < (int64_t)n_p * n_theta; ++i) {
            table[4 * i] = p_list[i / n_theta];
            table[4 * i + 1] = theta_list[i % n_theta];
            table[4 * i + 2] = table[4 * i + 3] = -1.0;
        }
    const int64_t ns = std::min<int64_t>(n_sample, n_nodes);
    const std::vector<int64_t> sample = tune_sample(n_nodes, ns, seed);
    std::vector<double> xs(3 * (size_t)ns);
    for (int64_t i = 0; i < ns; ++i)
        for (int k = 0; k < 3; ++k) xs[3 * (size_t)i + k] = nodes[3 * sample[(size_t)i] + k];
    double *dM = nullptr, *du = nullptr, *dref = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    tfmm_plan ref = nullptr, cand = nullptr;
    auto cleanup = [&]() {
        if (cand) tfmm_plan_destroy(cand);
        if (ref) tfmm_plan_destroy(ref);
        if (st) (void)hipStreamSynchronize(st);
        if (dM) (void)hipFree(dM);
        if (du) (void)hipFree(du);
        if (dref) (void)hipFree(dref);
        if (ea) (void)hipEventDestroy(ea);
        if (eb) (void)hipEventDestroy(eb);
        if (st) (void)hipStreamDestroy(st);
    };
    int rc = guarded([&]() -> int {
        DeviceScope ds(base->device);
        tfmm::hip_check(hipStreamCreate(&st), "hipStreamCreate");
        tfmm::hip_check(hipEventCreate(&ea), "hipEventCreate");
        tfmm::hip_check(hipEventCreate(&eb), "hipEventCreate");
        tfmm::hip_check(hipMalloc(&dM, sizeof(double) * 3 * (size_t)n_nodes), "hipMalloc M");
        tfmm::hip_check(hipMalloc(&du, sizeof(double) * (size_t)n_nodes), "hipMalloc u");
        tfmm::hip_check(hipMalloc(&dref, sizeof(double) * (size_t)ns), "hipMalloc reference");
        tfmm::hip_check(hipMemcpy(dM, M, sizeof(double) * 3 * (size_t)n_nodes, hipMemcpyHostToDevice), "hipMemcpy M");
        // reference: FP64 direct sum at the sampled nodes
        tfmm_params rp = *base;
        rp.surrogate = TFMM_SUR_OFF;
        rp.p = 2;
        rp.theta = 0.5;
        int r = create(xs.data(), ns, &rp, &ref);
        if (r) return r;
        if ((r = tfmm_direct(ref, dM, 1, dref, st))) return r;
        std::vector<double> uref((size_t)ns), u((size_t)n_nodes);
        tfmm::hip_check(hipMemcpyAsync(uref.data(), dref, sizeof(double) * (size_t)ns, hipMemcpyDeviceToHost, st),
                        "hipMemcpy reference");
        tfmm::hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        tfmm_plan_destroy(ref);
        ref = nullptr;
        double nref = 0.0;
        for (double v : uref) nref += v * v;
        nref = std::sqrt(nref);
        bool any = false;
        double best_err = -1.0;
        // p ascending; per p the largest theta first (the cheapest); the first
        // theta whose sampled error is within half the tolerance is timed and
        // the smaller thetas of that p (more work) are skipped
        for (int32_t ip = 0; ip < n_p; ++ip) {
            std::vector<int32_t> order((size_t)n_theta);
            for (int32_t i = 0; i < n_theta; ++i) order[(size_t)i] = i;
            std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return theta_list[a] > theta_list[b]; });
            for (int32_t it : order) {
                tfmm_params cp = *base;
                cp.surrogate = TFMM_SUR_OFF;  // the search is over the exact method's knobs
                cp.p = p_list[ip];
                cp.theta = theta_list[it];
                if ((r = create(nullptr, 0, &cp, &cand))) return r;
                if ((r = tfmm_evaluate(cand, dM, 1, du, st))) return r;
                tfmm::hip_check(hipMemcpyAsync(u.data(), du, sizeof(double) * (size_t)n_nodes, hipMemcpyDeviceToHost, st),
                                "hipMemcpy u");
                tfmm::hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                double e2 = 0.0;
                for (int64_t i = 0; i < ns; ++i) {
                    const double d = u[(size_t)sample[(size_t)i]] - uref[(size_t)i];
                    e2 += d * d;
                }
                const double err = nref > 0.0 ? std::sqrt(e2) / nref : std::sqrt(e2);
                ++out->n_tried;
                double *row = table ? table + 4 * ((int64_t)ip * n_theta + it) : nullptr;
                if (row) row[2] = err;
                const bool ok = err <= 0.5 * tol;
                if (ok) {
                    float best_ms = -1.f;
                    for (int rep = 0; rep < 3; ++rep) {
                        tfmm::hip_check(hipEventRecord(ea, st), "hipEventRecord");
                        if ((r = tfmm_evaluate(cand, dM, 1, du, st))) return r;
                        tfmm::hip_check(hipEventRecord(eb, st), "hipEventRecord");
                        tfmm::hip_check(hipEventSynchronize(eb), "hipEventSynchronize");
                        float ms = 0.f;
                        tfmm::hip_check(hipEventElapsedTime(&ms, ea, eb), "hipEventElapsedTime");
                        if (best_ms < 0.f || ms < best_ms) best_ms = ms;
                    }
                    if (row) row[3] = best_ms;
                    if (!any || best_ms < out->ms) {
                        out->p = cp.p;
                        out->theta = cp.theta;
                        out->err = err;
                        out->ms = best_ms;
                    }
                    any = true;
                } else if (!any && (best_err < 0.0 || err < best_err)) {
                    // the most accurate candidate so far stands in until one meets the tolerance
                    best_err = err;
                    out->p = cp.p;
                    out->theta = cp.theta;
                    out->err = err;
                    out->ms = -1.0;
                }
                tfmm_plan_destroy(cand);
                cand = nullptr;
                if (ok) break;
            }
        }
        out->met = any ? 1 : 0;
        return TFMM_OK;
    });
    cleanup();
    return rc;
}

int tfmm_tune_accuracy(const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                       const tfmm_params *base, const double *M, double tol, int32_t n_sample, uint64_t seed,
                       const int32_t *p_list, int32_t n_p, const double *theta_list, int32_t n_theta,
                       tfmm_tune_result *out, double *table)
{
    if (!tets) return set_error(TFMM_EINVAL, "NULL argument");
    return tune_accuracy(nodes, n_nodes, tets, n_tets, base, M, tol, n_sample, seed, p_list, n_p, theta_list, n_theta,
                         out, table);
}

int tfmm_tune_accuracy_points(const double *points, int64_t n_points, const tfmm_params *base, const double *M,
                              double tol, int32_t n_sample, uint64_t seed, const int32_t *p_list, int32_t n_p,
                              const double *theta_list, int32_t n_theta, tfmm_tune_result *out, double *table)
{
    return tune_accuracy(points, n_points, nullptr, n_points, base, M, tol, n_sample, seed, p_list, n_p, theta_list,
                         n_theta, out, table);
}

static void batch_drop_graph(tfmm_batch b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->keyM.clear();
    b->keyU.clear();
    b->keyGen.clear();
    b->key_merged = false;
}

int tfmm_batch_destroy(tfmm_batch batch)
{
    if (!batch) return TFMM_OK;
    return guarded([&]() -> int {
        {
            DeviceScope ds(batch->device);
            batch_drop_graph(batch);
            if (batch->capture) (void)hipStreamDestroy(batch->capture);
            for (int k = 0; k < kBatchBranches; ++k) {
                if (batch->branch[k]) (void)hipStreamDestroy(batch->branch[k]);
                if (batch->join[k]) (void)hipEventDestroy(batch->join[k]);
            }
            if (batch->fork) (void)hipEventDestroy(batch->fork);
            void *bufs[] = {batch->mM, batch->mU, batch->d_scale, batch->d_off, batch->dM, batch->dU};
            for (void *q : bufs)
                if (q) (void)hipFree(q);
        }
        int rc = TFMM_OK;
        if (batch->merged) rc = tfmm_plan_destroy(batch->merged);
        for (tfmm_plan p : batch->plans) {
            const int r = tfmm_plan_destroy(p);
            if (r && !rc) rc = r;
        }
        delete batch;
        return rc;
    });
}

int tfmm_batch_create(int32_t n_meshes, const double *const *nodes, const int64_t *n_nodes, const int32_t *const *tets,
                      const int64_t *n_tets, const tfmm_params *prm, tfmm_batch *out)
{
    if (out) *out = nullptr;
    if (!out || !prm || n_meshes < 1 || !nodes || !n_nodes || !tets || !n_tets)
        return set_error(TFMM_EINVAL, "n_meshes >= 1 and non-NULL arrays required");
    if (prm->device < 0) return set_error(TFMM_EINVAL, "a batch needs a device");
    tfmm_batch b = nullptr;
    int rc = guarded([&]() -> int {
        b = new tfmm_batch_s();
        b->device = prm->device;
        return TFMM_OK;
    });
    if (rc) return rc;
    for (int32_t i = 0; i < n_meshes; ++i) {
        tfmm_plan p = nullptr;
        rc = tfmm_plan_create(nodes[i], n_nodes[i], tets[i], n_tets[i], nullptr, 0, prm, &p);
        if (rc) {
            const std::string msg = "mesh " + std::to_string(i) + ": " + g_last_error;
            (void)tfmm_batch_destroy(b);
            return set_error(rc, msg);
        }
        b->plans.push_back(p);
    }
    rc = guarded([&]() -> int {
        DeviceScope ds(b->device);
        tfmm::hip_check(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "hipStreamCreate");
        tfmm::hip_check(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "hipEventCreate");
        for (int k = 0; k < kBatchBranches; ++k) {
            tfmm::hip_check(hipStreamCreateWithFlags(&b->branch[k], hipStreamNonBlocking), "hipStreamCreate");
            tfmm::hip_check(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming), "hipEventCreate");
        }
        // the merged plan over all meshes
        std::vector<const tfmm::HostPlan *> hps;
        for (tfmm_plan p : b->plans) hps.push_back(&p->dp.hp);
        std::unique_ptr<tfmm_plan_s> P(new tfmm_plan_s());
        tfmm::merge_host_plans(hps, P->dp.hp, b->scale, b->off);
        P->dp.ncoef = (prm->p + 1) * (prm->p + 2) * (prm->p + 3) / 6;
        P->dp.m2l_precision = prm->m2l_precision;
        P->dp.sur_mode = TFMM_SUR_OFF;
        for (int l = 0; l < tfmm::kMaxLevels; ++l) P->dp.lo.q[l] = (int8_t)prm->p;
        P->dp.device = b->device;
        try {
            tfmm::upload_plan(P->dp);
        } catch (...) {
            tfmm::free_plan(P->dp);
            throw;
        }
        P->on_device = true;
        b->merged = P.release();
        const size_t n = b->plans.size();
        const int64_t N = b->off[n];
        tfmm::hip_check(hipMalloc(&b->mM, sizeof(double) * 3 * (size_t)std::max<int64_t>(N, 1)), "hipMalloc batch M");
        tfmm::hip_check(hipMalloc(&b->mU, sizeof(double) * (size_t)std::max<int64_t>(N, 1)), "hipMalloc batch u");
        tfmm::hip_check(hipMalloc(&b->d_scale, sizeof(double) * n), "hipMalloc batch scale");
        tfmm::hip_check(hipMalloc(&b->d_off, sizeof(int64_t) * (n + 1)), "hipMalloc batch offsets");
        tfmm::hip_check(hipMalloc(&b->dM, sizeof(double *) * n), "hipMalloc batch M pointers");
        tfmm::hip_check(hipMalloc(&b->dU, sizeof(double *) * n), "hipMalloc batch u pointers");
        tfmm::hip_check(hipMemcpy(b->d_scale, b->scale.data(), sizeof(double) * n, hipMemcpyHostToDevice), "hipMemcpy");
        tfmm::hip_check(hipMemcpy(b->d_off, b->off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice), "hipMemcpy");
        return TFMM_OK;
    });
    if (rc) {
        (void)tfmm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return TFMM_OK;
}

int tfmm_batch_evaluate(tfmm_batch batch, const double *const *M, double *const *u, void *hip_stream)
{
    if (!batch || !M || !u) return set_error(TFMM_EINVAL, "NULL argument");
    const size_t n = batch->plans.size();
    for (size_t i = 0; i < n; ++i)
        if (!M[i] || !u[i]) return set_error(TFMM_EINVAL, "NULL M or u of mesh " + std::to_string(i));
    return guarded([&]() -> int {
        DeviceScope ds(batch->device);
        hipStream_t st = (hipStream_t)hip_stream;
        if (batch->use_merged && batch->merged) {
            tfmm::DevicePlan &dp = batch->merged->dp;
            const int nm = (int)n;
            const int64_t N = batch->off[n];
            auto put_pointers = [&]() {
                tfmm::hip_check(hipMemcpy(batch->dM, M, sizeof(double *) * n, hipMemcpyHostToDevice), "hipMemcpy");
                tfmm::hip_check(hipMemcpy(batch->dU, u, sizeof(double *) * n, hipMemcpyHostToDevice), "hipMemcpy");
            };
            if (dp.timing) {  // per-phase events cannot live in a graph: run eagerly
                batch_drop_graph(batch);
                put_pointers();
                tfmm::batch_gather(batch->dM, batch->d_off, batch->d_scale, nm, N, batch->mM, st);
                tfmm::run_evaluate(dp, batch->mM, 1, batch->mU, st);
                tfmm::batch_scatter(batch->mU, batch->d_off, nm, N, batch->dU, st);
                return TFMM_OK;
            }
            const bool same = batch->exec && batch->key_merged && std::equal(batch->keyM.begin(), batch->keyM.end(), M) &&
                              std::equal(batch->keyU.begin(), batch->keyU.end(), u) && batch->keyGen.size() == 1 &&
                              batch->keyGen[0] == dp.schedule_gen;
            if (!same) {
                batch_drop_graph(batch);
                tfmm::prepare_evaluate(dp, 1);
                put_pointers();
                tfmm::hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
                tfmm::hip_check(hipStreamBeginCapture(batch->capture, hipStreamCaptureModeThreadLocal),
                                "hipStreamBeginCapture");
                try {
                    tfmm::batch_gather(batch->dM, batch->d_off, batch->d_scale, nm, N, batch->mM, batch->capture);
                    tfmm::run_evaluate(dp, batch->mM, 1, batch->mU, batch->capture);
                    tfmm::batch_scatter(batch->mU, batch->d_off, nm, N, batch->dU, batch->capture);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(batch->capture, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                tfmm::hip_check(hipStreamEndCapture(batch->capture, &batch->graph), "hipStreamEndCapture");
                tfmm::hip_check(hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0),
                                "hipGraphInstantiate");
                batch->keyM.assign(M, M + n);
                batch->keyU.assign(u, u + n);
                batch->keyGen.assign(1, dp.schedule_gen);
                batch->key_merged = true;
            }
            tfmm::hip_check(hipGraphLaunch(batch->exec, st), "hipGraphLaunch");
            return TFMM_OK;
        }
        bool timing = false;
        for (tfmm_plan p : batch->plans) timing = timing || p->dp.timing;
        if (timing) {  // per-phase events cannot live in a graph: run eagerly
            for (size_t i = 0; i < n; ++i) tfmm::run_evaluate(batch->plans[i]->dp, M[i], 1, u[i], st);
            return TFMM_OK;
        }
        std::vector<uint64_t> gen(n);
        for (size_t i = 0; i < n; ++i) gen[i] = batch->plans[i]->dp.schedule_gen;
        const bool same = batch->exec && !batch->key_merged && std::equal(batch->keyM.begin(), batch->keyM.end(), M) &&
                          std::equal(batch->keyU.begin(), batch->keyU.end(), u) && gen == batch->keyGen;
        if (!same) {
            batch_drop_graph(batch);
            for (tfmm_plan p : batch->plans) tfmm::prepare_evaluate(p->dp, 1);
            tfmm::hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
            tfmm::hip_check(hipStreamBeginCapture(batch->capture, hipStreamCaptureModeThreadLocal),
                            "hipStreamBeginCapture");
            try {
                // deal the meshes to the branches: longest first, least loaded branch
                std::vector<size_t> ord(n);
                std::vector<double> cost(n);
                for (size_t i = 0; i < n; ++i) {
                    const tfmm::HostPlan &hp = batch->plans[i]->dp.hp;
                    ord[i] = i;
                    cost[i] = (double)hp.n_p2p_pairs + 300.0 * (double)hp.m2l_src.size() + 1e5;
                }
                std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
                double load[kBatchBranches] = {};
                tfmm::hip_check(hipEventRecord(batch->fork, batch->capture), "hipEventRecord");
                for (int k = 0; k < kBatchBranches; ++k)
                    tfmm::hip_check(hipStreamWaitEvent(batch->branch[k], batch->fork, 0), "hipStreamWaitEvent");
                for (size_t i : ord) {
                    const int k = (int)(std::min_element(load, load + kBatchBranches) - load);
                    load[k] += cost[i];
                    tfmm::run_evaluate(batch->plans[i]->dp, M[i], 1, u[i], batch->branch[k]);
                }
                for (int k = 0; k < kBatchBranches; ++k) {
                    tfmm::hip_check(hipEventRecord(batch->join[k], batch->branch[k]), "hipEventRecord");
                    tfmm::hip_check(hipStreamWaitEvent(batch->capture, batch->join[k], 0), "hipStreamWaitEvent");
                }
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(batch->capture, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            tfmm::hip_check(hipStreamEndCapture(batch->capture, &batch->graph), "hipStreamEndCapture");
            tfmm::hip_check(hipGraphInstantiate(&batch->exec, batch->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            batch->keyM.assign(M, M + n);
            batch->keyU.assign(u, u + n);
            // prepare_evaluate above may have reallocated buffers (and bumped
            // the generations); the graph holds the buffers of now
            for (size_t i = 0; i < n; ++i) gen[i] = batch->plans[i]->dp.schedule_gen;
            batch->keyGen = gen;
        }
        tfmm::hip_check(hipGraphLaunch(batch->exec, st), "hipGraphLaunch");
        return TFMM_OK;
    });
}

int tfmm_batch_autotune(tfmm_batch batch, void *hip_stream)
{
    if (!batch) return set_error(TFMM_EINVAL, "NULL batch");
    if (batch->use_merged && batch->merged) return tfmm_plan_autotune(batch->merged, hip_stream);
    for (tfmm_plan p : batch->plans) {
        const int rc = tfmm_plan_autotune(p, hip_stream);
        if (rc) return rc;
    }
    return guarded([&]() -> int {
        DeviceScope ds(batch->device);
        batch_drop_graph(batch);
        return TFMM_OK;
    });
}

int tfmm_batch_plan(tfmm_batch batch, int32_t i, tfmm_plan *out)
{
    if (!batch || !out || i < 0 || (size_t)i >= batch->plans.size()) return set_error(TFMM_EINVAL, "bad batch index");
    *out = batch->plans[i];
    return TFMM_OK;
}

int tfmm_batch_merged_plan(tfmm_batch batch, tfmm_plan *out)
{
    if (!batch || !out) return set_error(TFMM_EINVAL, "NULL argument");
    *out = batch->merged;
    return TFMM_OK;
}

int tfmm_batch_set_merged(tfmm_batch batch, int32_t on)
{
    if (!batch || (on != 0 && on != 1)) return set_error(TFMM_EINVAL, "NULL batch or on not 0/1");
    return guarded([&]() -> int {
        DeviceScope ds(batch->device);
        if (batch->use_merged != (on != 0)) batch_drop_graph(batch);
        batch->use_merged = on != 0;
        return TFMM_OK;
    });
}

int tfmm_demag_energy(tfmm_plan plan, const double *M, const double *u, double *H_tet, double *energy,
                      void *hip_stream)
{
    if (!plan || !M || !u || !energy) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    if (!plan->dp.hp.targets_are_nodes) return set_error(TFMM_EINVAL, "the plan's targets are not its nodes");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        *energy = tfmm::run_demag(plan->dp, M, u, H_tet, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

int tfmm_surrogate_param_count(int32_t hidden) { return tfmm::surrogate_param_count(hidden); }

static int write_surrogate(const char *path, int32_t hidden, const std::vector<float> &params)
{
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_error(TFMM_EINVAL, std::string("cannot write ") + path);
    const char magic[8] = {'T', 'F', 'M', 'M', 'S', 'U', 'R', '1'};
    const int32_t hdr[2] = {hidden, (int32_t)params.size()};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 2, f) == 2 &&
              std::fwrite(params.data(), sizeof(float), params.size(), f) == params.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? TFMM_OK : set_error(TFMM_EINVAL, std::string("write failed: ") + path);
}

int tfmm_surrogate_train(tfmm_plan plan, const tfmm_train_cfg *cfg, const char *out_path, double *final_loss)
{
    if (!plan || !cfg) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    if ((cfg->hidden != 32 && cfg->hidden != 64 && cfg->hidden != 128) || cfg->steps < 1 || cfg->batch < 1 ||
        !(cfg->lr > 0.f))
        return set_error(TFMM_EINVAL, "hidden must be 32, 64 or 128; steps, batch and lr positive");
    std::vector<float> params;
    int rc = guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        const double loss =
            tfmm::surrogate_train(plan->dp, cfg->hidden, cfg->steps, cfg->batch, cfg->lr, cfg->seed, params);
        if (final_loss) *final_loss = loss;
        return TFMM_OK;
    });
    if (rc || !out_path) return rc;
    return write_surrogate(out_path, cfg->hidden, params);
}

int tfmm_surrogate_load(tfmm_plan plan, const char *path)
{
    if (!plan || !path) return set_error(TFMM_EINVAL, "NULL argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_error(TFMM_EINVAL, std::string("cannot read ") + path);
    char magic[8];
    int32_t hdr[2] = {0, 0};
    std::vector<float> params;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TFMMSUR1", 8) == 0 &&
              std::fread(hdr, sizeof(int32_t), 2, f) == 2 && hdr[1] == tfmm::surrogate_param_count(hdr[0]) &&
              hdr[1] > 0;
    if (ok) {
        params.resize((size_t)hdr[1]);
        ok = std::fread(params.data(), sizeof(float), params.size(), f) == params.size();
    }
    std::fclose(f);
    if (!ok) return set_error(TFMM_EINVAL, std::string("not a surrogate file of a supported width: ") + path);
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::surrogate_set(plan->dp, hdr[0], params);
        return TFMM_OK;
    });
}

int tfmm_surrogate_samples(tfmm_plan plan, uint64_t seed, int32_t n, float *X, float *Y)
{
    if (!plan || !X || !Y || n < 1) return set_error(TFMM_EINVAL, "bad argument");
    if (!plan->on_device) return set_error(TFMM_EINVAL, "host-only plan");
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::surrogate_samples(plan->dp, seed, n, X, Y);
        return TFMM_OK;
    });
}

int tfmm_surrogate_grad(int32_t hidden, const float *params, const float *X, const float *Y, int32_t batch,
                        float *grad, double *loss, int32_t device)
{
    if (!params || !X || !Y || !grad || !loss || batch < 1 || tfmm::surrogate_param_count(hidden) <= 0)
        return set_error(TFMM_EINVAL, "bad argument");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_error(TFMM_EDEVICE, "no such HIP device");
    return guarded([&]() -> int {
        DeviceScope ds(device);
        tfmm::surrogate_grad(hidden, params, X, Y, batch, grad, loss);
        return TFMM_OK;
    });
}

int tfmm_band_potential(tfmm_plan plan, int32_t use_surrogate, const double *M, double *u, void *hip_stream)
{
    int rc = check_eval_args(plan, M, 1, u);
    if (rc) return rc;
    if (plan->dp.hp.points) return set_error(TFMM_ENOTSUP, "not available for point-dipole plans");
    if (use_surrogate && !plan->dp.sur_wb) return set_error(TFMM_EINVAL, "no surrogate attached to the plan");
    return guarded([&]() -> int {
        DeviceScope ds(plan->dp.device);
        tfmm::run_band(plan->dp, use_surrogate != 0, M, u, (hipStream_t)hip_stream);
        return TFMM_OK;
    });
}

}  // extern "C"

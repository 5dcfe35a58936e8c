// Batches of independent tensors of any shapes through the whole hot path.
//
// A plan turns the items into per-stage task tables that live in the
// caller's workspace, so every stage is one launch over all tensors:
// transform tiles, Jacobi (slice, block pair) tasks driven by one global round
// counter (each slice follows its own tournament of nb_s - 1 rounds per
// sweep), per-tensor rank selection, per-slice packing, reconstruction tiles,
// back-transform tiles and per-tensor error sums.  Descriptor tables hold
// workspace addresses, so they are rebuilt when the workspace moves.  The
// plan keeps the tables in pinned host memory and copies them into the
// workspace at the start of every run (a copy node of a captured graph), so
// it owns no device memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

using namespace tsvdm;

struct tsvdm_batch_plan_s {
    std::vector<tsvdm_batch_item> items;
    int in_dt = TSVDM_F32, dt = TSVDM_F32, ttm_compute = TSVDM_F32;
    int max_sweeps = 40, max_steps = 0;
    std::vector<int> nb2;  // pair width 2b per item
    // workspace layout (byte offsets)
    std::vector<size_t> off_ahat, off_w, off_s2, off_tf, off_tb, off_keys, off_stats, off_part,
        off_upk, off_gpk, off_spk;
    std::vector<int64_t> cap;  // effective capacity per item
    size_t off_ctl = 0, ws_total = 0;
    int64_t nslices = 0;
    // host tables (addresses filled per workspace); transform tasks are
    // sorted by tile shape and Jacobi tasks by pair width
    std::vector<int4> ttm_tasks, lr_tasks;
    std::vector<int2> jtasks;
    int64_t ttm_group[TTM_SHAPES] = {}, back_group[TTM_SHAPES] = {}, jgroup[2] = {0, 0};
    // slice SVD form per item: FORM_ROT (rotation form), FORM_GRAM_ROUNDS
    // (Gram form, Jacobi on the factor in the block rounds), FORM_GRAM_LDS
    // (Gram form, in-LDS Jacobi).  Slices are numbered by form: rotation
    // [0, n_rot), Gram in rounds [n_rot, n_jac), in LDS [n_jac, nslices);
    // the batched Jacobi covers [0, n_jac), Gram slice gi is slice n_rot + gi
    std::vector<char> form;
    std::vector<int64_t> slice_base;
    int64_t n_rot = 0, n_jac = 0, n_gram = 0, n_lds = 0;
    std::vector<size_t> off_gG, off_gL, off_gsh, off_gfl, off_gperm;
    std::vector<size_t> off_trk;     // Jacobi pair records (nbe^2 int32 per slice)
    std::vector<int2> gtasks;        // (Gram slice, lower-triangle tile)
    std::vector<int4> ftasks;        // (Gram slice, kept-column tile, position tile)
    std::vector<int> glists;         // Gram slices by Cholesky class, then in-LDS slices by class
    int64_t chol_off[GRAM_CHOL_CLASSES] = {}, chol_cnt[GRAM_CHOL_CLASSES] = {};
    int64_t lds_off[GRAM_LDS_CLASSES] = {}, lds_cnt[GRAM_LDS_CLASSES] = {};
    int lds_maxr[GRAM_LDS_CLASSES] = {};
    size_t o_gs = 0, o_gt = 0, o_gl = 0, o_gf = 0;
    // tables: pinned host copy (filled for one workspace address) and their
    // place in the workspace
    char* htab = nullptr;
    size_t tab_bytes = 0, off_tab = 0;
    size_t o_fwd = 0, o_back = 0, o_ttm = 0, o_bt = 0, o_sl = 0, o_jt = 0, o_ps = 0, o_lr = 0,
           o_sel = 0, o_err = 0;
    int64_t n_back = 0, n_back_tasks = 0;
    int n_err = 0;
    void* tables_ws = nullptr;
    // captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    void* graph_ws = nullptr;
    hipStream_t graph_stream = nullptr;
    int32_t* graph_status = nullptr;
};

namespace {

enum { FORM_ROT = 0, FORM_GRAM_ROUNDS = 1, FORM_GRAM_LDS = 2 };

size_t esz(int dt) { return dt == TSVDM_F64 ? 8 : 4; }

int validate_item(const tsvdm_batch_item& it, int idx) {
    const std::string where = "batch item " + std::to_string(idx) + ": ";
    if (!(it.m > 0 && it.p > 0 && it.n > 0 && it.m < (1 << 30) && it.p < (1 << 30) && it.n < 65536)) {
        set_error(where + "m, p, n must be positive (n < 65536)");
        return TSVDM_E_SHAPE;
    }
    if (std::min(it.m, it.p) > 4096) {
        set_error(where + "min(m, p) must be <= 4096");
        return TSVDM_E_SHAPE;
    }
    if (!it.A || !it.M || !it.rho || !it.offsets) {
        set_error(where + "A, M, rho and offsets must be non-NULL");
        return TSVDM_E_ARG;
    }
    if (it.reserved != 0) {
        set_error(where + "reserved must be 0");
        return TSVDM_E_ARG;
    }
    if (!(it.block == 0 || it.block == 16 || it.block == 32)) {
        set_error(where + "block must be 0, 16 or 32");
        return TSVDM_E_ARG;
    }
    if (it.ttm_tile < 0 || it.ttm_tile > TTM_SHAPES) {
        set_error(where + "ttm_tile must be in [0, 8]");
        return TSVDM_E_ARG;
    }
    if (it.mode == 1) {
        if (it.k < 1) { set_error(where + "k must be >= 1"); return TSVDM_E_ARG; }
    } else if (it.mode == 2) {
        if (!(it.eps > 0.0 && it.eps < 1.0)) { set_error(where + "eps must lie in (0, 1)"); return TSVDM_E_ARG; }
    } else {
        set_error(where + "mode must be 1 or 2");
        return TSVDM_E_ARG;
    }
    if (!std::isfinite(it.inv_scale)) { set_error(where + "inv_scale must be finite"); return TSVDM_E_ARG; }
    if (it.U_pk && (!it.G_pk || !it.S_pk || it.capacity < 0)) {
        set_error(where + "U_pk, G_pk, S_pk must be given together with capacity >= 0");
        return TSVDM_E_ARG;
    }
    if (it.err && !it.A_rec) { set_error(where + "err needs A_rec"); return TSVDM_E_ARG; }
    return TSVDM_OK;
}

// Offsets of the tables inside their block; returns the block size.
size_t layout_tables(tsvdm_batch_plan_s* P) {
    size_t off = 0;
    auto place = [&](size_t bytes) { off = align_up(off); size_t o = off; off += bytes; return o; };
    P->o_fwd = place(sizeof(TtmProblem) * P->items.size());
    P->o_back = place(sizeof(TtmProblem) * std::max<size_t>((size_t)P->n_back, 1));
    P->o_ttm = place(sizeof(int4) * P->ttm_tasks.size());
    P->o_bt = place(sizeof(int4) * std::max<size_t>((size_t)P->n_back_tasks, 1));
    P->o_sl = place(sizeof(BatchSlice) * std::max<size_t>((size_t)P->n_jac, 1));
    P->o_jt = place(sizeof(int2) * P->jtasks.size());
    P->o_ps = place(sizeof(PackSlice) * (size_t)P->nslices);
    P->o_lr = place(sizeof(int4) * std::max<size_t>(P->lr_tasks.size(), 1));
    P->o_sel = place(sizeof(SelTensor) * P->items.size());
    P->o_err = place(sizeof(ErrJob) * std::max<size_t>((size_t)P->n_err, 1));
    P->o_gs = place(sizeof(GramSlice) * std::max<size_t>((size_t)P->n_gram, 1));
    P->o_gt = place(sizeof(int2) * std::max<size_t>(P->gtasks.size(), 1));
    P->o_gl = place(sizeof(int) * std::max<size_t>(P->glists.size(), 1));
    P->o_gf = place(sizeof(int4) * std::max<size_t>(P->ftasks.size(), 1));
    return align_up(off);
}

// Fill the host copy of the tables for workspace base `ws`.
int build_tables(tsvdm_batch_plan_s* P, char* ws) {
    const int cnt = (int)P->items.size();
    std::vector<TtmProblem> fwd(cnt), back;
    std::vector<BatchSlice> sl((size_t)P->n_jac);
    std::vector<PackSlice> ps((size_t)P->nslices);
    std::vector<GramSlice> gsl((size_t)P->n_gram);
    std::vector<SelTensor> sel(cnt);
    std::vector<ErrJob> err;
    std::vector<int4> back_by[TTM_SHAPES];
    const size_t e = esz(P->dt);
    const int VW = 16 / (int)e;
    for (int t = 0; t < cnt; ++t) {
        const tsvdm_batch_item& it = P->items[t];
        const SliceGeom g = slice_geom(it.m, it.p);
        char* ahat = ws + P->off_ahat[t];
        char* w = ws + P->off_w[t];
        double* s2 = reinterpret_cast<double*>(ws + P->off_s2[t]);
        fwd[t] = TtmProblem{it.A, ahat, it.M, ws + P->off_tf[t], it.m * it.p, (int)it.n, 0, 1.0};
        void* upk = it.U_pk ? it.U_pk : ws + P->off_upk[t];
        void* gpk = it.U_pk ? it.G_pk : ws + P->off_gpk[t];
        void* spk = it.U_pk ? it.S_pk : ws + P->off_spk[t];
        const int b = P->nb2[t] / 2;
        const int nb = (int)((g.r + b - 1) / b);
        const int nbe = nb + (nb & 1);
        const double ueps = P->dt == TSVDM_F64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
        double tol = 8.0 * std::sqrt((double)std::max<int64_t>(g.L, 1)) * ueps;
        tol = P->dt == TSVDM_F64 ? std::max(tol, 1e-14) : std::max(tol, 2e-6);
        const int form = P->form[t];
        for (int64_t i = 0; i < it.n; ++i) {
            const int64_t slice = P->slice_base[t] + i;
            BatchSlice d;
            d.A = ahat + (size_t)(i * it.m * it.p) * e;
            d.W = w + (size_t)(i * g.r * g.r) * e;
            d.s2 = s2 + i * g.r;
            d.g = g;
            d.nbe = nbe;
            d.vec_a = (g.m % VW == 0) ? 1 : 0;
            d.vec_w = (g.r % VW == 0) ? 1 : 0;
            d.tensor = t;
            d.tol = tol;
            d.track = form == FORM_GRAM_LDS ? nullptr
                      : reinterpret_cast<int32_t*>(ws + P->off_trk[t]) + i * nbe * nbe;
            if (form != FORM_ROT) {
                GramSlice gd;
                gd.A = static_cast<const float*>(d.A);
                gd.B = static_cast<float*>(d.W);
                gd.G = reinterpret_cast<double*>(ws + P->off_gG[t]) + i * g.r * g.r;
                gd.Lw = reinterpret_cast<double*>(ws + P->off_gL[t]) + i * g.r * g.r;
                gd.s2 = d.s2;
                gd.shift = reinterpret_cast<double*>(ws + P->off_gsh[t]) + i;
                gd.flag = reinterpret_cast<int32_t*>(ws + P->off_gfl[t]) + i;
                gd.perm = reinterpret_cast<int32_t*>(ws + P->off_gperm[t]) + i * g.r;
                gd.g = g;
                gd.tol = gram_tol(g.r);
                gsl[(size_t)(slice - P->n_rot)] = gd;
                if (form == FORM_GRAM_ROUNDS) {
                    // the rounds orthogonalise the columns of the r x r
                    // factor, accumulating no rotations
                    BatchSlice f = d;
                    f.A = gd.B;
                    f.W = nullptr;
                    f.g = slice_geom(g.r, g.r);
                    f.vec_a = (g.r % VW == 0) ? 1 : 0;
                    f.vec_w = 0;
                    f.tol = gd.tol;
                    sl[(size_t)slice] = f;
                }
            } else {
                sl[(size_t)slice] = d;
            }
            PackSlice q;
            q.A = d.A;
            q.W = d.W;
            q.s2 = d.s2;
            q.g = g;
            q.rho = it.rho + i;
            q.off = it.offsets + i;
            q.U_pk = upk;
            q.G_pk = gpk;
            q.S_pk = spk;
            q.capacity = P->cap[t];
            q.C = d.A;  // the reconstruction overwrites A-hat, no longer needed
            q.status = nullptr;
            ps[(size_t)slice] = q;
        }
        SelTensor s;
        s.s2 = s2;
        s.rho = it.rho;
        s.offsets = it.offsets;
        s.stats = it.stats ? it.stats : reinterpret_cast<double*>(ws + P->off_stats[t]);
        s.keys = reinterpret_cast<unsigned long long*>(ws + P->off_keys[t]);
        s.r = g.r;
        s.n = it.n;
        s.np2 = select_np2(g.r * it.n);
        s.mode = it.mode;
        s.pad = 0;
        s.k = it.k;
        s.eps = it.eps;
        sel[t] = s;
        if (it.A_rec) {
            TtmProblem bk{ahat, it.A_rec, it.M, ws + P->off_tb[t], it.m * it.p, (int)it.n, 0,
                          it.inv_scale};
            const int bi = (int)back.size();
            back.push_back(bk);
            int64_t n_rt;
            int n_ct;
            const int shp = ttm_resolve_tile(it.ttm_tile, it.n, P->ttm_compute);
            ttm_tile_counts(shp, it.m * it.p, it.n, &n_rt, &n_ct);
            for (int64_t rt = 0; rt < n_rt; ++rt)
                for (int ct = 0; ct < n_ct; ++ct) back_by[shp - 1].push_back(int4{bi, (int)rt, ct, 0});
            if (it.err) {
                ErrJob j;
                j.A = it.A;
                j.B = it.A_rec;
                j.count = it.m * it.p * it.n;
                j.out = it.err;
                j.part = reinterpret_cast<double*>(ws + P->off_part[t]);
                err.push_back(j);
            }
        }
    }
    std::vector<int4> back_tasks;
    for (int q = 0; q < TTM_SHAPES; ++q) {
        P->back_group[q] = (int64_t)back_by[q].size();
        back_tasks.insert(back_tasks.end(), back_by[q].begin(), back_by[q].end());
    }
    if ((int64_t)back.size() != P->n_back || (int64_t)back_tasks.size() != P->n_back_tasks ||
        (int)err.size() != P->n_err || P->n_jac + P->n_gram - (P->n_jac - P->n_rot) != P->nslices) {
        set_error("internal: batch table sizes differ from the plan's layout");
        return TSVDM_E_ARG;
    }
    if (!P->htab) {
        TSVDM_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&P->htab), P->tab_bytes, hipHostMallocDefault));
    } else {
        // a copy of the previous tables may still be in flight
        TSVDM_HIP_CHECK(hipDeviceSynchronize());
    }
    char* host = P->htab;
    memset(host, 0, P->tab_bytes);
    auto put = [&](size_t o, const void* src, size_t bytes) { if (bytes) memcpy(host + o, src, bytes); };
    put(P->o_fwd, fwd.data(), sizeof(TtmProblem) * fwd.size());
    put(P->o_back, back.data(), sizeof(TtmProblem) * back.size());
    put(P->o_ttm, P->ttm_tasks.data(), sizeof(int4) * P->ttm_tasks.size());
    put(P->o_bt, back_tasks.data(), sizeof(int4) * back_tasks.size());
    put(P->o_sl, sl.data(), sizeof(BatchSlice) * sl.size());
    put(P->o_jt, P->jtasks.data(), sizeof(int2) * P->jtasks.size());
    put(P->o_ps, ps.data(), sizeof(PackSlice) * ps.size());
    put(P->o_lr, P->lr_tasks.data(), sizeof(int4) * P->lr_tasks.size());
    put(P->o_sel, sel.data(), sizeof(SelTensor) * sel.size());
    put(P->o_err, err.data(), sizeof(ErrJob) * err.size());
    put(P->o_gs, gsl.data(), sizeof(GramSlice) * gsl.size());
    put(P->o_gt, P->gtasks.data(), sizeof(int2) * P->gtasks.size());
    put(P->o_gl, P->glists.data(), sizeof(int) * P->glists.size());
    put(P->o_gf, P->ftasks.data(), sizeof(int4) * P->ftasks.size());
    P->tables_ws = ws;
    return TSVDM_OK;
}

// The status word of each PackSlice is set per run (it is the caller's).
__global__ void set_pack_status(PackSlice* ps, int64_t n, int32_t* status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ps[i].status = status;
}

__global__ void merge_status(int32_t* status, const int32_t* jacobi_status) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *status == TSVDM_OK) *status = *jacobi_status;
}

// a fill kernel rather than a memset, so that graph replays stay exact
__global__ void clear_status(int32_t* status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = TSVDM_OK;
}

int run_stages(tsvdm_batch_plan_s* P, char* ws, int host_poll, int32_t* status, hipStream_t st) {
    char* D = ws + P->off_tab;
    const int cnt = (int)P->items.size();
    int rc;
    TSVDM_HIP_CHECK(hipMemcpyAsync(D, P->htab, P->tab_bytes, hipMemcpyHostToDevice, st));
    int32_t* jstatus = reinterpret_cast<int32_t*>(ws + P->off_ctl);
    int32_t* gstatus = reinterpret_cast<int32_t*>(ws + P->off_ctl + 64);
    void* ctl_ws = ws + P->off_ctl + 256;
    clear_status<<<1, 64, 0, st>>>(status);
    TSVDM_LAUNCH_CHECK();
    clear_status<<<1, 64, 0, st>>>(jstatus);
    TSVDM_LAUNCH_CHECK();
    // 1. transform
    rc = run_ttm_batch(reinterpret_cast<const TtmProblem*>(D + P->o_fwd), cnt,
                       reinterpret_cast<const int4*>(D + P->o_ttm), P->ttm_group,
                       P->in_dt, P->dt, P->ttm_compute, 0, st);
    if (rc) return rc;
    // 2. slice SVDs: FP64 Gram and Cholesky factor of the Gram-form slices;
    //    the block rounds of the rotation-form slices and of the factors
    //    whose Jacobi runs in the rounds; the in-LDS Jacobi of the others
    const GramSlice* gs = reinterpret_cast<const GramSlice*>(D + P->o_gs);
    const int* glists = reinterpret_cast<const int*>(D + P->o_gl);
    if (P->n_gram > 0) {
        rc = run_gram_prep_batch(gs, P->n_gram, reinterpret_cast<const int2*>(D + P->o_gt),
                                 (int64_t)P->gtasks.size(), glists, P->chol_off, P->chol_cnt, st);
        if (rc) return rc;
    }
    if (P->n_jac > 0) {
        rc = run_jacobi_batch(P->dt, reinterpret_cast<const BatchSlice*>(D + P->o_sl), P->n_jac,
                              reinterpret_cast<const int2*>(D + P->o_jt), P->jgroup, P->max_steps,
                              host_poll, ctl_ws, jstatus, st);
        if (rc) return rc;
        rc = run_gram_unshift_batch(gs, P->n_jac - P->n_rot, st);
        if (rc) return rc;
    }
    if (P->n_lds > 0) {
        rc = run_gram_lds_batch(gs, glists, P->lds_off, P->lds_cnt, P->lds_maxr, P->max_sweeps,
                                gs + (P->n_jac - P->n_rot), P->n_lds, gstatus, st);
        if (rc) return rc;
    }
    // 3. ranks
    rc = run_select_batch(reinterpret_cast<const SelTensor*>(D + P->o_sel), cnt, st);
    if (rc) return rc;
    // 4. factors (the caller's status word collects capacity overflows)
    set_pack_status<<<(unsigned)((P->nslices + 255) / 256), 256, 0, st>>>(
        reinterpret_cast<PackSlice*>(D + P->o_ps), P->nslices, status);
    TSVDM_LAUNCH_CHECK();
    if (P->n_rot > 0) {
        rc = run_pack_batch(P->dt, reinterpret_cast<const PackSlice*>(D + P->o_ps), P->n_rot, st);
        if (rc) return rc;
    }
    if (P->n_gram > 0) {
        rc = run_gram_pack_batch(gs, reinterpret_cast<const PackSlice*>(D + P->o_ps) + P->n_rot, P->n_gram,
                                 reinterpret_cast<const int4*>(D + P->o_gf), (int64_t)P->ftasks.size(), st);
        if (rc) return rc;
    }
    // 5. reconstruction and back-transform
    if (!P->lr_tasks.empty()) {
        rc = run_lowrank_batch(P->dt, reinterpret_cast<const PackSlice*>(D + P->o_ps),
                               reinterpret_cast<const int4*>(D + P->o_lr),
                               (int64_t)P->lr_tasks.size(), st);
        if (rc) return rc;
        int nback = 0;
        for (const auto& it : P->items) nback += it.A_rec ? 1 : 0;
        rc = run_ttm_batch(reinterpret_cast<const TtmProblem*>(D + P->o_back), nback,
                           reinterpret_cast<const int4*>(D + P->o_bt), P->back_group, P->dt,
                           P->dt, P->ttm_compute, 1, st);
        if (rc) return rc;
    }
    // 6. error sums
    if (P->n_err > 0) {
        rc = run_error_batch(P->in_dt, P->dt, reinterpret_cast<const ErrJob*>(D + P->o_err),
                             P->n_err, st);
        if (rc) return rc;
    }
    merge_status<<<1, 64, 0, st>>>(status, jstatus);
    TSVDM_LAUNCH_CHECK();
    if (P->n_lds > 0) {
        merge_status<<<1, 64, 0, st>>>(status, gstatus);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

}  // namespace

extern "C" {

int tsvdm_batch_plan_create(const tsvdm_batch_item* items, int32_t count, int in_dtype, int dtype,
                            int ttm_compute, int block, int max_sweeps, tsvdm_batch_plan* plan,
                            size_t* ws_bytes) {
    clear_error();
    TSVDM_REQUIRE(items && plan && ws_bytes, TSVDM_E_ARG, "items, plan and ws_bytes must be non-NULL");
    TSVDM_REQUIRE(count >= 1 && count < 65536, TSVDM_E_SHAPE, "count must be in [1, 65535]");
    TSVDM_REQUIRE(in_dtype == TSVDM_F64 || in_dtype == TSVDM_F32, TSVDM_E_UNSUPPORTED, "in_dtype must be F64 or F32");
    TSVDM_REQUIRE(dtype == TSVDM_F64 || dtype == TSVDM_F32, TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    TSVDM_REQUIRE(ttm_compute >= TSVDM_F64 && ttm_compute <= TSVDM_BF16X3, TSVDM_E_UNSUPPORTED, "unknown ttm_compute");
    TSVDM_REQUIRE(!(ttm_compute >= TSVDM_BF16 && dtype != TSVDM_F32), TSVDM_E_UNSUPPORTED,
                  "BF16 transforms need dtype F32");
    TSVDM_REQUIRE(block == 0 || block == 16 || block == 32, TSVDM_E_ARG, "block must be 0, 16 or 32");
    TSVDM_REQUIRE(max_sweeps >= 0 && max_sweeps <= 200, TSVDM_E_ARG, "max_sweeps must be in [0, 200]");
    for (int t = 0; t < count; ++t) {
        const int rc = validate_item(items[t], t);
        if (rc) return rc;
    }
    tsvdm_batch_plan_s* P = new tsvdm_batch_plan_s();
    P->items.assign(items, items + count);
    P->in_dt = in_dtype;
    P->dt = dtype;
    P->ttm_compute = ttm_compute;
    P->max_sweeps = max_sweeps ? max_sweeps : 40;
    int64_t rmax = 0;
    for (const auto& it : P->items) rmax = std::max(rmax, std::min(it.m, it.p));
    const int plan_block = block ? block : (rmax >= 256 ? 32 : 16);
    for (const auto& it : P->items) P->nb2.push_back(2 * (it.block ? it.block : plan_block));
    const size_t e = esz(dtype);
    size_t wsoff = 0;
    auto take = [&](size_t bytes) {
        wsoff = align_up(wsoff);
        const size_t o = wsoff;
        wsoff += bytes;
        return o;
    };
    // FP32 items with min(m, p) <= GRAM_MAX_R take the Gram form, the
    // others the rotation form.  The Gram form's Jacobi runs in LDS only when
    // every item is that small: the block rounds run for as many steps as
    // the largest slice needs, and small slices then ride along at a lower
    // cost than a separate in-LDS launch (latency bound, one workgroup per
    // slice), even one overlapped on a second stream.
    bool all_small = dtype == TSVDM_F32;
    for (const auto& it : P->items) all_small = all_small && std::min(it.m, it.p) <= GRAM_LDS_MAX_R;
    for (const auto& it : P->items) {
        const int64_t r = std::min(it.m, it.p);
        P->form.push_back(dtype != TSVDM_F32 || r > GRAM_MAX_R ? FORM_ROT
                          : (all_small ? FORM_GRAM_LDS : FORM_GRAM_ROUNDS));
    }
    P->slice_base.assign(count, 0);
    for (int pass = FORM_ROT; pass <= FORM_GRAM_LDS; ++pass)
        for (int t = 0; t < count; ++t) {
            if (P->form[t] != pass) continue;
            P->slice_base[t] = P->nslices;
            P->nslices += P->items[t].n;
            if (pass == FORM_ROT) P->n_rot += P->items[t].n;
            if (pass != FORM_GRAM_LDS) P->n_jac += P->items[t].n;
            if (pass != FORM_ROT) P->n_gram += P->items[t].n;
            if (pass == FORM_GRAM_LDS) P->n_lds += P->items[t].n;
        }
    std::vector<int> ccls[GRAM_CHOL_CLASSES], lcls[GRAM_LDS_CLASSES];
    int max_rounds = 1;
    std::vector<int4> ttm_by[TTM_SHAPES];
    std::vector<int2> jt_by[2];
    for (int t = 0; t < count; ++t) {
        const tsvdm_batch_item& it = P->items[t];
        const SliceGeom g = slice_geom(it.m, it.p);
        const int form = P->form[t];
        if (form != FORM_ROT) {
            P->off_gG.push_back(take((size_t)(g.r * g.r * it.n) * 8));
            P->off_gL.push_back(take((size_t)(g.r * g.r * it.n) * 8));
            P->off_gsh.push_back(take((size_t)it.n * 8));
            P->off_gfl.push_back(take((size_t)it.n * 4));
            P->off_gperm.push_back(take((size_t)(g.r * it.n) * 4));
        } else {
            P->off_gG.push_back(0);
            P->off_gL.push_back(0);
            P->off_gsh.push_back(0);
            P->off_gfl.push_back(0);
            P->off_gperm.push_back(0);
        }
        if (form != FORM_GRAM_LDS) {
            const int b = P->nb2[t] / 2;
            const int64_t nb = (g.r + b - 1) / b, nbe = nb + (nb & 1);
            P->off_trk.push_back(take((size_t)(nbe * nbe * it.n) * 4));
        } else {
            P->off_trk.push_back(0);
        }
        P->off_ahat.push_back(take((size_t)(it.m * it.p * it.n) * e));
        P->off_w.push_back(take((size_t)(g.r * g.r * it.n) * e));
        P->off_s2.push_back(take((size_t)(g.r * it.n) * 8));
        P->off_tf.push_back(take((size_t)(it.n * it.n) * 8));
        P->off_tb.push_back(take((size_t)(it.n * it.n) * 8));
        P->off_keys.push_back(take(it.mode == 2 ? (size_t)select_np2(g.r * it.n) * 8 : 8));
        P->off_stats.push_back(take(32));
        P->off_part.push_back(take(sizeof(double) * 2 * ERR_SEGS));
        int64_t cap = it.capacity;
        if (!it.U_pk) {
            cap = (it.mode == 1 ? std::min<int64_t>(it.k, g.r) : g.r) * it.n;
            P->off_upk.push_back(take((size_t)(it.m * cap) * e));
            P->off_gpk.push_back(take((size_t)(it.p * cap) * e));
            P->off_spk.push_back(take((size_t)cap * e));
        } else {
            P->off_upk.push_back(0);
            P->off_gpk.push_back(0);
            P->off_spk.push_back(0);
        }
        P->cap.push_back(cap);
        const int b = P->nb2[t] / 2;
        const int nb = (int)((g.r + b - 1) / b);
        const int nbe = nb + (nb & 1);
        if (form != FORM_GRAM_LDS) max_rounds = std::max(max_rounds, nbe - 1);
        // task tables
        int64_t n_rt;
        int n_ct;
        const int shp = ttm_resolve_tile(it.ttm_tile, it.n, P->ttm_compute);
        ttm_tile_counts(shp, it.m * it.p, it.n, &n_rt, &n_ct);
        for (int64_t rt = 0; rt < n_rt; ++rt)
            for (int ct = 0; ct < n_ct; ++ct) ttm_by[shp - 1].push_back(int4{t, (int)rt, ct, 0});
        const int ta = (int)((it.m + 63) / 64), tb = (int)((it.p + 63) / 64);
        std::vector<int2>& jt = jt_by[P->nb2[t] == 64 ? 1 : 0];
        const int nt = (int)((g.r + 63) / 64), ntri = nt * (nt + 1) / 2;
        const int ntl = (int)((g.L + 63) / 64);
        const int lcl = gram_lds_class(g.r), ccl = gram_chol_class(g.r);
        for (int64_t i = 0; i < it.n; ++i) {
            const int s = (int)(P->slice_base[t] + i);
            if (form != FORM_ROT) {
                const int gi = (int)(s - P->n_rot);
                for (int q = 0; q < ntri; ++q) P->gtasks.push_back(int2{gi, q});
                for (int tc = 0; tc < nt; ++tc)
                    for (int tt = 0; tt < ntl; ++tt) P->ftasks.push_back(int4{gi, tc, tt, 0});
                ccls[ccl].push_back(gi);
            }
            if (form == FORM_GRAM_LDS) {
                lcls[lcl].push_back((int)(s - P->n_rot));
                P->lds_maxr[lcl] = std::max(P->lds_maxr[lcl], (int)g.r);
            } else {
                for (int k = 0; k < nbe / 2; ++k) jt.push_back(int2{s, k});
            }
            if (it.A_rec)
                for (int y = 0; y < tb; ++y)
                    for (int x = 0; x < ta; ++x) P->lr_tasks.push_back(int4{s, x, y, 0});
        }
    }
    for (int c = 0; c < GRAM_CHOL_CLASSES; ++c) {
        P->chol_off[c] = (int64_t)P->glists.size();
        P->chol_cnt[c] = (int64_t)ccls[c].size();
        P->glists.insert(P->glists.end(), ccls[c].begin(), ccls[c].end());
    }
    for (int c = 0; c < GRAM_LDS_CLASSES; ++c) {
        P->lds_off[c] = (int64_t)P->glists.size();
        P->lds_cnt[c] = (int64_t)lcls[c].size();
        P->glists.insert(P->glists.end(), lcls[c].begin(), lcls[c].end());
    }
    for (int q = 0; q < TTM_SHAPES; ++q) {
        P->ttm_group[q] = (int64_t)ttm_by[q].size();
        P->ttm_tasks.insert(P->ttm_tasks.end(), ttm_by[q].begin(), ttm_by[q].end());
    }
    for (int q = 0; q < 2; ++q) {
        P->jgroup[q] = (int64_t)jt_by[q].size();
        P->jtasks.insert(P->jtasks.end(), jt_by[q].begin(), jt_by[q].end());
    }
    for (const auto& it : P->items) {
        if (!it.A_rec) continue;
        int64_t n_rt;
        int n_ct;
        ttm_tile_counts(ttm_resolve_tile(it.ttm_tile, it.n, P->ttm_compute), it.m * it.p, it.n, &n_rt, &n_ct);
        P->n_back += 1;
        P->n_back_tasks += n_rt * n_ct;
        P->n_err += it.err ? 1 : 0;
    }
    P->tab_bytes = layout_tables(P);
    P->off_tab = take(P->tab_bytes);
    P->max_steps = P->max_sweeps * max_rounds;
    if (P->max_steps > 100000) P->max_steps = 100000;
    P->off_ctl = take(256 + jacobi_batch_ctl_bytes(P->nslices, P->max_steps));
    P->ws_total = align_up(wsoff);
    if ((int64_t)P->jtasks.size() >= ((int64_t)1 << 31) || (int64_t)P->ttm_tasks.size() >= ((int64_t)1 << 31) ||
        (int64_t)P->lr_tasks.size() >= ((int64_t)1 << 31) || (int64_t)P->gtasks.size() >= ((int64_t)1 << 31) ||
        (int64_t)P->ftasks.size() >= ((int64_t)1 << 31)) {
        delete P;
        set_error("batch too large for one launch per stage");
        return TSVDM_E_SHAPE;
    }
    *plan = P;
    *ws_bytes = P->ws_total;
    return TSVDM_OK;
}

int tsvdm_batch_run(tsvdm_batch_plan P, void* ws, size_t ws_bytes, int host_poll, int use_graph,
                    int32_t* status, void* stream) {
    clear_error();
    TSVDM_REQUIRE(P != nullptr, TSVDM_E_ARG, "plan is NULL");
    TSVDM_REQUIRE(ws != nullptr && status != nullptr, TSVDM_E_ARG, "ws and status must be non-NULL");
    TSVDM_REQUIRE(host_poll == 0 || host_poll == 1, TSVDM_E_ARG, "host_poll must be 0 or 1");
    TSVDM_REQUIRE(use_graph == 0 || use_graph == 1, TSVDM_E_ARG, "use_graph must be 0 or 1");
    if (ws_bytes < P->ws_total) {
        set_error("workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(P->ws_total));
        return TSVDM_E_WORKSPACE;
    }
    hipStream_t st = as_stream(stream);
    char* base = static_cast<char*>(ws);
    if (P->n_lds > 0) {
        // the in-LDS Jacobi's dynamic LDS limit (a host attribute, set once
        // per process, before any capture below)
        const int rc = gram_lds_prepare();
        if (rc) return rc;
    }
    if (P->tables_ws != ws) {
        // tables embed workspace addresses; a captured graph of another
        // workspace is stale
        if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
        if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
        const int rc = build_tables(P, base);
        if (rc) return rc;
    }
    if (!use_graph) return run_stages(P, base, host_poll, status, st);
    TSVDM_REQUIRE(st != nullptr, TSVDM_E_ARG, "graph capture needs a non-default stream");
    TSVDM_REQUIRE(!stats_enabled(), TSVDM_E_ARG, "kernel statistics cannot be captured in a graph");
    if (!P->gexec || P->graph_ws != ws || P->graph_stream != st || P->graph_status != status) {
        if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
        if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
        TSVDM_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = run_stages(P, base, 0, status, st);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (ec != hipSuccess) {
            set_error(std::string("graph capture failed: ") + hipGetErrorString(ec));
            return TSVDM_E_HIP;
        }
        P->graph = g;
        TSVDM_HIP_CHECK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
        P->graph_ws = ws;
        P->graph_stream = st;
        P->graph_status = status;
    }
    TSVDM_HIP_CHECK(hipGraphLaunch(P->gexec, st));
    return TSVDM_OK;
}

int tsvdm_batch_plan_destroy(tsvdm_batch_plan P) {
    clear_error();
    if (!P) return TSVDM_OK;
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->htab) (void)hipHostFree(P->htab);
    delete P;
    return TSVDM_OK;
}

}  // extern "C"

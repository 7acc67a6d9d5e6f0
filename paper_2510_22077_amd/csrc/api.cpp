// C ABI: context life cycle, device uploads, FGMRES and Newton drivers.
//
// Paper: Newton x^{k+1} = x^k + delta^k with J^k delta^k = -r^k (Section 1);
// right-preconditioned GMRES stopped at ||A x - b|| / ||r(u=0,p=0)|| < tol
// (Section 8), here in its flexible form so that an FP32 preconditioner can sit
// inside the FP64 outer iteration; gPLMM built once from J~_w and reused for all
// Newton iterations, with the Stokes velocity as the fallback wind (Section 4).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace gp {
void cgs2(gplmm_ctx* c, const double* V, int64_t ldv, int k, double* w, int64_t n, double* hout);
void dots2(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* y, int64_t n, double* a, double* b);
double update2(gplmm_ctx* c, double* V, int64_t ldv, int j, const double* t, const double* s, double sj,
               double ainv, double* w, int64_t n);
void lincomb(gplmm_ctx* c, const double* Z, int64_t ldz, int k, const double* y_host, double* x, int64_t n);
int64_t red_scratch_doubles();

void timer_begin(gplmm_ctx* c, const char* name) {
    if (!c->timing) return;
    Timer& t = c->timers[name];
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, c->stream);
    t.ev0.push_back(e);
}

void timer_end(gplmm_ctx* c, const char* name, double bytes) {
    if (!c->timing) return;
    Timer& t = c->timers[name];
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, c->stream);
    t.ev1.push_back(e);
    t.bytes.push_back(bytes);
}
}  // namespace gp

using namespace gp;

namespace {

template <typename V>
int upload(gplmm_ctx* c, V** dst, const std::vector<V>& src) {
    size_t bytes = sizeof(V) * std::max<size_t>(src.size(), 1);
    GP_HIP(c, hipMalloc((void**)dst, bytes));
    if (!src.empty()) GP_HIP(c, hipMemcpy(*dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice));
    return GPLMM_OK;
}

#define GP_TRY(x)                    \
    do {                             \
        int rc_ = (x);               \
        if (rc_ != GPLMM_OK) return rc_; \
    } while (0)

int alloc(gplmm_ctx* c, void** p, size_t bytes) {
    GP_HIP(c, hipMalloc(p, std::max<size_t>(bytes, 16)));
    GP_HIP(c, hipMemset(*p, 0, std::max<size_t>(bytes, 16)));
    return GPLMM_OK;
}

size_t real_size(const gplmm_ctx* c) { return c->opt.precision == GPLMM_FP32 ? 4 : 8; }

// Position of coarse entry (row, col) in the block-diagonal storage (same block assumed).
int64_t coarse_pos(const gplmm_ctx* c, int row, int col) {
    const int b = c->co_blk[row];
    return c->cblk_moff[b] + (int64_t)c->co_loc[row] * c->cblk_n[b] + c->co_loc[col];
}

int upload_all(gplmm_ctx* c) {
    const int64_t nc = c->ncell, N = c->N;
    const int T = c->tile;
    // the Krylov kernels address a vector with 32-bit byte offsets
    if (N > (int64_t)INT32_MAX / 8) return fail(c, GPLMM_E_ARG, "more than 2^28 unknowns");
    // geometry
    GP_TRY(upload(c, &c->d_nb6, c->nbr));
    GP_TRY(upload(c, &c->d_tag, c->tagcell));
    if (!c->csamp.empty()) {   // batch: per-cell sample, per-sample physics and slot ranges
        GP_TRY(upload(c, &c->d_csamp, c->csamp));
        GP_TRY(upload(c, &c->d_sphys, c->sphys));
        std::vector<int64_t> seg;
        for (const SampleGeo& sg : c->samples) seg.push_back((int64_t)c->nrec * sg.coff);
        seg.push_back(N);
        GP_TRY(upload(c, &c->d_seg, seg));
        GP_TRY(alloc(c, (void**)&c->d_sscale, sizeof(double) * 2 * c->samples.size()));
        const size_t nb = sizeof(double) * c->samples.size() * 2 * (size_t)(c->opt.restart + 2);
        GP_TRY(alloc(c, (void**)&c->d_bres, nb));
        GP_TRY(alloc(c, (void**)&c->d_bcoef, nb));
        GP_TRY(alloc(c, (void**)&c->d_bsc, sizeof(double) * 2 * c->samples.size()));
        GP_HIP(c, hipHostMalloc((void**)&c->h_bres, nb, hipHostMallocDefault));
        std::vector<int32_t> ss(c->subs.size());   // sample of each subdomain (of its first unknown)
        for (size_t i = 0; i < c->subs.size(); ++i) {
            const Sub& sb = c->subs[i];
            ss[i] = c->csamp[c->sub_slots[sb.slot_off] / c->nrec];
        }
        GP_TRY(upload(c, &c->d_sub_samp, ss));
        GP_TRY(upload(c, &c->d_sact, std::vector<uint8_t>(c->samples.size(), 1)));
        GP_TRY(alloc(c, (void**)&c->d_alist, sizeof(int32_t) * c->samples.size()));
    }
    c->geo = DevGeo{c->nx, c->ny, c->nz, c->ndim, c->nrec, {c->opt.periodic[0], c->opt.periodic[1], c->opt.periodic[2]},
                    nc, (int)c->pin, c->opt.h, c->d_nb6, c->d_tag, c->d_csamp, c->d_sphys};
    // local problems
    const int nsub = c->Np + c->Nc;
    const int nall = (int)c->subs.size();   // with the split parts
    std::vector<int32_t> row_sub(c->sub_slots.size()), sorted_slot(c->sub_slots.size()), sorted_loc(c->sub_slots.size());
    std::vector<int64_t> local_off(nall + 1, 0);
    for (int s = 0; s < nall; ++s) {
        const Sub& sb = c->subs[s];
        std::vector<std::pair<int32_t, int32_t>> p(sb.n);
        for (int r = 0; r < sb.n; ++r) {
            row_sub[sb.slot_off + r] = s;
            p[r] = {c->sub_slots[sb.slot_off + r], r};
        }
        std::sort(p.begin(), p.end());
        for (int r = 0; r < sb.n; ++r) {
            sorted_slot[sb.slot_off + r] = p[r].first;
            sorted_loc[sb.slot_off + r] = p[r].second;
        }
        local_off[s + 1] = local_off[s] + (int64_t)sb.nT * T;
    }
    std::vector<int32_t> slot_class(N);
    for (int64_t s = 0; s < N; ++s) {
        int64_t q = s / c->nrec;
        int comp = (int)(s % c->nrec);
        slot_class[s] = comp < c->ndim ? c->owner[s] : (c->prim[q] >= 0 ? c->prim[q] : -4);
    }
    std::vector<int32_t> sub_ids(nall);
    for (int s = 0; s < nall; ++s) sub_ids[s] = s;
    GP_TRY(upload(c, &c->d_subs, c->subs));
    GP_TRY(upload(c, &c->d_sub_slots, c->sub_slots));
    GP_TRY(upload(c, &c->d_row_sub, row_sub));
    GP_TRY(upload(c, &c->d_sorted_slot, sorted_slot));
    GP_TRY(upload(c, &c->d_sorted_loc, sorted_loc));
    GP_TRY(upload(c, &c->d_slot_class, slot_class));
    GP_TRY(upload(c, &c->d_noclose, c->noclose));
    GP_TRY(upload(c, &c->d_local_off, local_off));
    GP_TRY(upload(c, &c->d_sub_ids, sub_ids));
    GP_TRY(upload(c, &c->d_tfc, c->env_tfc));
    GP_TRY(upload(c, &c->d_tfr, c->env_tfr));
    GP_TRY(upload(c, &c->d_lrow, c->env_lrow));
    GP_TRY(upload(c, &c->d_urow, c->env_urow));
    GP_TRY(upload(c, &c->d_tlc, c->env_tlc));
    for (int set = 0; set < 3; ++set) {
        GP_TRY(upload(c, &c->d_step_pairs[set], c->lu_step_pairs[set]));
        GP_TRY(upload(c, &c->d_sub_list[set], c->lu_sub_list[set]));
    }
    // triangular solves: each set's subdomains, largest first (they bound the launch)
    for (int set = 0; set < 2; ++set) {
        int s0 = set == 0 ? 0 : c->Np, s1 = set == 0 ? c->Np : nsub;
        std::vector<int32_t> ord;
        for (int sidx = s0; sidx < s1; ++sidx) ord.push_back(sidx);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return c->subs[a].nT > c->subs[b].nT; });
        c->maxT_set[set] = ord.empty() ? 0 : c->subs[ord[0]].nT;
        GP_TRY(upload(c, &c->d_sub_order[set], ord));
    }
    // split primaries: phase 1 = forward over the unsplit primaries (whole solves) and the
    // halves, phase 3 = backward over the halves; separators' inverses
    if (!c->splits.empty()) {
        std::vector<int32_t> p1, p3, sep;
        for (int s = 0; s < nall; ++s) {
            const Sub& sb = c->subs[s];
            if ((sb.kind == 0 && sb.split < 0) || sb.kind == 2) p1.push_back(s);
            if (sb.kind == 2) p3.push_back(s);
        }
        auto by_size = [&](int a, int b) { return c->subs[a].nT > c->subs[b].nT; };
        std::stable_sort(p1.begin(), p1.end(), by_size);
        std::stable_sort(p3.begin(), p3.end(), by_size);
        c->n_phase1 = (int)p1.size();
        c->n_phase3 = (int)p3.size();
        c->maxT_phase1 = c->subs[p1[0]].nT;
        c->maxT_phase3 = c->subs[p3[0]].nT;
        std::vector<int64_t> inv_off(nall, 0);
        std::vector<int32_t> inv_cols(nall, 0);
        for (const Split& sp : c->splits) {
            sep.push_back(sp.s_sub);
            inv_off[sp.s_sub] = sp.inv_off;
            inv_cols[sp.s_sub] = sp.nS;
        }
        GP_TRY(upload(c, &c->d_phase_order[0], p1));
        GP_TRY(upload(c, &c->d_phase_order[1], p3));
        GP_TRY(upload(c, &c->d_sep_ids, sep));
        GP_TRY(upload(c, &c->d_sinv_off, inv_off));
        GP_TRY(upload(c, &c->d_sinv_ncols, inv_cols));
        GP_TRY(upload(c, &c->d_splits, c->splits));
        GP_TRY(alloc(c, &c->d_sinv, real_size(c) * c->sinv_elems));
        int64_t used = 0;
        for (int s = 0; s < nall; ++s) {
            const Sub& sb = c->subs[s];
            if (sb.kind == 0 && sb.split < 0) {
                used += (s + 1 < nall ? c->subs[s + 1].diag_off : c->factor_elems) - sb.diag_off;
            } else if (sb.kind == 2) {
                const int stop = sb.sep0 / T;
                for (int I = 0; I < sb.nT; ++I) {
                    const int tfc = c->env_tfc[sb.env_off + I];
                    used += (int64_t)std::max(std::min(I, stop) - tfc, 0) * T * T;
                    if (I < stop) used += (int64_t)(1 + c->env_tlc[sb.env_off + I] - I) * T * T;
                }
            }
        }
        for (const Split& sp : c->splits) used += (int64_t)sp.ld * sp.nS;
        c->split_apply_elems = used;
        c->split_row0 = c->subs[c->nsub_main].slot_off;
        c->split_row1 = (int64_t)c->sub_slots.size();
    }
    // the blocks of A^f_f (mg_form 1, 2): after the duals, largest first
    if (c->n_fsub > 0) {
        std::vector<int32_t> fo;
        for (int s = nsub; s < nsub + c->n_fsub; ++s) fo.push_back(s);
        std::stable_sort(fo.begin(), fo.end(), [&](int a, int b) { return c->subs[a].nT > c->subs[b].nT; });
        c->maxT_f = c->subs[fo[0]].nT;
        GP_TRY(upload(c, &c->d_fsub_order, fo));
        c->f_row0 = c->subs[nsub].slot_off;
        c->f_row1 = nsub + c->n_fsub < nall ? c->subs[nsub + c->n_fsub].slot_off : (int64_t)c->sub_slots.size();
    }
    c->prim_factor_elems = nall > c->Np ? c->subs[c->Np].diag_off : c->factor_elems;
    c->prim_rows = nall > c->Np ? c->subs[c->Np].slot_off : (int64_t)c->sub_slots.size();
    GP_TRY(alloc(c, &c->d_factor, real_size(c) * c->factor_elems));
    GP_TRY(alloc(c, (void**)&c->d_inv64, sizeof(double) * 1024 * std::max(nall, 1)));
    GP_TRY(alloc(c, &c->d_local, real_size(c) * local_off[nall]));
    // shape/correction blocks: column-major with ld = nT * T, right-hand sides built here
    std::vector<int64_t> phi_off(c->Np + 1, 0);
    std::vector<int32_t> phi_ncols(std::max(nsub, 1), 0);
    c->max_phi_cols = 0;
    for (int i = 0; i < c->Np; ++i) {
        int nck = (int)c->Cp[i].size() + 1;
        phi_ncols[i] = nck;
        c->max_phi_cols = std::max(c->max_phi_cols, nck);
        phi_off[i + 1] = phi_off[i] + (int64_t)c->subs[i].nT * T * nck;
    }
    c->phi_elems = phi_off[c->Np];
    std::vector<double> rhs(c->phi_elems, 0.0);
    const double ih = 1.0 / c->opt.h;
    for (int i = 0; i < c->Np; ++i) {
        const Sub& sb = c->subs[i];
        const int ld = sb.nT * T;
        const int ncp = (int)c->Cp[i].size();
        for (int r = 0; r < sb.n; ++r) {
            int64_t s = c->sub_slots[sb.slot_off + r];
            int64_t q = s / c->nrec;
            int comp = (int)(s % c->nrec);
            if (comp >= c->ndim) continue;
            int64_t L = c->nbr[q * 6 + 2 * comp];
            int jq = c->iface[q], jl = L >= 0 ? c->iface[L] : -1;
            for (int k = 0; k < ncp; ++k) {
                int j = c->Cp[i][k];
                double g = 0.0;
                if (jq == j) g -= ih;   // -X[F, p_R] with X[F, p_R] = +1/h
                if (jl == j) g += ih;   // -X[F, p_L] with X[F, p_L] = -1/h
                rhs[phi_off[i] + (int64_t)k * ld + r] = g;
            }
            const Phys& ph = c->csamp.empty() ? c->phys : c->sphys[c->csamp[q]];
            rhs[phi_off[i] + (int64_t)ncp * ld + r] = ph.rho * ph.body[comp];
        }
    }
    if (c->opt.precision == GPLMM_FP32) {
        std::vector<float> rf(rhs.begin(), rhs.end());
        GP_TRY(alloc(c, &c->d_phi_rhs, sizeof(float) * rf.size()));
        if (!rf.empty()) GP_HIP(c, hipMemcpy(c->d_phi_rhs, rf.data(), sizeof(float) * rf.size(), hipMemcpyHostToDevice));
    } else {
        GP_TRY(alloc(c, &c->d_phi_rhs, sizeof(double) * rhs.size()));
        if (!rhs.empty()) GP_HIP(c, hipMemcpy(c->d_phi_rhs, rhs.data(), sizeof(double) * rhs.size(), hipMemcpyHostToDevice));
    }
    GP_TRY(alloc(c, &c->d_phi, real_size(c) * c->phi_elems));
    phi_off.resize(std::max(nsub, 1) + 1, phi_off.back());
    GP_TRY(upload(c, &c->d_phi_off, phi_off));
    GP_TRY(upload(c, &c->d_phi_ncols, phi_ncols));
    GP_TRY(upload(c, &c->d_phi_cols, c->phi_cols));
    GP_TRY(upload(c, &c->d_phi_cols_off, c->phi_cols_off));
    {   // prolongation workgroups: each primary's rows in chunks of 256
        std::vector<int32_t> pb;
        c->max_pcols = 0;
        for (int i = 0; i < c->Np; ++i) {
            for (int ch = 0; ch * 256 < c->subs[i].n; ++ch) {
                pb.push_back(i);
                pb.push_back(ch);
            }
            c->max_pcols = std::max(c->max_pcols, (int)(c->phi_cols_off[i + 1] - c->phi_cols_off[i]));
        }
        c->n_prolong_blk = (int)(pb.size() / 2);
        GP_TRY(upload(c, &c->d_prolong_blk, pb));
    }
    // row groups of Rhat: interfaces (their cells' pressures), then corrections (every slot of S_i)
    std::vector<int64_t> gptr(1, 0);
    std::vector<int32_t> gslot;
    for (int j = 0; j < c->Nc; ++j) {
        for (int32_t q : c->icells[j]) gslot.push_back((int32_t)((int64_t)c->nrec * q + c->ndim));
        gptr.push_back((int64_t)gslot.size());
    }
    for (int i = 0; i < c->Np; ++i) {
        if (c->ycol[i] < 0) continue;
        const Sub& sb = c->subs[i];
        for (int r = 0; r < sb.n; ++r) gslot.push_back(c->sub_slots[sb.slot_off + r]);
        gptr.push_back((int64_t)gslot.size());
    }
    GP_TRY(upload(c, &c->d_grp_ptr, gptr));
    GP_TRY(upload(c, &c->d_grp_slot, gslot));
    // dual gather lists: for each slot, the local rows of the dual grids that contain it
    std::vector<int64_t> dcount(N + 1, 0);
    for (int s = c->Np; s < nsub; ++s) {
        const Sub& sb = c->subs[s];
        for (int r = 0; r < sb.n; ++r) dcount[c->sub_slots[sb.slot_off + r] + 1]++;
    }
    for (int64_t s = 0; s < N; ++s) dcount[s + 1] += dcount[s];
    std::vector<int64_t> dsrc(dcount[N]);
    std::vector<int64_t> fillp(dcount.begin(), dcount.end() - 1);
    for (int s = c->Np; s < nsub; ++s) {   // ascending dual id, so each slot's order is fixed
        const Sub& sb = c->subs[s];
        for (int r = 0; r < sb.n; ++r) dsrc[fillp[c->sub_slots[sb.slot_off + r]]++] = local_off[s] + r;
    }
    GP_TRY(upload(c, &c->d_dinv_ptr, dcount));
    GP_TRY(upload(c, &c->d_dinv, dsrc));
    // probing
    GP_TRY(upload(c, &c->d_probe, c->probe));
    GP_TRY(upload(c, &c->d_color_cols, c->color_cols));
    const int nco = c->nco;
    const int64_t coe = std::max<int64_t>(c->co_elems, 1);
    GP_TRY(alloc(c, (void**)&c->d_Ao, sizeof(double) * coe));
    GP_TRY(alloc(c, (void**)&c->d_Aowork, sizeof(double) * coe));
    GP_TRY(alloc(c, (void**)&c->d_Aoasm, sizeof(double) * coe));
    GP_TRY(alloc(c, (void**)&c->d_piv, sizeof(int32_t) * 2 * std::max(c->cblk_max, 1)));
    GP_TRY(alloc(c, (void**)&c->d_panel, sizeof(double) * 32 * std::max(c->cblk_max, 1)));
    GP_TRY(upload(c, &c->d_co_blk, c->co_blk));
    GP_TRY(upload(c, &c->d_co_loc, c->co_loc));
    GP_TRY(upload(c, &c->d_cblk_n, c->cblk_n));
    GP_TRY(upload(c, &c->d_cblk_idx, c->cblk_idx));
    GP_TRY(upload(c, &c->d_cblk_ioff, c->cblk_ioff));
    GP_TRY(upload(c, &c->d_cblk_moff, c->cblk_moff));
    GP_TRY(alloc(c, (void**)&c->d_cv, sizeof(double) * 2 * std::max(nco, 1)));
    GP_TRY(alloc(c, (void**)&c->d_probe_e, sizeof(double) * 2 * kProbeColors * std::max(nco, 1)));
    GP_TRY(alloc(c, (void**)&c->d_flag, sizeof(int) * 4));
    // vectors
    const int m = c->opt.restart;
    GP_TRY(alloc(c, (void**)&c->d_wind, sizeof(double) * N));
    const int slots = 1 + 2 * c->ndim + (c->opt.build_matrix == GPLMM_BUILD_JACOBIAN ? 4 * (c->ndim - 1) : 0);
    const int64_t ncoef = (int64_t)slots * c->ndim * nc;
    GP_TRY(alloc(c, (void**)&c->d_xcoef, sizeof(double) * ncoef));
    if (c->opt.precision == GPLMM_FP32) GP_TRY(alloc(c, (void**)&c->d_xcoef_f, sizeof(float) * ncoef));
    GP_TRY(alloc(c, (void**)&c->d_r, sizeof(double) * N));
    GP_TRY(alloc(c, (void**)&c->d_tmp, sizeof(double) * N));
    GP_TRY(alloc(c, (void**)&c->d_dx, sizeof(double) * N));
    GP_TRY(alloc(c, (void**)&c->d_zero, sizeof(double) * N));
    GP_TRY(alloc(c, (void**)&c->d_V, sizeof(double) * (int64_t)(m + 1) * N));
    GP_TRY(alloc(c, (void**)&c->d_Z, sizeof(double) * (int64_t)m * N));
    GP_TRY(alloc(c, (void**)&c->d_red, sizeof(double) * red_scratch_doubles()));
    GP_HIP(c, hipHostMalloc((void**)&c->h_red, sizeof(double) * 8 * (kMaxRestart + 2), hipHostMallocDefault));
    GP_TRY(alloc(c, &c->d_pv, real_size(c) * 6 * N));
    return GPLMM_OK;
}

int do_build(gplmm_ctx* c) {
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    launch_xcoef(c, c->stream);
    if (c->opt.precision == GPLMM_FP32) {
        rc = build_precond<float>(c);
    } else {
        rc = build_precond<double>(c);
    }
    c->last_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

static int apply_eager(gplmm_ctx* c, const double* v, double* z) {
    return c->opt.precision == GPLMM_FP32 ? apply_precond<float>(c, v, z) : apply_precond<double>(c, v, z);
}

// Capture one application, from the staging input to the staging output, on a private
// stream (the context's stream may be the default stream, which cannot be captured).
static int capture_apply(gplmm_ctx* c) {
    if (c->apply_exec) {
        (void)hipGraphExecDestroy(c->apply_exec);
        c->apply_exec = nullptr;
    }
    if (c->apply_graph) {
        (void)hipGraphDestroy(c->apply_graph);
        c->apply_graph = nullptr;
    }
    if (!c->cap_stream) GP_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->d_gin) {
        GP_TRY(alloc(c, (void**)&c->d_gin, sizeof(double) * c->N));
        GP_TRY(alloc(c, (void**)&c->d_gout, sizeof(double) * c->N));
    }
    GP_HIP(c, hipStreamSynchronize(c->stream));
    hipStream_t keep = c->stream;
    c->stream = c->cap_stream;
    GP_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = apply_eager(c, c->d_gin, c->d_gout);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = keep;
    if (rc != GPLMM_OK) return rc;
    if (e != hipSuccess) return fail(c, GPLMM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    c->apply_graph = g;
    GP_HIP(c, hipGraphInstantiate(&c->apply_exec, g, nullptr, nullptr, 0));
    c->graph_valid = true;
    return GPLMM_OK;
}

int do_apply(gplmm_ctx* c, const double* v, double* z) {
    if (c->opt.use_graph && !c->timing) {
        if (!c->graph_valid) GP_TRY(capture_apply(c));
        GP_HIP(c, hipMemcpyAsync(c->d_gin, v, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream));
        GP_HIP(c, hipGraphLaunch(c->apply_exec, c->stream));
        GP_HIP(c, hipMemcpyAsync(z, c->d_gout, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream));
        return GPLMM_OK;
    }
    timer_begin(c, "precond_apply");
    int rc = apply_eager(c, v, z);
    timer_end(c, "precond_apply", c->apply_bytes);
    return rc;
}

// FGMRES(m) for J(xk) d = b, d = 0 initially; |residual| <= tol_abs.  Returns iterations.
//
// Arnoldi with classical Gram-Schmidt applied twice, the second projection of each basis
// vector delayed into the next step (DCGS2: Bielich, Langou, Thomas, Swirydowicz, Yamazaki
// and Boman, Parallel Computing 2022): step j computes the dots of V[0..j] with both the
// tentative v_j and the new w = J z_j in one pass, then, in a second pass, finishes v_j
// (v_j <- (v_j - V t) / alpha) and projects w against the finished basis.  The Hessenberg
// column j - 1, whose subdiagonal entry referred to the tentative v_j, is corrected by the
// same coefficients (J z_{j-1} = sum_i h_i v_i + beta (alpha v_j' + V t)) and only then
// rotated, so the residual estimate lags the basis by one step.  z_j = M^-1 (tentative v_j)
// is kept as computed: flexible GMRES needs only J Z = V H with orthonormal V.
int fgmres(gplmm_ctx* c, const double* xk, const double* b, double* d, double tol_abs, int maxit, bool* ok) {
    const int64_t N = c->N;
    const int m = c->opt.restart;
    double* V = c->d_V;
    double* Z = c->d_Z;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), a(m + 2), bb(m + 2);
    auto Hx = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    auto rotate = [&](int col) {   // previous rotations, then a new one eliminating H[col+1][col]
        for (int i = 0; i < col; ++i) {
            const double t = cs[i] * Hx(i, col) + sn[i] * Hx(i + 1, col);
            Hx(i + 1, col) = -sn[i] * Hx(i, col) + cs[i] * Hx(i + 1, col);
            Hx(i, col) = t;
        }
        const double den = std::hypot(Hx(col, col), Hx(col + 1, col));
        cs[col] = den > 0.0 ? Hx(col, col) / den : 1.0;
        sn[col] = den > 0.0 ? Hx(col + 1, col) / den : 0.0;
        Hx(col, col) = den;
        Hx(col + 1, col) = 0.0;
        g[col + 1] = -sn[col] * g[col];
        g[col] = cs[col] * g[col];
    };
    hipMemsetAsync(d, 0, sizeof(double) * N, c->stream);
    hipMemcpyAsync(V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream);
    double beta = nrm2(c, V, N);
    int total = 0;
    *ok = beta <= tol_abs;
    while (!*ok && total < maxit) {
        scal_copy(c, 1.0 / beta, V, V, N);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kdone = 0;          // finished Hessenberg columns
        bool stop = false;
        double bprev = 0.0;     // norm of the projected w of the previous step
        int j = 0;
        for (; j < m && total < maxit; ++j) {
            double* vj = V + (int64_t)j * N;
            double* zj = Z + (int64_t)j * N;
            double* w = V + (int64_t)(j + 1) * N;
            int rc = do_apply(c, vj, zj);
            if (rc) return -1;
            timer_begin(c, "jv");
            launch_jv(c, xk, zj, w, c->stream);
            timer_end(c, "jv", c->jv_bytes);
            ++total;
            timer_begin(c, "arnoldi");
            dots2(c, V, N, j + 1, w, N, a.data(), bb.data());
            double tt = 0.0, tb = 0.0;
            for (int i = 0; i < j; ++i) {
                tt += a[i] * a[i];
                tb += a[i] * bb[i];
            }
            const double alpha = std::sqrt(std::max(a[j] - tt, 1e-300));
            const double sj = (bb[j] - tb) / alpha;
            const double wn2 = update2(c, V, N, j, a.data(), bb.data(), sj, 1.0 / alpha, w, N);
            // algorithmic bytes of the step: the dots read V[0..j] and w (j + 2 vectors), the
            // update reads V[0..j) and reads and writes v_j and w (j + 4 vectors)
            timer_end(c, "arnoldi", 8.0 * (double)N * (double)(2 * j + 6));
            if (!std::isfinite(wn2) || !std::isfinite(alpha) || !std::isfinite(sj)) {
                // a non-finite preconditioner or Jacobian output: the step is a failure, and
                // d keeps the finite update of the cycles before (zero in the first)
                *ok = false;
                return total;
            }
            const double hn = std::sqrt(std::max(wn2, 0.0));
            if (j >= 1) {   // column j - 1 referred to the tentative v_j
                for (int i = 0; i < j; ++i) Hx(i, j - 1) += bprev * a[i];
                Hx(j, j - 1) = bprev * alpha;
                rotate(j - 1);
                kdone = j;
                if (std::fabs(g[j]) <= tol_abs) {
                    stop = true;
                    break;
                }
            }
            for (int i = 0; i < j; ++i) Hx(i, j) = bb[i];
            Hx(j, j) = sj;
            Hx(j + 1, j) = hn;
            bprev = hn;
            // residual estimate with column j as it stands (its subdiagonal entry changes only
            // by the rounding-level reorthogonalisation of v_{j+1}): when it meets the
            // tolerance, or w lies in the span of the basis, column j is final
            double hj, hj1;
            {
                std::vector<double> col(j + 2);
                for (int i = 0; i <= j; ++i) col[i] = Hx(i, j);
                col[j + 1] = hn;
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                    col[i] = t;
                }
                hj = col[j];
                hj1 = col[j + 1];
            }
            const double den = std::hypot(hj, hj1);
            const double est = den > 0.0 ? std::fabs(hj1 / den * g[j]) : 0.0;
            if (est <= tol_abs || !(hn > 0.0)) {
                rotate(j);
                kdone = j + 1;
                stop = true;
                ++j;
                break;
            }
            scal_copy(c, 1.0 / hn, w, w, N);
        }
        if (!stop && kdone < j) {
            // the last column: one more pass gives the delayed projection of v_j
            dots2(c, V, N, j + 1, V + (int64_t)j * N, N, a.data(), bb.data());
            double tt = 0.0;
            for (int i = 0; i < j; ++i) tt += a[i] * a[i];
            const double alpha = std::sqrt(std::max(a[j] - tt, 1e-300));
            for (int i = 0; i < j; ++i) Hx(i, j - 1) += bprev * a[i];
            Hx(j, j - 1) = bprev * alpha;
            rotate(j - 1);
            kdone = j;
            if (std::fabs(g[j]) <= tol_abs) stop = true;
        }
        const int k = kdone;
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= Hx(i, l) * y[l];
            y[i] = s / Hx(i, i);
        }
        for (int i = 0; i < k; ++i)
            if (!std::isfinite(y[i])) {
                *ok = false;
                return total;
            }
        if (k > 0) lincomb(c, Z, N, k, y.data(), d, N);
        if (stop && std::fabs(g[k]) <= tol_abs) {   // converged (the estimate met the tolerance)
            *ok = true;
            break;
        }
        if (c->progress) c->progress(c->progress_user, c->progress_newton, total, -1.0);
        // restart from the true residual b - J d
        launch_jv(c, xk, d, c->d_tmp, c->stream);
        scal_copy(c, -1.0, c->d_tmp, V, N);
        axpy(c, 1.0, b, V, N);
        beta = nrm2(c, V, N);
        if (!std::isfinite(beta)) return total;
        if (beta <= tol_abs) *ok = true;
    }
    return total;
}

// FGMRES for a batch: one Arnoldi process per sample, run in lockstep.  The preconditioner
// and the Jacobian act on all samples at once (the batch is block diagonal); the dot
// products, Gram-Schmidt coefficients, norms, Hessenberg matrices, rotations and stopping
// tests are per sample (the same delayed CGS2 steps as fgmres()), so each sample converges
// to its own tolerance tol_abs[s] in as many iterations as it would need alone.  A sample
// that has converged has its slice of the basis set to zero, which keeps it at zero.
int fgmres_batch(gplmm_ctx* c, const double* xk, const double* b, double* d, const double* tol_abs, int maxit,
                 bool* ok) {
    const int64_t N = c->N;
    const int m = c->opt.restart;
    const int ns = (int)c->samples.size();
    const int ld = m + 2;
    double* V = c->d_V;
    double* Z = c->d_Z;
    std::vector<double> H((size_t)ns * (m + 1) * m, 0.0), cs((size_t)ns * m), sn((size_t)ns * m),
        g((size_t)ns * (m + 1)), y((size_t)ns * ld, 0.0), a((size_t)ns * (m + 2)), bb((size_t)ns * (m + 2)),
        coef((size_t)ns * 2 * ld, 0.0), sc((size_t)ns * 2), nrm(ns), beta(ns), bprev(ns), scale(ns);
    std::vector<int> kdone(ns, 0);
    std::vector<int32_t> alist;
    std::vector<char> done(ns, 0), active(ns, 0);
    auto Hx = [&](int s, int i, int j) -> double& { return H[((size_t)s * (m + 1) + i) * m + j]; };
    auto rotate = [&](int s, int col) {
        double* css = cs.data() + (size_t)s * m;
        double* sns = sn.data() + (size_t)s * m;
        double* gs = g.data() + (size_t)s * (m + 1);
        for (int i = 0; i < col; ++i) {
            const double t = css[i] * Hx(s, i, col) + sns[i] * Hx(s, i + 1, col);
            Hx(s, i + 1, col) = -sns[i] * Hx(s, i, col) + css[i] * Hx(s, i + 1, col);
            Hx(s, i, col) = t;
        }
        const double den = std::hypot(Hx(s, col, col), Hx(s, col + 1, col));
        css[col] = den > 0.0 ? Hx(s, col, col) / den : 1.0;
        sns[col] = den > 0.0 ? Hx(s, col + 1, col) / den : 0.0;
        Hx(s, col, col) = den;
        Hx(s, col + 1, col) = 0.0;
        gs[col + 1] = -sns[col] * gs[col];
        gs[col] = css[col] * gs[col];
    };
    auto seg_norms = [&](const double* v) {
        seg_sumsq(c, v, nrm.data());
        for (int s = 0; s < ns; ++s) beta[s] = std::sqrt(std::max(nrm[s], 0.0));
    };
    auto set_scale = [&](double* v) -> int {   // v slice of sample s *= scale[s]
        GP_HIP(c, hipMemcpyAsync(c->d_sscale, scale.data(), sizeof(double) * ns, hipMemcpyHostToDevice, c->stream));
        seg_scale(c, c->d_sscale, v);
        return GPLMM_OK;
    };
    hipMemsetAsync(d, 0, sizeof(double) * N, c->stream);
    hipMemcpyAsync(V, b, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream);
    seg_norms(V);
    int total = 0, ndone = 0;
    for (int s = 0; s < ns; ++s)
        if (beta[s] <= tol_abs[s]) {
            done[s] = 1;
            ++ndone;
        }
    std::vector<uint8_t> act8(ns, 1);
    auto push_active = [&]() -> int {   // finished samples skip their local solves
        for (int s = 0; s < ns; ++s) act8[s] = active[s] ? 1 : 0;
        GP_HIP(c, hipMemcpyAsync(c->d_sact, act8.data(), ns, hipMemcpyHostToDevice, c->stream));
        GP_HIP(c, hipStreamSynchronize(c->stream));
        return GPLMM_OK;
    };
    while (ndone < ns && total < maxit) {
        for (int s = 0; s < ns; ++s) {
            active[s] = !done[s];
            scale[s] = done[s] ? 0.0 : 1.0 / beta[s];
            kdone[s] = 0;
            std::fill(g.begin() + (size_t)s * (m + 1), g.begin() + (size_t)(s + 1) * (m + 1), 0.0);
            g[(size_t)s * (m + 1)] = done[s] ? 0.0 : beta[s];
        }
        GP_TRY(set_scale(V));
        GP_TRY(push_active());
        int nact = ns - ndone, j = 0;
        for (; j < m && total < maxit && nact > 0; ++j) {
            double* vj = V + (int64_t)j * N;
            double* zj = Z + (int64_t)j * N;
            double* w = V + (int64_t)(j + 1) * N;
            if (do_apply(c, vj, zj)) return -1;
            timer_begin(c, "jv");
            launch_jv(c, xk, zj, w, c->stream);
            timer_end(c, "jv", c->jv_bytes);
            ++total;
            timer_begin(c, "arnoldi");
            const int k = j + 1;
            alist.clear();
            for (int s = 0; s < ns; ++s)
                if (active[s]) alist.push_back(s);
            const int na = (int)alist.size();
            seg_dots2(c, V, N, k, w, alist.data(), na, a.data(), bb.data());
            for (int yy = 0; yy < na; ++yy) {
                const int s = alist[yy];
                double* as = a.data() + (size_t)yy * k;
                const double* bs = bb.data() + (size_t)yy * k;
                double* cf = coef.data() + (size_t)s * 2 * ld;
                double tt = 0.0, tb = 0.0;
                for (int i = 0; i < j; ++i) {
                    tt += as[i] * as[i];
                    tb += as[i] * bs[i];
                    cf[i] = as[i];
                    cf[ld + i] = bs[i];
                }
                const double alpha = std::sqrt(std::max(as[j] - tt, 1e-300));
                sc[2 * s] = (bs[j] - tb) / alpha;
                sc[2 * s + 1] = 1.0 / alpha;
                as[j] = alpha;   // kept for the column correction below
            }
            seg_update2(c, V, N, j, coef.data(), ld, sc.data(), alist.data(), na, w, nrm.data());
            timer_end(c, "arnoldi", 0.0);
            bool changed = false;
            for (int s = 0; s < ns; ++s) scale[s] = 0.0;
            for (int yy = 0; yy < na; ++yy) {
                const int s = alist[yy];
                const double* as = a.data() + (size_t)yy * k;
                const double* bs = bb.data() + (size_t)yy * k;
                const double alpha = as[j];
                if (!std::isfinite(nrm[yy]) || !std::isfinite(alpha) || !std::isfinite(sc[2 * s])) {
                    // non-finite preconditioner or Jacobian output: the step fails
                    std::fill(active.begin(), active.end(), 1);
                    GP_TRY(push_active());
                    *ok = false;
                    return total;
                }
                const double hn = std::sqrt(std::max(nrm[yy], 0.0));
                double* gs = g.data() + (size_t)s * (m + 1);
                bool conv = false;
                if (j >= 1) {
                    for (int i = 0; i < j; ++i) Hx(s, i, j - 1) += bprev[s] * as[i];
                    Hx(s, j, j - 1) = bprev[s] * alpha;
                    rotate(s, j - 1);
                    kdone[s] = j;
                    conv = std::fabs(gs[j]) <= tol_abs[s];
                }
                if (!conv) {
                    for (int i = 0; i < j; ++i) Hx(s, i, j) = bs[i];
                    Hx(s, j, j) = sc[2 * s];
                    Hx(s, j + 1, j) = hn;
                    bprev[s] = hn;
                    std::vector<double> col(j + 2);
                    for (int i = 0; i <= j; ++i) col[i] = Hx(s, i, j);
                    col[j + 1] = hn;
                    const double* css = cs.data() + (size_t)s * m;
                    const double* sns = sn.data() + (size_t)s * m;
                    for (int i = 0; i < j; ++i) {
                        const double t = css[i] * col[i] + sns[i] * col[i + 1];
                        col[i + 1] = -sns[i] * col[i] + css[i] * col[i + 1];
                        col[i] = t;
                    }
                    const double den = std::hypot(col[j], col[j + 1]);
                    const double est = den > 0.0 ? std::fabs(col[j + 1] / den * gs[j]) : 0.0;
                    if (est <= tol_abs[s] || !(hn > 0.0)) {
                        rotate(s, j);
                        kdone[s] = j + 1;
                        conv = true;
                    } else {
                        scale[s] = 1.0 / hn;
                    }
                }
                if (conv) {
                    active[s] = 0;
                    --nact;
                    changed = true;
                }
            }
            GP_TRY(set_scale(w));
            if (changed) GP_TRY(push_active());
        }
        // samples still active at the end of the cycle: the delayed projection of their last
        // basis vector completes the last Hessenberg column
        if (nact > 0 && j >= 1) {
            const int k = j + 1;
            alist.clear();
            for (int s = 0; s < ns; ++s)
                if (active[s]) alist.push_back(s);
            seg_dots2(c, V, N, k, V + (int64_t)j * N, alist.data(), (int)alist.size(), a.data(), bb.data());
            for (int yy = 0; yy < (int)alist.size(); ++yy) {
                const int s = alist[yy];
                const double* as = a.data() + (size_t)yy * k;
                double tt = 0.0;
                for (int i = 0; i < j; ++i) tt += as[i] * as[i];
                const double alpha = std::sqrt(std::max(as[j] - tt, 1e-300));
                for (int i = 0; i < j; ++i) Hx(s, i, j - 1) += bprev[s] * as[i];
                Hx(s, j, j - 1) = bprev[s] * alpha;
                rotate(s, j - 1);
                kdone[s] = j;
            }
        }
        int kmax = 0;
        for (int s = 0; s < ns; ++s) {
            double* ys = y.data() + (size_t)s * ld;
            std::fill(ys, ys + ld, 0.0);
            const int k = done[s] ? 0 : kdone[s];
            const double* gs = g.data() + (size_t)s * (m + 1);
            for (int i = k - 1; i >= 0; --i) {
                double t = gs[i];
                for (int l = i + 1; l < k; ++l) t -= Hx(s, i, l) * ys[l];
                ys[i] = t / Hx(s, i, i);
            }
            kmax = std::max(kmax, k);
            if (!done[s] && (std::fabs(gs[k]) <= tol_abs[s])) {
                done[s] = 1;
                ++ndone;
            }
        }
        if (kmax > 0) seg_lincomb(c, Z, N, kmax, y.data(), ld, d);
        if (ndone == ns) break;
        if (c->progress) c->progress(c->progress_user, c->progress_newton, total, -1.0);
        // restart the unfinished samples from the true residual b - J d
        launch_jv(c, xk, d, c->d_tmp, c->stream);
        scal_copy(c, -1.0, c->d_tmp, V, N);
        axpy(c, 1.0, b, V, N);
        seg_norms(V);
        for (int s = 0; s < ns; ++s)
            if (!done[s] && beta[s] <= tol_abs[s]) {
                done[s] = 1;
                ++ndone;
            }
    }
    std::fill(active.begin(), active.end(), 1);   // later builds and applications cover every sample
    GP_TRY(push_active());
    *ok = ndone == ns;
    return total;
}

}  // namespace

extern "C" {

void gplmm_default_options(gplmm_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->nx = o->ny = 0;
    o->nz = 1;
    o->h = 1.0;
    o->periodic[0] = 1;
    o->precision = GPLMM_FP64;
    o->wind_mode = GPLMM_WIND_STOKES;
    o->tag_layers = 1;
    o->dual_dilations = -1;
    o->restart = 30;
    o->newton_tol = 1e-8;
    o->lin_tol = 1e-9;
    o->line_search = 0;
    o->use_graph = 1;
    o->newton_maxit = 30;
    o->lin_maxit = 600;
    o->tile = 0;
    o->stream = nullptr;
}

// Options check shared by the single-image and batch set-ups.
static int check_options(gplmm_ctx* c, const gplmm_options* opt, double rho, double mu) {
    if (c->opt.restart <= 0) c->opt.restart = 30;
    if (c->opt.tile == 0) c->opt.tile = 32;
    if (c->opt.restart > kMaxRestart) return fail(c, GPLMM_E_ARG, "restart must be <= 1024");
    if (c->opt.tile != 32) return fail(c, GPLMM_E_ARG, "only tile = 32 is supported");
    if (c->opt.build_matrix != GPLMM_BUILD_GEOMETRIC && c->opt.build_matrix != GPLMM_BUILD_JACOBIAN)
        return fail(c, GPLMM_E_ARG, "build_matrix must be GPLMM_BUILD_GEOMETRIC or GPLMM_BUILD_JACOBIAN");
    if (c->opt.split_tiles < -1) return fail(c, GPLMM_E_ARG, "split_tiles must be -1, 0 or positive");
    if (c->opt.mg_form < 0 || c->opt.mg_form > 2) return fail(c, GPLMM_E_ARG, "mg_form must be 0, 1 or 2");
    if (c->opt.mg_form != 0 && c->opt.split_tiles > 0)
        return fail(c, GPLMM_E_ARG, "mg_form 1 and 2 do not combine with split_tiles");
    if (opt->nx <= 0 || opt->ny <= 0 || opt->nz <= 0) return fail(c, GPLMM_E_ARG, "image dimensions must be positive");
    if (opt->nx > 1024 || opt->ny > 1024 || opt->nz > 1024)
        return fail(c, GPLMM_E_ARG, "image dimensions must be <= 1024");
    if (!(rho > 0) || !(mu > 0) || !(opt->h > 0)) return fail(c, GPLMM_E_ARG, "rho, mu and h must be positive");
    return GPLMM_OK;
}

static void set_dims(gplmm_ctx* c, int nx, int ny, int nz) {
    c->tile = 32;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->ndim = nz == 1 ? 2 : 3;
    c->nrec = c->ndim + 1;
    c->nvox = (int64_t)nx * ny * nz;
}

// Everything after the decomposition: local problems, probing, coarse blocks, uploads.
static int finish_setup(gplmm_ctx* c) {
    int rc = build_local_problems(c);
    if (rc == GPLMM_OK) rc = build_probing(c);
    if (rc == GPLMM_OK) {
        build_coarse_blocks(c);
        for (const ProbeEntry& p : c->probe)   // every coarse coupling stays inside one block
            if (c->co_blk[p.row] != c->co_blk[p.col]) {
                rc = fail(c, GPLMM_E_GEOMETRY, "a coarse coupling crosses two samples");
                break;
            }
    }
    if (rc == GPLMM_OK && !c->opt.host_only) rc = upload_all(c);
    if (rc == GPLMM_OK && !c->opt.host_only) {   // X of the zero wind until the first build
        launch_xcoef(c, c->stream);
        if (hipStreamSynchronize(c->stream) != hipSuccess) rc = gp::fail(c, GPLMM_E_HIP, "coefficient table");
    }
    if (rc == GPLMM_OK && !c->opt.host_only) {
        // algorithmic bytes of one preconditioner application (for roofline reporting):
        // every local factor read once, the shape vectors once, the coarse inverse once,
        // and about 16 vector passes over N slots
        const double rs = (double)real_size(c);
        c->apply_bytes = rs * (double)c->factor_elems + rs * (double)c->phi_elems + 8.0 * (double)c->co_elems +
                         16.0 * rs * (double)c->N;
        c->jv_bytes = 8.0 * 3.0 * (double)c->N + 24.0 * (double)c->ncell;
        c->ready = true;
    }
    return rc;
}

int gplmm_setup(const uint8_t* mask, const int32_t* labels, double rho, double mu, const double body[3], double dt,
                const gplmm_options* opt, gplmm_ctx** out) {
    if (!mask || !labels || !opt || !out || !body) return GPLMM_E_ARG;
    *out = nullptr;
    gplmm_ctx* c = new gplmm_ctx();
    c->opt = *opt;
    *out = c;
    int rc = check_options(c, opt, rho, mu);
    if (rc != GPLMM_OK) return rc;
    set_dims(c, opt->nx, opt->ny, opt->nz);
    c->phys = Phys{rho, mu, {body[0], body[1], c->ndim == 3 ? body[2] : 0.0}, dt > 0 ? dt : 0.0};
    c->stream = (hipStream_t)opt->stream;
    rc = build_decomposition(c, mask, labels);
    c->samples.assign(1, SampleGeo{0, 0, c->nx, c->ny, c->nz, 0, 0});
    if (rc == GPLMM_OK) rc = finish_setup(c);
    return rc;
}

int gplmm_setup_pnm(const uint8_t* mask, const int32_t* throat_labels, const int32_t* pore_labels, double rho,
                    double mu, const double body[3], double dt, const gplmm_options* opt, gplmm_ctx** out) {
    if (!mask || !throat_labels || !pore_labels || !opt || !out || !body) return GPLMM_E_ARG;
    *out = nullptr;
    gplmm_ctx* c = new gplmm_ctx();
    c->opt = *opt;
    *out = c;
    int rc = check_options(c, opt, rho, mu);
    if (rc != GPLMM_OK) return rc;
    set_dims(c, opt->nx, opt->ny, opt->nz);
    c->phys = Phys{rho, mu, {body[0], body[1], c->ndim == 3 ? body[2] : 0.0}, dt > 0 ? dt : 0.0};
    c->stream = (hipStream_t)opt->stream;
    c->setup_groups = pore_labels;
    rc = build_decomposition(c, mask, throat_labels);
    c->setup_groups = nullptr;
    c->samples.assign(1, SampleGeo{0, 0, c->nx, c->ny, c->nz, 0, 0});
    if (rc == GPLMM_OK) rc = finish_setup(c);
    return rc;
}

int gplmm_setup_batch(int nsamples, const uint8_t* const* masks, const int32_t* const* labels, const int32_t* dims,
                      const double* rho, const double* mu, const double* body, const double* dt,
                      const gplmm_options* opt, gplmm_ctx** out) {
    if (!out) return GPLMM_E_ARG;
    *out = nullptr;
    if (nsamples < 1 || !masks || !labels || !dims || !rho || !mu || !body || !opt) return GPLMM_E_ARG;
    gplmm_ctx* c = new gplmm_ctx();
    c->opt = *opt;
    *out = c;
    if (opt->mg_form != 0) return fail(c, GPLMM_E_ARG, "mg_form 1 and 2 take a single image");
    c->stream = (hipStream_t)opt->stream;
    if (nsamples > kMaxSamples) return fail(c, GPLMM_E_ARG, "at most 1024 samples per batch");
    int rc0 = check_options(c, opt, rho[0], mu[0]);
    if (rc0 != GPLMM_OK) return rc0;
    const int nd = dims[2] == 1 ? 2 : 3;
    std::vector<gplmm_ctx*> parts;
    int rc = GPLMM_OK;
    for (int s = 0; s < nsamples && rc == GPLMM_OK; ++s) {
        gplmm_options o = *opt;
        o.nx = dims[3 * s];
        o.ny = dims[3 * s + 1];
        o.nz = dims[3 * s + 2];
        o.host_only = 1;
        gplmm_ctx* p = new gplmm_ctx();
        p->opt = o;
        parts.push_back(p);
        rc = check_options(p, &o, rho[s], mu[s]);
        if (rc == GPLMM_OK && (o.nz == 1 ? 2 : 3) != nd) rc = fail(p, GPLMM_E_ARG, "samples of mixed dimension");
        if (rc == GPLMM_OK && (!masks[s] || !labels[s])) rc = fail(p, GPLMM_E_ARG, "null image");
        if (rc == GPLMM_OK) {
            set_dims(p, o.nx, o.ny, o.nz);
            rc = build_decomposition(p, masks[s], labels[s]);
        }
        if (rc != GPLMM_OK) c->err = "sample " + std::to_string(s) + ": " + p->err;
        const double d = dt ? dt[s] : 0.0;
        c->sphys.push_back(Phys{rho[s], mu[s], {body[3 * s], body[3 * s + 1], nd == 3 ? body[3 * s + 2] : 0.0},
                                d > 0 ? d : 0.0});
    }
    if (rc == GPLMM_OK) {
        c->opt.nx = parts[0]->nx;
        c->opt.ny = parts[0]->ny;
        c->opt.nz = parts[0]->nz;
        set_dims(c, parts[0]->nx, parts[0]->ny, parts[0]->nz);
        c->phys = c->sphys[0];
        rc = merge_samples(c, parts);
    }
    for (gplmm_ctx* p : parts) delete p;
    if (rc == GPLMM_OK && nsamples == 1) {   // one sample: the plain context
        c->csamp.clear();
        c->sphys.clear();
    }
    if (rc == GPLMM_OK) rc = finish_setup(c);
    return rc;
}

int gplmm_batch_info(const gplmm_ctx* c, int* nsamples, int64_t* cell_off, int64_t* voxel_off, int32_t* prim_off,
                     int32_t* iface_off) {
    if (!c) return GPLMM_E_ARG;
    const int ns = (int)c->samples.size();
    if (nsamples) *nsamples = ns;
    for (int s = 0; s <= ns; ++s) {
        const bool end = s == ns;
        if (cell_off) cell_off[s] = end ? c->ncell : c->samples[s].coff;
        if (voxel_off) voxel_off[s] = end ? c->nvox : c->samples[s].voff;
        if (prim_off) prim_off[s] = end ? c->Np : c->samples[s].p0;
        if (iface_off) iface_off[s] = end ? c->Nc : c->samples[s].i0;
    }
    return GPLMM_OK;
}

int gplmm_layout_info(const gplmm_ctx* c, gplmm_layout* o) {
    if (!c || !o) return GPLMM_E_ARG;
    std::memset(o, 0, sizeof(*o));
    o->ndim = c->ndim;
    o->nrec = c->nrec;
    o->ncell = c->ncell;
    o->N = c->N;
    o->nface_active = c->nface;
    o->Np = c->Np;
    o->Nc = c->Nc;
    o->Ny = c->Ny;
    o->pin = c->pin;
    std::vector<uint8_t> cov(c->ncell, 0);
    for (auto& d : c->dual_cells)
        for (int32_t q : d) cov[q] = 1;
    o->ndual_cells = std::count(cov.begin(), cov.end(), 1);
    int64_t lu = 0;
    for (int i = 0; i < c->Np; ++i) lu += 2 * (int64_t)c->subs[i].n;
    for (int j = 0; j < c->Nc; ++j) lu += c->subs[c->Np + j].n;
    o->local_unknowns = lu;
    o->factor_bytes = (int64_t)(c->opt.precision == GPLMM_FP32 ? 4 : 8) * c->factor_elems;
    o->ncolors = c->ncolors;
    o->lu_flops = c->lu_flops[0] + c->lu_flops[1] + c->lu_flops[2];
    o->nsplit = (int)c->splits.size();
    for (const Split& sp : c->splits) o->sep_unknowns += sp.nS;
    o->nfblock = c->n_fsub;
    for (int k = 0; k < c->n_fsub; ++k) {
        const Sub& sb = c->subs[c->Np + c->Nc + k];
        o->max_fblock = std::max(o->max_fblock, sb.n);
        o->f_unknowns += sb.n;
    }
    return GPLMM_OK;
}

int gplmm_get_maps(const gplmm_ctx* c, int32_t* cell_voxel, int32_t* cell_iface, int32_t* cell_prim,
                   int32_t* face_owner, int8_t* face_tag) {
    if (!c) return GPLMM_E_ARG;
    if (cell_voxel) std::copy(c->cell_voxel.begin(), c->cell_voxel.end(), cell_voxel);
    if (cell_iface) std::copy(c->iface.begin(), c->iface.end(), cell_iface);
    if (cell_prim) std::copy(c->prim.begin(), c->prim.end(), cell_prim);
    if (face_owner) std::copy(c->owner.begin(), c->owner.end(), face_owner);
    if (face_tag)
        for (int64_t k = 0; k < c->N; ++k) face_tag[k] = (int8_t)(c->tagslot[k] | (c->noclose[k] << 1));
    return GPLMM_OK;
}

int gplmm_get_duals(const gplmm_ctx* c, int64_t* ptr, int32_t* cells) {
    if (!c || !ptr) return GPLMM_E_ARG;
    ptr[0] = 0;
    for (int j = 0; j < c->Nc; ++j) {
        ptr[j + 1] = ptr[j] + (int64_t)c->dual_cells[j].size();
        if (cells) std::copy(c->dual_cells[j].begin(), c->dual_cells[j].end(), cells + ptr[j]);
    }
    return GPLMM_OK;
}

int gplmm_get_split(const gplmm_ctx* c, int k, int32_t* info, int32_t* slots) {
    if (!c || !info) return GPLMM_E_ARG;
    if (k < 0 || k >= (int)c->splits.size()) return GPLMM_E_ARG;
    const Split& sp = c->splits[k];
    info[0] = sp.prim;
    info[1] = sp.nA;
    info[2] = sp.nB;
    info[3] = sp.nS;
    if (slots) {
        const Sub& a = c->subs[sp.a_sub];
        const Sub& b = c->subs[sp.b_sub];
        const int32_t* sa = c->sub_slots.data() + a.slot_off;
        const int32_t* sb = c->sub_slots.data() + b.slot_off;
        std::copy(sa, sa + sp.nA, slots);
        std::copy(sb, sb + sp.nB, slots + sp.nA);
        std::copy(sa + sp.nA, sa + sp.nA + sp.nS, slots + sp.nA + sp.nB);
    }
    return GPLMM_OK;
}

int gplmm_get_fblocks(const gplmm_ctx* c, int64_t* ptr, int32_t* slots) {
    if (!c || !ptr) return GPLMM_E_ARG;
    ptr[0] = 0;
    for (int k = 0; k < c->n_fsub; ++k) {
        const Sub& sb = c->subs[c->Np + c->Nc + k];
        ptr[k + 1] = ptr[k] + sb.n;
        if (slots) {   // each block's local order is its slot order
            const int32_t* sl = c->sub_slots.data() + sb.slot_off;
            std::copy(sl, sl + sb.n, slots + ptr[k]);
        }
    }
    return GPLMM_OK;
}

int gplmm_get_subdomains(const gplmm_ctx* c, int32_t* n, int64_t* factor_elems) {
    if (!c) return GPLMM_E_ARG;
    const int nsub = c->Np + c->Nc;   // the split parts are not reported
    const int nall = (int)c->subs.size();
    for (int s = 0; s < nsub; ++s) {
        if (n) n[s] = c->subs[s].n;
        if (factor_elems)
            factor_elems[s] = (s + 1 < nall ? c->subs[s + 1].diag_off : c->factor_elems) - c->subs[s].diag_off;
    }
    return GPLMM_OK;
}

int gplmm_residual(gplmm_ctx* c, const double* x, const double* xprev, double* r) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!x || !r) return GPLMM_E_ARG;
    launch_residual(c, x, xprev, r, c->stream);
    GP_HIP(c, hipGetLastError());
    return GPLMM_OK;
}

int gplmm_matvec(gplmm_ctx* c, const double* xlin, const double* v, double* y) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!xlin || !v || !y) return GPLMM_E_ARG;
    launch_jv(c, xlin, v, y, c->stream);
    GP_HIP(c, hipGetLastError());
    return GPLMM_OK;
}

int gplmm_build_matvec(gplmm_ctx* c, const double* v, double* y) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!v || !y) return GPLMM_E_ARG;
    launch_xv<double>(c, v, y, nullptr, c->stream);
    GP_HIP(c, hipGetLastError());
    return GPLMM_OK;
}

int gplmm_build(gplmm_ctx* c, const double* wind) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (wind) GP_HIP(c, hipMemcpyAsync(c->d_wind, wind, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream));
    else GP_HIP(c, hipMemsetAsync(c->d_wind, 0, sizeof(double) * c->N, c->stream));
    int rc = do_build(c);
    if (rc == GPLMM_OK) GP_HIP(c, hipGetLastError());
    return rc;
}

int gplmm_set_coarse_model(gplmm_ctx* c, gplmm_mlp* model) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (model && (gp::mlp_width_in(model) != gp::kCoarseFeatures || gp::mlp_width_out(model) != 1))
        return gp::fail(c, GPLMM_E_ARG, "the coarse model must map 16 features to one value");
    if (model && c->opt.mg_form == 1)
        return gp::fail(c, GPLMM_E_ARG, "the coarse model predicts Rhat X Phat, not the operator of mg_form 1");
    c->coarse_model = model;
    return GPLMM_OK;
}

int gplmm_coarse_entries(gplmm_ctx* c, int64_t* nent, int32_t* rows, int32_t* cols, float* feat, float* scale,
                         double* exact) {
    if (!c || !nent) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    std::vector<double> wh(c->N);
    GP_HIP(c, hipMemcpyAsync(wh.data(), c->d_wind, sizeof(double) * c->N, hipMemcpyDeviceToHost, c->stream));
    GP_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<float> f, s;
    gp::coarse_features(c, wh.data(), f, s);
    const int64_t ne = (int64_t)c->cl_row.size();
    *nent = ne;
    if (rows) std::copy(c->cl_row.begin(), c->cl_row.end(), rows);
    if (cols) std::copy(c->cl_col.begin(), c->cl_col.end(), cols);
    if (feat) std::copy(f.begin(), f.end(), feat);
    if (scale) std::copy(s.begin(), s.end(), scale);
    if (exact) {
        if (!c->built || c->last_coarse_learned)
            return gp::fail(c, GPLMM_E_STATE, "exact coarse values need a preceding build with the exact operator");
        std::vector<double> A((size_t)c->co_elems);
        GP_HIP(c, hipMemcpy(A.data(), c->d_Aoasm, sizeof(double) * A.size(), hipMemcpyDeviceToHost));
        for (int64_t e = 0; e < ne; ++e) exact[e] = A[coarse_pos(c, c->cl_row[e], c->cl_col[e])];
    }
    return GPLMM_OK;
}

int gplmm_get_coarse(gplmm_ctx* c, double* ao, int* nco_out) {
    if (!c) return GPLMM_E_ARG;
    if (nco_out) *nco_out = c->nco;
    if (!ao) return GPLMM_OK;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!c->built) return fail(c, GPLMM_E_STATE, "gplmm_build must precede gplmm_get_coarse");
    std::vector<double> A((size_t)c->co_elems);
    GP_HIP(c, hipMemcpyAsync(A.data(), c->d_Aoasm, sizeof(double) * A.size(), hipMemcpyDeviceToHost, c->stream));
    GP_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t nco = c->nco;
    std::fill(ao, ao + nco * nco, 0.0);
    for (size_t b = 0; b < c->cblk_n.size(); ++b) {
        const int n = c->cblk_n[b];
        const int32_t* idx = c->cblk_idx.data() + c->cblk_ioff[b];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) ao[idx[i] * nco + idx[j]] = A[c->cblk_moff[b] + (int64_t)i * n + j];
    }
    return GPLMM_OK;
}

int gplmm_precond_apply(gplmm_ctx* c, const double* v, double* z) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!v || !z || v == z) return GPLMM_E_ARG;
    if (!c->built) return fail(c, GPLMM_E_STATE, "gplmm_build must precede gplmm_precond_apply");
    int rc = do_apply(c, v, z);
    if (rc == GPLMM_OK) GP_HIP(c, hipGetLastError());
    return rc;
}

int gplmm_newton_solve(gplmm_ctx* c, const double* xprev, double* x, gplmm_stats* st) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!x) return GPLMM_E_ARG;
    gplmm_stats loc;
    gplmm_stats* S = st ? st : &loc;
    std::memset(S, 0, sizeof(*S));
    auto T0 = std::chrono::steady_clock::now();
    const int64_t N = c->N;
    const int64_t reorth0 = c->gs_reorth;
    // A batch is one block-diagonal system: FGMRES runs one Arnoldi process per sample
    // (fgmres_batch) to lin_tol * ||r_s(0)|| on every sample s, and Newton stops when the
    // largest relative residual max_s ||r_s|| / ||r_s(0)|| reaches newton_tol.
    const bool batch = !c->csamp.empty();
    const int ns = (int)c->samples.size();
    std::vector<double> r0s(ns, 0.0), rns(ns, 0.0), rts(ns, 0.0);
    double* d_r2 = nullptr;
    auto rel_max = [&](const std::vector<double>& v) {
        double m = 0.0;
        for (int s = 0; s < ns; ++s) m = std::max(m, v[s] / r0s[s]);
        return m;
    };
    // ||r(0)||: the residual at the origin (previous time level also zero)
    launch_residual(c, c->d_zero, c->d_zero, c->d_r, c->stream);
    const double r0 = nrm2(c, c->d_r, N);
    S->r0_norm = r0;
    if (!(r0 > 0)) return fail(c, GPLMM_E_ARG, "the residual at the origin is zero (no driving force)");
    std::vector<double> lin_tols(ns);
    if (batch) {
        seg_sumsq(c, c->d_r, r0s.data());
        for (int s = 0; s < ns; ++s) {
            r0s[s] = std::sqrt(r0s[s]);
            if (!(r0s[s] > 0))
                return fail(c, GPLMM_E_ARG, "sample " + std::to_string(s) + " has no driving force");
            lin_tols[s] = c->opt.lin_tol * r0s[s];
        }
        d_r2 = (double*)c->d_V;   // trial residuals of the line search (the Krylov basis is free then)
    }
    const double lin_abs = c->opt.lin_tol * r0;
    auto solve_step = [&](bool* ok) {
        return batch ? fgmres_batch(c, x, c->d_r, c->d_dx, lin_tols.data(), c->opt.lin_maxit, ok)
                     : fgmres(c, x, c->d_r, c->d_dx, lin_abs, c->opt.lin_maxit, ok);
    };
    const int mode = c->opt.wind_mode;
    if (mode != GPLMM_WIND_CALLER || !c->built) {
        if (mode != GPLMM_WIND_CALLER) hipMemsetAsync(c->d_wind, 0, sizeof(double) * N, c->stream);
        int rc = do_build(c);
        S->t_build_ms += c->last_build_ms;
        S->builds++;
        S->t_coarse_ms += c->last_coarse_ms;
        S->learned_builds += c->last_coarse_learned ? 1 : 0;
        if (rc) return rc;
    }
    launch_residual(c, x, xprev, c->d_r, c->stream);
    double rn = nrm2(c, c->d_r, N);
    double rel = rn / r0;
    if (batch) {
        seg_sumsq(c, c->d_r, rns.data());
        for (auto& v : rns) v = std::sqrt(v);
        rel = rel_max(rns);
    }
    S->res_hist[0] = rel;
    int rcode = 1;
    for (int k = 0; k < c->opt.newton_maxit && k < 64; ++k) {
        if (rel <= c->opt.newton_tol) {
            rcode = 0;
            break;
        }
        if (k == 1 && mode == GPLMM_WIND_STOKES) {
            hipMemcpyAsync(c->d_wind, x, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream);
            int rc = do_build(c);
            S->t_build_ms += c->last_build_ms;
            S->builds++;
            S->t_coarse_ms += c->last_coarse_ms;
            S->learned_builds += c->last_coarse_learned ? 1 : 0;
            if (rc) return rc;
        }
        scal_copy(c, -1.0, c->d_r, c->d_r, N);   // b = -r (fgmres leaves d_r alone)
        auto t1 = std::chrono::steady_clock::now();
        bool ok = false;
        c->progress_newton = k + 1;
        int its = solve_step(&ok);
        if (its < 0) return GPLMM_E_HIP;
        if (!ok && c->last_coarse_learned) {
            // the learned coarse operator did not carry FGMRES to the tolerance: rebuild with
            // the exact one (same wind) for the rest of the solve and redo this step
            gplmm_mlp* model = c->coarse_model;
            c->coarse_model = nullptr;
            int rc = do_build(c);
            c->coarse_model = model;
            S->t_build_ms += c->last_build_ms;
            S->builds++;
            S->t_coarse_ms += c->last_coarse_ms;
            S->coarse_fallbacks++;
            if (rc) return rc;
            its += solve_step(&ok);
        }
        S->t_solve_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
        S->lin_its[k] = its;
        S->lin_its_total += its;
        S->newton_its = k + 1;
        if (batch && c->opt.line_search) {
            // backtracking per sample: each sample keeps the first trial step that meets its
            // own sufficient-decrease test (the samples are independent)
            std::vector<char> acc(ns, 0);
            int nacc = 0;
            double lam = 1.0, lam_min = 1.0;
            for (;;) {
                GP_HIP(c, hipMemcpyAsync(c->d_tmp, x, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
                axpy(c, lam, c->d_dx, c->d_tmp, N);
                launch_residual(c, c->d_tmp, xprev, d_r2, c->stream);
                seg_sumsq(c, d_r2, rts.data());
                const bool last = lam <= 1.0 / 64.0;
                for (int s = 0; s < ns; ++s) {
                    if (acc[s]) continue;
                    const double rt = std::sqrt(rts[s]);
                    if (last && !std::isfinite(rt))
                        return fail(c, GPLMM_E_BREAKDOWN, "Newton step " + std::to_string(k + 1) + ": sample " +
                                                              std::to_string(s) + " has a non-finite residual at "
                                                              "every trial step");
                    if (rt <= (1.0 - 1e-4 * lam) * rns[s] || last) {
                        acc[s] = 1;
                        ++nacc;
                        rns[s] = rt;
                        lam_min = std::min(lam_min, lam);
                        const int64_t a = (int64_t)c->nrec * c->samples[s].coff;
                        const int64_t b = s + 1 < ns ? (int64_t)c->nrec * c->samples[s + 1].coff : N;
                        GP_HIP(c, hipMemcpyAsync(x + a, c->d_tmp + a, sizeof(double) * (b - a),
                                                 hipMemcpyDeviceToDevice, c->stream));
                        GP_HIP(c, hipMemcpyAsync(c->d_r + a, d_r2 + a, sizeof(double) * (b - a),
                                                 hipMemcpyDeviceToDevice, c->stream));
                    }
                }
                if (nacc == ns) break;
                lam *= 0.5;
            }
            rel = rel_max(rns);
            S->step_length[k] = lam_min;
        } else if (c->opt.line_search) {
            // backtracking on ||r||, trial points in d_tmp; d_r ends holding r(x_new)
            double lam = 1.0;
            for (;;) {
                GP_HIP(c, hipMemcpyAsync(c->d_tmp, x, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
                axpy(c, lam, c->d_dx, c->d_tmp, N);
                launch_residual(c, c->d_tmp, xprev, c->d_r, c->stream);
                const double rt = nrm2(c, c->d_r, N);
                if (!std::isfinite(rt) && lam <= 1.0 / 64.0)
                    return fail(c, GPLMM_E_BREAKDOWN, "Newton step " + std::to_string(k + 1) +
                                                          ": non-finite residual at every trial step");
                if (rt <= (1.0 - 1e-4 * lam) * rn || lam <= 1.0 / 64.0) {
                    GP_HIP(c, hipMemcpyAsync(x, c->d_tmp, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
                    rn = rt;
                    break;
                }
                lam *= 0.5;
            }
            rel = rn / r0;
            S->step_length[k] = lam;
        } else {
            // full Newton step x + delta (the paper's update); the trial point is kept in d_tmp
            // until its residual is known to be finite, so x never takes a non-finite step
            GP_HIP(c, hipMemcpyAsync(c->d_tmp, x, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
            axpy(c, 1.0, c->d_dx, c->d_tmp, N);
            launch_residual(c, c->d_tmp, xprev, c->d_r, c->stream);
            rn = nrm2(c, c->d_r, N);
            if (!std::isfinite(rn))
                return fail(c, GPLMM_E_BREAKDOWN, "Newton step " + std::to_string(k + 1) +
                                                      ": non-finite residual; x keeps the last finite iterate");
            GP_HIP(c, hipMemcpyAsync(x, c->d_tmp, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
            rel = rn / r0;
            if (batch) {
                seg_sumsq(c, c->d_r, rns.data());
                for (auto& v : rns) v = std::sqrt(v);
                rel = rel_max(rns);
            }
            S->step_length[k] = 1.0;
        }
        S->res_hist[k + 1] = rel;
        if (c->progress) c->progress(c->progress_user, k + 1, its, rel);
    }
    if (rel <= c->opt.newton_tol) rcode = 0;
    S->converged = rcode == 0;
    S->gs_reorth = (int)(c->gs_reorth - reorth0);
    GP_HIP(c, hipStreamSynchronize(c->stream));
    GP_HIP(c, hipGetLastError());
    S->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - T0).count();
    return rcode;
}

void gplmm_coarse_default_options(gplmm_coarse_options* o) {
    if (!o) return;
    o->increments = 1;
    o->newton_maxit = 50;
    o->tol = 1e-6;
}

int gplmm_coarse_solve(gplmm_ctx* c, const gplmm_coarse_options* opt, double* x, gplmm_coarse_stats* st) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!x || !opt) return GPLMM_E_ARG;
    if (!c->csamp.empty()) return fail(c, GPLMM_E_ARG, "the coarse-scale solver takes a single image");
    if (c->phys.dt > 0.0) return fail(c, GPLMM_E_ARG, "the coarse-scale solver is for the steady equations");
    if (c->opt.tag_layers < 1) return fail(c, GPLMM_E_ARG, "the coarse-scale solver needs tag_layers >= 1");
    if (c->nco <= 0) return fail(c, GPLMM_E_ARG, "no coarse unknowns (a single pore)");
    if (opt->increments < 1 || opt->increments > 64 || opt->newton_maxit < 1 || !(opt->tol > 0.0))
        return fail(c, GPLMM_E_ARG, "coarse options: 1 <= increments <= 64, newton_maxit >= 1, tol > 0");
    gplmm_coarse_stats loc;
    gplmm_coarse_stats* S = st ? st : &loc;
    std::memset(S, 0, sizeof(*S));
    auto T0 = std::chrono::steady_clock::now();
    const int64_t N = c->N;
    const int nco = c->nco;
    const bool fp32 = c->opt.precision == GPLMM_FP32;
    const Phys full = c->phys;
    double* rc = c->d_dx;          // coarse residual (nco), then the coarse step (nco)
    double* dc = c->d_dx + nco;
    std::vector<double> h(nco);
    auto coarse_norm = [&]() -> double {
        launch_residual(c, x, nullptr, c->d_r, c->stream, true);
        coarse_restrict(c, c->d_r, rc);
        hipMemcpyAsync(h.data(), rc, sizeof(double) * nco, hipMemcpyDeviceToHost, c->stream);
        hipStreamSynchronize(c->stream);
        double s2 = 0.0;
        for (double v : h) s2 += v * v;
        return std::sqrt(s2);
    };
    int rcode = 0;
    GP_HIP(c, hipMemsetAsync(x, 0, sizeof(double) * N, c->stream));
    const int n = opt->increments;
    S->converged = 1;
    for (int m = 1; m <= n && rcode >= 0; ++m) {
        const double f = (double)m / n;
        for (int a = 0; a < 3; ++a) c->phys.body[a] = full.body[a] * f;
        // wind: the velocity of the previous step (zero at the first); pressures are ignored
        GP_HIP(c, hipMemcpyAsync(c->d_wind, x, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
        int rc_b = do_build(c);
        S->t_build_ms += c->last_build_ms;
        if (rc_b != GPLMM_OK) {
            rcode = rc_b;
            break;
        }
        const double r0 = coarse_norm();
        double rel = r0 > 0.0 ? 1.0 : 0.0;
        int its = 0;
        while (its < opt->newton_maxit && rel >= opt->tol && r0 > 0.0) {
            int rj = fp32 ? coarse_jacobian<float>(c, x) : coarse_jacobian<double>(c, x);
            if (rj != GPLMM_OK) {
                rcode = rj;
                break;
            }
            if (fp32) coarse_update<float>(c, rc, dc, c->d_tmp, x);
            else coarse_update<double>(c, rc, dc, c->d_tmp, x);
            ++its;
            const double rn = coarse_norm();
            if (!std::isfinite(rn)) {
                rcode = fail(c, GPLMM_E_BREAKDOWN, "coarse-scale solver: non-finite coarse residual");
                break;
            }
            rel = rn / r0;
        }
        S->increments = m;
        S->newton_its[m - 1] = its;
        S->rc_rel[m - 1] = rel;
        if (rel >= opt->tol) S->converged = 0;
    }
    c->phys = full;
    c->built = false;            // the coarse blocks hold J_c^-1 and the factors the last step's
    c->graph_valid = false;
    if (rcode < 0) return rcode;
    // true residual of the approximate solution, against r(0) of the full driving force
    launch_residual(c, c->d_zero, c->d_zero, c->d_r, c->stream);
    const double r0f = nrm2(c, c->d_r, N);
    launch_residual(c, x, nullptr, c->d_r, c->stream);
    S->fine_rel_residual = nrm2(c, c->d_r, N) / r0f;
    GP_HIP(c, hipStreamSynchronize(c->stream));
    GP_HIP(c, hipGetLastError());
    S->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - T0).count();
    return S->converged ? GPLMM_OK : 1;
}

int gplmm_continuation(gplmm_ctx* c, int steps, const double* scales, double* x, gplmm_stats* st) {
    if (!c) return GPLMM_E_ARG;
    if (!c->ready) return fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    if (!x || !scales || !st) return GPLMM_E_ARG;
    if (!c->csamp.empty()) return fail(c, GPLMM_E_ARG, "the continuation takes a single image");
    if (c->phys.dt > 0.0) return fail(c, GPLMM_E_ARG, "the continuation is for the steady equations");
    if (steps < 1 || steps > 64) return fail(c, GPLMM_E_ARG, "continuation: 1 <= steps <= 64");
    for (int k = 0; k < steps; ++k)
        if (!(scales[k] > (k ? scales[k - 1] : 0.0)) || scales[k] > 1.0)
            return fail(c, GPLMM_E_ARG, "continuation: scales must increase within (0, 1]");
    if (scales[steps - 1] != 1.0) return fail(c, GPLMM_E_ARG, "continuation: the last scale must be 1");
    const Phys full = c->phys;
    const int mode = c->opt.wind_mode;
    int rc = GPLMM_OK;
    for (int k = 0; k < steps; ++k) {
        for (int a = 0; a < 3; ++a) c->phys.body[a] = full.body[a] * scales[k];
        std::memset(&st[k], 0, sizeof(gplmm_stats));
        if (k > 0) {
            // the preconditioner of each later step is built once from the velocity of the
            // step before (Section 8's protocol), and Newton starts from that state
            auto t0 = std::chrono::steady_clock::now();
            GP_HIP(c, hipMemcpyAsync(c->d_wind, x, sizeof(double) * c->N, hipMemcpyDeviceToDevice, c->stream));
            rc = do_build(c);
            if (rc != GPLMM_OK) break;
            c->opt.wind_mode = GPLMM_WIND_CALLER;
            const double tb = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            rc = gplmm_newton_solve(c, nullptr, x, &st[k]);
            st[k].t_build_ms += tb;
            st[k].t_total_ms += tb;
            st[k].builds += 1;
        } else {
            rc = gplmm_newton_solve(c, nullptr, x, &st[k]);
        }
        c->opt.wind_mode = mode;
        if (rc != GPLMM_OK) break;
    }
    c->phys = full;
    c->opt.wind_mode = mode;
    return rc;
}

int gplmm_sample_residuals(gplmm_ctx* c, const double* x, const double* xprev, double* out) {
    if (!c || !x || !out) return GPLMM_E_ARG;
    if (!c->ready) return gp::fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    const int ns = (int)c->samples.size();
    std::vector<double> a(ns), b(ns);
    auto norms = [&](std::vector<double>& v) {
        if (c->csamp.empty()) v[0] = dot(c, c->d_tmp, c->d_tmp, c->N);
        else seg_sumsq(c, c->d_tmp, v.data());
        for (auto& t : v) t = std::sqrt(std::max(0.0, t));
    };
    launch_residual(c, c->d_zero, c->d_zero, c->d_tmp, c->stream);
    norms(a);
    launch_residual(c, x, xprev, c->d_tmp, c->stream);
    norms(b);
    GP_HIP(c, hipGetLastError());
    for (int s = 0; s < ns; ++s) out[s] = a[s] > 0 ? b[s] / a[s] : b[s];
    return GPLMM_OK;
}

int gplmm_set_progress(gplmm_ctx* c, gplmm_progress_fn fn, void* user) {
    if (!c) return GPLMM_E_ARG;
    c->progress = fn;
    c->progress_user = user;
    return GPLMM_OK;
}

int gplmm_set_timing(gplmm_ctx* c, int on) {
    if (!c) return GPLMM_E_ARG;
    c->timing = on != 0;
    return GPLMM_OK;
}

int gplmm_kernel_time(gplmm_ctx* c, const char* name, double* avg_ms, double* bytes) {
    if (!c || !name) return GPLMM_E_ARG;
    auto it = c->timers.find(name);
    if (it == c->timers.end()) return 0;
    hipStreamSynchronize(c->stream);
    Timer& t = it->second;
    size_t n = std::min(t.ev0.size(), t.ev1.size());
    double sum = 0.0, bsum = 0.0;
    for (size_t k = 0; k < n; ++k) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, t.ev0[k], t.ev1[k]);
        sum += ms;
        bsum += t.bytes[k];
    }
    if (avg_ms) *avg_ms = n ? sum / n : 0.0;
    if (bytes) *bytes = n ? bsum / n : 0.0;
    return (int)n;
}

void gplmm_reset_timers(gplmm_ctx* c) {
    if (!c) return;
    for (auto& kv : c->timers) {
        for (auto e : kv.second.ev0) hipEventDestroy(e);
        for (auto e : kv.second.ev1) hipEventDestroy(e);
    }
    c->timers.clear();
}

const char* gplmm_last_error(const gplmm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void gplmm_destroy(gplmm_ctx* c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    gplmm_reset_timers(c);
    if (c->apply_exec) (void)hipGraphExecDestroy(c->apply_exec);
    if (c->apply_graph) (void)hipGraphDestroy(c->apply_graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    void* ptrs[] = {c->d_co_pinned, c->d_panel, c->d_gin, c->d_gout, c->d_cl_row, c->d_cl_col, c->d_cl_feat, c->d_cl_pred, c->d_cl_scale, c->d_nb6, c->d_xcoef, c->d_xcoef_f, c->d_tag, c->d_sub_slots, c->d_subs, c->d_tfc, c->d_tfr, c->d_lrow,
                    c->d_urow, c->d_tlc, c->d_step_pairs[0], c->d_step_pairs[1], c->d_sub_list[0], c->d_sub_list[1],
                    c->d_step_pairs[2], c->d_sub_list[2], c->d_splits, c->d_phase_order[0], c->d_phase_order[1],
                    c->d_sep_ids, c->d_sinv_off, c->d_sinv_ncols, c->d_sinv, c->d_fsub_order,
                    c->d_factor, c->d_phi, c->d_phi_rhs, c->d_phi_off, c->d_phi_cols, c->d_phi_cols_off, c->d_prolong_blk, c->d_probe_e,
                    c->d_phi_ncols, c->d_grp_ptr, c->d_grp_slot, c->d_dinv_ptr, c->d_dinv, c->d_Ao, c->d_Aowork,
                    c->d_piv, c->d_probe, c->d_color_cols, c->d_flag, c->d_wind, c->d_r, c->d_tmp,
                    c->d_dx, c->d_zero, c->d_V, c->d_Z, c->d_red, c->d_pv, c->d_local, c->d_cv, c->d_row_sub,
                    c->d_sorted_slot, c->d_sorted_loc, c->d_slot_class, c->d_local_off, c->d_sub_ids,
                    c->d_noclose, c->d_Aoasm, c->d_sub_order[0], c->d_sub_order[1], c->d_co_blk, c->d_co_loc,
                    c->d_cblk_n, c->d_cblk_idx, c->d_cblk_ioff, c->d_cblk_moff, c->d_csamp, c->d_sphys, c->d_seg,
                    c->d_sscale, c->d_inv64, c->d_bres, c->d_bcoef, c->d_bsc, c->d_sub_samp, c->d_sact, c->d_alist};
    for (void* p : ptrs)
        if (p) hipFree(p);
    if (c->h_red) hipHostFree(c->h_red);
    if (c->h_bres) hipHostFree(c->h_bres);
    delete c;
}

}  // extern "C"

// Internal state of a gplmm context: host decomposition, device buffers and
// the launch helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "gplmm.h"

namespace gp {

constexpr int kMaxRestart = 1024;
constexpr int kMaxSamples = 1024;   // samples of one batch

struct Phys {
    double rho, mu, body[3], dt;   // dt <= 0: steady
};

constexpr uint8_t kPinBit = 0x80;   // tag bit of a pinned cell (one per sample)

// Geometry as the device kernels see it.
struct DevGeo {
    int nx, ny, nz, ndim, nrec;
    int per[3];
    int64_t ncell;
    int pin;                 // pinned cell of the first sample (the kernels test kPinBit)
    double h;
    const int32_t* nb6;      // cell * 6 + 2 d + t -> cell -/+ e_d (periodic wrap) or -1
    const uint8_t* tag;      // cell -> bit a: lower a-face carries no inertia in X; kPinBit: pinned
    const int32_t* csamp;    // cell -> sample of a batch, or nullptr for one sample
    const Phys* sphys;       // per-sample physics of a batch (indexed by csamp)
};

// Physics of a cell: its sample's in a batch, else the context's.
__host__ __device__ __forceinline__ const Phys& cell_phys(const DevGeo& g, const Phys& ph, int64_t c) {
    return g.csamp ? g.sphys[g.csamp[c]] : ph;
}

// One sample of a batch: its voxels, cells, primaries and interfaces are contiguous
// ranges starting at these offsets; the image dimensions place its voxels.
struct SampleGeo {
    int64_t voff, coff;
    int nx, ny, nz;
    int p0, i0;              // first primary, first interface
};

// One local problem (primary closure / primary block / dual block / split parts).
struct Sub {
    int kind;                // 0 primary (closure and Schwarz block), 1 dual, 2 half of a split
                             // primary with the separator appended, 3 separator of a split primary
    int id;                  // primary or interface id
    int n;                   // local unknowns
    int nT;                  // tiles per side
    int64_t slot_off;        // into sub_slots
    int64_t env_off;         // into env arrays (tfc, tfr, tlc, lrow, urow), nT entries each
    int64_t diag_off;        // element offset of the first diagonal tile in the factor buffer
    int sep0;                // kind 2: first local row of the separator (a multiple of the tile)
    int skip_ss;             // kind 2: 1 = the separator-separator block is not assembled here
    int split;               // index of the split that the subdomain belongs to, or -1
};

// A primary whose Schwarz block is solved by one level of nested dissection: the halves A
// and B (B in reverse order along the cut axis) each factorised with the separator S
// appended ([A, S] and [B, S], elimination stopped after the half), the separator's Schur
// complement S' = the sum of the two trailing blocks, factorised and inverted.
struct Split {
    int prim;
    int a_sub, b_sub, s_sub;
    int nA, nB, nS;
    int ld;                  // padded separator size (its tiles times the tile)
    int64_t inv_off;         // element offset of S'^-1 (column-major, ld x ld) in the inverse buffer
};

// Coarse probing: one colour = set of coarse columns whose restricted images do not overlap.
struct ProbeEntry {
    int32_t row, col;
};

struct Timer {
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<double> bytes;   // algorithmic bytes of each timed launch
};

}  // namespace gp

struct gplmm_ctx {
    gplmm_options opt;
    gp::Phys phys;
    int ndim = 2, nrec = 3;
    int nx = 0, ny = 0, nz = 0;
    int64_t nvox = 0, ncell = 0, N = 0, nface = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // ---- host decomposition
    std::vector<int32_t> cidx;        // voxel -> cell
    std::vector<int32_t> cell_voxel;  // cell -> voxel
    std::vector<int32_t> nbr;         // cell * 6 + 2*d + (s>0) -> cell or -1
    std::vector<int32_t> iface, prim; // per cell
    std::vector<int32_t> owner;       // per slot (see gplmm_get_maps)
    std::vector<int8_t> tagslot;      // per slot
    std::vector<uint8_t> noclose;     // per slot: face of a wall-free group (no closure sums)
    std::vector<uint8_t> tagcell;     // per cell bits
    int Np = 0, Nc = 0, Ny = 0;
    int64_t pin = 0;
    std::vector<gp::SampleGeo> samples; // one entry for a single image
    std::vector<gp::Phys> sphys;      // per-sample physics (batch)
    std::vector<int32_t> csamp;       // cell -> sample (batch only)
    std::vector<std::vector<int32_t>> Cp;          // interfaces of each primary
    std::vector<std::vector<int32_t>> icells;      // cells of each interface
    std::vector<std::vector<int32_t>> dual_cells;  // cells of each dual grid
    std::vector<int32_t> ycol;        // primary -> coarse y column (or -1)
    const int32_t* setup_groups = nullptr;   // interface groups during gplmm_setup_pnm only

    // ---- local problems
    int tile = 32;
    std::vector<gp::Sub> subs;        // [0, Np): primaries, [Np, Np + Nc): duals
    std::vector<int32_t> sub_slots;   // global slot of each local unknown, local order
    std::vector<int32_t> env_tfc, env_tfr;   // per tile row/col: first tile col/row of L/U
    std::vector<int32_t> env_tlc;            // per tile row: last tile column of U (inclusive)
    std::vector<int64_t> env_lrow, env_urow; // element offsets of the L and U tile rows
    int64_t factor_elems = 0;
    int maxT = 0;
    int maxT_set[2] = {0, 0};          // largest tile count among the primaries / the duals
    // LU schedule: per step K, (sub, I) pairs for the row-update kernel
    // set 0 = primaries' Schwarz blocks (split halves in place of split primaries, stopped
    // after the half), 1 = primaries' closures + duals, 2 = separators of split primaries
    std::vector<int64_t> lu_step_off[3];     // [set][K]
    std::vector<int32_t> lu_step_pairs[3];
    std::vector<int64_t> lu_sub_off[3];
    std::vector<int32_t> lu_sub_list[3];
    double lu_flops[3] = {0.0, 0.0, 0.0};   // flops of the tile products of each schedule (2 T^3 each)
    std::vector<gp::Split> splits;       // primaries solved by nested dissection
    int nsub_main = 0;                   // Np + Nc + Nf: the subdomains before the split parts
    int n_fsub = 0, maxT_f = 0;          // mg_form 1: blocks of A^f_f (components of the f-faces)
    int64_t f_row0 = 0, f_row1 = 0;      // their rows in the slot lists
    int32_t* d_fsub_order = nullptr;     // their subdomain ids, largest first
    int64_t sinv_elems = 0;              // separators' inverses, all splits
    int64_t split_apply_elems = 0;       // factor and inverse elements one primary solve reads
    int max_sep_ld = 0;                  // largest padded separator
    int n_phase1 = 0, n_phase3 = 0;      // split solves: unsplit primaries and halves / halves only
    int maxT_phase1 = 0, maxT_phase3 = 0;
    int64_t split_row0 = 0, split_row1 = 0;   // slot-list rows of the split parts
    gp::Split* d_splits = nullptr;
    int32_t* d_phase_order[2] = {nullptr, nullptr};   // phase 1 (largest first), phase 3
    int32_t* d_sep_ids = nullptr;        // the separators' subdomain ids
    int64_t* d_sinv_off = nullptr;       // per subdomain: offset of its inverse (separators)
    int32_t* d_sinv_ncols = nullptr;     // per subdomain: columns of its inverse (separators)
    void* d_sinv = nullptr;              // separators' inverses (real)

    // ---- shape vectors
    std::vector<int64_t> phi_off;     // per primary: element offset of its |S| x (|Cp|+1) block
    int64_t phi_elems = 0;
    std::vector<int32_t> phi_cols;    // per primary: coarse column of each shape column (concat)
    std::vector<int64_t> phi_cols_off;

    // ---- coarse operator probing
    int ncolors = 0;
    std::vector<int64_t> color_off;   // entries of colour c: [color_off[c], color_off[c+1])
    std::vector<gp::ProbeEntry> probe;
    std::vector<int64_t> color_col_off;
    std::vector<int32_t> color_cols;
    int nco = 0;                      // coarse size Nc + Ny
    // block-diagonal coarse storage: one dense block per sample, over the coarse indices
    // cblk_idx[cblk_ioff[b] .. cblk_ioff[b+1]) (row-major n_b x n_b at cblk_moff[b])
    std::vector<int32_t> cblk_n, cblk_idx, co_blk, co_loc;
    std::vector<int64_t> cblk_ioff, cblk_moff;
    int64_t co_elems = 0;             // sum of n_b^2
    int cblk_max = 0;

    // ---- device buffers
    gp::DevGeo geo{};
    int32_t* d_nb6 = nullptr;
    double* d_xcoef = nullptr;           // tabulated momentum rows of X, FP64
    float* d_xcoef_f = nullptr;          // the same in FP32 (FP32 preconditioner)
    uint8_t* d_tag = nullptr;
    int32_t* d_sub_slots = nullptr;      // local order, concatenated over subs
    int32_t* d_row_sub = nullptr;        // sub of each concatenated row
    int32_t* d_sorted_slot = nullptr;    // per sub: its slots ascending ...
    int32_t* d_sorted_loc = nullptr;     // ... and their local indices
    int32_t* d_slot_class = nullptr;     // per slot: owner primary, -1 f-face, -2 void, -4 interface cell
    uint8_t* d_noclose = nullptr;        // per slot: 1 = keep the plain row in the closure matrix
    int64_t* d_local_off = nullptr;      // per sub: offset of its padded local vector
    int32_t* d_sub_ids = nullptr;        // 0 .. Np+Nc-1
    gp::Sub* d_subs = nullptr;
    int32_t* d_tfc = nullptr;
    int32_t* d_tfr = nullptr;
    int64_t* d_lrow = nullptr;
    int64_t* d_urow = nullptr;
    int32_t* d_tlc = nullptr;
    int32_t* d_step_pairs[3] = {nullptr, nullptr, nullptr};
    int32_t* d_sub_list[3] = {nullptr, nullptr, nullptr};
    void* d_factor = nullptr;            // real (float or double) tiles
    double* d_inv64 = nullptr;           // per subdomain: FP64 inverses of the current LU step's diagonal tile
    int64_t prim_factor_elems = 0;       // primaries' tiles come first
    int64_t prim_rows = 0;               // primaries' rows come first in the slot lists
    void* d_phi = nullptr;               // real shape/correction vectors (column-major, ld = nT*T)
    void* d_phi_rhs = nullptr;           // their right-hand sides
    int max_phi_cols = 0;
    int64_t* d_phi_off = nullptr;
    int32_t* d_phi_ncols = nullptr;
    int32_t* d_phi_cols = nullptr;
    int64_t* d_phi_cols_off = nullptr;
    int32_t* d_prolong_blk = nullptr;    // prolongation workgroups: (primary, 256-row chunk) pairs
    double* d_probe_e = nullptr;         // probing: kProbeColors coarse indicator and image vectors
    int n_prolong_blk = 0, max_pcols = 0;
    int64_t* d_grp_ptr = nullptr;        // Rhat row groups: interfaces, then corrections
    int32_t* d_grp_slot = nullptr;
    int64_t* d_dinv_ptr = nullptr;       // per slot: local rows of the dual grids holding it
    int64_t* d_dinv = nullptr;
    int32_t* d_co_blk = nullptr;         // per coarse index: block, local index within it
    int32_t* d_co_loc = nullptr;
    int32_t* d_cblk_n = nullptr;
    int32_t* d_cblk_idx = nullptr;
    int64_t* d_cblk_ioff = nullptr;
    int64_t* d_cblk_moff = nullptr;
    int32_t* d_csamp = nullptr;          // batch: cell -> sample
    gp::Phys* d_sphys = nullptr;         // batch: per-sample physics
    int64_t* d_seg = nullptr;            // batch: slot offset of each sample (nsamples + 1)
    double* d_sscale = nullptr;          // batch: per-sample scale factors
    double* d_bres = nullptr;            // batch Arnoldi: per-sample dot products / norms
    double* h_bres = nullptr;            //   (pinned host mirror)
    double* d_bcoef = nullptr;           //   per-sample projection / combination coefficients
    double* d_bsc = nullptr;             //   per-sample (sj, 1/alpha)
    int32_t* d_sub_samp = nullptr;       // batch: sample of each subdomain
    uint8_t* d_sact = nullptr;           // batch: per-sample flag, 0 = skip its local solves
    int32_t* d_alist = nullptr;          // batch: samples still iterating in FGMRES
    double* d_Ao = nullptr;              // coarse operator blocks, then their inverses
    double* d_Aowork = nullptr;
    double* d_Aoasm = nullptr;           // the assembled coarse operator (kept for inspection)
    int32_t* d_piv = nullptr;
    gp::ProbeEntry* d_probe = nullptr;
    int32_t* d_color_cols = nullptr;
    int* d_flag = nullptr;               // breakdown flags
    // triangular solves: subdomains of each set (0 primaries, 1 duals), largest first
    int32_t* d_sub_order[2] = {nullptr, nullptr};

    // work vectors (FP64 unless noted)
    double* d_wind = nullptr;            // N
    double* d_r = nullptr;
    double* d_tmp = nullptr;
    double* d_dx = nullptr;
    double* d_zero = nullptr;
    double* d_V = nullptr;               // (m+1) x N
    double* d_Z = nullptr;               // m x N
    double* d_red = nullptr;             // reduction scratch
    double* h_red = nullptr;             // pinned host mirror
    void* d_pv = nullptr;                // preconditioner vectors (real): 6 x N
    void* d_local = nullptr;             // local solutions (real)
    double* d_cv = nullptr;              // coarse vectors (2 x nco)
    bool ready = false;
    bool built = false;
    // learned coarse operator: pattern (the probing entries), device staging, model
    gplmm_mlp* coarse_model = nullptr;
    std::vector<int32_t> cl_row, cl_col;
    int32_t* d_cl_row = nullptr;
    int32_t* d_cl_col = nullptr;
    float* d_cl_feat = nullptr;
    float* d_cl_pred = nullptr;
    float* d_cl_scale = nullptr;
    uint8_t* d_co_pinned = nullptr;      // coarse rows coupled to a primary holding a pinned cell
    bool last_coarse_learned = false;    // the last build took the learned coarse operator
    double last_coarse_ms = 0.0;         // coarse assembly time of the last build (host clock)
    // launch parameters chosen by gplmm_autotune (defaults until then)
    int red_blocks = 1024;               // blocks of the Krylov reductions (<= 2048)
    int stencil_block = 256;             // threads per block of the stencil kernels (<= 512)
    int trsv_mode = 2;                   // primary-solve variant (gplmm_tuning.trsv_mode)
    // graph of one preconditioner application (captured on first use, replayed after)
    hipGraph_t apply_graph = nullptr;
    hipGraphExec_t apply_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    double* d_gin = nullptr;
    double* d_gout = nullptr;
    bool graph_valid = false;
    double* d_panel = nullptr;            // coarse LU panel scratch (32 x nco)
    int builds = 0;
    int64_t gs_passes = 0, gs_reorth = 0;   // Gram-Schmidt steps, and those reorthogonalised
    double last_build_ms = 0.0;
    bool timing = false;
    double apply_bytes = 0.0, jv_bytes = 0.0;

    std::map<std::string, gp::Timer> timers;
    gplmm_progress_fn progress = nullptr;   // called after every Newton step and FGMRES cycle
    void* progress_user = nullptr;
    int progress_newton = 0;                // Newton step under way (for the FGMRES-cycle calls)
};

namespace gp {

int fail(gplmm_ctx* c, int code, const std::string& msg);
#define GP_HIP(ctx, call)                                                               \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return gp::fail(ctx, GPLMM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// setup.cpp
int build_decomposition(gplmm_ctx* c, const uint8_t* mask, const int32_t* labels);
int build_local_problems(gplmm_ctx* c);
int build_probing(gplmm_ctx* c);
void build_coarse_blocks(gplmm_ctx* c);
int merge_samples(gplmm_ctx* c, std::vector<gplmm_ctx*>& parts);

// stencil.hip
void launch_residual(gplmm_ctx* c, const double* x, const double* xprev, double* r, hipStream_t s,
                     bool tagged = false);
void launch_jv(gplmm_ctx* c, const double* xk, const double* v, double* y, hipStream_t s, bool tagged = false);
template <typename T>
void launch_xv(gplmm_ctx* c, const T* v, T* y, const T* sub_from, hipStream_t s);
void launch_xcoef(gplmm_ctx* c, hipStream_t s);
constexpr int kCoarseFeatures = 16;
int mlp_width_in(const gplmm_mlp* m);
int mlp_width_out(const gplmm_mlp* m);
int coarse_features(gplmm_ctx* c, const double* wind_host, std::vector<float>& feat, std::vector<float>& scale);
void launch_bB(gplmm_ctx* c, double* bB, hipStream_t s);
// y = Xcheck v: the primary and interface-cell rows of the column-summed build matrix (FP64)
void launch_xcheck_v(gplmm_ctx* c, const double* v, double* y, hipStream_t s);
// y = X v for kProbeColors vectors interleaved per slot (FP64, the tabulated rows read once)
constexpr int kProbeColors = 8;
void launch_xv_multi(gplmm_ctx* c, const double* v, double* y, hipStream_t s);

// krylov.hip
double dot(gplmm_ctx* c, const double* a, const double* b, int64_t n);
double nrm2(gplmm_ctx* c, const double* a, int64_t n);
void seg_sumsq(gplmm_ctx* c, const double* a, double* out_host);   // per-sample sums of squares
void seg_scale(gplmm_ctx* c, const double* scale_dev, double* a);   // a *= scale[sample] (in place)
void seg_dots2(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* y, const int32_t* alist, int na,
               double* a, double* b);
void seg_update2(gplmm_ctx* c, double* V, int64_t ldv, int j, const double* coef_host, int ldc,
                 const double* sc_host, const int32_t* alist, int na, double* w, double* nrm2);
void seg_lincomb(gplmm_ctx* c, const double* Z, int64_t ldz, int k, const double* y_host, int ldy, double* x);
void axpy(gplmm_ctx* c, double alpha, const double* x, double* y, int64_t n);
void scal_copy(gplmm_ctx* c, double alpha, const double* x, double* y, int64_t n);
template <typename A, typename B>
void convert(gplmm_ctx* c, const A* x, B* y, int64_t n);

// precond.hip
template <typename T>
int build_precond(gplmm_ctx* c);
template <typename T>
int apply_precond(gplmm_ctx* c, const double* v, double* z);

// coarse-scale solver pieces (precond.hip)
template <typename T>
int coarse_jacobian(gplmm_ctx* c, const double* xk);
void coarse_restrict(gplmm_ctx* c, const double* v, double* out);
template <typename T>
void coarse_update(gplmm_ctx* c, const double* rc, double* dc, double* tmp, double* x);

// coarse.hip
int coarse_invert(gplmm_ctx* c);

// timing (api.cpp)
void timer_begin(gplmm_ctx* c, const char* name);
void timer_end(gplmm_ctx* c, const char* name, double bytes);

}  // namespace gp

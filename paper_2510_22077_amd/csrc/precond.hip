// gPLMM build and apply on the device.
//
// Paper: M^-1 = M_G^-1 + M_L^-1 (I - A M_G^-1) with M_L = M_dp (Section 3.1);
// M_dp^-1 = M_d^-1 + M_p^-1 (I - A M_d^-1) (Section 3.2.3); the compact
// coarse form M_G^-1 = Phat (Rhat A Phat)^-1 Rhat with A itself in place of the
// column-summed operator (Section 3.2.2, Remark 1); A = X = J~_w for gPLMM
// (Section 4).  Phat puts the shape vectors phi_ij and correction vectors chi_i
// on each primary, the coarse pressure on each interface's cells and zero on
// the f-faces; Rhat sums over each interface's cells and over every row of
// each primary.
//
// The coarse operator Rhat X Phat is assembled by probing: the columns of one
// colour have restricted images on disjoint coarse rows, so one prolongation,
// one stencil application and one restriction of the colour's indicator give
// all of their entries.
#include <chrono>

#include "internal.h"

namespace gp {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
    __syncthreads();
    return s;
}

// coarse[g] = sum of v over the slots of row group g (interfaces: their cells' pressures;
// correction unknowns: every slot of the primary).
template <typename V>
__global__ void restrict_kernel(const V* __restrict__ v, const int64_t* __restrict__ gptr,
                                const int32_t* __restrict__ gslot, double* __restrict__ out) {
    __shared__ double sh[16];
    const int g = blockIdx.x;
    double acc = 0.0;
    const int64_t e = gptr[g + 1];
    int64_t t = gptr[g] + threadIdx.x;
    // four entries per pass, their index and value loads in flight together
    for (; t + 3 * (int64_t)blockDim.x < e; t += 4 * (int64_t)blockDim.x) {
        int32_t q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = gslot[t + u * (int64_t)blockDim.x];
        double w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = (double)v[q[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += w[u];
    }
    for (; t < e; t += blockDim.x) acc += (double)v[gslot[t]];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[g] = s;
}

// z on the primaries' slots: sum_k phi_k coef[col_k] over the primary's shape and
// correction vectors, one workgroup per 256-row chunk of one primary (blk: (primary,
// chunk) pairs): the primary's column indices and coefficients are read once per
// workgroup into LDS, and each thread issues its row's shape-vector loads eight at a
// time; the sum keeps the column order and skips zero coefficients.
template <typename T, typename O>
__global__ void __launch_bounds__(256) prolong_blk_kernel(const T* __restrict__ phi, const int64_t* __restrict__ phi_off,
                                                          const int64_t* __restrict__ pcol_off,
                                                          const int32_t* __restrict__ pcols,
                                                          const Sub* __restrict__ subs, const int32_t* __restrict__ blk,
                                                          const int32_t* __restrict__ slots,
                                                          const double* __restrict__ coef, O* __restrict__ z, int kT) {
    extern __shared__ double acoef[];
    const int i = blk[2 * blockIdx.x], chunk = blk[2 * blockIdx.x + 1];
    const Sub sb = subs[i];
    const int64_t c0 = pcol_off[i];
    const int nc = (int)(pcol_off[i + 1] - c0);
    for (int k = threadIdx.x; k < nc; k += blockDim.x) {
        const int32_t cl = pcols[c0 + k];
        acoef[k] = cl >= 0 ? coef[cl] : 0.0;
    }
    __syncthreads();
    const int r = chunk * 256 + (int)threadIdx.x;
    if (r >= sb.n) return;
    const int64_t ld = (int64_t)sb.nT * kT;
    const T* ph = phi + phi_off[i] + r;
    double acc = 0.0;
    int k = 0;
    for (; k + 8 <= nc; k += 8) {
        T p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = ph[(int64_t)(k + u) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (acoef[k + u] != 0.0) acc += acoef[k + u] * (double)p[u];
    }
    for (; k < nc; ++k)
        if (acoef[k] != 0.0) acc += acoef[k] * (double)ph[(int64_t)k * ld];
    z[slots[sb.slot_off + r]] = (O)acc;
}

// z on interface cells' pressures: the coarse pressure of their interface.
template <typename O>
__global__ void prolong_iface_kernel(const int64_t* __restrict__ gptr, const int32_t* __restrict__ gslot, int Nc,
                                     const double* __restrict__ coef, O* __restrict__ z) {
    const int j = blockIdx.x;
    if (j >= Nc) return;
    for (int64_t t = gptr[j] + threadIdx.x; t < gptr[j + 1]; t += blockDim.x) z[gslot[t]] = (O)coef[j];
}

// Probing K colours at once (K = 1, or K = kProbeColors with the colours of a slot
// interleaved: vector q of slot s at z[s K + q], nb <= K of them in use and the rest zero;
// coarse vectors at stride nco): the same sums as the single-vector prolongation and
// restriction for every colour, each in its own order, with the shared reads (shape
// vectors, slot lists) done once and every load unconditional.
template <typename T, int K>
__global__ void __launch_bounds__(256) prolong_blk_multi_kernel(const T* __restrict__ phi,
                                                                const int64_t* __restrict__ phi_off,
                                                                const int64_t* __restrict__ pcol_off,
                                                                const int32_t* __restrict__ pcols,
                                                                const Sub* __restrict__ subs,
                                                                const int32_t* __restrict__ blk,
                                                                const int32_t* __restrict__ slots,
                                                                const double* __restrict__ coef, int nco, int nb,
                                                                double* __restrict__ z, int kT) {
    extern __shared__ double acoefm[];   // [column][colour]
    const int i = blk[2 * blockIdx.x], chunk = blk[2 * blockIdx.x + 1];
    const Sub sb = subs[i];
    const int64_t c0 = pcol_off[i];
    const int nc = (int)(pcol_off[i + 1] - c0);
    for (int x = threadIdx.x; x < nc * K; x += blockDim.x) {
        const int k = x / K, q = x % K;
        const int32_t cl = pcols[c0 + k];
        acoefm[x] = (cl >= 0 && q < nb) ? coef[(int64_t)q * nco + cl] : 0.0;
    }
    __syncthreads();
    const int r = chunk * 256 + (int)threadIdx.x;
    if (r >= sb.n) return;
    const int64_t ld = (int64_t)sb.nT * kT;
    const T* ph = phi + phi_off[i] + r;
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    for (int k = 0; k < nc; ++k) {
        const double p = (double)ph[(int64_t)k * ld];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double a = acoefm[k * K + q];
            if (a != 0.0) acc[q] += a * p;
        }
    }
    const int64_t sl = slots[sb.slot_off + r];
#pragma unroll
    for (int q = 0; q < K; ++q) z[sl * K + q] = acc[q];
}

template <int K>
__global__ void prolong_iface_multi_kernel(const int64_t* __restrict__ gptr, const int32_t* __restrict__ gslot,
                                           int Nc, const double* __restrict__ coef, int nco, int nb,
                                           double* __restrict__ z) {
    const int j = blockIdx.x;
    if (j >= Nc) return;
    for (int64_t t = gptr[j] + threadIdx.x; t < gptr[j + 1]; t += blockDim.x) {
        const int64_t sl = gslot[t];
#pragma unroll
        for (int q = 0; q < K; ++q) z[sl * K + q] = q < nb ? coef[(int64_t)q * nco + j] : 0.0;
    }
}

template <int K>
__global__ void restrict_multi_kernel(const double* __restrict__ v, int nb, const int64_t* __restrict__ gptr,
                                      const int32_t* __restrict__ gslot, double* __restrict__ out, int nco) {
    __shared__ double sh[16][K];
    const int g = blockIdx.x;
    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;
    for (int64_t t = gptr[g] + threadIdx.x; t < gptr[g + 1]; t += blockDim.x) {
        const int64_t sl = gslot[t];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += v[sl * K + q];
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_down(acc[q], off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) sh[wv][q] = acc[q];
    __syncthreads();
    if ((int)threadIdx.x < nb) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w][threadIdx.x];
        out[(int64_t)threadIdx.x * nco + g] = t;
    }
}

// e_q = indicator of colour k0 + q's columns, for q < nb: the colours' entries are
// contiguous in the column (or probe-entry) list, colour k0 + q at [off[q], off[q + 1])
struct ColorSpan {
    int64_t off[kProbeColors + 1];
};

__global__ void set_ones_multi_kernel(const int32_t* __restrict__ cols, ColorSpan sp, int nb, double* __restrict__ e,
                                      int nco) {
    const int64_t k = sp.off[0] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= sp.off[nb]) return;
    int q = 0;
    while (k >= sp.off[q + 1]) ++q;
    e[(int64_t)q * nco + cols[k]] = 1.0;
}

// Block-diagonal coarse storage: one dense row-major block per sample over the coarse
// indices idx[ioff[b] .. ioff[b+1]); blk/loc give each coarse index's block and position.
struct CoBlk {
    const int32_t* blk;
    const int32_t* loc;
    const int32_t* n;
    const int32_t* idx;
    const int64_t* ioff;
    const int64_t* moff;
};

__device__ __forceinline__ int64_t co_pos(const CoBlk& cb, int row, int col) {
    const int b = cb.blk[row];
    return cb.moff[b] + (int64_t)cb.loc[row] * cb.n[b] + cb.loc[col];
}

// Ao[row, col] = t_q[row] for the (row, col) entries of colour k0 + q.
__global__ void probe_scatter_multi_kernel(const ProbeEntry* __restrict__ ent, ColorSpan sp, int nb,
                                           const double* __restrict__ t, int nco, double* __restrict__ Ao, CoBlk cb) {
    const int64_t k = sp.off[0] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= sp.off[nb]) return;
    int q = 0;
    while (k >= sp.off[q + 1]) ++q;
    const ProbeEntry p = ent[k];
    Ao[co_pos(cb, p.row, p.col)] = t[(int64_t)q * nco + p.row];
}

// zp[slot] = local solution (primaries are disjoint)
template <typename T>
__global__ void scatter_prim_kernel(const int32_t* __restrict__ slots, const int32_t* __restrict__ row_sub,
                                    const Sub* __restrict__ subs, const int64_t* __restrict__ local_off,
                                    const T* __restrict__ loc, T* __restrict__ z, int64_t nrows_prim) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows_prim) return;
    const int s = row_sub[t];
    if (subs[s].split >= 0) return;   // solved by its halves
    const int r = (int)(t - subs[s].slot_off);
    z[slots[t]] = loc[local_off[s] + r];
}

// zp[slot] = the halves' local solutions of the split primaries: the first half's rows
// ([x_A, x_S]) and the second half's own rows (x_B)
template <typename T>
__global__ void scatter_split_kernel(const int32_t* __restrict__ slots, const int32_t* __restrict__ row_sub,
                                     const Sub* __restrict__ subs, const int64_t* __restrict__ local_off,
                                     const T* __restrict__ loc, T* __restrict__ z, int64_t row0, int64_t row1) {
    const int64_t t = row0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= row1) return;
    const int s = row_sub[t];
    const Sub sb = subs[s];
    if (sb.kind != 2) return;
    const int r = (int)(t - sb.slot_off);
    if (sb.skip_ss && r >= sb.sep0) return;
    z[slots[t]] = loc[local_off[s] + r];
}

// z[slot] = local solution for the rows row0 .. row1 of the slot lists (disjoint blocks)
template <typename T>
__global__ void scatter_rows_kernel(const int32_t* __restrict__ slots, const int32_t* __restrict__ row_sub,
                                    const Sub* __restrict__ subs, const int64_t* __restrict__ local_off,
                                    const T* __restrict__ loc, T* __restrict__ z, int64_t row0, int64_t row1) {
    const int64_t t = row0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= row1) return;
    const int s = row_sub[t];
    z[slots[t]] = loc[local_off[s] + (t - subs[s].slot_off)];
}

// zd[slot] = sum over the dual grids containing the slot, in a fixed order
template <typename T>
__global__ void gather_dual_kernel(const int64_t* __restrict__ ptr, const int64_t* __restrict__ src,
                                   const T* __restrict__ loc, T* __restrict__ z, int64_t N) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    T acc = 0;
    for (int64_t k = ptr[s]; k < ptr[s + 1]; ++k) acc += loc[src[k]];
    z[s] = acc;
}

template <typename T>
__global__ void combine_kernel(const T* __restrict__ a, const T* __restrict__ b, const T* __restrict__ c,
                               double* __restrict__ z, int64_t N) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < N) z[s] = (double)a[s] + (double)b[s] + (double)c[s];
}

// y = A x for the block-diagonal coarse inverse, one workgroup per coarse row: the row
// of its sample's block against x gathered over the block's coarse indices.
__global__ void gemv_kernel(const double* __restrict__ A, CoBlk cb, const double* __restrict__ x,
                            double* __restrict__ y) {
    __shared__ double sh[16];
    const int i = blockIdx.x;
    const int b = cb.blk[i], n = cb.n[b];
    const double* a = A + cb.moff[b] + (int64_t)cb.loc[i] * n;
    const int32_t* idx = cb.idx + cb.ioff[b];
    double acc = 0.0;
    int j = threadIdx.x;
    // four entries per pass, their loads in flight together
    for (; j + 3 * (int)blockDim.x < n; j += 4 * (int)blockDim.x) {
        double av[4];
        int32_t iv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            av[u] = a[j + u * blockDim.x];
            iv[u] = idx[j + u * blockDim.x];
        }
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = x[iv[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += av[u] * xv[u];
    }
    for (; j < n; j += blockDim.x) acc += a[j] * x[idx[j]];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) y[i] = s;
}

// Ao[row, col] = sinh(prediction) * scale for the learned coarse entries
__global__ void learned_scatter_kernel(const int32_t* __restrict__ row, const int32_t* __restrict__ col,
                                       const float* __restrict__ pred, const float* __restrict__ scale, int64_t n,
                                       double* __restrict__ Ao, CoBlk cb) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    // predictions are clipped to asinh(+-4000): no entry of the normalised operator is larger
    const double z = fmin(fmax((double)pred[k], -9.0), 9.0);
    Ao[co_pos(cb, row[k], col[k])] = sinh(z) * (double)scale[k];
}

// Conservation structure of the learned coarse operator.  The shape vectors of a primary
// sum to a uniform pressure (partition of unity) wherever the primary holds no pinned
// cell, and X maps a uniform pressure to zero, so every coarse row not coupled to a pinned
// primary has zero sum over the interface columns.  Interface rows: the diagonal is set
// to minus the sum of the predicted off-diagonal interface entries; correction rows: the
// predicted interface entries are shifted equally to a zero sum.  One workgroup per
// coarse row of its sample's dense block; rows flagged in `pinned` keep the prediction.
__global__ void coarse_structure_kernel(double* __restrict__ Ao, CoBlk cb, int Nc, const uint8_t* __restrict__ pinned) {
    __shared__ double sh[16];
    __shared__ double shc[16];
    const int r = blockIdx.x;
    if (pinned[r]) return;
    const int b = cb.blk[r], n = cb.n[b];
    double* row = Ao + cb.moff[b] + (int64_t)cb.loc[r] * n;
    const int32_t* idx = cb.idx + cb.ioff[b];
    double acc = 0.0, cnt = 0.0;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        const int col = idx[l];
        if (col < Nc && col != r && row[l] != 0.0) {
            acc += row[l];
            cnt += 1.0;
        }
    }
    const double sum = block_sum(acc, sh);
    const double num = block_sum(cnt, shc);
    __shared__ double tot, m;
    if (threadIdx.x == 0) {
        tot = sum;
        m = num;
    }
    __syncthreads();
    if (r < Nc) {
        if (threadIdx.x == 0) row[cb.loc[r]] = -tot;
    } else if (m > 0.0) {
        const double shift = tot / m;
        for (int l = threadIdx.x; l < n; l += blockDim.x) {
            const int col = idx[l];
            if (col < Nc && row[l] != 0.0) row[l] -= shift;
        }
    }
}

template <typename T>
__global__ void zero_kernel(T* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// zero fill as a kernel (the application is captured in a graph, which gets no memset nodes)
template <typename T>
void zero_fill(gplmm_ctx* c, T* p, int64_t n) {
    if (n > 0) zero_kernel<T><<<nb(n), kB, 0, c->stream>>>(p, n);
}

}  // namespace

template <typename T>
void trsv_gather(gplmm_ctx* c, const int32_t* sub_ids_dev, int nsub, const T* vin, T* out_local);
template <typename T>
void trsv_phi(gplmm_ctx* c, int maxcols);
template <typename T>
int assemble_subs(gplmm_ctx* c, int first_sub, int nsub, bool closure);
template <typename T>
int factor_set(gplmm_ctx* c, int set);
template <typename T>
void trsv_split(gplmm_ctx* c, const T* vin, T* loc);
template <typename T>
void trsv_fblocks(gplmm_ctx* c, const T* vin, T* out_local);
template <typename T>
int build_separators(gplmm_ctx* c);

static CoBlk coblk(const gplmm_ctx* c) {
    return CoBlk{c->d_co_blk, c->d_co_loc, c->d_cblk_n, c->d_cblk_idx, c->d_cblk_ioff, c->d_cblk_moff};
}

template <typename T>
static T* pvec(gplmm_ctx* c, int k) {
    return (T*)c->d_pv + (int64_t)k * c->N;
}

// Phat coef (FP64 coarse vector) -> z (type O)
template <typename T, typename O>
static void prolong(gplmm_ctx* c, const double* coef, O* z) {
    zero_fill<O>(c, z, c->N);
    if (c->n_prolong_blk > 0)
        prolong_blk_kernel<T, O><<<c->n_prolong_blk, 256, sizeof(double) * std::max(c->max_pcols, 1), c->stream>>>(
            (const T*)c->d_phi, c->d_phi_off, c->d_phi_cols_off, c->d_phi_cols, c->d_subs, c->d_prolong_blk,
            c->d_sub_slots, coef, z, c->tile);
    if (c->Nc > 0)
        prolong_iface_kernel<O><<<c->Nc, 64, 0, c->stream>>>(c->d_grp_ptr, c->d_grp_slot, c->Nc, coef, z);
}

template <typename V>
static void restrict_(gplmm_ctx* c, const V* v, double* out) {
    if (c->nco > 0) restrict_kernel<V><<<c->nco, kB, 0, c->stream>>>(v, c->d_grp_ptr, c->d_grp_slot, out);
}

// Learned coarse entries: features from the current wind (host), network inference,
// scatter into the dense coarse operator.
static int learned_coarse(gplmm_ctx* c) {
    hipStream_t s = c->stream;
    std::vector<double> wh(c->N);
    GP_HIP(c, hipMemcpyAsync(wh.data(), c->d_wind, sizeof(double) * c->N, hipMemcpyDeviceToHost, s));
    GP_HIP(c, hipStreamSynchronize(s));
    std::vector<float> feat, scale;
    coarse_features(c, wh.data(), feat, scale);
    const int64_t ne = (int64_t)c->cl_row.size();
    if (!c->d_cl_row) {   // first learned build: device staging of the pattern
        const size_t n1 = (size_t)std::max<int64_t>(ne, 1);
        GP_HIP(c, hipMalloc((void**)&c->d_cl_row, sizeof(int32_t) * n1));
        GP_HIP(c, hipMalloc((void**)&c->d_cl_col, sizeof(int32_t) * n1));
        GP_HIP(c, hipMalloc((void**)&c->d_cl_feat, sizeof(float) * n1 * kCoarseFeatures));
        GP_HIP(c, hipMalloc((void**)&c->d_cl_pred, sizeof(float) * n1));
        GP_HIP(c, hipMalloc((void**)&c->d_cl_scale, sizeof(float) * n1));
        GP_HIP(c, hipMemcpy(c->d_cl_row, c->cl_row.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice));
        GP_HIP(c, hipMemcpy(c->d_cl_col, c->cl_col.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice));
    }
    GP_HIP(c, hipMemcpyAsync(c->d_cl_feat, feat.data(), sizeof(float) * feat.size(), hipMemcpyHostToDevice, s));
    GP_HIP(c, hipMemcpyAsync(c->d_cl_scale, scale.data(), sizeof(float) * ne, hipMemcpyHostToDevice, s));
    GP_HIP(c, hipStreamSynchronize(s));
    int rc = gplmm_mlp_forward(c->coarse_model, c->d_cl_feat, (int)ne, c->d_cl_pred);
    if (rc != GPLMM_OK) return fail(c, rc, "coarse model inference failed");
    GP_HIP(c, hipDeviceSynchronize());
    learned_scatter_kernel<<<nb(ne), kB, 0, s>>>(c->d_cl_row, c->d_cl_col, c->d_cl_pred, c->d_cl_scale, ne, c->d_Ao,
                                                 coblk(c));
    if (!c->d_co_pinned) {   // coarse rows coupled to a primary that holds a pinned cell
        std::vector<uint8_t> pin(c->nco, 0);
        for (int64_t q = 0; q < c->ncell; ++q) {
            if (!(c->tagcell[q] & kPinBit) || c->prim[q] < 0) continue;
            const int i = c->prim[q];
            if (c->ycol[i] >= 0) pin[c->ycol[i]] = 1;
            for (int32_t j : c->Cp[i]) pin[j] = 1;
        }
        GP_HIP(c, hipMalloc((void**)&c->d_co_pinned, std::max<size_t>(pin.size(), 1)));
        GP_HIP(c, hipMemcpy(c->d_co_pinned, pin.data(), pin.size(), hipMemcpyHostToDevice));
    }
    coarse_structure_kernel<<<c->nco, kB, 0, s>>>(c->d_Ao, coblk(c), c->Nc, c->d_co_pinned);
    GP_HIP(c, hipGetLastError());
    GP_HIP(c, hipStreamSynchronize(s));
    return GPLMM_OK;
}

// The coarse blocks <- Rhat A Phat by probing: the columns of one colour are prolonged
// together, A is applied, the result restricted and scattered into the entries of those
// columns.  K colours go through each pass side by side, interleaved per slot
// (mvm(pv, xv, nq) applies A to them); K = 1 is one plain vector per colour.  Scratch:
// the first 2K Krylov basis vectors, which hold nothing between FGMRES solves (the
// Newton residual and step vectors must survive a rebuild).
template <typename T, int K, typename MVM>
static void probe_coarse(gplmm_ctx* c, MVM mvm) {
    hipStream_t s = c->stream;
    const int nco = c->nco;
    const int64_t N = c->N;
    hipMemsetAsync(c->d_Ao, 0, sizeof(double) * c->co_elems, s);
    double* E = c->d_probe_e;
    double* tc = c->d_probe_e + (int64_t)kProbeColors * nco;
    double* pv = c->d_V;
    double* xv = c->d_V + (int64_t)K * N;
    for (int k0 = 0; k0 < c->ncolors; k0 += K) {
        const int nq = std::min(K, c->ncolors - k0);
        ColorSpan cs{}, ps{};
        for (int q = 0; q <= nq; ++q) {
            cs.off[q] = c->color_col_off[k0 + q];
            ps.off[q] = c->color_off[k0 + q];
        }
        zero_fill<double>(c, E, (int64_t)nq * nco);
        if (cs.off[nq] > cs.off[0])
            set_ones_multi_kernel<<<nb(cs.off[nq] - cs.off[0]), kB, 0, s>>>(c->d_color_cols, cs, nq, E, nco);
        zero_fill<double>(c, pv, (int64_t)K * N);
        if (c->n_prolong_blk > 0)
            prolong_blk_multi_kernel<T, K><<<c->n_prolong_blk, 256, sizeof(double) * K * std::max(c->max_pcols, 1), s>>>(
                (const T*)c->d_phi, c->d_phi_off, c->d_phi_cols_off, c->d_phi_cols, c->d_subs, c->d_prolong_blk,
                c->d_sub_slots, E, nco, nq, pv, c->tile);
        if (c->Nc > 0)
            prolong_iface_multi_kernel<K><<<c->Nc, 64, 0, s>>>(c->d_grp_ptr, c->d_grp_slot, c->Nc, E, nco, nq, pv);
        mvm(pv, xv, nq);
        if (nco > 0) restrict_multi_kernel<K><<<nco, kB, 0, s>>>(xv, nq, c->d_grp_ptr, c->d_grp_slot, tc, nco);
        if (ps.off[nq] > ps.off[0])
            probe_scatter_multi_kernel<<<nb(ps.off[nq] - ps.off[0]), kB, 0, s>>>(c->d_probe, ps, nq, tc, nco, c->d_Ao,
                                                                               coblk(c));
    }
}

// Coarse-scale solver (Section 5): the coarse Jacobian J_c = Rhat J~(xk) Phat, J~ the
// Jacobian of the residual without inertia on tagged faces, assembled with the probing
// colours of the coarse operator (with at least one tag layer every coupling J~ adds to
// X stays inside one primary, so the pattern is the same) and inverted in place.
template <typename T>
int coarse_jacobian(gplmm_ctx* c, const double* xk) {
    probe_coarse<T, 1>(c, [&](const double* pv, double* xv, int) { launch_jv(c, xk, pv, xv, c->stream, true); });
    return coarse_invert(c);
}

// out = Rhat v (FP64, nco entries).
void coarse_restrict(gplmm_ctx* c, const double* v, double* out) { restrict_<double>(c, v, out); }

// x <- x - Phat (J_c^-1 rc): the coarse Newton update with delta_c = -J_c^-1 r_c; the
// coarse inverse is in the coarse blocks, delta at dc (nco), the prolonged step at tmp (N).
template <typename T>
void coarse_update(gplmm_ctx* c, const double* rc, double* dc, double* tmp, double* x) {
    gemv_kernel<<<c->nco, kB, 0, c->stream>>>(c->d_Ao, coblk(c), rc, dc);
    prolong<T, double>(c, dc, tmp);
    axpy(c, -1.0, tmp, x, c->N);
}

template <typename T>
int build_precond(gplmm_ctx* c) {
    hipStream_t s = c->stream;
    T* F = (T*)c->d_factor;
    GP_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    // 1. closure matrices of the primaries and the dual blocks, factorised together
    timer_begin(c, "build_closure_dual_lu");
    GP_HIP(c, hipMemsetAsync(F, 0, sizeof(T) * c->factor_elems, s));
    assemble_subs<T>(c, 0, c->Np, true);
    assemble_subs<T>(c, c->Np, c->Nc, false);
    if (c->n_fsub > 0) assemble_subs<T>(c, c->Np + c->Nc, c->n_fsub, false);   // A^f_f (Eq. xf)
    factor_set<T>(c, 1);
    timer_end(c, "build_closure_dual_lu", c->lu_flops[1]);
    // 2. shape and correction vectors: Abar_i^-1 [g_i1 .. g_im, b_B]
    timer_begin(c, "build_shape");
    GP_HIP(c, hipMemcpyAsync(c->d_phi, c->d_phi_rhs, sizeof(T) * c->phi_elems, hipMemcpyDeviceToDevice, s));
    trsv_phi<T>(c, c->max_phi_cols);
    timer_end(c, "build_shape", 0.0);
    // 3. primary Schwarz blocks X[S_i, S_i] replace the closure factors
    timer_begin(c, "build_primary_lu");
    GP_HIP(c, hipMemsetAsync(F, 0, sizeof(T) * c->prim_factor_elems, s));
    assemble_subs<T>(c, 0, c->Np, false);
    const int nall = (int)c->subs.size();
    if (nall > c->nsub_main) {   // split primaries: both halves with the separator appended
        const int64_t e0 = c->subs[c->nsub_main].diag_off;
        GP_HIP(c, hipMemsetAsync(F + e0, 0, sizeof(T) * (c->factor_elems - e0), s));
        assemble_subs<T>(c, c->nsub_main, nall - c->nsub_main, false);
    }
    factor_set<T>(c, 0);
    build_separators<T>(c);
    timer_end(c, "build_primary_lu", c->lu_flops[0] + c->lu_flops[2]);
    int flag = 0;
    GP_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(c, hipStreamSynchronize(s));
    if (flag) return fail(c, GPLMM_E_BREAKDOWN, "zero or non-finite pivot in a local factorisation");
    // 4. coarse operator Rhat X Phat: predicted by the learned model when one is set (an
    //    operator that cannot be factorised falls back to the exact one), else by probing
    const int nco = c->nco;
    c->last_coarse_learned = false;
    auto tc0 = std::chrono::steady_clock::now();
    if (nco > 0 && c->coarse_model) {
        GP_HIP(c, hipMemsetAsync(c->d_Ao, 0, sizeof(double) * c->co_elems, s));
        int rc = learned_coarse(c);
        if (rc == GPLMM_OK) {
            c->last_coarse_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc0).count();
            rc = coarse_invert(c);
            if (rc == GPLMM_OK) {
                c->last_coarse_learned = true;
                GP_HIP(c, hipStreamSynchronize(s));
                c->built = true;
                c->builds++;
                return GPLMM_OK;
            }
        }
        if (rc != GPLMM_E_BREAKDOWN) return rc;
        c->err.clear();
        tc0 = std::chrono::steady_clock::now();
    }
    if (nco > 0) {
        timer_begin(c, "build_coarse");
        if (c->opt.mg_form == 1)   // Eq. iMG: Rhat Xcheck Phat
            probe_coarse<T, 1>(c, [&](const double* pv, double* xv, int) { launch_xcheck_v(c, pv, xv, s); });
        else if (c->opt.restart + 1 >= 2 * kProbeColors)
            probe_coarse<T, kProbeColors>(c, [&](const double* pv, double* xv, int) { launch_xv_multi(c, pv, xv, s); });
        else
            probe_coarse<T, 1>(c, [&](const double* pv, double* xv, int) { launch_xv<double>(c, pv, xv, nullptr, s); });
        GP_HIP(c, hipGetLastError());
        GP_HIP(c, hipStreamSynchronize(s));
        c->last_coarse_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tc0).count();
        int rc = coarse_invert(c);
        timer_end(c, "build_coarse", 0.0);
        if (rc != GPLMM_OK) return rc;
    }
    GP_HIP(c, hipStreamSynchronize(s));
    c->built = true;
    c->builds++;
    return GPLMM_OK;
}

template <typename T>
int apply_precond(gplmm_ctx* c, const double* v, double* z) {
    hipStream_t s = c->stream;
    const int64_t N = c->N;
    T* zG = pvec<T>(c, 0);
    T* vt = pvec<T>(c, 1);
    T* r1 = pvec<T>(c, 2);
    T* zd = pvec<T>(c, 3);
    T* r2 = pvec<T>(c, 4);
    T* zp = pvec<T>(c, 5);
    T* loc = (T*)c->d_local;
    // coarse correction z_G = Phat Ao^-1 Rhat v
    if (c->nco > 0) {
        restrict_<double>(c, v, c->d_cv);
        gemv_kernel<<<c->nco, kB, 0, s>>>(c->d_Ao, coblk(c), c->d_cv, c->d_cv + c->nco);
        prolong<T, T>(c, c->d_cv + c->nco, zG);
    } else {
        zero_fill<T>(c, zG, N);
    }
    const T* vin;
    if constexpr (sizeof(T) == sizeof(double)) {
        vin = (const T*)v;
    } else {
        convert<double, T>(c, v, vt, N);
        vin = vt;
    }
    // r1 = v - X z_G ; z_d = M_d^-1 r1 (overlapping duals, deterministic gather-sum)
    launch_xv<T>(c, zG, r1, vin, s);
    if (c->n_fsub > 0) {   // Eq. xf: z_G's f entries (zero so far) = (A^f_f)^-1 r1_f, then r1 again
        trsv_fblocks<T>(c, r1, loc);
        const int64_t nr = c->f_row1 - c->f_row0;
        scatter_rows_kernel<T><<<nb(nr), kB, 0, s>>>(c->d_sub_slots, c->d_row_sub, c->d_subs, c->d_local_off, loc, zG,
                                                     c->f_row0, c->f_row1);
        launch_xv<T>(c, zG, r1, vin, s);
    }
    if (c->Nc > 0) {
        trsv_gather<T>(c, c->d_sub_ids + c->Np, c->Nc, r1, loc);
        gather_dual_kernel<T><<<nb(N), kB, 0, s>>>(c->d_dinv_ptr, c->d_dinv, loc, zd, N);
    } else {
        zero_fill<T>(c, zd, N);
    }
    // r2 = r1 - X z_d ; z_p = M_p^-1 r2 (disjoint primaries)
    launch_xv<T>(c, zd, r2, r1, s);
    zero_fill<T>(c, zp, N);
    if (c->splits.empty()) {
        trsv_gather<T>(c, c->d_sub_ids, c->Np, r2, loc);
    } else {
        trsv_split<T>(c, r2, loc);
        const int64_t nr = c->split_row1 - c->split_row0;
        scatter_split_kernel<T><<<nb(nr), kB, 0, s>>>(c->d_sub_slots, c->d_row_sub, c->d_subs, c->d_local_off, loc, zp,
                                                      c->split_row0, c->split_row1);
    }
    scatter_prim_kernel<T><<<nb(c->prim_rows), kB, 0, s>>>(c->d_sub_slots, c->d_row_sub, c->d_subs, c->d_local_off,
                                                           loc, zp, c->prim_rows);
    combine_kernel<T><<<nb(N), kB, 0, s>>>(zG, zd, zp, z, N);
    return GPLMM_OK;
}

template int coarse_jacobian<float>(gplmm_ctx*, const double*);
template int coarse_jacobian<double>(gplmm_ctx*, const double*);
template void coarse_update<float>(gplmm_ctx*, const double*, double*, double*, double*);
template void coarse_update<double>(gplmm_ctx*, const double*, double*, double*, double*);
template int build_precond<float>(gplmm_ctx*);
template int build_precond<double>(gplmm_ctx*);
template int apply_precond<float>(gplmm_ctx*, const double*, double*);
template int apply_precond<double>(gplmm_ctx*, const double*, double*);

}  // namespace gp

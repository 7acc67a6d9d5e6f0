// Vector kernels for FGMRES: multi-vector dot products and updates for
// classical Gram-Schmidt (applied twice), norms, linear combinations and
// precision casts.  Reductions are two-pass with a fixed block count, so
// results do not depend on scheduling (bitwise reproducible run to run).
#include "internal.h"

namespace gp {

namespace {

constexpr int kMaxRedBlocks = 2048;   // scratch is sized for this many reduction blocks
constexpr int kThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // wavefront (64 lanes) shuffle reduction, then across the block's waves in LDS
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

// partial[j * nblk + b] = sum over block b's rows of V_j . w.  Vectors are taken eight at
// a time (eight independent streams in flight per thread, w read once per group),
// rows grid-strided, and the eight block sums reduced together.
constexpr int kGroup = 8;

__global__ void __launch_bounds__(kThreads) multidot_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                                            const double* __restrict__ w, int64_t n,
                                                            double* __restrict__ partial) {
    __shared__ double sh[kThreads / 64][kGroup];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < k; j0 += kGroup) {
        const int kk = min(kGroup, k - j0);
        const double* Vg = V + (int64_t)j0 * ldv;
        double acc[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) acc[q] = 0.0;
        for (int64_t r = r0; r < n; r += stride) {
            const double wr = w[r];
#pragma unroll
            for (int q = 0; q < kGroup; ++q)
                if (q < kk) acc[q] += Vg[(int64_t)q * ldv + r] * wr;
        }
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            double v = acc[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) sh[wv][q] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < kk) {
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < kThreads / 64; ++u) t += sh[u][threadIdx.x];
            partial[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// out[j] = sum_b partial[j * nblk + b]   (one block per j)
__global__ void reduce_kernel(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[(int64_t)j * nblk + b];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[j] = s;
}

// w -= sum_j V_j h_j ; optionally partial sums of w_new^2.  The coefficients sit in LDS;
// the k column reads of a row are independent loads, eight in flight at a time.
__global__ void __launch_bounds__(kThreads) update_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                                          const double* __restrict__ hcoef, double* __restrict__ w,
                                                          int64_t n, double* __restrict__ partial_nrm) {
    __shared__ double sh[16];
    __shared__ double hs[kMaxRestart + 2];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = hcoef[j];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        double x = w[r];
        int j = 0;
        for (; j + kGroup <= k; j += kGroup) {
            double t[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) t[q] = V[(int64_t)(j + q) * ldv + r];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) x -= t[q] * hs[j + q];
        }
        for (; j < k; ++j) x -= V[(int64_t)j * ldv + r] * hs[j];
        w[r] = x;
        acc += x * x;
    }
    if (partial_nrm) {
        double s = block_sum(acc, sh);
        if (threadIdx.x == 0) partial_nrm[blockIdx.x] = s;
    }
}

__global__ void axpy_kernel(double alpha, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += alpha * x[i];
}

__global__ void scal_copy_kernel(double alpha, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = alpha * x[i];
}

// Wave-wide sums of the 16 values a[0..8), b[0..8) of every lane, written to out[0..16)
// (a's sums first): a butterfly reduce-scatter (each exchange halves the values a lane
// keeps: 8 + 4 + 2 + 1 lane exchanges, then two plain ones) instead of a separate
// six-step tree per value.
__device__ __forceinline__ void wave_sums16(const double (&a)[kGroup], const double (&b)[kGroup], int lane,
                                            double* out) {
    static_assert(kGroup == 8, "the reduce-scatter is written for 16 values");
    double u8[8];
    const bool h32 = lane & 32;
#pragma unroll
    for (int i = 0; i < 8; ++i) {   // keep b (upper) on lanes with bit 5 set, a otherwise
        const double keep = h32 ? b[i] : a[i], send = h32 ? a[i] : b[i];
        u8[i] = keep + __shfl_xor(send, 32, 64);
    }
    double u4[4];
    const bool h16 = lane & 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = h16 ? u8[4 + i] : u8[i], send = h16 ? u8[i] : u8[4 + i];
        u4[i] = keep + __shfl_xor(send, 16, 64);
    }
    double u2[2];
    const bool h8 = lane & 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = h8 ? u4[2 + i] : u4[i], send = h8 ? u4[i] : u4[2 + i];
        u2[i] = keep + __shfl_xor(send, 8, 64);
    }
    const bool h4 = lane & 4;
    double v = (h4 ? u2[1] : u2[0]) + __shfl_xor(h4 ? u2[0] : u2[1], 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    // value index held: 8 h32 + 4 h16 + 2 h8 + h4 (a: 0..7, b: 8..15)
    if ((lane & 3) == 0) out[((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1)] = v;
}

// Delayed classical Gram-Schmidt (the reorthogonalisation of v_j is carried out in the
// step that projects w, so each Arnoldi step reads the basis twice): partial sums of
// V_i . x and V_i . y for i < k in one pass; partial[i * nblk + b] and
// partial[(k + i) * nblk + b].
__global__ void __launch_bounds__(kThreads) multidot2_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ y, int64_t n,
                                                             double* __restrict__ partial) {
    __shared__ double sh[kThreads / 64][2 * kGroup];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j0 = 0; j0 < k; j0 += kGroup) {
        const int kk = min(kGroup, k - j0);
        const double* Vg = V + (int64_t)j0 * ldv;
        double ax[kGroup], ay[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) ax[q] = ay[q] = 0.0;
        // two rows per trip through bounds-checked buffers (one per column, x and y: loads
        // past the end or of columns past k return zero), twenty loads in flight per thread
        // with one row offset each
        __amdgpu_buffer_rsrc_t rv[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q)
            rv[q] = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(Vg + (int64_t)q * ldv), 0,
                                                      q < kk ? (int)(n * 8) : 0, 0x00020000);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(x), 0, (int)(n * 8), 0x00020000);
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(y), 0, (int)(n * 8), 0x00020000);
        auto ld = [](__amdgpu_buffer_rsrc_t rs, int64_t row) {
            return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(row * 8), 0, 0));
        };
        for (int64_t r = r0; r < n; r += 2 * stride) {
            const int64_t r2 = r + stride;
            double v1[kGroup], v2[kGroup];
            const double x1 = ld(rx, r), y1 = ld(ry, r), x2 = ld(rx, r2), y2 = ld(ry, r2);
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                v1[q] = ld(rv[q], r);
                v2[q] = ld(rv[q], r2);
            }
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                ax[q] += v1[q] * x1;
                ay[q] += v1[q] * y1;
                ax[q] += v2[q] * x2;
                ay[q] += v2[q] * y2;
            }
        }
        wave_sums16(ax, ay, lane, sh[wv]);
        __syncthreads();
        if ((int)threadIdx.x < 2 * kk) {
            const int q = threadIdx.x < kk ? threadIdx.x : threadIdx.x - kk;
            const int col = threadIdx.x < kk ? q : kGroup + q;
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < kThreads / 64; ++u) t += sh[u][col];
            const int out = threadIdx.x < kk ? j0 + q : k + j0 + q;
            partial[(int64_t)out * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// One pass over V[0..j): v_j <- (v_j - sum_i V_i t_i) * ainv, then
// w <- w - sum_i V_i s_i - v_j sj, with partial sums of the new ||w||^2.
__global__ void __launch_bounds__(kThreads) update2_kernel(const double* __restrict__ V, int64_t ldv, int j,
                                                           const double* __restrict__ coef, double sj, double ainv,
                                                           double* __restrict__ vj, double* __restrict__ w,
                                                           int64_t n, double* __restrict__ partial_nrm) {
    __shared__ double sh[16];
    __shared__ double ts[kMaxRestart], ss[kMaxRestart];
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        ts[i] = coef[i];
        ss[i] = coef[kMaxRestart + i];
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
        double av = 0.0, aw = 0.0;
        int i = 0;
        for (; i + kGroup <= j; i += kGroup) {
            double t[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) t[q] = V[(int64_t)(i + q) * ldv + r];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                av += t[q] * ts[i + q];
                aw += t[q] * ss[i + q];
            }
        }
        for (; i < j; ++i) {
            const double t = V[(int64_t)i * ldv + r];
            av += t * ts[i];
            aw += t * ss[i];
        }
        const double vn = (vj[r] - av) * ainv;
        vj[r] = vn;
        const double wn = w[r] - aw - vn * sj;
        w[r] = wn;
        acc += wn * wn;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial_nrm[blockIdx.x] = t;
}

// Batches: the same Arnoldi kernels per sample, over the samples still iterating
// (alist): block (ch, y) strides over the slots [seg[s], seg[s+1]) of sample s = alist[y]
// (nch blocks per sample), so every sample keeps its own dot products, coefficients and
// norms.  partial[((y * 2k) + q) * nch + ch]: q < k dots with x = V[k-1], q >= k with y.
__global__ void __launch_bounds__(kThreads) seg_multidot2_kernel(const double* __restrict__ V, int64_t ldv, int k,
                                                                 const double* __restrict__ y,
                                                                 const int64_t* __restrict__ seg,
                                                                 const int32_t* __restrict__ alist,
                                                                 double* __restrict__ partial) {
    __shared__ double sh[kThreads / 64][2 * kGroup];
    const int s = alist[blockIdx.y], nch = gridDim.x, ys = blockIdx.y;
    const int64_t e = seg[s + 1];
    const int64_t stride = (int64_t)nch * blockDim.x;
    const int64_t r0 = seg[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double* x = V + (int64_t)(k - 1) * ldv;
    for (int j0 = 0; j0 < k; j0 += kGroup) {
        const int kk = min(kGroup, k - j0);
        const double* Vg = V + (int64_t)j0 * ldv;
        double ax[kGroup], ay[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) ax[q] = ay[q] = 0.0;
        for (int64_t r = r0; r < e; r += stride) {
            const double xr = x[r], yr = y[r];
#pragma unroll
            for (int q = 0; q < kGroup; ++q)
                if (q < kk) {
                    const double v = Vg[(int64_t)q * ldv + r];
                    ax[q] += v * xr;
                    ay[q] += v * yr;
                }
        }
        wave_sums16(ax, ay, lane, sh[wv]);
        __syncthreads();
        if ((int)threadIdx.x < 2 * kk) {
            const int q = threadIdx.x < kk ? threadIdx.x : threadIdx.x - kk;
            const int col = threadIdx.x < kk ? q : kGroup + q;
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < kThreads / 64; ++u) t += sh[u][col];
            const int out = threadIdx.x < kk ? j0 + q : k + j0 + q;
            partial[((int64_t)ys * 2 * k + out) * nch + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// Per sample s = alist[y]: v_j <- (v_j - V[0..j) t_s) ainv_s, w <- w - V[0..j) s_s - v_j sj_s;
// partial sums of the sample's new ||w||^2 at partial_nrm[y * nch + ch].  coef: per sample
// 2 * ldc values (t, then s at + ldc); sc: per sample (sj, ainv).
__global__ void __launch_bounds__(kThreads) seg_update2_kernel(const double* __restrict__ V, int64_t ldv, int j,
                                                               const double* __restrict__ coef, int ldc,
                                                               const double* __restrict__ sc,
                                                               double* __restrict__ vj, double* __restrict__ w,
                                                               const int64_t* __restrict__ seg,
                                                               const int32_t* __restrict__ alist,
                                                               double* __restrict__ partial_nrm) {
    __shared__ double sh[16];
    __shared__ double ts[kMaxRestart], ss[kMaxRestart];
    const int s = alist[blockIdx.y], nch = gridDim.x, ys = blockIdx.y;
    const double* cs = coef + (int64_t)s * 2 * ldc;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        ts[i] = cs[i];
        ss[i] = cs[ldc + i];
    }
    __syncthreads();
    const double sj = sc[2 * s], ainv = sc[2 * s + 1];
    const int64_t e = seg[s + 1];
    const int64_t stride = (int64_t)nch * blockDim.x;
    double acc = 0.0;
    for (int64_t r = seg[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < e; r += stride) {
        double av = 0.0, aw = 0.0;
        int i = 0;
        for (; i + kGroup <= j; i += kGroup) {
            double t[kGroup];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) t[q] = V[(int64_t)(i + q) * ldv + r];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                av += t[q] * ts[i + q];
                aw += t[q] * ss[i + q];
            }
        }
        for (; i < j; ++i) {
            const double t = V[(int64_t)i * ldv + r];
            av += t * ts[i];
            aw += t * ss[i];
        }
        const double vn = (vj[r] - av) * ainv;
        vj[r] = vn;
        const double wn = w[r] - aw - vn * sj;
        w[r] = wn;
        acc += wn * wn;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial_nrm[(int64_t)ys * nch + blockIdx.x] = t;
}

// x += sum_j Z_j y[sample][j] with per-sample coefficients (ldy per sample)
__global__ void seg_lincomb_kernel(const double* __restrict__ Z, int64_t ldz, int k, const double* __restrict__ y,
                                   int ldy, const int32_t* __restrict__ csamp, int nrec, double* __restrict__ x,
                                   int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* ys = y + (int64_t)csamp[i / nrec] * ldy;
    double s = x[i];
    for (int j = 0; j < k; ++j) s += Z[(int64_t)j * ldz + i] * ys[j];
    x[i] = s;
}

// x += sum_j Z_j y_j
__global__ void lincomb_kernel(const double* __restrict__ Z, int64_t ldz, int k, const double* __restrict__ y,
                               double* __restrict__ x, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = x[i];
    for (int j = 0; j < k; ++j) s += Z[(int64_t)j * ldz + i] * y[j];
    x[i] = s;
}

template <typename A, typename B>
__global__ void convert_kernel(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (B)x[i];
}

// Per-sample partial sums of squares: block (ch, s) strides over sample s's slots
// [seg[s], seg[s+1]); partial[s * gridDim.x + ch].
__global__ void __launch_bounds__(kThreads) seg_sumsq_kernel(const double* __restrict__ a,
                                                             const int64_t* __restrict__ seg,
                                                             double* __restrict__ partial) {
    __shared__ double sh[16];
    const int s = blockIdx.y;
    const int64_t e = seg[s + 1];
    double acc = 0.0;
    for (int64_t r = seg[s] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < e;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double v = a[r];
        acc += v * v;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// a[r] *= scale[sample of r's cell]
__global__ void seg_scale_kernel(const int32_t* __restrict__ csamp, int nrec, const double* __restrict__ scale,
                                 double* __restrict__ a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] *= scale[csamp[i / nrec]];
}

inline unsigned nb_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

// Device scratch layout in c->d_red: [0, kMaxRedBlocks * 2 (kMaxRestart + 2)) partials, then
// results: h (kMaxRestart + 2), h2 / the dots of V with w, norms, lincomb coefficients, then
// the coefficients of the delayed Gram-Schmidt update at 4 (kMaxRestart + 2).
constexpr int64_t kPart = (int64_t)kMaxRedBlocks * 2 * (kMaxRestart + 2);
constexpr int kRs = kMaxRestart + 2;
static double* partials(gplmm_ctx* c) { return c->d_red; }
static double* results(gplmm_ctx* c) { return c->d_red + kPart; }

double dot(gplmm_ctx* c, const double* a, const double* b, int64_t n) {
    multidot_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(a, 0, 1, b, n, partials(c));
    reduce_kernel<<<1, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, results(c));
    hipMemcpyAsync(c->h_red, results(c), sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    return c->h_red[0];
}

double nrm2(gplmm_ctx* c, const double* a, int64_t n) { return std::sqrt(std::max(0.0, dot(c, a, a, n))); }

void seg_sumsq(gplmm_ctx* c, const double* a, double* out_host) {
    constexpr int kChunks = 64;
    const int ns = (int)c->samples.size();
    seg_sumsq_kernel<<<dim3(kChunks, ns), kThreads, 0, c->stream>>>(a, c->d_seg, partials(c));
    reduce_kernel<<<ns, kThreads, 0, c->stream>>>(partials(c), kChunks, results(c));
    hipMemcpyAsync(c->h_red, results(c), sizeof(double) * ns, hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int s = 0; s < ns; ++s) out_host[s] = c->h_red[s];
}

void seg_scale(gplmm_ctx* c, const double* scale_dev, double* a) {
    seg_scale_kernel<<<nb_for(c->N), kThreads, 0, c->stream>>>(c->d_csamp, c->nrec, scale_dev, a, c->N);
}

void axpy(gplmm_ctx* c, double alpha, const double* x, double* y, int64_t n) {
    axpy_kernel<<<nb_for(n), kThreads, 0, c->stream>>>(alpha, x, y, n);
}

void scal_copy(gplmm_ctx* c, double alpha, const double* x, double* y, int64_t n) {
    scal_copy_kernel<<<nb_for(n), kThreads, 0, c->stream>>>(alpha, x, y, n);
}

// h = V[0..k)^T w into device results(c)[0..k) (no host sync)
static void multi_dot_dev(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* w, int64_t n,
                          double* out_dev) {
    multidot_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(V, ldv, k, w, n, partials(c));
    reduce_kernel<<<k, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, out_dev);
}

// Classical Gram-Schmidt with the Daniel-Gragg-Kaufman-Stewart reorthogonalisation
// test: h = V^T w and ||w||^2 in one pass over V (w must be the column after V's k
// columns, so the k + 1 dots include w.w), w <- w - V h with ||w||^2 fused; if the new
// norm dropped below 1/sqrt(2) of the old one (cancellation), a second projection
// h2 = V^T w, w <- w - V h2 follows and h += h2.  Returns h (k values) and ||w|| in
// hout[k] (host).  Passes over V: two, four when the test fires.
void cgs2(gplmm_ctx* c, const double* V, int64_t ldv, int k, double* w, int64_t n, double* hout) {
    double* r = results(c);
    double* h1 = r;
    double* h2 = r + (kMaxRestart + 2);
    double* nr = r + 2 * (kMaxRestart + 2);
    const bool fused = w == V + (int64_t)k * ldv;
    multi_dot_dev(c, V, ldv, fused ? k + 1 : k, w, n, h1);
    if (!fused) {
        multidot_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(w, 0, 1, w, n, partials(c));
        reduce_kernel<<<1, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, h1 + k);
    }
    update_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(V, ldv, k, h1, w, n, partials(c));
    reduce_kernel<<<1, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, nr);
    hipMemcpyAsync(c->h_red, h1, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(c->h_red + (kMaxRestart + 2), nr, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int j = 0; j < k; ++j) hout[j] = c->h_red[j];
    const double before = c->h_red[k];
    double after = c->h_red[kMaxRestart + 2];
    c->gs_passes++;
    if (!(after > 0.5 * before)) {
        multi_dot_dev(c, V, ldv, k, w, n, h2);
        update_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(V, ldv, k, h2, w, n, partials(c));
        reduce_kernel<<<1, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, nr);
        hipMemcpyAsync(c->h_red, h2, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream);
        hipMemcpyAsync(c->h_red + (kMaxRestart + 2), nr, sizeof(double), hipMemcpyDeviceToHost, c->stream);
        hipStreamSynchronize(c->stream);
        for (int j = 0; j < k; ++j) hout[j] += c->h_red[j];
        after = c->h_red[kMaxRestart + 2];
        c->gs_reorth++;
    }
    hout[k] = std::sqrt(std::max(0.0, after));
}

void lincomb(gplmm_ctx* c, const double* Z, int64_t ldz, int k, const double* y_host, double* x, int64_t n) {
    double* yd = results(c) + 3 * (kMaxRestart + 2);
    hipMemcpyAsync(yd, y_host, sizeof(double) * k, hipMemcpyHostToDevice, c->stream);
    lincomb_kernel<<<nb_for(n), kThreads, 0, c->stream>>>(Z, ldz, k, yd, x, n);
    hipStreamSynchronize(c->stream);
}

template <typename A, typename B>
void convert(gplmm_ctx* c, const A* x, B* y, int64_t n) {
    convert_kernel<A, B><<<nb_for(n), kThreads, 0, c->stream>>>(x, y, n);
}

template void convert<double, float>(gplmm_ctx*, const double*, float*, int64_t);
template void convert<float, double>(gplmm_ctx*, const float*, double*, int64_t);
template void convert<double, double>(gplmm_ctx*, const double*, double*, int64_t);

int64_t red_scratch_doubles() { return kPart + 8 * (int64_t)kRs + 64; }

// Dots of V[0..k) with x = V[k-1] (the vector being reorthogonalised) and with y, one pass:
// a[i] = V_i . x, b[i] = V_i . y (host).
void dots2(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* y, int64_t n, double* a, double* b) {
    const double* x = V + (int64_t)(k - 1) * ldv;
    multidot2_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(V, ldv, k, x, y, n, partials(c));
    reduce_kernel<<<2 * k, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, results(c));
    hipMemcpyAsync(c->h_red, results(c), sizeof(double) * 2 * k, hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int i = 0; i < k; ++i) {
        a[i] = c->h_red[i];
        b[i] = c->h_red[k + i];
    }
    c->gs_passes++;
}

// v_j <- (v_j - V[0..j) t) ainv, w <- w - V[0..j) s - v_j sj; returns ||w||^2.
double update2(gplmm_ctx* c, double* V, int64_t ldv, int j, const double* t, const double* s, double sj,
               double ainv, double* w, int64_t n) {
    double* coef = results(c) + 4 * (int64_t)kRs;   // t at [0, kMaxRestart), s at [kMaxRestart, 2 kMaxRestart)
    double* hc = c->h_red + 4 * kRs;
    for (int i = 0; i < j; ++i) {
        hc[i] = t[i];
        hc[kMaxRestart + i] = s[i];
    }
    if (j > 0) {
        hipMemcpyAsync(coef, hc, sizeof(double) * j, hipMemcpyHostToDevice, c->stream);
        hipMemcpyAsync(coef + kMaxRestart, hc + kMaxRestart, sizeof(double) * j, hipMemcpyHostToDevice, c->stream);
    }
    double* nr = results(c) + 6 * (int64_t)kRs;
    update2_kernel<<<c->red_blocks, kThreads, 0, c->stream>>>(V, ldv, j, coef, sj, ainv, V + (int64_t)j * ldv, w, n,
                                                             partials(c));
    reduce_kernel<<<1, kThreads, 0, c->stream>>>(partials(c), c->red_blocks, nr);
    hipMemcpyAsync(c->h_red + 2 * kRs, nr, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    c->gs_reorth++;
    return c->h_red[2 * kRs];
}


// ---- batches: per-sample Arnoldi (see fgmres_batch), over the active samples alist[0..na)
static int seg_chunks(int na, int rows_per_sample) {
    const int64_t cap = kPart / ((int64_t)std::max(na, 1) * std::max(rows_per_sample, 1));
    const int64_t want = (kMaxRedBlocks + na - 1) / std::max(na, 1);   // about kMaxRedBlocks blocks in all
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, cap));
}

static void push_alist(gplmm_ctx* c, const int32_t* alist, int na) {
    hipMemcpyAsync(c->d_alist, alist, sizeof(int32_t) * na, hipMemcpyHostToDevice, c->stream);
}

// a[y * k + i] = V_i . V[k-1], b[y * k + i] = V_i . w on sample alist[y] (host arrays of na * k)
void seg_dots2(gplmm_ctx* c, const double* V, int64_t ldv, int k, const double* y, const int32_t* alist, int na,
               double* a, double* b) {
    const int nch = seg_chunks(na, 2 * k);
    push_alist(c, alist, na);
    seg_multidot2_kernel<<<dim3(nch, na), kThreads, 0, c->stream>>>(V, ldv, k, y, c->d_seg, c->d_alist, partials(c));
    reduce_kernel<<<na * 2 * k, kThreads, 0, c->stream>>>(partials(c), nch, c->d_bres);
    hipMemcpyAsync(c->h_bres, c->d_bres, sizeof(double) * na * 2 * k, hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int q = 0; q < na; ++q)
        for (int i = 0; i < k; ++i) {
            a[(int64_t)q * k + i] = c->h_bres[(int64_t)q * 2 * k + i];
            b[(int64_t)q * k + i] = c->h_bres[(int64_t)q * 2 * k + k + i];
        }
    c->gs_passes++;
}

// per active sample s = alist[y]: v_j <- (v_j - V t_s) ainv_s, w <- w - V s_s - v_j sj_s;
// nrm2[y] = new ||w_s||^2.  coef_host: ns x 2 x ldc (t then s) and sc_host: ns x 2 (sj, ainv),
// both indexed by sample.
void seg_update2(gplmm_ctx* c, double* V, int64_t ldv, int j, const double* coef_host, int ldc, const double* sc_host,
                 const int32_t* alist, int na, double* w, double* nrm2) {
    const int ns = (int)c->samples.size();
    const int nch = seg_chunks(na, 1);
    push_alist(c, alist, na);
    if (j > 0) hipMemcpyAsync(c->d_bcoef, coef_host, sizeof(double) * ns * 2 * ldc, hipMemcpyHostToDevice, c->stream);
    hipMemcpyAsync(c->d_bsc, sc_host, sizeof(double) * ns * 2, hipMemcpyHostToDevice, c->stream);
    seg_update2_kernel<<<dim3(nch, na), kThreads, 0, c->stream>>>(V, ldv, j, c->d_bcoef, ldc, c->d_bsc,
                                                                 V + (int64_t)j * ldv, w, c->d_seg, c->d_alist,
                                                                 partials(c));
    reduce_kernel<<<na, kThreads, 0, c->stream>>>(partials(c), nch, c->d_bres);
    hipMemcpyAsync(c->h_bres, c->d_bres, sizeof(double) * na, hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int q = 0; q < na; ++q) nrm2[q] = c->h_bres[q];
    c->gs_reorth++;
}

// x += Z[0..k) y_s on each sample's slots (y_host: ns x ldy)
void seg_lincomb(gplmm_ctx* c, const double* Z, int64_t ldz, int k, const double* y_host, int ldy, double* x) {
    const int ns = (int)c->samples.size();
    hipMemcpyAsync(c->d_bcoef, y_host, sizeof(double) * ns * ldy, hipMemcpyHostToDevice, c->stream);
    seg_lincomb_kernel<<<nb_for(c->N), kThreads, 0, c->stream>>>(Z, ldz, k, c->d_bcoef, ldy, c->d_csamp, c->nrec, x,
                                                                c->N);
    hipStreamSynchronize(c->stream);
}

}  // namespace gp

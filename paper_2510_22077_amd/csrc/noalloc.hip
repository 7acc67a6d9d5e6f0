// Allocation-free variant of gplmm_sample_residuals for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops): the per-block
// partial sums live in a file-scope device array instead of context buffers, and the
// norms are written to a caller-owned device array, so the call makes no allocation, no
// host copy and no synchronisation.
//
// Each block of the partial kernel owns one slice of one sample's cells (grid-stride),
// evaluates the residual record of every cell at x and at the origin (Section 1; the
// normalisation ||r(u = 0, p = 0)|| of Section 8), and writes its two sums of squares to
// the scratch array; the finishing kernel adds a sample's partial sums in block order
// (deterministic) and writes ||r_s(x)|| / ||r_s(0)||.  Every scratch entry that is read
// is written earlier in the same call, so nothing needs clearing between calls; calls
// that overlap on one GPU share the array and race.
#include <mutex>

#include "internal.h"
#include "stencil_dev.h"

namespace gp {
namespace {

constexpr int kNaBlock = 256;
constexpr int kNaMaxBlocksPerSample = 1024;
constexpr int64_t kNaScratchDoubles = 131072;   // 1 MiB: two partial sums per (sample, block)
constexpr int kNaMaxDevices = 64;

__device__ __align__(256) double scratch[kNaScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kNaMaxDevices] = {};

// part[(s * nblk + b) * 2 + {0, 1}] = sum over block b's cells of sample s of
// |r(x)|^2 and |r(0)|^2.  seg: slot offsets of the samples (nullptr for one image).
template <int ND>
__global__ void __launch_bounds__(kNaBlock) resnorm_partial_kernel(DevGeo g, Phys ph, const double* __restrict__ x,
                                                                   const double* __restrict__ xold,
                                                                   const double* __restrict__ zero,
                                                                   const int64_t* __restrict__ seg, int nblk,
                                                                   double* __restrict__ part) {
    constexpr int nr = ND + 1;
    const int s = blockIdx.y;
    const int64_t c0 = seg ? seg[s] / nr : 0;
    const int64_t c1 = seg ? seg[s + 1] / nr : g.ncell;
    double sx = 0.0, s0 = 0.0;
    for (int64_t c = c0 + (int64_t)blockIdx.x * kNaBlock + threadIdx.x; c < c1; c += (int64_t)nblk * kNaBlock) {
        double rx[nr], r0[nr];
        residual_cell<ND>(g, ph, x, xold, c, rx);
        residual_cell<ND>(g, ph, zero, zero, c, r0);
#pragma unroll
        for (int a = 0; a < nr; ++a) {
            sx += rx[a] * rx[a];
            s0 += r0[a] * r0[a];
        }
    }
    // wave reduction (64 lanes), then the four waves of the block in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        s0 += __shfl_down(s0, off, 64);
    }
    __shared__ double red[2][kNaBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = sx;
        red[1][wave] = s0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kNaBlock / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        const int64_t k = ((int64_t)s * nblk + blockIdx.x) * 2;
        part[k] = a;
        part[k + 1] = b;
    }
}

// out[s] = ||r_s(x)|| / ||r_s(0)|| (||r_s(x)|| when the origin residual is zero).
__global__ void resnorm_finish_kernel(const double* __restrict__ part, int nblk, int ns, double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
        a += part[((int64_t)s * nblk + k) * 2];
        b += part[((int64_t)s * nblk + k) * 2 + 1];
    }
    const double nx = sqrt(a), n0 = sqrt(b);
    out[s] = n0 > 0.0 ? nx / n0 : nx;
}

// Device address of this GPU's copy of the scratch array (looked up once per device).
int scratch_for_current_device(gplmm_ctx* c, double** out) {
    int dev = 0;
    GP_HIP(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(c, GPLMM_E_ARG, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GP_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return GPLMM_OK;
}

}  // namespace
}  // namespace gp

using namespace gp;

extern "C" int gplmm_sample_residuals_noalloc(gplmm_ctx* c, const double* x, const double* xprev, double* out) {
    if (!c || !x || !out) return GPLMM_E_ARG;
    if (!c->ready) return fail(c, GPLMM_E_STATE, "no device state (host-only context)");
    const int ns = (int)c->samples.size();
    const int64_t per_sample = kNaScratchDoubles / (2 * (int64_t)std::max(ns, 1));
    if (per_sample < 1)
        return fail(c, GPLMM_E_ARG, "gplmm_sample_residuals_noalloc: " + std::to_string(ns) +
                                        " samples exceed the static scratch (" + std::to_string(kNaScratchDoubles / 2) +
                                        " samples at most)");
    const int nblk = (int)std::min<int64_t>(per_sample, kNaMaxBlocksPerSample);
    double* part = nullptr;
    int rc = scratch_for_current_device(c, &part);
    if (rc != GPLMM_OK) return rc;
    const int64_t* seg = c->csamp.empty() ? nullptr : c->d_seg;
    const dim3 grid((unsigned)nblk, (unsigned)ns);
    if (c->ndim == 3)
        resnorm_partial_kernel<3><<<grid, kNaBlock, 0, c->stream>>>(c->geo, c->phys, x, xprev, c->d_zero, seg, nblk, part);
    else
        resnorm_partial_kernel<2><<<grid, kNaBlock, 0, c->stream>>>(c->geo, c->phys, x, xprev, c->d_zero, seg, nblk, part);
    resnorm_finish_kernel<<<(ns + 255) / 256, 256, 0, c->stream>>>(part, nblk, ns, out);
    GP_HIP(c, hipGetLastError());
    return GPLMM_OK;
}

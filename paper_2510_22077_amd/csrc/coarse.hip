// Coarse system of the global preconditioner: Ao = Rhat X Phat (Remark 1 of
// Section 3.2.2), of size Nc + Ny, factorised in FP64 with partial pivoting and
// turned into an explicit inverse so that each application of M_G is one dense
// GEMV (the coarse system is small and ill-conditioned; the paper solves it
// directly at every application, Section 8's complexity discussion).
#include "internal.h"

namespace gp {

namespace {

constexpr int kB = 256;

// Pivot search in column k (rows k..n-1), row swap, column scaling.  One block.
__global__ void lu_pivot_kernel(double* __restrict__ A, int n, int k, int32_t* __restrict__ piv,
                                int* __restrict__ flag) {
    __shared__ double bv[kB];
    __shared__ int bi[kB];
    double best = -1.0;
    int bidx = k;
    for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
        double v = fabs(A[(int64_t)i * n + k]);
        if (v > best) {
            best = v;
            bidx = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            double o = bv[threadIdx.x + off];
            int oi = bi[threadIdx.x + off];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (threadIdx.x == 0) {
        piv[k] = p;
        if (!(bv[0] > 0.0) || !isfinite(bv[0])) atomicOr(flag, 2);
    }
    if (p != k)
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double t = A[(int64_t)k * n + j];
            A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
            A[(int64_t)p * n + j] = t;
        }
    __syncthreads();
    const double d = A[(int64_t)k * n + k];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[(int64_t)i * n + k] /= d;
}

// Trailing update A[i][j] -= A[i][k] A[k][j], i, j > k.
__global__ void lu_update_kernel(double* __restrict__ A, int n, int k) {
    const int j = k + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int i = k + 1 + blockIdx.y;
    if (j >= n || i >= n) return;
    A[(int64_t)i * n + j] -= A[(int64_t)i * n + k] * A[(int64_t)k * n + j];
}

// Inverse from P A = L U: column t of X solves L U x = P e_t.  One thread per column;
// L and U entries are read by all threads at once (broadcast), X rows are coalesced.
__global__ void lu_inverse_kernel(const double* __restrict__ LU, const int32_t* __restrict__ piv, int n,
                                  double* __restrict__ X) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    // b = P e_t: apply the recorded swaps to the unit vector
    int pos = t;
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (pos == k) pos = p;
        else if (pos == p) pos = k;
    }
    for (int i = 0; i < n; ++i) X[(int64_t)i * n + t] = (i == pos) ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i) {            // L y = b (unit lower)
        double s = X[(int64_t)i * n + t];
        for (int m = 0; m < i; ++m) s -= LU[(int64_t)i * n + m] * X[(int64_t)m * n + t];
        X[(int64_t)i * n + t] = s;
    }
    for (int i = n - 1; i >= 0; --i) {       // U x = y
        double s = X[(int64_t)i * n + t];
        for (int m = i + 1; m < n; ++m) s -= LU[(int64_t)i * n + m] * X[(int64_t)m * n + t];
        X[(int64_t)i * n + t] = s / LU[(int64_t)i * n + i];
    }
}

}  // namespace

int coarse_invert(gplmm_ctx* c) {
    const int n = c->nco;
    hipStream_t s = c->stream;
    double* A = c->d_Aowork;
    GP_HIP(c, hipMemcpyAsync(A, c->d_Ao, sizeof(double) * (int64_t)n * n, hipMemcpyDeviceToDevice, s));
    GP_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    for (int k = 0; k < n; ++k) {
        lu_pivot_kernel<<<1, kB, 0, s>>>(A, n, k, c->d_piv, c->d_flag);
        if (k + 1 < n) {
            dim3 grid((unsigned)((n - k - 1 + kB - 1) / kB), (unsigned)(n - k - 1));
            lu_update_kernel<<<grid, kB, 0, s>>>(A, n, k);
        }
    }
    lu_inverse_kernel<<<(n + 63) / 64, 64, 0, s>>>(A, c->d_piv, n, c->d_Ao);
    int flag = 0;
    GP_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(c, hipStreamSynchronize(s));
    if (flag) return fail(c, GPLMM_E_BREAKDOWN, "the coarse operator is singular");
    return GPLMM_OK;
}

}  // namespace gp

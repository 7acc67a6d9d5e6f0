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

// Position of the 1 in column t of P (P A = L U): the recorded swaps applied in order.
__global__ void perm_pos_kernel(const int32_t* __restrict__ piv, int n, int32_t* __restrict__ pos) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int p = t;
    for (int k = 0; k < n; ++k) {
        const int q = piv[k];
        if (p == k) p = q;
        else if (p == q) p = k;
    }
    pos[t] = p;
}

// Inverse from P A = L U, blocked: block b owns columns [32b, 32b + 32) of X and solves
// L U X = P I on them, 64 rows at a time (forward with unit L, then backward with U);
// the off-diagonal updates are 64 x 16 x 32 products staged through LDS.
constexpr int kIR = 64, kIC = 32, kIK = 16;

__global__ void __launch_bounds__(256) inverse_trsm_kernel(const double* __restrict__ LU,
                                                           const int32_t* __restrict__ pos, int n,
                                                           double* __restrict__ X) {
    __shared__ double At[kIR][kIC + 1];
    __shared__ double Lk[kIR][kIK + 1];
    __shared__ double Xk[kIK][kIC + 1];
    const int c0 = blockIdx.x * kIC;
    const int tid = threadIdx.x;
    const int tr = tid >> 3;          // 0..31: rows tr and tr + 32
    const int tc = (tid & 7) * 4;     // 4 columns
    const int nb = (n + kIR - 1) / kIR;
    // X = P I on the owned columns
    for (int x = tid; x < n * kIC; x += blockDim.x) {
        int i = x / kIC, t = c0 + x % kIC;
        if (t < n) X[(int64_t)i * n + t] = (pos[t] == i) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        const bool fwd = pass == 0;
        for (int bi = 0; bi < nb; ++bi) {
            const int I = fwd ? bi : nb - 1 - bi;
            const int r0 = I * kIR;
            double acc[2][4];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 4; ++b) {
                    int i = r0 + tr + 32 * a, t = c0 + tc + b;
                    acc[a][b] = (i < n && t < n) ? X[(int64_t)i * n + t] : 0.0;
                }
            // off-diagonal blocks: rows [0, r0) forward, [r0 + 64, n) backward
            const int k_lo = fwd ? 0 : r0 + kIR, k_hi = fwd ? r0 : n;
            for (int k0 = k_lo; k0 < k_hi; k0 += kIK) {
                __syncthreads();
                for (int x = tid; x < kIR * kIK; x += blockDim.x) {
                    int i = x / kIK, k = x % kIK;
                    int gi = r0 + i, gk = k0 + k;
                    Lk[i][k] = (gi < n && gk < k_hi) ? LU[(int64_t)gi * n + gk] : 0.0;
                }
                for (int x = tid; x < kIK * kIC; x += blockDim.x) {
                    int k = x / kIC, t = x % kIC;
                    int gk = k0 + k, gt = c0 + t;
                    Xk[k][t] = (gk < k_hi && gt < n) ? X[(int64_t)gk * n + gt] : 0.0;
                }
                __syncthreads();
#pragma unroll 4
                for (int k = 0; k < kIK; ++k) {
                    double l0 = Lk[tr][k], l1 = Lk[tr + 32][k];
                    for (int b = 0; b < 4; ++b) {
                        double xv = Xk[k][tc + b];
                        acc[0][b] -= l0 * xv;
                        acc[1][b] -= l1 * xv;
                    }
                }
            }
            __syncthreads();
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 4; ++b) At[tr + 32 * a][tc + b] = acc[a][b];
            // diagonal block: unit-lower forward or upper backward substitution, column-parallel
            __syncthreads();
            const int rows = min(kIR, n - r0);
            for (int st = 0; st < rows; ++st) {
                const int r = fwd ? st : rows - 1 - st;
                if (!fwd) {
                    if (tid < kIC) At[r][tid] /= LU[(int64_t)(r0 + r) * n + (r0 + r)];
                }
                __syncthreads();
                for (int x = tid; x < kIR * kIC; x += blockDim.x) {
                    int i = x / kIC, t = x % kIC;
                    bool below = fwd ? (i > r && i < rows) : (i < r);
                    if (below) At[i][t] -= LU[(int64_t)(r0 + i) * n + (r0 + r)] * At[r][t];
                }
                __syncthreads();
            }
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 4; ++b) {
                    int i = r0 + tr + 32 * a, t = c0 + tc + b;
                    if (i < n && t < n) X[(int64_t)i * n + t] = At[tr + 32 * a][tc + b];
                }
            __syncthreads();
        }
    }
}

}  // namespace

int coarse_invert(gplmm_ctx* c) {
    const int n = c->nco;
    hipStream_t s = c->stream;
    double* A = c->d_Aowork;
    GP_HIP(c, hipMemcpyAsync(A, c->d_Ao, sizeof(double) * (int64_t)n * n, hipMemcpyDeviceToDevice, s));
    GP_HIP(c, hipMemcpyAsync(c->d_Aoasm, c->d_Ao, sizeof(double) * (int64_t)n * n, hipMemcpyDeviceToDevice, s));
    GP_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    for (int k = 0; k < n; ++k) {
        lu_pivot_kernel<<<1, kB, 0, s>>>(A, n, k, c->d_piv, c->d_flag);
        if (k + 1 < n) {
            dim3 grid((unsigned)((n - k - 1 + kB - 1) / kB), (unsigned)(n - k - 1));
            lu_update_kernel<<<grid, kB, 0, s>>>(A, n, k);
        }
    }
    perm_pos_kernel<<<(n + 255) / 256, 256, 0, s>>>(c->d_piv, n, c->d_piv + n);
    inverse_trsm_kernel<<<(n + kIC - 1) / kIC, 256, 0, s>>>(A, c->d_piv + n, n, c->d_Ao);
    int flag = 0;
    GP_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(c, hipStreamSynchronize(s));
    if (flag) return fail(c, GPLMM_E_BREAKDOWN, "the coarse operator is singular");
    return GPLMM_OK;
}

}  // namespace gp

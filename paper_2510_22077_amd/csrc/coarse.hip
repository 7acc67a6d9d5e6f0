// Coarse system of the global preconditioner: Ao = Rhat X Phat (Remark 1 of
// Section 3.2.2), of size Nc + Ny, factorised in FP64 with partial pivoting and
// turned into an explicit inverse so that each application of M_G is one dense
// GEMV (the coarse system is small and ill-conditioned; the paper solves it
// directly at every application, Section 9.3's complexity discussion).
//
// Blocked right-looking LU with panels of 32 columns: the panel is factorised by
// one workgroup (pivot search, row interchange, rank-1 updates inside sub-panels of
// 8 columns and a rank-8 update of the rest of the panel after each), the
// interchanges are applied to the other columns, the block row of U is a
// unit-lower triangular solve, and the trailing matrix takes a rank-32 update (a
// tiled FP64 product).  The inverse U^-1 L^-1 P is formed by the same two
// kernels: a forward sweep (triangular solve of a block row, rank-32 update of the
// rows below) and a backward sweep with U.
#include "internal.h"

namespace gp {

namespace {

constexpr int kNB = 32;        // panel width
constexpr int kPT = 1024;      // panel workgroup
constexpr int kS = 8;          // sub-panel width inside a panel
constexpr int kBig = 128;      // columns (rows) per rank-kBig trailing update
constexpr int kGT = 64;        // update tile (kGT x kGT outputs, 256 threads, 4 x 4 each)
constexpr int kTr = 4;         // 32 x 32 blocks per pass of the register panel's transposes

// Factor columns [k0, k0 + w) of rows [k0, n) (row-major A, leading dimension n) through
// a column-major copy P (w columns of length n, so that every pass over the panel is a
// contiguous, coalesced sweep held in L2); pivot rows are chosen by largest magnitude,
// lowest index on ties.
__global__ void __launch_bounds__(kPT) panel_kernel(double* __restrict__ A, int n, int k0, int w,
                                                    int32_t* __restrict__ piv, int* __restrict__ flag,
                                                    double* __restrict__ P) {
    __shared__ double bv[kPT / 64];
    __shared__ int bi[kPT / 64];
    __shared__ double prow[kNB];
    __shared__ int pivot;
    __shared__ double tile[kNB][kNB + 1];
    __shared__ double Ub[kS][kNB];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // 32 x 32 blocks transposed through LDS: row segments read and panel columns written
    // with whole waves on contiguous addresses
    const int ty = tid >> 5, tx = tid & 31;
    for (int rb = k0; rb < n; rb += kNB) {
        const int r = rb + ty;
        tile[ty][tx] = (r < n && tx < w) ? A[(int64_t)r * n + k0 + tx] : 0.0;
        __syncthreads();
        const int rr = rb + tx;
        if (rr < n && ty < w) P[(int64_t)ty * n + rr] = tile[tx][ty];
        __syncthreads();
    }
    // sub-panels of kS columns: the rank-1 updates of a pivot step touch only the columns
    // of its sub-panel; then the sub-panel's rows of the remaining panel columns are
    // finished by forward substitution (a block of U) and every row below takes one
    // rank-kS update of those columns.  Each entry sees its updates in the same order as
    // with whole-panel rank-1 updates, at a fraction of the passes over the panel.
    for (int sb = 0; sb < w; sb += kS) {
        const int se = min(sb + kS, w);   // sub-panel columns [sb, se)
        for (int j = sb; j < se; ++j) {
            const int col = k0 + j;
            const double* pc = P + (int64_t)j * n;
            double best = -1.0;
            int bidx = n;
            // rows visited in increasing order: ties keep the lower index (four loads in flight)
            for (int r0 = col + tid; r0 < n; r0 += 4 * kPT) {
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = r0 + u * kPT;
                    v[u] = r < n ? fabs(pc[r]) : -1.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (v[u] > best) {
                        best = v[u];
                        bidx = r0 + u * kPT;
                    }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_down(best, off, 64);
                const int oi = __shfl_down(bidx, off, 64);
                if (ov > best || (ov == best && oi < bidx)) {
                    best = ov;
                    bidx = oi;
                }
            }
            if (lane == 0) {
                bv[wv] = best;
                bi[wv] = bidx;
            }
            __syncthreads();
            if (tid == 0) {
                double b = bv[0];
                int p = bi[0];
                for (int u = 1; u < kPT / 64; ++u)
                    if (bv[u] > b || (bv[u] == b && bi[u] < p)) {
                        b = bv[u];
                        p = bi[u];
                    }
                if (!(b > 0.0) || !isfinite(b) || p >= n) {
                    atomicOr(flag, 2);
                    p = col;
                }
                pivot = p;
                piv[col] = p;
            }
            __syncthreads();
            const int p = pivot;
            if (tid < w) {   // interchange across the whole panel; keep the pivot row
                double* q = P + (int64_t)tid * n;
                const double a = q[col], b = q[p];
                q[col] = b;
                q[p] = a;
                prow[tid] = b;
            }
            __syncthreads();
            const double d = prow[j];
            for (int r = col + 1 + tid; r < n; r += kPT) {
                const double l = P[(int64_t)j * n + r] / d;
                P[(int64_t)j * n + r] = l;
                for (int t = j + 1; t < se; ++t) P[(int64_t)t * n + r] -= l * prow[t];
            }
            __syncthreads();
        }
        if (se < w) {
            // U block: rows k0 + [sb, se) of columns [se, w) (unit-lower forward substitution)
            if (tid < w - se) {
                const int c = se + tid;
                double u[kS];
#pragma unroll
                for (int i = 0; i < kS; ++i) {
                    if (sb + i >= se) break;
                    double v = P[(int64_t)c * n + k0 + sb + i];
                    for (int t = 0; t < i; ++t) v -= P[(int64_t)(sb + t) * n + k0 + sb + i] * u[t];
                    u[i] = v;
                    P[(int64_t)c * n + k0 + sb + i] = v;
                    Ub[i][c] = v;
                }
            }
            __syncthreads();
            // rank-(se - sb) update of rows k0 + se .. n - 1 in columns [se, w), eight at a time
            const int ks = se - sb;
            for (int r = k0 + se + tid; r < n; r += kPT) {
                double l[kS];
#pragma unroll
                for (int t = 0; t < kS; ++t) l[t] = t < ks ? P[(int64_t)(sb + t) * n + r] : 0.0;
#pragma unroll 1
                for (int c0 = se; c0 < w; c0 += 8) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (c0 + u < w) v[u] = P[(int64_t)(c0 + u) * n + r];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (c0 + u < w) {
                            double acc = v[u];
#pragma unroll
                            for (int t = 0; t < kS; ++t)
                                if (t < ks) acc -= l[t] * Ub[t][c0 + u];
                            P[(int64_t)(c0 + u) * n + r] = acc;
                        }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int rb = k0; rb < n; rb += kNB) {
        const int rr = rb + tx;
        tile[tx][ty] = (rr < n && ty < w) ? P[(int64_t)ty * n + rr] : 0.0;
        __syncthreads();
        const int r = rb + ty;
        if (r < n && tx < w) A[(int64_t)r * n + k0 + tx] = tile[ty][tx];
        __syncthreads();
    }
}

// The factorisation of panel_kernel with each S-column sub-panel held in registers
// (S = kS: the same pivots and operations in the same order, so the same bits; S < kS
// where R kS values would not fit): thread t owns rows k0 + t + kPT q (q < R, so
// n - k0 <= R kPT) and reads them from the row-major matrix itself (each thread's S
// values of a row are contiguous; no column-major copy).  A pivot step touches no memory but the
// block's candidates and the two interchanged rows, which pass through LDS (two
// barriers); the sub-panel's interchanges reach the panel's other columns in one
// permutation of the few rows involved at its end.
template <int R, int S>
__global__ void __launch_bounds__(kPT) panel_reg_kernel(double* __restrict__ A, int n, int k0, int w,
                                                        int32_t* __restrict__ piv, int* __restrict__ flag,
                                                        double* __restrict__ P) {
    __shared__ double bv[kPT / 64];
    __shared__ int bi[kPT / 64];
    __shared__ double rowA[S], rowB[S];
    __shared__ int pvs[S];
    __shared__ int arow[2 * S], asrc[2 * S];
    __shared__ int na_s;
    __shared__ double xbuf[2 * S][kNB];
    __shared__ double tile[kTr][kNB][kNB + 1];
    __shared__ double Ub[S][kNB];
    __shared__ double Lb[S][S];
    constexpr int kC = R <= 3 ? 4 : 2;   // columns per pass of the rank update
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ty = tid >> 5, tx = tid & 31;
    // the panel into the column-major copy, kTr 32 x 32 blocks per pass through LDS
    for (int rb = k0; rb < n; rb += kTr * kNB) {
#pragma unroll
        for (int u = 0; u < kTr; ++u) {
            const int r = rb + u * kNB + ty;
            tile[u][ty][tx] = (r < n && tx < w) ? A[(int64_t)r * n + k0 + tx] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTr; ++u) {
            const int rr = rb + u * kNB + tx;
            if (rr < n && ty < w) P[(int64_t)ty * n + rr] = tile[u][tx][ty];
        }
        __syncthreads();
    }
    for (int sb = 0; sb < w; sb += S) {
        const int se = min(sb + S, w);
        double v[R][S];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = k0 + tid + kPT * q;
#pragma unroll
            for (int t = 0; t < S; ++t) v[q][t] = (r < n && sb + t < se) ? P[(int64_t)(sb + t) * n + r] : 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < S; ++jj) {
            if (sb + jj >= se) break;
            const int col = k0 + sb + jj;
            double best = -1.0;
            int bidx = n;
#pragma unroll
            for (int q = 0; q < R; ++q) {   // own rows in increasing order: ties keep the lower
                const int r = k0 + tid + kPT * q;
                if (r >= col && r < n) {
                    const double a = fabs(v[q][jj]);
                    if (a > best) {
                        best = a;
                        bidx = r;
                    }
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_down(best, off, 64);
                const int oi = __shfl_down(bidx, off, 64);
                if (ov > best || (ov == best && oi < bidx)) {
                    best = ov;
                    bidx = oi;
                }
            }
            if (lane == 0) {
                bv[wv] = best;
                bi[wv] = bidx;
            }
            __syncthreads();
            double b = bv[0];
            int p = bi[0];
            for (int u = 1; u < kPT / 64; ++u)
                if (bv[u] > b || (bv[u] == b && bi[u] < p)) {
                    b = bv[u];
                    p = bi[u];
                }
            const bool bad = !(b > 0.0) || !isfinite(b) || p >= n;
            if (bad) p = col;
            if (tid == 0) {
                if (bad) atomicOr(flag, 2);
                piv[col] = p;
                pvs[jj] = p;
            }
            // interchange rows col and p of the sub-panel through LDS; rowB is the pivot row
            const int oc = col - k0, op = p - k0;
            if (tid == oc % kPT) {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (q == oc / kPT)
#pragma unroll
                        for (int t = 0; t < S; ++t) rowA[t] = v[q][t];
            }
            if (tid == op % kPT) {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (q == op / kPT)
#pragma unroll
                        for (int t = 0; t < S; ++t) rowB[t] = v[q][t];
            }
            __syncthreads();
            if (p != col) {
                if (tid == oc % kPT) {
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        if (q == oc / kPT)
#pragma unroll
                            for (int t = 0; t < S; ++t) v[q][t] = rowB[t];
                }
                if (tid == op % kPT) {
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        if (q == op / kPT)
#pragma unroll
                            for (int t = 0; t < S; ++t) v[q][t] = rowA[t];
                }
            }
            const double d = rowB[jj];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = k0 + tid + kPT * q;
                if (r > col && r < n) {
                    const double l = v[q][jj] / d;
                    v[q][jj] = l;
#pragma unroll
                    for (int t = jj + 1; t < S; ++t)
                        if (sb + t < se) v[q][t] -= l * rowB[t];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = k0 + tid + kPT * q;
#pragma unroll
            for (int t = 0; t < S; ++t)
                if (r < n && sb + t < se) P[(int64_t)(sb + t) * n + r] = v[q][t];
        }
        // the multipliers of the sub-panel's own rows k0 + sb + i (thread sb + i, first slot)
        if (tid >= sb && tid < se) {
#pragma unroll
            for (int t = 0; t < S; ++t) Lb[tid - sb][t] = v[0][t];
        }
        // the sub-panel's interchanges, in order, on the panel's other columns: the rows they
        // touch and the row each one's final value comes from
        if (tid == 0) {
            int na = 0;
            for (int jj = 0; jj < se - sb; ++jj) {
                const int r1 = k0 + sb + jj, r2 = pvs[jj];
                int a1 = -1, a2 = -1;
                for (int a = 0; a < na; ++a) {
                    if (arow[a] == r1) a1 = a;
                    if (arow[a] == r2) a2 = a;
                }
                if (a1 < 0) {
                    arow[na] = r1;
                    asrc[na] = r1;
                    a1 = na++;
                }
                if (a2 < 0) {
                    arow[na] = r2;
                    asrc[na] = r2;
                    a2 = na++;
                }
                const int tsrc = asrc[a1];
                asrc[a1] = asrc[a2];
                asrc[a2] = tsrc;
            }
            na_s = na;
        }
        __syncthreads();
        const int na = na_s;
        for (int x = tid; x < na * w; x += kPT) {
            const int a = x / w, cc = x % w;
            if (cc < sb || cc >= se) xbuf[a][cc] = P[(int64_t)cc * n + asrc[a]];
        }
        __syncthreads();
        for (int x = tid; x < na * w; x += kPT) {
            const int a = x / w, cc = x % w;
            if (cc < sb || cc >= se) P[(int64_t)cc * n + arow[a]] = xbuf[a][cc];
        }
        __syncthreads();
        if (se < w) {
            // U block: rows k0 + [sb, se) of columns [se, w) (unit-lower forward substitution,
            // the column's entries loaded together)
            if (tid < w - se) {
                const int c = se + tid;
                double u[S];
#pragma unroll
                for (int i = 0; i < S; ++i) u[i] = sb + i < se ? P[(int64_t)c * n + k0 + sb + i] : 0.0;
#pragma unroll
                for (int i = 0; i < S; ++i) {
                    if (sb + i >= se) break;
                    double x = u[i];
#pragma unroll
                    for (int t = 0; t < i; ++t) x -= Lb[i][t] * u[t];
                    u[i] = x;
                    P[(int64_t)c * n + k0 + sb + i] = x;
                    Ub[i][c] = x;
                }
            }
            __syncthreads();
            // rank-(se - sb) update of the rows below in columns [se, w), kC columns per pass,
            // every held row's loads of a pass in flight together; the multipliers are the
            // held values of the sub-panel
            const int ks = se - sb;
            for (int c0 = se; c0 < w; c0 += kC) {
                double x[R][kC];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = k0 + tid + kPT * q;
#pragma unroll
                    for (int u = 0; u < kC; ++u)
                        x[q][u] = (r >= k0 + se && r < n && c0 + u < w) ? P[(int64_t)(c0 + u) * n + r] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = k0 + tid + kPT * q;
                    if (r < k0 + se || r >= n) continue;
#pragma unroll
                    for (int u = 0; u < kC; ++u)
                        if (c0 + u < w) {
                            double acc = x[q][u];
#pragma unroll
                            for (int t = 0; t < S; ++t)
                                if (t < ks) acc -= v[q][t] * Ub[t][c0 + u];
                            P[(int64_t)(c0 + u) * n + r] = acc;
                        }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int rb = k0; rb < n; rb += kTr * kNB) {
#pragma unroll
        for (int u = 0; u < kTr; ++u) {
            const int rr = rb + u * kNB + tx;
            tile[u][tx][ty] = (rr < n && ty < w) ? P[(int64_t)ty * n + rr] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kTr; ++u) {
            const int r = rb + u * kNB + ty;
            if (r < n && tx < w) A[(int64_t)r * n + k0 + tx] = tile[u][ty][tx];
        }
        __syncthreads();
    }
}

// Apply the interchanges of rows k0 .. k0 + w - 1 (in order) to every column outside
// [k0, k0 + w), one thread per column.
__global__ void swap_kernel(double* __restrict__ A, int n, int k0, int w, const int32_t* __restrict__ piv) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || (c >= k0 && c < k0 + w)) return;
    for (int j = 0; j < w; ++j) {
        const int r = k0 + j, p = piv[r];
        if (p != r) {
            const double t = A[(int64_t)r * n + c];
            A[(int64_t)r * n + c] = A[(int64_t)p * n + c];
            A[(int64_t)p * n + c] = t;
        }
    }
}

// Triangular solve of the w-row block starting at row k0 of B (leading dimension ldb),
// for columns [c0, c1), with the w x w diagonal block of the factor F (leading
// dimension n) at (k0, k0): lower = 1: unit lower (L), lower = 0: upper with diagonal (U).
__global__ void __launch_bounds__(256) block_trsm_kernel(const double* __restrict__ F, int n, int k0, int w,
                                                         double* __restrict__ B, int64_t ldb, int c0, int c1,
                                                         int lower) {
    __shared__ double T[kNB][kNB + 1];
    for (int x = threadIdx.x; x < kNB * kNB; x += blockDim.x) {
        const int i = x / kNB, j = x % kNB;
        T[i][j] = (i < w && j < w) ? F[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
    }
    __syncthreads();
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    double x[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i) x[i] = i < w ? B[(int64_t)(k0 + i) * ldb + c] : 0.0;
    if (lower) {
#pragma unroll
        for (int i = 0; i < kNB; ++i) {
            double v = x[i];
#pragma unroll
            for (int s = 0; s < i; ++s) v -= T[i][s] * x[s];
            x[i] = v;
        }
    } else {
#pragma unroll
        for (int i = kNB - 1; i >= 0; --i) {
            if (i >= w) continue;
            double v = x[i];
#pragma unroll
            for (int s = i + 1; s < kNB; ++s)
                if (s < w) v -= T[i][s] * x[s];
            x[i] = v / T[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < kNB; ++i)
        if (i < w) B[(int64_t)(k0 + i) * ldb + c] = x[i];
}

// C[r0 + i][c0 + j] -= sum_{t < w} L[r0 + i][kc + t] * B[kb + t][c0 + j], i < M, j < N
// (any rank w: taken kNB columns at a time, C read and written once).
// L has leading dimension n, B and C leading dimension ldb (C aliases B).  64 x 64 output
// tiles, 256 threads, 4 x 4 outputs per thread; operand tiles staged in LDS.
__global__ void __launch_bounds__(256) rank_update_kernel(const double* __restrict__ L, int n, int kc,
                                                          const double* B, int64_t ldb, int kb, double* C,
                                                          int r0, int M, int c0, int N, int w) {
    __shared__ double La[kGT][kNB + 1];
    __shared__ double Bb[kNB][kGT + 1];
    const int ti = blockIdx.y * kGT, tj = blockIdx.x * kGT;
    const int tid = threadIdx.x;
    const int ty = tid / 16, tx = tid % 16;
    double acc[4][4] = {};
    // the rank w in chunks of kNB (operands through LDS), one read-modify-write of C
    for (int t0 = 0; t0 < w; t0 += kNB) {
        const int wc = min(kNB, w - t0);
        __syncthreads();
        for (int x = tid; x < kGT * kNB; x += 256) {
            const int i = x / kNB, t = x % kNB;
            La[i][t] = (ti + i < M && t < wc) ? L[(int64_t)(r0 + ti + i) * n + kc + t0 + t] : 0.0;
        }
        for (int x = tid; x < kNB * kGT; x += 256) {
            const int t = x / kGT, j = x % kGT;
            Bb[t][j] = (t < wc && tj + j < N) ? B[(int64_t)(kb + t0 + t) * ldb + c0 + tj + j] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int t = 0; t < kNB; ++t) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = La[ty + 16 * u][t];
                b[u] = Bb[t][tx + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = ti + ty + 16 * u;
        if (i >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = tj + tx + 16 * v;
            if (j < N) C[(int64_t)(r0 + i) * ldb + c0 + j] -= acc[u][v];
        }
    }
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

// X = P I: X[i][t] = (pos[t] == i)
__global__ void perm_matrix_kernel(const int32_t* __restrict__ pos, int n, double* __restrict__ X) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)n * n) return;
    const int i = (int)(x / n), t = (int)(x % n);
    X[x] = pos[t] == i ? 1.0 : 0.0;
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// Invert one dense block in place: A (n x n, row-major) is overwritten by its LU factors and
// X receives the inverse.
static void invert_block(gplmm_ctx* c, double* A, double* X, int n) {
    hipStream_t s = c->stream;
    // LU with partial pivoting in blocks of kBig columns: the panels of a block update
    // only the block's own columns as they go; the block's rows of the columns to its
    // right are then solved with the block's unit-lower factor, and the trailing matrix
    // takes one rank-kBig update
    for (int K0 = 0; K0 < n; K0 += kBig) {
        const int K1 = std::min(K0 + kBig, n);
        for (int k0 = K0; k0 < K1; k0 += kNB) {
            const int w = std::min(kNB, K1 - k0);
            switch ((n - k0 + kPT - 1) / kPT) {   // rows per thread of the register-held variant
                case 1: panel_reg_kernel<1, kS><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                case 2: panel_reg_kernel<2, kS><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                case 3: panel_reg_kernel<3, kS><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                case 4: panel_reg_kernel<4, 4><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                case 5: panel_reg_kernel<5, 4><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                case 6: panel_reg_kernel<6, 4><<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel); break;
                default: panel_kernel<<<1, kPT, 0, s>>>(A, n, k0, w, c->d_piv, c->d_flag, c->d_panel);
            }
            swap_kernel<<<blocks(n, 256), 256, 0, s>>>(A, n, k0, w, c->d_piv);
            const int r = k0 + w;
            if (r < K1) {
                block_trsm_kernel<<<blocks(K1 - r, 256), 256, 0, s>>>(A, n, k0, w, A, n, r, K1, 1);
                rank_update_kernel<<<dim3(blocks(K1 - r, kGT), blocks(n - r, kGT)), 256, 0, s>>>(
                    A, n, k0, A, n, k0, A, r, n - r, r, K1 - r, w);
            }
        }
        if (K1 < n) {
            for (int k0 = K0; k0 < K1; k0 += kNB) {
                const int w = std::min(kNB, K1 - k0);
                block_trsm_kernel<<<blocks(n - K1, 256), 256, 0, s>>>(A, n, k0, w, A, n, K1, n, 1);
                const int r = k0 + w;
                if (r < K1)
                    rank_update_kernel<<<dim3(blocks(n - K1, kGT), blocks(K1 - r, kGT)), 256, 0, s>>>(
                        A, n, k0, A, n, k0, A, r, K1 - r, K1, n - K1, w);
            }
            rank_update_kernel<<<dim3(blocks(n - K1, kGT), blocks(n - K1, kGT)), 256, 0, s>>>(
                A, n, K0, A, n, K0, A, K1, n - K1, K1, n - K1, K1 - K0);
        }
    }
    // inverse: X = P I, then L^-1 (forward sweep), then U^-1 (backward sweep), both in
    // blocks of kBig rows with one rank-kBig update of the rows beyond each block
    perm_pos_kernel<<<blocks(n, 256), 256, 0, s>>>(c->d_piv, n, c->d_piv + n);
    perm_matrix_kernel<<<blocks((int64_t)n * n, 256), 256, 0, s>>>(c->d_piv + n, n, X);
    for (int K0 = 0; K0 < n; K0 += kBig) {
        const int K1 = std::min(K0 + kBig, n);
        for (int k0 = K0; k0 < K1; k0 += kNB) {
            const int w = std::min(kNB, K1 - k0);
            block_trsm_kernel<<<blocks(n, 256), 256, 0, s>>>(A, n, k0, w, X, n, 0, n, 1);
            const int r = k0 + w;
            if (r < K1)
                rank_update_kernel<<<dim3(blocks(n, kGT), blocks(K1 - r, kGT)), 256, 0, s>>>(A, n, k0, X, n, k0, X, r,
                                                                                          K1 - r, 0, n, w);
        }
        if (K1 < n)
            rank_update_kernel<<<dim3(blocks(n, kGT), blocks(n - K1, kGT)), 256, 0, s>>>(A, n, K0, X, n, K0, X, K1,
                                                                                      n - K1, 0, n, K1 - K0);
    }
    for (int K0 = ((n - 1) / kBig) * kBig; K0 >= 0; K0 -= kBig) {
        const int K1 = std::min(K0 + kBig, n);
        for (int k0 = K0 + ((K1 - 1 - K0) / kNB) * kNB; k0 >= K0; k0 -= kNB) {
            const int w = std::min(kNB, K1 - k0);
            block_trsm_kernel<<<blocks(n, 256), 256, 0, s>>>(A, n, k0, w, X, n, 0, n, 0);
            if (k0 > K0)
                rank_update_kernel<<<dim3(blocks(n, kGT), blocks(k0 - K0, kGT)), 256, 0, s>>>(A, n, k0, X, n, k0, X, K0,
                                                                                           k0 - K0, 0, n, w);
        }
        if (K0 > 0)
            rank_update_kernel<<<dim3(blocks(n, kGT), blocks(K0, kGT)), 256, 0, s>>>(A, n, K0, X, n, K0, X, 0, K0, 0,
                                                                                  n, K1 - K0);
    }
}

// The coarse operator is block diagonal (one block per sample of a batch, one block for a
// single image): each block is factorised and inverted on its own.
int coarse_invert(gplmm_ctx* c) {
    hipStream_t s = c->stream;
    const int64_t ne = c->co_elems;
    timer_begin(c, "coarse_inv");
    GP_HIP(c, hipMemcpyAsync(c->d_Aowork, c->d_Ao, sizeof(double) * ne, hipMemcpyDeviceToDevice, s));
    GP_HIP(c, hipMemcpyAsync(c->d_Aoasm, c->d_Ao, sizeof(double) * ne, hipMemcpyDeviceToDevice, s));
    GP_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), s));
    for (size_t b = 0; b < c->cblk_n.size(); ++b) {
        const int n = c->cblk_n[b];
        if (n > 0) invert_block(c, c->d_Aowork + c->cblk_moff[b], c->d_Ao + c->cblk_moff[b], n);
    }
    timer_end(c, "coarse_inv", 0.0);
    int flag = 0;
    GP_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(c, hipStreamSynchronize(s));
    if (flag) return fail(c, GPLMM_E_BREAKDOWN, "the coarse operator is singular");
    return GPLMM_OK;
}

}  // namespace gp

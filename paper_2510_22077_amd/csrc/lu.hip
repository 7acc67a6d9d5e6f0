// Batched local problems of the preconditioner: assembly, no-pivot LU and
// triangular solves on a tile skyline.
//
// Paper: the closure matrices Abar_i of the primaries (Section 3.2.2, the two
// reduction steps) and the additive-Schwarz blocks of the primary and dual
// grids (Section 3.2.3) are factorised once and reused for every right-hand
// side (the paper pre-factorises its local systems with LU).
//
// Layout: each local matrix (n x n, unknowns in the pressure-after-faces
// raster order) is cut into T x T tiles.  Lower tiles (I, J), J < I, exist for
// J >= tfc[I]; upper tiles (I, J), I < J, exist for I >= tfr[J], i.e. for
// J <= tlc[I]; both are stored tile-row by tile-row (L row I: columns tfc[I]..
// I-1, U row I: columns I+1..tlc[I]), so a substitution streams each factor
// as one contiguous range.  tfc and tfr are non-decreasing, so fill-in of an
// LU without pivoting stays inside (the envelope property).  Tiles are
// row-major.  Pivoting is not needed in this
// order: every pressure follows all of its faces, so each leading block is a
// saddle-point matrix with a positive-real velocity block and a full-rank
// divergence block.
#include "internal.h"
#include "stencil_dev.h"

namespace gp {

constexpr int kT = 32;
constexpr int kTT = kT * kT;

struct Env {
    const Sub* subs;
    const int32_t* tfc;
    const int32_t* tfr;
    const int32_t* tlc;
    const int64_t* lrow;
    const int64_t* urow;
    const int32_t* sub_samp;   // batch: sample of each subdomain (nullptr for one image)
    const uint8_t* sact;       // batch: 0 for a sample whose Krylov process has finished
    const Split* splits;       // primaries solved by nested dissection
};

// A subdomain of a finished sample of a batch: its right-hand side is zero, so is its
// solution; the block writes the zeros and leaves.
__device__ __forceinline__ bool skip_solve(const Env& e, int s) { return e.sub_samp && !e.sact[e.sub_samp[s]]; }

template <typename T>
__device__ __forceinline__ T* tile_ptr(T* F, const Env& e, const Sub& sb, int I, int J) {
    if (I == J) return F + sb.diag_off + (int64_t)I * kTT;
    if (J < I) return F + e.lrow[sb.env_off + I] + (int64_t)(J - e.tfc[sb.env_off + I]) * kTT;
    return F + e.urow[sb.env_off + I] + (int64_t)(J - I - 1) * kTT;
}

// ---------------------------------------------------------------------------------------
// Assembly: one thread per local row; the row of X = J~_w comes from the tabulated
// momentum coefficients (or the mass / pin row), its columns are located in the
// subdomain through the sorted slot list.  closure != 0 (primaries only): entries in
// columns of f-faces or of other primaries' unknowns are added to the diagonal
// (Section 3.2.2, both reduction steps), except on rows of wall-free faces.
// ---------------------------------------------------------------------------------------
template <int ND, typename T, bool kJac>
__global__ void assemble_kernel(DevGeo g, const double* __restrict__ coef, Env e, T* __restrict__ F,
                                const int32_t* __restrict__ row_sub, const int32_t* __restrict__ slots,
                                const int32_t* __restrict__ sorted_slot, const int32_t* __restrict__ sorted_loc,
                                const int32_t* __restrict__ slot_class, const uint8_t* __restrict__ noclose,
                                int64_t nrows, int first_sub, int nsub, int closure) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows) return;
    const int s = row_sub[t];
    if (s < first_sub || s >= first_sub + nsub) return;
    constexpr int nr = ND + 1;
    const Sub sb = e.subs[s];
    if (sb.kind == 3) return;   // separators: formed from the halves' trailing blocks
    const int r = (int)(t - sb.slot_off);
    // a half assembled without the separator-separator block (the other half holds it)
    const int sep_skip = sb.skip_ss && r >= sb.sep0 ? sb.sep0 : sb.n;
    const int64_t gs = slots[t];
    const int64_t c = gs / nr;
    const int comp = (int)(gs % nr);
    if (noclose[gs]) closure = 0;
    double diag_extra = 0.0;
    const int32_t* ss = sorted_slot + sb.slot_off;
    const int32_t* sl = sorted_loc + sb.slot_off;
    auto emit = [&](int64_t col64, double val) {
        const int32_t col = (int32_t)col64;
        int lo = 0, hi = sb.n;   // binary search in the subdomain's sorted slots
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ss[mid] < col) lo = mid + 1; else hi = mid;
        }
        if (lo < sb.n && ss[lo] == col) {
            const int lc = sl[lo];
            if (lc >= sep_skip) return;
            T* tp = tile_ptr(F, e, sb, r / kT, lc / kT);
            tp[(r % kT) * kT + (lc % kT)] += (T)val;
        } else if (closure) {
            const int32_t cls = slot_class[col];
            if (cls == -1 || (cls >= 0 && cls != sb.id)) diag_extra += val;
        }
    };
    const Nb<ND> nc = load_nb<ND>(g, c);
    const double ih = 1.0 / g.h;
    const int64_t nce = g.ncell;
    if (comp < ND) {
        const int a = comp;
        const int32_t L = nc.n[a][0];
        if (L >= 0) {
            const Nb<ND> nl = load_nb<ND>(g, L);
            const FaceNb<ND> f = face_nb(nc, nl, a);
            emit(gs, coef[a * nce + c]);
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (f.kind[d][q] == kActive) emit((int64_t)nr * f.P[d][q] + a, coef[((1 + 2 * d + q) * ND + a) * nce + c]);
            emit(nr * c + ND, ih);
            emit((int64_t)nr * L + ND, -ih);
            if (kJac) {   // transverse couplings of the Newton Jacobian
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    if (d == a) continue;
                    const int dd = d < a ? d : d - 1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double w = coef[((1 + 2 * ND + 4 * dd + q) * ND + a) * nce + c];
                        if (w != 0.0) emit((int64_t)nr * jac_col_cell<ND>(nc, nl, c, L, d, q) + d, w);
                    }
                }
            }
        }
    } else if ((g.tag[c] & kPinBit)) {
        emit(gs, 1.0);
    } else {
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            if (nc.n[a][0] >= 0) emit(nr * c + a, ih);
            if (nc.n[a][1] >= 0) emit((int64_t)nr * nc.n[a][1] + a, -ih);
        }
    }
    if (diag_extra != 0.0) {
        T* tp = tile_ptr(F, e, sb, r / kT, r / kT);
        tp[(r % kT) * kT + (r % kT)] += (T)diag_extra;
    }
}

// Identity on the padding rows of the last diagonal tile.
template <typename T>
__global__ void pad_kernel(Env e, T* F, int first_sub, int nsub) {
    int s = first_sub + blockIdx.x;
    if (s >= first_sub + nsub) return;
    const Sub sb = e.subs[s];
    const int I = sb.nT - 1;
    T* tp = F + sb.diag_off + (int64_t)I * kTT;
    for (int r = sb.n - I * kT + threadIdx.x; r < kT; r += blockDim.x) tp[r * kT + r] = (T)1;
}

// ---------------------------------------------------------------------------------------
// Tile products on the matrix cores (FP32 factors).  v_mfma_f32_32x32x2f32 takes, in lane
// l, A[l % 32][k] and B[k][l % 32] with k = l / 32, and accumulates the 32 x 32 product
// into 16 registers per lane: register v of lane l holds C[8 (v / 4) + 4 (l / 32) + v % 4]
// [l % 32].  Sixteen such steps (k = 2 s + l / 32, s = 0..15) make one 32 x 32 x 32 product.
// ---------------------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int mrow(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__device__ __forceinline__ f32x16 mfma_tile(f32x16 acc, const float (&a)[16], const float (&b)[16]) {
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b[s], acc, 0, 0, 0);
    return acc;
}

// b[s] = B[2 s + l / 32][l % 32] of a row-major tile in global memory (coalesced rows)
__device__ __forceinline__ void load_b(float (&b)[16], const float* tile, int lane) {
#pragma unroll
    for (int s = 0; s < 16; ++s) b[s] = tile[(2 * s + (lane >> 5)) * kT + (lane & 31)];
}

// ---------------------------------------------------------------------------------------
// LU step K, part 1 (one block per active subdomain): factor the diagonal tile in FP64,
// store its packed inverses (inv(L_KK) strictly below the diagonal, unit diagonal
// implied; inv(U_KK) on and above it: the form the triangular solves use), and form the
// U panel U_KJ = inv(L_KK) A_KJ.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) lu_diag_kernel(Env e, T* __restrict__ F, const int32_t* __restrict__ list,
                                                      int K, int* __restrict__ flag, double* __restrict__ inv64) {
    __shared__ double A[kT][kT + 1];
    __shared__ double X[kT][kT + 1];
    __shared__ double W[kT][kT + 1];
    const int sub = list[blockIdx.x];
    const Sub sb = e.subs[sub];
    const int tid = threadIdx.x;
    T* dp = F + sb.diag_off + (int64_t)K * kTT;
    for (int x = tid; x < kTT; x += blockDim.x) A[x / kT][x % kT] = (double)dp[x];
    __syncthreads();
    // one barrier per elimination step: every thread forms the multipliers of its own
    // rows (the same division), and the multipliers are kept in X until the end, since
    // column k of A is still read during step k.  The block is 256 threads: each takes
    // its four entries of a step together
    static_assert(kTT % 256 == 0, "four entries per thread");
    for (int k = 0; k < kT; ++k) {
        const double piv = A[k][k];
        if (tid == 0 && (!(piv == piv) || piv == 0.0 || fabs(piv) > 1e300)) atomicOr(flag, 1);
#pragma unroll
        for (int u = 0; u < kTT / 256; ++u) {
            const int x = tid + 256 * u;
            const int i = x / kT, j = x % kT;
            if (i > k && j >= k) {
                const double l = A[i][k] / piv;
                if (j == k) X[i][k] = l;
                else A[i][j] -= l * A[k][j];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kTT / 256; ++u) {
        const int x = tid + 256 * u;
        const int i = x / kT, j = x % kT;
        if (i > j) A[i][j] = X[i][j];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTT / 256; ++u) {
        const int x = tid + 256 * u;
        X[x / kT][x % kT] = x / kT == x % kT ? 1.0 : 0.0;
    }
    __syncthreads();
    // packed inverses by substitution in column (axpy) form, both in the same 32 steps,
    // every entry of a step on its own thread: step s is step k = s of inv(L) (entries
    // (i > k, c <= k) of X lose L_ik X_kc, X_kk = 1 implied) and step k = 31 - s of inv(U)
    // (row k of inv(U) is X_k. / U_kk, written to W, and entries (i < k, c >= k) lose
    // U_ik times it).  Each entry sees its updates in the same order as a column-by-column
    // substitution, so the values are those of one.
    for (int st = 0; st < kT; ++st) {
        const int kl = st, ku = kT - 1 - st;
        const int nl = (kT - 1 - kl) * (kl + 1);   // inv(L) entries of this step
        const int nu = (ku + 1) * (kT - ku);       // inv(U) row ku and the rows above it
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int t = tid + 256 * u;
            if (t < nl) {
                const int i = kl + 1 + t / (kl + 1), c = t % (kl + 1);
                X[i][c] -= A[i][kl] * (c == kl ? 1.0 : X[kl][c]);
            } else if (t < nl + nu) {
                const int t2 = t - nl;
                const int i = t2 / (kT - ku), c = ku + t2 % (kT - ku);
                const double xk = X[ku][c] / A[ku][ku];
                if (i == ku) W[ku][c] = xk;
                else X[i][c] -= A[i][ku] * xk;
            }
        }
        __syncthreads();
    }
    for (int x = tid; x < kTT; x += blockDim.x) {
        const int i = x / kT, j = x % kT;
        const double pv = i > j ? X[i][j] : W[i][j];
        dp[x] = (T)pv;
        inv64[(int64_t)sub * kTT + x] = pv;   // FP64 copy for the L panel of this step
    }
    const int32_t* tfr = e.tfr + sb.env_off;
    int J1 = K + 1;
    while (J1 < sb.nT && tfr[J1] <= K) ++J1;   // U tiles of row K: columns K+1 .. J1-1
    if constexpr (sizeof(T) == 4) {
        // U panel on the matrix cores, one wave per tile: U_KJ = inv(L_KK) A_KJ (unit lower
        // inverse, rounded to FP32; the product accumulates from zero)
        const int lane = tid & 63, w = tid >> 6;
        float a[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int i = lane & 31, k = 2 * s + (lane >> 5);
            a[s] = k < i ? (float)X[i][k] : (k == i ? 1.f : 0.f);
        }
        for (int J = K + 1 + w; J < J1; J += 4) {
            T* up = tile_ptr(F, e, sb, K, J);
            float b[16];
            load_b(b, up, lane);
            f32x16 acc = {};
            acc = mfma_tile(acc, a, b);
#pragma unroll
            for (int v = 0; v < 16; ++v) up[mrow(v, lane) * kT + (lane & 31)] = acc[v];
        }
    } else {
        // U panel in FP64 on the vector units
        __shared__ double B[kT][kT + 1];
        for (int J = K + 1; J < J1; ++J) {
            T* up = tile_ptr(F, e, sb, K, J);
            __syncthreads();
            for (int x = tid; x < kTT; x += blockDim.x) B[x / kT][x % kT] = (double)up[x];
            __syncthreads();
            for (int x = tid; x < kTT; x += blockDim.x) {
                const int i = x / kT, j = x % kT;
                double acc = B[i][j];
                for (int m = 0; m < i; ++m) acc += X[i][m] * B[m][j];
                up[x] = (T)acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// LU step K, part 2 (one block per (subdomain, tile row I > K)): L_IK = A_IK inv(U_KK),
// then A_IJ -= L_IK U_KJ for every J > K in the envelope.  FP32: the products run on the
// matrix cores, one wave per trailing tile; FP64: on the vector units through LDS.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) lu_row_kernel(Env e, T* __restrict__ F, const int32_t* __restrict__ pairs,
                                                     int K, const double* __restrict__ inv64) {
    __shared__ T Lt[kT][kT + 1];
    __shared__ T Bt[kT][kT + 1];
    const int sub = pairs[2 * blockIdx.x];
    const Sub sb = e.subs[sub];
    const int I = pairs[2 * blockIdx.x + 1];
    const int tid = threadIdx.x;
    const double* ip = inv64 + (int64_t)sub * kTT;   // packed FP64 inverses of step K; inv(U_KK) on and above
    T* lp = tile_ptr(F, e, sb, I, K);
    const int32_t* tfr = e.tfr + sb.env_off;
    int J1 = K + 1;
    while (J1 < sb.nT && tfr[J1] <= K) ++J1;
    if constexpr (sizeof(T) == 4) {
        // L panel on the matrix cores (wave 0): L_IK = A_IK inv(U_KK), inverse rounded to FP32
        const int lane = tid & 63;
        if (tid < 64) {
            float a[16], b[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int k = 2 * s + (lane >> 5), j = lane & 31;
                a[s] = lp[(lane & 31) * kT + k];
                b[s] = k <= j ? (float)ip[k * kT + j] : 0.f;
            }
            f32x16 acc = {};
            acc = mfma_tile(acc, a, b);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = mrow(v, lane), j = lane & 31;
                Lt[i][j] = acc[v];
                lp[i * kT + j] = acc[v];
            }
        }
    } else {
        // L panel in FP64: L_IK = A_IK inv(U_KK)
        __shared__ double Ad[kT][kT + 1];
        __shared__ double Ui[kT][kT + 1];
        for (int x = tid; x < kTT; x += blockDim.x) {
            Ad[x / kT][x % kT] = (double)lp[x];
            Ui[x / kT][x % kT] = ip[x];
        }
        __syncthreads();
        for (int x = tid; x < kTT; x += blockDim.x) {
            const int i = x / kT, j = x % kT;
            double acc = 0.0;
            for (int m = 0; m <= j; ++m) acc += Ad[i][m] * Ui[m][j];
            Lt[i][j] = (T)acc;
            lp[x] = (T)acc;
        }
    }
    __syncthreads();
    if constexpr (sizeof(T) == 4) {
        const int lane = tid & 63, w = tid >> 6;
        float a[16];   // -L_IK in the A-operand layout
#pragma unroll
        for (int s = 0; s < 16; ++s) a[s] = -Lt[lane & 31][2 * s + (lane >> 5)];
        for (int J = K + 1 + w; J < J1; J += 4) {
            const T* up = tile_ptr(F, e, sb, K, J);
            T* ap = tile_ptr(F, e, sb, I, J);
            float b[16];
            load_b(b, up, lane);
            // the product is accumulated from zero and subtracted once, so A_IJ is rounded
            // once per step rather than once per k-pair
            f32x16 acc = {};
            acc = mfma_tile(acc, a, b);
#pragma unroll
            for (int v = 0; v < 16; ++v) ap[mrow(v, lane) * kT + (lane & 31)] += acc[v];
        }
    } else {
        for (int J = K + 1; J < J1; ++J) {
            const T* up = tile_ptr(F, e, sb, K, J);
            T* ap = tile_ptr(F, e, sb, I, J);
            __syncthreads();
            for (int x = tid; x < kTT; x += blockDim.x) Bt[x / kT][x % kT] = up[x];
            __syncthreads();
            for (int x = tid; x < kTT; x += blockDim.x) {
                int i = x / kT, j = x % kT;
                T acc = 0;
#pragma unroll 8
                for (int m = 0; m < kT; ++m) acc += Lt[i][m] * Bt[m][j];
                ap[x] -= acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Triangular solves, one block (256 threads) per (subdomain, right-hand side).
// mode 0: b gathered from a global vector through the slot list, x to `out` + local_off[s];
// mode 1: in place on column `col` of a column-major block (ld = nT*T) at `out` + off[s].
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum8(T v) {
    v += __shfl_down(v, 4, 8);
    v += __shfl_down(v, 2, 8);
    v += __shfl_down(v, 1, 8);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(256) trsv_kernel(Env e, const T* __restrict__ F, const int32_t* __restrict__ sub_ids,
                                                   const int32_t* __restrict__ slots, const T* __restrict__ vin,
                                                   T* __restrict__ out, const int64_t* __restrict__ off,
                                                   const int32_t* __restrict__ ncols, int mode) {
    __shared__ T yt[kT];
    __shared__ T part[kT];
    const int s = sub_ids[blockIdx.x];
    const Sub sb = e.subs[s];
    const int col = blockIdx.y;
    if (mode == 1 && col >= ncols[s]) return;
    const int tid = threadIdx.x;
    const int ld = sb.nT * kT;
    T* x = out + off[s] + (mode == 1 ? (int64_t)col * ld : 0);
    const int32_t* sl = slots + sb.slot_off;
    const int32_t* tfc = e.tfc + sb.env_off;
    const int32_t* tfr = e.tfr + sb.env_off;
    const int r = tid >> 3, q = tid & 7;      // row within a tile, 4-column chunk
    // forward: L y = b (unit lower), L stored by tile rows
    for (int I = 0; I < sb.nT; ++I) {
        // four tiles per pass with separate sums, so that their loads are in flight together
        T acc4[4] = {0, 0, 0, 0};
        int J = tfc[I];
        for (; J + 4 <= I; J += 4) {
            T lv[4][4], yv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T* lt = tile_ptr(const_cast<T*>(F), e, sb, I, J + u);
                const T* yj = x + (J + u) * kT;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    lv[u][m] = lt[r * kT + q * 4 + m];
                    yv[u][m] = yj[q * 4 + m];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int m = 0; m < 4; ++m) acc4[u] += lv[u][m] * yv[u][m];
        }
        for (; J < I; ++J) {
            const T* lt = tile_ptr(const_cast<T*>(F), e, sb, I, J);
            const T* yj = x + J * kT;
#pragma unroll
            for (int m = 0; m < 4; ++m) acc4[0] += lt[r * kT + q * 4 + m] * yj[q * 4 + m];
        }
        T acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
        acc = wave_sum8(acc);
        if (q == 0) {
            int gr = I * kT + r;
            T b;
            if (mode == 0) b = gr < sb.n ? vin[sl[gr]] : (T)0;
            else b = x[gr];
            part[r] = b - acc;
        }
        __syncthreads();
        {   // y_I = inv(L_II) part: strictly lower part of the inverted tile, unit diagonal
            const T* dt = F + sb.diag_off + (int64_t)I * kTT + r * kT + q * 4;
            T v = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = q * 4 + m;
                v += (k < r ? dt[m] : (k == r ? (T)1 : (T)0)) * part[k];
            }
            v = wave_sum8(v);
            if (q == 0) x[I * kT + r] = v;
        }
        __syncthreads();
    }
    // backward: U x = y, U stored by tile columns
    for (int J = sb.nT - 1; J >= 0; --J) {
        {   // x_J = inv(U_JJ) x_J: upper part (with diagonal) of the inverted tile
            const T* dt = F + sb.diag_off + (int64_t)J * kTT + r * kT + q * 4;
            T v = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = q * 4 + m;
                if (k >= r) v += dt[m] * x[J * kT + k];
            }
            v = wave_sum8(v);
            if (q == 0) yt[r] = v;
        }
        __syncthreads();
        if (tid < kT) x[J * kT + tid] = yt[tid];
        int I = tfr[J];
        for (; I + 4 <= J; I += 4) {   // four tiles per pass, loads in flight together
            T uv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T* ut = tile_ptr(const_cast<T*>(F), e, sb, I + u, J);
#pragma unroll
                for (int m = 0; m < 4; ++m) uv[u][m] = ut[r * kT + q * 4 + m];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                T acc = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m) acc += uv[u][m] * yt[q * 4 + m];
                acc = wave_sum8(acc);
                if (q == 0) x[(I + u) * kT + r] -= acc;
            }
        }
        for (; I < J; ++I) {
            const T* ut = tile_ptr(const_cast<T*>(F), e, sb, I, J);
            T acc = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) acc += ut[r * kT + q * 4 + m] * yt[q * 4 + m];
            acc = wave_sum8(acc);
            if (q == 0) x[I * kT + r] -= acc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Single-right-hand-side solves for the preconditioner application: one block of 1024
// threads per subdomain (largest first), no communication between blocks.  Thread
// (r, c) = (tid / 32, tid % 32) owns element (r, c) of every tile it touches, so the
// tiles of a tile row (L, stored row by row) or of a tile column (U, stored column by
// column) stream through the block as one contiguous, coalesced range with independent
// loads; partial sums are reduced over the 32 lanes of a row.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T sum32(T v);

// Lane permutations inside a wave: DPP within 16-lane rows, a swizzle across the two
// rows of a 32-lane group (bit mode: and 0x1f, xor 0x10).
template <int kCtrl>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xf, 0xf, true));
}
template <int kCtrl>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), kCtrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float swz16_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401f));
}
__device__ __forceinline__ double swz16_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), 0x401f);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401f);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 32 lanes of a half-wave, result in every lane: quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror (a 16-lane sum), then the other row.
template <>
__device__ __forceinline__ float sum32<float>(float v) {
    v += dpp_f<0xb1>(v);
    v += dpp_f<0x4e>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return v + swz16_f(v);
}
template <>
__device__ __forceinline__ double sum32<double>(double v) {
    v += dpp_d<0xb1>(v);
    v += dpp_d<0x4e>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return v + swz16_d(v);
}

constexpr size_t kTrsvLdsMax = 64 * 1024;   // dynamic LDS bound for the in-LDS solve
// tiles of a tile row (column) held per register buffer: 32 FP32 or 16 FP64 values per thread
template <typename T>
constexpr int pf_tiles() { return sizeof(T) == 4 ? 30 : 16; }

// Tiles t0..nt-1 of a long tile row (past the register buffer), eight loads in flight.
template <typename T>
__device__ __forceinline__ T tail_dot(const T* __restrict__ src, const T* y, int t0, int nt) {
    T acc = 0;
    int t = t0;
    for (; t + 8 <= nt; t += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = src[(int64_t)(t + q) * kTT];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q] * y[(t + q) * kT];
    }
    for (; t < nt; ++t) acc += src[(int64_t)t * kTT] * y[t * kT];
    return acc;
}

// buf[t] = tile t of a tile row for t < n (entries past the row keep stale values,
// which buf_dot drops)
// Buffer resource over the n tiles of a tile row (raw, bounds-checked: a load past the
// range returns zero without a memory access).  Flags: the data-format word of CDNA3/4.
constexpr int kBufFlags = 0x00020000;
// (the row pointer and count are the same in every lane: taken from the first lane, so the
// descriptor lives in scalar registers)
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T* row, int n) {
    const uint64_t a = reinterpret_cast<uint64_t>(row);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    T* base = reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, __builtin_amdgcn_readfirstlane(n) * kTT * (int)sizeof(T),
                                             kBufFlags);
}

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t rs, int byte_off) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, byte_off, 0, 0));
}

// buf[t] = element `el` of tile t of a tile row of n tiles, t < kPF.  Every call issues
// the same kPF loads (those past the row return zero and touch no memory): with a fixed
// count the waits on a buffer can count exactly, whereas loads skipped by branches make
// every later wait drain all loads in flight, including the rows prefetched ahead.
template <typename T, int kPF>
__device__ __forceinline__ void load_row(T (&buf)[kPF], const T* __restrict__ row, int n, int el) {
    const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, n);
#pragma unroll
    for (int t = 0; t < kPF; ++t) buf[t] = buf_ld<T>(rs, (t * kTT + el) * (int)sizeof(T));
}

// sum_{t < n} buf[t] y[t kT]; n is the same for the whole workgroup, so each term sits
// behind a uniform branch (no LDS read or product past the row)
template <typename T, int kPF>
__device__ __forceinline__ T buf_dot(const T (&buf)[kPF], const T* y, int n) {
    T acc = 0;
#pragma unroll
    for (int t = 0; t < kPF; ++t)
        if (t < n) acc += buf[t] * y[t * kT];
    return acc;
}

// The per-row envelope of a subdomain (first L tile column, last U tile column, and the
// offsets of the L and U tile rows from its first diagonal tile) staged in LDS, 4 nT ints
// at m.  The substitutions read them from LDS: global loads complete in order, so waiting
// for a global load of them would also wait for every factor load issued before it (the
// tile rows prefetched ahead of the substitution).
// An entry of the staged envelope, the same in every lane (read from LDS, made scalar so
// that row pointers, counts and buffer ranges live in scalar registers)
__device__ __forceinline__ int row_u(const int32_t* m, int i) { return __builtin_amdgcn_readfirstlane(m[i]); }

__device__ __forceinline__ void stage_rows(const Env& e, const Sub& sb, int32_t* m, int tid, int nthr) {
    for (int I = tid; I < sb.nT; I += nthr) {
        const int64_t k = sb.env_off + I;
        m[I] = e.tfc[k];
        m[sb.nT + I] = e.tlc[k];
        m[2 * sb.nT + I] = (int32_t)(e.lrow[k] - sb.diag_off);
        m[3 * sb.nT + I] = (int32_t)(e.urow[k] - sb.diag_off);
    }
}

// kLds: the subdomain's solution vector lives in LDS (dynamic, nT * T entries) during
// the solve and is written out once at the end; otherwise it is updated in place in
// `out`.  Diagonal tiles hold inv(L_II) (strictly lower, unit diagonal implied) and
// inv(U_II) (upper with diagonal), so each diagonal block is one 32 x 32 product.
// Both substitutions are row-oriented (one 32-lane reduction per tile row); the tiles
// of tile row I + 2 (I - 2 going backward) are loaded into registers while rows I and
// I + 1 are processed (two register buffers), which keeps two rows of factor loads in
// flight behind the dependency chain of the substitution.
//
// phase (split primaries, for the halves [A, S] only; other subdomains solve whole):
// 1 = forward substitution of the half (rows below sep0), then the separator rows minus
//     their half's part, r_S - L_SA y_A (for the second half, whose separator rows hold
//     no right-hand side, -L_SB y_B); no backward substitution;
// 2 = backward substitution of the half with the separator's solution read from the
//     separator's local vector.
template <typename T, bool kLds>
__global__ void __launch_bounds__(1024) trsv_sub_kernel(Env e, const T* __restrict__ F,
                                                        const int32_t* __restrict__ order,
                                                        const int32_t* __restrict__ slots, const T* __restrict__ vin,
                                                        T* __restrict__ out, const int64_t* __restrict__ off,
                                                        int phase, int mrows) {
    constexpr int kPF = pf_tiles<T>();
    extern __shared__ double2 sub_lds[];
    unsigned char* dyn_lds = reinterpret_cast<unsigned char*>(sub_lds);
    __shared__ T part[kT];
    const int s = order[blockIdx.x];
    const Sub sb = e.subs[s];
    const int nT = sb.nT;
    if (nT == 0) return;
    T* xo = out + off[s];
    if (skip_solve(e, s)) {
        for (int i = threadIdx.x; i < nT * kT; i += blockDim.x) xo[i] = (T)0;
        return;
    }
    const bool half = phase != 0 && sb.kind == 2;
    const int stop = half ? sb.sep0 / kT : nT;   // rows eliminated by the substitutions
    const bool fwd = !half || phase == 1, bwd = !half || phase == 2;
    T* x = kLds ? reinterpret_cast<T*>(dyn_lds + 16 * mrows) : xo;
    const int tid = threadIdx.x, r = tid >> 5, c = tid & 31;
    int32_t* meta = reinterpret_cast<int32_t*>(dyn_lds);
    stage_rows(e, sb, meta, tid, 1024);
    const int32_t* tfc = meta;
    const int32_t* tlc = meta + nT;
    const int32_t* lrow = meta + 2 * nT;
    const int32_t* urow = meta + 3 * nT;
    const int32_t* sl = slots + sb.slot_off;
    const T* Fd = F + sb.diag_off;
    const T* D = Fd + tid;
    const int len = nT * kT;
    if (fwd) {
        const int nb = sb.skip_ss ? sb.sep0 : sb.n;
        for (int i = tid; i < len; i += 1024) x[i] = i < nb ? vin[sl[i]] : (T)0;
    } else {
        const T* xs = out + off[e.splits[sb.split].s_sub];
        for (int i = tid; i < len; i += 1024) x[i] = i < stop * kT ? xo[i] : xs[i - stop * kT];
    }
    __syncthreads();
    T bufA[kPF], bufB[kPF];
#pragma unroll
    for (int t = 0; t < kPF; ++t) bufA[t] = bufB[t] = 0;
    int nA = 0, nB = 0;
    T dA, dB;
    // rows I and I + 1 are in flight while row I - 2 is solved; loads of rows past the
    // end are clamped to the last row (and never used)
    // (the diagonal value of a row is fetched only after the row's diagonal product has
    // consumed the previous one, so that it reuses its register without a copy)
    // L tiles of row I taken by the substitution: columns below both I and stop
    auto lcount = [&](int I) { return max(min(I, stop) - row_u(tfc, I), 0); };
    auto fetch_l = [&](int I, T(&buf)[kPF], int& nb) {
        const int Ic = min(I, nT - 1);
        nb = min(lcount(Ic), kPF);
        load_row(buf, Fd + row_u(lrow, Ic), nb, tid);
    };
    auto fetch_u = [&](int I, T(&buf)[kPF], int& nb) {
        const int Ic = max(I, 0);
        nb = min(row_u(tlc, Ic) - Ic, kPF);
        load_row(buf, Fd + row_u(urow, Ic), nb, tid);
    };
    if (fwd) {
        fetch_l(0, bufA, nA);
        fetch_l(1, bufB, nB);
        dA = D[0];
        dB = D[(int64_t)min(1, nT - 1) * kTT];
    }
    __syncthreads();
    // ---- forward: L y = b, row-oriented over L's contiguous tile rows
    auto fwd_row = [&](int I, T(&buf)[kPF], int& nb, T& db) {
        const int j0 = row_u(tfc, I), nt = lcount(I);
        const T* y = x + j0 * kT + c;
        T acc = buf_dot(buf, y, nb);
        if (nt > kPF) acc += tail_dot<T>(Fd + row_u(lrow, I) + tid, y, kPF, nt);
        fetch_l(I + 2, buf, nb);
        acc = sum32(acc);
        if (I >= stop) {   // separator row of a half: no elimination, no dependency
            if (c == 0) x[I * kT + r] -= acc;
            return;
        }
        if (c == 0) part[r] = x[I * kT + r] - acc;
        __syncthreads();
        const T v = sum32((c < r ? db : (c == r ? (T)1 : (T)0)) * part[c]);
        if (c == 0) x[I * kT + r] = v;
        db = D[(int64_t)min(I + 2, nT - 1) * kTT];
        __syncthreads();
    };
    // (the loop bodies have no exit between their two rows: a path from the first row back
    // to the top would make the compiler take the first buffer's loads as the latest at the
    // top and wait for every load in flight there)
    if (fwd) {
        int I = 0;
        for (; I + 1 < nT; I += 2) {
            fwd_row(I, bufA, nA, dA);
            fwd_row(I + 1, bufB, nB, dB);
        }
        if (I < nT) fwd_row(I, bufA, nA, dA);
        __syncthreads();
    }
    // ---- backward: U x = y, row-oriented over U's contiguous tile rows (descending)
    auto bwd_row = [&](int I, T(&buf)[kPF], int& nb, T& db) {
        const int nt = row_u(tlc, I) - I;
        const T* y = x + (I + 1) * kT + c;
        T acc = buf_dot(buf, y, nb);
        if (nt > kPF) acc += tail_dot<T>(Fd + row_u(urow, I) + tid, y, kPF, nt);
        fetch_u(I - 2, buf, nb);
        acc = sum32(acc);
        if (c == 0) part[r] = x[I * kT + r] - acc;
        __syncthreads();
        const T v = sum32((c >= r ? db : (T)0) * part[c]);
        if (c == 0) x[I * kT + r] = v;
        db = D[(int64_t)max(I - 2, 0) * kTT];
        __syncthreads();
    };
    if (bwd) {
        fetch_u(stop - 1, bufA, nA);
        fetch_u(stop - 2, bufB, nB);
        dA = D[(int64_t)(stop - 1) * kTT];
        dB = D[(int64_t)max(stop - 2, 0) * kTT];
        int I = stop - 1;
        for (; I >= 1; I -= 2) {
            bwd_row(I, bufA, nA, dA);
            bwd_row(I - 1, bufB, nB, dB);
        }
        if (I == 0) bwd_row(0, bufA, nA, dA);
    }
    if (kLds)
        for (int i = tid; i < len; i += 1024) xo[i] = x[i];
}

// Separators of the split primaries: x_S = S'^-1 r'_S with r'_S the sum of the two
// halves' separator rows after phase 1; one block per (split, 64 rows of S'^-1, column-
// major), four waves over interleaved columns, the solution written to the separator's
// local vector.
template <typename T>
__global__ void __launch_bounds__(256) sep_solve_kernel(Env e, const T* __restrict__ sinv, T* __restrict__ loc,
                                                        const int64_t* __restrict__ off) {
    extern __shared__ double2 sep_lds[];
    T* rs = reinterpret_cast<T*>(sep_lds);
    __shared__ T red[4][64];
    const Split sp = e.splits[blockIdx.x];
    const int row0 = blockIdx.y * 64;
    if (row0 >= sp.ld) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const T* xa = loc + off[sp.a_sub] + sp.nA;
    const T* xb = loc + off[sp.b_sub] + sp.nB;
    for (int i = tid; i < sp.nS; i += 256) rs[i] = xa[i] + xb[i];
    __syncthreads();
    const int row = row0 + lane;
    T acc = 0;
    if (row < sp.ld) {
        const T* m = sinv + sp.inv_off + row;
        for (int j = w; j < sp.nS; j += 4) acc += m[(int64_t)j * sp.ld] * rs[j];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < sp.ld) loc[off[sp.s_sub] + row] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// S' = the sum of the two halves' trailing separator blocks (after their eliminations
// stopped at the separator), one block per (split, separator tile); tiles outside a
// half's envelope are zero.
template <typename T>
__global__ void schur_sum_kernel(Env e, T* __restrict__ F) {
    const Split sp = e.splits[blockIdx.x];
    const int nts = sp.ld / kT;
    const int I = blockIdx.y, J = blockIdx.z;
    if (I >= nts || J >= nts) return;
    auto tile_if = [&](const Sub& sb, int a0) -> const T* {
        const int i = a0 + I, j = a0 + J;
        if (j < i && j < e.tfc[sb.env_off + i]) return nullptr;
        if (i < j && j > e.tlc[sb.env_off + i]) return nullptr;
        return tile_ptr(F, e, sb, i, j);
    };
    const Sub a = e.subs[sp.a_sub], b = e.subs[sp.b_sub], sv = e.subs[sp.s_sub];
    const T* ta = tile_if(a, sp.nA / kT);
    const T* tb = tile_if(b, sp.nB / kT);
    T* ts = tile_ptr(F, e, sv, I, J);
    for (int x = threadIdx.x; x < kTT; x += blockDim.x) ts[x] = (ta ? ta[x] : (T)0) + (tb ? tb[x] : (T)0);
}

// Identity columns 0 .. nS-1 of each separator's inverse block (solved in place).
template <typename T>
__global__ void sep_identity_kernel(Env e, T* __restrict__ sinv) {
    const Split sp = e.splits[blockIdx.x];
    const int j = blockIdx.y;
    if (j >= sp.nS) return;
    T* col = sinv + sp.inv_off + (int64_t)j * sp.ld;
    for (int i = threadIdx.x; i < sp.ld; i += blockDim.x) col[i] = i == j ? (T)1 : (T)0;
}

// ---------------------------------------------------------------------------------------
// The same substitutions for small subdomains (the dual grids): one 256-thread block per
// subdomain, so that many subdomains share a compute unit.  Thread (r, q) = (tid / 8,
// tid % 8) owns the four elements (r, 4q .. 4q + 3) of every tile it touches (one 16- or
// 32-byte load per tile), reads the four matching solution entries with one LDS read, and
// the row sums are reduced over the 8 lanes of a row (three DPP steps).
// ---------------------------------------------------------------------------------------
template <typename T>
struct Quad {
    T v[4];
};

template <typename T>
__device__ __forceinline__ Quad<T> ld4(const T* p) {
    Quad<T> q;
    if constexpr (sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        q.v[0] = a.x; q.v[1] = a.y; q.v[2] = a.z; q.v[3] = a.w;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 b = *reinterpret_cast<const double2*>(p + 2);
        q.v[0] = a.x; q.v[1] = a.y; q.v[2] = b.x; q.v[3] = b.y;
    }
    return q;
}

// the four elements at byte_off of a bounds-checked row buffer (zeros past the row)
template <typename T>
__device__ __forceinline__ Quad<T> buf_ld4(__amdgpu_buffer_rsrc_t rs, int byte_off) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 0);
        return __builtin_bit_cast(Quad<T>, v);
    } else {
        struct Two {
            u32x4 a, b;
        };
        Two w;
        w.a = __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off, 0, 0);
        w.b = __builtin_amdgcn_raw_buffer_load_b128(rs, byte_off + 16, 0, 0);
        return __builtin_bit_cast(Quad<T>, w);
    }
}

template <typename T>
__device__ __forceinline__ T dot4(const Quad<T>& a, const Quad<T>& b) {
    return a.v[0] * b.v[0] + a.v[1] * b.v[1] + a.v[2] * b.v[2] + a.v[3] * b.v[3];
}

// Sum over the 8 lanes of a row, result in every lane: quad_perm [1,0,3,2], [2,3,0,1],
// then row_half_mirror (lane i <-> 7 - i inside each group of 8).
template <typename T>
__device__ __forceinline__ T sum8(T v) {
    if constexpr (sizeof(T) == 4) {
        v += dpp_f<0xb1>(v);
        v += dpp_f<0x4e>(v);
        return v + dpp_f<0x141>(v);
    } else {
        v += dpp_d<0xb1>(v);
        v += dpp_d<0x4e>(v);
        return v + dpp_d<0x141>(v);
    }
}

template <typename T>
constexpr int pf_small() { return sizeof(T) == 4 ? 6 : 3; }

template <typename T>
__global__ void __launch_bounds__(256) trsv_small_kernel(Env e, const T* __restrict__ F,
                                                         const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ slots,
                                                         const T* __restrict__ vin, T* __restrict__ out,
                                                         const int64_t* __restrict__ off, int mrows) {
    constexpr int kPF = pf_small<T>();
    extern __shared__ double2 small_lds[];
    __shared__ __align__(16) T part[kT];
    const int s = order[blockIdx.x];
    const Sub sb = e.subs[s];
    const int nT = sb.nT;
    if (nT == 0) return;
    T* xo = out + off[s];
    if (skip_solve(e, s)) {
        for (int i = threadIdx.x; i < nT * kT; i += blockDim.x) xo[i] = (T)0;
        return;
    }
    T* x = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(small_lds) + 16 * mrows);
    const int tid = threadIdx.x, r = tid >> 3, q = tid & 7;
    const int el = r * kT + 4 * q;   // first of this thread's four elements in a tile
    int32_t* meta = reinterpret_cast<int32_t*>(small_lds);
    stage_rows(e, sb, meta, tid, 256);
    const int32_t* tfc = meta;
    const int32_t* tlc = meta + nT;
    const int32_t* lrow = meta + 2 * nT;
    const int32_t* urow = meta + 3 * nT;
    const int32_t* sl = slots + sb.slot_off;
    const T* Fd = F + sb.diag_off;
    const T* D = Fd + el;
    const int len = nT * kT;
    for (int i = tid; i < len; i += 256) x[i] = i < sb.n ? vin[sl[i]] : (T)0;
    __syncthreads();
    Quad<T> bufA[kPF], bufB[kPF];
    int nA = 0, nB = 0;
    Quad<T> dA, dB;
    // a fixed count of bounds-checked loads per row (see load_row)
    auto load = [&](Quad<T>(&buf)[kPF], const T* row, int n) {
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, n);
#pragma unroll
        for (int t = 0; t < kPF; ++t) buf[t] = buf_ld4<T>(rs, (t * kTT + el) * (int)sizeof(T));
    };
    auto dot = [&](const Quad<T>(&buf)[kPF], const T* y, int n) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < kPF; ++t)
            if (t < n) acc += dot4(buf[t], ld4(y + t * kT));
        return acc;
    };
    auto tail = [&](const T* src, const T* y, int t0, int nt) {
        T acc = 0;
        int t = t0;
        for (; t + 4 <= nt; t += 4) {
            Quad<T> a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = ld4(src + (int64_t)(t + u) * kTT);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += dot4(a[u], ld4(y + (t + u) * kT));
        }
        for (; t < nt; ++t) acc += dot4(ld4(src + (int64_t)t * kTT), ld4(y + t * kT));
        return acc;
    };
    auto fetch_l = [&](int I, Quad<T>(&buf)[kPF], int& nb) {
        const int Ic = min(I, nT - 1);
        nb = min(Ic - row_u(tfc, Ic), kPF);
        load(buf, Fd + row_u(lrow, Ic), nb);
    };
    auto fetch_u = [&](int I, Quad<T>(&buf)[kPF], int& nb) {
        const int Ic = max(I, 0);
        nb = min(row_u(tlc, Ic) - Ic, kPF);
        load(buf, Fd + row_u(urow, Ic), nb);
    };
    fetch_l(0, bufA, nA);
    fetch_l(1, bufB, nB);
    dA = ld4(D);
    dB = ld4(D + (int64_t)min(1, nT - 1) * kTT);
    __syncthreads();
    // ---- forward: L y = b (inv(L_II) strictly lower, unit diagonal implied)
    auto fwd_row = [&](int I, Quad<T>(&buf)[kPF], int& nb, Quad<T>& db) {
        const int j0 = row_u(tfc, I), nt = I - j0;
        const T* y = x + j0 * kT + 4 * q;
        T acc = dot(buf, y, nb);
        if (nt > kPF) acc += tail(Fd + row_u(lrow, I) + el, y, kPF, nt);
        fetch_l(I + 2, buf, nb);
        acc = sum8(acc);
        if (q == 0) part[r] = x[I * kT + r] - acc;
        __syncthreads();
        const Quad<T> p4 = ld4(part + 4 * q);
        T v = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int col = 4 * q + m;
            v += (col < r ? db.v[m] : (col == r ? (T)1 : (T)0)) * p4.v[m];
        }
        v = sum8(v);
        if (q == 0) x[I * kT + r] = v;
        db = ld4(D + (int64_t)min(I + 2, nT - 1) * kTT);
        __syncthreads();
    };
    int I0 = 0;
    for (; I0 + 1 < nT; I0 += 2) {   // no exit between the two rows (see trsv_sub_kernel)
        fwd_row(I0, bufA, nA, dA);
        fwd_row(I0 + 1, bufB, nB, dB);
    }
    if (I0 < nT) fwd_row(I0, bufA, nA, dA);
    // ---- backward: U x = y (inv(U_II) on and above the diagonal)
    auto bwd_row = [&](int I, Quad<T>(&buf)[kPF], int& nb, Quad<T>& db) {
        const int nt = row_u(tlc, I) - I;
        const T* y = x + (I + 1) * kT + 4 * q;
        T acc = dot(buf, y, nb);
        if (nt > kPF) acc += tail(Fd + row_u(urow, I) + el, y, kPF, nt);
        fetch_u(I - 2, buf, nb);
        acc = sum8(acc);
        if (q == 0) part[r] = x[I * kT + r] - acc;
        __syncthreads();
        const Quad<T> p4 = ld4(part + 4 * q);
        T v = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) v += (4 * q + m >= r ? db.v[m] : (T)0) * p4.v[m];
        v = sum8(v);
        if (q == 0) x[I * kT + r] = v;
        db = ld4(D + (int64_t)max(I - 2, 0) * kTT);
        __syncthreads();
    };
    fetch_u(nT - 1, bufA, nA);
    fetch_u(nT - 2, bufB, nB);
    dA = ld4(D + (int64_t)(nT - 1) * kTT);
    dB = ld4(D + (int64_t)max(nT - 2, 0) * kTT);
    int I1 = nT - 1;
    for (; I1 >= 1; I1 -= 2) {
        bwd_row(I1, bufA, nA, dA);
        bwd_row(I1 - 1, bufB, nB, dB);
    }
    if (I1 == 0) bwd_row(0, bufA, nA, dA);
    for (int i = tid; i < len; i += 256) xo[i] = x[i];
}

// ---------------------------------------------------------------------------------------
// The primary-grid substitutions with 16-byte loads: the 1024 threads form four groups
// of 256; group g takes the tiles t = g, g + 4, ... of every tile row, and thread (r, q)
// of a group owns the four elements (r, 4q .. 4q + 3) of each of its tiles, as in
// trsv_small_kernel.  A row's sums are reduced over the 8 lanes of a row, then over the
// four groups through LDS, and group 0 applies the diagonal block.  Same bytes as
// trsv_sub_kernel with a quarter of the load instructions.
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024) trsv_quad_kernel(Env e, const T* __restrict__ F,
                                                         const int32_t* __restrict__ order,
                                                         const int32_t* __restrict__ slots,
                                                         const T* __restrict__ vin, T* __restrict__ out,
                                                         const int64_t* __restrict__ off, int mrows) {
    // tiles per group held per register buffer (FP32: rows of up to 32 tiles, FP64: 16)
    constexpr int kPF = sizeof(T) == 4 ? 8 : 4;
    extern __shared__ double2 quad_lds[];
    __shared__ T part4[4][kT];
    const int s = order[blockIdx.x];
    const Sub sb = e.subs[s];
    const int nT = sb.nT;
    if (nT == 0) return;
    T* xo = out + off[s];
    if (skip_solve(e, s)) {
        for (int i = threadIdx.x; i < nT * kT; i += blockDim.x) xo[i] = (T)0;
        return;
    }
    T* x = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(quad_lds) + 16 * mrows);
    const int tid = threadIdx.x, g = tid >> 8, r = (tid & 255) >> 3, q = tid & 7;
    const int el = r * kT + 4 * q;
    int32_t* meta = reinterpret_cast<int32_t*>(quad_lds);
    stage_rows(e, sb, meta, tid, 1024);
    const int32_t* tfc = meta;
    const int32_t* tlc = meta + nT;
    const int32_t* lrow = meta + 2 * nT;
    const int32_t* urow = meta + 3 * nT;
    const int32_t* sl = slots + sb.slot_off;
    const T* Fd = F + sb.diag_off;
    const T* D = Fd + el;
    const int len = nT * kT;
    for (int i = tid; i < len; i += 1024) x[i] = i < sb.n ? vin[sl[i]] : (T)0;
    __syncthreads();
    Quad<T> bufA[kPF], bufB[kPF];
    int nA = 0, nB = 0;
    Quad<T> dA, dB;
    // this group's tiles of a row of nt tiles: g, g + 4, ... (a count uniform over each wave)
    auto mine = [&](int nt) { return nt > g ? min((nt - g + 3) >> 2, kPF) : 0; };
    // a fixed count of bounds-checked loads per row (see load_row): tiles g, g + 4, ... of
    // a row of nt tiles
    auto load = [&](Quad<T>(&buf)[kPF], const T* row, int nt) {
        const __amdgpu_buffer_rsrc_t rs = row_rsrc(row, min(nt, 4 * kPF));
#pragma unroll
        for (int u = 0; u < kPF; ++u) buf[u] = buf_ld4<T>(rs, ((g + 4 * u) * kTT + el) * (int)sizeof(T));
    };
    auto dot = [&](const Quad<T>(&buf)[kPF], const T* y, int n) {
        T acc = 0;
#pragma unroll
        for (int u = 0; u < kPF; ++u)
            if (u < n) acc += dot4(buf[u], ld4(y + (g + 4 * u) * kT));
        return acc;
    };
    auto tail = [&](const T* src, const T* y, int nt) {
        T acc = 0;
        for (int t = g + 4 * kPF; t < nt; t += 4) acc += dot4(ld4(src + (int64_t)t * kTT), ld4(y + t * kT));
        return acc;
    };
    auto fetch_l = [&](int I, Quad<T>(&buf)[kPF], int& nb) {
        const int Ic = min(I, nT - 1);
        const int nt = Ic - row_u(tfc, Ic);
        nb = mine(nt);
        load(buf, Fd + row_u(lrow, Ic), nt);
    };
    auto fetch_u = [&](int I, Quad<T>(&buf)[kPF], int& nb) {
        const int Ic = max(I, 0);
        const int nt = row_u(tlc, Ic) - Ic;
        nb = mine(nt);
        load(buf, Fd + row_u(urow, Ic), nt);
    };
    fetch_l(0, bufA, nA);
    fetch_l(1, bufB, nB);
    dA = ld4(D);
    dB = ld4(D + (int64_t)min(1, nT - 1) * kTT);
    __syncthreads();
    // b_c - (the row sums of the four groups) for this thread's four columns; group 0 folds
    // -b_r into its sum before the barrier, so nothing reads x[I kT ..] after it (group 0
    // overwrites that row with the solution)
    auto rhs4 = [&](int I) {
        Quad<T> p;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int col = 4 * q + m;
            p.v[m] = -(part4[0][col] + part4[1][col] + part4[2][col] + part4[3][col]);
        }
        return p;
    };
    // ---- forward: L y = b (inv(L_II) strictly lower, unit diagonal implied)
    auto fwd_row = [&](int I, Quad<T>(&buf)[kPF], int& nb, Quad<T>& db) {
        const int j0 = row_u(tfc, I), nt = I - j0;
        const T* y = x + j0 * kT + 4 * q;
        T acc = dot(buf, y, nb);
        if (nt > 4 * kPF) acc += tail(Fd + row_u(lrow, I) + el, y, nt);
        fetch_l(I + 2, buf, nb);
        acc = sum8(acc);
        if (q == 0) part4[g][r] = g == 0 ? acc - x[I * kT + r] : acc;
        __syncthreads();
        if (g == 0) {
            const Quad<T> p4 = rhs4(I);
            T v = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int col = 4 * q + m;
                v += (col < r ? db.v[m] : (col == r ? (T)1 : (T)0)) * p4.v[m];
            }
            v = sum8(v);
            if (q == 0) x[I * kT + r] = v;
            db = ld4(D + (int64_t)min(I + 2, nT - 1) * kTT);
        }
        __syncthreads();
    };
    int I0 = 0;
    for (; I0 + 1 < nT; I0 += 2) {   // no exit between the two rows (see trsv_sub_kernel)
        fwd_row(I0, bufA, nA, dA);
        fwd_row(I0 + 1, bufB, nB, dB);
    }
    if (I0 < nT) fwd_row(I0, bufA, nA, dA);
    // ---- backward: U x = y (inv(U_II) on and above the diagonal)
    auto bwd_row = [&](int I, Quad<T>(&buf)[kPF], int& nb, Quad<T>& db) {
        const int nt = row_u(tlc, I) - I;
        const T* y = x + (I + 1) * kT + 4 * q;
        T acc = dot(buf, y, nb);
        if (nt > 4 * kPF) acc += tail(Fd + row_u(urow, I) + el, y, nt);
        fetch_u(I - 2, buf, nb);
        acc = sum8(acc);
        if (q == 0) part4[g][r] = g == 0 ? acc - x[I * kT + r] : acc;
        __syncthreads();
        if (g == 0) {
            const Quad<T> p4 = rhs4(I);
            T v = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) v += (4 * q + m >= r ? db.v[m] : (T)0) * p4.v[m];
            v = sum8(v);
            if (q == 0) x[I * kT + r] = v;
            db = ld4(D + (int64_t)max(I - 2, 0) * kTT);
        }
        __syncthreads();
    };
    if (g == 0) {
        dA = ld4(D + (int64_t)(nT - 1) * kTT);
        dB = ld4(D + (int64_t)max(nT - 2, 0) * kTT);
    }
    fetch_u(nT - 1, bufA, nA);
    fetch_u(nT - 2, bufB, nB);
    int I1 = nT - 1;
    for (; I1 >= 1; I1 -= 2) {
        bwd_row(I1, bufA, nA, dA);
        bwd_row(I1 - 1, bufB, nB, dB);
    }
    if (I1 == 0) bwd_row(0, bufA, nA, dA);
    for (int i = tid; i < len; i += 1024) xo[i] = x[i];
}

// ---------------------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------------------
static Env make_env(gplmm_ctx* c) {
    return Env{c->d_subs, c->d_tfc, c->d_tfr, c->d_tlc, c->d_lrow, c->d_urow, c->d_sub_samp, c->d_sact, c->d_splits};
}

template <typename T>
int assemble_subs(gplmm_ctx* c, int first_sub, int nsub, bool closure) {
    Env e = make_env(c);
    T* F = (T*)c->d_factor;
    const int64_t nrows = (int64_t)c->sub_slots.size();
    const unsigned nb = (unsigned)((nrows + 255) / 256);
    const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
    auto launch = [&](auto kern) {
        kern<<<nb, 256, 0, c->stream>>>(c->geo, c->d_xcoef, e, F, c->d_row_sub, c->d_sub_slots, c->d_sorted_slot,
                                        c->d_sorted_loc, c->d_slot_class, c->d_noclose, nrows, first_sub, nsub,
                                        closure ? 1 : 0);
    };
    if (c->ndim == 3) {
        if (jac) launch(assemble_kernel<3, T, true>);
        else launch(assemble_kernel<3, T, false>);
    } else {
        if (jac) launch(assemble_kernel<2, T, true>);
        else launch(assemble_kernel<2, T, false>);
    }
    if (nsub > 0) pad_kernel<T><<<nsub, 64, 0, c->stream>>>(e, F, first_sub, nsub);
    return GPLMM_OK;
}

template <typename T>
int factor_set(gplmm_ctx* c, int set) {
    Env e = make_env(c);
    T* F = (T*)c->d_factor;
    const auto& soff = c->lu_sub_off[set];
    const auto& poff = c->lu_step_off[set];
    timer_begin(c, "lu");
    for (int K = 0; K + 1 < (int)soff.size(); ++K) {
        int ns = (int)(soff[K + 1] - soff[K]);
        if (ns == 0) break;
        lu_diag_kernel<T><<<ns, 256, 0, c->stream>>>(e, F, c->d_sub_list[set] + soff[K], K, c->d_flag, c->d_inv64);
        int np = (int)(poff[K + 1] - poff[K]);
        if (np > 0)
            lu_row_kernel<T><<<np, 256, 0, c->stream>>>(e, F, c->d_step_pairs[set] + 2 * poff[K], K, c->d_inv64);
    }
    timer_end(c, "lu", c->lu_flops[set]);
    return GPLMM_OK;
}

template <typename T>
void trsv_gather(gplmm_ctx* c, const int32_t* sub_ids_dev, int nsub, const T* vin, T* out_local) {
    if (nsub <= 0) return;
    Env e = make_env(c);
    const bool duals = sub_ids_dev != c->d_sub_ids;
    const int set = duals ? 1 : 0;
    // algorithmic bytes: every factor tile of these subdomains once, the gathered
    // right-hand side (value + slot index) and the solution written and re-read
    const int s0 = duals ? c->Np : 0, s1 = duals ? c->Np + c->Nc : c->Np;
    const int64_t e0 = c->subs[s0].diag_off;
    const int64_t e1 = s1 < (int)c->subs.size() ? c->subs[s1].diag_off : c->factor_elems;
    const int64_t rows = (s1 < (int)c->subs.size() ? c->subs[s1].slot_off : (int64_t)c->sub_slots.size()) -
                         c->subs[s0].slot_off;
    const double bytes = (double)sizeof(T) * (double)(e1 - e0) + (double)rows * (3.0 * sizeof(T) + 4.0);
    timer_begin(c, "trsv");
    timer_begin(c, duals ? "trsv_d" : "trsv_p");
    // dynamic LDS: the staged row envelopes (16 bytes per tile row), then the solution
    const int mt = c->maxT_set[set];
    const size_t meta = (size_t)16 * mt;
    const size_t lds = meta + (size_t)mt * kT * sizeof(T);
    const T* F = (const T*)c->d_factor;
    const int32_t* ord = c->d_sub_order[set];
    if (duals && lds <= kTrsvLdsMax)
        trsv_small_kernel<T><<<nsub, 256, lds, c->stream>>>(e, F, ord, c->d_sub_slots, vin, out_local, c->d_local_off, mt);
    else if (lds <= kTrsvLdsMax && c->trsv_mode == 2)
        trsv_quad_kernel<T><<<nsub, 1024, lds, c->stream>>>(e, F, ord, c->d_sub_slots, vin, out_local, c->d_local_off, mt);
    else if (lds <= kTrsvLdsMax && c->trsv_mode == 0)
        trsv_sub_kernel<T, true><<<nsub, 1024, lds, c->stream>>>(e, F, ord, c->d_sub_slots, vin, out_local,
                                                                c->d_local_off, 0, mt);
    else
        trsv_sub_kernel<T, false><<<nsub, 1024, meta, c->stream>>>(e, F, ord, c->d_sub_slots, vin, out_local,
                                                                  c->d_local_off, 0, mt);
    timer_end(c, duals ? "trsv_d" : "trsv_p", bytes);
    timer_end(c, "trsv", bytes);
}

// Eq. xf: x_f = (A^f_f)^-1 r_f, one workgroup per diagonal block of A^f_f (the f-faces'
// connected sets; blocks of a few tiles, so the dual-block kernel).
template <typename T>
void trsv_fblocks(gplmm_ctx* c, const T* vin, T* out_local) {
    if (c->n_fsub <= 0) return;
    Env e = make_env(c);
    const int s0 = c->Np + c->Nc, s1 = s0 + c->n_fsub;
    const int64_t e0 = c->subs[s0].diag_off;
    const int64_t e1 = s1 < (int)c->subs.size() ? c->subs[s1].diag_off : c->factor_elems;
    const double bytes = (double)sizeof(T) * (double)(e1 - e0) + (double)(c->f_row1 - c->f_row0) * (3.0 * sizeof(T) + 4.0);
    timer_begin(c, "trsv");
    timer_begin(c, "trsv_f");
    const int mt = c->maxT_f;
    const size_t meta = (size_t)16 * mt;
    const size_t lds = meta + (size_t)mt * kT * sizeof(T);
    const T* F = (const T*)c->d_factor;
    if (lds <= kTrsvLdsMax)
        trsv_small_kernel<T><<<c->n_fsub, 256, lds, c->stream>>>(e, F, c->d_fsub_order, c->d_sub_slots, vin, out_local,
                                                                 c->d_local_off, mt);
    else
        trsv_sub_kernel<T, false><<<c->n_fsub, 1024, meta, c->stream>>>(e, F, c->d_fsub_order, c->d_sub_slots, vin,
                                                                       out_local, c->d_local_off, 0, mt);
    timer_end(c, "trsv_f", bytes);
    timer_end(c, "trsv", bytes);
}

// The primaries' solves with split primaries: phase 1 (unsplit primaries whole, halves
// forward), the separators, phase 2 (halves backward).  The halves' local vectors then
// hold [x_A, x_S] and [x_B, x_S].
template <typename T>
void trsv_split(gplmm_ctx* c, const T* vin, T* loc) {
    Env e = make_env(c);
    const T* F = (const T*)c->d_factor;
    const int nsp = (int)c->splits.size();
    // algorithmic bytes: the factor tiles the substitutions read (every tile of an unsplit
    // primary; of a half the tiles of its eliminated rows and the separator rows' L tiles
    // left of the separator), the separators' inverses, the gathered right-hand side
    // (value + slot index) and the solution written and re-read
    const double bytes = (double)sizeof(T) * (double)c->split_apply_elems + (double)c->prim_rows * (3.0 * sizeof(T) + 4.0);
    timer_begin(c, "trsv");
    timer_begin(c, "trsv_p");
    const int m1 = c->maxT_phase1, m3 = c->maxT_phase3;
    const size_t lds1 = (size_t)16 * m1 + (size_t)m1 * kT * sizeof(T);
    const size_t lds3 = (size_t)16 * m3 + (size_t)m3 * kT * sizeof(T);
    timer_begin(c, "trsv_p_fwd");
    if (lds1 <= kTrsvLdsMax)
        trsv_sub_kernel<T, true><<<c->n_phase1, 1024, lds1, c->stream>>>(e, F, c->d_phase_order[0], c->d_sub_slots, vin,
                                                                          loc, c->d_local_off, 1, m1);
    else
        trsv_sub_kernel<T, false><<<c->n_phase1, 1024, (size_t)16 * m1, c->stream>>>(
            e, F, c->d_phase_order[0], c->d_sub_slots, vin, loc, c->d_local_off, 1, m1);
    timer_end(c, "trsv_p_fwd", 0.0);
    timer_begin(c, "trsv_sep");
    sep_solve_kernel<T><<<dim3(nsp, (c->max_sep_ld + 63) / 64), 256, (size_t)c->max_sep_ld * sizeof(T), c->stream>>>(
        e, (const T*)c->d_sinv, loc, c->d_local_off);
    timer_end(c, "trsv_sep", 0.0);
    timer_begin(c, "trsv_p_bwd");
    if (lds3 <= kTrsvLdsMax)
        trsv_sub_kernel<T, true><<<c->n_phase3, 1024, lds3, c->stream>>>(e, F, c->d_phase_order[1], c->d_sub_slots, vin,
                                                                          loc, c->d_local_off, 2, m3);
    else
        trsv_sub_kernel<T, false><<<c->n_phase3, 1024, (size_t)16 * m3, c->stream>>>(
            e, F, c->d_phase_order[1], c->d_sub_slots, vin, loc, c->d_local_off, 2, m3);
    timer_end(c, "trsv_p_bwd", 0.0);
    timer_end(c, "trsv_p", bytes);
    timer_end(c, "trsv", bytes);
}

// Separators after the halves' stopped eliminations: S' assembled from the trailing
// blocks, factorised (schedule 2) and inverted column by column.
template <typename T>
int build_separators(gplmm_ctx* c) {
    const int nsp = (int)c->splits.size();
    if (nsp == 0) return GPLMM_OK;
    Env e = make_env(c);
    T* F = (T*)c->d_factor;
    const int mt = c->max_sep_ld / kT;
    schur_sum_kernel<T><<<dim3(nsp, mt, mt), 256, 0, c->stream>>>(e, F);
    int rc = factor_set<T>(c, 2);
    if (rc != GPLMM_OK) return rc;
    int maxs = 0;
    for (const Split& sp : c->splits) maxs = std::max(maxs, sp.nS);
    sep_identity_kernel<T><<<dim3(nsp, maxs), 256, 0, c->stream>>>(e, (T*)c->d_sinv);
    trsv_kernel<T><<<dim3(nsp, maxs), 256, 0, c->stream>>>(e, F, c->d_sep_ids, c->d_sub_slots, nullptr, (T*)c->d_sinv,
                                                          c->d_sinv_off, c->d_sinv_ncols, 1);
    return GPLMM_OK;
}

template <typename T>
void trsv_phi(gplmm_ctx* c, int maxcols) {
    if (c->Np <= 0 || maxcols <= 0) return;
    Env e = make_env(c);
    trsv_kernel<T><<<dim3(c->Np, maxcols), 256, 0, c->stream>>>(e, (const T*)c->d_factor, c->d_sub_ids,
                                                               c->d_sub_slots, nullptr, (T*)c->d_phi, c->d_phi_off,
                                                               c->d_phi_ncols, 1);
}

template int assemble_subs<float>(gplmm_ctx*, int, int, bool);
template int assemble_subs<double>(gplmm_ctx*, int, int, bool);
template int factor_set<float>(gplmm_ctx*, int);
template int factor_set<double>(gplmm_ctx*, int);
template void trsv_gather<float>(gplmm_ctx*, const int32_t*, int, const float*, float*);
template void trsv_gather<double>(gplmm_ctx*, const int32_t*, int, const double*, double*);
template void trsv_fblocks<float>(gplmm_ctx*, const float*, float*);
template void trsv_fblocks<double>(gplmm_ctx*, const double*, double*);
template void trsv_split<float>(gplmm_ctx*, const float*, float*);
template void trsv_split<double>(gplmm_ctx*, const double*, double*);
template int build_separators<float>(gplmm_ctx*);
template int build_separators<double>(gplmm_ctx*);
template void trsv_phi<float>(gplmm_ctx*, int);
template void trsv_phi<double>(gplmm_ctx*, int);

}  // namespace gp

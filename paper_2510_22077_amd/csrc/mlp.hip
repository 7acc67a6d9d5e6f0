// Small multilayer perceptron with BF16 MFMA forward and backward passes, FP32
// master weights and an Adam optimiser, used to predict coarse-operator
// coefficients from geometric features of pores and throats.
//
// Network: h_0 = x, h_l = gelu(h_{l-1} W_l + b_l) for the hidden layers,
// y = h_L W_out + b_out, GELU in its tanh form.  Loss: mean squared error.
// Products run on v_mfma_f32_16x16x16bf16_1k (one wave per 16 x 16 output tile,
// BF16 operands, FP32 accumulation); activations are kept in FP32 (pre-activation,
// for the backward pass) and BF16 (input of the next product).  Every dimension
// is padded to a multiple of 16 with zeros.
#include "internal.h"

#include <cmath>
#include <cstring>

struct gplmm_mlp {
    int nin = 0, nh = 0, nl = 0, nout = 0;
    int cap = 0;                         // batch capacity (padded rows)
    std::vector<int> dim;                // padded widths d_0 .. d_{nl+1}
    std::vector<int> rdim;               // true widths
    std::vector<int64_t> woff, boff;     // offsets of W_l, b_l in the padded parameter vector
    int64_t nparam = 0;                  // padded parameter count
    hipStream_t stream = nullptr;
    float* d_w = nullptr;                // padded FP32 master parameters
    float* d_g = nullptr;                // gradients (same layout)
    float* d_m = nullptr;                // Adam moments
    float* d_v = nullptr;
    uint16_t* d_wbf = nullptr;           // BF16 copy of the weights
    std::vector<float*> d_z;             // pre-activations, FP32 [cap x d_l], l = 1..nl+1
    std::vector<uint16_t*> d_h;          // activations, BF16 [cap x d_l], l = 0..nl
    uint16_t* d_dz = nullptr;            // BF16 [cap x max d]: upstream gradient of the current layer
    uint16_t* d_dz2 = nullptr;
    uint8_t* d_live = nullptr;           // 1 where the padded parameter vector holds a real parameter
    double* d_red = nullptr;             // loss partials
    double* h_red = nullptr;
    int adam_t = 0;
    std::string err;
};

namespace gp {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLossBlocks = 256;

__device__ __forceinline__ uint16_t to_bf16(float f) {   // round to nearest even
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2 / pi)
constexpr float kGeluA = 0.044715f;
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + tanhf(kGeluC * (z + kGeluA * z * z * z))); }
__device__ __forceinline__ float gelu_grad(float z) {
    const float t = tanhf(kGeluC * (z + kGeluA * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * kGeluC * (1.0f + 3.0f * kGeluA * z * z);
}

// C(m, n) = sum_k A(m, k) B(k, n) over BF16 operands addressed by strides, one wave per
// 16 x 16 tile of C.  Fragment layout of the instruction: lane l holds A(l % 16, 4 (l / 16)
// + j), B(4 (l / 16) + j, l % 16) and C(4 (l / 16) + j, l % 16), j = 0..3.
enum Epi : int {
    kEpiHidden = 0,    // z = C + b -> zout (FP32), gelu(z) -> hout (BF16)
    kEpiOutput = 1,    // z = C + b -> zout (FP32)
    kEpiBackAct = 2,   // dz = C * gelu'(zin) -> hout (BF16)
    kEpiStore = 3      // C -> zout (FP32)
};

template <int EPI>
__global__ void __launch_bounds__(64) gemm_bf16_kernel(int M, int N, int K, const uint16_t* __restrict__ A,
                                                       int64_t sam, int64_t sak, const uint16_t* __restrict__ B,
                                                       int64_t sbk, int64_t sbn, const float* __restrict__ bias,
                                                       const float* __restrict__ zin, float* __restrict__ zout,
                                                       uint16_t* __restrict__ hout, int ldo) {
    const int tm = blockIdx.x, tn = blockIdx.y;
    const int l = threadIdx.x;
    const int r16 = l & 15, q = l >> 4;
    const int am = tm * 16 + r16, bn = tn * 16 + r16;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + 4 * q + j;
            a[j] = (short)A[am * sam + k * sak];
            b[j] = (short)B[k * sbk + bn * sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = tm * 16 + 4 * q + j, n = tn * 16 + r16;
        const int64_t o = (int64_t)m * ldo + n;
        const float c = acc[j];
        if (EPI == kEpiHidden) {
            const float z = c + bias[n];
            zout[o] = z;
            hout[o] = to_bf16(gelu(z));
        } else if (EPI == kEpiOutput) {
            zout[o] = c + bias[n];
        } else if (EPI == kEpiBackAct) {
            hout[o] = to_bf16(c * gelu_grad(zin[o]));
        } else {
            zout[o] = c;
        }
    }
}

// x (FP32, [n x nin], row-major) -> h0 (BF16, [cap x d0]), zero padding
__global__ void input_kernel(const float* __restrict__ x, int n, int nin, int d0, int rows, uint16_t* __restrict__ h0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)rows * d0) return;
    const int r = (int)(t / d0), c = (int)(t % d0);
    h0[t] = (r < n && c < nin) ? to_bf16(x[(int64_t)r * nin + c]) : (uint16_t)0;
}

// y (FP32, [n x nout]) <- z_out
__global__ void output_kernel(const float* __restrict__ z, int n, int nout, int d, float* __restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nout) return;
    const int r = (int)(t / nout), c = (int)(t % nout);
    y[t] = z[(int64_t)r * d + c];
}

// dz_out = 2 (z - t) / (n nout) on the true rows and columns, 0 elsewhere (BF16 and FP32);
// per-block partial sums of (z - t)^2
__global__ void loss_grad_kernel(const float* __restrict__ z, const float* __restrict__ tg, int n, int nout, int d,
                                 int rows, uint16_t* __restrict__ dz, float* __restrict__ dzf,
                                 double* __restrict__ part) {
    __shared__ double sh[4];
    double acc = 0.0;
    const double scale = 2.0 / ((double)n * nout);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)rows * d;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t / d), c = (int)(t % d);
        float g = 0.f;
        if (r < n && c < nout) {
            const double e = (double)z[t] - (double)tg[(int64_t)r * nout + c];
            acc += e * e;
            g = (float)(scale * e);
        }
        dz[t] = to_bf16(g);
        dzf[t] = g;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// db[n] = sum over rows of dz[:, n] (BF16 gradient values), one block per column
__global__ void colsum_kernel(const uint16_t* __restrict__ dz, int rows, int d, float* __restrict__ db) {
    __shared__ float sh[4];
    const int n = blockIdx.x;
    float acc = 0.f;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) acc += from_bf16(dz[(int64_t)r * d + n]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) db[n] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, const uint8_t* __restrict__ live, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || !live[t]) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    w[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

__global__ void to_bf16_kernel(const float* __restrict__ w, int64_t n, uint16_t* __restrict__ o) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) o[t] = to_bf16(w[t]);
}

inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
inline int pad16(int x) { return (x + 15) / 16 * 16; }

}  // namespace

}  // namespace gp

using namespace gp;

namespace {

int mlp_fail(gplmm_mlp* m, const char* msg) {
    m->err = msg;
    return GPLMM_E_ARG;
}

#define MLP_HIP(m, call)                                           \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) {                                    \
            (m)->err = std::string("HIP: ") + hipGetErrorString(e_); \
            return GPLMM_E_HIP;                                    \
        }                                                          \
    } while (0)

// mask of the parameters that exist (not padding) in the padded layout
std::vector<uint8_t> live_mask(const gplmm_mlp* m) {
    std::vector<uint8_t> live(m->nparam, 0);
    const int L = m->nl + 1;
    for (int l = 0; l < L; ++l) {
        for (int i = 0; i < m->rdim[l]; ++i)
            for (int j = 0; j < m->rdim[l + 1]; ++j) live[m->woff[l] + (int64_t)i * m->dim[l + 1] + j] = 1;
        for (int j = 0; j < m->rdim[l + 1]; ++j) live[m->boff[l] + j] = 1;
    }
    return live;
}

// forward pass over rows [0, rows) of h0 (already filled)
int run_forward(gplmm_mlp* m, int rows) {
    const int L = m->nl + 1;
    for (int l = 0; l < L; ++l) {
        const int K = m->dim[l], N = m->dim[l + 1];
        dim3 grid(rows / 16, N / 16);
        const uint16_t* W = m->d_wbf + m->woff[l];
        const float* b = m->d_w + m->boff[l];
        if (l + 1 < L)
            gemm_bf16_kernel<kEpiHidden><<<grid, 64, 0, m->stream>>>(rows, N, K, m->d_h[l], K, 1, W, N, 1, b, nullptr,
                                                                     m->d_z[l + 1], m->d_h[l + 1], N);
        else
            gemm_bf16_kernel<kEpiOutput><<<grid, 64, 0, m->stream>>>(rows, N, K, m->d_h[l], K, 1, W, N, 1, b, nullptr,
                                                                     m->d_z[l + 1], nullptr, N);
    }
    MLP_HIP(m, hipGetLastError());
    return GPLMM_OK;
}

}  // namespace

extern "C" {

int gplmm_mlp_create(int nin, int nhidden, int nlayers, int nout, int max_batch, void* stream, gplmm_mlp** out) {
    if (!out) return GPLMM_E_ARG;
    *out = nullptr;
    if (nin < 1 || nhidden < 1 || nlayers < 1 || nout < 1 || max_batch < 1 || nin > 4096 || nhidden > 4096 ||
        nout > 4096 || nlayers > 16)
        return GPLMM_E_ARG;
    gplmm_mlp* m = new gplmm_mlp;
    m->nin = nin;
    m->nh = nhidden;
    m->nl = nlayers;
    m->nout = nout;
    m->cap = pad16(max_batch);
    m->stream = (hipStream_t)stream;
    m->rdim.push_back(nin);
    for (int l = 0; l < nlayers; ++l) m->rdim.push_back(nhidden);
    m->rdim.push_back(nout);
    for (int d : m->rdim) m->dim.push_back(pad16(d));
    const int L = nlayers + 1;
    int64_t off = 0;
    int maxd = 0;
    for (int l = 0; l < L; ++l) {
        m->woff.push_back(off);
        off += (int64_t)m->dim[l] * m->dim[l + 1];
        m->boff.push_back(off);
        off += m->dim[l + 1];
        maxd = std::max(maxd, m->dim[l + 1]);
    }
    m->nparam = off;
    *out = m;
    auto al = [&](void** p, size_t bytes) -> int {
        if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) return GPLMM_E_HIP;
        if (hipMemset(*p, 0, std::max<size_t>(bytes, 16)) != hipSuccess) return GPLMM_E_HIP;
        return GPLMM_OK;
    };
    int rc = GPLMM_OK;
    rc |= al((void**)&m->d_w, sizeof(float) * off);
    rc |= al((void**)&m->d_g, sizeof(float) * off);
    rc |= al((void**)&m->d_m, sizeof(float) * off);
    rc |= al((void**)&m->d_v, sizeof(float) * off);
    rc |= al((void**)&m->d_wbf, sizeof(uint16_t) * off);
    m->d_z.assign(L + 1, nullptr);
    m->d_h.assign(L, nullptr);
    for (int l = 0; l <= L; ++l) {
        if (l >= 1) rc |= al((void**)&m->d_z[l], sizeof(float) * (int64_t)m->cap * m->dim[l]);
        if (l < L) rc |= al((void**)&m->d_h[l], sizeof(uint16_t) * (int64_t)m->cap * m->dim[l]);
    }
    rc |= al((void**)&m->d_dz, sizeof(uint16_t) * (int64_t)m->cap * maxd);
    rc |= al((void**)&m->d_dz2, sizeof(uint16_t) * (int64_t)m->cap * maxd);
    rc |= al((void**)&m->d_red, sizeof(double) * kLossBlocks);
    rc |= al((void**)&m->d_live, (size_t)off);
    if (rc == GPLMM_OK) {
        std::vector<uint8_t> live = live_mask(m);
        if (hipMemcpy(m->d_live, live.data(), live.size(), hipMemcpyHostToDevice) != hipSuccess) rc = GPLMM_E_HIP;
    }
    if (hipHostMalloc((void**)&m->h_red, sizeof(double) * kLossBlocks, hipHostMallocDefault) != hipSuccess)
        rc = GPLMM_E_HIP;
    if (rc != GPLMM_OK) {
        m->err = "device allocation failed";
        return GPLMM_E_HIP;
    }
    return GPLMM_OK;
}

void gplmm_mlp_destroy(gplmm_mlp* m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    else (void)hipDeviceSynchronize();
    void* ps[] = {m->d_w, m->d_g, m->d_m, m->d_v, m->d_wbf, m->d_dz, m->d_dz2, m->d_red, m->d_live};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (float* p : m->d_z)
        if (p) (void)hipFree(p);
    for (uint16_t* p : m->d_h)
        if (p) (void)hipFree(p);
    if (m->h_red) (void)hipHostFree(m->h_red);
    delete m;
}

const char* gplmm_mlp_last_error(const gplmm_mlp* m) { return m ? m->err.c_str() : "null model"; }

}  // extern "C"

namespace gp {
int mlp_width_in(const gplmm_mlp* m) { return m ? m->nin : -1; }
int mlp_width_out(const gplmm_mlp* m) { return m ? m->nout : -1; }
}  // namespace gp

extern "C" {

int64_t gplmm_mlp_num_params(const gplmm_mlp* m) {
    if (!m) return -1;
    int64_t n = 0;
    for (int l = 0; l + 1 < (int)m->rdim.size(); ++l) n += (int64_t)m->rdim[l] * m->rdim[l + 1] + m->rdim[l + 1];
    return n;
}

// Packed host layout: for each layer, W (fan_in x fan_out, row-major) then b (fan_out).
static int pack_io(gplmm_mlp* m, float* host, const float* dev_src, bool to_host) {
    std::vector<float> pad(m->nparam, 0.f);
    if (to_host) MLP_HIP(m, hipMemcpy(pad.data(), dev_src, sizeof(float) * m->nparam, hipMemcpyDeviceToHost));
    int64_t p = 0;
    const int L = m->nl + 1;
    for (int l = 0; l < L; ++l) {
        for (int i = 0; i < m->rdim[l]; ++i)
            for (int j = 0; j < m->rdim[l + 1]; ++j) {
                float& d = pad[m->woff[l] + (int64_t)i * m->dim[l + 1] + j];
                if (to_host) host[p++] = d; else d = host[p++];
            }
        for (int j = 0; j < m->rdim[l + 1]; ++j) {
            float& d = pad[m->boff[l] + j];
            if (to_host) host[p++] = d; else d = host[p++];
        }
    }
    if (!to_host) {
        MLP_HIP(m, hipMemcpy(m->d_w, pad.data(), sizeof(float) * m->nparam, hipMemcpyHostToDevice));
        to_bf16_kernel<<<blocks(m->nparam), 256, 0, m->stream>>>(m->d_w, m->nparam, m->d_wbf);
        MLP_HIP(m, hipGetLastError());
        MLP_HIP(m, hipMemsetAsync(m->d_m, 0, sizeof(float) * m->nparam, m->stream));
        MLP_HIP(m, hipMemsetAsync(m->d_v, 0, sizeof(float) * m->nparam, m->stream));
        m->adam_t = 0;
        MLP_HIP(m, hipStreamSynchronize(m->stream));
    }
    return GPLMM_OK;
}

int gplmm_mlp_set_params(gplmm_mlp* m, const float* host) {
    if (!m || !host) return GPLMM_E_ARG;
    return pack_io(m, const_cast<float*>(host), nullptr, false);
}

int gplmm_mlp_get_params(gplmm_mlp* m, float* host) {
    if (!m || !host) return GPLMM_E_ARG;
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    return pack_io(m, host, m->d_w, true);
}

int gplmm_mlp_forward(gplmm_mlp* m, const float* x, int n, float* y) {
    if (!m || !x || !y || n < 0) return GPLMM_E_ARG;
    for (int r0 = 0; r0 < n; r0 += m->cap) {
        const int nb = std::min(m->cap, n - r0), rows = pad16(nb);
        input_kernel<<<blocks((int64_t)rows * m->dim[0]), 256, 0, m->stream>>>(x + (int64_t)r0 * m->nin, nb, m->nin,
                                                                               m->dim[0], rows, m->d_h[0]);
        int rc = run_forward(m, rows);
        if (rc) return rc;
        output_kernel<<<blocks((int64_t)nb * m->nout), 256, 0, m->stream>>>(m->d_z[m->nl + 1], nb, m->nout,
                                                                           m->dim[m->nl + 1], y + (int64_t)r0 * m->nout);
    }
    MLP_HIP(m, hipGetLastError());
    return GPLMM_OK;
}

// Loss and gradient of the MSE over one batch (n <= capacity); gradients stay on the device
// (and are copied to grad_host, packed, when it is not NULL).
int gplmm_mlp_grad(gplmm_mlp* m, const float* x, const float* t, int n, double* loss, float* grad_host) {
    if (!m || !x || !t || n < 1) return GPLMM_E_ARG;
    if (n > m->cap) return mlp_fail(m, "batch larger than the capacity given at creation");
    const int rows = pad16(n);
    const int L = m->nl + 1;
    input_kernel<<<blocks((int64_t)rows * m->dim[0]), 256, 0, m->stream>>>(x, n, m->nin, m->dim[0], rows, m->d_h[0]);
    int rc = run_forward(m, rows);
    if (rc) return rc;
    // output layer gradient (FP32 copy kept in d_z[L] is not needed afterwards: reuse it)
    float* dzf = m->d_z[L];
    loss_grad_kernel<<<kLossBlocks, 256, 0, m->stream>>>(m->d_z[L], t, n, m->nout, m->dim[L], rows, m->d_dz, dzf,
                                                         m->d_red);
    uint16_t* dz = m->d_dz;
    uint16_t* dzn = m->d_dz2;
    for (int l = L - 1; l >= 0; --l) {
        const int K = m->dim[l], N = m->dim[l + 1];
        // dW_l = h_l^T dz  (M = K, N = N, sum over rows)
        gemm_bf16_kernel<kEpiStore><<<dim3(K / 16, N / 16), 64, 0, m->stream>>>(
            K, N, rows, m->d_h[l], 1, K, dz, N, 1, nullptr, nullptr, m->d_g + m->woff[l], nullptr, N);
        colsum_kernel<<<N, 256, 0, m->stream>>>(dz, rows, N, m->d_g + m->boff[l]);
        if (l > 0) {
            // dz_{l-1} = (dz W_l^T) * gelu'(z_l-1)
            gemm_bf16_kernel<kEpiBackAct><<<dim3(rows / 16, K / 16), 64, 0, m->stream>>>(
                rows, K, N, dz, N, 1, m->d_wbf + m->woff[l], 1, N, nullptr, m->d_z[l], nullptr, dzn, K);
            std::swap(dz, dzn);
        }
    }
    MLP_HIP(m, hipGetLastError());
    MLP_HIP(m, hipMemcpyAsync(m->h_red, m->d_red, sizeof(double) * kLossBlocks, hipMemcpyDeviceToHost, m->stream));
    MLP_HIP(m, hipStreamSynchronize(m->stream));
    if (loss) {
        double s = 0.0;
        for (int b = 0; b < kLossBlocks; ++b) s += m->h_red[b];
        *loss = s / ((double)n * m->nout);
    }
    if (grad_host) return pack_io(m, grad_host, m->d_g, true);
    return GPLMM_OK;
}

int gplmm_mlp_adam(gplmm_mlp* m, double lr, double b1, double b2, double eps) {
    if (!m) return GPLMM_E_ARG;
    m->adam_t++;
    const float c1 = (float)(1.0 - std::pow(b1, m->adam_t)), c2 = (float)(1.0 - std::pow(b2, m->adam_t));
    adam_kernel<<<blocks(m->nparam), 256, 0, m->stream>>>(m->d_w, m->d_g, m->d_m, m->d_v, m->d_live, m->nparam,
                                                          (float)lr, (float)b1, (float)b2, (float)eps, c1, c2);
    to_bf16_kernel<<<blocks(m->nparam), 256, 0, m->stream>>>(m->d_w, m->nparam, m->d_wbf);
    MLP_HIP(m, hipGetLastError());
    return GPLMM_OK;
}

// Minibatch Adam over n samples in the given order (the caller shuffles), `epochs`
// passes; *loss_out = mean of the last epoch's batch losses.
int gplmm_mlp_train(gplmm_mlp* m, const float* x, const float* t, int n, int epochs, int batch, double lr,
                    double* loss_out) {
    if (!m || !x || !t || n < 1 || epochs < 1 || batch < 1) return GPLMM_E_ARG;
    batch = std::min(batch, m->cap);
    double last = 0.0;
    for (int e = 0; e < epochs; ++e) {
        double sum = 0.0;
        int nb = 0;
        for (int r0 = 0; r0 < n; r0 += batch) {
            const int k = std::min(batch, n - r0);
            double l = 0.0;
            int rc = gplmm_mlp_grad(m, x + (int64_t)r0 * m->nin, t + (int64_t)r0 * m->nout, k, &l, nullptr);
            if (rc) return rc;
            rc = gplmm_mlp_adam(m, lr, 0.9, 0.999, 1e-8);
            if (rc) return rc;
            sum += l;
            ++nb;
        }
        last = sum / std::max(nb, 1);
    }
    if (loss_out) *loss_out = last;
    return GPLMM_OK;
}

}  // extern "C"

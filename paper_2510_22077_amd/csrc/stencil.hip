// MAC stencils on the cell-record layout (one thread per fluid cell).
//
// Paper: governing equations (Section 1) discretised on the MAC grid
// (Section 2); the Newton Jacobian J = dr/dx (Section 1); the gPLMM build
// matrix X = J~_w, the Jacobian of the modified residual with the inertia
// linearised about the wind w and switched off on tagged faces (Section 4).
//
// Discretisation (the paper gives none; the same reading as the oracle):
// viscous -(mu/h^2) sum_nb (g - u_F) over the 2*ndim neighbour faces, with
// g = neighbour value if active, 0 on a grain surface (the neighbour face
// touches a fluid cell), -u_F when both cells of the neighbour face are
// grain (wall half a cell away); first-order upwind inertia
// rho * sum_d a_d D_d u with a_x = u_F and transverse a_d the mean of the four
// d-faces of the face's two cells; gradient (p_R - p_L)/h; mass row -div u;
// the pinned cell's mass row (one per sample of a batch) is p = 0.
//
// X is fixed between builds, so its momentum rows are tabulated once per build
// (kNC coefficients per face, structure of arrays over cells); X v is then a
// gather over the face's stencil with no classification work.  The Newton
// Jacobian changes with every Newton iterate and is applied matrix-free.
#include "internal.h"
#include "stencil_dev.h"

namespace gp {

namespace {

constexpr int kBlock = 512;   // largest block size the stencil kernels are compiled for

// r(x): momentum and mass residual.
template <int ND, bool kTagged>
__global__ void __launch_bounds__(kBlock) residual_kernel(DevGeo g, Phys ph0, const double* __restrict__ x,
                                                          const double* __restrict__ xold, double* __restrict__ r) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    double out[ND + 1];
    residual_cell<ND, kTagged>(g, ph0, x, xold, c, out);
#pragma unroll
    for (int a = 0; a <= ND; ++a) r[(ND + 1) * c + a] = out[a];
}

// y = J(xk) v with the upwind branches frozen at xk.  kTagged: the Jacobian of the
// residual without inertia on tagged faces (coarse-scale solver).
template <int ND, bool kTagged>
__global__ void __launch_bounds__(kBlock) jv_kernel(DevGeo g, Phys ph0, const double* __restrict__ xk,
                                                    const double* __restrict__ v, double* __restrict__ y) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Phys ph = cell_phys(g, ph0, c);
    constexpr int nr = ND + 1;
    const Nb<ND> nc = load_nb<ND>(g, c);
    const double ih = 1.0 / g.h, vis = ph.mu * ih * ih;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        double out = 0.0;
        const int32_t L = nc.n[a][0];
        if (L >= 0) {
            const Nb<ND> nl = load_nb<ND>(g, L);
            const FaceNb<ND> f = face_nb(nc, nl, a);
            const double uF = xk[nr * c + a], vF = v[nr * c + a];
            double visc = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int t = 0; t < 2; ++t) visc += vF - nb_value(f, d, t, v, nr, a, vF);
            out = vis * visc + (v[nr * c + ND] - v[(int64_t)nr * L + ND]) * ih;
            if (ph.dt > 0.0) out += ph.rho * vF / ph.dt;
            if (!kTagged || !((g.tag[c] >> a) & 1u)) {
                double conv = 0.0;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    const double ad = advecting(nc, nl, c, L, a, d, xk, nr);
                    const double adv = advecting(nc, nl, c, L, a, d, v, nr);
                    const int t = ad >= 0.0 ? 0 : 1;
                    const double gu = nb_value(f, d, t, xk, nr, a, uF), gv = nb_value(f, d, t, v, nr, a, vF);
                    const double Du = t == 0 ? uF - gu : gu - uF;
                    const double Dv = t == 0 ? vF - gv : gv - vF;
                    conv += (ad * Dv + adv * Du) * ih;
                }
                out += ph.rho * conv;
            }
        }
        y[nr * c + a] = out;
    }
    double m;
    if ((g.tag[c] & kPinBit)) {
        m = v[nr * c + ND];
    } else {
        m = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            const double up = nc.n[a][1] >= 0 ? v[(int64_t)nr * nc.n[a][1] + a] : 0.0;
            const double lo = nc.n[a][0] >= 0 ? v[nr * c + a] : 0.0;
            m -= (up - lo) * ih;
        }
    }
    y[nr * c + ND] = m;
}

// Momentum rows of the build matrix: coef[(k * ND + a) * ncell + c], k = 0 diagonal,
// k = 1 + 2 d + t neighbour face (d, t); all zero for an inactive face.  kJac = false:
// X = J~_w (Section 4: Oseen with wind w, no inertia on tagged faces); kJac = true: the
// Newton Jacobian J(w) at the state w (no tags), with its transverse slots.  FP64 and,
// if cf32 != nullptr, FP32.
template <int ND, bool kJac>
__global__ void __launch_bounds__(kBlock) xcoef_kernel(DevGeo g, Phys ph0, const double* __restrict__ wind,
                                                       double* __restrict__ cf64, float* __restrict__ cf32) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Phys ph = cell_phys(g, ph0, c);
    constexpr int nr = ND + 1;
    constexpr int ns = coef_slots<ND>(kJac);
    const Nb<ND> nc = load_nb<ND>(g, c);
    const int64_t nce = g.ncell;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        double co[ns > kNC ? ns : kNC];   // x_face_coefs fills kNC slots
#pragma unroll
        for (int k = 0; k < (ns > kNC ? ns : kNC); ++k) co[k] = 0.0;
        const int32_t L = nc.n[a][0];
        if (L >= 0) {
            const Nb<ND> nl = load_nb<ND>(g, L);
            const FaceNb<ND> f = face_nb(nc, nl, a);
            const bool tagged = !kJac && ((g.tag[c] >> a) & 1u);
            x_face_coefs(ph, g.h, nc, nl, f, c, a, tagged ? (const double*)nullptr : wind, nr, co);
            if (kJac) jac_extra<ND>(ph, g.h, nc, nl, f, c, a, wind, nr, co);
        }
#pragma unroll
        for (int k = 0; k < ns; ++k) {
            cf64[(k * ND + a) * nce + c] = co[k];
            if (cf32) cf32[(k * ND + a) * nce + c] = (float)co[k];
        }
    }
}

// y = a - A b  (a == nullptr: y = A b) from the tabulated rows of the build matrix A.
template <int ND, typename T, bool kJac>
__global__ void __launch_bounds__(kBlock) xv_kernel(DevGeo g, const T* __restrict__ coef, const T* __restrict__ a,
                                                    const T* __restrict__ b, T* __restrict__ y) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    constexpr int nr = ND + 1;
    const Nb<ND> nc = load_nb<ND>(g, c);
    const int64_t nce = g.ncell;
    const T ih = (T)(1.0 / g.h);
    const T pc = b[nr * c + ND];
#pragma unroll
    for (int ax = 0; ax < ND; ++ax) {
        const int64_t s = nr * c + ax;
        T acc = 0;
        const int32_t L = nc.n[ax][0];
        if (L >= 0) {
            acc = coef[ax * nce + c] * b[s] + ih * (pc - b[(int64_t)nr * L + ND]);
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const T w = coef[((1 + 2 * d + t) * ND + ax) * nce + c];
                    const int32_t P = nc.n[d][t];   // (ax, t = 0) -> L itself
                    if (w != (T)0 && P >= 0) acc += w * b[(int64_t)nr * P + ax];
                }
            if (kJac) {
                const Nb<ND> nl = load_nb<ND>(g, L);
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    if (d == ax) continue;
                    const int dd = d < ax ? d : d - 1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const T w = coef[((1 + 2 * ND + 4 * dd + q) * ND + ax) * nce + c];
                        if (w != (T)0) acc += w * b[(int64_t)nr * jac_col_cell<ND>(nc, nl, c, L, d, q) + d];
                    }
                }
            }
        }
        y[s] = a ? (T)(a[s] - acc) : acc;
    }
    T m;
    if ((g.tag[c] & kPinBit)) {
        m = pc;
    } else {
        m = 0;
#pragma unroll
        for (int ax = 0; ax < ND; ++ax) {
            if (nc.n[ax][0] >= 0) m += ih * b[nr * c + ax];
            if (nc.n[ax][1] >= 0) m -= ih * b[(int64_t)nr * nc.n[ax][1] + ax];
        }
    }
    const int64_t s = nr * c + ND;
    y[s] = a ? (T)(a[s] - m) : m;
}

// y = X b for kProbeColors vectors interleaved per slot (vector q of slot s at s K + q,
// FP64): the operation of xv_kernel with a = nullptr on each vector, in the same order, the
// tabulated coefficients and the neighbour table read once and each neighbour's K values
// read as one contiguous 64-byte run (the probing of the coarse operator).
template <int ND, bool kJac>
__global__ void __launch_bounds__(kBlock) xv_multi_kernel(DevGeo g, const double* __restrict__ coef,
                                                          const double* __restrict__ b, double* __restrict__ y) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    constexpr int nr = ND + 1;
    constexpr int K = kProbeColors;
    const Nb<ND> nc = load_nb<ND>(g, c);
    const int64_t nce = g.ncell;
    const double ih = 1.0 / g.h;
    auto ldv = [&](int64_t slot, double (&out)[K]) {
#pragma unroll
        for (int q = 0; q < K; ++q) out[q] = b[slot * K + q];
    };
    double pc[K];
    ldv(nr * c + ND, pc);
#pragma unroll
    for (int ax = 0; ax < ND; ++ax) {
        const int64_t s = nr * c + ax;
        double acc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] = 0.0;
        const int32_t L = nc.n[ax][0];
        if (L >= 0) {
            const double cd = coef[ax * nce + c];
            double bs[K], bl[K];
            ldv(s, bs);
            ldv((int64_t)nr * L + ND, bl);
#pragma unroll
            for (int q = 0; q < K; ++q) acc[q] = cd * bs[q] + ih * (pc[q] - bl[q]);
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const double w = coef[((1 + 2 * d + t) * ND + ax) * nce + c];
                    const int32_t P = nc.n[d][t];
                    if (w != 0.0 && P >= 0) {
                        double bp[K];
                        ldv((int64_t)nr * P + ax, bp);
#pragma unroll
                        for (int q = 0; q < K; ++q) acc[q] += w * bp[q];
                    }
                }
            if (kJac) {
                const Nb<ND> nl = load_nb<ND>(g, L);
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    if (d == ax) continue;
                    const int dd = d < ax ? d : d - 1;
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) {
                        const double w = coef[((1 + 2 * ND + 4 * dd + q4) * ND + ax) * nce + c];
                        if (w != 0.0) {
                            double bj[K];
                            ldv((int64_t)nr * jac_col_cell<ND>(nc, nl, c, L, d, q4) + d, bj);
#pragma unroll
                            for (int q = 0; q < K; ++q) acc[q] += w * bj[q];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) y[s * K + q] = acc[q];
    }
    const int64_t sp = nr * c + ND;
    if ((g.tag[c] & kPinBit)) {
#pragma unroll
        for (int q = 0; q < K; ++q) y[sp * K + q] = pc[q];
    } else {
        double m[K];
#pragma unroll
        for (int q = 0; q < K; ++q) m[q] = 0.0;
#pragma unroll
        for (int ax = 0; ax < ND; ++ax) {
            if (nc.n[ax][0] >= 0) {
                double bv[K];
                ldv(nr * c + ax, bv);
#pragma unroll
                for (int q = 0; q < K; ++q) m[q] += ih * bv[q];
            }
            if (nc.n[ax][1] >= 0) {
                double bv[K];
                ldv((int64_t)nr * nc.n[ax][1] + ax, bv);
#pragma unroll
                for (int q = 0; q < K; ++q) m[q] -= ih * bv[q];
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) y[sp * K + q] = m[q];
    }
}

// y = Xcheck b, the rows of Eq. iMG's column-summed operator that the restriction Rhat
// reads (Section 3.2.2): a row of a primary's unknown keeps its columns in that primary
// and on interface cells, an interface cell's mass row keeps every column but the
// f-faces; each dropped column's coefficient is added to the row's diagonal (both
// reduction steps), except on faces of wall-free groups, which drop it.  Every other row
// (f-faces, inactive faces) is zero.  cls: per slot, owner primary, -1 f-face, -4
// interface cell; keep: per slot, 1 = no diagonal sums.
template <int ND, bool kJac>
__global__ void __launch_bounds__(kBlock) xcheck_kernel(DevGeo g, const double* __restrict__ coef,
                                                        const int32_t* __restrict__ cls,
                                                        const uint8_t* __restrict__ keep,
                                                        const double* __restrict__ b, double* __restrict__ y) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    constexpr int nr = ND + 1;
    const Nb<ND> nc = load_nb<ND>(g, c);
    const int64_t nce = g.ncell;
    const double ih = 1.0 / g.h;
#pragma unroll
    for (int ax = 0; ax <= ND; ++ax) {
        const int64_t s = nr * c + ax;
        const int32_t rc = cls[s];
        const bool prow = rc >= 0, crow = rc == -4;
        double acc = 0.0, dsum = 0.0;
        auto add = [&](int64_t col, double w) {
            const int32_t cc = cls[col];
            const bool kept = prow ? (cc == rc || cc == -4) : cc != -1;
            if (kept) acc += w * b[col];
            else dsum += w;
        };
        if (!(prow || crow)) {
            y[s] = 0.0;
            continue;
        }
        if (ax < ND) {
            const int32_t L = nc.n[ax][0];
            if (L >= 0) {
                acc = coef[ax * nce + c] * b[s];
                add(nr * c + ND, ih);
                add((int64_t)nr * L + ND, -ih);
#pragma unroll
                for (int d = 0; d < ND; ++d)
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const double w = coef[((1 + 2 * d + t) * ND + ax) * nce + c];
                        const int32_t P = nc.n[d][t];
                        if (w != 0.0 && P >= 0) add((int64_t)nr * P + ax, w);
                    }
                if (kJac) {
                    const Nb<ND> nl = load_nb<ND>(g, L);
#pragma unroll
                    for (int d = 0; d < ND; ++d) {
                        if (d == ax) continue;
                        const int dd = d < ax ? d : d - 1;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const double w = coef[((1 + 2 * ND + 4 * dd + q) * ND + ax) * nce + c];
                            if (w != 0.0) add((int64_t)nr * jac_col_cell<ND>(nc, nl, c, L, d, q) + d, w);
                        }
                    }
                }
            }
        } else if ((g.tag[c] & kPinBit)) {
            acc = b[s];
        } else {
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                if (nc.n[d][0] >= 0) add(nr * c + d, ih);
                if (nc.n[d][1] >= 0) add((int64_t)nr * nc.n[d][1] + d, -ih);
            }
        }
        y[s] = keep[s] ? acc : acc + dsum * b[s];
    }
}

// b_B = -r(u = 0, p = 0) of the steady equations: rho * body on every active face.
template <int ND>
__global__ void bB_kernel(DevGeo g, Phys ph0, double* __restrict__ out) {
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    const Phys ph = cell_phys(g, ph0, c);
    constexpr int nr = ND + 1;
    const Nb<ND> nc = load_nb<ND>(g, c);
#pragma unroll
    for (int a = 0; a < ND; ++a) out[nr * c + a] = nc.n[a][0] >= 0 ? ph.rho * ph.body[a] : 0.0;
    out[nr * c + ND] = 0.0;
}

inline dim3 grid_for(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

void launch_residual(gplmm_ctx* c, const double* x, const double* xprev, double* r, hipStream_t s, bool tagged) {
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    if (c->ndim == 3) {
        if (tagged) residual_kernel<3, true><<<gr, b, 0, s>>>(c->geo, c->phys, x, xprev, r);
        else residual_kernel<3, false><<<gr, b, 0, s>>>(c->geo, c->phys, x, xprev, r);
    } else {
        if (tagged) residual_kernel<2, true><<<gr, b, 0, s>>>(c->geo, c->phys, x, xprev, r);
        else residual_kernel<2, false><<<gr, b, 0, s>>>(c->geo, c->phys, x, xprev, r);
    }
}

void launch_jv(gplmm_ctx* c, const double* xk, const double* v, double* y, hipStream_t s, bool tagged) {
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    if (c->ndim == 3) {
        if (tagged) jv_kernel<3, true><<<gr, b, 0, s>>>(c->geo, c->phys, xk, v, y);
        else jv_kernel<3, false><<<gr, b, 0, s>>>(c->geo, c->phys, xk, v, y);
    } else {
        if (tagged) jv_kernel<2, true><<<gr, b, 0, s>>>(c->geo, c->phys, xk, v, y);
        else jv_kernel<2, false><<<gr, b, 0, s>>>(c->geo, c->phys, xk, v, y);
    }
}

void launch_xcoef(gplmm_ctx* c, hipStream_t s) {
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
    if (c->ndim == 3) {
        if (jac) xcoef_kernel<3, true><<<gr, b, 0, s>>>(c->geo, c->phys, c->d_wind, c->d_xcoef, c->d_xcoef_f);
        else xcoef_kernel<3, false><<<gr, b, 0, s>>>(c->geo, c->phys, c->d_wind, c->d_xcoef, c->d_xcoef_f);
    } else {
        if (jac) xcoef_kernel<2, true><<<gr, b, 0, s>>>(c->geo, c->phys, c->d_wind, c->d_xcoef, c->d_xcoef_f);
        else xcoef_kernel<2, false><<<gr, b, 0, s>>>(c->geo, c->phys, c->d_wind, c->d_xcoef, c->d_xcoef_f);
    }
}

template <typename T>
static const T* xcoef_table(gplmm_ctx* c);
template <>
const double* xcoef_table<double>(gplmm_ctx* c) { return c->d_xcoef; }
template <>
const float* xcoef_table<float>(gplmm_ctx* c) { return c->d_xcoef_f; }

template <typename T>
void launch_xv(gplmm_ctx* c, const T* v, T* y, const T* sub_from, hipStream_t s) {
    const T* cf = xcoef_table<T>(c);
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
    if (c->ndim == 3) {
        if (jac) xv_kernel<3, T, true><<<gr, b, 0, s>>>(c->geo, cf, sub_from, v, y);
        else xv_kernel<3, T, false><<<gr, b, 0, s>>>(c->geo, cf, sub_from, v, y);
    } else {
        if (jac) xv_kernel<2, T, true><<<gr, b, 0, s>>>(c->geo, cf, sub_from, v, y);
        else xv_kernel<2, T, false><<<gr, b, 0, s>>>(c->geo, cf, sub_from, v, y);
    }
}

void launch_xcheck_v(gplmm_ctx* c, const double* v, double* y, hipStream_t s) {
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
    const double* cf = c->d_xcoef;
    if (c->ndim == 3) {
        if (jac) xcheck_kernel<3, true><<<gr, b, 0, s>>>(c->geo, cf, c->d_slot_class, c->d_noclose, v, y);
        else xcheck_kernel<3, false><<<gr, b, 0, s>>>(c->geo, cf, c->d_slot_class, c->d_noclose, v, y);
    } else {
        if (jac) xcheck_kernel<2, true><<<gr, b, 0, s>>>(c->geo, cf, c->d_slot_class, c->d_noclose, v, y);
        else xcheck_kernel<2, false><<<gr, b, 0, s>>>(c->geo, cf, c->d_slot_class, c->d_noclose, v, y);
    }
}

void launch_xv_multi(gplmm_ctx* c, const double* v, double* y, hipStream_t s) {
    const dim3 gr = grid_for(c->ncell, c->stencil_block);
    const int b = c->stencil_block;
    const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
    const double* cf = c->d_xcoef;
    if (c->ndim == 3) {
        if (jac) xv_multi_kernel<3, true><<<gr, b, 0, s>>>(c->geo, cf, v, y);
        else xv_multi_kernel<3, false><<<gr, b, 0, s>>>(c->geo, cf, v, y);
    } else {
        if (jac) xv_multi_kernel<2, true><<<gr, b, 0, s>>>(c->geo, cf, v, y);
        else xv_multi_kernel<2, false><<<gr, b, 0, s>>>(c->geo, cf, v, y);
    }
}

void launch_bB(gplmm_ctx* c, double* bB, hipStream_t s) {
    if (c->ndim == 3) bB_kernel<3><<<grid_for(c->ncell, c->stencil_block), c->stencil_block, 0, s>>>(c->geo, c->phys, bB);
    else bB_kernel<2><<<grid_for(c->ncell, c->stencil_block), c->stencil_block, 0, s>>>(c->geo, c->phys, bB);
}

template void launch_xv<float>(gplmm_ctx*, const float*, float*, const float*, hipStream_t);
template void launch_xv<double>(gplmm_ctx*, const double*, double*, const double*, hipStream_t);

}  // namespace gp

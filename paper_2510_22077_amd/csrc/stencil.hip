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
// the pinned cell's mass row is p = 0.
#include "internal.h"
#include "stencil_dev.h"

namespace gp {

namespace {

constexpr int kBlock = 256;

// r(x): momentum and mass residual.
__global__ void residual_kernel(DevGeo g, Phys ph, const double* __restrict__ x,
                                const double* __restrict__ xold, double* __restrict__ r) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    Nbhd nb;
    load_nbhd(g, c, nb);
    const int nd = g.ndim, nr = g.nrec;
    const double h = g.h, ih = 1.0 / h, vis = ph.mu / (h * h);
    for (int a = 0; a < nd; ++a) {
        double out = 0.0;
        if (nb.L[a] >= 0) {
            const double uF = x[nr * c + a];
            FaceKinds fk;
            classify(g, nb, a, fk);
            double visc = 0.0;
            for (int d = 0; d < nd; ++d)
                for (int t = 0; t < 2; ++t) visc += uF - nbval(fk, d, t, x, nr, a, uF);
            out = vis * visc + (x[nr * c + nd] - x[nr * (int64_t)nb.L[a] + nd]) * ih - ph.rho * ph.body[a];
            if (ph.dt > 0.0) out += ph.rho * (uF - (xold ? xold[nr * c + a] : 0.0)) / ph.dt;
            double conv = 0.0;
            for (int d = 0; d < nd; ++d) {
                double ad = advecting(g, nb, a, d, x, c);
                double gm = nbval(fk, d, 0, x, nr, a, uF), gp_ = nbval(fk, d, 1, x, nr, a, uF);
                conv += ad * (ad >= 0.0 ? (uF - gm) : (gp_ - uF)) * ih;
            }
            out += ph.rho * conv;
        }
        r[nr * c + a] = out;
    }
    double m;
    if (c == g.pin) {
        m = x[nr * c + nd];
    } else {
        m = 0.0;
        for (int a = 0; a < nd; ++a) {
            double up = nb.n[a][1] >= 0 ? x[nr * (int64_t)nb.n[a][1] + a] : 0.0;
            double lo = nb.L[a] >= 0 ? x[nr * c + a] : 0.0;
            m -= (up - lo) * ih;
        }
    }
    r[nr * c + nd] = m;
}

// y = J(xk) v with upwind branches frozen at xk.
__global__ void jv_kernel(DevGeo g, Phys ph, const double* __restrict__ xk, const double* __restrict__ v,
                          double* __restrict__ y) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    Nbhd nb;
    load_nbhd(g, c, nb);
    const int nd = g.ndim, nr = g.nrec;
    const double h = g.h, ih = 1.0 / h, vis = ph.mu / (h * h);
    for (int a = 0; a < nd; ++a) {
        double out = 0.0;
        if (nb.L[a] >= 0) {
            const double uF = xk[nr * c + a], vF = v[nr * c + a];
            FaceKinds fk;
            classify(g, nb, a, fk);
            double visc = 0.0;
            for (int d = 0; d < nd; ++d)
                for (int t = 0; t < 2; ++t) visc += vF - nbval(fk, d, t, v, nr, a, vF);
            out = vis * visc + (v[nr * c + nd] - v[nr * (int64_t)nb.L[a] + nd]) * ih;
            if (ph.dt > 0.0) out += ph.rho * vF / ph.dt;
            double conv = 0.0;
            for (int d = 0; d < nd; ++d) {
                double ad = advecting(g, nb, a, d, xk, c);
                double adv = advecting(g, nb, a, d, v, c);
                bool bw = ad >= 0.0;
                double Du = bw ? (uF - nbval(fk, d, 0, xk, nr, a, uF)) : (nbval(fk, d, 1, xk, nr, a, uF) - uF);
                double Dv = bw ? (vF - nbval(fk, d, 0, v, nr, a, vF)) : (nbval(fk, d, 1, v, nr, a, vF) - vF);
                conv += (ad * Dv + adv * Du) * ih;
            }
            out += ph.rho * conv;
        }
        y[nr * c + a] = out;
    }
    double m;
    if (c == g.pin) {
        m = v[nr * c + nd];
    } else {
        m = 0.0;
        for (int a = 0; a < nd; ++a) {
            double up = nb.n[a][1] >= 0 ? v[nr * (int64_t)nb.n[a][1] + a] : 0.0;
            double lo = nb.L[a] >= 0 ? v[nr * c + a] : 0.0;
            m -= (up - lo) * ih;
        }
    }
    y[nr * c + nd] = m;
}

// y = a - X b  (a == nullptr: y = X b), X = J~_w with tags; T = float or double.
template <typename T, typename W>
__global__ void xv_kernel(DevGeo g, Phys ph, const W* __restrict__ wind, const T* __restrict__ a,
                          const T* __restrict__ b, T* __restrict__ y) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    Nbhd nb;
    load_nbhd(g, c, nb);
    const int nr = g.nrec;
    for (int comp = 0; comp < nr; ++comp) {
        int64_t cols[kMaxRow];
        double vals[kMaxRow];
        int cnt = x_row(g, ph, nb, c, comp, wind, cols, vals);
        T acc = 0;
        for (int k = 0; k < cnt; ++k) acc += (T)vals[k] * b[cols[k]];
        int64_t s = (int64_t)nr * c + comp;
        y[s] = a ? (T)(a[s] - acc) : acc;
    }
}

// b_B = -r(u = 0, p = 0) of the steady equations: rho * body on every active face.
__global__ void bB_kernel(DevGeo g, Phys ph, double* __restrict__ out) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.ncell) return;
    Nbhd nb;
    load_nbhd(g, c, nb);
    for (int a = 0; a < g.ndim; ++a) out[g.nrec * c + a] = nb.L[a] >= 0 ? ph.rho * ph.body[a] : 0.0;
    out[g.nrec * c + g.ndim] = 0.0;
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

void launch_residual(gplmm_ctx* c, const double* x, const double* xprev, double* r, hipStream_t s) {
    residual_kernel<<<grid_for(c->ncell), kBlock, 0, s>>>(c->geo, c->phys, x, xprev, r);
}

void launch_jv(gplmm_ctx* c, const double* xk, const double* v, double* y, hipStream_t s) {
    jv_kernel<<<grid_for(c->ncell), kBlock, 0, s>>>(c->geo, c->phys, xk, v, y);
}

template <typename T>
void launch_xv(gplmm_ctx* c, const T* v, T* y, const T* sub_from, hipStream_t s) {
    xv_kernel<T, double><<<grid_for(c->ncell), kBlock, 0, s>>>(c->geo, c->phys, c->d_wind, sub_from, v, y);
}

void launch_bB(gplmm_ctx* c, double* bB, hipStream_t s) {
    bB_kernel<<<grid_for(c->ncell), kBlock, 0, s>>>(c->geo, c->phys, bB);
}

template void launch_xv<float>(gplmm_ctx*, const float*, float*, const float*, hipStream_t);
template void launch_xv<double>(gplmm_ctx*, const double*, double*, const double*, hipStream_t);

}  // namespace gp

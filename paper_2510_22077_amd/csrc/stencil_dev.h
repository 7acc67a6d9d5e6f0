// Device helpers for the MAC stencils on the cell-record layout: the neighbour
// faces of a face and their kind, the advecting velocities, and the
// coefficients of one momentum row of the build matrix X.
//
// Neighbourhoods come from the per-cell table nb6[6 c + 2 d + t] = the fluid
// cell c -/+ e_d (periodic wrap applied) or -1.  The neighbour faces of the
// lower a-face of cell C (between L = C - e_a and C) are lower a-faces of L,
// of C + e_a and of C -/+ e_d, so C's and L's table rows describe the whole
// stencil.
#pragma once

#include "internal.h"

namespace gp {

enum : int { kActive = 0, kZero = 1, kGhost = 2 };

// The chip hands workgroups to its eight XCDs round-robin (workgroup i to XCD i % 8), and
// each XCD has its own L2.  A one-thread-per-cell stencil reads the records of the
// neighbouring cells, which belong to neighbouring workgroups; renumbering the
// workgroups so that XCD x works on one contiguous range of cells keeps those
// neighbours in the same L2 (round-robin order left every neighbour row on another
// XCD: the Jacobian stencil fetched 12x its algorithmic bytes from beyond L2).
// A bijection of [0, n) onto itself.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t n) {
    const int64_t q = n / kXcds, r = n % kXcds;
    const int64_t x = i % kXcds, k = i / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}
constexpr int kNC = 7;   // coefficients per momentum row: diagonal, then (d, t) -> 1 + 2 d + t
// With the Newton Jacobian as build matrix, each row also couples to the four d-faces of
// its two cells on every transverse axis d (the derivative of the advecting velocity):
// slot 1 + 2 ND + 4 dd + q, dd the rank of d among the axes other than a, q = lower and
// upper d-face of L, lower and upper d-face of C.
template <int ND>
constexpr int coef_slots(bool jac) { return jac ? 1 + 2 * ND + 4 * (ND - 1) : 1 + 2 * ND; }

template <int ND>
struct Nb {
    int32_t n[ND][2];
};

template <int ND>
__device__ __forceinline__ Nb<ND> load_nb(const DevGeo& g, int64_t c) {
    Nb<ND> r;
    const int32_t* p = g.nb6 + 6 * c;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        r.n[d][0] = p[2 * d];
        r.n[d][1] = p[2 * d + 1];
    }
    return r;
}

// Neighbour faces (d, t) of the lower a-face of C: the cell whose lower a-face it
// is, and its kind: active (an unknown), zero (inactive, on a grain surface at
// distance h) or ghost (both of its cells grain: the wall is half a cell away).
// C's table row is `nc`, L's is `nl` (L = nc.n[a][0] >= 0).
template <int ND>
struct FaceNb {
    int32_t P[ND][2];
    int8_t kind[ND][2];
};

template <int ND>
__device__ __forceinline__ FaceNb<ND> face_nb(const Nb<ND>& nc, const Nb<ND>& nl, int a) {
    FaceNb<ND> f;
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (d == a) {
                f.P[d][t] = t ? nc.n[a][1] : nc.n[a][0];
                const int32_t q = t ? nc.n[a][1] : nl.n[a][0];
                f.kind[d][t] = q >= 0 ? kActive : kZero;
            } else {
                const int32_t P = nc.n[d][t], Q = nl.n[d][t];
                f.P[d][t] = P;
                f.kind[d][t] = (P >= 0 && Q >= 0) ? kActive : ((P >= 0 || Q >= 0) ? kZero : kGhost);
            }
        }
    return f;
}

// Value of neighbour face (d, t) of a face whose own value is `self`.
template <int ND, typename V>
__device__ __forceinline__ double nb_value(const FaceNb<ND>& f, int d, int t, const V* v, int nr, int a,
                                           double self) {
    const int k = f.kind[d][t];
    if (k == kActive) return (double)v[(int64_t)nr * f.P[d][t] + a];
    return k == kZero ? 0.0 : -self;
}

// Advecting velocity a_d at the lower a-face of C: the face's own value for d == a,
// else the mean of the four d-faces of L and C (inactive faces count zero).
template <int ND, typename V>
__device__ __forceinline__ double advecting(const Nb<ND>& nc, const Nb<ND>& nl, int64_t c, int32_t L, int a,
                                            int d, const V* v, int nr) {
    if (d == a) return (double)v[(int64_t)nr * c + a];
    double s = 0.0;
    if (nl.n[d][0] >= 0) s += (double)v[(int64_t)nr * L + d];
    if (nl.n[d][1] >= 0) s += (double)v[(int64_t)nr * nl.n[d][1] + d];
    if (nc.n[d][0] >= 0) s += (double)v[(int64_t)nr * c + d];
    if (nc.n[d][1] >= 0) s += (double)v[(int64_t)nr * nc.n[d][1] + d];
    return 0.25 * s;
}

// Momentum row of the active lower a-face of C in X = J~_w (Section 4): the
// coefficient of the face itself (diagonal) and of each neighbour face (d, t)
// (zero unless active); the pressure columns (+1/h at C, -1/h at L) are implied.
// Tagged faces (no inertia) pass wind == nullptr.
template <int ND, typename W>
__device__ __forceinline__ void x_face_coefs(const Phys& ph, double h, const Nb<ND>& nc, const Nb<ND>& nl,
                                             const FaceNb<ND>& f, int64_t c, int a, const W* wind, int nr,
                                             double* co) {
    const double ih = 1.0 / h, vis = ph.mu * ih * ih;
    double diag = ph.dt > 0.0 ? ph.rho / ph.dt : 0.0;
#pragma unroll
    for (int k = 1; k < kNC; ++k) co[k] = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int k = f.kind[d][t];
            if (k == kActive) {
                diag += vis;
                co[1 + 2 * d + t] -= vis;
            } else {
                diag += k == kZero ? vis : 2.0 * vis;
            }
        }
    if (wind) {
        const int32_t L = nc.n[a][0];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const double ad = advecting(nc, nl, c, L, a, d, wind, nr);
            if (ad == 0.0) continue;
            const double cf = ph.rho * ad * ih;
            if (ad >= 0.0) {          // a (u_F - g_-) / h
                diag += cf;
                if (f.kind[d][0] == kActive) co[1 + 2 * d] -= cf;
                else if (f.kind[d][0] == kGhost) diag += cf;
            } else {                  // a (g_+ - u_F) / h
                diag -= cf;
                if (f.kind[d][1] == kActive) co[2 + 2 * d] += cf;
                else if (f.kind[d][1] == kGhost) diag -= cf;
            }
        }
    }
    co[0] = diag;
}

// The terms by which the Newton Jacobian J(w) (Section 1) differs from the untagged Oseen
// row of X(w): the derivative of the advecting velocity a_a = u_F adds rho D_a u(w) to the
// diagonal; that of each transverse a_d (the mean of four d-faces) adds rho D_d u(w) / 4
// on each of those faces that is active.  D_d u(w) is the upwind difference on the branch
// a_d(w) selects (ties: backward), as in the Jacobian stencil.
template <int ND, typename W>
__device__ __forceinline__ void jac_extra(const Phys& ph, double h, const Nb<ND>& nc, const Nb<ND>& nl,
                                          const FaceNb<ND>& f, int64_t c, int a, const W* w, int nr,
                                          double* co) {
    const double ih = 1.0 / h;
    const int32_t L = nc.n[a][0];
    const double uF = (double)w[(int64_t)nr * c + a];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const double ad = advecting(nc, nl, c, L, a, d, w, nr);
        const int t = ad >= 0.0 ? 0 : 1;
        const double g = nb_value(f, d, t, w, nr, a, uF);
        const double Du = (t == 0 ? uF - g : g - uF) * ih;
        if (d == a) {
            co[0] += ph.rho * Du;
        } else {
            const int dd = d < a ? d : d - 1;
            const double cf = 0.25 * ph.rho * Du;
            double* tr = co + 1 + 2 * ND + 4 * dd;
            tr[0] = nl.n[d][0] >= 0 ? cf : 0.0;
            tr[1] = nl.n[d][1] >= 0 ? cf : 0.0;
            tr[2] = nc.n[d][0] >= 0 ? cf : 0.0;
            tr[3] = nc.n[d][1] >= 0 ? cf : 0.0;
        }
    }
}

// Record cell of transverse column q of a row (L = C - e_a): L, L + e_d, C, C + e_d.
template <int ND>
__device__ __forceinline__ int32_t jac_col_cell(const Nb<ND>& nc, const Nb<ND>& nl, int64_t c, int32_t L, int d,
                                                int q) {
    return q == 0 ? L : q == 1 ? nl.n[d][1] : q == 2 ? (int32_t)c : nc.n[d][1];
}

// Residual record of cell c (Section 1 momentum and mass equations on the MAC grid):
// out[a] for the lower a-face (0 when inactive), out[ND] for the mass row (p = 0 at a
// pinned cell).  Backward Euler against xold when dt > 0 (xold may be nullptr = 0).
// kTagged: the modified residual of Section 4 with the wind equal to the state, i.e.
// no inertia on tagged faces (the residual of the coarse-scale solver, Section 5).
template <int ND, bool kTagged = false>
__device__ __forceinline__ void residual_cell(const DevGeo& g, const Phys& ph0, const double* __restrict__ x,
                                              const double* __restrict__ xold, int64_t c, double* out) {
    const Phys ph = cell_phys(g, ph0, c);
    constexpr int nr = ND + 1;
    const Nb<ND> nc = load_nb<ND>(g, c);
    const double ih = 1.0 / g.h, vis = ph.mu * ih * ih;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        double o = 0.0;
        const int32_t L = nc.n[a][0];
        if (L >= 0) {
            const Nb<ND> nl = load_nb<ND>(g, L);
            const FaceNb<ND> f = face_nb(nc, nl, a);
            const double uF = x[nr * c + a];
            double visc = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d)
#pragma unroll
                for (int t = 0; t < 2; ++t) visc += uF - nb_value(f, d, t, x, nr, a, uF);
            o = vis * visc + (x[nr * c + ND] - x[(int64_t)nr * L + ND]) * ih - ph.rho * ph.body[a];
            if (ph.dt > 0.0) o += ph.rho * (uF - (xold ? xold[nr * c + a] : 0.0)) / ph.dt;
            if (!kTagged || !((g.tag[c] >> a) & 1u)) {
                double conv = 0.0;
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    const double ad = advecting(nc, nl, c, L, a, d, x, nr);
                    const double gm = nb_value(f, d, 0, x, nr, a, uF), gp_ = nb_value(f, d, 1, x, nr, a, uF);
                    conv += ad * (ad >= 0.0 ? (uF - gm) : (gp_ - uF)) * ih;
                }
                o += ph.rho * conv;
            }
        }
        out[a] = o;
    }
    double m;
    if ((g.tag[c] & kPinBit)) {
        m = x[nr * c + ND];
    } else {
        m = 0.0;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            const double up = nc.n[a][1] >= 0 ? x[(int64_t)nr * nc.n[a][1] + a] : 0.0;
            const double lo = nc.n[a][0] >= 0 ? x[nr * c + a] : 0.0;
            m -= (up - lo) * ih;
        }
    }
    out[ND] = m;
}

}  // namespace gp

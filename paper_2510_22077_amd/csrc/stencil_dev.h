// Device helpers for the MAC stencils: neighbourhood lookup, neighbour-face
// classification and the coefficients of one row of the build matrix X.
#pragma once

#include "internal.h"

namespace gp {

constexpr int kMaxRow = 16;
enum : int { kActive = 0, kZero = 1, kGhost = 2 };

// Cells around cell C (indices or -1): n[d][t] = C -/+ e_d, ll[a] = C - 2 e_a,
// e[a][d][t] = C - e_a -/+ e_d (d != a).  L[a] = n[a][0].
struct Nbhd {
    int32_t n[3][2];
    int32_t ll[3];
    int32_t e[3][3][2];
    int32_t L[3];
};

__device__ __forceinline__ int32_t cell_at(const DevGeo& g, int i, int j, int k) {
    if (i < 0 || i >= g.nx) {
        if (!g.per[0]) return -1;
        i = (i + g.nx) % g.nx;
    }
    if (j < 0 || j >= g.ny) {
        if (!g.per[1]) return -1;
        j = (j + g.ny) % g.ny;
    }
    if (k < 0 || k >= g.nz) {
        if (!g.per[2]) return -1;
        k = (k + g.nz) % g.nz;
    }
    return g.cidx[((int64_t)k * g.ny + j) * g.nx + i];
}

__device__ __forceinline__ void load_nbhd(const DevGeo& g, int64_t c, Nbhd& nb) {
    uint32_t cc = g.coord[c];
    int i = cc & 1023u, j = (cc >> 10) & 1023u, k = (cc >> 20) & 1023u;
    const int nd = g.ndim;
    int o[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        nb.n[d][0] = nb.n[d][1] = nb.ll[d] = -1;
        nb.L[d] = -1;
        for (int a = 0; a < 3; ++a) nb.e[d][a][0] = nb.e[d][a][1] = -1;
    }
    for (int d = 0; d < nd; ++d) {
        o[d] = -1;
        nb.n[d][0] = cell_at(g, i + o[0], j + o[1], k + o[2]);
        o[d] = 1;
        nb.n[d][1] = cell_at(g, i + o[0], j + o[1], k + o[2]);
        o[d] = -2;
        nb.ll[d] = cell_at(g, i + o[0], j + o[1], k + o[2]);
        o[d] = 0;
        nb.L[d] = nb.n[d][0];
    }
    for (int a = 0; a < nd; ++a)
        for (int d = 0; d < nd; ++d) {
            if (d == a) continue;
            int p[3] = {0, 0, 0};
            p[a] = -1;
            p[d] = -1;
            nb.e[a][d][0] = cell_at(g, i + p[0], j + p[1], k + p[2]);
            p[d] = 1;
            nb.e[a][d][1] = cell_at(g, i + p[0], j + p[1], k + p[2]);
        }
}

struct FaceKinds {
    int8_t kind[3][2];
    int32_t cell[3][2];
};

// Neighbour faces of the lower a-face of C in direction -/+ e_d.
__device__ __forceinline__ void classify(const DevGeo& g, const Nbhd& nb, int a, FaceKinds& fk) {
    for (int d = 0; d < g.ndim; ++d)
        for (int t = 0; t < 2; ++t) {
            int32_t P;
            int8_t kd;
            if (d == a) {
                if (t == 1) {
                    P = nb.n[a][1];
                    kd = P >= 0 ? kActive : kZero;
                } else {
                    P = nb.L[a];
                    kd = nb.ll[a] >= 0 ? kActive : kZero;
                }
            } else {
                P = nb.n[d][t];
                int32_t Q = nb.e[a][d][t];
                kd = (P >= 0 && Q >= 0) ? kActive : ((P >= 0 || Q >= 0) ? kZero : kGhost);
            }
            fk.kind[d][t] = kd;
            fk.cell[d][t] = P;
        }
}

template <typename V>
__device__ __forceinline__ double nbval(const FaceKinds& fk, int d, int t, const V* vec, int nr, int a,
                                        double self) {
    int8_t k = fk.kind[d][t];
    if (k == kActive) return (double)vec[(int64_t)nr * fk.cell[d][t] + a];
    return k == kZero ? 0.0 : -self;
}

// Advecting velocity a_d of the lower a-face of cell c: the face's own value for
// d == a, else the mean of the four d-faces of its two cells (inactive ones 0).
template <typename V>
__device__ __forceinline__ double advecting(const DevGeo& g, const Nbhd& nb, int a, int d, const V* vec,
                                            int64_t c) {
    const int nr = g.nrec;
    if (d == a) return (double)vec[(int64_t)nr * c + a];
    const int32_t Lc = nb.L[a];
    double s = 0.0;
    if (nb.e[a][d][0] >= 0) s += (double)vec[(int64_t)nr * Lc + d];              // lower d-face of L
    if (nb.e[a][d][1] >= 0) s += (double)vec[(int64_t)nr * nb.e[a][d][1] + d];   // upper d-face of L
    if (nb.n[d][0] >= 0) s += (double)vec[(int64_t)nr * c + d];                  // lower d-face of C
    if (nb.n[d][1] >= 0) s += (double)vec[(int64_t)nr * nb.n[d][1] + d];         // upper d-face of C
    return 0.25 * s;
}

// Row (c, comp) of X = J~_w: up to kMaxRow (column slot, value) pairs, columns may repeat.
template <typename W>
__device__ __forceinline__ int x_row(const DevGeo& g, const Phys& ph, const Nbhd& nb, int64_t c, int comp,
                                     const W* wind, int64_t* cols, double* vals) {
    const int nd = g.ndim, nr = g.nrec;
    const double ih = 1.0 / g.h, vis = ph.mu * ih * ih;
    int cnt = 0;
    const int64_t self = (int64_t)nr * c + comp;
    if (comp == nd) {
        if (c == g.pin) {
            cols[0] = self;
            vals[0] = 1.0;
            return 1;
        }
        for (int a = 0; a < nd; ++a) {
            if (nb.L[a] >= 0) {
                cols[cnt] = (int64_t)nr * c + a;
                vals[cnt++] = ih;
            }
            if (nb.n[a][1] >= 0) {
                cols[cnt] = (int64_t)nr * nb.n[a][1] + a;
                vals[cnt++] = -ih;
            }
        }
        return cnt;
    }
    const int a = comp;
    if (nb.L[a] < 0) return 0;
    FaceKinds fk;
    classify(g, nb, a, fk);
    double diag = ph.dt > 0.0 ? ph.rho / ph.dt : 0.0;
    for (int d = 0; d < nd; ++d)
        for (int t = 0; t < 2; ++t) {
            int8_t k = fk.kind[d][t];
            if (k == kActive) {
                diag += vis;
                cols[cnt] = (int64_t)nr * fk.cell[d][t] + a;
                vals[cnt++] = -vis;
            } else {
                diag += k == kZero ? vis : 2.0 * vis;
            }
        }
    if (!((g.tag[c] >> a) & 1u)) {
        for (int d = 0; d < nd; ++d) {
            double ad = wind ? advecting(g, nb, a, d, wind, c) : 0.0;
            if (ad == 0.0) continue;
            double cf = ph.rho * ad * ih;
            int t = ad >= 0.0 ? 0 : 1;
            int8_t k = fk.kind[d][t];
            if (t == 0) {          // a (u_F - g_-)/h
                diag += cf;
                if (k == kActive) {
                    cols[cnt] = (int64_t)nr * fk.cell[d][0] + a;
                    vals[cnt++] = -cf;
                } else if (k == kGhost) {
                    diag += cf;
                }
            } else {               // a (g_+ - u_F)/h
                diag -= cf;
                if (k == kActive) {
                    cols[cnt] = (int64_t)nr * fk.cell[d][1] + a;
                    vals[cnt++] = cf;
                } else if (k == kGhost) {
                    diag -= cf;
                }
            }
        }
    }
    cols[cnt] = (int64_t)nr * c + nd;
    vals[cnt++] = ih;
    cols[cnt] = (int64_t)nr * nb.L[a] + nd;
    vals[cnt++] = -ih;
    cols[cnt] = self;
    vals[cnt++] = diag;
    return cnt;
}

}  // namespace gp

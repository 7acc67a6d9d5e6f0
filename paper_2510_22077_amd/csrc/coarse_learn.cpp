// Features of the coarse operator's entries for the learned coefficients.
//
// The coarse operator Rhat X Phat (Section 3.2.2, Remark 1) couples the coarse
// pressures of the contact interfaces ("throats") and the correction unknowns of
// the primaries ("pores").  Its structural pattern is the probing pattern.  Each
// entry (row object, column object) is described by: its kind (interface-interface
// diagonal / off-diagonal, interface-pore, pore-interface, pore-pore diagonal /
// off-diagonal); for both objects the log size (cells), the log of its wall contact
// relative to its size (a shape factor: grain-touching cells per cell for a throat
// sheet, grain faces per cell for a pore), and log(1 + Re) of a local Reynolds number rho |w| l / mu
// from the wind (mean face speed over the object's cells, l = size^(1/ndim-1) for a
// throat, size^(1/ndim) for a pore); and a relation feature (size of the pore two
// throats share, adjacency of a throat and a pore, throats two pores share), for
// each object the log size of its neighbourhood (a throat: its pores' cells; a pore:
// its coordination number), and the row object's shape factor G = A / P^2 (its size
// over its squared wall contact).  The network predicts asinh(entry / scale) with the
// scale mu l_r^(1/2) l_c^(1/2) built from the objects' lengths: targets of order one
// that keep their sign, with the large diagonal entries compressed.  The operator
// assembled from the predictions then takes the conservation structure of the exact
// one (zero sums over the interface columns, see learned_coarse).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace gp {

namespace {

struct ObjGeo {
    double size = 0, wall = 0, len = 1, around = 0;   // around: log of the neighbourhood's size
    std::vector<int32_t> cells;
};

}  // namespace

// Per coarse object: its cells, size, wall contact and length.
static void coarse_geometry(gplmm_ctx* c, std::vector<ObjGeo>& obj) {
    const int nd = c->ndim;
    const int nco = c->nco;
    obj.assign(nco, ObjGeo());
    for (int j = 0; j < c->Nc; ++j) {
        ObjGeo& o = obj[j];
        o.cells = c->icells[j];
        o.size = (double)o.cells.size();
        for (int32_t q : o.cells) {
            bool touch = false;
            for (int e = 0; e < 2 * nd; ++e) touch |= c->nbr[(int64_t)q * 6 + e] < 0;
            o.wall += touch ? 1.0 : 0.0;
        }
        o.len = std::pow(std::max(o.size, 1.0), nd == 3 ? 0.5 : 1.0);
    }
    std::vector<std::vector<int32_t>> pc(c->Np);
    for (int64_t q = 0; q < c->ncell; ++q)
        if (c->prim[q] >= 0) pc[c->prim[q]].push_back((int32_t)q);
    for (int i = 0; i < c->Np; ++i) {
        if (c->ycol[i] < 0) continue;
        ObjGeo& o = obj[c->ycol[i]];
        o.cells = pc[i];
        o.size = (double)o.cells.size();
        for (int32_t q : o.cells)
            for (int e = 0; e < 2 * nd; ++e) o.wall += c->nbr[(int64_t)q * 6 + e] < 0 ? 1.0 : 0.0;
        o.len = std::pow(std::max(o.size, 1.0), 1.0 / nd);
        o.around = std::log1p((double)c->Cp[i].size());   // coordination number
    }
    for (int i = 0; i < c->Np; ++i)   // throats: total size of the pores they join
        for (int32_t j : c->Cp[i]) obj[j].around += (double)pc[i].size();
    for (int j = 0; j < c->Nc; ++j) obj[j].around = std::log1p(obj[j].around);
}

int coarse_features(gplmm_ctx* c, const double* wind_host, std::vector<float>& feat, std::vector<float>& scale) {
    const int nco = c->nco;
    if (c->cl_row.empty()) {   // pattern: the probing entries, in colour order
        c->cl_row.reserve(c->probe.size());
        for (const ProbeEntry& p : c->probe) {
            c->cl_row.push_back(p.row);
            c->cl_col.push_back(p.col);
        }
    }
    std::vector<ObjGeo> obj;
    coarse_geometry(c, obj);
    const int nd = c->ndim, nr = c->nrec;
    // object speed from the wind: mean over the object's cells of |w| at their lower faces
    std::vector<double> re(nco, 0.0);
    for (int g = 0; g < nco; ++g) {
        const ObjGeo& o = obj[g];
        if (o.cells.empty() || !wind_host) continue;
        double s = 0.0;
        for (int32_t q : o.cells) {
            double w2 = 0.0;
            for (int a = 0; a < nd; ++a) {
                const double w = wind_host[(int64_t)q * nr + a];
                w2 += w * w;
            }
            s += std::sqrt(w2);
        }
        const Phys& ph = c->csamp.empty() ? c->phys : c->sphys[c->csamp[o.cells[0]]];
        re[g] = ph.rho * (s / (double)o.cells.size()) * o.len * c->opt.h / ph.mu;
    }
    // pores of each interface; interfaces of each pore (coarse ids)
    std::vector<std::vector<int32_t>> iface_pores(c->Nc);
    for (int i = 0; i < c->Np; ++i)
        for (int32_t j : c->Cp[i]) iface_pores[j].push_back(i);
    std::vector<int32_t> prim_of(nco, -1);
    for (int i = 0; i < c->Np; ++i)
        if (c->ycol[i] >= 0) prim_of[c->ycol[i]] = i;
    const int64_t ne = (int64_t)c->cl_row.size();
    feat.assign(ne * kCoarseFeatures, 0.f);
    scale.assign(ne, 0.f);
    for (int64_t e = 0; e < ne; ++e) {
        const int r = c->cl_row[e], k = c->cl_col[e];
        const bool ri = r < c->Nc, ki = k < c->Nc;
        int kind;
        if (ri && ki) kind = r == k ? 0 : 1;
        else if (ri) kind = 2;
        else if (ki) kind = 3;
        else kind = r == k ? 4 : 5;
        float* f = &feat[e * kCoarseFeatures];
        f[kind] = 1.f;
        auto put = [&](int base, int g) {
            const ObjGeo& o = obj[g];
            f[base] = (float)std::log(std::max(o.size, 1.0));
            f[base + 1] = (float)std::log((1.0 + o.wall) / std::max(o.size, 1.0));
            f[base + 2] = (float)std::log1p(re[g]);
        };
        put(6, r);
        put(9, k);
        f[13] = (float)obj[r].around;
        f[14] = (float)obj[k].around;
        double rel = 0.0;
        if (kind == 1) {   // size of a pore both throats touch
            for (int32_t a : iface_pores[r])
                for (int32_t b : iface_pores[k])
                    if (a == b && c->ycol[a] >= 0) rel = std::max(rel, std::log(std::max(obj[c->ycol[a]].size, 1.0)));
        } else if (kind == 2 || kind == 3) {   // is the throat a throat of the pore
            const int j = ri ? r : k, y = ri ? k : r;
            for (int32_t a : iface_pores[j]) rel = std::max(rel, (double)(c->ycol[a] == y));
        } else if (kind == 5) {   // throats the two pores share
            const int na = prim_of[r], nb = prim_of[k];
            if (na >= 0 && nb >= 0) {
                int cnt = 0;
                for (int32_t j : c->Cp[na])
                    for (int32_t j2 : c->Cp[nb]) cnt += j == j2;
                rel = std::log1p((double)cnt);
            }
        }
        f[12] = (float)rel;
        // shape factor G = A / P^2 of the row object: its size against its wall contact
        f[15] = (float)std::log(std::max(obj[r].size, 1.0) / ((1.0 + obj[r].wall) * (1.0 + obj[r].wall)));
        const double mu = (c->csamp.empty() || obj[r].cells.empty()) ? c->phys.mu : c->sphys[c->csamp[obj[r].cells[0]]].mu;
        scale[e] = (float)(mu * std::sqrt(obj[r].len * obj[k].len));
    }
    return GPLMM_OK;
}

}  // namespace gp

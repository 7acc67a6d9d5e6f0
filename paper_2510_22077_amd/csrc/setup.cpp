// Host setup: fluid cells, pore decomposition, local problems, probing colours.
//
// Paper, Section 3.2.1 (primary grids, contact interfaces, dual grids) and the
// permutation paragraph of Section 3.2.2 (a face with a flanking cell in a
// primary belongs to it; a face flanked by neither belongs to the interface).
// The rules that turn pore labels into interfaces (carving on the higher-label
// side, the closure exemption of wall-free face groups, the merge of interfaces that touch no
// primary, the pin, tags and dual growth) are this library's reading of the
// paper, stated where each step is implemented.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <map>
#include <queue>

#include "internal.h"
#include <array>

namespace gp {

int fail(gplmm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

namespace {

struct UF {
    std::vector<int64_t> p;
    explicit UF(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int64_t find(int64_t a) {
        while (p[a] != a) {
            p[a] = p[p[a]];
            a = p[a];
        }
        return a;
    }
    void unite(int64_t a, int64_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

inline int64_t slot(const gplmm_ctx* c, int64_t cell, int comp) { return (int64_t)c->nrec * cell + comp; }

}  // namespace

// Voxel neighbour (with periodic wrap) or -1 outside the image.
static inline int64_t vox_nb(const gplmm_ctx* c, int64_t v, int d, int s) {
    int64_t i = v % c->nx, j = (v / c->nx) % c->ny, k = v / ((int64_t)c->nx * c->ny);
    int64_t q[3] = {i, j, k};
    int64_t n[3] = {c->nx, c->ny, c->nz};
    q[d] += s;
    if (q[d] < 0 || q[d] >= n[d]) {
        if (!c->opt.periodic[d]) return -1;
        q[d] = (q[d] + n[d]) % n[d];
    }
    return (q[2] * c->ny + q[1]) * c->nx + q[0];
}

int build_decomposition(gplmm_ctx* c, const uint8_t* mask, const int32_t* labels) {
    const int64_t nvox = c->nvox;
    const int nd = c->ndim;
    // ---- largest face-connected fluid component (periodic axes wrap); ties: earliest first voxel
    std::vector<int32_t> comp(nvox, -1);
    std::vector<int64_t> comp_size;
    {
        std::vector<int64_t> stack;
        for (int64_t v = 0; v < nvox; ++v) {
            if (!mask[v] || comp[v] >= 0) continue;
            int32_t id = (int32_t)comp_size.size();
            int64_t cnt = 0;
            comp[v] = id;
            stack.push_back(v);
            while (!stack.empty()) {
                int64_t u = stack.back();
                stack.pop_back();
                ++cnt;
                for (int d = 0; d < nd; ++d)
                    for (int s = -1; s <= 1; s += 2) {
                        int64_t w = vox_nb(c, u, d, s);
                        if (w >= 0 && mask[w] && comp[w] < 0) {
                            comp[w] = id;
                            stack.push_back(w);
                        }
                    }
            }
            comp_size.push_back(cnt);
        }
    }
    if (comp_size.empty()) return fail(c, GPLMM_E_GEOMETRY, "the image has no fluid voxel");
    int32_t keep = (int32_t)(std::max_element(comp_size.begin(), comp_size.end()) - comp_size.begin());
    c->cidx.assign(nvox, -1);
    c->cell_voxel.clear();
    for (int64_t v = 0; v < nvox; ++v)
        if (comp[v] == keep) {
            c->cidx[v] = (int32_t)c->cell_voxel.size();
            c->cell_voxel.push_back((int32_t)v);
        }
    const int64_t nc = (int64_t)c->cell_voxel.size();
    c->ncell = nc;
    c->N = (int64_t)c->nrec * nc;
    // ---- cell neighbours through active faces
    c->nbr.assign(nc * 6, -1);
    for (int64_t q = 0; q < nc; ++q)
        for (int d = 0; d < nd; ++d)
            for (int t = 0; t < 2; ++t) {
                int64_t w = vox_nb(c, c->cell_voxel[q], d, t ? 1 : -1);
                c->nbr[q * 6 + 2 * d + t] = w >= 0 ? c->cidx[w] : -1;
            }
    auto NB = [&](int64_t q, int d, int t) -> int64_t { return q < 0 ? -1 : c->nbr[q * 6 + 2 * d + t]; };
    // ---- labels
    std::vector<int64_t> L(nc);
    for (int64_t q = 0; q < nc; ++q) {
        L[q] = labels[c->cell_voxel[q]];
        if (L[q] <= 0) return fail(c, GPLMM_E_ARG, "a fluid voxel has a non-positive pore label");
    }
    std::vector<uint8_t> is_if(nc);
    std::vector<int64_t> minlow(nc);
    auto carve = [&]() {
        for (int64_t q = 0; q < nc; ++q) {
            int64_t m = INT64_MAX;
            for (int e = 0; e < 2 * nd; ++e) {
                int64_t w = c->nbr[q * 6 + e];
                if (w >= 0 && L[w] > 0 && L[w] < L[q]) m = std::min(m, L[w]);
            }
            is_if[q] = m != INT64_MAX;
            minlow[q] = m;
        }
    };
    // an a-face "at" cell q is its lower a-face; active iff the lower neighbour is fluid
    auto face_active = [&](int64_t q, int a) { return q >= 0 && NB(q, a, 0) >= 0; };
    carve();
    // ---- interfaces: sorted (lower label, own label) pairs; with interface groups (the
    // pore-network decomposition of Section 3.3) one interface per group label instead
    std::vector<int64_t> G;
    if (c->setup_groups) {
        G.assign(nc, 0);
        for (int64_t q = 0; q < nc; ++q) {
            G[q] = c->setup_groups[c->cell_voxel[q]];
            if (is_if[q] && G[q] <= 0) return fail(c, GPLMM_E_ARG, "an interface cell has a non-positive group label");
        }
    }
    auto key_of = [&](int64_t q) {
        return G.empty() ? std::make_pair(minlow[q], L[q]) : std::make_pair(G[q], (int64_t)0);
    };
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int64_t q = 0; q < nc; ++q)
        if (is_if[q]) pairs.push_back(key_of(q));
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    c->iface.assign(nc, -1);
    for (int64_t q = 0; q < nc; ++q)
        if (is_if[q])
            c->iface[q] = (int32_t)(std::lower_bound(pairs.begin(), pairs.end(), key_of(q)) - pairs.begin());
    // ---- degenerate interfaces: touched by no primary cell, or only by primary pieces that touch
    // no other interface (a dead-end pocket seen by the rest of the void only through faces
    // between interface cells, which the coarse space leaves at zero; a piece is a face-connected
    // set of one label's primary cells, since carving can cut a fragment off a pore).  The
    // lowest-id one that shares a face with another interface joins the interface it shares the
    // most faces with.
    std::vector<int64_t> piece(nc);
    {
        UF uf(nc);
        for (int64_t q = 0; q < nc; ++q) {
            if (is_if[q]) continue;
            for (int e = 0; e < 2 * nd; ++e) {
                int64_t w = c->nbr[q * 6 + e];
                if (w >= 0 && !is_if[w] && L[w] == L[q]) uf.unite(q, w);
            }
        }
        for (int64_t q = 0; q < nc; ++q) piece[q] = uf.find(q);
    }
    for (;;) {
        int nif = (int)pairs.size();
        std::vector<std::vector<int64_t>> if_labs(nif);                 // primary pieces touching j
        std::map<int64_t, std::vector<int32_t>> lab_ifs;                 // interfaces touched by a piece
        std::vector<uint8_t> shares(nif, 0);
        for (int64_t q = 0; q < nc; ++q) {
            int j = c->iface[q];
            if (j < 0) continue;
            for (int e = 0; e < 2 * nd; ++e) {
                int64_t w = c->nbr[q * 6 + e];
                if (w < 0) continue;
                if (c->iface[w] < 0) {
                    if_labs[j].push_back(piece[w]);
                    lab_ifs[piece[w]].push_back(j);
                } else if (c->iface[w] != j) {
                    shares[j] = 1;
                }
            }
        }
        for (auto& kv : lab_ifs) {
            std::sort(kv.second.begin(), kv.second.end());
            kv.second.erase(std::unique(kv.second.begin(), kv.second.end()), kv.second.end());
        }
        int j = -1;
        for (int t = 0; t < nif && j < 0; ++t) {
            if (!shares[t]) continue;
            bool dead = true;
            for (int64_t l : if_labs[t]) {
                const auto& v = lab_ifs[l];
                if (!(v.size() == 1 && v[0] == t)) {
                    dead = false;
                    break;
                }
            }
            if (dead) j = t;
        }
        if (j < 0) break;
        std::vector<int64_t> cnt(nif, 0);
        for (int64_t q = 0; q < nc; ++q) {
            if (c->iface[q] != j) continue;
            for (int e = 0; e < 2 * nd; ++e) {
                int64_t w = c->nbr[q * 6 + e];
                if (w >= 0 && c->iface[w] >= 0 && c->iface[w] != j) cnt[c->iface[w]]++;
            }
        }
        int k = (int)(std::max_element(cnt.begin(), cnt.end()) - cnt.begin());
        for (int64_t q = 0; q < nc; ++q) {
            if (c->iface[q] == j) c->iface[q] = k;
            if (c->iface[q] > j) c->iface[q] -= 1;
        }
        pairs.erase(pairs.begin() + j);
    }
    c->Nc = (int)pairs.size();
    // ---- primaries in label order
    std::vector<int64_t> plab;
    for (int64_t q = 0; q < nc; ++q)
        if (c->iface[q] < 0) plab.push_back(L[q]);
    std::sort(plab.begin(), plab.end());
    plab.erase(std::unique(plab.begin(), plab.end()), plab.end());
    c->Np = (int)plab.size();
    c->prim.assign(nc, -1);
    for (int64_t q = 0; q < nc; ++q)
        if (c->iface[q] < 0) c->prim[q] = (int32_t)(std::lower_bound(plab.begin(), plab.end(), L[q]) - plab.begin());
    c->pin = -1;
    for (int64_t q = 0; q < nc; ++q)
        if (c->iface[q] < 0) {
            c->pin = q;
            break;
        }
    if (c->pin < 0) return fail(c, GPLMM_E_GEOMETRY, "no primary cell");
    // ---- ownership of every slot
    c->owner.assign(c->N, -3);
    c->nface = 0;
    for (int64_t q = 0; q < nc; ++q)
        for (int a = 0; a < nd; ++a) {
            int64_t s = slot(c, q, a);
            if (!face_active(q, a)) {
                c->owner[s] = -2;
                continue;
            }
            ++c->nface;
            int64_t l0 = NB(q, a, 0);
            int pq = c->prim[q], pl = c->prim[l0];
            if (pq >= 0 && pl >= 0 && pq != pl)
                return fail(c, GPLMM_E_GEOMETRY, "a face lies between two different primaries");
            c->owner[s] = pq >= 0 ? pq : (pl >= 0 ? pl : -1);
        }
    // ---- wall-free face groups: a primary's same-axis faces linked through the viscous
    // stencil, none of which reaches a non-active face position, keep their plain rows in
    // the closure matrix (the column sums would leave their common velocity undetermined)
    c->noclose.assign(c->N, 0);
    for (int a = 0; a < nd; ++a) {
        UF uf(nc);
        std::vector<uint8_t> walled(nc, 0);
        auto own = [&](int64_t q) -> int32_t { return face_active(q, a) ? c->owner[slot(c, q, a)] : -9; };
        for (int64_t q = 0; q < nc; ++q) {
            if (!face_active(q, a)) continue;
            for (int d = 0; d < nd; ++d)
                for (int t = 0; t < 2; ++t) {
                    int64_t p = NB(q, d, t);
                    bool act = face_active(p, a);
                    if (!act) walled[q] = 1;
                    if (t == 1 && act && own(q) >= 0 && own(q) == own(p)) uf.unite(q, p);
                }
        }
        std::vector<uint8_t> root_wall(nc, 0);
        for (int64_t q = 0; q < nc; ++q)
            if (own(q) >= 0 && walled[q]) root_wall[uf.find(q)] = 1;
        for (int64_t q = 0; q < nc; ++q)
            if (own(q) >= 0 && !root_wall[uf.find(q)]) c->noclose[slot(c, q, a)] = 1;
    }
    // ---- interfaces adjacent to each primary
    c->Cp.assign(c->Np, {});
    for (int64_t q = 0; q < nc; ++q) {
        if (c->prim[q] < 0) continue;
        for (int e = 0; e < 2 * nd; ++e) {
            int64_t w = c->nbr[q * 6 + e];
            if (w >= 0 && c->iface[w] >= 0) c->Cp[c->prim[q]].push_back(c->iface[w]);
        }
    }
    for (auto& v : c->Cp) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    c->icells.assign(c->Nc, {});
    for (int64_t q = 0; q < nc; ++q)
        if (c->iface[q] >= 0) c->icells[c->iface[q]].push_back((int32_t)q);
    // ---- tags: faces with a cell within Chebyshev distance tag_layers of an interface cell
    {
        std::vector<uint8_t> near(nvox, 0);
        for (int64_t q = 0; q < nc; ++q)
            if (c->iface[q] >= 0) near[c->cell_voxel[q]] = 1;
        for (int d = 0; d < nd; ++d) {
            std::vector<uint8_t> acc = near;
            for (int64_t v = 0; v < nvox; ++v) {
                if (!near[v]) continue;
                for (int s = -1; s <= 1; s += 2) {
                    int64_t w = v;
                    for (int r = 1; r <= c->opt.tag_layers; ++r) {
                        w = vox_nb(c, w, d, s);
                        if (w < 0) break;
                        acc[w] = 1;
                    }
                }
            }
            near.swap(acc);
        }
        c->tagslot.assign(c->N, 0);
        c->tagcell.assign(nc, 0);
        for (int64_t q = 0; q < nc; ++q)
            for (int a = 0; a < nd; ++a) {
                if (!face_active(q, a)) continue;
                int64_t l0 = NB(q, a, 0);
                if (near[c->cell_voxel[q]] || near[c->cell_voxel[l0]]) {
                    c->tagslot[slot(c, q, a)] = 1;
                    c->tagcell[q] |= (uint8_t)(1u << a);
                }
            }
        c->tagcell[c->pin] |= kPinBit;
    }
    // ---- dual grids: each interface grown dual_dilations times through face neighbours
    int dd = c->opt.dual_dilations >= 0 ? c->opt.dual_dilations : (nd == 2 ? 1 : 0);
    c->dual_cells.assign(c->Nc, {});
    for (int j = 0; j < c->Nc; ++j) {
        std::vector<int32_t> cur = c->icells[j];
        for (int it = 0; it < dd; ++it) {
            std::vector<int32_t> nxt = cur;
            for (int32_t q : cur)
                for (int e = 0; e < 2 * nd; ++e) {
                    int64_t w = c->nbr[(int64_t)q * 6 + e];
                    if (w >= 0) nxt.push_back((int32_t)w);
                }
            std::sort(nxt.begin(), nxt.end());
            nxt.erase(std::unique(nxt.begin(), nxt.end()), nxt.end());
            cur.swap(nxt);
        }
        c->dual_cells[j] = cur;
    }
    return GPLMM_OK;
}

// ------------------------------------------------------------------------------------------
// Local problems: unknown sets, pressure-after-faces raster order, tile envelopes, LU schedule
// ------------------------------------------------------------------------------------------

namespace {

// Unknowns of a cell set: its cells plus every active face with a flanking cell in the set.
std::vector<int64_t> unknowns_of(const gplmm_ctx* c, const std::vector<int32_t>& cells) {
    std::vector<int64_t> u;
    const int nd = c->ndim;
    for (int32_t q : cells) {
        u.push_back(slot(c, q, nd));
        for (int a = 0; a < nd; ++a) {
            if (c->nbr[(int64_t)q * 6 + 2 * a] >= 0) u.push_back(slot(c, q, a));
            int64_t up = c->nbr[(int64_t)q * 6 + 2 * a + 1];
            if (up >= 0) u.push_back(slot(c, up, a));
        }
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    return u;
}

// Frame of a set's unknowns: the record position of each face (for a face whose
// record cell is outside the set, one step above its lower neighbour) and the cell
// position of each pressure, in the set's own coordinates, and the raster strides.
struct LocalFrame {
    std::vector<std::array<int, 3>> pos;   // per unknown
    std::vector<int> comp;                 // per unknown: face axis, or ndim for a pressure
    int64_t stride[3] = {0, 0, 0};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int slow = 0;
    int nd = 3;
};

LocalFrame local_frame(const gplmm_ctx* c, const std::vector<int32_t>& cells, const std::vector<int64_t>& u) {
    const int nd = c->ndim;
    const int n = (int)cells.size();
    LocalFrame f;
    f.nd = nd;
    // the sample holding the set (a subdomain never spans two samples of a batch)
    size_t si = 0;
    while (si + 1 < c->samples.size() && c->samples[si + 1].coff <= (int64_t)cells[0]) ++si;
    const SampleGeo& sg = c->samples[si];
    const int dims[3] = {sg.nx, sg.ny, sg.nz};
    std::vector<std::array<int, 3>> co(n);
    for (int t = 0; t < n; ++t) {
        int64_t v = c->cell_voxel[cells[t]] - sg.voff;
        co[t] = {(int)(v % sg.nx), (int)((v / sg.nx) % sg.ny), (int)(v / ((int64_t)sg.nx * sg.ny))};
    }
    for (int a = 0; a < 3; ++a) {
        if (!c->opt.periodic[a] || dims[a] < 2) continue;
        std::vector<char> occ(dims[a], 0);
        for (int t = 0; t < n; ++t) occ[co[t][a]] = 1;
        int best = -1, bestlen = 0;
        for (int x0 = 0; x0 < dims[a]; ++x0) {
            if (occ[x0] || !occ[(x0 + dims[a] - 1) % dims[a]]) continue;   // an empty run starts at x0
            int len = 0;
            while (len < dims[a] && !occ[(x0 + len) % dims[a]]) ++len;
            if (len > bestlen) {
                bestlen = len;
                best = x0;
            }
        }
        if (best < 0) continue;   // occupies the whole ring: keep the image coordinates
        const int start = (best + bestlen) % dims[a];
        for (int t = 0; t < n; ++t) co[t][a] = (co[t][a] - start + dims[a]) % dims[a];
    }
    for (int a = 0; a < 3; ++a) {
        f.lo[a] = 1 << 30;
        f.hi[a] = -1;
    }
    for (int t = 0; t < n; ++t)
        for (int a = 0; a < 3; ++a) {
            f.lo[a] = std::min(f.lo[a], co[t][a]);
            f.hi[a] = std::max(f.hi[a], co[t][a]);
        }
    int ax[3] = {0, 1, 2};   // fastest .. slowest; ties keep x fastest
    std::stable_sort(ax, ax + nd, [&](int a, int b) { return f.hi[a] - f.lo[a] < f.hi[b] - f.lo[b]; });
    int64_t st = 1;
    for (int q = 0; q < nd; ++q) {
        f.stride[ax[q]] = st;
        st *= (int64_t)(f.hi[ax[q]] - f.lo[ax[q]] + 2);   // +1 for the upper faces of the top layer
    }
    f.slow = ax[nd - 1];
    auto idx = [&](int64_t q) -> int {
        auto it = std::lower_bound(cells.begin(), cells.end(), (int32_t)q);
        return (it != cells.end() && *it == q) ? (int)(it - cells.begin()) : -1;
    };
    f.pos.resize(u.size());
    f.comp.resize(u.size());
    for (size_t t = 0; t < u.size(); ++t) {
        const int64_t q = u[t] / c->nrec;
        const int comp = (int)(u[t] % c->nrec);
        int k = idx(q);
        f.comp[t] = comp;
        if (comp < nd) {
            if (k >= 0) {
                f.pos[t] = co[k];
            } else {   // record cell outside the set: one step above its lower neighbour
                f.pos[t] = co[idx(c->nbr[q * 6 + 2 * comp])];
                f.pos[t][comp] += 1;
            }
        } else {
            f.pos[t] = co[k];
        }
    }
    return f;
}

// Raster key of unknown t: faces at their record position (axis order within it), a
// pressure after the upper face of its cell along the slowest axis.  reverse: the slowest
// axis runs downwards (a pressure then still follows every face of its cell).
int64_t frame_key(const LocalFrame& f, size_t t, bool reverse) {
    const auto& p = f.pos[t];
    int64_t l = 0;
    for (int a = 0; a < f.nd; ++a) {
        const int x = (reverse && a == f.slow) ? f.hi[a] + 1 - p[a] : p[a] - f.lo[a];
        l += (int64_t)x * f.stride[a];
    }
    return f.comp[t] < f.nd ? l * 8 + f.comp[t] : (l + f.stride[f.slow]) * 8 + 7;
}

// Local order of a subdomain's unknowns: a raster order over the set's own bounding
// box (periodic axes cut at their longest empty run, so a set that wraps is
// contiguous), with the longest extent as the slowest axis, which keeps the
// envelope (the slab of unknowns between a row and its furthest lower neighbour)
// small.  Every pressure follows all of its faces, so the velocity-first leading blocks
// of the saddle-point matrix stay nonsingular without pivoting.
std::vector<int64_t> local_keys(const gplmm_ctx* c, const std::vector<int32_t>& cells, const std::vector<int64_t>& u) {
    LocalFrame f = local_frame(c, cells, u);
    std::vector<int64_t> keys(u.size());
    for (size_t t = 0; t < u.size(); ++t) keys[t] = frame_key(f, t, false);
    return keys;
}

// Structural columns of row s of X (viscous/convective neighbours, gradient, divergence).
void row_pattern(const gplmm_ctx* c, int64_t s, std::vector<int64_t>& cols) {
    cols.clear();
    const int nd = c->ndim;
    int64_t q = s / c->nrec;
    int comp = (int)(s % c->nrec);
    auto NB = [&](int64_t x, int d, int t) -> int64_t { return x < 0 ? -1 : c->nbr[x * 6 + 2 * d + t]; };
    cols.push_back(s);
    if (comp < nd) {
        int a = comp;
        int64_t l0 = NB(q, a, 0);
        for (int d = 0; d < nd; ++d)
            for (int t = 0; t < 2; ++t) {
                int64_t p = (d == a && t == 0) ? l0 : NB(q, d, t);
                if (p >= 0 && NB(p, a, 0) >= 0) cols.push_back(slot(c, p, a));
            }
        cols.push_back(slot(c, q, nd));
        cols.push_back(slot(c, l0, nd));
        if (c->opt.build_matrix == GPLMM_BUILD_JACOBIAN) {
            // the Newton Jacobian's transverse couplings: the d-faces of the face's two cells
            for (int d = 0; d < nd; ++d) {
                if (d == a) continue;
                for (int64_t cell : {l0, q}) {
                    if (NB(cell, d, 0) >= 0) cols.push_back(slot(c, cell, d));
                    int64_t up = NB(cell, d, 1);
                    if (up >= 0) cols.push_back(slot(c, up, d));
                }
            }
        }
    } else if (!(c->tagcell[q] & kPinBit)) {
        for (int a = 0; a < nd; ++a) {
            if (NB(q, a, 0) >= 0) cols.push_back(slot(c, q, a));
            int64_t up = NB(q, a, 1);
            if (up >= 0) cols.push_back(slot(c, up, a));
        }
    }
}

// One level of nested dissection of a primary's unknown set (its Schwarz block is solved
// as the halves A and B in parallel and the separator S between them):
// * S: every unknown whose position along the slowest axis is the median plane k0 (a face
//   at its record cell, a pressure at its cell); A below, B above.  The X stencil couples
//   unknowns at most one position apart, so A and B are uncoupled;
// * A in raster order, B in raster order reversed along the cut axis (its separator
//   neighbours come last), each trimmed to a whole number of tiles by moving its last
//   unknowns to the front of S;
// * any pressure with an incident face ordered after it (in the global order [A, B, S])
//   moves to the end of S, so every pressure still follows its faces and the elimination
//   without pivoting stays defined; trimming and moving repeat until nothing moves.
// Returns false when the set does not split (too few planes, a coupling across the cut,
// or a separator above a quarter of the unknowns or above 4096).
bool plan_split(const gplmm_ctx* c, const std::vector<int32_t>& cells, std::vector<int64_t>& A,
                std::vector<int64_t>& B, std::vector<int64_t>& S) {
    const int T = c->tile, nd = c->ndim;
    std::vector<int64_t> u = unknowns_of(c, cells);
    const LocalFrame f = local_frame(c, cells, u);
    const int n = (int)u.size();
    const int sl = f.slow;
    const int z0 = f.lo[sl], z1 = f.hi[sl] + 1;
    std::vector<int> cnt(z1 - z0 + 1, 0);
    for (int t = 0; t < n; ++t) cnt[f.pos[t][sl] - z0]++;
    int k0 = z0, acc = 0;
    while (k0 < z1 && acc + cnt[k0 - z0] < n / 2) acc += cnt[k0++ - z0];
    if (k0 <= z0 || k0 >= z1) return false;
    std::vector<std::pair<int64_t, int>> ka, kb, ks;
    for (int t = 0; t < n; ++t) {
        const int z = f.pos[t][sl];
        if (z < k0) ka.push_back({frame_key(f, t, false), t});
        else if (z > k0) kb.push_back({frame_key(f, t, true), t});
        else ks.push_back({frame_key(f, t, false), t});
    }
    std::sort(ka.begin(), ka.end());
    std::sort(kb.begin(), kb.end());
    std::sort(ks.begin(), ks.end());
    std::vector<int> a, b, core, rep;
    std::deque<int> movA, movB;
    for (auto& p : ka) a.push_back(p.second);
    for (auto& p : kb) b.push_back(p.second);
    for (auto& p : ks) core.push_back(p.second);
    // slot -> unknown index
    std::vector<std::pair<int64_t, int>> inv(n);
    for (int t = 0; t < n; ++t) inv[t] = {u[t], t};
    std::sort(inv.begin(), inv.end());
    auto index_of = [&](int64_t s) -> int {
        auto it = std::lower_bound(inv.begin(), inv.end(), std::make_pair(s, -1));
        return (it != inv.end() && it->first == s) ? it->second : -1;
    };
    std::vector<int> place(n);
    for (int round = 0; round < 64; ++round) {
        while (a.size() % T) {
            movA.push_front(a.back());
            a.pop_back();
        }
        while (b.size() % T) {
            movB.push_front(b.back());
            b.pop_back();
        }
        int pos = 0;
        for (int t : a) place[t] = pos++;
        for (int t : b) place[t] = pos++;
        for (int t : movA) place[t] = pos++;
        for (int t : movB) place[t] = pos++;
        for (int t : core) place[t] = pos++;
        for (int t : rep) place[t] = pos++;
        // pressures ordered before one of their faces move to the end of S
        std::vector<char> late(n, 0);
        bool any = false;
        for (int t = 0; t < n; ++t) {
            if (f.comp[t] != nd) continue;
            const int64_t q = u[t] / c->nrec;
            bool bad = false;
            for (int d = 0; d < nd && !bad; ++d) {
                int64_t lo_s = c->nbr[q * 6 + 2 * d] >= 0 ? (int64_t)c->nrec * q + d : -1;
                int64_t up = c->nbr[q * 6 + 2 * d + 1];
                int64_t hi_s = up >= 0 ? (int64_t)c->nrec * up + d : -1;
                for (int64_t fs : {lo_s, hi_s}) {
                    if (fs < 0) continue;
                    const int k = index_of(fs);
                    if (k >= 0 && place[k] > place[t]) bad = true;
                }
            }
            if (bad && std::find(rep.begin(), rep.end(), t) == rep.end()) {
                late[t] = 1;
                any = true;
            }
        }
        if (!any) break;
        auto drop = [&](std::vector<int>& v) { v.erase(std::remove_if(v.begin(), v.end(), [&](int t) { return late[t]; }), v.end()); };
        auto dropq = [&](std::deque<int>& v) { v.erase(std::remove_if(v.begin(), v.end(), [&](int t) { return late[t]; }), v.end()); };
        drop(a);
        drop(b);
        dropq(movA);
        dropq(movB);
        drop(core);
        for (int t = 0; t < n; ++t)
            if (late[t]) rep.push_back(t);
        if (round == 63) return false;
    }
    const int nS = (int)(movA.size() + movB.size() + core.size() + rep.size());
    if (a.empty() || b.empty() || nS * 4 > n || nS > 4096) return false;
    // the halves must be uncoupled
    std::vector<char> part(n, 2);
    for (int t : a) part[t] = 0;
    for (int t : b) part[t] = 1;
    std::vector<int64_t> cols;
    for (int t = 0; t < n; ++t) {
        if (part[t] == 2) continue;
        row_pattern(c, u[t], cols);
        for (int64_t s : cols) {
            const int k = index_of(s);
            if (k >= 0 && part[k] != 2 && part[k] != part[t]) return false;
        }
    }
    A.clear();
    B.clear();
    S.clear();
    for (int t : a) A.push_back(u[t]);
    for (int t : b) B.push_back(u[t]);
    for (int t : movA) S.push_back(u[t]);
    for (int t : movB) S.push_back(u[t]);
    for (int t : core) S.push_back(u[t]);
    for (int t : rep) S.push_back(u[t]);
    return true;
}

}  // namespace

int build_local_problems(gplmm_ctx* c) {
    const int T = c->tile;
    const int nsub = c->Np + c->Nc;
    c->nsub_main = nsub;
    c->subs.assign(nsub, {});
    c->splits.clear();
    c->sinv_elems = 0;
    c->max_sep_ld = 0;
    c->sub_slots.clear();
    c->env_tfc.clear();
    c->env_tfr.clear();
    c->env_lrow.clear();
    c->env_urow.clear();
    c->env_tlc.clear();
    std::vector<std::vector<int32_t>> prim_cells(c->Np);
    for (int64_t q = 0; q < c->ncell; ++q)
        if (c->prim[q] >= 0) prim_cells[c->prim[q]].push_back((int32_t)q);
    int64_t elems = 0;
    c->maxT = 0;
    std::vector<int64_t> cols;
    // the tile skyline of a subdomain whose unknowns are `ordered` (its local order); dense:
    // every tile present (the separators, whose Schur complement fills in)
    auto add_sub = [&](Sub& sb, const std::vector<int64_t>& ordered, bool dense) {
        const int n = (int)ordered.size();
        sb.n = n;
        sb.nT = (n + T - 1) / T;
        c->maxT = std::max(c->maxT, sb.nT);
        sb.slot_off = (int64_t)c->sub_slots.size();
        for (int64_t v : ordered) c->sub_slots.push_back((int32_t)v);
        // global slot -> local index (sorted lookup)
        std::vector<std::pair<int64_t, int>> inv(n);
        for (int t = 0; t < n; ++t) inv[t] = {ordered[t], t};
        std::sort(inv.begin(), inv.end());
        auto local = [&](int64_t s) -> int {
            auto it = std::lower_bound(inv.begin(), inv.end(), std::make_pair(s, -1));
            return (it != inv.end() && it->first == s) ? it->second : -1;
        };
        std::vector<int> fc(n), fr(n);
        for (int r = 0; r < n; ++r) fc[r] = fr[r] = dense ? 0 : r;
        if (!dense)
            for (int r = 0; r < n; ++r) {
                row_pattern(c, ordered[r], cols);
                for (int64_t s : cols) {
                    int lc = local(s);
                    if (lc < 0) continue;
                    fc[r] = std::min(fc[r], lc);
                    fr[lc] = std::min(fr[lc], r);
                }
            }
        sb.env_off = (int64_t)c->env_tfc.size();
        std::vector<int> tfc(sb.nT), tfr(sb.nT);
        for (int I = 0; I < sb.nT; ++I) {
            tfc[I] = I;
            tfr[I] = I;
            for (int r = I * T; r < std::min(n, (I + 1) * T); ++r) {
                tfc[I] = std::min(tfc[I], fc[r] / T);
                tfr[I] = std::min(tfr[I], fr[r] / T);
            }
        }
        for (int I = sb.nT - 2; I >= 0; --I) {   // monotone skyline
            tfc[I] = std::min(tfc[I], tfc[I + 1]);
            tfr[I] = std::min(tfr[I], tfr[I + 1]);
        }
        sb.diag_off = elems;
        elems += (int64_t)sb.nT * T * T;
        for (int I = 0; I < sb.nT; ++I) {
            c->env_tfc.push_back(tfc[I]);
            c->env_tfr.push_back(tfr[I]);
            c->env_lrow.push_back(elems);
            elems += (int64_t)(I - tfc[I]) * T * T;
        }
        // U by tile rows: row I holds columns I+1 .. tlc[I], tlc[I] = last J with tfr[J] <= I
        for (int I = 0, J = 0; I < sb.nT; ++I) {
            while (J + 1 < sb.nT && tfr[J + 1] <= I) ++J;
            const int last = std::max(J, I);
            c->env_tlc.push_back(last);
            c->env_urow.push_back(elems);
            elems += (int64_t)(last - I) * T * T;
        }
    };
    for (int sidx = 0; sidx < nsub; ++sidx) {
        Sub& sb = c->subs[sidx];
        sb.kind = sidx < c->Np ? 0 : 1;
        sb.id = sidx < c->Np ? sidx : sidx - c->Np;
        sb.sep0 = 0;
        sb.skip_ss = 0;
        const std::vector<int32_t>& cells = sb.kind == 0 ? prim_cells[sb.id] : c->dual_cells[sb.id];
        std::vector<int64_t> u = unknowns_of(c, cells);
        std::vector<std::pair<int64_t, int64_t>> keyed(u.size());
        std::vector<int64_t> keys = local_keys(c, cells, u);
        for (size_t t = 0; t < u.size(); ++t) keyed[t] = {keys[t], u[t]};
        std::sort(keyed.begin(), keyed.end());
        std::vector<int64_t> ordered(u.size());
        for (size_t t = 0; t < u.size(); ++t) ordered[t] = keyed[t].second;
        add_sub(sb, ordered, false);
    }
    // ---- Eq. xf (mg_form 1, 2): the f-faces' block A^f_f, one subdomain per connected
    // component of the f-faces under X's couplings, unknowns in slot order
    c->n_fsub = 0;
    if (c->opt.mg_form != 0) {
        std::vector<int64_t> fslots;
        for (int64_t sl = 0; sl < c->N; ++sl)
            if ((int)(sl % c->nrec) < c->ndim && c->owner[sl] == -1) fslots.push_back(sl);
        const int64_t nf = (int64_t)fslots.size();
        auto fidx = [&](int64_t sl) -> int64_t {
            auto it = std::lower_bound(fslots.begin(), fslots.end(), sl);
            return (it != fslots.end() && *it == sl) ? (int64_t)(it - fslots.begin()) : -1;
        };
        UF uf(nf);
        for (int64_t k = 0; k < nf; ++k) {
            row_pattern(c, fslots[k], cols);
            for (int64_t cl : cols) {
                const int64_t m = fidx(cl);
                if (m >= 0) uf.unite(k, m);
            }
        }
        std::vector<int64_t> comp_of(nf, -1);
        std::vector<std::vector<int64_t>> comps;
        for (int64_t k = 0; k < nf; ++k) {   // components numbered by their first slot
            const int64_t r = uf.find(k);
            if (comp_of[r] < 0) {
                comp_of[r] = (int64_t)comps.size();
                comps.emplace_back();
            }
            comps[comp_of[r]].push_back(fslots[k]);
        }
        for (size_t k = 0; k < comps.size(); ++k) {
            Sub sb{};
            sb.kind = 4;
            sb.id = (int)k;
            sb.split = -1;
            add_sub(sb, comps[k], false);
            c->subs.push_back(sb);
        }
        c->n_fsub = (int)comps.size();
        c->nsub_main = nsub + c->n_fsub;
    }
    // ---- nested dissection of the primaries whose blocks span more than split_tiles tiles
    // (single images; the split parts follow the duals)
    const int thr = c->opt.split_tiles;   // 0 (default) and -1: never
    if (thr > 0 && c->samples.size() <= 1) {
        for (int i = 0; i < c->Np; ++i) {
            if (c->subs[i].nT <= thr) continue;
            std::vector<int64_t> A, B, S;
            if (!plan_split(c, prim_cells[i], A, B, S)) continue;
            Split sp;
            sp.prim = i;
            sp.nA = (int)A.size();
            sp.nB = (int)B.size();
            sp.nS = (int)S.size();
            std::vector<int64_t> as(A), bs(B);
            as.insert(as.end(), S.begin(), S.end());
            bs.insert(bs.end(), S.begin(), S.end());
            Sub sa{}, sbb{}, ss{};
            sa.split = sbb.split = ss.split = -1;
            sa.kind = sbb.kind = 2;
            ss.kind = 3;
            sa.id = sbb.id = ss.id = i;
            sa.sep0 = sp.nA;
            sbb.sep0 = sp.nB;
            sbb.skip_ss = 1;
            add_sub(sa, as, false);
            add_sub(sbb, bs, false);
            add_sub(ss, S, true);
            sp.ld = ss.nT * T;
            sp.inv_off = c->sinv_elems;
            c->sinv_elems += (int64_t)sp.ld * sp.ld;
            c->max_sep_ld = std::max(c->max_sep_ld, sp.ld);
            sp.a_sub = (int)c->subs.size();
            c->subs.push_back(sa);
            sp.b_sub = (int)c->subs.size();
            c->subs.push_back(sbb);
            sp.s_sub = (int)c->subs.size();
            c->subs.push_back(ss);
            c->splits.push_back(sp);
        }
    }
    c->factor_elems = elems;
    // the solves address a subdomain's tiles by 32-bit offsets from its first diagonal tile
    for (size_t k = 0; k < c->subs.size(); ++k) {
        const int64_t end = k + 1 < c->subs.size() ? c->subs[k + 1].diag_off : elems;
        if (end - c->subs[k].diag_off > (int64_t)INT32_MAX)
            return fail(c, GPLMM_E_ARG, "a local factor exceeds 2^31 elements");
    }
    // ---- LU schedules: set 0 = the primaries' Schwarz blocks (split primaries by their two
    // halves, eliminated up to the separator), set 1 = the primaries' closures and the
    // duals, set 2 = the separators' Schur complements
    std::vector<int> stop(c->subs.size());
    for (size_t s = 0; s < c->subs.size(); ++s) {
        Sub& sb = c->subs[s];
        sb.split = -1;
        stop[s] = sb.nT;
    }
    for (size_t k = 0; k < c->splits.size(); ++k) {
        const Split& sp = c->splits[k];
        c->subs[sp.prim].split = c->subs[sp.a_sub].split = c->subs[sp.b_sub].split = c->subs[sp.s_sub].split = (int)k;
        stop[sp.a_sub] = sp.nA / T;
        stop[sp.b_sub] = sp.nB / T;
    }
    for (int set = 0; set < 3; ++set) {
        std::vector<int> members;
        for (int s = 0; s < (int)c->subs.size(); ++s) {
            const Sub& sb = c->subs[s];
            const bool in = set == 0 ? ((sb.kind == 0 && sb.split < 0) || sb.kind == 2)
                                     : (set == 1 ? s < c->nsub_main : sb.kind == 3);
            if (in) members.push_back(s);
        }
        auto& off = c->lu_step_off[set];
        auto& pr = c->lu_step_pairs[set];
        auto& soff = c->lu_sub_off[set];
        auto& sl = c->lu_sub_list[set];
        off.assign(1, 0);
        soff.assign(1, 0);
        pr.clear();
        sl.clear();
        double products = 0.0;   // T x T tile products of the factorisation (panels, updates)
        int steps = 0;
        for (int s : members) steps = std::max(steps, stop[s]);
        for (int K = 0; K < steps; ++K) {
            for (int s : members) {
                const Sub& sb = c->subs[s];
                if (stop[s] <= K) continue;
                sl.push_back(s);
                const int* tfc = &c->env_tfc[sb.env_off];
                const int width = c->env_tlc[sb.env_off + K] - K;   // U panel tiles of step K
                products += width;
                for (int I = K + 1; I < sb.nT && tfc[I] <= K; ++I) {
                    pr.push_back(s);
                    pr.push_back(I);
                    products += 1.0 + width;                         // L panel tile, trailing row
                }
            }
            off.push_back((int64_t)pr.size() / 2);
            soff.push_back((int64_t)sl.size());
        }
        c->lu_flops[set] = 2.0 * (double)T * T * T * products;
    }
    // ---- shape/correction blocks: per primary |S| x (|Cp| + 1), column-major
    c->phi_off.assign(c->Np, 0);
    c->phi_cols_off.assign(c->Np + 1, 0);
    c->phi_cols.clear();
    c->ycol.assign(c->Np, -1);
    int64_t pe = 0;
    int ny = 0;
    for (int i = 0; i < c->Np; ++i) {
        c->phi_off[i] = pe;
        pe += (int64_t)c->subs[i].n * ((int64_t)c->Cp[i].size() + 1);
        for (int32_t j : c->Cp[i]) c->phi_cols.push_back(j);
        // a correction vector (and a coarse y unknown) only when b_B is nonzero on the primary
        bool nonzero = false;
        for (int t = 0; t < c->subs[i].n && !nonzero; ++t) {
            int64_t s = c->sub_slots[c->subs[i].slot_off + t];
            int comp = (int)(s % c->nrec);
            const Phys& ph = c->csamp.empty() ? c->phys : c->sphys[c->csamp[s / c->nrec]];
            if (comp < c->ndim && ph.body[comp] != 0.0) nonzero = true;
        }
        if (nonzero) c->ycol[i] = c->Nc + ny++;
        c->phi_cols.push_back(c->ycol[i]);
        c->phi_cols_off[i + 1] = (int64_t)c->phi_cols.size();
    }
    c->phi_elems = pe;
    c->Ny = ny;
    c->nco = c->Nc + ny;
    return GPLMM_OK;
}

// Coarse operator by probing: columns whose restricted images Rhat X Phat e_col touch
// disjoint coarse rows share a colour; Rhat X Phat (sum of a colour's columns) then
// yields every entry of those columns at once.
int build_probing(gplmm_ctx* c) {
    const int nd = c->ndim;
    const int64_t nc = c->ncell;
    const int nco = c->nco;
    // record cells of each row group (interfaces: their cells; primaries: cells holding S_i slots)
    std::vector<std::vector<int32_t>> group_cells(nco);
    for (int j = 0; j < c->Nc; ++j) group_cells[j] = c->icells[j];
    std::vector<std::vector<int32_t>> prim_rec(c->Np);
    for (int i = 0; i < c->Np; ++i) {
        const Sub& sb = c->subs[i];
        std::vector<int32_t> cells;
        for (int t = 0; t < sb.n; ++t) cells.push_back(c->sub_slots[sb.slot_off + t] / c->nrec);
        std::sort(cells.begin(), cells.end());
        cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
        prim_rec[i] = cells;
        if (c->ycol[i] >= 0) group_cells[c->ycol[i]] = cells;
    }
    // cell -> groups containing it
    std::vector<std::vector<int32_t>> cell_groups(nc);
    for (int g = 0; g < nco; ++g)
        for (int32_t q : group_cells[g]) cell_groups[q].push_back(g);
    // support cells of each coarse column
    std::vector<std::vector<int32_t>> col_cells(nco);
    for (int j = 0; j < c->Nc; ++j) col_cells[j] = c->icells[j];
    for (int i = 0; i < c->Np; ++i) {
        for (int32_t j : c->Cp[i])
            col_cells[j].insert(col_cells[j].end(), prim_rec[i].begin(), prim_rec[i].end());
        if (c->ycol[i] >= 0) col_cells[c->ycol[i]] = prim_rec[i];
    }
    std::vector<int32_t> mark_cell(nc, -1), mark_group(nco, -1);
    std::vector<std::vector<int32_t>> Q(nco);
    for (int col = 0; col < nco; ++col) {
        std::vector<int32_t>& q = Q[col];
        auto visit = [&](int64_t x) {
            if (x < 0 || mark_cell[x] == col) return;
            mark_cell[x] = col;
            for (int32_t g : cell_groups[x])
                if (mark_group[g] != col) {
                    mark_group[g] = col;
                    q.push_back(g);
                }
        };
        const bool jac = c->opt.build_matrix == GPLMM_BUILD_JACOBIAN;
        for (int32_t x : col_cells[col]) {
            visit(x);
            for (int e = 0; e < 2 * nd; ++e) {
                const int64_t y = c->nbr[(int64_t)x * 6 + e];
                visit(y);
                // the Jacobian's transverse couplings also reach the diagonal neighbours
                if (jac && y >= 0)
                    for (int e2 = 0; e2 < 2 * nd; ++e2)
                        if (e2 / 2 != e / 2) visit(c->nbr[y * 6 + e2]);
            }
        }
        std::sort(q.begin(), q.end());
    }
    // greedy colouring
    std::vector<std::vector<uint64_t>> used;   // per row: bitset of colours claiming it
    std::vector<int> color(nco, -1);
    std::vector<std::vector<uint64_t>> claim;  // claim[color] bitset over rows
    int ncol = 0;
    for (int col = 0; col < nco; ++col) {
        int chosen = -1;
        for (int k = 0; k < ncol && chosen < 0; ++k) {
            bool ok = true;
            for (int32_t r : Q[col])
                if (claim[k][r >> 6] >> (r & 63) & 1ull) {
                    ok = false;
                    break;
                }
            if (ok) chosen = k;
        }
        if (chosen < 0) {
            chosen = ncol++;
            claim.emplace_back((nco + 63) / 64, 0ull);
        }
        color[col] = chosen;
        for (int32_t r : Q[col]) claim[chosen][r >> 6] |= 1ull << (r & 63);
    }
    c->ncolors = ncol;
    c->color_off.assign(ncol + 1, 0);
    c->color_col_off.assign(ncol + 1, 0);
    std::vector<std::vector<int32_t>> cols_of(ncol);
    for (int col = 0; col < nco; ++col) cols_of[color[col]].push_back(col);
    c->probe.clear();
    c->color_cols.clear();
    for (int k = 0; k < ncol; ++k) {
        for (int32_t col : cols_of[k]) {
            c->color_cols.push_back(col);
            for (int32_t r : Q[col]) c->probe.push_back({r, col});
        }
        c->color_off[k + 1] = (int64_t)c->probe.size();
        c->color_col_off[k + 1] = (int64_t)c->color_cols.size();
    }
    return GPLMM_OK;
}


// ------------------------------------------------------------------------------------------
// Batches: the decompositions of independent samples placed side by side
// ------------------------------------------------------------------------------------------

// Concatenate the decompositions of the parts (each built alone from its own image): cells,
// primaries, interfaces and slots of sample s follow those of samples 0..s-1, every index
// shifted by the offsets of its kind.  No cell of one sample neighbours a cell of another, so
// the stencils, subdomains and coarse couplings of the batch are those of the samples.
int merge_samples(gplmm_ctx* c, std::vector<gplmm_ctx*>& parts) {
    c->samples.clear();
    c->cidx.clear();
    c->cell_voxel.clear();
    c->nbr.clear();
    c->iface.clear();
    c->prim.clear();
    c->owner.clear();
    c->tagslot.clear();
    c->noclose.clear();
    c->tagcell.clear();
    c->Cp.clear();
    c->icells.clear();
    c->dual_cells.clear();
    c->csamp.clear();
    c->Np = c->Nc = 0;
    c->nface = 0;
    int64_t voff = 0, coff = 0;
    for (size_t si = 0; si < parts.size(); ++si) {
        const gplmm_ctx* p = parts[si];
        if (p->ndim != c->ndim) return fail(c, GPLMM_E_ARG, "all samples of a batch must have the same dimension");
        c->samples.push_back(SampleGeo{voff, coff, p->nx, p->ny, p->nz, c->Np, c->Nc});
        for (int32_t q : p->cidx) c->cidx.push_back(q >= 0 ? (int32_t)(q + coff) : -1);
        for (int32_t v : p->cell_voxel) c->cell_voxel.push_back((int32_t)(v + voff));
        for (int32_t q : p->nbr) c->nbr.push_back(q >= 0 ? (int32_t)(q + coff) : -1);
        for (int32_t j : p->iface) c->iface.push_back(j >= 0 ? j + c->Nc : -1);
        for (int32_t i : p->prim) c->prim.push_back(i >= 0 ? i + c->Np : -1);
        for (int32_t o : p->owner) c->owner.push_back(o >= 0 ? o + c->Np : o);
        c->tagslot.insert(c->tagslot.end(), p->tagslot.begin(), p->tagslot.end());
        c->noclose.insert(c->noclose.end(), p->noclose.begin(), p->noclose.end());
        c->tagcell.insert(c->tagcell.end(), p->tagcell.begin(), p->tagcell.end());
        for (const auto& v : p->Cp) {
            std::vector<int32_t> w(v);
            for (auto& j : w) j += c->Nc;
            c->Cp.push_back(w);
        }
        for (const auto& v : p->icells) {
            std::vector<int32_t> w(v);
            for (auto& q : w) q += (int32_t)coff;
            c->icells.push_back(w);
        }
        for (const auto& v : p->dual_cells) {
            std::vector<int32_t> w(v);
            for (auto& q : w) q += (int32_t)coff;
            c->dual_cells.push_back(w);
        }
        c->csamp.insert(c->csamp.end(), (size_t)p->ncell, (int32_t)si);
        if (si == 0) c->pin = p->pin;
        c->Np += p->Np;
        c->Nc += p->Nc;
        c->nface += p->nface;
        voff += p->nvox;
        coff += p->ncell;
    }
    if (coff > INT32_MAX / 8) return fail(c, GPLMM_E_ARG, "the batch has too many cells");
    c->nvox = voff;
    c->ncell = coff;
    c->N = (int64_t)c->nrec * coff;
    return GPLMM_OK;
}

// Coarse blocks: the interfaces and correction unknowns of one sample couple only among
// themselves, so the coarse operator is block diagonal with one block per sample.
void build_coarse_blocks(gplmm_ctx* c) {
    c->cblk_n.clear();
    c->cblk_idx.clear();
    c->cblk_ioff.assign(1, 0);
    c->cblk_moff.assign(1, 0);
    c->co_blk.assign(c->nco, -1);
    c->co_loc.assign(c->nco, -1);
    const int ns = (int)c->samples.size();
    for (int si = 0; si < ns; ++si) {
        const int i0 = c->samples[si].i0, i1 = si + 1 < ns ? c->samples[si + 1].i0 : c->Nc;
        const int p0 = c->samples[si].p0, p1 = si + 1 < ns ? c->samples[si + 1].p0 : c->Np;
        const int b = (int)c->cblk_n.size();
        int n = 0;
        auto add = [&](int g) {
            c->co_blk[g] = b;
            c->co_loc[g] = n++;
            c->cblk_idx.push_back(g);
        };
        for (int j = i0; j < i1; ++j) add(j);
        for (int i = p0; i < p1; ++i)
            if (c->ycol[i] >= 0) add(c->ycol[i]);
        c->cblk_n.push_back(n);
        c->cblk_ioff.push_back((int64_t)c->cblk_idx.size());
        c->cblk_moff.push_back(c->cblk_moff.back() + (int64_t)n * n);
    }
    c->co_elems = c->cblk_moff.back();
    c->cblk_max = c->cblk_n.empty() ? 0 : *std::max_element(c->cblk_n.begin(), c->cblk_n.end());
}

}  // namespace gp

// Host-side mesh setup for the WLS-ENO library: geometry, sibling half-facets
// (Sec. 3.3.1), k-ring stencils with fractional increments (Sec. 3.2),
// reverse Cuthill-McKee renumbering and the device-order records the kernels
// read.  Runs once per mesh / parameter set.
//
// This file is compiled with -ffp-contract=off: the centroid and squared
// centroid distance that order and truncate stencils are part of the
// documented interface and must not pick up fused multiply-adds.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <numeric>
#include <utility>

#include "internal.hpp"

namespace wlseno {

int num_coeffs(int dim, int p)
{
    int count = 0;
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < (dim >= 2 ? p : 1); ++b)
            for (int c = 0; c < (dim >= 3 ? p : 1); ++c)
                if (a + b + c <= p - 1) ++count;
    return count;
}

int points_per_face(int dim, int p)
{
    if (dim == 1) return 1;
    if (dim == 2) return std::max(1, (p + 1) / 2);
    return 3;
}

static Error inval(const std::string &s) { return Error{WLSENO_EINVAL, s}; }

// Graded exponent list (degree ascending, descending lexicographic in a degree).
static std::vector<std::array<int, 3>> basis_exponents(int dim, int p)
{
    std::vector<std::array<int, 3>> out;
    for (int q = 0; q <= p - 1; ++q) {
        if (dim == 1) {
            out.push_back({q, 0, 0});
        } else if (dim == 2) {
            for (int a = q; a >= 0; --a) out.push_back({a, q - a, 0});
        } else {
            for (int a = q; a >= 0; --a)
                for (int b = q - a; b >= 0; --b) out.push_back({a, b, q - a - b});
        }
    }
    return out;
}

// ------------------------------------------------------------------ mesh

void mesh_setup(HostMesh &out, int dim, int64_t nv, const double *xyz, int64_t nc,
                const int32_t *cells, uint32_t flags)
{
    if (dim < 1 || dim > 3) throw inval("dim must be 1, 2 or 3");
    if (!xyz || !cells) throw inval("null mesh array");
    if (nv < dim + 1 || nc < 1) throw inval("mesh needs at least one cell and dim+1 vertices");
    if (nc > (int64_t)(INT32_MAX / 8) || nv > (int64_t)INT32_MAX)
        throw inval("mesh too large for 32-bit indices");
    if (flags & ~(WLSENO_MESH_PERIODIC_1D | WLSENO_MESH_PERIODIC_2D)) throw inval("unknown mesh flags");
    if ((flags & WLSENO_MESH_PERIODIC_1D) && dim != 1) throw inval("WLSENO_MESH_PERIODIC_1D requires dim = 1");
    if ((flags & WLSENO_MESH_PERIODIC_2D) && dim != 2) throw inval("WLSENO_MESH_PERIODIC_2D requires dim = 2");
    const bool periodic = (flags & (WLSENO_MESH_PERIODIC_1D | WLSENO_MESH_PERIODIC_2D)) != 0;

    HostMesh m;
    m.dim = dim;
    m.nv = nv;
    m.nc = nc;
    m.periodic = periodic;
    const int nvc = dim + 1;
    m.xyz.assign(xyz, xyz + nv * dim);
    m.cells.assign(cells, cells + nc * nvc);
    for (int64_t t = 0; t < nc * nvc; ++t)
        if (m.cells[t] < 0 || m.cells[t] >= nv)
            throw inval("cell " + std::to_string(t / nvc) + " references vertex " +
                        std::to_string(m.cells[t]) + " out of range");
    if (periodic && dim == 1) {
        m.period = xyz[nv - 1] - xyz[0];
        if (!(m.period > 0.0)) throw inval("periodic 1-D mesh: last node must lie right of the first");
    }
    m.vid = m.cells;
    if (periodic && dim == 1)
        for (auto &v : m.vid)
            if (v == nv - 1) v = 0;
    if (periodic && dim == 2) {
        // one id per point of the torus: a vertex on an upper side stands for
        // its partner on the lower side (same other coordinate)
        double lo[2] = {xyz[0], xyz[1]}, hi[2] = {xyz[0], xyz[1]};
        for (int64_t v = 0; v < nv; ++v)
            for (int d = 0; d < 2; ++d) {
                lo[d] = std::min(lo[d], xyz[v * 2 + d]);
                hi[d] = std::max(hi[d], xyz[v * 2 + d]);
            }
        m.period = hi[0] - lo[0];
        m.period_y = hi[1] - lo[1];
        if (!(m.period > 0.0) || !(m.period_y > 0.0)) throw inval("periodic 2-D mesh: degenerate bounding box");
        const double tol[2] = {1e-12 * m.period, 1e-12 * m.period_y};
        std::map<std::pair<double, double>, int32_t> rep;
        std::vector<int32_t> ident(nv);
        std::vector<char> upper(nv, 0);
        for (int64_t v = 0; v < nv; ++v) {
            double c[2];
            for (int d = 0; d < 2; ++d) {
                c[d] = xyz[v * 2 + d];
                if (std::fabs(c[d] - lo[d]) <= tol[d]) c[d] = lo[d];
                if (std::fabs(c[d] - hi[d]) <= tol[d]) upper[v] = 1;
            }
            if (!upper[v]) ident[v] = rep.emplace(std::make_pair(c[0], c[1]), (int32_t)v).first->second;
        }
        for (int64_t v = 0; v < nv; ++v) {
            if (!upper[v]) continue;
            double c[2];
            for (int d = 0; d < 2; ++d) {
                c[d] = xyz[v * 2 + d];
                if (std::fabs(c[d] - lo[d]) <= tol[d] || std::fabs(c[d] - hi[d]) <= tol[d]) c[d] = lo[d];
            }
            auto it = rep.find(std::make_pair(c[0], c[1]));
            if (it == rep.end())
                throw inval("periodic 2-D mesh: vertex " + std::to_string(v) + " on an upper side has no partner");
            ident[v] = it->second;
        }
        for (auto &v : m.vid) v = ident[v];
    }

    // measures and centroids
    m.vol.resize(nc);
    m.cent.resize(nc * dim);
    for (int64_t c = 0; c < nc; ++c) {
        const int32_t *cv = &m.cells[c * nvc];
        const double *x0 = &xyz[(int64_t)cv[0] * dim];
        double vol;
        if (dim == 1) {
            vol = xyz[cv[1]] - xyz[cv[0]];
        } else if (dim == 2) {
            const double *x1 = &xyz[(int64_t)cv[1] * 2], *x2 = &xyz[(int64_t)cv[2] * 2];
            vol = 0.5 * ((x1[0] - x0[0]) * (x2[1] - x0[1]) - (x1[1] - x0[1]) * (x2[0] - x0[0]));
        } else {
            const double *x1 = &xyz[(int64_t)cv[1] * 3], *x2 = &xyz[(int64_t)cv[2] * 3],
                         *x3 = &xyz[(int64_t)cv[3] * 3];
            double a[3], b[3], e[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = x1[d] - x0[d];
                b[d] = x2[d] - x0[d];
                e[d] = x3[d] - x0[d];
            }
            double det = a[0] * (b[1] * e[2] - b[2] * e[1]) - a[1] * (b[0] * e[2] - b[2] * e[0]) +
                         a[2] * (b[0] * e[1] - b[1] * e[0]);
            vol = det / 6.0;
        }
        if (!(vol > 0.0))
            throw inval("cell " + std::to_string(c) + " has non-positive measure (orientation or degenerate)");
        m.vol[c] = vol;
        for (int d = 0; d < dim; ++d) {
            double s = xyz[(int64_t)cv[0] * dim + d];
            for (int v = 1; v < nvc; ++v) s = s + xyz[(int64_t)cv[v] * dim + d];
            m.cent[c * dim + d] = s / (double)nvc;
        }
    }

    // sibling half-facets: equal sorted vertex sets
    struct HF {
        int32_t k[3];
        int32_t cell, lf;
    };
    std::vector<HF> hf;
    hf.reserve(nc * nvc);
    for (int64_t c = 0; c < nc; ++c)
        for (int lf = 0; lf < nvc; ++lf) {
            HF h{{-1, -1, -1}, (int32_t)c, lf};
            int t = 0;
            for (int v = 0; v < nvc; ++v)
                if (v != lf) h.k[t++] = m.vid[c * nvc + v];
            std::sort(h.k, h.k + t);
            hf.push_back(h);
        }
    auto key_less = [](const HF &a, const HF &b) {
        if (a.k[0] != b.k[0]) return a.k[0] < b.k[0];
        if (a.k[1] != b.k[1]) return a.k[1] < b.k[1];
        if (a.k[2] != b.k[2]) return a.k[2] < b.k[2];
        if (a.cell != b.cell) return a.cell < b.cell;
        return a.lf < b.lf;
    };
    auto key_eq = [](const HF &a, const HF &b) {
        return a.k[0] == b.k[0] && a.k[1] == b.k[1] && a.k[2] == b.k[2];
    };
    std::sort(hf.begin(), hf.end(), key_less);
    m.sib.assign(nc * nvc, -1);
    for (size_t t = 0; t < hf.size();) {
        size_t u = t + 1;
        while (u < hf.size() && key_eq(hf[t], hf[u])) ++u;
        if (u - t > 2)
            throw inval("facet shared by more than two cells (cell " + std::to_string(hf[t].cell) + ")");
        if (u - t == 2) {
            const HF &a = hf[t], &b = hf[t + 1];
            m.sib[(int64_t)a.cell * nvc + a.lf] = (b.cell << 2) | b.lf;
            m.sib[(int64_t)b.cell * nvc + b.lf] = (a.cell << 2) | a.lf;
        }
        t = u;
    }

    // vertex -> cells
    m.v2c_ptr.assign(nv + 1, 0);
    for (int64_t t = 0; t < nc * nvc; ++t) m.v2c_ptr[m.vid[t] + 1]++;
    for (int64_t v = 0; v < nv; ++v) m.v2c_ptr[v + 1] += m.v2c_ptr[v];
    m.v2c.assign(m.v2c_ptr[nv], 0);
    {
        std::vector<int32_t> fill(m.v2c_ptr.begin(), m.v2c_ptr.end() - 1);
        for (int64_t c = 0; c < nc; ++c)
            for (int v = 0; v < nvc; ++v) {
                int32_t vv = m.vid[c * nvc + v];
                // a cell lists a vertex once (distinct ids since measure > 0)
                m.v2c[fill[vv]++] = (int32_t)c;
            }
    }

    // unique vertex pairs: edges (mean length h) and, in 3-D, edge -> cells
    if (dim == 1) {
        double s = 0.0;
        for (int64_t c = 0; c < nc; ++c) s += m.vol[c];
        m.h = s / (double)nc;
    } else {
        const int np = dim == 2 ? 3 : 6;
        static const int pr[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        static const int pr2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        std::vector<std::pair<int64_t, int64_t>> ek;   // (key, cell*8 + local pair)
        ek.reserve(nc * np);
        for (int64_t c = 0; c < nc; ++c)
            for (int t = 0; t < np; ++t) {
                int a = dim == 2 ? pr2[t][0] : pr[t][0], b = dim == 2 ? pr2[t][1] : pr[t][1];
                int64_t va = m.vid[c * nvc + a], vb = m.vid[c * nvc + b];
                if (va > vb) std::swap(va, vb);
                ek.push_back({va * nv + vb, c * 8 + t});
            }
        std::sort(ek.begin(), ek.end());
        double sum = 0.0;
        int64_t ne = 0;
        if (dim == 3) m.cell_edges.assign(nc * 6, -1);
        std::vector<int32_t> e2c_ptr{0}, e2c;
        for (size_t t = 0; t < ek.size();) {
            size_t u = t;
            int64_t key = ek[t].first;
            int64_t va = key / nv, vb = key % nv;
            double l2 = 0.0;
            for (int d = 0; d < dim; ++d) {
                double dx = xyz[vb * dim + d] - xyz[va * dim + d];
                l2 += dx * dx;
            }
            sum += std::sqrt(l2);
            while (u < ek.size() && ek[u].first == key) {
                if (dim == 3) {
                    int64_t c = ek[u].second / 8;
                    int lt = (int)(ek[u].second % 8);
                    m.cell_edges[c * 6 + lt] = (int32_t)ne;
                    e2c.push_back((int32_t)c);
                }
                ++u;
            }
            if (dim == 3) e2c_ptr.push_back((int32_t)e2c.size());
            ++ne;
            t = u;
        }
        m.h = sum / (double)ne;
        if (dim == 3) {
            m.e2c_ptr = std::move(e2c_ptr);
            m.e2c = std::move(e2c);
        }
    }
    out = std::move(m);
}

// -------------------------------------------------------------- stencils

namespace {

enum Kind { FACET = 0, EDGE = 1, VERTEX = 2 };

struct RingSet {
    std::vector<int32_t> mark;   // mark[c] == stamp  <=>  c in the current set
    int32_t stamp = 0;
    std::vector<int32_t> items;

    explicit RingSet(int64_t nc) : mark(nc, 0) {}
    void clear()
    {
        items.clear();
        if (++stamp == INT32_MAX) {
            std::fill(mark.begin(), mark.end(), 0);
            stamp = 1;
        }
    }
    void add(int32_t c)
    {
        if (mark[c] != stamp) {
            mark[c] = stamp;
            items.push_back(c);
        }
    }
};

void add_ring(const HostMesh &m, Kind kind, int32_t j, RingSet &s)
{
    const int nvc = m.dim + 1;
    s.add(j);
    if (kind == FACET) {
        for (int lf = 0; lf < nvc; ++lf) {
            int32_t sb = m.sib[(int64_t)j * nvc + lf];
            if (sb >= 0) s.add(sb >> 2);
        }
        return;
    }
    if (kind == EDGE) {
        for (int t = 0; t < 6; ++t) {
            int32_t e = m.cell_edges[(int64_t)j * 6 + t];
            for (int32_t k = m.e2c_ptr[e]; k < m.e2c_ptr[e + 1]; ++k) s.add(m.e2c[k]);
        }
        return;
    }
    for (int v = 0; v < nvc; ++v) {
        int32_t vv = m.vid[(int64_t)j * nvc + v];
        for (int32_t k = m.v2c_ptr[vv]; k < m.v2c_ptr[vv + 1]; ++k) s.add(m.v2c[k]);
    }
}

double sqdist(const HostMesh &m, int64_t i, int64_t j)
{
    double d2 = 0.0;
    for (int d = 0; d < m.dim; ++d) {
        double dx = m.cent[j * m.dim + d] - m.cent[i * m.dim + d];
        const double L = m.periodic ? (d == 0 ? m.period : (d == 1 ? m.period_y : 0.0)) : 0.0;
        if (L > 0.0) {
            if (dx > 0.5 * L)
                dx -= L;
            else if (dx < -0.5 * L)
                dx += L;
        }
        d2 = d2 + dx * dx;
    }
    return d2;
}

// Stencil of cell i (user ids), centre first, per the documented size rule.
void one_stencil(const HostMesh &m, int64_t i, int n_lo, int n_hi, RingSet &a, RingSet &b,
                 std::vector<std::pair<double, int32_t>> &tmp, int32_t *out, int *count)
{
    std::vector<Kind> kinds;
    if (m.dim == 1)
        kinds = {VERTEX};
    else if (m.dim == 2)
        kinds = {FACET, VERTEX};
    else
        kinds = {FACET, EDGE, VERTEX};
    RingSet *S = &a;
    bool done = false;
    for (Kind k : kinds) {
        S->clear();
        add_ring(m, k, (int32_t)i, *S);
        if ((int)S->items.size() >= n_lo) {
            done = true;
            break;
        }
    }
    if (!done) {
        RingSet *cur = &a, *nxt = &b;   // cur holds the integer level
        while (true) {
            bool big = false;
            for (Kind k : kinds) {
                nxt->clear();
                for (int32_t j : cur->items) nxt->add(j);
                for (size_t t = 0; t < cur->items.size(); ++t) add_ring(m, k, cur->items[t], *nxt);
                if ((int)nxt->items.size() >= n_lo) {
                    big = true;
                    break;
                }
            }
            S = nxt;
            if (big || nxt->items.size() == cur->items.size()) break;
            std::swap(cur, nxt);
        }
    }
    tmp.clear();
    for (int32_t j : S->items)
        if (j != i) tmp.push_back({sqdist(m, i, j), j});
    std::sort(tmp.begin(), tmp.end());
    int keep = std::min<int>((int)tmp.size(), n_hi - 1);
    out[0] = (int32_t)i;
    for (int t = 0; t < keep; ++t) out[t + 1] = tmp[t].second;
    *count = keep + 1;
}

// Reverse Cuthill-McKee over the facet-adjacency graph; returns perm[device] = user.
std::vector<int32_t> rcm_order(const HostMesh &m)
{
    const int64_t nc = m.nc;
    const int nvc = m.dim + 1;
    std::vector<int32_t> deg(nc, 0);
    for (int64_t c = 0; c < nc; ++c)
        for (int lf = 0; lf < nvc; ++lf) deg[c] += m.sib[c * nvc + lf] >= 0;
    std::vector<char> placed(nc, 0);
    std::vector<int32_t> level(nc, -1), order;
    order.reserve(nc);
    std::vector<int32_t> q, touched, nb;
    auto bfs_levels = [&](int32_t root, int32_t &last_level_best, int32_t &ecc) {
        touched.clear();
        q.clear();
        q.push_back(root);
        level[root] = 0;
        touched.push_back(root);
        for (size_t h = 0; h < q.size(); ++h) {
            int32_t x = q[h];
            for (int lf = 0; lf < nvc; ++lf) {
                int32_t s = m.sib[(int64_t)x * nvc + lf];
                if (s < 0) continue;
                int32_t y = s >> 2;
                if (level[y] < 0 && !placed[y]) {
                    level[y] = level[x] + 1;
                    q.push_back(y);
                    touched.push_back(y);
                }
            }
        }
        ecc = level[q.back()];
        int32_t best = q.back();
        for (int32_t x : q)
            if (level[x] == ecc && (deg[x] < deg[best] || (deg[x] == deg[best] && x < best))) best = x;
        last_level_best = best;
        for (int32_t x : touched) level[x] = -1;
    };
    for (int64_t s0 = 0; s0 < nc; ++s0) {
        if (placed[s0]) continue;
        int32_t root = (int32_t)s0, cand, ecc, ecc_prev = -1;
        for (int it = 0; it < 8; ++it) {
            bfs_levels(root, cand, ecc);
            if (ecc <= ecc_prev) break;
            ecc_prev = ecc;
            root = cand;
        }
        size_t head = order.size();
        order.push_back(root);
        placed[root] = 1;
        while (head < order.size()) {
            int32_t x = order[head++];
            nb.clear();
            for (int lf = 0; lf < nvc; ++lf) {
                int32_t s = m.sib[(int64_t)x * nvc + lf];
                if (s >= 0 && !placed[s >> 2]) nb.push_back(s >> 2);
            }
            std::sort(nb.begin(), nb.end(), [&](int32_t p1, int32_t p2) {
                return deg[p1] != deg[p2] ? deg[p1] < deg[p2] : p1 < p2;
            });
            for (int32_t y : nb)
                if (!placed[y]) {
                    placed[y] = 1;
                    order.push_back(y);
                }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

}  // namespace

// --------------------------------------------------------------- build

void build_setup(const HostMesh &m, const wlseno_params &prm, Build &out)
{
    const int dim = m.dim, nvc = dim + 1;
    const int64_t nc = m.nc;
    if (prm.p < 2 || prm.p > 5) throw inval("p must be in 2..5");
    if (dim == 3 && prm.p > 3) throw Error{WLSENO_EUNSUPPORTED, "3-D supports p <= 3"};
    if (dim == 2 && prm.p > 5) throw Error{WLSENO_EUNSUPPORTED, "2-D supports p <= 5"};
    if (prm.flux != WLSENO_FLUX_ADVECTION && prm.flux != WLSENO_FLUX_BURGERS && prm.flux != WLSENO_FLUX_EULER)
        throw inval("flux must be advection, Burgers or Euler");
    if (prm.flux == WLSENO_FLUX_EULER && dim != 2)
        throw Error{WLSENO_EUNSUPPORTED, "the Euler system is compiled for 2-D meshes"};
    if (prm.flux == WLSENO_FLUX_EULER && !(prm.gamma > 1.0)) throw inval("gamma > 1 required");
    if (prm.weight_mode != 0 && prm.weight_mode != 1) throw inval("weight_mode must be 0 or 1");
    if (prm.bc < 0 || prm.bc > 3) throw inval("bc must be 0, 1, 2 or 3");
    if (prm.bc == 3 && prm.flux != WLSENO_FLUX_EULER) throw inval("bc = 3 (slip wall) applies to the Euler system only");
    if (prm.bc == 1 && prm.flux == WLSENO_FLUX_EULER) throw inval("bc = 1 (zero outside state) is not valid for Euler");
    if (prm.characteristic != 0 && prm.characteristic != 1) throw inval("characteristic must be 0 or 1");
    if (prm.characteristic && prm.flux != WLSENO_FLUX_EULER)
        throw inval("characteristic = 1 applies to the Euler system only");
    if (prm.balance != 0 && prm.balance != 1) throw inval("balance must be 0 or 1");
    if (prm.lf_alpha != 0 && prm.lf_alpha != 1) throw inval("lf_alpha must be 0 or 1");
    if (prm.h_mode != 0 && prm.h_mode != 1) throw inval("h_mode must be 0 or 1");
    if (prm.balance && prm.flux == WLSENO_FLUX_EULER) throw inval("balance = 1 applies to scalar fluxes only");
    if (prm.balance && !((dim == 2 || dim == 3) && prm.p == 3))
        throw Error{WLSENO_EUNSUPPORTED, "balanced stencils are compiled for p = 3 in 2-D and 3-D"};
    if (prm.lanes != 0 && prm.lanes != 2 && prm.lanes != 4 && prm.lanes != 8 && prm.lanes != 16)
        throw inval("lanes must be 0, 2, 4, 8 or 16");
    if (!(prm.eps >= 0.0) || !(prm.alpha_w > 0.0) || !(prm.rank_tol >= 0.0))
        throw inval("eps >= 0, alpha_w > 0 and rank_tol >= 0 required");
    // WLS-ENO weights 1/((u_j - u_i)^2 + eps h^2): eps h^2 is the positive
    // constant that keeps them finite where neighbouring averages are equal
    if (prm.weight_mode == 0 && !(prm.eps > 0.0)) throw inval("eps > 0 required with WLS-ENO weights (weight_mode 0)");
    Build b;
    b.prm = prm;
    b.m = num_coeffs(dim, prm.p);
    b.nq = points_per_face(dim, prm.p);
    b.nf = nvc;
    b.nvars = prm.flux == WLSENO_FLUX_EULER ? dim + 2 : 1;
    if (prm.n_lo < 1 || prm.n_hi < prm.n_lo) throw inval("need 1 <= n_lo <= n_hi");
    if (prm.n_hi < b.m) throw inval("n_hi must be at least the number of coefficients m");
    if (prm.n_hi > 64) throw Error{WLSENO_EUNSUPPORTED, "n_hi above 64"};

    // stencils in user order
    const int cap = prm.n_hi;
    std::vector<int32_t> flat(nc * cap);
    std::vector<int32_t> cnt(nc);
    int bad = -1;
#pragma omp parallel
    {
        RingSet a(nc), bb(nc);
        std::vector<std::pair<double, int32_t>> tmp;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < nc; ++i) {
            int k = 0;
            one_stencil(m, i, prm.n_lo, prm.n_hi, a, bb, tmp, &flat[i * cap], &k);
            cnt[i] = k;
        }
    }
    for (int64_t i = 0; i < nc; ++i)
        if (cnt[i] < b.m) {
            bad = (int)i;
            break;
        }
    if (bad >= 0)
        throw inval("stencil of cell " + std::to_string(bad) + " has " + std::to_string(cnt[bad]) +
                    " cells, fewer than the " + std::to_string(b.m) + " coefficients");
    b.row_ptr.assign(nc + 1, 0);
    for (int64_t i = 0; i < nc; ++i) b.row_ptr[i + 1] = b.row_ptr[i] + cnt[i];
    b.col.resize(b.row_ptr[nc]);
    b.min_stencil = INT32_MAX;
    b.max_stencil = 0;
    for (int64_t i = 0; i < nc; ++i) {
        std::memcpy(&b.col[b.row_ptr[i]], &flat[i * cap], cnt[i] * sizeof(int32_t));
        b.min_stencil = std::min(b.min_stencil, cnt[i]);
        b.max_stencil = std::max(b.max_stencil, cnt[i]);
    }

    // renumbering: reverse Cuthill-McKee, then a stable partition into the
    // reconstruction kernel's stencil-size buckets
    std::vector<int32_t> rcm = rcm_order(m);
    const std::vector<int> variants = stencil_capacities(dim, prm.p);
    if (variants.empty() || (int)variants.size() > kMaxBuckets) {
        b.perm = std::move(rcm);
        b.nbuckets = 0;
        b.bucket_cell0[0] = 0;
        for (int t = 1; t <= kMaxBuckets; ++t) b.bucket_cell0[t] = nc;
    } else {
        const int nbk = (int)variants.size();
        auto bucket_of = [&](int64_t u) {
            for (int t = 0; t < nbk; ++t)
                if (variants[t] >= cnt[u]) return t;
            return nbk - 1;   // too large: reported as unsupported by the device upload
        };
        b.perm.clear();
        b.perm.reserve(nc);
        b.nbuckets = nbk;
        for (int t = 0; t < nbk; ++t) {
            b.bucket_cap[t] = variants[t];
            b.bucket_cell0[t] = (int64_t)b.perm.size();
            for (int32_t u : rcm)
                if (bucket_of(u) == t) b.perm.push_back(u);
        }
        for (int t = nbk; t <= kMaxBuckets; ++t) b.bucket_cell0[t] = nc;
    }
    b.iperm.assign(nc, 0);
    for (int64_t d = 0; d < nc; ++d) b.iperm[b.perm[d]] = (int32_t)d;

    // device-order CSR
    b.sptr.assign(nc + 1, 0);
    for (int64_t d = 0; d < nc; ++d) b.sptr[d + 1] = b.sptr[d] + cnt[b.perm[d]];
    b.scol.resize(b.sptr[nc]);
    for (int64_t d = 0; d < nc; ++d) {
        int32_t u = b.perm[d];
        for (int32_t t = 0; t < cnt[u]; ++t) b.scol[b.sptr[d] + t] = b.iperm[b.col[b.row_ptr[u] + t]];
    }
    // balanced-stencil refit: enlarged stencils (the same rule, twice the
    // sizes), device order, padded
    if (prm.balance) {
        const int cap2 = 2 * prm.n_hi;
        std::vector<int32_t> flat2(nc * cap2);
        std::vector<int32_t> cnt2(nc);
#pragma omp parallel
        {
            RingSet a(nc), bb(nc);
            std::vector<std::pair<double, int32_t>> tmp;
#pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < nc; ++i) {
                int k = 0;
                one_stencil(m, i, 2 * prm.n_lo, 2 * prm.n_hi, a, bb, tmp, &flat2[i * cap2], &k);
                cnt2[i] = k;
            }
        }
        int pc = 0;
        for (int64_t i = 0; i < nc; ++i) pc = std::max(pc, (int)cnt2[i]);
        b.pool_cap = pc;
        b.pool.assign(nc * pc, -1);
        for (int64_t d = 0; d < nc; ++d) {
            const int32_t u = b.perm[d];
            for (int32_t t = 0; t < cnt2[u]; ++t) b.pool[d * pc + t] = b.iperm[flat2[u * cap2 + t]];
        }
    }

    // h_mode 1: eps h_i^2 with h_i the mean length of cell i's edges
    if (prm.h_mode == 1) {
        b.eh2_cell.resize(nc);
        for (int64_t dd = 0; dd < nc; ++dd) {
            const int64_t u = b.perm[dd];
            double hi;
            if (dim == 1) {
                hi = m.vol[u];
            } else {
                double s = 0.0;
                int ne = 0;
                for (int v = 0; v < nvc; ++v)
                    for (int w = v + 1; w < nvc; ++w) {
                        double l2 = 0.0;
                        for (int k = 0; k < dim; ++k) {
                            const double t = m.xyz[(int64_t)m.cells[u * nvc + w] * dim + k] -
                                             m.xyz[(int64_t)m.cells[u * nvc + v] * dim + k];
                            l2 = l2 + t * t;
                        }
                        s = s + std::sqrt(l2);
                        ++ne;
                    }
                hi = s / ne;
            }
            b.eh2_cell[dd] = prm.eps * hi * hi;
        }
    }

    // padded per-bucket stencil table (no row-pointer load in the kernel)
    {
        int64_t off = 0;
        for (int t = 0; t < kMaxBuckets; ++t) {
            b.spad_off[t] = off;
            if (t < b.nbuckets) off += (b.bucket_cell0[t + 1] - b.bucket_cell0[t]) * b.bucket_cap[t];
        }
        b.spad_off[kMaxBuckets] = off;
        b.spad.assign(off, -1);
        for (int t = 0; t < b.nbuckets; ++t) {
            const int stride = b.bucket_cap[t];
            for (int64_t d = b.bucket_cell0[t]; d < b.bucket_cell0[t + 1]; ++d) {
                const int64_t base = b.spad_off[t] + (d - b.bucket_cell0[t]) * stride;
                const int32_t n = b.sptr[d + 1] - b.sptr[d];
                for (int32_t r = 0; r < n && r < stride; ++r) b.spad[base + r] = b.scol[b.sptr[d] + r];
            }
        }
    }

    // geometry records: centroid + moments nu(alpha) = mu(alpha)/alpha!, 2 <= |alpha| <= p-1
    auto ex = basis_exponents(dim, prm.p);
    const int nmom = b.m - 1 - dim;
    b.gs = dim + nmom;
    if (b.gs & 1) b.gs += 1;
    b.geo.assign(nc * b.gs, 0.0);
    b.vrel.assign(nc * nvc * dim, 0.0);
    b.rvol.resize(nc);
    const double fact[5] = {1, 1, 2, 6, 24};
    for (int64_t d = 0; d < nc; ++d) {
        int64_t u = b.perm[d];
        double e[4][3] = {{0}};
        for (int v = 0; v < nvc; ++v)
            for (int k = 0; k < dim; ++k) {
                e[v][k] = m.xyz[(int64_t)m.cells[u * nvc + v] * dim + k] - m.cent[u * dim + k];
                b.vrel[(d * nvc + v) * dim + k] = e[v][k];
            }
        for (int k = 0; k < dim; ++k) b.geo[d * b.gs + k] = m.cent[u * dim + k];
        // S(idx) = sum_v prod_t e[v][idx_t]
        auto S = [&](const int *idx, int q) {
            double s = 0.0;
            for (int v = 0; v < nvc; ++v) {
                double pr = 1.0;
                for (int t = 0; t < q; ++t) pr *= e[v][idx[t]];
                s += pr;
            }
            return s;
        };
        for (int t = 0; t < nmom; ++t) {
            const auto &a = ex[1 + dim + t];
            int idx[4], q = 0;
            for (int k = 0; k < 3; ++k)
                for (int r = 0; r < a[k]; ++r) idx[q++] = k;
            // central moments of the uniform density on a simplex, from the
            // Dirichlet(1,..,1) moments of the barycentric coordinates:
            //   |a|=2: S/((d+1)(d+2)),  |a|=3: 2 S/((d+1)(d+2)(d+3)),
            //   |a|=4: d!/(d+4)! (6 S + sum over the 3 pairings of S2 S2)
            double mu;
            if (q == 2) {
                mu = S(idx, 2) / ((dim + 1.0) * (dim + 2.0));
            } else if (q == 3) {
                mu = 2.0 * S(idx, 3) / ((dim + 1.0) * (dim + 2.0) * (dim + 3.0));
            } else {
                int p01[2] = {idx[0], idx[1]}, p23[2] = {idx[2], idx[3]};
                int p02[2] = {idx[0], idx[2]}, p13[2] = {idx[1], idx[3]};
                int p03[2] = {idx[0], idx[3]}, p12[2] = {idx[1], idx[2]};
                double pairs = S(p01, 2) * S(p23, 2) + S(p02, 2) * S(p13, 2) + S(p03, 2) * S(p12, 2);
                double df4 = 1.0;
                for (int k = dim + 1; k <= dim + 4; ++k) df4 /= k;   // d!/(d+4)!
                mu = (6.0 * S(idx, 4) + pairs) * df4;
            }
            double af = fact[a[0]] * fact[a[1]] * fact[a[2]];
            b.geo[d * b.gs + dim + t] = mu / af;
        }
        b.rvol[d] = 1.0 / m.vol[u];
    }
    if (!m.mesh_of.empty()) {
        b.mid.resize(nc);
        for (int64_t d = 0; d < nc; ++d) b.mid[d] = m.mesh_of[b.perm[d]];
    }

    // facets: normals, areas, sibling map, point correspondence
    const int F = nvc, Q = b.nq;
    b.dsib.assign(nc * F, -1);
    b.qperm.assign(nc * F, 0);
    b.normal.assign(nc * F * dim, 0.0);
    b.nsum.assign(nc * F, 0.0);
    b.area.assign(nc * F, 0.0);
    double min_ins = INFINITY;
    auto own_normal = [&](int64_t u, int lf, double *n, double *ar) {
        const int32_t *cv = &m.cells[u * nvc];
        if (dim == 1) {
            n[0] = lf == 0 ? 1.0 : -1.0;
            *ar = 1.0;
        } else if (dim == 2) {
            const double *a = &m.xyz[(int64_t)cv[(lf + 1) % 3] * 2];
            const double *bb = &m.xyz[(int64_t)cv[(lf + 2) % 3] * 2];
            double tx = bb[0] - a[0], ty = bb[1] - a[1];
            double len = std::sqrt(tx * tx + ty * ty);
            n[0] = ty / len;
            n[1] = -tx / len;
            *ar = len;
        } else {
            const double *a = &m.xyz[(int64_t)cv[(lf + 1) % 4] * 3];
            const double *bb = &m.xyz[(int64_t)cv[(lf + 2) % 4] * 3];
            const double *cc = &m.xyz[(int64_t)cv[(lf + 3) % 4] * 3];
            const double *op = &m.xyz[(int64_t)cv[lf] * 3];
            double u1[3], u2[3], w[3];
            for (int k = 0; k < 3; ++k) {
                u1[k] = bb[k] - a[k];
                u2[k] = cc[k] - a[k];
                w[k] = op[k] - a[k];
            }
            double cr[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                            u1[0] * u2[1] - u1[1] * u2[0]};
            double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            double sgn = (cr[0] * w[0] + cr[1] * w[1] + cr[2] * w[2]) > 0.0 ? -1.0 : 1.0;
            for (int k = 0; k < 3; ++k) n[k] = sgn * cr[k] / len;
            *ar = 0.5 * len;
        }
    };
    for (int64_t d = 0; d < nc; ++d) {
        int64_t u = b.perm[d];
        double perim = 0.0;
        for (int lf = 0; lf < F; ++lf) {
            int32_t s = m.sib[u * F + lf];
            double n[3] = {0, 0, 0}, ar = 0.0;
            if (s < 0) {
                own_normal(u, lf, n, &ar);
                for (int k = 0; k < dim; ++k) b.normal[(lf * nc + d) * dim + k] = ar * n[k];
                for (int k = 0; k < dim; ++k) b.nsum[lf * nc + d] += n[k];
                b.area[lf * nc + d] = ar;
            } else {
                int64_t u2 = s >> 2;
                int lf2 = s & 3;
                int64_t d2 = b.iperm[u2];
                // the half-facet of the lower device id defines normal and area
                bool owner = d < d2;
                if (owner) {
                    own_normal(u, lf, n, &ar);
                } else {
                    own_normal(u2, lf2, n, &ar);
                    for (int k = 0; k < dim; ++k) n[k] = -n[k];
                }
                // scaled by the facet measure; the sibling's is the exact negation
                for (int k = 0; k < dim; ++k) b.normal[(lf * nc + d) * dim + k] = ar * n[k];
                for (int k = 0; k < dim; ++k) b.nsum[lf * nc + d] += n[k];
                b.area[lf * nc + d] = ar;
                b.dsib[lf * nc + d] = (int32_t)((d2 << 2) | lf2);
                // sibling point index of each own point
                int32_t code = 0;
                for (int q = 0; q < Q; ++q) {
                    int q2 = 0;
                    if (dim == 2) {
                        q2 = Q - 1 - q;
                    } else if (dim == 3) {
                        int32_t gv = m.vid[u * nvc + (lf + 1 + q) % 4];
                        for (int t = 0; t < 3; ++t)
                            if (m.vid[u2 * nvc + (lf2 + 1 + t) % 4] == gv) q2 = t;
                    }
                    code |= q2 << (2 * q);
                }
                b.qperm[lf * nc + d] = code;
            }
            perim += b.area[lf * nc + d];
        }
        double ins = dim == 1 ? m.vol[u] : 2.0 * dim * m.vol[u] / perim;
        min_ins = std::min(min_ins, ins);
    }
    b.min_insphere = min_ins;
    out = std::move(b);
}

void transpose_tables(const Build &b, int64_t nc, int nf, std::vector<int64_t> &tptr, std::vector<int32_t> &tpos)
{
    const int64_t npad = b.spad_off[kMaxBuckets];
    const int64_t nslot = npad + (int64_t)nf * nc;
    if (nslot > (int64_t)INT32_MAX) throw inval("mesh too large for the adjoint tables");
    tptr.assign(nc + 1, 0);
    for (int64_t t = 0; t < npad; ++t)
        if (b.spad[t] >= 0) ++tptr[b.spad[t] + 1];
    for (int64_t t = 0; t < (int64_t)nf * nc; ++t)
        if (b.dsib[t] >= 0) ++tptr[(b.dsib[t] >> 2) + 1];
    for (int64_t j = 0; j < nc; ++j) tptr[j + 1] += tptr[j];
    tpos.assign(nslot, -1);
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t t = 0; t < npad; ++t)
        if (b.spad[t] >= 0) tpos[t] = (int32_t)fill[b.spad[t]]++;
    for (int64_t t = 0; t < (int64_t)nf * nc; ++t)
        if (b.dsib[t] >= 0) tpos[npad + t] = (int32_t)fill[b.dsib[t] >> 2]++;
}

}  // namespace wlseno

// Host partitioner: overlapping subdomains and their index sets.
//
//   Def. 2.8   extension of a subdomain by one layer of elements: every element in the support of a
//              basis function whose support meets the subdomain.  Basis functions belong to interior
//              vertices (V^h is inside H^1_0), and supp(phi_l) meets the open subdomain exactly when
//              l is a vertex of one of its elements; the subdomain's own elements are kept.
//   Def. 2.12  ovdof(D): dofs whose support meets D (interior vertices of elements of D);
//              dof(D): dofs whose support lies in closure(D) (every element around the vertex in D).
//   Def. 2.13  mu_l = number of subdomains with l in dof(D).
//   Sec. 2.4   Lambda = max over elements of the number of subdomains containing it.
//
// Local orderings are ascending global dof ids, dof(D) first and Gamma = ovdof \ dof after it.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace hkg {

int32_t build_partition(const hkgeneo_problem *p, Partition *out, int *bad_sub,
                        const std::vector<std::vector<int32_t>> *sets) {
    const int ne = p->n_elem, nv = p->n_vert, nd = p->n_dof, ns = sets ? (int)sets->size() : p->n_sub;
    const int npe = (p->dim == 2) ? (p->elem_type == HKG_P1 ? 3 : 4) : (p->elem_type == HKG_P1 ? 4 : 8);
    Partition &P = *out;
    P = Partition();
    P.n_sub = ns;
    P.n_dof = nd;
    P.npe = npe;
    *bad_sub = -1;

    // vertex -> element adjacency (CSR)
    std::vector<int32_t> v_ptr(nv + 1, 0), v_el((size_t)ne * npe);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < npe; ++a) {
            int v = p->elem_vert[(size_t)e * npe + a];
            if (v < 0 || v >= nv) return HKG_EINVAL;
            v_ptr[v + 1]++;
        }
    for (int v = 0; v < nv; ++v) v_ptr[v + 1] += v_ptr[v];
    {
        std::vector<int32_t> fill(v_ptr.begin(), v_ptr.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int a = 0; a < npe; ++a) v_el[fill[p->elem_vert[(size_t)e * npe + a]]++] = e;
    }
    for (int v = 0; v < nv; ++v)
        if (p->vert_dof[v] < -1 || p->vert_dof[v] >= nd) return HKG_EINVAL;

    // elements of each block of the non-overlapping partition (or the given element sets, which are
    // taken as they are: no layers added)
    std::vector<std::vector<int32_t>> block(ns);
    if (sets) {
        block = *sets;
        for (auto &b : block)
            for (int e : b)
                if (e < 0 || e >= ne) return HKG_EINVAL;
    } else {
        for (int e = 0; e < ne; ++e) {
            int s = p->elem_part[e];
            if (s < 0 || s >= ns) return HKG_EINVAL;
            block[s].push_back(e);
        }
    }
    P.el_ptr.assign(ns + 1, 0);

    std::vector<uint8_t> inD(ne, 0);
    std::vector<int32_t> vmark(nv, -1);         // stamp per vertex
    std::vector<int32_t> gloc(nd, -1);          // Gamma-local index of a dof, during one subdomain
    std::vector<int32_t> elem_count(ne, 0);     // subdomains containing each element (for Lambda)
    P.nI.resize(ns);
    P.nG.resize(ns);
    P.offI.assign(ns + 1, 0);
    P.offG.assign(ns + 1, 0);
    P.band_ptr.assign(ns + 1, 0);
    P.mu.assign(nd, 0);
    int stamp = 0;

    for (int s = 0; s < ns; ++s) {
        const int layers = sets ? 0 : p->overlap[s];
        if (layers < 0) return HKG_EINVAL;
        std::vector<int32_t> elems = block[s];
        for (int e : elems) inD[e] = 1;
        for (int layer = 0; layer < layers; ++layer) {
            // interior vertices of the current elements: their basis functions meet D'
            ++stamp;
            std::vector<int32_t> verts;
            for (int e : elems)
                for (int a = 0; a < npe; ++a) {
                    int v = p->elem_vert[(size_t)e * npe + a];
                    if (p->vert_dof[v] >= 0 && vmark[v] != stamp) {
                        vmark[v] = stamp;
                        verts.push_back(v);
                    }
                }
            // union of their supports
            for (int v : verts)
                for (int t = v_ptr[v]; t < v_ptr[v + 1]; ++t) {
                    int e = v_el[t];
                    if (!inD[e]) {
                        inD[e] = 1;
                        elems.push_back(e);
                    }
                }
        }
        // ovdof and dof
        ++stamp;
        std::vector<int32_t> ovv;
        for (int e : elems) {
            elem_count[e]++;
            for (int a = 0; a < npe; ++a) {
                int v = p->elem_vert[(size_t)e * npe + a];
                if (p->vert_dof[v] >= 0 && vmark[v] != stamp) {
                    vmark[v] = stamp;
                    ovv.push_back(v);
                }
            }
        }
        std::vector<int32_t> dofs, gam;
        for (int v : ovv) {
            bool inside = true;
            for (int t = v_ptr[v]; t < v_ptr[v + 1]; ++t)
                if (!inD[v_el[t]]) { inside = false; break; }
            if (inside) dofs.push_back(p->vert_dof[v]);
            else gam.push_back(p->vert_dof[v]);
        }
        std::sort(dofs.begin(), dofs.end());
        std::sort(gam.begin(), gam.end());
        if (dofs.empty()) { *bad_sub = s; return HKG_EINVAL; }
        {
            std::vector<int32_t> sorted(elems);
            std::sort(sorted.begin(), sorted.end());
            P.el_list.insert(P.el_list.end(), sorted.begin(), sorted.end());
            P.el_ptr[s + 1] = (int32_t)P.el_list.size();
        }
        P.nI[s] = (int32_t)dofs.size();
        P.nG[s] = (int32_t)gam.size();
        P.offI[s + 1] = P.offI[s] + P.nI[s];
        P.offG[s + 1] = P.offG[s] + P.nG[s];
        P.I_idx.insert(P.I_idx.end(), dofs.begin(), dofs.end());
        P.G_idx.insert(P.G_idx.end(), gam.begin(), gam.end());
        for (int d : dofs) P.mu[d]++;

        // band elements: elements of D with a Gamma vertex, and the Gamma-local index per vertex
        for (int g = 0; g < (int)gam.size(); ++g) gloc[gam[g]] = g;
        auto vloc = [&](int v) { return p->vert_dof[v] >= 0 ? gloc[p->vert_dof[v]] : -1; };
        std::sort(elems.begin(), elems.end());
        for (int e : elems) {
            bool touches = false;
            for (int a = 0; a < npe; ++a)
                if (vloc(p->elem_vert[(size_t)e * npe + a]) >= 0) touches = true;
            if (!touches) continue;
            P.band_elem.push_back(e);
            for (int a = 0; a < npe; ++a) P.band_loc.push_back(vloc(p->elem_vert[(size_t)e * npe + a]));
        }
        P.band_ptr[s + 1] = (int32_t)P.band_elem.size();
        for (int g : gam) gloc[g] = -1;
        for (int e : elems) inD[e] = 0;
    }
    for (int d = 0; d < nd; ++d)
        if (P.mu[d] == 0) return HKG_EINVAL;       // a dof internal to no subdomain: no partition of unity
    P.lambda_overlap = 0;
    for (int e = 0; e < ne; ++e) P.lambda_overlap = std::max(P.lambda_overlap, elem_count[e]);

    // transpose map, ordered by subdomain
    P.tp_ptr.assign(nd + 1, 0);
    for (int32_t d : P.I_idx) P.tp_ptr[d + 1]++;
    for (int d = 0; d < nd; ++d) P.tp_ptr[d + 1] += P.tp_ptr[d];
    P.tp_pos.resize(P.I_idx.size());
    {
        std::vector<int32_t> fill(P.tp_ptr.begin(), P.tp_ptr.end() - 1);
        for (int s = 0; s < ns; ++s)
            for (int a = 0; a < P.nI[s]; ++a) {
                int d = P.I_idx[P.offI[s] + a];
                P.tp_pos[fill[d]++] = (int32_t)(P.offI[s] + a);
            }
    }
    return HKG_OK;
}

// First-level subdomains of the nested decomposition (Sec. 2.3): the elements of each overlapping
// coarse subdomain are split by the fine element partition into pieces, ordered by fine block id,
// and each piece is expanded by `layers` layers of Def. 2.8 restricted to the coarse subdomain, so
// that the pieces of a coarse subdomain cover it.  Pieces without an interior dof are dropped.
int32_t build_nested_sets(const hkgeneo_problem *p, const Partition &Pc, int layers,
                          std::vector<std::vector<int32_t>> *sets, std::vector<int32_t> *owner) {
    const int ne = p->n_elem, nv = p->n_vert;
    const int npe = Pc.npe;
    std::vector<int32_t> v_ptr(nv + 1, 0), v_el((size_t)ne * npe);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < npe; ++a) v_ptr[p->elem_vert[(size_t)e * npe + a] + 1]++;
    for (int v = 0; v < nv; ++v) v_ptr[v + 1] += v_ptr[v];
    {
        std::vector<int32_t> fill(v_ptr.begin(), v_ptr.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int a = 0; a < npe; ++a) v_el[fill[p->elem_vert[(size_t)e * npe + a]]++] = e;
    }
    sets->clear();
    owner->clear();
    std::vector<uint8_t> inC(ne, 0), inF(ne, 0);
    std::vector<int32_t> vmark(nv, -1);
    int stamp = 0;
    for (int i = 0; i < Pc.n_sub; ++i) {
        const int32_t *ce = Pc.el_list.data() + Pc.el_ptr[i];
        const int nce = Pc.el_ptr[i + 1] - Pc.el_ptr[i];
        for (int q = 0; q < nce; ++q) inC[ce[q]] = 1;
        std::vector<int32_t> ids;
        for (int q = 0; q < nce; ++q) {
            const int f = p->fine_part[ce[q]];
            if (f < 0) return HKG_EINVAL;
            ids.push_back(f);
        }
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        for (int fid : ids) {
            std::vector<int32_t> elems;
            for (int q = 0; q < nce; ++q)
                if (p->fine_part[ce[q]] == fid) elems.push_back(ce[q]);
            for (int e : elems) inF[e] = 1;
            for (int layer = 0; layer < layers; ++layer) {
                ++stamp;
                std::vector<int32_t> verts;
                for (int e : elems)
                    for (int a = 0; a < npe; ++a) {
                        const int v = p->elem_vert[(size_t)e * npe + a];
                        if (p->vert_dof[v] >= 0 && vmark[v] != stamp) {
                            vmark[v] = stamp;
                            verts.push_back(v);
                        }
                    }
                for (int v : verts)
                    for (int t = v_ptr[v]; t < v_ptr[v + 1]; ++t) {
                        const int e = v_el[t];
                        if (inC[e] && !inF[e]) {
                            inF[e] = 1;
                            elems.push_back(e);
                        }
                    }
            }
            // keep the piece if some interior vertex has all its elements in it
            bool has_dof = false;
            for (int e : elems) {
                for (int a = 0; a < npe && !has_dof; ++a) {
                    const int v = p->elem_vert[(size_t)e * npe + a];
                    if (p->vert_dof[v] < 0) continue;
                    bool inside = true;
                    for (int t = v_ptr[v]; t < v_ptr[v + 1]; ++t)
                        if (!inF[v_el[t]]) { inside = false; break; }
                    has_dof = inside;
                }
                if (has_dof) break;
            }
            for (int e : elems) inF[e] = 0;
            if (!has_dof) continue;
            std::sort(elems.begin(), elems.end());
            sets->push_back(std::move(elems));
            owner->push_back(i);
        }
        for (int q = 0; q < nce; ++q) inC[ce[q]] = 0;
    }
    return sets->empty() ? HKG_EINVAL : HKG_OK;
}

void build_coarse_pairs(const Partition &P, CoarsePairs *out) {
    // owner subdomain of each concatenated internal position
    std::vector<int32_t> pos_sub(P.I_idx.size());
    for (int s = 0; s < P.n_sub; ++s)
        for (int64_t t = P.offI[s]; t < P.offI[s + 1]; ++t) pos_sub[t] = s;
    CoarsePairs &C = *out;
    C = CoarsePairs();
    C.ptr.push_back(0);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per_j(P.n_sub);
    for (int i = 0; i < P.n_sub; ++i) {
        std::vector<int32_t> touched;
        const int nI = P.nI[i], nG = P.nG[i];
        for (int q = 0; q < nI + nG; ++q) {
            int d = q < nI ? P.I_idx[P.offI[i] + q] : P.G_idx[P.offG[i] + (q - nI)];
            for (int t = P.tp_ptr[d]; t < P.tp_ptr[d + 1]; ++t) {
                int pos = P.tp_pos[t];
                int j = pos_sub[pos];
                if (per_j[j].empty()) touched.push_back(j);
                per_j[j].push_back({q, (int32_t)(pos - P.offI[j])});
            }
        }
        std::sort(touched.begin(), touched.end());
        for (int j : touched) {
            C.pi.push_back(i);
            C.pj.push_back(j);
            for (auto &x : per_j[j]) {
                C.qi.push_back(x.first);
                C.qj.push_back(x.second);
            }
            C.ptr.push_back((int32_t)C.qi.size());
            per_j[j].clear();
        }
    }
}

}  // namespace hkg

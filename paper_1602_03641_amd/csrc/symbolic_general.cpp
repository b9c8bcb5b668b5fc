// Symbolic phase of a general mesh: cells given by their faces, faces by their
// nodes in cyclic order (§3.1 states the scheme for such cells; §5.4 and §5.5
// run it on tetrahedra and prisms).  Runs once per mesh on the host:
//
//  - each cell's nodes (the union of its faces' nodes, in order of first
//    appearance) and, per local face, the local indices of its nodes,
//  - fracture faces (given as face indices) and the cells on each side,
//  - unknowns of the cell-eliminated system (eq eqschur): free nodes by node
//    index, then every fracture face (no group elimination on this path),
//  - the sparsity pattern (union over cells of the cliques of their
//    unknowns) and its renumbered sliced-ELL form (shared with hexahedra),
//  - for every stored entry of the system, the list of local-matrix entries
//    that add up to it (cell Schur blocks, fracture blocks), and for every row
//    the Dirichlet columns that go to b: the device assembles by gathering
//    these lists in a fixed order, without atomics,
//  - the fluxes as edges between control volumes (cell-node, cell-face,
//    face-node) and, per control volume, its incident edges: the CFL bound and
//    the upwind operator treat every control volume alike.
#include <algorithm>
#include <array>
#include <string>

#include "vag_internal.h"

namespace vag {

void build_symbolic_general(int64_t nn64, int64_t nc64, int64_t nface64, const int64_t *cfp, const int32_t *cf,
                            const int64_t *fnp, const int32_t *fnd, int64_t nf64, const int32_t *face_ids,
                            const uint8_t *dirichlet, Symbolic &S, GenSym &G) {
    if (nn64 <= 0 || nc64 <= 0 || nface64 <= 0 || nf64 < 0 || nn64 >= INT32_MAX || nc64 >= INT32_MAX / 8 ||
        nface64 >= INT32_MAX / 4 || nf64 > nface64)
        throw Error(VAG_ERR_ARG, "mesh sizes out of range");
    const int32_t nn = (int32_t)nn64, nc = (int32_t)nc64, nF = (int32_t)nface64, nf = (int32_t)nf64;
    S.nn = nn;
    S.nc = nc;
    S.nf = nf;

    // faces: 3 or 4 distinct nodes
    if (fnp[0] != 0) throw Error(VAG_ERR_ARG, "face_node_ptr[0] must be 0");
    for (int32_t f = 0; f < nF; ++f) {
        const int64_t k = fnp[f + 1] - fnp[f];
        if (k < 3 || k > kGenMaxFaceNodes)
            throw Error(VAG_ERR_UNSUPPORTED,
                        "face " + std::to_string(f) + " has " + std::to_string(k) + " nodes (3 or 4 supported)");
        for (int64_t i = fnp[f]; i < fnp[f + 1]; ++i) {
            if (fnd[i] < 0 || fnd[i] >= nn)
                throw Error(VAG_ERR_ARG, "face " + std::to_string(f) + ": node index out of range");
            for (int64_t j = fnp[f]; j < i; ++j)
                if (fnd[j] == fnd[i]) throw Error(VAG_ERR_ARG, "face " + std::to_string(f) + " repeats a node");
        }
    }
    // cells: 4 to 6 faces, each face in at most two cells
    if (cfp[0] != 0) throw Error(VAG_ERR_ARG, "cell_face_ptr[0] must be 0");
    std::vector<int32_t> fcell(2 * (size_t)nF, -1);
    for (int32_t K = 0; K < nc; ++K) {
        const int64_t k = cfp[K + 1] - cfp[K];
        if (k < 4 || k > kGenMaxFaces)
            throw Error(VAG_ERR_UNSUPPORTED,
                        "cell " + std::to_string(K) + " has " + std::to_string(k) + " faces (4 to 6 supported)");
        for (int64_t q = cfp[K]; q < cfp[K + 1]; ++q) {
            const int32_t f = cf[q];
            if (f < 0 || f >= nF) throw Error(VAG_ERR_ARG, "cell " + std::to_string(K) + ": face index out of range");
            for (int64_t p = cfp[K]; p < q; ++p)
                if (cf[p] == f) throw Error(VAG_ERR_MESH, "cell " + std::to_string(K) + " lists a face twice");
            if (fcell[2 * (size_t)f] < 0) fcell[2 * (size_t)f] = K;
            else if (fcell[2 * (size_t)f + 1] < 0) fcell[2 * (size_t)f + 1] = K;
            else throw Error(VAG_ERR_MESH, "face " + std::to_string(f) + " belongs to more than two cells");
        }
    }

    // each cell's nodes and the local indices of its faces' nodes
    G.cnode_ptr.assign((size_t)nc + 1, 0);
    G.cnode.clear();
    G.cnode.reserve(8 * (size_t)nc);
    G.cface_k.assign(kGenMaxFaces * (size_t)nc, 0);
    G.cface_loc.assign(kGenMaxFaces * kGenMaxFaceNodes * (size_t)nc, 0xff);
    for (int32_t K = 0; K < nc; ++K) {
        const size_t base = G.cnode.size();
        int lf = 0;
        for (int64_t q = cfp[K]; q < cfp[K + 1]; ++q, ++lf) {
            const int32_t f = cf[q];
            const int k = (int)(fnp[f + 1] - fnp[f]);
            G.cface_k[kGenMaxFaces * (size_t)K + lf] = (uint8_t)k;
            for (int i = 0; i < k; ++i) {
                const int32_t s = fnd[fnp[f] + i];
                size_t l = base;
                while (l < G.cnode.size() && G.cnode[l] != s) ++l;
                if (l == G.cnode.size()) {
                    if (l - base >= (size_t)kGenMaxNodes)
                        throw Error(VAG_ERR_UNSUPPORTED, "cell " + std::to_string(K) + " has more than 8 nodes");
                    G.cnode.push_back(s);
                }
                G.cface_loc[(kGenMaxFaces * (size_t)K + lf) * kGenMaxFaceNodes + i] = (uint8_t)(l - base);
            }
        }
        if (G.cnode.size() - base < 4) throw Error(VAG_ERR_MESH, "cell " + std::to_string(K) + " has fewer than 4 nodes");
        G.cnode_ptr[K + 1] = (int32_t)G.cnode.size();
        G.max_nv = std::max(G.max_nv, (int)(G.cnode.size() - base));
        G.max_nf = std::max(G.max_nf, lf);
        for (int f = 0; f < lf; ++f) G.max_fk = std::max(G.max_fk, (int)G.cface_k[kGenMaxFaces * (size_t)K + f]);
    }
    G.ncn = (int64_t)G.cnode.size();

    // fracture faces
    std::vector<int32_t> frac_of(nF, -1);
    for (int32_t g = 0; g < nf; ++g) {
        const int32_t f = face_ids[g];
        if (f < 0 || f >= nF) throw Error(VAG_ERR_ARG, "fracture face " + std::to_string(g) + ": face index out of range");
        if (frac_of[f] >= 0) throw Error(VAG_ERR_ARG, "fracture face " + std::to_string(g) + " is listed twice");
        if (fcell[2 * (size_t)f] < 0)
            throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(g) + " is not a face of any cell");
        frac_of[f] = g;
    }
    S.frac_cell.assign(2 * (size_t)nf, -1);
    S.cell_frac.assign(kGenMaxFaces * (size_t)nc, -1);
    S.fmask.assign(nc, 0);
    for (int32_t g = 0; g < nf; ++g) {
        const int32_t f = face_ids[g];
        const int32_t a = fcell[2 * (size_t)f], b = fcell[2 * (size_t)f + 1];
        S.frac_cell[2 * (size_t)g] = (b >= 0 && b < a) ? b : a;  // ascending cell index
        S.frac_cell[2 * (size_t)g + 1] = (b >= 0 && b < a) ? a : b;
    }
    for (int32_t K = 0; K < nc; ++K) {
        int lf = 0;
        for (int64_t q = cfp[K]; q < cfp[K + 1]; ++q, ++lf)
            if (frac_of[cf[q]] >= 0) {
                S.cell_frac[kGenMaxFaces * (size_t)K + lf] = frac_of[cf[q]];
                S.fmask[K] |= (uint8_t)(1u << lf);
            }
    }
    G.fnode_ptr.assign((size_t)nf + 1, 0);
    G.fnode.clear();
    S.frac_node.assign(nn, 0);
    for (int32_t g = 0; g < nf; ++g) {
        const int32_t f = face_ids[g];
        for (int64_t i = fnp[f]; i < fnp[f + 1]; ++i) {
            G.fnode.push_back(fnd[i]);
            S.frac_node[fnd[i]] = 1;
        }
        G.fnode_ptr[g + 1] = (int32_t)G.fnode.size();
    }
    G.nfn = (int64_t)G.fnode.size();

    // unknowns: free nodes, then every fracture face
    S.node_unk.assign(nn, -1);
    int32_t nfree = 0;
    for (int32_t s = 0; s < nn; ++s)
        if (!dirichlet[s]) S.node_unk[s] = nfree++;
    if (nfree == nn) throw Error(VAG_ERR_ARG, "no Dirichlet node: the Darcy problem is singular");
    S.nfree = nfree;
    S.frac_unk.resize(nf);
    for (int32_t g = 0; g < nf; ++g) S.frac_unk[g] = nfree + g;
    S.nunk = S.nx = nfree + nf;
    S.ngroup = S.ngcolor = 0;
    S.grp_ptr.assign(1, 0);
    S.grp_nptr.assign(1, 0);
    S.grp_off.assign(1, 0);
    S.grp_poff.assign(1, 0);
    S.gcolor_ptr.assign(1, 0);
    S.grp_face.clear();
    S.grp_node.clear();
    S.grp_pos.clear();
    S.face_grp.assign(nf, -1);
    S.face_loc.assign(nf, -1);

    // the unknowns of each cell: its nodes (local order), then its fracture
    // faces (local face order); -1 for a Dirichlet node
    auto cell_unknowns = [&](int32_t K, int32_t *u, int32_t *node) {
        int m = 0;
        for (int32_t q = G.cnode_ptr[K]; q < G.cnode_ptr[K + 1]; ++q) {
            node[m] = G.cnode[q];
            u[m++] = S.node_unk[G.cnode[q]];
        }
        for (int lf = 0; lf < kGenMaxFaces; ++lf) {
            const int32_t g = S.cell_frac[kGenMaxFaces * (size_t)K + lf];
            if (g >= 0) {
                node[m] = -1;
                u[m++] = S.frac_unk[g];
            }
        }
        return m;
    };
    G.unk_off.assign((size_t)nc + 1, 0);
    {
        int32_t u[kGenMaxNodes + kGenMaxFaces], node[kGenMaxNodes + kGenMaxFaces];
        for (int32_t K = 0; K < nc; ++K) G.unk_off[K + 1] = G.unk_off[K] + cell_unknowns(K, u, node);
    }

    // node -> cells
    std::vector<int32_t> ncp(nn + 1, 0), ncl;
    for (int64_t q = 0; q < G.ncn; ++q) ncp[G.cnode[q] + 1]++;
    for (int32_t s = 0; s < nn; ++s) ncp[s + 1] += ncp[s];
    ncl.resize(ncp[nn]);
    {
        std::vector<int32_t> fill(ncp.begin(), ncp.end() - 1);
        for (int32_t K = 0; K < nc; ++K)
            for (int32_t q = G.cnode_ptr[K]; q < G.cnode_ptr[K + 1]; ++q) ncl[fill[G.cnode[q]]++] = K;
    }

    // CSR pattern in unknown order: a row couples to every unknown of every
    // cell that holds its node or face
    S.row_ptr.assign((size_t)S.nunk + 1, 0);
    S.col.clear();
    {
        std::vector<int32_t> marker((size_t)S.nunk, -1), cols;
        int32_t u[kGenMaxNodes + kGenMaxFaces], node[kGenMaxNodes + kGenMaxFaces];
        auto add_cell = [&](int32_t row, int32_t K) {
            const int m = cell_unknowns(K, u, node);
            for (int i = 0; i < m; ++i)
                if (u[i] >= 0 && marker[u[i]] != row) {
                    marker[u[i]] = row;
                    cols.push_back(u[i]);
                }
        };
        std::vector<std::vector<int32_t>> rows((size_t)S.nunk);
        for (int32_t s = 0; s < nn; ++s) {
            const int32_t row = S.node_unk[s];
            if (row < 0) continue;
            cols.clear();
            for (int32_t q = ncp[s]; q < ncp[s + 1]; ++q) add_cell(row, ncl[q]);
            rows[row] = cols;
        }
        for (int32_t g = 0; g < nf; ++g) {
            const int32_t row = S.frac_unk[g];
            cols.clear();
            for (int side = 0; side < 2; ++side)
                if (S.frac_cell[2 * (size_t)g + side] >= 0) add_cell(row, S.frac_cell[2 * (size_t)g + side]);
            rows[row] = cols;
        }
        int64_t total = 0;
        for (int32_t r = 0; r < S.nunk; ++r) {
            total += (int64_t)rows[r].size();
            S.row_ptr[r + 1] = (int32_t)total;
        }
        if (total >= INT32_MAX) throw Error(VAG_ERR_UNSUPPORTED, "system has more than 2^31 nonzeros");
        S.col.reserve(total);
        for (auto &v : rows) S.col.insert(S.col.end(), v.begin(), v.end());
    }
    S.nnz = S.row_ptr[S.nunk];
    finish_symbolic_pattern(S);

    // local value blocks: m x m per cell, (k + 1)^2 per fracture face
    G.loc_off.assign((size_t)nc + nf + 1, 0);
    for (int32_t K = 0; K < nc; ++K) {
        const int64_t m = G.unk_off[K + 1] - G.unk_off[K];
        G.loc_off[K + 1] = G.loc_off[K] + m * m;
    }
    for (int32_t g = 0; g < nf; ++g) {
        const int64_t k1 = G.fnode_ptr[g + 1] - G.fnode_ptr[g] + 1;
        G.loc_off[nc + g + 1] = G.loc_off[nc + g] + k1 * k1;
    }

    // contributions to the stored entries and to b, in cell then face order
    auto slot = [&](int32_t row, int32_t col) -> int64_t {
        const int32_t *b = S.col.data() + S.row_ptr[row], *e = S.col.data() + S.row_ptr[row + 1];
        const int32_t *p = std::lower_bound(b, e, col);
        if (p == e || *p != col) throw Error(VAG_ERR_ARG, "internal: a local coupling is missing from the pattern");
        return S.sell_ptr[row / kSliceRows] + (int64_t)(p - b) * kSliceRows + row % kSliceRows;
    };
    std::vector<std::pair<int64_t, int64_t>> ent;   // (slot, local value index)
    std::vector<std::array<int64_t, 3>> bent;       // (row, local value index, node)
    {
        int32_t u[kGenMaxNodes + kGenMaxFaces], node[kGenMaxNodes + kGenMaxFaces];
        for (int32_t K = 0; K < nc; ++K) {
            const int m = cell_unknowns(K, u, node);
            for (int i = 0; i < m; ++i) {
                if (u[i] < 0) continue;
                for (int j = 0; j < m; ++j) {
                    const int64_t v = G.loc_off[K] + (int64_t)i * m + j;
                    if (u[j] >= 0) ent.push_back({slot(u[i], u[j]), v});
                    else bent.push_back({u[i], v, node[j]});
                }
            }
        }
        for (int32_t g = 0; g < nf; ++g) {
            const int k = G.fnode_ptr[g + 1] - G.fnode_ptr[g];
            int32_t fu[kGenMaxFaceNodes + 1], fn[kGenMaxFaceNodes + 1];
            fu[0] = S.frac_unk[g];
            fn[0] = -1;
            for (int i = 0; i < k; ++i) {
                fn[1 + i] = G.fnode[G.fnode_ptr[g] + i];
                fu[1 + i] = S.node_unk[fn[1 + i]];
            }
            for (int i = 0; i <= k; ++i) {
                if (fu[i] < 0) continue;
                for (int j = 0; j <= k; ++j) {
                    const int64_t v = G.loc_off[nc + g] + (int64_t)i * (k + 1) + j;
                    if (fu[j] >= 0) ent.push_back({slot(fu[i], fu[j]), v});
                    else bent.push_back({fu[i], v, fn[j]});
                }
            }
        }
    }
    const int64_t stored = S.sell_ptr.back();
    G.con_ptr.assign((size_t)stored + 1, 0);
    for (auto &e : ent) G.con_ptr[e.first + 1]++;
    for (int64_t q = 0; q < stored; ++q) G.con_ptr[q + 1] += G.con_ptr[q];
    G.con.resize(ent.size());
    {
        std::vector<int64_t> fill(G.con_ptr.begin(), G.con_ptr.end() - 1);
        for (auto &e : ent) G.con[fill[e.first]++] = e.second;
    }
    G.bcon_ptr.assign((size_t)S.nunk + 1, 0);
    for (auto &e : bent) G.bcon_ptr[e[0] + 1]++;
    for (int32_t r = 0; r < S.nunk; ++r) G.bcon_ptr[r + 1] += G.bcon_ptr[r];
    G.bcon.resize(bent.size());
    G.bcon_node.resize(bent.size());
    {
        std::vector<int32_t> fill(G.bcon_ptr.begin(), G.bcon_ptr.end() - 1);
        for (auto &e : bent) {
            const int32_t q = fill[e[0]]++;
            G.bcon[q] = e[1];
            G.bcon_node[q] = (int32_t)e[2];
        }
    }

    // fluxes and control volumes: cells [0, nc), fracture faces [nc, nc + nf),
    // nodes [nc + nf, nc + nf + nn); flux array [cell-node | cell-face | face-node]
    G.nflux = G.ncn + 2 * (int64_t)nf + G.nfn;
    if (G.nflux >= INT32_MAX / 2) throw Error(VAG_ERR_UNSUPPORTED, "too many fluxes for 31-bit edge indices");
    const int64_t nrow = (int64_t)nc + nf + nn;
    std::vector<std::array<int32_t, 3>> edges;  // (cv where F > 0 leaves, cv it enters, flux index)
    edges.reserve((size_t)G.nflux);
    for (int32_t K = 0; K < nc; ++K)
        for (int32_t q = G.cnode_ptr[K]; q < G.cnode_ptr[K + 1]; ++q)
            edges.push_back({K, (int32_t)(nc + nf + G.cnode[q]), q});
    for (int32_t g = 0; g < nf; ++g)
        for (int side = 0; side < 2; ++side) {
            const int32_t K = S.frac_cell[2 * (size_t)g + side];
            if (K >= 0) edges.push_back({K, nc + g, (int32_t)(G.ncn + 2 * g + side)});
        }
    for (int32_t g = 0; g < nf; ++g)
        for (int32_t q = G.fnode_ptr[g]; q < G.fnode_ptr[g + 1]; ++q)
            edges.push_back({nc + g, (int32_t)(nc + nf + G.fnode[q]), (int32_t)(G.ncn + 2 * nf + q)});
    G.inc_ptr.assign((size_t)nrow + 1, 0);
    for (auto &e : edges) {
        G.inc_ptr[e[0] + 1]++;
        G.inc_ptr[e[1] + 1]++;
    }
    for (int64_t i = 0; i < nrow; ++i) {
        // the upwind operator stores a row's entry count in 8 bits
        if (G.inc_ptr[i + 1] > 255)
            throw Error(VAG_ERR_UNSUPPORTED, "a control volume has more than 255 fluxes (node " +
                                                 std::to_string(i - nc - nf) + ")");
        G.inc_ptr[i + 1] += G.inc_ptr[i];
    }
    G.inc_edge.resize(G.inc_ptr[nrow]);
    G.inc_other.resize(G.inc_ptr[nrow]);
    {
        std::vector<int64_t> fill(G.inc_ptr.begin(), G.inc_ptr.end() - 1);
        for (auto &e : edges) {
            int64_t q = fill[e[0]]++;
            G.inc_edge[q] = e[2] << 1;
            G.inc_other[q] = e[1];
            q = fill[e[1]]++;
            G.inc_edge[q] = (e[2] << 1) | 1;
            G.inc_other[q] = e[0];
        }
    }
}

}  // namespace vag

// Symbolic phase: everything that depends only on the mesh topology, the
// fracture face list and the Dirichlet flags.  Runs once per mesh on the host.
//
//  - match fracture faces to cell faces (the conforming assumption of §3.1),
//  - number the unknowns of the cell-eliminated system (eq eqschur): free
//    nodes by node index, then fracture faces,
//  - group the fracture faces that share a cell: after the cell elimination
//    the face-face block is block diagonal over these groups, so a group can
//    be eliminated exactly onto the free nodes of its cells (dense Schur
//    complement per group); eliminated faces are numbered after the system,
//  - sparsity pattern: the unknowns of a cell (its free nodes and fracture
//    faces) are pairwise coupled after eliminating u_K, so the pattern is the
//    union over cells of these cliques, plus the node cliques of the
//    eliminated groups,
//  - greedy cell colouring such that cells of one colour share no node: the
//    assembly scatters one colour at a time without atomics (deterministic),
//  - per-cell slot maps: position in the CSR values of each local pair,
//  - node -> (cell, slot) and node -> (fracture, vertex) adjacency.
#include <algorithm>
#include <array>
#include <unordered_map>

#include "vag_internal.h"

namespace vag {

namespace {

struct Key4 {
    std::array<int32_t, 4> v;
    bool operator==(const Key4 &o) const { return v == o.v; }
};
struct Key4Hash {
    size_t operator()(const Key4 &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int32_t x : k.v) {
            h ^= static_cast<uint32_t>(x);
            h *= 1099511628211ull;
        }
        return static_cast<size_t>(h);
    }
};

Key4 sorted_key(const int32_t *n) {
    Key4 k{{n[0], n[1], n[2], n[3]}};
    std::sort(k.v.begin(), k.v.end());
    return k;
}

// true if b lists the same 4-cycle as a (any rotation, either direction)
bool same_cycle(const int32_t *a, const int32_t *b) {
    int p = -1;
    for (int i = 0; i < 4; ++i)
        if (a[i] == b[0]) p = i;
    if (p < 0) return false;
    bool fwd = true, bwd = true;
    for (int i = 0; i < 4; ++i) {
        fwd &= (a[(p + i) & 3] == b[i]);
        bwd &= (a[(p - i + 4) & 3] == b[i]);
    }
    return fwd || bwd;
}

}  // namespace

void build_symbolic(int64_t nn64, int64_t nc64, int64_t nf64, const int32_t *hex8,
                    const int32_t *frac_nodes, const uint8_t *dirichlet, bool eliminate, Symbolic &S) {
    if (nn64 <= 0 || nc64 <= 0 || nf64 < 0 || nn64 >= INT32_MAX || nc64 >= INT32_MAX / 8 ||
        nf64 >= INT32_MAX / 4)
        throw Error(VAG_ERR_ARG, "mesh sizes out of range");
    const int32_t nn = (int32_t)nn64, nc = (int32_t)nc64, nf = (int32_t)nf64;
    S.nn = nn;
    S.nc = nc;
    S.nf = nf;

    for (int64_t i = 0; i < 8 * (int64_t)nc; ++i)
        if (hex8[i] < 0 || hex8[i] >= nn)
            throw Error(VAG_ERR_ARG, "hex8 node index out of range at cell " + std::to_string(i / 8));
    for (int64_t i = 0; i < 4 * (int64_t)nf; ++i)
        if (frac_nodes[i] < 0 || frac_nodes[i] >= nn)
            throw Error(VAG_ERR_ARG, "fracture face node index out of range at face " + std::to_string(i / 4));

    // node -> (cell, slot)
    S.node_cell_ptr.assign(nn + 1, 0);
    for (int64_t i = 0; i < 8 * (int64_t)nc; ++i) S.node_cell_ptr[hex8[i] + 1]++;
    for (int32_t s = 0; s < nn; ++s) S.node_cell_ptr[s + 1] += S.node_cell_ptr[s];
    S.node_cell.resize(S.node_cell_ptr[nn]);
    {
        std::vector<int32_t> fill(S.node_cell_ptr.begin(), S.node_cell_ptr.end() - 1);
        for (int32_t K = 0; K < nc; ++K)
            for (int a = 0; a < 8; ++a) S.node_cell[fill[hex8[8 * (int64_t)K + a]]++] = K * 8 + a;
    }

    // fracture faces: match against cell faces
    S.frac_node.assign(nn, 0);
    for (int64_t i = 0; i < 4 * (int64_t)nf; ++i) S.frac_node[frac_nodes[i]] = 1;
    std::unordered_map<Key4, int32_t, Key4Hash> fmap;
    fmap.reserve((size_t)nf * 2 + 1);
    for (int32_t f = 0; f < nf; ++f) {
        const int32_t *fn = frac_nodes + 4 * (int64_t)f;
        Key4 k = sorted_key(fn);
        if (k.v[0] == k.v[1] || k.v[1] == k.v[2] || k.v[2] == k.v[3])
            throw Error(VAG_ERR_ARG, "fracture face " + std::to_string(f) + " repeats a node");
        if (!fmap.emplace(k, f).second)
            throw Error(VAG_ERR_ARG, "fracture face " + std::to_string(f) + " is listed twice");
    }
    S.fmask.assign(nc, 0);
    S.cell_frac.assign(6 * (size_t)nc, -1);
    S.frac_cell.assign(2 * (size_t)nf, -1);
    if (nf > 0) {
        for (int32_t K = 0; K < nc; ++K) {
            const int32_t *cn = hex8 + 8 * (int64_t)K;
            for (int lf = 0; lf < 6; ++lf) {
                int32_t q[4];
                bool all = true;
                for (int i = 0; i < 4; ++i) {
                    q[i] = cn[hexf(lf, i)];
                    all &= S.frac_node[q[i]] != 0;
                }
                if (!all) continue;
                auto it = fmap.find(sorted_key(q));
                if (it == fmap.end()) continue;
                int32_t f = it->second;
                if (!same_cycle(q, frac_nodes + 4 * (int64_t)f))
                    throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(f) +
                                                  " nodes are not in cyclic order");
                int side = S.frac_cell[2 * (size_t)f] < 0 ? 0 : (S.frac_cell[2 * (size_t)f + 1] < 0 ? 1 : 2);
                if (side == 2)
                    throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(f) + " has more than two cells");
                S.frac_cell[2 * (size_t)f + side] = K;  // cells visited in ascending order
                S.cell_frac[6 * (size_t)K + lf] = f;
                S.fmask[K] |= (uint8_t)(1u << lf);
            }
        }
    }
    S.frac_slot.assign(4 * (size_t)nf, -1);
    for (int32_t f = 0; f < nf; ++f) {
        int32_t K = S.frac_cell[2 * (size_t)f];
        if (K < 0) throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(f) + " is not a face of the mesh");
        for (int i = 0; i < 4; ++i)
            for (int a = 0; a < 8; ++a)
                if (hex8[8 * (int64_t)K + a] == frac_nodes[4 * (int64_t)f + i]) S.frac_slot[4 * (size_t)f + i] = a;
    }

    // node -> (fracture, vertex)
    S.node_frac_ptr.assign(nn + 1, 0);
    for (int64_t i = 0; i < 4 * (int64_t)nf; ++i) S.node_frac_ptr[frac_nodes[i] + 1]++;
    for (int32_t s = 0; s < nn; ++s) S.node_frac_ptr[s + 1] += S.node_frac_ptr[s];
    S.node_frac.resize(S.node_frac_ptr[nn]);
    {
        std::vector<int32_t> fill(S.node_frac_ptr.begin(), S.node_frac_ptr.end() - 1);
        for (int32_t f = 0; f < nf; ++f)
            for (int i = 0; i < 4; ++i) S.node_frac[fill[frac_nodes[4 * (int64_t)f + i]]++] = f * 4 + i;
    }

    // fracture-face groups: faces of one cell are coupled after the cell
    // elimination, so the face-face block is block diagonal over the
    // connected components of "shares a cell"
    std::vector<int32_t> uf(nf);
    for (int32_t f = 0; f < nf; ++f) uf[f] = f;
    auto find = [&](int32_t f) {
        while (uf[f] != f) f = uf[f] = uf[uf[f]];
        return f;
    };
    for (int32_t K = 0; K < nc; ++K) {
        int32_t first = -1;
        for (int lf = 0; lf < 6; ++lf) {
            if (!(S.fmask[K] >> lf & 1)) continue;
            const int32_t f = S.cell_frac[6 * (size_t)K + lf];
            if (first < 0) {
                first = f;
            } else {
                const int32_t a = find(first), b = find(f);
                if (a != b) uf[std::max(a, b)] = std::min(a, b);
            }
        }
    }

    // free nodes first
    S.node_unk.assign(nn, -1);
    int32_t nfree = 0;
    for (int32_t s = 0; s < nn; ++s)
        if (!dirichlet[s]) S.node_unk[s] = nfree++;
    if (nfree == nn) throw Error(VAG_ERR_ARG, "no Dirichlet node: the Darcy problem is singular");
    S.nfree = nfree;

    // candidate groups (faces ascending within a group, groups by first face)
    std::vector<int32_t> root_id(nf, -1), cand_ptr(1, 0), cand_face;
    {
        std::vector<int32_t> cnt;
        for (int32_t f = 0; f < nf; ++f) {
            const int32_t r = find(f);
            if (root_id[r] < 0) {
                root_id[r] = (int32_t)cnt.size();
                cnt.push_back(0);
            }
            cnt[root_id[r]]++;
        }
        cand_ptr.resize(cnt.size() + 1, 0);
        for (size_t g = 0; g < cnt.size(); ++g) cand_ptr[g + 1] = cand_ptr[g] + cnt[g];
        cand_face.resize(nf);
        std::vector<int32_t> fill(cand_ptr.begin(), cand_ptr.end() - 1);
        for (int32_t f = 0; f < nf; ++f) cand_face[fill[root_id[find(f)]]++] = f;
    }
    const int32_t ncand = (int32_t)cand_ptr.size() - 1;
    // free nodes (as node unknowns) of the cells of each candidate group
    std::vector<int32_t> cand_nptr(ncand + 1, 0), cand_node;
    std::vector<uint8_t> elim(ncand, 0);
    {
        std::vector<int32_t> mark(nfree, -1), cells;
        for (int32_t g = 0; g < ncand; ++g) {
            const size_t start = cand_node.size();
            for (int32_t q = cand_ptr[g]; q < cand_ptr[g + 1]; ++q)
                for (int side = 0; side < 2; ++side) {
                    const int32_t K = S.frac_cell[2 * (size_t)cand_face[q] + side];
                    if (K < 0) continue;
                    for (int a = 0; a < 8; ++a) {
                        const int32_t u = S.node_unk[hex8[8 * (int64_t)K + a]];
                        if (u >= 0 && mark[u] != g) {
                            mark[u] = g;
                            cand_node.push_back(u);
                        }
                    }
                }
            std::sort(cand_node.begin() + start, cand_node.end());
            cand_nptr[g + 1] = (int32_t)cand_node.size();
            elim[g] = eliminate && cand_ptr[g + 1] - cand_ptr[g] <= kGroupMaxFaces &&
                      cand_nptr[g + 1] - cand_nptr[g] <= kGroupMaxNodes;
        }
    }
    // colour the eliminated groups: groups of one colour share no free node
    std::vector<int32_t> gcol(ncand, -1);
    {
        std::vector<std::vector<int32_t>> node_colors(nfree);
        std::vector<int32_t> seen;
        for (int32_t g = 0; g < ncand; ++g) {
            if (!elim[g]) continue;
            seen.clear();
            for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q)
                for (int32_t c : node_colors[cand_node[q]]) seen.push_back(c);
            std::sort(seen.begin(), seen.end());
            int32_t c = 0;
            for (int32_t x : seen)
                if (x == c) ++c; else if (x > c) break;
            gcol[g] = c;
            S.ngcolor = std::max(S.ngcolor, c + 1);
            for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q) node_colors[cand_node[q]].push_back(c);
        }
    }
    // eliminated groups by colour
    std::vector<int32_t> order;
    S.gcolor_ptr.assign(S.ngcolor + 1, 0);
    for (int32_t g = 0; g < ncand; ++g)
        if (elim[g]) S.gcolor_ptr[gcol[g] + 1]++;
    for (int c = 0; c < S.ngcolor; ++c) S.gcolor_ptr[c + 1] += S.gcolor_ptr[c];
    order.resize(S.gcolor_ptr[S.ngcolor]);
    {
        std::vector<int32_t> fill(S.gcolor_ptr.begin(), S.gcolor_ptr.end() - 1);
        for (int32_t g = 0; g < ncand; ++g)
            if (elim[g]) order[fill[gcol[g]]++] = g;
    }
    S.ngroup = (int32_t)order.size();

    // unknowns: free nodes, kept faces, then eliminated faces group by group
    S.frac_unk.assign(nf, -1);
    std::vector<int32_t> face_grp(nf, -1), face_loc(nf, -1);
    int32_t nkept = 0;
    for (int32_t f = 0; f < nf; ++f)
        if (!elim[root_id[find(f)]]) S.frac_unk[f] = nfree + nkept++;
    S.nunk = nfree + nkept;
    S.nx = nfree + nf;
    S.grp_ptr.assign(S.ngroup + 1, 0);
    S.grp_nptr.assign(S.ngroup + 1, 0);
    S.grp_off.assign(S.ngroup + 1, 0);
    S.grp_poff.assign(S.ngroup + 1, 0);
    S.grp_face.clear();
    S.grp_node.clear();
    {
        int32_t next = S.nunk;
        for (int32_t G = 0; G < S.ngroup; ++G) {
            const int32_t g = order[G];
            const int32_t ng = cand_ptr[g + 1] - cand_ptr[g], mg = cand_nptr[g + 1] - cand_nptr[g];
            for (int32_t q = cand_ptr[g]; q < cand_ptr[g + 1]; ++q) {
                const int32_t f = cand_face[q];
                S.frac_unk[f] = next++;
                face_grp[f] = G;
                face_loc[f] = q - cand_ptr[g];
                S.grp_face.push_back(f);
            }
            for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q) S.grp_node.push_back(cand_node[q]);
            S.grp_ptr[G + 1] = S.grp_ptr[G] + ng;
            S.grp_nptr[G + 1] = S.grp_nptr[G] + mg;
            S.grp_off[G + 1] = S.grp_off[G] + (int64_t)ng * (ng + mg);
            S.grp_poff[G + 1] = S.grp_poff[G] + (int64_t)mg * mg;
            S.grp_max_g = std::max(S.grp_max_g, ng);
            S.grp_max_m = std::max(S.grp_max_m, mg);
        }
    }
    // node (system unknown) -> eliminated groups, for the fill of the pattern
    std::vector<int32_t> ngp_ptr(nfree + 1, 0), ngp;
    for (int32_t q = 0; q < (int32_t)S.grp_node.size(); ++q) ngp_ptr[S.grp_node[q] + 1]++;
    for (int32_t u = 0; u < nfree; ++u) ngp_ptr[u + 1] += ngp_ptr[u];
    ngp.resize(ngp_ptr[nfree]);
    {
        std::vector<int32_t> fill(ngp_ptr.begin(), ngp_ptr.end() - 1);
        for (int32_t G = 0; G < S.ngroup; ++G)
            for (int32_t q = S.grp_nptr[G]; q < S.grp_nptr[G + 1]; ++q) ngp[fill[S.grp_node[q]]++] = G;
    }

    auto cell_unknowns = [&](int32_t K, int32_t *u) {
        int m = 0;
        for (int a = 0; a < 8; ++a) u[m++] = S.node_unk[hex8[8 * (int64_t)K + a]];
        for (int lf = 0; lf < 6; ++lf)
            if (S.fmask[K] >> lf & 1) u[m++] = S.frac_unk[S.cell_frac[6 * (size_t)K + lf]];
        return m;
    };

    // CSR pattern: row = free node or kept fracture face; a node also couples
    // to every free node of each eliminated group it belongs to (fill)
    S.row_ptr.assign((size_t)S.nunk + 1, 0);
    std::vector<int32_t> marker((size_t)S.nunk, -1);
    std::vector<int32_t> cols;
    cols.reserve(128);
    // two passes: count then fill
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            for (int32_t r = 0; r < S.nunk; ++r) S.row_ptr[r + 1] += S.row_ptr[r];
            if (S.row_ptr[S.nunk] < 0 || (int64_t)S.row_ptr[S.nunk] >= INT32_MAX)
                throw Error(VAG_ERR_UNSUPPORTED, "system has more than 2^31 nonzeros");
            S.col.resize(S.row_ptr[S.nunk]);
            std::fill(marker.begin(), marker.end(), -1);
        }
        auto add = [&](int32_t row, int32_t c) {
            if (c >= 0 && c < S.nunk && marker[c] != row) {
                marker[c] = row;
                cols.push_back(c);
            }
        };
        auto finish_row = [&](int32_t row) {
            if (pass == 0) {
                S.row_ptr[row + 1] = (int32_t)cols.size();
            } else {
                std::sort(cols.begin(), cols.end());
                std::copy(cols.begin(), cols.end(), S.col.begin() + S.row_ptr[row]);
            }
        };
        for (int32_t s = 0; s < nn; ++s) {
            const int32_t row = S.node_unk[s];
            if (row < 0) continue;
            cols.clear();
            for (int32_t q = S.node_cell_ptr[s]; q < S.node_cell_ptr[s + 1]; ++q) {
                int32_t u[14];
                const int m = cell_unknowns(S.node_cell[q] >> 3, u);
                for (int i = 0; i < m; ++i) add(row, u[i]);
            }
            for (int32_t q = ngp_ptr[row]; q < ngp_ptr[row + 1]; ++q) {
                const int32_t G = ngp[q];
                for (int32_t k = S.grp_nptr[G]; k < S.grp_nptr[G + 1]; ++k) add(row, S.grp_node[k]);
            }
            finish_row(row);
        }
        for (int32_t f = 0; f < nf; ++f) {
            const int32_t row = S.frac_unk[f];
            if (row >= S.nunk) continue;
            cols.clear();
            for (int side = 0; side < 2; ++side) {
                const int32_t K = S.frac_cell[2 * (size_t)f + side];
                if (K < 0) continue;
                int32_t u[14];
                const int m = cell_unknowns(K, u);
                for (int i = 0; i < m; ++i) add(row, u[i]);
            }
            finish_row(row);
        }
    }
    S.nnz = S.row_ptr[S.nunk];

    // sliced ELL copy of the pattern (64-row slices, column-major in a slice)
    {
        const int32_t n = S.nunk;
        const int64_t nslice = (n + kSliceRows - 1) / kSliceRows;
        S.sell_ptr.assign(nslice + 1, 0);
        for (int64_t sl = 0; sl < nslice; ++sl) {
            int32_t w = 0;
            for (int32_t r = (int32_t)(sl * kSliceRows); r < std::min<int64_t>(n, (sl + 1) * kSliceRows); ++r)
                w = std::max(w, S.row_ptr[r + 1] - S.row_ptr[r]);
            S.sell_ptr[sl + 1] = S.sell_ptr[sl] + (int64_t)w * kSliceRows;
        }
        if (S.sell_ptr[nslice] >= INT32_MAX)
            throw Error(VAG_ERR_UNSUPPORTED, "padded system has more than 2^31 entries");
        S.sell_col.assign(S.sell_ptr[nslice], 0);
        S.csr2sell.assign(S.nnz, -1);
        for (int64_t sl = 0; sl < nslice; ++sl) {
            const int32_t w = (int32_t)((S.sell_ptr[sl + 1] - S.sell_ptr[sl]) / kSliceRows);
            for (int lane = 0; lane < kSliceRows; ++lane) {
                const int64_t r = sl * kSliceRows + lane;
                for (int32_t k = 0; k < w; ++k) {
                    const int64_t pos = S.sell_ptr[sl] + (int64_t)k * kSliceRows + lane;
                    if (r < n && k < S.row_ptr[r + 1] - S.row_ptr[r]) {
                        S.sell_col[pos] = S.col[S.row_ptr[r] + k];
                        S.csr2sell[S.row_ptr[r] + k] = (int32_t)pos;
                    } else {
                        S.sell_col[pos] = r < n ? (int32_t)r : 0;  // padding: own row, value 0
                    }
                }
            }
        }
    }
    S.diag_pos.assign(S.nunk, -1);
    for (int32_t r = 0; r < S.nunk; ++r)
        for (int32_t q = S.row_ptr[r]; q < S.row_ptr[r + 1]; ++q)
            if (S.col[q] == r) S.diag_pos[r] = S.csr2sell[q];

    auto sell_pos = [&](int32_t r, int32_t c) {
        const int32_t *c0 = S.col.data() + S.row_ptr[r];
        const int32_t *c1 = S.col.data() + S.row_ptr[r + 1];
        const int32_t *it = std::lower_bound(c0, c1, c);
        if (it == c1 || *it != c) throw Error(VAG_ERR_ARG, "internal: pattern misses an entry");
        return S.csr2sell[it - S.col.data()];
    };
    auto node_local = [&](int32_t G, int32_t u) {
        const int32_t *b0 = S.grp_node.data() + S.grp_nptr[G];
        const int32_t *b1 = S.grp_node.data() + S.grp_nptr[G + 1];
        return (int32_t)(std::lower_bound(b0, b1, u) - b0);
    };

    // slot maps
    S.slot_ptr.assign((size_t)nc + 1, 0);
    for (int32_t K = 0; K < nc; ++K) {
        int m = 8 + __builtin_popcount(S.fmask[K]);
        S.slot_ptr[K + 1] = S.slot_ptr[K] + m * m;
    }
    S.slots.resize(S.slot_ptr[nc]);
    for (int32_t K = 0; K < nc; ++K) {
        int32_t u[14], fid[14];
        int m = cell_unknowns(K, u);
        for (int a = 0, lf = 0; a < m; ++a) {
            fid[a] = -1;
            if (a >= 8) {
                while (!(S.fmask[K] >> lf & 1)) ++lf;
                fid[a] = S.cell_frac[6 * (size_t)K + lf++];
            }
        }
        int32_t *out = S.slots.data() + S.slot_ptr[K];
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                int32_t v;
                if (u[a] < 0) {
                    v = -1;
                } else if (u[b] < 0) {
                    v = -2;
                } else if (u[a] >= S.nunk) {
                    const int32_t G = face_grp[fid[a]];
                    const int32_t g = S.grp_ptr[G + 1] - S.grp_ptr[G];
                    const int32_t W = g + S.grp_nptr[G + 1] - S.grp_nptr[G];
                    const int32_t col = u[b] >= S.nunk ? face_loc[fid[b]] : g + node_local(G, u[b]);
                    const int64_t off = S.grp_off[G] + (int64_t)face_loc[fid[a]] * W + col;
                    if (off >= INT32_MAX) throw Error(VAG_ERR_UNSUPPORTED, "fracture-face groups too large");
                    v = (int32_t)off;
                } else if (u[b] >= S.nunk) {
                    v = -1;
                } else {
                    v = sell_pos(u[a], u[b]);
                }
                out[a * m + b] = v;
            }
    }
    // system positions of the node pairs of each group
    S.grp_pos.resize(S.grp_poff[S.ngroup]);
    for (int32_t G = 0; G < S.ngroup; ++G) {
        const int32_t m = S.grp_nptr[G + 1] - S.grp_nptr[G];
        const int32_t *B = S.grp_node.data() + S.grp_nptr[G];
        for (int32_t p = 0; p < m; ++p)
            for (int32_t q = 0; q < m; ++q) S.grp_pos[S.grp_poff[G] + (int64_t)p * m + q] = sell_pos(B[p], B[q]);
    }

    // greedy colouring: cells sharing a node get different colours
    std::vector<int32_t> color(nc, -1);
    std::vector<int32_t> seen(64, -1);
    int ncolor = 0;
    for (int32_t K = 0; K < nc; ++K) {
        for (int a = 0; a < 8; ++a) {
            int32_t s = hex8[8 * (int64_t)K + a];
            for (int32_t q = S.node_cell_ptr[s]; q < S.node_cell_ptr[s + 1]; ++q) {
                int32_t L = S.node_cell[q] >> 3;
                if (color[L] >= 0) {
                    if (color[L] >= (int)seen.size()) seen.resize(color[L] + 1, -1);
                    seen[color[L]] = K;
                }
            }
        }
        int c = 0;
        while (c < (int)seen.size() && seen[c] == K) ++c;
        color[K] = c;
        ncolor = std::max(ncolor, c + 1);
        if (c >= (int)seen.size()) seen.resize(c + 1, -1);
    }
    S.ncolor = ncolor;
    S.color_ptr.assign(ncolor + 1, 0);
    for (int32_t K = 0; K < nc; ++K) S.color_ptr[color[K] + 1]++;
    for (int c = 0; c < ncolor; ++c) S.color_ptr[c + 1] += S.color_ptr[c];
    S.color_cells.resize(nc);
    {
        std::vector<int32_t> fill(S.color_ptr.begin(), S.color_ptr.end() - 1);
        for (int32_t K = 0; K < nc; ++K) S.color_cells[fill[color[K]]++] = K;
    }
}

}  // namespace vag

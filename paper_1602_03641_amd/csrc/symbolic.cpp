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
//  - sliced-ELL slice pointers of that pattern (the device fills the columns),
//  - node -> (cell, slot) and node -> (fracture, vertex) adjacency, used by the
//    row-by-row assembly and by the transport.
#include <algorithm>
#include <array>
#include <exception>
#include <thread>
#include <memory>
#include <unordered_map>

#include "host_parallel.h"
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

namespace {
// sorts a short row in place (rows hold at most a few dozen columns)
inline void sort_row(int32_t *b, int32_t *e) {
    if (e - b > 48) {
        std::sort(b, e);
        return;
    }
    for (int32_t *i = b + 1; i < e; ++i) {
        const int32_t v = *i;
        int32_t *j = i;
        for (; j > b && j[-1] > v; --j) *j = j[-1];
        *j = v;
    }
}
}  // namespace

namespace {
// the rows in the system numbering, sorted: new row r is natural row
// order[r], whose columns (natural numbering) src(o) lists
template <class Src>
uvector<int32_t> sorted_rows(const Symbolic &S, const std::vector<int32_t> &rp, const Src &src) {
    const int32_t n = S.nunk;
    uvector<int32_t> cl((size_t)rp[n]);
    parallel_chunks(n, [&](int, int64_t r0, int64_t r1) {
        for (int32_t r = (int32_t)r0; r < (int32_t)r1; ++r) {
            const int32_t *in = src(S.sys_old[r]);
            int32_t *out = cl.data() + rp[r];
            const int32_t len = rp[r + 1] - rp[r];
            for (int32_t k = 0; k < len; ++k) out[k] = S.sys_new[in[k]];
            sort_row(out, out + len);
        }
    });
    return cl;
}
}  // namespace

void finish_symbolic_pattern(Symbolic &S, const std::vector<const int32_t *> *row_src, bool columns) {
    const int32_t nn = S.nn, nf = S.nf, nfree = S.nfree;
    // Renumber the system rows so that, inside windows of kSortWindow rows
    // (node rows and face rows apart), longer rows come first (stable):
    // slices then hold rows of similar length and carry little padding,
    // while rows of equal length keep their order and their locality.
    // Old row o lists its columns at row_src[o] (or in S.col from
    // S.row_ptr[o]), unsorted and in the old numbering.
    {
        const int32_t n = S.nunk;
        std::vector<int32_t> order(n);
        auto len = [&](int32_t r) { return S.row_ptr[r + 1] - S.row_ptr[r]; };
        // every row holds its own unknown, through a cell of its node or face
        for (int32_t r = 0; r < nfree; ++r)
            if (len(r) < 1) throw Error(VAG_ERR_MESH, "a free node of no cell (system row " + std::to_string(r) + ")");
        // a counting sort by decreasing length inside each window (stable)
        auto windows = [&](int32_t b0, int32_t b1) {
            const int64_t nw = ((int64_t)b1 - b0 + kSortWindow - 1) / kSortWindow;
            parallel_chunks(nw, [&](int, int64_t w0, int64_t w1) {
                std::vector<int32_t> cnt;
                for (int64_t w = w0; w < w1; ++w) {
                    const int32_t r0 = b0 + (int32_t)(w * kSortWindow), r1 = std::min(b1, r0 + kSortWindow);
                    int32_t lmax = 0;
                    for (int32_t r = r0; r < r1; ++r) lmax = std::max(lmax, len(r));
                    cnt.assign((size_t)lmax + 2, 0);
                    for (int32_t r = r0; r < r1; ++r) cnt[lmax - len(r) + 1]++;
                    for (int32_t l = 0; l <= lmax; ++l) cnt[l + 1] += cnt[l];
                    for (int32_t r = r0; r < r1; ++r) order[r0 + cnt[lmax - len(r)]++] = r;
                }
            }, 64);
        };
        windows(0, nfree);
        windows(nfree, n);
        S.sys_old.swap(order);  // new row -> old row
        S.sys_new.resize(n);    // old row -> new row
        std::vector<int32_t> rp(n + 1);
        parallel_chunks(n, [&](int, int64_t r0, int64_t r1) {
            for (int64_t r = r0; r < r1; ++r) {
                S.sys_new[S.sys_old[r]] = (int32_t)r;
                rp[r + 1] = len(S.sys_old[r]);
            }
        });
        // row pointers in the new numbering
        rp[0] = 0;
        for (int32_t r = 0; r < n; ++r) rp[r + 1] += rp[r];
        if (columns) {
            uvector<int32_t> cl = row_src ? sorted_rows(S, rp, [&](int32_t o) { return (*row_src)[o]; })
                                          : sorted_rows(S, rp, [&](int32_t o) { return S.col.data() + S.row_ptr[o]; });
            S.col.swap(cl);
            S.col_on_host = true;
        } else {
            S.col = uvector<int32_t>();  // the device builds the columns
            S.col_on_host = false;
        }
        S.row_ptr.swap(rp);
        parallel_chunks(nn, [&](int, int64_t s0, int64_t s1) {
            for (int64_t v = s0; v < s1; ++v)
                if (S.node_unk[v] >= 0) S.node_unk[v] = S.sys_new[S.node_unk[v]];
        });
        for (auto &u : S.frac_unk)
            if (u < n) u = S.sys_new[u];
        for (int32_t G = 0; G < S.ngroup; ++G) {
            for (int32_t q = S.grp_nptr[G]; q < S.grp_nptr[G + 1]; ++q) S.grp_node[q] = S.sys_new[S.grp_node[q]];
            std::sort(S.grp_node.begin() + S.grp_nptr[G], S.grp_node.begin() + S.grp_nptr[G + 1]);
        }
    }

    // sliced ELL slice pointers (64-row slices, width = longest row); the
    // column array itself is filled on the device from the CSR pattern
    {
        const int32_t n = S.nunk;
        const int64_t nslice = (n + kSliceRows - 1) / kSliceRows;
        S.sell_ptr.assign(nslice + 1, 0);
        parallel_chunks(nslice, [&](int, int64_t l0, int64_t l1) {
            for (int64_t sl = l0; sl < l1; ++sl) {
                int32_t w = 0;
                for (int32_t r = (int32_t)(sl * kSliceRows); r < std::min<int64_t>(n, (sl + 1) * kSliceRows); ++r)
                    w = std::max(w, S.row_ptr[r + 1] - S.row_ptr[r]);
                S.sell_ptr[sl + 1] = (int64_t)w * kSliceRows;
            }
        }, 1024);
        for (int64_t sl = 0; sl < nslice; ++sl) S.sell_ptr[sl + 1] += S.sell_ptr[sl];
        if (S.sell_ptr[nslice] >= INT32_MAX)
            throw Error(VAG_ERR_UNSUPPORTED, "padded system has more than 2^31 entries");
    }

    // row -> node or kept face, face -> (group, local index)
    S.unk_node.assign(nfree, -1);
    parallel_chunks(nn, [&](int, int64_t s0, int64_t s1) {
        for (int64_t v = s0; v < s1; ++v)
            if (S.node_unk[v] >= 0) S.unk_node[S.node_unk[v]] = (int32_t)v;
    });
    S.unk_face.assign(S.nunk - nfree, -1);
    for (int32_t f = 0; f < nf; ++f)
        if (S.frac_unk[f] < S.nunk) S.unk_face[S.frac_unk[f] - nfree] = f;
}

void build_symbolic(int64_t nn64, int64_t nc64, int64_t nf64, const int32_t *hex8,
                    const int32_t *frac_nodes, const uint8_t *dirichlet, bool eliminate, Symbolic &S,
                    bool rows_on_device) {
    if (nn64 <= 0 || nc64 <= 0 || nf64 < 0 || nn64 >= INT32_MAX || nc64 >= INT32_MAX / 8 ||
        nf64 >= INT32_MAX / 4)
        throw Error(VAG_ERR_ARG, "mesh sizes out of range");
    const int32_t nn = (int32_t)nn64, nc = (int32_t)nc64, nf = (int32_t)nf64;
    S.nn = nn;
    S.nc = nc;
    S.nf = nf;

    {
        // the first cell (in index order) naming a node out of range
        std::vector<int64_t> bad((size_t)chunk_count(nc), INT64_MAX);
        parallel_chunks(nc, [&](int t, int64_t k0, int64_t k1) {
            for (int64_t i = 8 * k0; i < 8 * k1; ++i)
                if (hex8[i] < 0 || hex8[i] >= nn) {
                    bad[t] = i / 8;
                    return;
                }
        });
        const int64_t K = *std::min_element(bad.begin(), bad.end());
        if (K != INT64_MAX) throw Error(VAG_ERR_ARG, "hex8 node index out of range at cell " + std::to_string(K));
    }
    for (int64_t i = 0; i < 4 * (int64_t)nf; ++i)
        if (frac_nodes[i] < 0 || frac_nodes[i] >= nn)
            throw Error(VAG_ERR_ARG, "fracture face node index out of range at face " + std::to_string(i / 4));

    // node -> (cell, slot), K * 8 + a in ascending order.  With the rows on
    // the device, the device builds it too (launch_node_cell) and the host
    // only lists the cells around the first node of each fracture face.
    std::vector<int32_t> lead_id, lead_ptr, lead_cell;
    if (!rows_on_device) {
        S.node_cell_ptr.assign(nn + 1, 0);
        for (int64_t i = 0; i < 8 * (int64_t)nc; ++i) S.node_cell_ptr[hex8[i] + 1]++;
        for (int32_t s = 0; s < nn; ++s) S.node_cell_ptr[s + 1] += S.node_cell_ptr[s];
        S.node_cell.resize(S.node_cell_ptr[nn]);
        std::vector<int32_t> fill(S.node_cell_ptr.begin(), S.node_cell_ptr.end() - 1);
        for (int64_t i = 0; i < 8 * (int64_t)nc; ++i) S.node_cell[fill[hex8[i]]++] = (int32_t)i;
    } else if (nf > 0) {
        S.node_cell_ptr.clear();
        S.node_cell.clear();
        lead_id.assign(nn, -1);
        int32_t nl = 0;
        for (int32_t f = 0; f < nf; ++f)
            if (lead_id[frac_nodes[4 * (int64_t)f]] < 0) lead_id[frac_nodes[4 * (int64_t)f]] = nl++;
        std::vector<std::vector<int32_t>> part((size_t)chunk_count(nc));
        parallel_chunks(nc, [&](int t, int64_t k0, int64_t k1) {
            for (int64_t i = 8 * k0; i < 8 * k1; ++i)
                if (lead_id[hex8[i]] >= 0) part[t].push_back((int32_t)i);
        });
        lead_ptr.assign((size_t)nl + 1, 0);
        for (const auto &p : part)
            for (int32_t i : p) lead_ptr[lead_id[hex8[i]] + 1]++;
        for (int32_t l = 0; l < nl; ++l) lead_ptr[l + 1] += lead_ptr[l];
        lead_cell.resize(lead_ptr[nl]);
        std::vector<int32_t> fill(lead_ptr.begin(), lead_ptr.end() - 1);
        for (const auto &p : part)
            for (int32_t i : p) lead_cell[fill[lead_id[hex8[i]]]++] = i;
    }
    // the cells (K * 8 + a, ascending) around node s, a first node of a fracture face
    auto around = [&](int32_t s, const int32_t *&b, const int32_t *&e) {
        if (rows_on_device) {
            b = lead_cell.data() + lead_ptr[lead_id[s]];
            e = lead_cell.data() + lead_ptr[lead_id[s] + 1];
        } else {
            b = S.node_cell.data() + S.node_cell_ptr[s];
            e = S.node_cell.data() + S.node_cell_ptr[s + 1];
        }
    };

    // fracture faces: each matched against the faces of the cells around its
    // first node (cells in ascending order, then local faces in order)
    S.frac_node.assign(nn, 0);
    for (int64_t i = 0; i < 4 * (int64_t)nf; ++i) S.frac_node[frac_nodes[i]] = 1;
    {
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
    }
    S.fmask.assign(nc, 0);
    S.cell_frac.assign(6 * (size_t)nc, -1);
    S.frac_cell.assign(2 * (size_t)nf, -1);
    for (int32_t f = 0; f < nf; ++f) {
        const int32_t *fn = frac_nodes + 4 * (int64_t)f;
        const Key4 key = sorted_key(fn);
        int32_t prev = -1;
        const int32_t *qb, *qe;
        around(fn[0], qb, qe);
        for (const int32_t *q = qb; q < qe; ++q) {
            const int32_t K = *q >> 3;
            if (K == prev) continue;  // a cell that names the node twice
            prev = K;
            const int32_t *cn = hex8 + 8 * (int64_t)K;
            for (int lf = 0; lf < 6; ++lf) {
                int32_t c[4];
                for (int i = 0; i < 4; ++i) c[i] = cn[hexf(lf, i)];
                if (!(sorted_key(c) == key)) continue;
                if (!same_cycle(c, fn))
                    throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(f) + " nodes are not in cyclic order");
                const int side = S.frac_cell[2 * (size_t)f] < 0 ? 0 : (S.frac_cell[2 * (size_t)f + 1] < 0 ? 1 : 2);
                if (side == 2)
                    throw Error(VAG_ERR_MESH, "fracture face " + std::to_string(f) + " has more than two cells");
                S.frac_cell[2 * (size_t)f + side] = K;
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
    for (int32_t f = 0; f < nf; ++f)
        for (int side = 0; side < 2; ++side) {
            const int32_t K = S.frac_cell[2 * (size_t)f + side];
            if (K < 0) continue;
            int lf = 0;
            while (!(S.fmask[K] >> lf & 1)) ++lf;  // K's first fracture face
            const int32_t a = find(S.cell_frac[6 * (size_t)K + lf]), b = find(f);
            if (a != b) uf[std::max(a, b)] = std::min(a, b);
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
    // colour the eliminated groups: groups of one colour share no free node;
    // greedy in group order, the least colour that no node of the group has
    // yet (colours below 64 as a bit mask per node, higher ones listed)
    std::vector<int32_t> gcol(ncand, -1);
    {
        std::vector<uint64_t> low(nfree, 0);
        std::unordered_map<int32_t, std::vector<int32_t>> high;
        std::vector<int32_t> seen;
        for (int32_t g = 0; g < ncand; ++g) {
            if (!elim[g]) continue;
            uint64_t m = 0;
            for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q) m |= low[cand_node[q]];
            int32_t c;
            if (~m) {
                c = __builtin_ctzll(~m);
            } else {
                seen.clear();
                for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q) {
                    auto it = high.find(cand_node[q]);
                    if (it != high.end()) seen.insert(seen.end(), it->second.begin(), it->second.end());
                }
                std::sort(seen.begin(), seen.end());
                c = 64;
                for (int32_t x : seen)
                    if (x == c) ++c; else if (x > c) break;
            }
            gcol[g] = c;
            S.ngcolor = std::max(S.ngcolor, c + 1);
            for (int32_t q = cand_nptr[g]; q < cand_nptr[g + 1]; ++q) {
                if (c < 64) low[cand_node[q]] |= 1ull << c;
                else high[cand_node[q]].push_back(c);
            }
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
    std::vector<int32_t> &ngp_ptr = S.node_grp_ptr, &ngp = S.node_grp;
    ngp_ptr.assign(nfree + 1, 0);
    for (int32_t q = 0; q < (int32_t)S.grp_node.size(); ++q) ngp_ptr[S.grp_node[q] + 1]++;
    for (int32_t u = 0; u < nfree; ++u) ngp_ptr[u + 1] += ngp_ptr[u];
    ngp.resize(ngp_ptr[nfree]);
    {
        std::vector<int32_t> fill(ngp_ptr.begin(), ngp_ptr.end() - 1);
        for (int32_t G = 0; G < S.ngroup; ++G)
            for (int32_t q = S.grp_nptr[G]; q < S.grp_nptr[G + 1]; ++q) ngp[fill[S.grp_node[q]]++] = G;
    }
    S.face_grp = std::move(face_grp);
    S.face_loc = std::move(face_loc);
    if (rows_on_device) return;  // finish_symbolic_lengths follows, with the device's row lengths

    // unknowns of each cell: 8 nodes, then its fracture faces by local face
    uvector<int32_t> cu(14 * (size_t)nc);
    uvector<uint8_t> cm(nc);
    parallel_chunks(nc, [&](int, int64_t k0, int64_t k1) {
        for (int32_t K = (int32_t)k0; K < (int32_t)k1; ++K) {
            int32_t *u = cu.data() + 14 * (size_t)K;
            int m = 0;
            for (int a = 0; a < 8; ++a) u[m++] = S.node_unk[hex8[8 * (int64_t)K + a]];
            for (int lf = 0; lf < 6; ++lf)
                if (S.fmask[K] >> lf & 1) u[m++] = S.frac_unk[S.cell_frac[6 * (size_t)K + lf]];
            cm[K] = (uint8_t)m;
        }
    });

    // CSR pattern, rows in unknown order (node rows by node index, then kept
    // faces by face index): row = free node or kept fracture face; a node
    // also couples to every free node of each eliminated group it belongs to
    // (fill)
    S.row_ptr.assign((size_t)S.nunk + 1, 0);
    // rows are built in chunks of nodes (then of faces), each chunk into its
    // own column list; the renumbering reads every row from there
    std::vector<std::vector<int32_t>> part;
    std::vector<const int32_t *> row_src;
    {
        const int Tn = chunk_count(nn), Tf = chunk_count(nf);
        part.resize(Tn + Tf);
        auto build_rows = [&](std::vector<int32_t> &out, bool faces, int64_t i0, int64_t i1) {
            std::vector<int32_t> marker((size_t)S.nunk, -1);
            std::vector<int32_t> cols;
            cols.reserve(128);
            out.reserve((size_t)(i1 - i0) * (faces ? 20 : 28));
            auto add = [&](int32_t row, int32_t c) {
                if (c >= 0 && c < S.nunk && marker[c] != row) {
                    marker[c] = row;
                    cols.push_back(c);
                }
            };
            auto add_cell = [&](int32_t row, int32_t K) {
                const int32_t *u = cu.data() + 14 * (size_t)K;
                for (int i = 0; i < cm[K]; ++i) add(row, u[i]);
            };
            for (int64_t i = i0; i < i1; ++i) {
                int32_t row;
                cols.clear();
                if (!faces) {
                    const int32_t s = (int32_t)i;
                    row = S.node_unk[s];
                    if (row < 0) continue;
                    for (int32_t q = S.node_cell_ptr[s]; q < S.node_cell_ptr[s + 1]; ++q)
                        add_cell(row, S.node_cell[q] >> 3);
                    for (int32_t q = ngp_ptr[row]; q < ngp_ptr[row + 1]; ++q) {
                        const int32_t G = ngp[q];
                        for (int32_t k = S.grp_nptr[G]; k < S.grp_nptr[G + 1]; ++k) add(row, S.grp_node[k]);
                    }
                } else {
                    const int32_t f = (int32_t)i;
                    row = S.frac_unk[f];
                    if (row >= S.nunk) continue;
                    for (int side = 0; side < 2; ++side)
                        if (S.frac_cell[2 * (size_t)f + side] >= 0) add_cell(row, S.frac_cell[2 * (size_t)f + side]);
                }
                // unsorted here: the renumbering sorts every row once
                out.insert(out.end(), cols.begin(), cols.end());
                S.row_ptr[row + 1] = (int32_t)cols.size();
            }
        };
        parallel_chunks(nn, [&](int t, int64_t i0, int64_t i1) { build_rows(part[t], false, i0, i1); });
        parallel_chunks(nf, [&](int t, int64_t i0, int64_t i1) { build_rows(part[Tn + t], true, i0, i1); });
        int64_t total = 0;
        for (auto &v : part) total += (int64_t)v.size();
        if (total >= INT32_MAX) throw Error(VAG_ERR_UNSUPPORTED, "system has more than 2^31 nonzeros");
        // where each row's list starts in its chunk's buffer (rows of a chunk
        // are consecutive unknowns: node_unk and frac_unk increase with the
        // node and face index)
        row_src.assign((size_t)S.nunk, nullptr);
        for (int t = 0; t < Tn + Tf; ++t) {
            const bool faces = t >= Tn;
            const int T = faces ? Tf : Tn, c = faces ? t - Tn : t;
            const int64_t n_items = faces ? nf : nn, i0 = n_items * c / T, i1 = n_items * (c + 1) / T;
            const int32_t *p = part[t].data();
            for (int64_t i = i0; i < i1; ++i) {
                const int32_t row = faces ? (S.frac_unk[i] < S.nunk ? S.frac_unk[i] : -1) : S.node_unk[i];
                if (row < 0) continue;
                row_src[row] = p;
                p += S.row_ptr[row + 1];
            }
        }
        for (int32_t r = 0; r < S.nunk; ++r) S.row_ptr[r + 1] += S.row_ptr[r];
    }
    S.nnz = S.row_ptr[S.nunk];

    finish_symbolic_pattern(S, &row_src);
}

void finish_symbolic_lengths(Symbolic &S, const int32_t *len) {
    const int32_t n = S.nunk;
    S.row_ptr.assign((size_t)n + 1, 0);
    int64_t total = 0;
    for (int32_t r = 0; r < n; ++r) {
        total += std::max(len[r], 0);
        if (total >= INT32_MAX) throw Error(VAG_ERR_UNSUPPORTED, "system has more than 2^31 nonzeros");
        S.row_ptr[r + 1] = (int32_t)total;
    }
    S.nnz = total;
    finish_symbolic_pattern(S, nullptr, false);
}

}  // namespace vag

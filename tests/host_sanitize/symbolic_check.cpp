// Drives the library's host symbolic phases (hexahedral and general cells)
// on meshes read from a file, for a build with the host address and
// undefined-behaviour sanitizers: every input is run through the phase and
// the pattern it builds is checked (rows sorted, columns in range, slices
// covering the rows), and the hexahedral phase run again in the mode that
// leaves the rows to the device must reach the same numbering from the row
// lengths; inputs marked invalid must end in a vag::Error.
// File layout (little endian): int64 kind (0 hexahedra, 1 general), int64
// expect_error, then the arrays of that kind (see read_* below).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "vag_internal.h"

using namespace vag;

namespace {

template <class T>
std::vector<T> read_vec(FILE *f, int64_t n) {
    std::vector<T> v((size_t)n);
    if (n && fread(v.data(), sizeof(T), (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "short read\n");
        exit(3);
    }
    return v;
}

int64_t read_i64(FILE *f) { return read_vec<int64_t>(f, 1)[0]; }

int check_pattern(const Symbolic &S) {
    if ((int64_t)S.row_ptr.size() != (int64_t)S.nunk + 1) return 10;
    for (int32_t r = 0; r < S.nunk; ++r) {
        if (S.row_ptr[r + 1] < S.row_ptr[r]) return 11;
        bool diag = false;
        for (int32_t q = S.row_ptr[r]; q < S.row_ptr[r + 1]; ++q) {
            if (S.col[q] < 0 || S.col[q] >= S.nunk) return 12;
            if (q > S.row_ptr[r] && S.col[q] <= S.col[q - 1]) return 13;
            diag |= S.col[q] == r;
        }
        if (!diag) return 14;
    }
    const int64_t nslice = ((int64_t)S.nunk + kSliceRows - 1) / kSliceRows;
    if ((int64_t)S.sell_ptr.size() != nslice + 1) return 15;
    for (int64_t sl = 0; sl < nslice; ++sl)
        for (int64_t r = sl * kSliceRows; r < std::min<int64_t>(S.nunk, (sl + 1) * kSliceRows); ++r)
            if ((int64_t)(S.row_ptr[r + 1] - S.row_ptr[r]) * kSliceRows > S.sell_ptr[sl + 1] - S.sell_ptr[sl])
                return 16;
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    const int64_t kind = read_i64(f), expect_error = read_i64(f);
    int rc = 0;
    try {
        if (kind == 0) {
            const int64_t nn = read_i64(f), nc = read_i64(f), nf = read_i64(f);
            auto hex8 = read_vec<int32_t>(f, 8 * nc);
            auto fn = read_vec<int32_t>(f, 4 * nf);
            auto dir = read_vec<uint8_t>(f, nn);
            for (int elim = 0; elim < 2 && rc == 0; ++elim) {
                Symbolic S;
                build_symbolic(nn, nc, nf, hex8.data(), fn.data(), dir.data(), elim != 0, S);
                rc = check_pattern(S);
                // the same phase with the rows left to the device: given the row
                // lengths (natural order), it must reach the same numbering
                if (rc == 0) {
                    Symbolic D;
                    build_symbolic(nn, nc, nf, hex8.data(), fn.data(), dir.data(), elim != 0, D, true);
                    std::vector<int32_t> len((size_t)D.nunk);
                    for (int32_t o = 0; o < D.nunk; ++o)
                        len[o] = S.row_ptr[S.sys_new[o] + 1] - S.row_ptr[S.sys_new[o]];
                    finish_symbolic_lengths(D, len.data());
                    if (D.sys_old != S.sys_old || D.row_ptr != S.row_ptr || D.sell_ptr != S.sell_ptr ||
                        D.node_unk != S.node_unk || D.frac_unk != S.frac_unk || D.grp_node != S.grp_node ||
                        D.frac_cell != S.frac_cell || D.cell_frac != S.cell_frac || D.col_on_host)
                        rc = 18;
                }
                printf("hex eliminate=%d: %d unknowns, %lld nonzeros, %d groups, check %d\n", elim, S.nunk,
                       (long long)S.nnz, S.ngroup, rc);
            }
        } else {
            const int64_t nn = read_i64(f), nc = read_i64(f), nface = read_i64(f);
            auto cfp = read_vec<int64_t>(f, nc + 1);
            auto cf = read_vec<int32_t>(f, cfp.back());
            auto fnp = read_vec<int64_t>(f, nface + 1);
            auto fnodes = read_vec<int32_t>(f, fnp.back());
            const int64_t nf = read_i64(f);
            auto fid = read_vec<int32_t>(f, nf);
            auto dir = read_vec<uint8_t>(f, nn);
            Symbolic S;
            GenSym G;
            build_symbolic_general(nn, nc, nface, cfp.data(), cf.data(), fnp.data(), fnodes.data(), nf, fid.data(),
                                   dir.data(), S, G);
            rc = check_pattern(S);
            if (rc == 0 && (int64_t)G.inc_ptr.size() != nc + nf + nn + 1) rc = 20;
            printf("general: %d unknowns, %lld nonzeros, %lld flux entries, check %d\n", S.nunk, (long long)S.nnz,
                   (long long)G.nflux, rc);
        }
    } catch (const Error &e) {
        printf("error %d: %s\n", (int)e.status, e.what());
        fclose(f);
        return expect_error ? 0 : 4;
    }
    fclose(f);
    if (expect_error) return 5;
    return rc;
}

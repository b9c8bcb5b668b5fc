// Block-Jacobi ILU(0) preconditioner (the third preconditioner of the solver
// study in §5.3, where GMRES and BiCGStab use it with one block per MPI
// process).  Here a block is a run of `B` consecutive unknowns of the
// system's natural order (free nodes by node index, then kept fracture faces
// by face index), factored without fill in that order; the device rows are
// stored in another order (sorted by length inside windows), so every row
// carries its device row and its factor entries their position in the
// device matrix.
#pragma once

#include "vag_internal.h"

namespace vag {

constexpr int kIluMaxBlock = 8192;  // rows per block: the solve keeps a block's vector in LDS
constexpr int kIluDefaultBlock = 128;

struct IluArgs {
    int32_t n, B, nblk;
    const int32_t *fptr;    // [n+1] factor entries of natural row o: [fptr[o], fptr[o+1])
    const uint16_t *fcol;   // local column (natural column - block start), ascending per row
    const int32_t *fsrc;    // position of the entry in the device matrix
    const int32_t *fdiag;   // [n] index of row o's diagonal entry
    const int32_t *rdev;    // [n] device row of natural row o
    // level schedules of the lower (forward) and upper (backward) dependency
    // graphs: block b's levels are [lvb[b], lvb[b+1]); level l's rows are
    // rows[lptr[l] .. lptr[l+1]) (natural indices, a permutation of the block)
    const int32_t *lvb_f, *lptr_f, *rows_f;
    const int32_t *lvb_b, *lptr_b, *rows_b;
    // per schedule slot, what the substitutions read in one 16-byte load:
    // forward {row - block start, first entry, diagonal entry, 0},
    // backward {row - block start, diagonal entry, end of the row, 0}
    const int4 *slot_f, *slot_b;
    double *fval;           // factor values: L below the diagonal (unit diagonal implied), U from it
};

class Ilu {
public:
    // Host symbolic phase from the device matrix's pattern (once per handle
    // and block size); uploads on the stream.
    void build(hipStream_t s, Tracker &tr, const Symbolic &S, int B);
    bool ready(int B) const { return B_ == B && a_.n > 0; }
    // Copies the device matrix values into the factor and factors every
    // block; *bad (device) receives 1 + the natural row of a zero or
    // non-finite pivot.
    void factor(hipStream_t s, const double *A, int *bad);
    // z = (L U)^-1 r block by block (device order vectors); skipped when
    // st && st->done.
    void apply(hipStream_t s, const double *r, double *z, const PcgState *st) const;
    int levels() const { return nlev_; }
    int64_t entries() const { return nent_; }

private:
    int B_ = 0, nlev_ = 0;
    int64_t nent_ = 0;
    IluArgs a_{};
    DBuf<int32_t> fptr_, fsrc_, fdiag_, rdev_, lvb_f_, lptr_f_, rows_f_, lvb_b_, lptr_b_, rows_b_;
    DBuf<int4> slot_f_, slot_b_;
    DBuf<uint16_t> fcol_;
    DBuf<double> fval_;
};

}  // namespace vag

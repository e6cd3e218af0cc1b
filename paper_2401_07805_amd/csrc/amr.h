// Once-refined meshes with hanging nodes: argument block and launchers
// (kernels in amr.hip, tables built on the host by vpp_amr_create).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace vpp {

struct AmrArgs {
    MeshArgs mc;                  // coarse lattice (cell size h)
    MeshArgs mf;                  // fine lattice over the whole box (h / 2)
    int64_t nc;                   // coarse lattice entries; the fine lattice follows
    int64_t n;                    // vector length (coarse + fine lattice)
    const int* cells;             // active cells: coarse index c >= 0, or -(1 + fine index)
    int ncells;
    const int* fkind;             // per fine node: -1 free, -2 unused, else its constraint list
    const int* cptr;              // constraint lists: terms cptr[i] .. cptr[i+1]
    const int* ccol;              // coarse vector entry of each term
    const double* cw;             // its weight
    const unsigned char* ident;   // per entry: 1 = identity row (not a free unknown, or Dirichlet)
    // Apply and diagonal in two launches each, no atomics.  Every active cell
    // e stores its (k+1)^3 results at scratch[q * ncells + e]; then entry g of
    // y sums scratch[nidx[j]] * nw[j] for j in [nptr[g], nptr[g+1]) (free
    // nodes with weight 1, constrained nodes through their constraint
    // weights), in increasing scratch index.  The diagonal also stores, for
    // every coarse node a fine cell reaches through constraints (in the order
    // the cell meets them), e^T K_e e at scratch[nfree_slots + soff[e] + i];
    // entry g of diag sums scratch[didx[j]] for j in [dptr[g], dptr[g+1]).
    double* scratch;
    const int* nptr;
    const int* nidx;
    const double* nw;
    const int* soff;
    const int* dptr;
    const int* didx;
    int64_t nfree_slots;
};

// y = A x (zeroes y first); every entry of y is written.
hipError_t launch_amr_apply(int k, const AmrArgs& a, const double* phi, const double* x, double* y, hipStream_t s);
// diag(A) with 1 on identity rows, and its FP64 / FP32 inverses.
hipError_t launch_amr_diag(int k, const AmrArgs& a, const double* phi, double* diag, double* inv64, float* inv32,
                           hipStream_t s);

}  // namespace vpp

// Kernel argument blocks and host-side launchers (implemented in the .hip
// files of this directory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace vpp {

template <typename T>
struct ApplyArgs {
    MeshArgs m;
    const T* x;
    T* y;
    const T* phi;
    double* dot;        // optional: atomically accumulates x . y (FP64)
    const int* done;    // optional: the kernel returns at once when *done != 0
};

// Per-problem launch configuration.
struct LaunchCfg {
    int variant;        // 0 cell per thread, 1 plane per thread
    int tile[3];
};

// y = A_D x (y must be zeroed before: nodes on shared tile faces are added
// atomically).  Returns hipErrorInvalidValue for a configuration that is not
// instantiated.
hipError_t launch_apply_f64(const LaunchCfg& c, int k, const ApplyArgs<double>& a, int nblocks,
                            hipStream_t s);
hipError_t launch_apply_f32(const LaunchCfg& c, int k, const ApplyArgs<float>& a, int nblocks,
                            hipStream_t s);
bool apply_config_supported(const LaunchCfg& c, int k);
int list_apply_configs(int k, LaunchCfg* out, int cap);

// Diagonal of A_D: accumulates into diag (zeroed before), then fix_diagonal
// writes 1 on Dirichlet rows and the FP64 / FP32 inverses.
hipError_t launch_diag(int k, const MeshArgs& m, const double* phi, double* diag, hipStream_t s);
hipError_t launch_fix_diagonal(const MeshArgs& m, double* diag, double* inv64, float* inv32,
                               hipStream_t s);

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);

// Adjoint kernels.
hipError_t launch_grad_coef(int k, const MeshArgs& m, const double* p, const double* lam, double* g,
                            hipStream_t s);
hipError_t launch_grad_phi(int k, const MeshArgs& m, const double* phi, const double* g, double* out,
                           hipStream_t s);

// Batched persistent apply (FP64).
struct BatchProblem {
    MeshArgs m;
    const double* phi;
    int tile_begin;      // first global work item of this problem
    int nrhs;
    int rhs_begin;       // first entry in the pointer tables
};

struct BatchArgs {
    const BatchProblem* probs;
    int nprob;
    int nitems;
    const double* const* x;
    double* const* y;
    int* queue;          // work counter, zero at launch
};

hipError_t launch_batch_apply(const LaunchCfg& c, int k, const BatchArgs& a, int nblocks, hipStream_t s);
int batch_blocks_per_cu(const LaunchCfg& c, int k);

struct MultiFillArgs {
    double* const* ptr;
    const int64_t* offset;   // prefix sums of the lengths, nvec + 1 entries
    int nvec;
    int* queue;              // also zeroed (may be null)
};
hipError_t launch_multi_zero(const MultiFillArgs& a, hipStream_t s);

}  // namespace vpp

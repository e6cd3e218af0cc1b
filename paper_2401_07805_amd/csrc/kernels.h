// Kernel argument blocks and host-side launchers (implemented in the .hip
// files of this directory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "blas.h"
#include "shared_nodes.h"

namespace vpp {

template <typename T>
struct ApplyArgs {
    MeshArgs m;
    const T* x;
    T* y;
    const T* phi;
    T* part;            // partial values of shared nodes: part[rank * nshared + f]
    int64_t nshared;    // stride of the rank arrays (shared_stride)
    double* dot_part;   // optional: per-workgroup partial sums of x . y (ntiles entries)
    double* dot;        // optional: x . y, written by the assembly kernel
    const int* done;    // optional: the kernels return at once when *done != 0
    bool tiles_only;    // launch the tile kernel only; the caller assembles the shared nodes
};

// Per-problem launch configuration.
struct LaunchCfg {
    int variant;        // 0 cell per thread (LDS atomics), 1 plane per thread, 2 half cell per thread (k = 3),
                        // 4 cell per thread (LDS slots)
    int tile[3];
};

inline int block_nodes(const LaunchCfg& c, int k)
{
    return (k * c.tile[0] + 1) * (k * c.tile[1] + 1) * (k * c.tile[2] + 1);
}

// Nodes lying in more than one tile (on interior tile boundary planes).
inline int64_t shared_node_count(const MeshArgs& m)
{
    const int64_t nbx = m.ntile[0] - 1, nby = m.ntile[1] - 1, nbz = m.ntile[2] - 1;
    return nbz * m.nn[1] * m.nn[0] + nby * (m.nn[2] - nbz) * m.nn[0] + nbx * (m.nn[1] - nby) * (m.nn[2] - nbz);
}

// Stride between the rank arrays of the partials: the count rounded up to a
// multiple of 4, so that every rank array starts 32-byte aligned.
inline int64_t shared_stride(const MeshArgs& m) { return (shared_node_count(m) + 3) & ~int64_t(3); }

// y = A_D x as two launches on s: the tile kernel (interior nodes of y, partials
// of shared nodes) and the assembly of the shared nodes.  y needs no
// initialisation.  hipErrorInvalidValue for a configuration that is not
// instantiated.
hipError_t launch_apply_f64(const LaunchCfg& c, int k, const ApplyArgs<double>& a, hipStream_t s);
hipError_t launch_apply_f32(const LaunchCfg& c, int k, const ApplyArgs<float>& a, hipStream_t s);
// The per-degree units behind launch_apply_f64 / launch_apply_f32.
hipError_t launch_apply_f64_k2(const LaunchCfg& c, const ApplyArgs<double>& a, hipStream_t s);
hipError_t launch_apply_f64_k3(const LaunchCfg& c, const ApplyArgs<double>& a, hipStream_t s);
hipError_t launch_apply_f64_k4(const LaunchCfg& c, const ApplyArgs<double>& a, hipStream_t s);
hipError_t launch_apply_f32_k2(const LaunchCfg& c, const ApplyArgs<float>& a, hipStream_t s);
hipError_t launch_apply_f32_k3(const LaunchCfg& c, const ApplyArgs<float>& a, hipStream_t s);
hipError_t launch_apply_f32_k4(const LaunchCfg& c, const ApplyArgs<float>& a, hipStream_t s);
bool apply_config_supported(const LaunchCfg& c, int k);
// Out-of-bounds accesses the instrumented kernels of one source file dropped
// since the last call (the count is reset); the debug library only (0 in the
// release library, ~0 if the counter could not be read).
unsigned long long bounds_count_apply_f64_k2();
unsigned long long bounds_count_apply_f64_k3();
unsigned long long bounds_count_apply_f64_k4();
unsigned long long bounds_count_apply_f32_k2();
unsigned long long bounds_count_apply_f32_k3();
unsigned long long bounds_count_apply_f32_k4();
unsigned long long bounds_count_misc();
int list_apply_configs(int k, LaunchCfg* out, int cap);
// Configurations instantiated with the mass shift (a problem with mu != 0 runs these only).
bool mass_config_supported(const LaunchCfg& c, int k);
int list_mass_configs(int k, LaunchCfg* out, int cap);
// Configurations instantiated with the arithmetic density mean (laws 2, 3: the
// only ones such a problem runs).
bool arith_config_supported(const LaunchCfg& c, int k);
int list_arith_configs(int k, LaunchCfg* out, int cap);

// Assembly of shared-face nodes from the tile partials (and of x . y).
template <typename T>
struct AssembleArgs {
    MeshArgs m;
    SharedEnum e;        // enumeration of the shared nodes (built on the host)
    const T* part;
    int64_t nshared;     // stride of the rank arrays (shared_stride); count = e.cz + e.cy + e.cx
    T* y;
    const double* dot_part;
    int ndot;
    double* dot;
    const int* done;
};
template <typename T>
hipError_t launch_assemble(const AssembleArgs<T>& a, hipStream_t s);
int device_cu_count();

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
// cv: cell scratch of cell_values(k, m) doubles (the cells' contributions,
// summed into out by launch_node_sum in a fixed order).
hipError_t launch_grad_phi(int k, const MeshArgs& m, const double* phi, const double* g, double* out, double* cv,
                           hipStream_t s);

// Values per cell-major scratch array of a mesh: (k+1)^3 per cell.
int64_t cell_values(int k, const MeshArgs& m);
// out[g] = the sum over the cells holding node g, in increasing cell index, of
// cv[q * ncell + c] (q: the node's position in cell c); every node written.
hipError_t launch_node_sum(int k, const MeshArgs& m, const double* cv, double* out, hipStream_t s);

// Closest-point projection onto {phi_h = 0} (one thread per point).
struct CpArgs {
    MeshArgs m;
    double lo[3], hi[3], h[3];   // domain box and cell size
    const double* phi;           // nodal phi (N)
    const double* nrm[3];        // nodal normal field (N each), or null: the gradient of phi_h
    const double* pts;           // n points, xyz interleaved; null: the N mesh nodes
    int64_t n;
    double phi_lim;              // band of the node mode: |phi_g| < phi_lim
    double eps, tol;
    int max_iter, normal_steps;
    double* y;                   // 3 n
    int* info;                   // n: outer steps to convergence, 0 not converged, -1 outside the band
};
// list: N ints (band nodes of the node mode), ctr: 2 ints (reset here by a fill
// kernel); nblocks: persistent workgroups (closest_point_blocks).
hipError_t launch_closest_points(int k, const CpArgs& a, int* list, int* ctr, int nblocks, hipStream_t s);
int closest_point_blocks(int k);
// out[g] = f_h(a.y[g]) where a.info[g] >= 0, else f[g] (a.n = N mesh nodes).
hipError_t launch_extend(int k, const CpArgs& a, const double* f, double* out, hipStream_t s);

// Right-hand sides of the level-set filter systems (all rows assembled).
struct RhsGeo {
    MeshArgs m;
    double ih[3];   // 1 / h_d
    double vol;     // hx hy hz
};
// b_d = (grad phi_h / |grad phi_h|, v)_d for d = 0, 1, 2; cv: 3 cell_values(k, m) doubles.
hipError_t launch_normal_rhs(int k, const RhsGeo& g, const double* phi, double* b0, double* b1, double* b2,
                             double* cv, hipStream_t s);
// b = (-div n_h, v) for the nodal components n0, n1, n2; cv: cell_values(k, m) doubles.
hipError_t launch_curvature_rhs(int k, const RhsGeo& g, const double* n0, const double* n1, const double* n2,
                                double* b, double* cv, hipStream_t s);

// One semi-implicit step of the level-set reinitialization:
//   A psi' = b,  A = M/dtau + eps K_n,  K_n = ((grad u . n)(grad v . n)),
//   b = (psi, v)/dtau + ((1 - psi^2)/2 n, grad v).
struct ReinitArgs {
    RhsGeo g;
    double eps, idtau;
    const double* n0;   // nodal normal components (N each)
    const double* n1;
    const double* n2;
};
// cv: cell_values(k, m) doubles of scratch each.
hipError_t launch_reinit_apply(int k, const ReinitArgs& r, const double* x, double* y, double* cv, hipStream_t s);
hipError_t launch_reinit_diag(int k, const ReinitArgs& r, double* diag, double* cv, hipStream_t s);
hipError_t launch_reinit_rhs(int k, const ReinitArgs& r, const double* psi, double* b, double* cv, hipStream_t s);
// part[b] = partial of x . y over the elements workgroup b visits (nblocks <= 1024).
hipError_t launch_dot_partials(const double* x, const double* y, int64_t n, double* part, int nblocks,
                               hipStream_t s);

// Batched persistent apply (FP64).
// Work items of one problem of a batch: a (tile) at degree 2, whose
// coefficient serves all right-hand sides, a (tile, rhs) at degree 3, the
// items of one tile consecutive (batch_apply_kernel).
__host__ __device__ inline int batch_items(int k, int ntiles, int nrhs) { return k == 2 ? ntiles : ntiles * nrhs; }

struct BatchProblem {
    MeshArgs m;
    const double* phi;
    int tile_begin;      // first global work item of this problem
    int nrhs;
    int rhs_begin;       // first entry in the pointer tables
    int64_t part_begin;  // first partial entry of this problem's first right-hand side
    int64_t nshared;     // stride of this problem's rank arrays (8 * nshared partial entries per rhs)
    SharedEnum se;       // their enumeration
    int ntiles;          // tiles of this problem
    int dot_begin;       // first p.Ap partial of this problem's first rhs (ntiles per rhs)
};

struct BatchArgs {
    const BatchProblem* probs;
    int nprob;
    int nitems;
    const double* const* x;
    double* const* y;
    double* part;        // partial slots of every (problem, rhs)
    int* queue;          // work counter, zero at launch (reset by the assembly kernel)
    int heaviside;       // shared by every problem of the batch
    // batched PCG (st null: plain apply): the (problem, rhs) vectors whose state
    // st[rhs].halt[par] is set are skipped, and every tile writes its partial of
    // x.y to dot_part[dot_begin + rhs_in_problem * ntiles + tile]
    const CgState* st;
    int par;
    double* dot_part;
    int any_mass = 0;    // some problem has a mass shift (at degree 3 it selects the kernel instantiation)
};

// Persistent tile kernel over all work items, then (unless tiles_only) one
// assembly launch over all (problem, rhs) vectors, which also resets the work
// counter; with tiles_only the caller assembles and resets it.
hipError_t launch_batch_apply(const LaunchCfg& c, int k, const BatchArgs& a, int nblocks, int total_rhs,
                              bool tiles_only, hipStream_t s);
int batch_blocks_per_cu(const LaunchCfg& c, int k);
// Instantiated batch configurations of degree k (writes up to cap, returns the count).
int list_batch_configs(int k, LaunchCfg* out, int cap);

}  // namespace vpp

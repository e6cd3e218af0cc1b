// Diagonal, fill and batched kernels and their launchers.
#include "apply_impl.h"
#include "shared_nodes.h"

namespace vpp {

// ---------------------------------------------------------------------------
// Diagonal: diag_a = sum_q cw_q sum_d rd[d] (dN_a/dxi_d (x_q))^2 (+ the mass
// shift's mu hx hy hz sum_q wref_q N_a(x_q)^2), from squared 1D tables (each
// term is a product of three 1D factors).  Runs once per phi, one launch per
// cell colour (cell_color), adding into the zeroed diagonal without atomics.

template <int K, int HV>
__global__ void __launch_bounds__(64) diag_kernel(MeshArgs m, const double* __restrict__ phi,
                                                   double* __restrict__ diag, CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    // phi is gathered by the (instrumented) coefficient helper
    VPP_BC_BEGIN((const double*)nullptr, (const double*)nullptr, phi, (const double*)nullptr,
                 (const double*)nullptr, (const double*)nullptr, (int64_t)m.nn[0] * m.nn[1] * m.nn[2], 0, 0, 0);
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
    double A[N3], Z[N3], Y[N3], out[N3];
    cell_coefficient<K, HV>(m, phi, cx, cy, cz, A);
#pragma unroll
    for (int q = 0; q < N3; ++q) Z[q] = A[q];
    sweep3<K, MS2, true, 2>(Z);
#pragma unroll
    for (int q = 0; q < N3; ++q) Y[q] = Z[q];
    sweep3<K, MS2, true, 1>(Y);
    sweep3<K, MD2, true, 0>(Y);
#pragma unroll
    for (int q = 0; q < N3; ++q) out[q] = m.rd[0] * Y[q];
#pragma unroll
    for (int q = 0; q < N3; ++q) Y[q] = Z[q];
    sweep3<K, MD2, true, 1>(Y);
    sweep3<K, MS2, true, 0>(Y);
#pragma unroll
    for (int q = 0; q < N3; ++q) out[q] = fma(m.rd[1], Y[q], out[q]);
    sweep3<K, MD2, true, 2>(A);
    sweep3<K, MS2, true, 1>(A);
    sweep3<K, MS2, true, 0>(A);
#pragma unroll
    for (int q = 0; q < N3; ++q) out[q] = fma(m.rd[2], A[q], out[q]);
    if (m.mass != 0.0) {
        // mass shift: mu hx hy hz sum_q wref_q N_a(x_q)^2
#pragma unroll
        for (int q = 0; q < N3; ++q) A[q] = m.mass * wref<K>(q % N, (q / N) % N, q / (N * N));
        sweep3<K, MS2, true, 2>(A);
        sweep3<K, MS2, true, 1>(A);
        sweep3<K, MS2, true, 0>(A);
#pragma unroll
        for (int q = 0; q < N3; ++q) out[q] += A[q];
    }
    const int64_t nx = m.nn[0], nxy = (int64_t)m.nn[0] * m.nn[1];
    const int64_t base = node_index(m, (int64_t)K * cx, (int64_t)K * cy, (int64_t)K * cz);
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0)
                diag[base + a0 + nx * a1 + nxy * a2] += out[a0 + N * (a1 + N * a2)];
}

__global__ void fix_diagonal_kernel(MeshArgs m, double* __restrict__ diag, double* __restrict__ inv64,
                                    float* __restrict__ inv32)
{
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(g % m.nn[0]), j = (int)((g / m.nn[0]) % m.nn[1]),
                  l = (int)(g / ((int64_t)m.nn[0] * m.nn[1]));
        double d = diag[g];
        if (is_dirichlet(m, i, j, l)) d = 1.0;
        diag[g] = d;
        const double r = 1.0 / d;
        inv64[g] = r;
        inv32[g] = (float)r;
    }
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host launchers.

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<int>(int*, int64_t, int, hipStream_t);

hipError_t launch_diag(int k, const MeshArgs& m, const double* phi, double* diag, hipStream_t s)
{
    // one launch per cell colour: the scatter into the nodes needs no atomics
#define VPP_DIAG(K)                                                                                              \
    return for_each_color(m, 64, [&](const CellColor& cc, int blocks) {                                         \
        if (m.heaviside == 0) hipLaunchKernelGGL((diag_kernel<K, 0>), dim3(blocks), dim3(64), 0, s, m, phi, diag, cc); \
        else if (m.heaviside == 1)                                                                               \
            hipLaunchKernelGGL((diag_kernel<K, 1>), dim3(blocks), dim3(64), 0, s, m, phi, diag, cc);            \
        else if (m.heaviside == 2)                                                                               \
            hipLaunchKernelGGL((diag_kernel<K, 2>), dim3(blocks), dim3(64), 0, s, m, phi, diag, cc);            \
        else hipLaunchKernelGGL((diag_kernel<K, 3>), dim3(blocks), dim3(64), 0, s, m, phi, diag, cc);           \
    });
    switch (k) {
    case 2: VPP_DIAG(2)
    case 3: VPP_DIAG(3)
    case 4: VPP_DIAG(4)
    default: return hipErrorInvalidValue;
    }
#undef VPP_DIAG
}

hipError_t launch_fix_diagonal(const MeshArgs& m, double* diag, double* inv64, float* inv32, hipStream_t s)
{
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(fix_diagonal_kernel, dim3(blocks), dim3(256), 0, s, m, diag, inv64, inv32);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Assembly of shared-face nodes.  A node lies in one or two tiles along each
// direction (two when it sits on an interior tile boundary); its value is the
// sum of the partial slots of all tiles holding it, taken in a fixed order
// (z, y, x tile index ascending), so the result is deterministic.

// Shared nodes, streamed in the order of their enumeration f, two per thread:
// the value is the sum of the partials the 2, 4 or 8 tiles holding the node
// wrote to part[rank * stride + f], taken in rank order (so the result is
// deterministic).  Every shared node has at least two sharers, so ranks 0 and 1
// are read as 16-byte pairs (stride and f are even).
template <typename T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

template <typename T>
__device__ __forceinline__ void assemble_one(const SharedEnum& e, const MeshArgs& m, const T* __restrict__ part,
                                             int64_t stride, int64_t f, T v, T* __restrict__ y)
{
    int i, j, l;
    shared_node(e, f, i, j, l);
    if (is_dirichlet(m, i, j, l)) return;
    const int n = sharer_count(e, i, j, l);
    for (int c = 2; c < n; ++c) v += VPP_LD(&part[c * stride + f], BC_PART);
    VPP_ST(&y[i + (int64_t)m.nn[0] * (j + (int64_t)m.nn[1] * l)], BC_Y, v);
}

template <typename T>
__global__ void __launch_bounds__(256) assemble_kernel(AssembleArgs<T> a)
{
    VPP_BC_BEGIN((const T*)nullptr, a.y, (const T*)nullptr, a.part, a.dot_part, (const T*)nullptr,
                 (int64_t)a.m.nn[0] * a.m.nn[1] * a.m.nn[2], 8 * a.nshared, (int64_t)a.ndot, 0);
    if (a.done && *a.done) return;
    if (a.dot && blockIdx.x == 0) {
        // x . y from the per-workgroup partials, summed in a fixed order
        __shared__ double red[256];
        double s = 0.0;
        for (int i = threadIdx.x; i < a.ndot; i += 256) s += VPP_LD(&a.dot_part[i], BC_DOT);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *a.dot = red[0];
    }
    const SharedEnum& e = a.e;
    const int64_t count = e.cz + e.cy + e.cx;
    using P = typename Pair<T>::type;
    for (int64_t f = 2 * ((int64_t)blockIdx.x * 256 + threadIdx.x); f < count; f += 2 * (int64_t)gridDim.x * 256) {
        // positions and sharer counts of nodes f and f + 1 first (no memory),
        // then every partial of both nodes loaded before any is used
        int i0, j0, l0, i1 = 0, j1 = 0, l1 = 0;
        shared_node(e, f, i0, j0, l0);
        const bool has1 = f + 1 < count;
        if (has1) shared_node(e, f + 1, i1, j1, l1);
        const int n0 = is_dirichlet(a.m, i0, j0, l0) ? 0 : sharer_count(e, i0, j0, l0);
        const int n1 = !has1 || is_dirichlet(a.m, i1, j1, l1) ? 0 : sharer_count(e, i1, j1, l1);
        const P r0 = VPP_LD(reinterpret_cast<const P*>(a.part + f), BC_PART);
        const P r1 = VPP_LD(reinterpret_cast<const P*>(a.part + a.nshared + f), BC_PART);
        T x0[6], x1[6];
#pragma unroll
        for (int c = 2; c < 8; ++c) {
            x0[c - 2] = c < n0 ? VPP_LD(&a.part[c * a.nshared + f], BC_PART) : T(0);
            x1[c - 2] = c < n1 ? VPP_LD(&a.part[c * a.nshared + f + 1], BC_PART) : T(0);
        }
        T v0 = r0.x + r1.x, v1 = r0.y + r1.y;
#pragma unroll
        for (int c = 2; c < 8; ++c) {
            if (c < n0) v0 += x0[c - 2];
            if (c < n1) v1 += x1[c - 2];
        }
        if (n0 > 0) VPP_ST(&a.y[i0 + (int64_t)a.m.nn[0] * (j0 + (int64_t)a.m.nn[1] * l0)], BC_Y, v0);
        if (n1 > 0) VPP_ST(&a.y[i1 + (int64_t)a.m.nn[0] * (j1 + (int64_t)a.m.nn[1] * l1)], BC_Y, v1);
    }
}

template <typename T>
hipError_t launch_assemble(const AssembleArgs<T>& a, hipStream_t s)
{
    const int64_t want = (a.e.cz + a.e.cy + a.e.cx + 511) / 512;
    const int blocks = (int)(want < 1 ? 1 : (want < 8192 ? want : 8192));
    hipLaunchKernelGGL(assemble_kernel<T>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_assemble<double>(const AssembleArgs<double>&, hipStream_t);
template hipError_t launch_assemble<float>(const AssembleArgs<float>&, hipStream_t);

int device_cu_count()
{
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 1;
        cached = n;
    }
    return cached;
}

// ---------------------------------------------------------------------------
// Batched persistent apply: one launch over the (problem, tile) work items of
// several independent meshes.  Workgroups pull items from a device counter
// until the list is exhausted (every workgroup leaves the loop once the
// counter passes the item count).  The coefficient of a tile is computed once
// and reused for all right-hand sides of its problem.  A second launch
// assembles the shared-face nodes of every (problem, rhs) and resets the counter.

template <int K, int TX, int TY, int TZ, int HV, int DM>
__global__ void __launch_bounds__(TX * TY * TZ) batch_apply_kernel(BatchArgs a)
{
    constexpr int N = K + 1, N3 = N * N * N, NT = TX * TY * TZ, CS = NT + 1;
    // Q2: a work item is a (problem, tile) whose coefficient is computed once
    // for all right-hand sides of the problem.  Q3: a work item is a (problem,
    // tile, rhs), the items of one tile consecutive, and the coefficient is
    // recomputed per item (its 64 values held across a loop over right-hand
    // sides, beside the cell's 64, would not fit in the registers; the tile's
    // phi is still in the caches for the next item).  The x . Ax partials of
    // the batched PCG (DM & 1) and the mass shift (DM & 2) are template
    // choices, as in the single-problem kernel, which keeps the branches they
    // would add out of the register allocation.
    constexpr bool per_tile = K == 2;
    __shared__ double slot[N3 * CS];
    __shared__ int item_s;
    const int tid = threadIdx.x;
    for (int q = tid; q < N3; q += NT) slot[q * CS + NT] = 0.0;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    for (;;) {
        if (tid == 0) item_s = atomicAdd(a.queue, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= a.nitems) break;
        int pi = 0;
        for (int i = 1; i < a.nprob; ++i)
            if (a.probs[i].tile_begin <= item) pi = i;
        const MeshArgs m = a.probs[pi].m;
        const double* phi = a.probs[pi].phi;
        const int nrhs = a.probs[pi].nrhs, rhs0 = a.probs[pi].rhs_begin;
        const int local = item - a.probs[pi].tile_begin;
        const int tile = per_tile ? local : local / nrhs;   // the inverse of batch_items
        const TileCoord tc = tile_coord<K, TX, TY, TZ>(m, tile);
        const int cx = tc.t[0] * TX + lx, cy = tc.t[1] * TY + ly, cz = tc.t[2] * TZ + lz;
        const bool active = cx < m.nc[0] && cy < m.nc[1] && cz < m.nc[2];
        // gathers from a wave-uniform tile base plus the lane's cell offset
        const int nx = m.nn[0], nxy = m.nn[0] * m.nn[1];
        const int64_t tile0 = uniform_i64(node_index(m, tc.n0[0], tc.n0[1], tc.n0[2]));
        const unsigned lane_b = (unsigned)(K * lx + nx * K * ly + nxy * K * lz) * (unsigned)sizeof(double);
        const int faces = active ? cell_dirichlet_faces(m, cx, cy, cz) : 0;
        auto coefficient = [&](double (&w)[N3]) {
            gather_cell_t<K>(phi + tile0, lane_b, nx, nxy, 0, w);
            sweep3<K, MS, false, 0>(w);
            sweep3<K, MS, false, 1>(w);
            sweep3<K, MS, false, 2>(w);
            coef_weights3<K, HV>(m, w);
        };
        // one right-hand side r of this tile with the coefficient cw
        auto one_rhs = [&](int r, const double (&cw)[N3]) {
            const double* x = a.x[rhs0 + r];
            double* y = a.y[rhs0 + r];
            double* part = a.part + a.probs[pi].part_begin + (int64_t)r * 8 * a.probs[pi].nshared;
            VPP_BC_SYNC();
            VPP_BC_BEGIN(x, y, phi, part, a.dot_part ? a.dot_part + a.probs[pi].dot_begin : nullptr, slot,
                         (int64_t)m.nn[0] * m.nn[1] * m.nn[2], 8 * a.probs[pi].nshared,
                         (int64_t)nrhs * a.probs[pi].ntiles, N3 * CS);
            double u[N3];
            if (active) {
                gather_cell_t<K>(x + tile0, lane_b, nx, nxy, faces, u);
                cell_operator<K, double, (DM & 2) != 0>(m, cw, u);   // a zero shift adds exact zeros
            }
            __syncthreads();   // the previous write-out has finished reading the slots
            if (active) {
#pragma unroll
                for (int q = 0; q < N3; ++q)
                    if (!owned_pos<K>(q % N, (q / N) % N, q / (N * N))) VPP_ST(&slot[q * CS + tid], BC_SLOT, u[q]);
            }
            __syncthreads();
            constexpr bool dot = (DM & 1) != 0;
            const double d = flush_two_pass<K, double, TX, TY, TZ>(m, tc, slot, CS, u, active, lx, ly, lz, cx, cy,
                                                                   cz, x, y, part, a.probs[pi].nshared, dot);
            if (dot) {
                const double sum = block_sum<NT>(d);
                if (tid == 0) VPP_ST(&a.dot_part[a.probs[pi].dot_begin + r * a.probs[pi].ntiles + tile], BC_DOT, sum);
            }
        };
        if constexpr (per_tile) {
            // systems of a batched PCG that have stopped are skipped
            bool any = true;
            if (a.st) {
                any = false;
                for (int r = 0; r < nrhs; ++r) any = any || !a.st[rhs0 + r].halt[a.par];
            }
            // the bounds table of the debug build: this problem's phi (the
            // barrier first: the previous item's write-out may still read it)
            VPP_BC_SYNC();
            VPP_BC_BEGIN((const double*)nullptr, (const double*)nullptr, phi, (const double*)nullptr,
                         (const double*)nullptr, slot, (int64_t)m.nn[0] * m.nn[1] * m.nn[2], 0, 0, N3 * CS);
            double cw[N3];
            if (active && any) coefficient(cw);
            for (int r = 0; r < nrhs; ++r) {
                if (a.st && a.st[rhs0 + r].halt[a.par]) continue;   // uniform over the workgroup
                one_rhs(r, cw);
            }
        } else {
            const int r = local - tile * nrhs;
            if (a.st && a.st[rhs0 + r].halt[a.par]) continue;   // uniform over the workgroup
            VPP_BC_SYNC();
            VPP_BC_BEGIN((const double*)nullptr, (const double*)nullptr, phi, (const double*)nullptr,
                         (const double*)nullptr, slot, (int64_t)m.nn[0] * m.nn[1] * m.nn[2], 0, 0, N3 * CS);
            double cw[N3];
            if (active) coefficient(cw);
            one_rhs(r, cw);
        }
    }
}

struct BatchAssembleArgs {
    const BatchProblem* probs;
    int nprob;
    double* const* y;
    double* part;
    int* queue;
};

// grid.y = (problem, rhs) pair; grid.x strides over that pair's shared nodes.
__global__ void __launch_bounds__(256) batch_assemble_kernel(BatchAssembleArgs a)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.queue = 0;
    int pr = blockIdx.y, pi = 0;
    for (; pi < a.nprob; ++pi) {
        if (pr < a.probs[pi].nrhs) break;
        pr -= a.probs[pi].nrhs;
    }
    if (pi >= a.nprob) return;
    const BatchProblem& P = a.probs[pi];
    const int64_t ns = P.nshared;
    const double* part = a.part + P.part_begin + (int64_t)pr * 8 * ns;
    double* y = a.y[P.rhs_begin + pr];
    VPP_BC_BEGIN((const double*)nullptr, y, (const double*)nullptr, part, (const double*)nullptr,
                 (const double*)nullptr, (int64_t)P.m.nn[0] * P.m.nn[1] * P.m.nn[2], 8 * ns, 0, 0);
    const SharedEnum& e = P.se;
    const int64_t count = e.cz + e.cy + e.cx;
    for (int64_t f = 2 * ((int64_t)blockIdx.x * 256 + threadIdx.x); f < count; f += 2 * (int64_t)gridDim.x * 256) {
        const double2 r0 = VPP_LD(reinterpret_cast<const double2*>(part + f), BC_PART);
        const double2 r1 = VPP_LD(reinterpret_cast<const double2*>(part + ns + f), BC_PART);
        assemble_one(e, P.m, part, ns, f, r0.x + r1.x, y);
        if (f + 1 < count) assemble_one(e, P.m, part, ns, f + 1, r0.y + r1.y, y);
    }
}

#define VPP_BATCH_CONFIGS(X) \
    X(2, 16, 8, 4)           \
    X(2, 32, 4, 4)           \
    X(2, 8, 8, 4)            \
    X(2, 16, 4, 4)           \
    X(2, 8, 4, 4)            \
    X(3, 8, 4, 4)            \
    X(3, 4, 4, 4)

template <int K, int TX, int TY, int TZ, int HV>
static void launch_batch_tiles(const BatchArgs& a, int nblocks, hipStream_t s)
{
    const dim3 g(nblocks), blk(TX * TY * TZ);
    switch ((a.st ? 1 : 0) | (a.any_mass ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((batch_apply_kernel<K, TX, TY, TZ, HV, 0>), g, blk, 0, s, a); break;
    case 1: hipLaunchKernelGGL((batch_apply_kernel<K, TX, TY, TZ, HV, 1>), g, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL((batch_apply_kernel<K, TX, TY, TZ, HV, 2>), g, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((batch_apply_kernel<K, TX, TY, TZ, HV, 3>), g, blk, 0, s, a); break;
    }
}

hipError_t launch_batch_apply(const LaunchCfg& c, int k, const BatchArgs& a, int nblocks, int total_rhs,
                              bool tiles_only, hipStream_t s)
{
#define VPP_BL(K, TX, TY, TZ)                                                                       \
    if (k == K && c.variant == 4 && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) {       \
        if (a.heaviside == 0) launch_batch_tiles<K, TX, TY, TZ, 0>(a, nblocks, s);                  \
        else launch_batch_tiles<K, TX, TY, TZ, 1>(a, nblocks, s);                                   \
        hipError_t e = hipGetLastError();                                                           \
        if (e != hipSuccess || tiles_only) return e;                                                \
        BatchAssembleArgs b{a.probs, a.nprob, a.y, a.part, a.queue};                                \
        hipLaunchKernelGGL(batch_assemble_kernel, dim3(512, (unsigned)total_rhs), dim3(256), 0, s, b);  \
        return hipGetLastError();                                                                   \
    }
    VPP_BATCH_CONFIGS(VPP_BL)
#undef VPP_BL
    return hipErrorInvalidValue;
}

int list_batch_configs(int k, LaunchCfg* out, int cap)
{
    int n = 0;
#define VPP_BLIST(K, TX, TY, TZ)                                      \
    if (k == K) {                                                     \
        if (n < cap && out) out[n] = LaunchCfg{4, {TX, TY, TZ}};     \
        ++n;                                                          \
    }
    VPP_BATCH_CONFIGS(VPP_BLIST)
#undef VPP_BLIST
    return n;
}

int batch_blocks_per_cu(const LaunchCfg& c, int k)
{
    int nb = 0;
#define VPP_BO(K, TX, TY, TZ)                                                                      \
    if (k == K && c.variant == 4 && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) {      \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_apply_kernel<K, TX, TY, TZ, 0, 0>,\
                                                         TX * TY * TZ, 0) != hipSuccess)          \
            return 0;                                                                              \
        return nb;                                                                                 \
    }
    VPP_BATCH_CONFIGS(VPP_BO)
#undef VPP_BO
    return 0;
}

unsigned long long bounds_count_misc() { return bc_count_here(); }

}  // namespace vpp

// C ABI of the library (include/vpp.h): problem set-up, apply, diagonal,
// Jacobi PCG (FP64 and FP64/FP32 defect correction), adjoint, batches and the
// autotuner.  Host side only; the kernels live in the .hip files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <initializer_list>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/vpp.h"
#include "blas.h"
#include "tridiag.h"
#include "amr.h"
#include "kernels.h"
#include "noalloc.h"

using namespace vpp;

namespace {

thread_local std::string g_err;

vpp_status fail(vpp_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

// True if a non-null caller vector is not aligned to its element size (a
// caller's error: the kernels take whole elements).
bool misaligned(size_t elem, std::initializer_list<const void*> ptrs)
{
    for (const void* q : ptrs)
        if (q && reinterpret_cast<uintptr_t>(q) % elem != 0) return true;
    return false;
}
#define VPP_ALIGNED(elem, ...)                                                                  \
    do {                                                                                        \
        if (misaligned((elem), {__VA_ARGS__}))                                                  \
            return fail(VPP_ERR_INVALID_ARG, "vector not aligned to its element size");         \
    } while (0)

#define VPP_HIP(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(VPP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

LaunchCfg default_config(int k)
{
    if (k == 2) return LaunchCfg{4, {8, 8, 4}};
    if (k == 3) return LaunchCfg{1, {4, 4, 2}};
    return LaunchCfg{1, {4, 2, 2}};
}

template <typename T>
vpp_status dev_alloc(T** p, size_t n, const char* what)
{
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(VPP_ERR_OUT_OF_MEMORY, std::string("hipMalloc failed for ") + what);
    }
    return VPP_OK;
}

template <typename T>
void dev_free(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------

struct CgWork {
    // FP64 solver vectors
    double *x = nullptr, *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
    // FP32 inner solver vectors
    float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
    double* xb = nullptr;         // FP64 iterate kept across a mixed-precision phase
    CgState* st = nullptr;        // device
    CgState* st32 = nullptr;      // device
    CgState* hst = nullptr;       // pinned host mirror
    double* rr = nullptr;         // device scalar for residual norms
    double* red = nullptr;        // per-workgroup partial sums of the reductions
    double* hrr = nullptr;        // pinned host mirror
    hipGraphExec_t g64 = nullptr, g32 = nullptr;
    int graph_iters = 0;
    LaunchCfg graph_cfg{-1, {0, 0, 0}};
    LaunchCfg graph_cfg32{-1, {0, 0, 0}};
    // deflation of the mixed-precision solver (allocated on first use)
    float* hist = nullptr;        // FP32 residuals of the first phase: hist_cap rows of hist_stride
    int hist_cap = 0;
    int64_t hist_stride = 0;
    double* coef = nullptr;       // alpha, beta, r.z of every recorded iteration
    double* dW = nullptr;         // Ritz vectors, kMaxDefl x N
    double* dAW = nullptr;        // the operator applied to them
    double* dC = nullptr;         // their coefficients on the recorded residuals
    double* dred = nullptr;       // kMaxDefl x kMaxRedBlocks partial sums
    double* dout = nullptr;       // kMaxDefl dot products
    double* hout = nullptr;       // pinned host mirror of dout
};

// Workspace of the reinitialization step (allocated on first use).
struct ReinitWork {
    double *b = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *x = nullptr;
    double *diag = nullptr, *invd = nullptr, *red = nullptr, *dot = nullptr, *rr = nullptr, *hrr = nullptr;
    float* inv32 = nullptr;
    CgState* st = nullptr;
    CgState* hst = nullptr;
};

struct vpp_problem_s {
    vpp_desc desc;
    int k = 2;
    int64_t N = 0, NQ = 0, ncell = 0;
    MeshArgs m{};                   // FP64 apply (tile counts of cfg)
    LaunchCfg cfg{};
    MeshArgs m32{};                 // FP32 apply (tile counts of cfg32)
    LaunchCfg cfg32{};
    double* phi64 = nullptr;
    float* phi32 = nullptr;
    double* diag = nullptr;
    double* inv64 = nullptr;
    float* inv32 = nullptr;
    double* part = nullptr;         // shared-face partials of the apply (sized for cfg)
    size_t part_bytes = 0;
    double* dot_part = nullptr;     // per-workgroup partial dot products
    size_t dot_part_n = 0;
    double* cellbuf = nullptr;      // cell-major scratch of the node-sum kernels
    size_t cellbuf_n = 0;
    hipEvent_t cell_evt = nullptr;  // last use of cellbuf (orders users on different streams)
    bool phi_set = false;
    hipStream_t stream = nullptr;   // library stream for solves and graph capture
    CgWork w;
    int* cp_list = nullptr;         // band nodes of the closest-point projection (N)
    int* cp_ctr = nullptr;          // its band count and queue head (2)
    ReinitWork* rw = nullptr;       // reinitialization step
};

static void free_reinit(ReinitWork* w)
{
    if (!w) return;
    dev_free(w->b); dev_free(w->r); dev_free(w->p); dev_free(w->q); dev_free(w->x);
    dev_free(w->diag); dev_free(w->invd); dev_free(w->red); dev_free(w->dot); dev_free(w->rr);
    dev_free(w->inv32); dev_free(w->st);
    if (w->hst) (void)hipHostFree(w->hst);
    if (w->hrr) (void)hipHostFree(w->hrr);
    delete w;
}

struct vpp_batch_s {
    std::vector<vpp_problem> probs;
    std::vector<int> nrhs;
    int k = 2;
    int total_rhs = 0;
    int nitems = 0;
    int64_t total_dofs = 0;
    LaunchCfg cfg{};
    int nblocks = 0;
    BatchProblem* d_probs = nullptr;
    double** d_x = nullptr;
    double** d_y = nullptr;
    double* d_part = nullptr;
    size_t part_n = 0;
    int* d_queue = nullptr;
    std::vector<const double*> cur_x;
    std::vector<double*> cur_y;
    hipGraphExec_t graph = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<BatchProblem> tab;     // host copy of d_probs
    // batched FP64 PCG workspace (set up by the first batched solve): one system
    // per (problem, rhs), its vectors at offsets cg_off in cg_x/r/p/q
    std::vector<int> cg_prob;          // problems whose systems advance in lockstep
    std::vector<int> cg_index;         // system (problem-major) -> lockstep system, -1 if solved alone
    BatchProblem* cg_probs = nullptr;  // device table of the lockstep problems
    int cg_nitems = 0, cg_nblocks = 0, cg_nsys = 0;
    std::vector<int64_t> cg_off;
    double *cg_x = nullptr, *cg_r = nullptr, *cg_p = nullptr, *cg_q = nullptr;
    double** cg_tx = nullptr;          // device pointer tables of x, p, q per system
    double** cg_tp = nullptr;
    double** cg_tq = nullptr;
    CgState* cg_st = nullptr;          // device, one per system
    CgState* cg_hst = nullptr;         // pinned mirror
    double* cg_red = nullptr;          // kRedDoubles per system
    double* cg_dot = nullptr;          // per-tile partials of p.Ap of every system
    double* cg_rr = nullptr;           // device, one residual norm per system
    double* cg_hrr = nullptr;          // pinned mirror
    CgSystem<double>* cg_sys = nullptr;
    int cg_blocks = 0;                 // workgroups of the batched vector launches
    hipGraphExec_t cg_graph = nullptr;
    int cg_graph_iters = 0;
};

static void set_tiles(MeshArgs& m, const LaunchCfg& c)
{
    for (int d = 0; d < 3; ++d) m.ntile[d] = (m.nc[d] + c.tile[d] - 1) / c.tile[d];
}

static int tile_count(const MeshArgs& m) { return m.ntile[0] * m.ntile[1] * m.ntile[2]; }

static MeshArgs make_mesh_args(const vpp_desc& d)
{
    MeshArgs m{};
    const int k = d.degree;
    double h[3];
    for (int i = 0; i < 3; ++i) {
        m.nc[i] = d.ncells[i];
        m.nn[i] = k * d.ncells[i] + 1;
        h[i] = d.extent[i] / d.ncells[i];
    }
    m.bcmask = 0;
    for (int f = 0; f < 6; ++f)
        if (d.bc[f] == VPP_BC_DIRICHLET) m.bcmask |= 1 << f;
    m.heaviside = d.heaviside;
    // W_q h_d^-2 = wref_q hx hy hz / h_d^2 = wref_q r0 rd[d]
    m.r0 = h[1] * h[2] / h[0];
    m.rd[0] = 1.0;
    m.rd[1] = (h[0] * h[0]) / (h[1] * h[1]);
    m.rd[2] = (h[0] * h[0]) / (h[2] * h[2]);
    const double il = 1.0 / d.rho_l, ig = 1.0 / d.rho_g;
    // linear H = (phi+1)/2:  c = ig + (il - ig)(phi+1)/2
    m.ca = m.r0 * (ig + 0.5 * (il - ig));
    m.cb = m.r0 * 0.5 * (il - ig);
    // sine ramp:  c = ig + (il - ig) H
    m.cg = m.r0 * ig;
    m.cd = m.r0 * (il - ig);
    // arithmetic density mean: rho = rho_g + (rho_l - rho_g) H, c' = r0 / rho
    m.qa = (d.rho_g + 0.5 * (d.rho_l - d.rho_g)) / m.r0;
    m.qb = 0.5 * (d.rho_l - d.rho_g) / m.r0;
    m.qs = d.rho_g / m.r0;
    m.qd = (d.rho_l - d.rho_g) / m.r0;
    m.dcdphi = il - ig;
    m.rho_l = d.rho_l;
    m.rho_g = d.rho_g;
    return m;
}

// Scratch of the apply for the current configurations of both precisions: the
// partials of shared-face nodes (8 ranks x shared nodes, FP64-sized) and one
// partial dot product per tile.
// Cell-major scratch of the kernels that sum per-cell contributions into the
// nodes (dJ/dphi, the filter right-hand sides, the reinitialization pieces):
// nvec arrays of cell_values entries.  The calls using it are ordered by an
// event, also when they run on different streams.
static vpp_status cell_scratch_begin(vpp_problem p, int nvec, hipStream_t s, double** out)
{
    const size_t need = (size_t)nvec * (size_t)cell_values(p->k, p->m);
    if (need > p->cellbuf_n) {
        if (p->cellbuf) {
            VPP_HIP(hipDeviceSynchronize());   // a previous call may still read it
            dev_free(p->cellbuf);
        }
        p->cellbuf = nullptr;
        p->cellbuf_n = 0;
        vpp_status st = dev_alloc(&p->cellbuf, need, "cell scratch");
        if (st) return st;
        p->cellbuf_n = need;
    }
    if (!p->cell_evt) VPP_HIP(hipEventCreateWithFlags(&p->cell_evt, hipEventDisableTiming));
    else VPP_HIP(hipStreamWaitEvent(s, p->cell_evt, 0));
    *out = p->cellbuf;
    return VPP_OK;
}

static vpp_status cell_scratch_end(vpp_problem p, hipStream_t s)
{
    VPP_HIP(hipEventRecord(p->cell_evt, s));
    return VPP_OK;
}

static vpp_status ensure_apply_scratch(vpp_problem p)
{
    const int64_t ns = std::max(shared_stride(p->m), shared_stride(p->m32));
    if (8 * ns >= (int64_t(1) << 32))
        return fail(VPP_ERR_UNSUPPORTED, "mesh too large for 32-bit partial indices with this tile configuration");
    const size_t need = (size_t)std::max<int64_t>(1, 8 * ns) * sizeof(double);
    if (need > p->part_bytes) {
        if (p->part) (void)hipFree(p->part);
        p->part = nullptr;
        p->part_bytes = 0;
        vpp_status s = dev_alloc(&p->part, need / sizeof(double), "apply partials");
        if (s) return s;
        p->part_bytes = need;
    }
    const size_t nd = (size_t)std::max(tile_count(p->m), tile_count(p->m32));
    if (nd > p->dot_part_n) {
        if (p->dot_part) (void)hipFree(p->dot_part);
        p->dot_part = nullptr;
        p->dot_part_n = 0;
        vpp_status s = dev_alloc(&p->dot_part, nd, "dot partials");
        if (s) return s;
        p->dot_part_n = nd;
    }
    return VPP_OK;
}

// y = A x on `s`; with `dot`, also x . y (written by the assembly kernel).
// Diagonal of A_D for the current phi and mass shift, and its inverses.
static vpp_status build_diagonal(vpp_problem p, hipStream_t s)
{
    VPP_HIP(launch_fill<double>(p->diag, p->N, 0.0, s));
    VPP_HIP(launch_diag(p->k, p->m, p->phi64, p->diag, s));
    VPP_HIP(launch_fix_diagonal(p->m, p->diag, p->inv64, p->inv32, s));
    return VPP_OK;
}

static void put_config(vpp_problem p, int prec, const LaunchCfg& c);

static bool arith_law(const vpp_desc& d) { return d.heaviside >= VPP_H_LINEAR_ARITH; }

// Configurations a problem may run: those instantiated with the arithmetic
// density mean or with the mass shift when it has one, else every
// configuration of its degree.
static bool config_ok(vpp_problem p, const LaunchCfg& c)
{
    if (arith_law(p->desc)) return arith_config_supported(c, p->k);
    return p->m.mass != 0.0 ? mass_config_supported(c, p->k) : apply_config_supported(c, p->k);
}

static int config_list(vpp_problem p, LaunchCfg* out, int cap)
{
    if (arith_law(p->desc)) return list_arith_configs(p->k, out, cap);
    return p->m.mass != 0.0 ? list_mass_configs(p->k, out, cap) : list_apply_configs(p->k, out, cap);
}

static vpp_status do_apply64(vpp_problem p, const double* x, double* y, double* dot, const int* done, hipStream_t s)
{
    ApplyArgs<double> a{p->m, x, y, p->phi64, p->part, shared_stride(p->m), dot ? p->dot_part : nullptr, dot,
                        done};
    VPP_HIP(launch_apply_f64(p->cfg, p->k, a, s));
    return VPP_OK;
}

static vpp_status do_apply32(vpp_problem p, const float* x, float* y, double* dot, const int* done, hipStream_t s)
{
    ApplyArgs<float> a{p->m32, x, y, p->phi32, reinterpret_cast<float*>(p->part), shared_stride(p->m32),
                       dot ? p->dot_part : nullptr, dot, done};
    VPP_HIP(launch_apply_f32(p->cfg32, p->k, a, s));
    return VPP_OK;
}

static void free_graphs(CgWork& w)
{
    if (w.g64) (void)hipGraphExecDestroy(w.g64);
    if (w.g32) (void)hipGraphExecDestroy(w.g32);
    w.g64 = w.g32 = nullptr;
}

static void free_work(CgWork& w)
{
    free_graphs(w);
    dev_free(w.x); dev_free(w.b); dev_free(w.r); dev_free(w.p); dev_free(w.q);
    dev_free(w.x32); dev_free(w.r32); dev_free(w.p32); dev_free(w.q32); dev_free(w.xb);
    dev_free(w.st); dev_free(w.st32); dev_free(w.rr); dev_free(w.red);
    dev_free(w.hist); dev_free(w.coef); dev_free(w.dW); dev_free(w.dAW); dev_free(w.dC); dev_free(w.dred);
    dev_free(w.dout);
    w.hist_cap = 0;
    if (w.hst) (void)hipHostFree(w.hst);
    if (w.hrr) (void)hipHostFree(w.hrr);
    if (w.hout) (void)hipHostFree(w.hout);
    w.hst = nullptr;
    w.hrr = nullptr;
    w.hout = nullptr;
}

static vpp_status ensure_work(vpp_problem p, bool mixed)
{
    CgWork& w = p->w;
    vpp_status s;
    const size_t n = (size_t)p->N;
    if (!w.x) {
        if ((s = dev_alloc(&w.x, n, "cg x")) || (s = dev_alloc(&w.b, n, "cg b")) ||
            (s = dev_alloc(&w.r, n, "cg r")) || (s = dev_alloc(&w.p, n, "cg p")) ||
            (s = dev_alloc(&w.q, n, "cg q")) || (s = dev_alloc(&w.st, 1, "cg state")) ||
            (s = dev_alloc(&w.st32, 1, "cg state")) || (s = dev_alloc(&w.rr, 1, "norm")) ||
            (s = dev_alloc(&w.red, kRedDoubles, "reduction partials")))
            return s;
        VPP_HIP(hipHostMalloc((void**)&w.hst, sizeof(CgState), hipHostMallocDefault));
        VPP_HIP(hipHostMalloc((void**)&w.hrr, sizeof(double), hipHostMallocDefault));
    }
    if (mixed && !w.x32) {
        if ((s = dev_alloc(&w.x32, n, "cg x32")) || (s = dev_alloc(&w.r32, n, "cg r32")) ||
            (s = dev_alloc(&w.p32, n, "cg p32")) || (s = dev_alloc(&w.q32, n, "cg q32")) ||
            (s = dev_alloc(&w.xb, n, "cg x kept")))
            return s;
    }
    return VPP_OK;
}

// Record `iters` (even) PCG iterations on the library stream into a graph.
template <typename T>
static vpp_status build_cg_graph(vpp_problem p, int iters, hipGraphExec_t* out)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    hipGraph_t g = nullptr;
    VPP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int it = 0; it < iters && err == hipSuccess; ++it) {
        const int par = it & 1;
        // tile kernel of q = A p (with p.q partials), then the update that also
        // assembles the shared nodes of q, then the search-direction update
        if constexpr (sizeof(T) == 8) {
            const int64_t stride = shared_stride(p->m);
            ApplyArgs<double> a{p->m, w.p, w.q, p->phi64, p->part, stride, p->dot_part, nullptr, &w.st->halt[par],
                                true};
            err = launch_apply_f64(p->cfg, p->k, a, s);
            if (err == hipSuccess)
                err = launch_cg_assemble_update<double>(w.st, par, w.red, p->dot_part, tile_count(p->m), p->m,
                                                        shared_enum(p->m, p->k, p->cfg.tile), p->part, stride,
                                                        w.r, w.q, p->inv64, p->N, s);
            if (err == hipSuccess)
                err = launch_cg_pupdate<double>(w.st, par, w.red, w.x, w.r, w.p, p->inv64, p->N, s);
        } else {
            const int64_t stride = shared_stride(p->m32);
            const float* part = reinterpret_cast<float*>(p->part);
            ApplyArgs<float> a{p->m32, w.p32, w.q32, p->phi32, reinterpret_cast<float*>(p->part), stride,
                               p->dot_part, nullptr, &w.st32->halt[par], true};
            err = launch_apply_f32(p->cfg32, p->k, a, s);
            if (err == hipSuccess)
                err = launch_cg_assemble_update<float>(w.st32, par, w.red, p->dot_part, tile_count(p->m32), p->m32,
                                                       shared_enum(p->m32, p->k, p->cfg32.tile), part, stride,
                                                       w.r32, w.q32, p->inv32, p->N, s);
            if (err == hipSuccess)
                err = launch_cg_pupdate<float>(w.st32, par, w.red, w.x32, w.r32, w.p32, p->inv32, p->N, s);
        }
    }
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(VPP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(err));
    }
    VPP_HIP(e2);
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    VPP_HIP(e3);
    *out = ex;
    return VPP_OK;
}

static bool same_cfg(const LaunchCfg& a, const LaunchCfg& b)
{
    return a.variant == b.variant && a.tile[0] == b.tile[0] && a.tile[1] == b.tile[1] && a.tile[2] == b.tile[2];
}

static vpp_status ensure_graphs(vpp_problem p, int iters, bool mixed)
{
    CgWork& w = p->w;
    if (w.graph_iters != iters || !same_cfg(w.graph_cfg, p->cfg) || !same_cfg(w.graph_cfg32, p->cfg32)) {
        free_graphs(w);
        w.graph_iters = iters;
        w.graph_cfg = p->cfg;
        w.graph_cfg32 = p->cfg32;
    }
    vpp_status s;
    if (!w.g64 && (s = build_cg_graph<double>(p, iters, &w.g64))) return s;
    if (mixed && !w.g32 && (s = build_cg_graph<float>(p, iters, &w.g32))) return s;
    return VPP_OK;
}

// Run graph chunks until the device sets a stop flag; returns the final state in *hs.
static vpp_status run_until_done(vpp_problem p, hipGraphExec_t g, CgState* st, CgState* hs, int max_iter)
{
    hipStream_t s = p->stream;
    const int chunk = p->w.graph_iters;
    const int max_launch = max_iter / chunk + 2;
    for (int l = 0; l < max_launch; ++l) {
        VPP_HIP(hipGraphLaunch(g, s));
        VPP_HIP(hipMemcpyAsync(hs, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        VPP_HIP(hipStreamSynchronize(s));
        if (hs->halt[0] || hs->halt[1]) break;
    }
    return VPP_OK;
}

// FP64 PCG on the workspace vectors (w.b, w.x in; w.x out).
static vpp_status pcg64(vpp_problem p, const vpp_cg_opts& o, vpp_cg_info& info, double* r0_out)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    vpp_status st;
    if ((st = do_apply64(p, w.x, w.q, nullptr, nullptr, s))) return st;
    CgState* hs = w.hst;
    std::memset(hs, 0, sizeof(CgState));
    VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
    VPP_HIP(launch_cg_init<double>(w.st, w.red, w.b, w.q, w.r, w.p, p->inv64, p->N, s));
    VPP_HIP(hipMemcpyAsync(hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    const double rr0 = hs->rr_last, rz0 = hs->rz[0];
    const double r0 = std::sqrt(rr0);
    *r0_out = r0;
    info.iterations = 0;
    info.rel_residual = r0 > 0 ? 1.0 : 0.0;
    if (!std::isfinite(rr0) || !std::isfinite(rz0)) {
        info.status = VPP_ERR_BREAKDOWN;
        return VPP_OK;
    }
    const double thr = std::max(o.rtol * r0, o.atol);
    if (r0 == 0.0 || r0 < o.atol) {
        info.status = VPP_OK;
        return VPP_OK;
    }
    CgState init{};
    init.rz[0] = rz0;
    init.tol2 = thr * thr;
    init.max_iter = o.max_iter;
    *hs = init;
    VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
    if ((st = run_until_done(p, w.g64, w.st, hs, o.max_iter))) return st;
    info.iterations = hs->iters;
    info.rel_residual = std::sqrt(hs->rr_last) / r0;
    if (hs->breakdown) info.status = VPP_ERR_BREAKDOWN;
    else if (hs->rr_last < init.tol2) info.status = VPP_OK;
    else info.status = VPP_ERR_NOT_CONVERGED;
    return VPP_OK;
}

// ||b - A x||^2 in FP64 on the workspace (r := b - A x).
static vpp_status residual64(vpp_problem p, double* rr)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    vpp_status st;
    if ((st = do_apply64(p, w.x, w.q, nullptr, nullptr, s))) return st;
    VPP_HIP(launch_residual(w.b, w.q, w.r, p->N, w.red, w.rr, s));
    VPP_HIP(hipMemcpyAsync(w.hrr, w.rr, sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    *rr = *w.hrr;
    return VPP_OK;
}

// ---------------------------------------------------------------------------
// Deflation of the mixed-precision solver.  FP32 PCG follows FP64 PCG
// iteration for iteration until its true residual stalls (near 1e-3 of the
// scaled residual at 64^3 and density ratio 1000), but every replacement of
// the residual puts FP32-sized perturbations back into the eigenvectors of the
// smallest eigenvalues, which the FP64 recurrence would have left resolved:
// the later phases then converge at the unaccelerated rate.  The first FP32
// phase is a Lanczos process: its CG coefficients define the tridiagonal
// matrix T of D^-1/2 A D^-1/2 on the basis v_j = D^-1/2 r_j / sqrt(r_j.z_j),
// whose smallest eigenpairs (theta, s) give Ritz vectors w = D^-1 sum_j s_j
// r_j / sqrt(r_j.z_j) in the original variables.  Only Ritz values followed by
// a gap (the next one at least 10 times larger) are used: an isolated
// near-null mode is resolved accurately by the FP32 Lanczos process, a cluster
// is not, and deflating part of one slows the later phases down.  At every
// replacement the FP64 iterate gets the Galerkin correction in span(W): x += W G^-1 W^T r,
// r -= A W G^-1 W^T r with G = W^T A W (a pivoted Cholesky factor that drops
// dependent columns).  A correction that would move r by more than a tenth of
// ||r|| (||A W c||, from the Gram matrix of A W) is not applied: the kept
// search direction would no longer fit the residual.  Converged Ritz vectors
// of the smallest eigenvalues move r very little (their eigenvalues are
// small); if the first correction is refused, the solve continues without
// deflation.

struct Defl {
    int k = 0;                     // Ritz vectors in W (0: off)
    int nk = 0;                    // columns kept by the pivoted factorization
    int perm[kMaxDefl] = {};
    double L[kMaxDefl][kMaxDefl] = {};
    double H[kMaxDefl][kMaxDefl] = {};   // (A W)^T (A W): ||A W c|| without a pass over the vectors
    bool accepted = false;
};

static vpp_status ensure_defl(vpp_problem p, int cap, int* got)
{
    CgWork& w = p->w;
    const int64_t stride = ((p->N + 63) / 64) * 64;
    if (w.hist && w.hist_stride == stride && w.hist_cap >= cap) {
        *got = cap;
        return VPP_OK;
    }
    dev_free(w.hist);
    dev_free(w.coef);
    w.hist_cap = 0;
    size_t fr = 0, tot = 0;
    VPP_HIP(hipMemGetInfo(&fr, &tot));
    // at most a quarter of the free device memory for the record
    const int64_t fit = (int64_t)(fr / 4 / ((size_t)stride * sizeof(float)));
    cap = (int)std::min<int64_t>(cap, fit);
    *got = 0;
    if (cap < 16) return VPP_OK;
    vpp_status st;
    const size_t n = (size_t)p->N;
    if ((st = dev_alloc(&w.hist, (size_t)cap * (size_t)stride, "deflation record")) ||
        (st = dev_alloc(&w.coef, 3 * (size_t)cap + 3, "deflation coefficients")))
        return st;
    if (!w.dW && ((st = dev_alloc(&w.dW, kMaxDefl * n, "Ritz vectors")) ||
                  (st = dev_alloc(&w.dAW, kMaxDefl * n, "Ritz images")) ||
                  (st = dev_alloc(&w.dred, (size_t)kMaxDefl * kMaxRedBlocks, "deflation partials")) ||
                  (st = dev_alloc(&w.dout, kMaxDefl, "deflation dots"))))
        return st;
    if (!w.hout) VPP_HIP(hipHostMalloc((void**)&w.hout, kMaxDefl * sizeof(double), hipHostMallocDefault));
    dev_free(w.dC);
    if ((st = dev_alloc(&w.dC, (size_t)cap * kMaxDefl, "Ritz coefficients"))) return st;
    w.hist_cap = cap;
    w.hist_stride = stride;
    *got = cap;
    return VPP_OK;
}

// out[t] = V[t] . y for t < k, on the host.
static vpp_status multi_dot_host(vpp_problem p, const double* V, int k, const double* y, double* out)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    VPP_HIP(launch_multi_dot(V, k, y, p->N, w.dred, w.dout, s));
    VPP_HIP(hipMemcpyAsync(w.hout, w.dout, k * sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    for (int t = 0; t < k; ++t) out[t] = w.hout[t];
    return VPP_OK;
}

// Ritz vectors of the first FP32 phase (m recorded iterations, m below the
// record's length) and the factor of G.
static vpp_status build_defl(vpp_problem p, int kreq, int m, Defl& df)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    df = Defl{};
    if (m < 2 || kreq < 1) return VPP_OK;
    std::vector<double> cf(3 * (size_t)(m + 1));
    VPP_HIP(hipMemcpyAsync(cf.data(), w.coef, cf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    std::vector<double> d(m), e(m), rz(m);
    for (int j = 0; j < m; ++j) {
        const double al = cf[3 * (j + 1)], be = cf[3 * (j + 1) + 1];
        rz[j] = cf[3 * j + 2];
        if (!(al > 0.0) || !(be >= 0.0) || !(rz[j] > 0.0) || !std::isfinite(al) || !std::isfinite(be) ||
            !std::isfinite(rz[j]))
            return VPP_OK;
        d[j] = 1.0 / al + (j > 0 ? cf[3 * j + 1] / cf[3 * j] : 0.0);
        e[j] = -std::sqrt(be) / al;
    }
    // Ritz values of the first phase: deflate the smallest ones only where a gap
    // of 10 follows them (isolated near-null modes, such as the nearly constant
    // pressure of a gas bubble); a cluster without a gap is left alone
    const int kmax = std::min(std::min(kreq, (int)kMaxDefl), m - 1);
    if (kmax < 1) return VPP_OK;
    std::vector<double> vals(kmax + 1);
    if (tridiag_smallest_values(m, d.data(), e.data(), kmax + 1, vals.data()) != kmax + 1) return VPP_OK;
    int k = 0;
    for (int i = 1; i <= kmax; ++i)
        if (vals[i - 1] > 0.0 && vals[i] >= 10.0 * vals[i - 1]) k = i;
    if (k == 0) return VPP_OK;
    std::vector<double> vecs((size_t)k * m), C((size_t)m * k);
    tridiag_vectors(m, d.data(), e.data(), k, vals.data(), vecs.data());
    for (int j = 0; j < m; ++j)
        for (int t = 0; t < k; ++t) C[(size_t)j * k + t] = vecs[(size_t)t * m + j] / std::sqrt(rz[j]);
    VPP_HIP(hipMemcpyAsync(w.dC, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
    VPP_HIP(hipStreamSynchronize(s));
    VPP_HIP(launch_ritz(w.hist, w.hist_stride, m, w.dC, k, p->inv64, w.dW, p->N, s));
    vpp_status st;
    for (int t = 0; t < k; ++t)
        if ((st = do_apply64(p, w.dW + (size_t)t * p->N, w.dAW + (size_t)t * p->N, nullptr, nullptr, s))) return st;
    double G[kMaxDefl][kMaxDefl];
    for (int t = 0; t < k; ++t) {
        double col[kMaxDefl];
        if ((st = multi_dot_host(p, w.dW, k, w.dAW + (size_t)t * p->N, col))) return st;
        for (int u = 0; u < k; ++u) G[u][t] = col[u];
    }
    for (int u = 0; u < k; ++u)
        for (int t = u + 1; t < k; ++t) G[u][t] = G[t][u] = 0.5 * (G[u][t] + G[t][u]);
    // pivoted Cholesky G(perm, perm) = L L^T, stopping at pivots below 1e-12 of the largest diagonal
    double gmax = 0.0;
    for (int t = 0; t < k; ++t) gmax = std::max(gmax, G[t][t]);
    if (!(gmax > 0.0) || !std::isfinite(gmax)) return VPP_OK;
    int idx[kMaxDefl];
    for (int t = 0; t < k; ++t) idx[t] = t;
    double S[kMaxDefl][kMaxDefl];
    for (int u = 0; u < k; ++u)
        for (int t = 0; t < k; ++t) S[u][t] = G[u][t];
    int nk = 0;
    for (; nk < k; ++nk) {
        int best = nk;
        for (int t = nk + 1; t < k; ++t)
            if (S[idx[t]][idx[t]] > S[idx[best]][idx[best]]) best = t;
        std::swap(idx[nk], idx[best]);
        const double piv = S[idx[nk]][idx[nk]];
        if (!(piv > 1e-12 * gmax) || !std::isfinite(piv)) break;
        const double lkk = std::sqrt(piv);
        df.L[nk][nk] = lkk;
        for (int t = nk + 1; t < k; ++t) df.L[t][nk] = S[idx[t]][idx[nk]] / lkk;
        for (int t = nk + 1; t < k; ++t)
            for (int u = nk + 1; u < k; ++u) S[idx[t]][idx[u]] -= df.L[t][nk] * df.L[u][nk];
    }
    if (nk == 0) return VPP_OK;
    for (int t = 0; t < k; ++t) {
        double col[kMaxDefl];
        if ((st = multi_dot_host(p, w.dAW, k, w.dAW + (size_t)t * p->N, col))) return st;
        for (int u = 0; u < k; ++u) df.H[u][t] = col[u];
    }
    df.k = k;
    df.nk = nk;
    for (int t = 0; t < k; ++t) df.perm[t] = idx[t];
    return VPP_OK;
}

// Coefficients of the Galerkin correction of the residual w.r in span(W).
static vpp_status defl_coef(vpp_problem p, const Defl& df, DeflCoef* c)
{
    vpp_status st;
    double dots[kMaxDefl];
    if ((st = multi_dot_host(p, p->w.dW, df.k, p->w.r, dots))) return st;
    double y[kMaxDefl];
    for (int i = 0; i < df.nk; ++i) {
        double v = dots[df.perm[i]];
        for (int j = 0; j < i; ++j) v -= df.L[i][j] * y[j];
        y[i] = v / df.L[i][i];
    }
    for (int i = df.nk - 1; i >= 0; --i) {
        double v = y[i];
        for (int j = i + 1; j < df.nk; ++j) v -= df.L[j][i] * y[j];
        y[i] = v / df.L[i][i];
    }
    *c = DeflCoef{};
    for (int i = 0; i < df.nk; ++i) c->c[df.perm[i]] = y[i];
    return VPP_OK;
}

// w.x += W c, w.r -= A W c; *rn = ||w.r|| afterwards.
static vpp_status defl_update(vpp_problem p, const Defl& df, const DeflCoef& c, double* rn)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    VPP_HIP(launch_defl_update(w.x, w.r, w.dW, w.dAW, c, df.k, p->N, w.red, w.rr, s));
    VPP_HIP(hipMemcpyAsync(w.hrr, w.rr, sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    *rn = std::sqrt(*w.hrr);
    return VPP_OK;
}

// Mixed precision PCG with reliable updates.  The Jacobi-PCG recurrences run
// in FP32 (operator, vectors) with FP64 scalars on a residual scaled to unit
// norm; whenever the scaled FP32 residual has dropped by inner_rtol since the
// last replacement, the FP32 correction is added to the FP64 solution, the
// true residual b - A x is recomputed with the FP64 operator, and it replaces
// the FP32 residual (rescaled) while the search direction is kept, so the
// Krylov recurrence continues instead of restarting.  Convergence is decided
// on the FP64 residual only.
static vpp_status pcg_mixed(vpp_problem p, const vpp_cg_opts& o, vpp_cg_info& info, double* r0_out)
{
    CgWork& w = p->w;
    hipStream_t s = p->stream;
    vpp_status st;
    double rr;
    if ((st = residual64(p, &rr))) return st;
    const double r0 = std::sqrt(rr);
    *r0_out = r0;
    info.iterations = 0;
    info.outer_iterations = 0;
    info.rel_residual = r0 > 0 ? 1.0 : 0.0;
    info.status = VPP_OK;
    info.deflation_corrections = 0;
    info.deflation_first_change = -1.0;
    if (!std::isfinite(rr)) {
        info.status = VPP_ERR_BREAKDOWN;
        return VPP_OK;
    }
    const double thr = std::max(o.rtol * r0, o.atol);
    if (!(r0 >= thr) || r0 == 0.0) return VPP_OK;
    const double delta = o.inner_rtol > 0 ? o.inner_rtol : 1e-2;
    CgState* hs = w.hst;
    // deflation: record the first FP32 phase (its residuals and CG coefficients)
    const int kdef = std::min(std::max(o.deflate, 0), (int)kMaxDefl);
    int rec_cap = 0;
    if (kdef > 0 && (st = ensure_defl(p, o.deflate_history > 0 ? std::min(o.deflate_history, 4096) : 512, &rec_cap)))
        return st;
    std::memset(hs, 0, sizeof(CgState));
    hs->tol2 = delta * delta;   // the replaced residual has unit norm
    hs->max_iter = o.max_iter;
    if (rec_cap > 0) {
        hs->hist = w.hist;
        hs->coef = w.coef;
        hs->hist_stride = w.hist_stride;
        hs->hist_cap = rec_cap;
    }
    VPP_HIP(hipMemcpyAsync(w.st32, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
    double rn = r0;
    VPP_HIP(launch_cg_replace32(w.st32, w.red, w.r, 1.0 / rn, 0.0, w.r32, w.p32, w.x32, p->inv32, p->N, s));
    if (rec_cap > 0) {
        // r_0 and r_0.z_0 of the record (the later ones come from the CG kernels)
        VPP_HIP(hipMemcpyAsync(w.hist, w.r32, p->N * sizeof(float), hipMemcpyDeviceToDevice, s));
        VPP_HIP(hipMemcpyAsync(w.coef + 2, &w.st32->rz[0], sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    Defl df;
    const int max_phases = 10000;
    int last_iters = 0, bad_phases = 0;
    while (true) {
        // per-phase iteration cap (inner_max_iter), within the overall max_iter
        int cap = o.max_iter;
        if (o.inner_max_iter > 0) cap = (int)std::min<int64_t>(cap, (int64_t)last_iters + o.inner_max_iter);
        hs->max_iter = cap;
        VPP_HIP(hipMemcpyAsync(&w.st32->max_iter, &hs->max_iter, sizeof(int), hipMemcpyHostToDevice, s));
        if ((st = run_until_done(p, w.g32, w.st32, hs, o.max_iter))) return st;
        const bool first_phase = info.outer_iterations == 0;
        if (first_phase && rec_cap > 0) {
            // the record covers the first phase only
            hs->hist_cap = 0;
            VPP_HIP(hipMemcpyAsync(&w.st32->hist_cap, &hs->hist_cap, sizeof(int), hipMemcpyHostToDevice, s));
        }
        last_iters = hs->iters;
        const bool broke = hs->breakdown != 0;
        // apply the phase's correction, keeping the previous iterate
        VPP_HIP(hipMemcpyAsync(w.xb, w.x, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
        VPP_HIP(launch_promote_add(w.x, w.x32, rn, p->N, s));
        if ((st = residual64(p, &rr))) return st;
        double rn_new = std::sqrt(rr);
        if (first_phase && rec_cap > 0 && !broke && rn_new < rn && rn_new >= thr && std::isfinite(rn_new))
            if ((st = build_defl(p, kdef, std::min(hs->iters, rec_cap - 1), df))) return st;
        if (df.k > 0 && rn_new >= thr) {
            DeflCoef c;
            if ((st = defl_coef(p, df, &c))) return st;
            double dr2 = 0.0;
            for (int u = 0; u < df.k; ++u)
                for (int t = 0; t < df.k; ++t) dr2 += c.c[u] * df.H[u][t] * c.c[t];
            const double change = std::sqrt(std::max(dr2, 0.0)) / rn_new;
            if (info.deflation_first_change < 0.0) info.deflation_first_change = change;
            if (std::isfinite(dr2) && change <= 0.1) {
                double rn_d = 0.0;
                if ((st = defl_update(p, df, c, &rn_d))) return st;
                rn_new = rn_d;
                df.accepted = true;
                info.deflation_corrections += 1;
            } else if (!df.accepted) {
                df.k = 0;   // Ritz vectors that do not describe the small eigenvalues
            }
        }
        info.outer_iterations += 1;
        if (rn_new < thr) {
            rn = rn_new;
            break;
        }
        if (!(rn_new < rn)) {
            // no progress (or a non-finite correction from an FP32 breakdown):
            // drop the phase, and hand over to FP64 PCG after two such phases
            VPP_HIP(hipMemcpyAsync(w.x, w.xb, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
            if ((st = residual64(p, &rr))) return st;
            if (++bad_phases >= 2 || hs->iters >= o.max_iter) {
                vpp_cg_info f64{};
                double r0f = 0.0;
                vpp_cg_opts of = o;
                of.max_iter = std::max(0, o.max_iter - hs->iters);
                of.atol = std::max(o.atol, thr);
                of.rtol = 0.0;
                if ((st = pcg64(p, of, f64, &r0f))) return st;
                info.iterations = hs->iters + f64.iterations;
                info.status = f64.status;
                double rr_end;
                if ((st = residual64(p, &rr_end))) return st;
                info.rel_residual = r0 > 0 ? std::sqrt(rr_end) / r0 : 0.0;
                return VPP_OK;
            }
            // restart the FP32 recurrence from the kept iterate's residual
            VPP_HIP(launch_cg_replace32(w.st32, w.red, w.r, 1.0 / rn, 0.0, w.r32, w.p32, w.x32, p->inv32, p->N, s));
            continue;
        }
        bad_phases = 0;
        if (hs->iters >= o.max_iter || info.outer_iterations >= max_phases) {
            info.status = VPP_ERR_NOT_CONVERGED;
            rn = rn_new;
            break;
        }
        // keep the direction (built on the residual scaled by 1/rn) unless the
        // FP32 recurrence broke down (p.Ap <= 0 from rounding): then restart it
        VPP_HIP(launch_cg_replace32(w.st32, w.red, w.r, 1.0 / rn_new, broke ? 0.0 : rn / rn_new, w.r32, w.p32, w.x32,
                                    p->inv32, p->N, s));
        rn = rn_new;
    }
    info.iterations = hs->iters;
    info.rel_residual = r0 > 0 ? rn / r0 : 0.0;
    return VPP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner cache: a JSON file {"entries": [{"key": ..., "variant": v,
// "tile": [tx, ty, tz], "us": t}, ...]} keyed by architecture, degree and
// problem-size bucket.

static std::string size_bucket_key(const char* what, int k, int64_t n)
{
    int b = 0;
    while ((int64_t(1) << (b + 1)) <= n) ++b;
    char buf[128];
    std::snprintf(buf, sizeof buf, "gfx950/%s/k%d/n2^%d", what, k, b);
    return buf;
}

struct CacheEntry {
    std::string key;
    LaunchCfg cfg;
    double us;
};

static std::vector<CacheEntry> read_cache(const char* path)
{
    std::vector<CacheEntry> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find("\"key\"", pos)) != std::string::npos) {
        CacheEntry e{};
        size_t q1 = s.find('"', s.find(':', pos) + 1);
        size_t q2 = s.find('"', q1 + 1);
        if (q1 == std::string::npos || q2 == std::string::npos) break;
        e.key = s.substr(q1 + 1, q2 - q1 - 1);
        size_t v = s.find("\"variant\"", q2);
        size_t t = s.find("\"tile\"", q2);
        size_t u = s.find("\"us\"", q2);
        if (v == std::string::npos || t == std::string::npos || u == std::string::npos) break;
        e.cfg.variant = std::atoi(s.c_str() + s.find(':', v) + 1);
        const char* tp = s.c_str() + s.find('[', t) + 1;
        char* end = nullptr;
        e.cfg.tile[0] = (int)std::strtol(tp, &end, 10);
        e.cfg.tile[1] = (int)std::strtol(end + 1, &end, 10);
        e.cfg.tile[2] = (int)std::strtol(end + 1, &end, 10);
        e.us = std::atof(s.c_str() + s.find(':', u) + 1);
        out.push_back(e);
        pos = u;
    }
    return out;
}

static void write_cache(const char* path, const std::vector<CacheEntry>& es)
{
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\"entries\": [\n";
        for (size_t i = 0; i < es.size(); ++i) {
            f << "  {\"key\": \"" << es[i].key << "\", \"variant\": " << es[i].cfg.variant << ", \"tile\": ["
              << es[i].cfg.tile[0] << ", " << es[i].cfg.tile[1] << ", " << es[i].cfg.tile[2]
              << "], \"us\": " << es[i].us << "}" << (i + 1 < es.size() ? "," : "") << "\n";
        }
        f << "]}\n";
    }
    std::rename(tmp.c_str(), path);
}

static bool cache_lookup(const char* path, const std::string& key, LaunchCfg* cfg)
{
    for (const auto& e : read_cache(path))
        if (e.key == key) {
            *cfg = e.cfg;
            return true;
        }
    return false;
}

static void cache_store(const char* path, const std::string& key, const LaunchCfg& cfg, double us)
{
    if (!path) return;
    auto es = read_cache(path);
    bool found = false;
    for (auto& e : es)
        if (e.key == key) {
            e.cfg = cfg;
            e.us = us;
            found = true;
        }
    if (!found) es.push_back(CacheEntry{key, cfg, us});
    write_cache(path, es);
}

// ---------------------------------------------------------------------------
// C ABI

// Argument checks of a problem description (vpp_create, vpp_apply_noalloc).
static vpp_status validate_desc(const vpp_desc* d)
{
    if (d->degree < 2 || d->degree > 4) return fail(VPP_ERR_INVALID_ARG, "degree must be 2, 3 or 4");
    for (int i = 0; i < 3; ++i) {
        if (d->ncells[i] < 1) return fail(VPP_ERR_INVALID_ARG, "ncells must be >= 1");
        if (!(d->extent[i] > 0.0) || !std::isfinite(d->extent[i]))
            return fail(VPP_ERR_INVALID_ARG, "extent must be positive");
        if (!std::isfinite(d->origin[i])) return fail(VPP_ERR_INVALID_ARG, "origin must be finite");
    }
    if (!(d->rho_l > 0.0) || !(d->rho_g > 0.0) || !std::isfinite(d->rho_l) || !std::isfinite(d->rho_g))
        return fail(VPP_ERR_INVALID_ARG, "densities must be positive");
    for (int f = 0; f < 6; ++f)
        if (d->bc[f] != VPP_BC_DIRICHLET && d->bc[f] != VPP_BC_NEUMANN)
            return fail(VPP_ERR_INVALID_ARG, "bc must be VPP_BC_DIRICHLET or VPP_BC_NEUMANN");
    if (d->heaviside != VPP_H_LINEAR && d->heaviside != VPP_H_PAPER && d->heaviside != VPP_H_LINEAR_ARITH &&
        d->heaviside != VPP_H_PAPER_ARITH)
        return fail(VPP_ERR_INVALID_ARG, "unknown heaviside");
    const int64_t k = d->degree;
    const int64_t N = (k * d->ncells[0] + 1) * (k * d->ncells[1] + 1) * (k * d->ncells[2] + 1);
    const int64_t ncell = (int64_t)d->ncells[0] * d->ncells[1] * d->ncells[2];
    if (N > (int64_t)INT32_MAX || ncell > (int64_t)INT32_MAX / 2)
        return fail(VPP_ERR_INVALID_ARG, "mesh too large (at most 2^31-1 nodes)");
    for (int i = 0; i < 3; ++i)
        if ((int64_t)k * d->ncells[i] + 1 >= (int64_t(1) << 20))
            return fail(VPP_ERR_INVALID_ARG, "mesh too large (at most 2^20-1 nodes per direction)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(VPP_ERR_HIP, "no HIP device available");
    }
    if (d->device < 0 || d->device >= ndev) return fail(VPP_ERR_INVALID_ARG, "device ordinal out of range");
    return VPP_OK;
}

extern "C" {

const char* vpp_last_error(void) { return g_err.c_str(); }
int32_t vpp_abi_version(void) { return VPP_ABI_VERSION; }

int64_t vpp_debug_bounds_violations(void)
{
#ifdef VPP_BOUNDS_CHECK
    if (hipDeviceSynchronize() != hipSuccess) return -2;
    const unsigned long long c[7] = {bounds_count_apply_f64_k2(), bounds_count_apply_f64_k3(),
                                     bounds_count_apply_f64_k4(), bounds_count_apply_f32_k2(),
                                     bounds_count_apply_f32_k3(), bounds_count_apply_f32_k4(),
                                     bounds_count_misc()};
    int64_t n = 0;
    for (unsigned long long v : c) {
        if (v == ~0ull) return -2;
        n += (int64_t)v;
    }
    return n;
#else
    return -1;
#endif
}

vpp_status vpp_create(const vpp_desc* d, vpp_problem* out)
{
    if (!d || !out) return fail(VPP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    vpp_status vs = validate_desc(d);
    if (vs) return vs;
    const int64_t k = d->degree;
    const int64_t N = (k * d->ncells[0] + 1) * (k * d->ncells[1] + 1) * (k * d->ncells[2] + 1);
    const int64_t ncell = (int64_t)d->ncells[0] * d->ncells[1] * d->ncells[2];
    DeviceGuard dg(d->device);
    vpp_problem p = new vpp_problem_s();
    p->desc = *d;
    p->k = d->degree;
    p->N = N;
    p->ncell = ncell;
    p->NQ = ncell * (k + 1) * (k + 1) * (k + 1);
    p->m = make_mesh_args(*d);
    p->cfg = default_config(p->k);
    if (arith_law(*d)) {
        LaunchCfg ac[4];
        if (list_arith_configs(p->k, ac, 4) < 1) {
            delete p;
            return fail(VPP_ERR_UNSUPPORTED, "no kernel configuration with the arithmetic density mean");
        }
        p->cfg = ac[0];
    }
    set_tiles(p->m, p->cfg);
    p->m32 = p->m;
    p->cfg32 = p->cfg;
    vpp_status s;
    if ((s = dev_alloc(&p->phi64, N, "phi")) || (s = dev_alloc(&p->phi32, N, "phi32")) ||
        (s = dev_alloc(&p->diag, N, "diag")) || (s = dev_alloc(&p->inv64, N, "invdiag")) ||
        (s = dev_alloc(&p->inv32, N, "invdiag32"))) {
        vpp_destroy(p);
        return s;
    }
    if ((s = ensure_apply_scratch(p))) {
        vpp_destroy(p);
        return s;
    }
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
        vpp_destroy(p);
        return fail(VPP_ERR_HIP, "hipStreamCreate failed");
    }
    *out = p;
    return VPP_OK;
}

vpp_status vpp_destroy(vpp_problem p)
{
    if (!p) return VPP_OK;
    DeviceGuard dg(p->desc.device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    free_work(p->w);
    dev_free(p->phi64); dev_free(p->phi32); dev_free(p->diag); dev_free(p->inv64); dev_free(p->inv32);
    dev_free(p->part); dev_free(p->dot_part); dev_free(p->cellbuf);
    if (p->cell_evt) (void)hipEventDestroy(p->cell_evt);
    dev_free(p->cp_list); dev_free(p->cp_ctr);
    free_reinit(p->rw);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return VPP_OK;
}

int64_t vpp_num_dofs(vpp_problem p) { return p ? p->N : -1; }
int64_t vpp_num_qpoints(vpp_problem p) { return p ? p->NQ : -1; }

vpp_status vpp_set_phi(vpp_problem p, const double* phi, void* stream)
{
    if (!p || !phi) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, phi);
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    VPP_HIP(hipMemcpyAsync(p->phi64, phi, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    VPP_HIP(launch_convert(p->phi64, p->phi32, p->N, s));
    vpp_status st = build_diagonal(p, s);
    if (st) return st;
    p->phi_set = true;
    return VPP_OK;
}

vpp_status vpp_set_mass(vpp_problem p, double mu, void* stream)
{
    if (!p) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(VPP_ERR_INVALID_ARG, "the mass shift must be finite and >= 0");
    if (mu != 0.0 && arith_law(p->desc))
        return fail(VPP_ERR_UNSUPPORTED, "the mass shift is not available with the arithmetic density mean");
    LaunchCfg mc[16];
    if (mu != 0.0 && list_mass_configs(p->k, mc, 16) < 1)
        return fail(VPP_ERR_UNSUPPORTED, "no kernel configuration with the mass shift for this degree");
    DeviceGuard dg(p->desc.device);
    VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (p->stream) VPP_HIP(hipStreamSynchronize(p->stream));
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= p->desc.extent[d] / p->desc.ncells[d];
    p->m.mass = p->m32.mass = mu * vol;
    if (mu != 0.0) {
        if (!mass_config_supported(p->cfg, p->k)) put_config(p, VPP_FP64, mc[0]);
        if (!mass_config_supported(p->cfg32, p->k)) put_config(p, VPP_FP32, mc[0]);
    }
    free_graphs(p->w);   // they hold the operator's arguments by value
    vpp_status st = ensure_apply_scratch(p);
    if (st) return st;
    if (p->phi_set && (st = build_diagonal(p, (hipStream_t)stream))) return st;
    return VPP_OK;
}

vpp_status vpp_apply(vpp_problem p, int32_t prec, const void* x, void* y, void* stream)
{
    if (!p || !x || !y) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (x == y) return fail(VPP_ERR_INVALID_ARG, "x and y must not alias");
    if (prec != VPP_FP64 && prec != VPP_FP32) return fail(VPP_ERR_INVALID_ARG, "precision must be FP64 or FP32");
    VPP_ALIGNED(prec == VPP_FP32 ? 4 : 8, x, y);
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    if (prec == VPP_FP64) return do_apply64(p, (const double*)x, (double*)y, nullptr, nullptr, s);
    return do_apply32(p, (const float*)x, (float*)y, nullptr, nullptr, s);
}

// Configuration of the allocation-free apply: fixed per degree and law (no
// autotuning, which needs a cache-flush buffer).
static LaunchCfg noalloc_config(const vpp_desc& d)
{
    if (arith_law(d)) {
        LaunchCfg c[4];
        list_arith_configs(d.degree, c, 4);
        return c[0];
    }
    if (d.degree == 2) return LaunchCfg{4, {16, 8, 4}};
    if (d.degree == 3) return LaunchCfg{2, {8, 4, 4}};
    return LaunchCfg{1, {4, 2, 2}};
}

vpp_status vpp_apply_noalloc(const vpp_desc* d, const double* phi, const double* x, double* y, void* stream)
{
    if (!d || !phi || !x || !y) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, phi, x, y);
    if ((const void*)x == y || (const void*)phi == y) return fail(VPP_ERR_INVALID_ARG, "y must not alias x or phi");
    vpp_status vs = validate_desc(d);
    if (vs) return vs;
    const LaunchCfg cfg = noalloc_config(*d);
    MeshArgs m = make_mesh_args(*d);
    set_tiles(m, cfg);
    const int64_t ns = shared_stride(m);
    if (8 * ns > (int64_t)kNoallocScratchDoubles)
        return fail(VPP_ERR_UNSUPPORTED, "mesh too large for the static scratch of vpp_apply_noalloc (its shared-face "
                                         "partials need " + std::to_string(8 * ns * 8) + " bytes, the scratch holds " +
                                         std::to_string(kNoallocScratchDoubles * 8) + ")");
    DeviceGuard dg(d->device);
    double* scratch = nullptr;
    VPP_HIP(noalloc_scratch(d->device, &scratch));
    ApplyArgs<double> a{m, x, y, phi, scratch, ns, nullptr, nullptr, nullptr, false};
    VPP_HIP(launch_apply_f64(cfg, d->degree, a, (hipStream_t)stream));
    return VPP_OK;
}

vpp_status vpp_diagonal(vpp_problem p, double* diag, void* stream)
{
    if (!p || !diag) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, diag);
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    DeviceGuard dg(p->desc.device);
    VPP_HIP(hipMemcpyAsync(diag, p->diag, p->N * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return VPP_OK;
}

vpp_status vpp_cg_solve(vpp_problem p, const double* b, double* x, const vpp_cg_opts* opts, vpp_cg_info* info,
                        void* stream)
{
    if (!p || !b || !x || !opts) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, b, x);
    if (!(opts->rtol >= 0.0) || !(opts->atol >= 0.0) || opts->max_iter < 0)
        return fail(VPP_ERR_INVALID_ARG, "tolerances must be >= 0 and max_iter >= 0");
    if (opts->precision != VPP_FP64 && opts->precision != VPP_MIXED)
        return fail(VPP_ERR_INVALID_ARG, "precision must be VPP_FP64 or VPP_MIXED");
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    DeviceGuard dg(p->desc.device);
    const bool mixed = opts->precision == VPP_MIXED;
    vpp_status st;
    if ((st = ensure_work(p, mixed))) return st;
    int chunk = opts->check_every > 0 ? opts->check_every : 32;
    chunk = std::max(2, std::min(chunk, 512));
    chunk += chunk & 1;
    if ((st = ensure_graphs(p, chunk, mixed))) return st;
    // Order after the caller's stream, then work on the library stream.
    VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
    hipStream_t s = p->stream;
    CgWork& w = p->w;
    VPP_HIP(hipMemcpyAsync(w.b, b, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    VPP_HIP(hipMemcpyAsync(w.x, x, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    vpp_cg_info inf{};
    inf.deflation_first_change = -1.0;
    double r0 = 0.0;
    if (mixed) st = pcg_mixed(p, *opts, inf, &r0);
    else st = pcg64(p, *opts, inf, &r0);
    if (st) return st;
    VPP_HIP(hipMemcpyAsync(x, w.x, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    double rr_true = 0.0;
    if ((st = residual64(p, &rr_true))) return st;
    inf.true_rel_residual = r0 > 0 ? std::sqrt(rr_true) / r0 : 0.0;
    if (info) *info = inf;
    if (inf.status == VPP_ERR_NOT_CONVERGED) return fail(VPP_ERR_NOT_CONVERGED, "CG did not converge");
    if (inf.status == VPP_ERR_BREAKDOWN) return fail(VPP_ERR_BREAKDOWN, "CG breakdown (p.Ap <= 0 or non-finite)");
    return VPP_OK;
}

vpp_status vpp_grad_coef(vpp_problem p, const double* pv, const double* lam, double* g_q, void* stream)
{
    if (!p || !pv || !lam || !g_q) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, pv, lam, g_q);
    DeviceGuard dg(p->desc.device);
    VPP_HIP(launch_grad_coef(p->k, p->m, pv, lam, g_q, (hipStream_t)stream));
    return VPP_OK;
}

vpp_status vpp_grad_phi(vpp_problem p, const double* g_q, double* g_phi, void* stream)
{
    if (!p || !g_q || !g_phi) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, g_q, g_phi);
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    if (arith_law(p->desc))
        return fail(VPP_ERR_UNSUPPORTED, "dJ/dphi is available for the reciprocal density mean (Eq. rhoEff) only");
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    vpp_status st;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_grad_phi(p->k, p->m, p->phi64, g_q, g_phi, cv, s));
    return cell_scratch_end(p, s);
}

static vpp_status closest_points(vpp_problem p, const double* pts, int64_t n, const double* const nrm[3],
                                 const vpp_cp_opts* o, double* y, int32_t* info, void* stream)
{
    if (!p || !o || !y || !info) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, pts, y, nrm ? nrm[0] : nullptr, nrm ? nrm[1] : nullptr, nrm ? nrm[2] : nullptr);
    VPP_ALIGNED(4, info);
    if (pts && n < 0) return fail(VPP_ERR_INVALID_ARG, "n must be >= 0");
    if (!(o->eps > 0.0) || !std::isfinite(o->eps) || !(o->tol > 0.0) || !std::isfinite(o->tol) ||
        !(o->phi_lim > 0.0 && o->phi_lim <= 1.0) || o->max_iter < 1 || o->max_iter > 10000 ||
        o->normal_steps < 0 || o->normal_steps > 100)
        return fail(VPP_ERR_INVALID_ARG, "closest-point options out of range");
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    // the queue head counts past the last point by at most one fetch per resident lane
    if ((pts ? n : p->N) > (int64_t)INT32_MAX - (int64_t(1) << 24))
        return fail(VPP_ERR_UNSUPPORTED, "too many points for the 32-bit work queue");
    DeviceGuard dg(p->desc.device);
    CpArgs a{};
    a.m = p->m;
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = p->desc.origin[d];
        a.hi[d] = p->desc.origin[d] + p->desc.extent[d];
        a.h[d] = p->desc.extent[d] / p->desc.ncells[d];
    }
    a.phi = p->phi64;
    for (int d = 0; d < 3; ++d) a.nrm[d] = nrm ? nrm[d] : nullptr;
    a.pts = pts;
    a.n = pts ? n : p->N;
    a.phi_lim = o->phi_lim;
    a.eps = o->eps;
    a.tol = o->tol;
    a.max_iter = o->max_iter;
    a.normal_steps = o->normal_steps;
    a.y = y;
    a.info = info;
    vpp_status st;
    if (!p->cp_ctr && (st = dev_alloc(&p->cp_ctr, 2, "closest-point counters"))) return st;
    if (!pts && !p->cp_list && (st = dev_alloc(&p->cp_list, (size_t)p->N, "closest-point band list"))) return st;
    VPP_HIP(launch_closest_points(p->k, a, p->cp_list, p->cp_ctr, closest_point_blocks(p->k), (hipStream_t)stream));
    return VPP_OK;
}

vpp_status vpp_closest_points(vpp_problem p, const double* pts, int64_t n, const vpp_cp_opts* o, double* y,
                              int32_t* info, void* stream)
{
    return closest_points(p, pts, n, nullptr, o, y, info, stream);
}

vpp_status vpp_closest_points_normal(vpp_problem p, const double* pts, int64_t n, const double* n0,
                                     const double* n1, const double* n2, const vpp_cp_opts* o, double* y,
                                     int32_t* info, void* stream)
{
    if (!n0 || !n1 || !n2) return fail(VPP_ERR_INVALID_ARG, "null normal component");
    const double* const nrm[3] = {n0, n1, n2};
    return closest_points(p, pts, n, nrm, o, y, info, stream);
}

vpp_status vpp_extend(vpp_problem p, const double* y, const int32_t* info, const double* f, double* out,
                      void* stream)
{
    if (!p || !y || !info || !f || !out) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, y, f, out);
    VPP_ALIGNED(4, info);
    if (f == out) return fail(VPP_ERR_INVALID_ARG, "f and out must not alias");
    DeviceGuard dg(p->desc.device);
    CpArgs a{};
    a.m = p->m;
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = p->desc.origin[d];
        a.hi[d] = p->desc.origin[d] + p->desc.extent[d];
        a.h[d] = p->desc.extent[d] / p->desc.ncells[d];
    }
    a.n = p->N;
    a.y = const_cast<double*>(y);
    a.info = const_cast<int32_t*>(info);
    VPP_HIP(launch_extend(p->k, a, f, out, (hipStream_t)stream));
    return VPP_OK;
}

static RhsGeo rhs_geometry(vpp_problem p)
{
    RhsGeo g{};
    g.m = p->m;
    g.vol = 1.0;
    for (int d = 0; d < 3; ++d) {
        const double h = p->desc.extent[d] / p->desc.ncells[d];
        g.ih[d] = 1.0 / h;
        g.vol *= h;
    }
    return g;
}

vpp_status vpp_normal_rhs(vpp_problem p, const double* phi, double* b0, double* b1, double* b2, void* stream)
{
    if (!p || !phi || !b0 || !b1 || !b2) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, phi, b0, b1, b2);
    if (b0 == b1 || b0 == b2 || b1 == b2 || (const void*)phi == b0 || (const void*)phi == b1 ||
        (const void*)phi == b2)
        return fail(VPP_ERR_INVALID_ARG, "phi and the outputs must not alias");
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    vpp_status st;
    if ((st = cell_scratch_begin(p, 3, s, &cv))) return st;
    VPP_HIP(launch_normal_rhs(p->k, rhs_geometry(p), phi, b0, b1, b2, cv, s));
    return cell_scratch_end(p, s);
}

vpp_status vpp_curvature_rhs(vpp_problem p, const double* n0, const double* n1, const double* n2, double* b,
                             void* stream)
{
    if (!p || !n0 || !n1 || !n2 || !b) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, n0, n1, n2, b);
    if ((const void*)b == n0 || (const void*)b == n1 || (const void*)b == n2)
        return fail(VPP_ERR_INVALID_ARG, "the output must not alias an input");
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    vpp_status st;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_curvature_rhs(p->k, rhs_geometry(p), n0, n1, n2, b, cv, s));
    return cell_scratch_end(p, s);
}

static vpp_status ensure_reinit_work(vpp_problem p)
{
    if (p->rw) return VPP_OK;
    ReinitWork* w = new ReinitWork();
    const size_t n = (size_t)p->N;
    vpp_status st;
    if ((st = dev_alloc(&w->b, n, "reinit b")) || (st = dev_alloc(&w->r, n, "reinit r")) ||
        (st = dev_alloc(&w->p, n, "reinit p")) || (st = dev_alloc(&w->q, n, "reinit q")) ||
        (st = dev_alloc(&w->x, n, "reinit x")) || (st = dev_alloc(&w->diag, n, "reinit diag")) ||
        (st = dev_alloc(&w->invd, n, "reinit inverse diag")) || (st = dev_alloc(&w->inv32, n, "reinit inverse diag")) ||
        (st = dev_alloc(&w->red, kRedDoubles, "reinit partials")) ||
        (st = dev_alloc(&w->dot, kMaxRedBlocks, "reinit dot partials")) || (st = dev_alloc(&w->rr, 1, "norm")) ||
        (st = dev_alloc(&w->st, 1, "reinit state"))) {
        free_reinit(w);
        return st;
    }
    if (hipHostMalloc((void**)&w->hst, sizeof(CgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&w->hrr, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        free_reinit(w);
        return fail(VPP_ERR_OUT_OF_MEMORY, "reinit host mirrors");
    }
    p->rw = w;
    return VPP_OK;
}

vpp_status vpp_reinit_step(vpp_problem p, const double* psi, const double* n0, const double* n1, const double* n2,
                           const vpp_reinit_opts* o, double* psi_out, vpp_cg_info* info, void* stream)
{
    if (!p || !psi || !n0 || !n1 || !n2 || !o || !psi_out) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, psi, n0, n1, n2, psi_out);
    if (!(o->eps > 0.0) || !std::isfinite(o->eps) || !(o->dtau > 0.0) || !std::isfinite(o->dtau) ||
        !(o->rtol >= 0.0) || !(o->atol >= 0.0) || o->max_iter < 0 || o->max_iter > 10000000)
        return fail(VPP_ERR_INVALID_ARG, "reinitialization options out of range");
    DeviceGuard dg(p->desc.device);
    vpp_status st;
    if ((st = ensure_reinit_work(p))) return st;
    VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
    hipStream_t s = p->stream;
    ReinitWork& w = *p->rw;
    const int64_t n = p->N;
    ReinitArgs ra{rhs_geometry(p), o->eps, 1.0 / o->dtau, n0, n1, n2};
    // natural conditions on every face: no identity rows, whatever the problem's faces
    ra.g.m.bcmask = 0;
    MeshArgs m1 = ra.g.m;
    m1.ntile[0] = m1.ntile[1] = m1.ntile[2] = 1;
    const int one[3] = {1, 1, 1};
    const SharedEnum none = shared_enum(m1, p->k, one);   // no shared nodes: q is used as it is
    const int gdot = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxRedBlocks, (n + 1023) / 1024));
    double* cv;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_reinit_rhs(p->k, ra, psi, w.b, cv, s));
    VPP_HIP(launch_reinit_diag(p->k, ra, w.diag, cv, s));
    VPP_HIP(launch_fix_diagonal(ra.g.m, w.diag, w.invd, w.inv32, s));
    VPP_HIP(hipMemcpyAsync(w.x, psi, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    VPP_HIP(launch_reinit_apply(p->k, ra, w.x, w.q, cv, s));
    CgState* hs = w.hst;
    std::memset(hs, 0, sizeof(CgState));
    VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
    VPP_HIP(launch_cg_init<double>(w.st, w.red, w.b, w.q, w.r, w.p, w.invd, n, s));
    VPP_HIP(hipMemcpyAsync(hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    vpp_cg_info inf{};
    inf.deflation_first_change = -1.0;
    const double r0 = std::sqrt(hs->rr_last), rz0 = hs->rz[0];
    const double thr = std::max(o->rtol * r0, o->atol);
    inf.rel_residual = r0 > 0 ? 1.0 : 0.0;
    bool iterate = true;
    if (!std::isfinite(r0) || !std::isfinite(rz0)) {
        inf.status = VPP_ERR_BREAKDOWN;
        iterate = false;
    } else if (r0 == 0.0 || r0 < o->atol) {
        inf.status = VPP_OK;
        iterate = false;
    } else if (o->max_iter == 0) {
        inf.status = VPP_ERR_NOT_CONVERGED;
        iterate = false;
    }
    if (iterate) {
        CgState init{};
        init.rz[0] = rz0;
        init.tol2 = thr * thr;
        init.max_iter = o->max_iter;
        *hs = init;
        VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
        constexpr int chunk = 16;
        for (int done = 0; done < o->max_iter + chunk;) {
            for (int it = 0; it < chunk; ++it, ++done) {
                const int par = done & 1;
                VPP_HIP(launch_reinit_apply(p->k, ra, w.p, w.q, cv, s));
                VPP_HIP(launch_dot_partials(w.p, w.q, n, w.dot, gdot, s));
                VPP_HIP(launch_cg_assemble_update<double>(w.st, par, w.red, w.dot, gdot, ra.g.m, none, nullptr, 0,
                                                          w.r, w.q, w.invd, n, s));
                VPP_HIP(launch_cg_pupdate<double>(w.st, par, w.red, w.x, w.r, w.p, w.invd, n, s));
            }
            VPP_HIP(hipMemcpyAsync(hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            VPP_HIP(hipStreamSynchronize(s));
            if (hs->halt[0] || hs->halt[1]) break;
        }
        inf.iterations = hs->iters;
        inf.rel_residual = std::sqrt(hs->rr_last) / r0;
        if (hs->breakdown) inf.status = VPP_ERR_BREAKDOWN;
        else if (hs->rr_last < init.tol2) inf.status = VPP_OK;
        else inf.status = VPP_ERR_NOT_CONVERGED;
    }
    // true residual, then the new level set
    VPP_HIP(launch_reinit_apply(p->k, ra, w.x, w.q, cv, s));
    VPP_HIP(launch_residual(w.b, w.q, nullptr, n, w.red, w.rr, s));
    if ((st = cell_scratch_end(p, s))) return st;
    VPP_HIP(hipMemcpyAsync(w.hrr, w.rr, sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipMemcpyAsync(psi_out, w.x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    VPP_HIP(hipStreamSynchronize(s));
    inf.true_rel_residual = r0 > 0 ? std::sqrt(*w.hrr) / r0 : 0.0;
    if (info) *info = inf;
    if (inf.status == VPP_ERR_NOT_CONVERGED) return fail(VPP_ERR_NOT_CONVERGED, "reinitialization CG did not converge");
    if (inf.status == VPP_ERR_BREAKDOWN) return fail(VPP_ERR_BREAKDOWN, "reinitialization CG breakdown");
    return VPP_OK;
}

// The reinitialization step's operator, diagonal and right-hand side on their
// own (the same launches vpp_reinit_step makes).
static vpp_status reinit_args(vpp_problem p, const double* n0, const double* n1, const double* n2,
                              const vpp_reinit_opts* o, ReinitArgs* ra)
{
    if (!o || !n0 || !n1 || !n2) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, n0, n1, n2);
    if (!(o->eps > 0.0) || !std::isfinite(o->eps) || !(o->dtau > 0.0) || !std::isfinite(o->dtau))
        return fail(VPP_ERR_INVALID_ARG, "reinitialization eps and dtau must be positive and finite");
    *ra = ReinitArgs{rhs_geometry(p), o->eps, 1.0 / o->dtau, n0, n1, n2};
    ra->g.m.bcmask = 0;
    return VPP_OK;
}

vpp_status vpp_reinit_apply(vpp_problem p, const double* n0, const double* n1, const double* n2,
                            const vpp_reinit_opts* o, const double* x, double* y, void* stream)
{
    if (!p || !x || !y) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, x, y);
    if ((const void*)x == y || (const void*)y == n0 || (const void*)y == n1 || (const void*)y == n2)
        return fail(VPP_ERR_INVALID_ARG, "y must not alias an input");
    ReinitArgs ra;
    vpp_status st;
    if ((st = reinit_args(p, n0, n1, n2, o, &ra))) return st;
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_reinit_apply(p->k, ra, x, y, cv, s));
    return cell_scratch_end(p, s);
}

vpp_status vpp_reinit_diagonal(vpp_problem p, const double* n0, const double* n1, const double* n2,
                               const vpp_reinit_opts* o, double* diag, void* stream)
{
    if (!p || !diag) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, diag);
    if ((const void*)diag == n0 || (const void*)diag == n1 || (const void*)diag == n2)
        return fail(VPP_ERR_INVALID_ARG, "diag must not alias an input");
    ReinitArgs ra;
    vpp_status st;
    if ((st = reinit_args(p, n0, n1, n2, o, &ra))) return st;
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_reinit_diag(p->k, ra, diag, cv, s));
    return cell_scratch_end(p, s);
}

vpp_status vpp_reinit_rhs(vpp_problem p, const double* psi, const double* n0, const double* n1, const double* n2,
                          const vpp_reinit_opts* o, double* b, void* stream)
{
    if (!p || !psi || !b) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, psi, b);
    if ((const void*)b == psi || (const void*)b == n0 || (const void*)b == n1 || (const void*)b == n2)
        return fail(VPP_ERR_INVALID_ARG, "b must not alias an input");
    ReinitArgs ra;
    vpp_status st;
    if ((st = reinit_args(p, n0, n1, n2, o, &ra))) return st;
    DeviceGuard dg(p->desc.device);
    hipStream_t s = (hipStream_t)stream;
    double* cv;
    if ((st = cell_scratch_begin(p, 1, s, &cv))) return st;
    VPP_HIP(launch_reinit_rhs(p->k, ra, psi, b, cv, s));
    return cell_scratch_end(p, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Once-refined meshes with hanging nodes.

struct vpp_amr_s {
    vpp_desc desc{};
    int k = 2;
    int64_t nc = 0, nf = 0, n = 0, nfree = 0;
    AmrArgs args{};
    int *d_cells = nullptr, *d_fkind = nullptr, *d_cptr = nullptr, *d_ccol = nullptr;
    double* d_cw = nullptr;
    int *d_nptr = nullptr, *d_nidx = nullptr;   // per entry: the cell results that reach it
    double *d_nw = nullptr, *d_scratch = nullptr;
    int *d_soff = nullptr, *d_dptr = nullptr, *d_didx = nullptr;   // the same for the diagonal
    unsigned char* d_ident = nullptr;
    double *phi = nullptr, *diag = nullptr, *inv64 = nullptr;
    float* inv32 = nullptr;
    bool phi_set = false;
    hipStream_t stream = nullptr;
    ReinitWork* w = nullptr;   // CG vectors (allocated by the first solve)
};

static double gll_point(int k, int i)
{
    if (k == 2) return Tab<2>::t.gll[i];
    if (k == 3) return Tab<3>::t.gll[i];
    return Tab<4>::t.gll[i];
}

// Lagrange polynomial a of the GLL points of degree k at x (product formula).
static double gll_lagrange(int k, int a, double x)
{
    double v = 1.0;
    for (int b = 0; b <= k; ++b)
        if (b != a) v *= (x - gll_point(k, b)) / (gll_point(k, a) - gll_point(k, b));
    return v;
}

static void amr_free(vpp_amr a)
{
    if (!a) return;
    dev_free(a->d_cells); dev_free(a->d_fkind); dev_free(a->d_cptr); dev_free(a->d_ccol); dev_free(a->d_cw);
    dev_free(a->d_ident); dev_free(a->phi); dev_free(a->diag); dev_free(a->inv64); dev_free(a->inv32);
    dev_free(a->d_nptr); dev_free(a->d_nidx); dev_free(a->d_nw); dev_free(a->d_scratch);
    dev_free(a->d_soff); dev_free(a->d_dptr); dev_free(a->d_didx);
    free_reinit(a->w);
    if (a->stream) (void)hipStreamDestroy(a->stream);
    delete a;
}

template <typename T>
static vpp_status upload(T** dst, const std::vector<T>& src, const char* what)
{
    vpp_status s = dev_alloc(dst, src.size(), what);
    if (s) return s;
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(VPP_ERR_HIP, std::string("upload of ") + what + " failed");
    return VPP_OK;
}

extern "C" vpp_status vpp_amr_create(const vpp_desc* d, const uint8_t* refined, vpp_amr* out)
{
    if (!d || !refined || !out) return fail(VPP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    vpp_status vs = validate_desc(d);
    if (vs) return vs;
    const int k = d->degree;
    const int nc[3] = {d->ncells[0], d->ncells[1], d->ncells[2]};
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    if (ncell > (int64_t(1) << 27)) return fail(VPP_ERR_INVALID_ARG, "mesh too large for the refined lattice");
    int64_t cn[3], fn[3];
    for (int i = 0; i < 3; ++i) {
        cn[i] = (int64_t)k * nc[i] + 1;
        fn[i] = 2 * (int64_t)k * nc[i] + 1;
    }
    const int64_t Nc = cn[0] * cn[1] * cn[2], Nf = fn[0] * fn[1] * fn[2];
    if (Nc + Nf > (int64_t)INT32_MAX) return fail(VPP_ERR_INVALID_ARG, "mesh too large (at most 2^31-1 entries)");
    auto ref = [&](int64_t cx, int64_t cy, int64_t cz) { return refined[cx + nc[0] * (cy + (int64_t)nc[1] * cz)] != 0; };
    // nodes of unrefined coarse cells; fine nodes of refined ones
    std::vector<uint8_t> cact(Nc, 0), fin(Nf, 0);
    std::vector<int> cells;
    for (int cz = 0; cz < nc[2]; ++cz)
        for (int cy = 0; cy < nc[1]; ++cy)
            for (int cx = 0; cx < nc[0]; ++cx) {
                if (ref(cx, cy, cz)) continue;
                cells.push_back(cx + nc[0] * (cy + nc[1] * cz));
                for (int a2 = 0; a2 <= k; ++a2)
                    for (int a1 = 0; a1 <= k; ++a1)
                        for (int a0 = 0; a0 <= k; ++a0)
                            cact[(k * cx + a0) + cn[0] * ((k * cy + a1) + cn[1] * (k * cz + a2))] = 1;
            }
    for (int fz = 0; fz < 2 * nc[2]; ++fz)
        for (int fy = 0; fy < 2 * nc[1]; ++fy)
            for (int fx = 0; fx < 2 * nc[0]; ++fx) {
                if (!ref(fx / 2, fy / 2, fz / 2)) continue;
                cells.push_back(-(1 + (fx + 2 * nc[0] * (fy + 2 * nc[1] * fz))));
                for (int a2 = 0; a2 <= k; ++a2)
                    for (int a1 = 0; a1 <= k; ++a1)
                        for (int a0 = 0; a0 <= k; ++a0)
                            fin[(k * fx + a0) + fn[0] * ((k * fy + a1) + fn[1] * (k * fz + a2))] = 1;
            }
    // a fine node on the closure of an unrefined coarse cell takes that cell's
    // Q_k interpolant (the first such cell in z, y, x order): its constraint list
    std::vector<int> fkind(Nf, -2), cptr(1, 0), ccol;
    std::vector<double> cwv;
    const int twok = 2 * k;
    for (int64_t gf = 0; gf < Nf; ++gf) {
        if (!fin[gf]) continue;
        const int64_t v[3] = {gf % fn[0], (gf / fn[0]) % fn[1], gf / (fn[0] * fn[1])};
        int lo[3], hi[3];
        for (int i = 0; i < 3; ++i) {
            const int c = (int)(v[i] / twok);
            lo[i] = (v[i] % twok == 0) ? c - 1 : c;
            hi[i] = c;
            lo[i] = std::max(lo[i], 0);
            hi[i] = std::min(hi[i], nc[i] - 1);
        }
        int own[3] = {-1, -1, -1};
        for (int cz = lo[2]; cz <= hi[2] && own[0] < 0; ++cz)
            for (int cy = lo[1]; cy <= hi[1] && own[0] < 0; ++cy)
                for (int cx = lo[0]; cx <= hi[0] && own[0] < 0; ++cx)
                    if (!ref(cx, cy, cz)) {
                        own[0] = cx; own[1] = cy; own[2] = cz;
                    }
        if (own[0] < 0) {
            fkind[gf] = -1;
            continue;
        }
        double xi[3];
        for (int i = 0; i < 3; ++i)
            xi[i] = ((double)(v[i] / k) + gll_point(k, (int)(v[i] % k))) * 0.5 - own[i];
        fkind[gf] = (int)cptr.size() - 1;
        for (int a2 = 0; a2 <= k; ++a2)
            for (int a1 = 0; a1 <= k; ++a1)
                for (int a0 = 0; a0 <= k; ++a0) {
                    const double w = gll_lagrange(k, a0, xi[0]) * gll_lagrange(k, a1, xi[1]) * gll_lagrange(k, a2, xi[2]);
                    if (w == 0.0) continue;
                    ccol.push_back((int)((k * own[0] + a0) + cn[0] * ((k * own[1] + a1) + cn[1] * (k * own[2] + a2))));
                    cwv.push_back(w);
                }
        cptr.push_back((int)ccol.size());
    }
    // identity rows: entries that are not free unknowns, and Dirichlet ones
    auto on_dirichlet = [&](const int64_t (&nn)[3], int64_t g) {
        const int64_t i = g % nn[0], j = (g / nn[0]) % nn[1], l = g / (nn[0] * nn[1]);
        const int64_t idx[3] = {i, j, l};
        for (int dd = 0; dd < 3; ++dd) {
            if (d->bc[2 * dd] == VPP_BC_DIRICHLET && idx[dd] == 0) return true;
            if (d->bc[2 * dd + 1] == VPP_BC_DIRICHLET && idx[dd] == nn[dd] - 1) return true;
        }
        return false;
    };
    std::vector<unsigned char> ident(Nc + Nf, 1);
    int64_t nfree = 0;
    for (int64_t g = 0; g < Nc; ++g)
        if (cact[g] && !on_dirichlet(cn, g)) {
            ident[g] = 0;
            ++nfree;
        }
    for (int64_t gf = 0; gf < Nf; ++gf)
        if (fkind[gf] == -1 && !on_dirichlet(fn, gf)) {
            ident[Nc + gf] = 0;
            ++nfree;
        }
    // the cell results reaching each entry (apply's second launch): cell e's
    // local node q is scratch slot q * ncells + e; a free node takes it with
    // weight 1, a constrained one passes it to its sources with their weights.
    // Slots are visited in increasing order, so each entry's list is sorted.
    const int64_t ncell_act = (int64_t)cells.size();
    const int n3 = (k + 1) * (k + 1) * (k + 1);
    if (ncell_act * n3 > (int64_t)INT32_MAX) return fail(VPP_ERR_INVALID_ARG, "too many active cells");
    std::vector<int> nptr((size_t)(Nc + Nf) + 1, 0), nidx;
    std::vector<double> nwv;
    {
        // local node q of every cell, as (target entry, weight) terms
        std::vector<int64_t> tgt;
        std::vector<double> tw;
        std::vector<int> tslot;
        for (int q = 0; q < n3; ++q) {
            const int a0 = q % (k + 1), a1 = (q / (k + 1)) % (k + 1), a2 = q / ((k + 1) * (k + 1));
            for (int64_t e = 0; e < ncell_act; ++e) {
                const int code = cells[e];
                const bool fine = code < 0;
                const int idx = fine ? -(code + 1) : code;
                const int64_t* nn = fine ? fn : cn;
                const int ncx = fine ? 2 * nc[0] : nc[0], ncy = fine ? 2 * nc[1] : nc[1];
                const int64_t cx = idx % ncx, cy = (idx / ncx) % ncy, cz = idx / ((int64_t)ncx * ncy);
                const int64_t gl = (k * cx + a0) + nn[0] * ((k * cy + a1) + nn[1] * (k * cz + a2));
                const int slot = (int)(q * ncell_act + e);
                if (!fine) {
                    tgt.push_back(gl); tw.push_back(1.0); tslot.push_back(slot);
                } else if (fkind[gl] < 0) {
                    tgt.push_back(Nc + gl); tw.push_back(1.0); tslot.push_back(slot);
                } else {
                    for (int p = cptr[fkind[gl]]; p < cptr[fkind[gl] + 1]; ++p) {
                        tgt.push_back(ccol[p]); tw.push_back(cwv[p]); tslot.push_back(slot);
                    }
                }
            }
        }
        if ((int64_t)tgt.size() > (int64_t)INT32_MAX) return fail(VPP_ERR_INVALID_ARG, "too many cell results");
        for (int64_t g : tgt) ++nptr[g + 1];
        for (size_t g = 0; g + 1 < nptr.size(); ++g) nptr[g + 1] += nptr[g];
        nidx.resize(tgt.size());
        nwv.resize(tgt.size());
        std::vector<int> pos(nptr.begin(), nptr.end() - 1);
        for (size_t t = 0; t < tgt.size(); ++t) {
            const int j = pos[tgt[t]]++;
            nidx[j] = tslot[t];
            nwv[j] = tw[t];
        }
    }
    // the diagonal's cell slots: free nodes as above (constrained ones have
    // none), then for every fine cell the coarse nodes its constrained nodes
    // reach, numbered in the order the diagonal kernel meets them (node q,
    // then term p; a coarse node at its first occurrence)
    std::vector<int> soff(ncell_act + 1, 0), dptr((size_t)(Nc + Nf) + 1, 0), didx;
    {
        std::vector<int64_t> tgt;
        std::vector<int64_t> tslot;
        for (int q = 0; q < n3; ++q) {
            const int a0 = q % (k + 1), a1 = (q / (k + 1)) % (k + 1), a2 = q / ((k + 1) * (k + 1));
            for (int64_t e = 0; e < ncell_act; ++e) {
                const int code = cells[e];
                const bool fine = code < 0;
                const int idx = fine ? -(code + 1) : code;
                const int64_t* nn = fine ? fn : cn;
                const int ncx = fine ? 2 * nc[0] : nc[0], ncy = fine ? 2 * nc[1] : nc[1];
                const int64_t cx = idx % ncx, cy = (idx / ncx) % ncy, cz = idx / ((int64_t)ncx * ncy);
                const int64_t gl = (k * cx + a0) + nn[0] * ((k * cy + a1) + nn[1] * (k * cz + a2));
                if (!fine) {
                    tgt.push_back(gl);
                    tslot.push_back(q * ncell_act + e);
                } else if (fkind[gl] < 0) {
                    tgt.push_back(Nc + gl);
                    tslot.push_back(q * ncell_act + e);
                }
            }
        }
        const int64_t nfree_slots = ncell_act * n3;
        std::vector<int> srcs;
        for (int64_t e = 0; e < ncell_act; ++e) {
            soff[e + 1] = soff[e];
            const int code = cells[e];
            if (code >= 0) continue;
            const int idx = -(code + 1);
            const int ncx = 2 * nc[0], ncy = 2 * nc[1];
            const int64_t cx = idx % ncx, cy = (idx / ncx) % ncy, cz = idx / ((int64_t)ncx * ncy);
            srcs.clear();
            for (int q = 0; q < n3; ++q) {
                const int a0 = q % (k + 1), a1 = (q / (k + 1)) % (k + 1), a2 = q / ((k + 1) * (k + 1));
                const int64_t gl = (k * cx + a0) + fn[0] * ((k * cy + a1) + fn[1] * (k * cz + a2));
                if (fkind[gl] < 0) continue;
                for (int p = cptr[fkind[gl]]; p < cptr[fkind[gl] + 1]; ++p)
                    if (std::find(srcs.begin(), srcs.end(), ccol[p]) == srcs.end()) srcs.push_back(ccol[p]);
            }
            if ((int64_t)soff[e] + (int64_t)srcs.size() + nfree_slots > (int64_t)INT32_MAX)
                return fail(VPP_ERR_INVALID_ARG, "too many cell results");
            for (size_t i = 0; i < srcs.size(); ++i) {
                tgt.push_back(srcs[i]);
                tslot.push_back(nfree_slots + soff[e] + (int64_t)i);
            }
            soff[e + 1] = soff[e] + (int)srcs.size();
        }
        for (int64_t g : tgt) ++dptr[g + 1];
        for (size_t g = 0; g + 1 < dptr.size(); ++g) dptr[g + 1] += dptr[g];
        didx.resize(tgt.size());
        std::vector<int> pos(dptr.begin(), dptr.end() - 1);
        for (size_t t = 0; t < tgt.size(); ++t) didx[pos[tgt[t]]++] = (int)tslot[t];
    }
    DeviceGuard dg(d->device);
    vpp_amr a = new vpp_amr_s();
    a->desc = *d;
    a->k = k;
    a->nc = Nc;
    a->nf = Nf;
    a->n = Nc + Nf;
    a->nfree = nfree;
    vpp_status st;
    if ((st = upload(&a->d_cells, cells, "amr cells")) || (st = upload(&a->d_fkind, fkind, "amr node kinds")) ||
        (st = upload(&a->d_cptr, cptr, "amr constraint lists")) || (st = upload(&a->d_ccol, ccol, "amr constraints")) ||
        (st = upload(&a->d_cw, cwv, "amr weights")) || (st = upload(&a->d_ident, ident, "amr identity rows")) ||
        (st = dev_alloc(&a->phi, a->n, "amr phi")) || (st = dev_alloc(&a->diag, a->n, "amr diag")) ||
        (st = dev_alloc(&a->inv64, a->n, "amr inverse diag")) || (st = dev_alloc(&a->inv32, a->n, "amr inverse diag")) ||
        (st = upload(&a->d_nptr, nptr, "amr entry lists")) || (st = upload(&a->d_nidx, nidx, "amr entry slots")) ||
        (st = upload(&a->d_nw, nwv, "amr entry weights")) || (st = upload(&a->d_soff, soff, "amr source slots")) ||
        (st = upload(&a->d_dptr, dptr, "amr diagonal lists")) || (st = upload(&a->d_didx, didx, "amr diagonal slots")) ||
        (st = dev_alloc(&a->d_scratch, (size_t)std::max<int64_t>(ncell_act * n3 + soff[ncell_act], 1),
                        "amr cell results"))) {
        amr_free(a);
        return st;
    }
    if (hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking) != hipSuccess) {
        amr_free(a);
        return fail(VPP_ERR_HIP, "hipStreamCreate failed");
    }
    AmrArgs& g = a->args;
    g.mc = make_mesh_args(*d);
    vpp_desc fd = *d;
    for (int i = 0; i < 3; ++i) fd.ncells[i] = 2 * d->ncells[i];
    g.mf = make_mesh_args(fd);
    for (int i = 0; i < 3; ++i) g.mc.ntile[i] = g.mf.ntile[i] = 1;
    g.nc = Nc;
    g.n = a->n;
    g.cells = a->d_cells;
    g.ncells = (int)cells.size();
    g.fkind = a->d_fkind;
    g.cptr = a->d_cptr;
    g.ccol = a->d_ccol;
    g.cw = a->d_cw;
    g.ident = a->d_ident;
    g.scratch = a->d_scratch;
    g.nptr = a->d_nptr;
    g.nidx = a->d_nidx;
    g.nw = a->d_nw;
    g.soff = a->d_soff;
    g.dptr = a->d_dptr;
    g.didx = a->d_didx;
    g.nfree_slots = ncell_act * n3;
    *out = a;
    return VPP_OK;
}

extern "C" vpp_status vpp_amr_destroy(vpp_amr a)
{
    if (!a) return fail(VPP_ERR_INVALID_ARG, "null argument");
    DeviceGuard dg(a->desc.device);
    (void)hipDeviceSynchronize();
    amr_free(a);
    return VPP_OK;
}

extern "C" int64_t vpp_amr_num_dofs(vpp_amr a) { return a ? a->n : -1; }
extern "C" int64_t vpp_amr_num_free(vpp_amr a) { return a ? a->nfree : -1; }

extern "C" vpp_status vpp_amr_set_phi(vpp_amr a, const double* phi, void* stream)
{
    if (!a || !phi) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, phi);
    DeviceGuard dg(a->desc.device);
    hipStream_t s = (hipStream_t)stream;
    VPP_HIP(hipMemcpyAsync(a->phi, phi, a->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    VPP_HIP(launch_amr_diag(a->k, a->args, a->phi, a->diag, a->inv64, a->inv32, s));
    a->phi_set = true;
    return VPP_OK;
}

extern "C" vpp_status vpp_amr_apply(vpp_amr a, const double* x, double* y, void* stream)
{
    if (!a || !x || !y) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, x, y);
    if ((const void*)x == y) return fail(VPP_ERR_INVALID_ARG, "x and y must not alias");
    if (!a->phi_set) return fail(VPP_ERR_STATE, "vpp_amr_set_phi has not been called");
    DeviceGuard dg(a->desc.device);
    VPP_HIP(launch_amr_apply(a->k, a->args, a->phi, x, y, (hipStream_t)stream));
    return VPP_OK;
}

extern "C" vpp_status vpp_amr_diagonal(vpp_amr a, double* diag, void* stream)
{
    if (!a || !diag) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, diag);
    if (!a->phi_set) return fail(VPP_ERR_STATE, "vpp_amr_set_phi has not been called");
    DeviceGuard dg(a->desc.device);
    VPP_HIP(hipMemcpyAsync(diag, a->diag, a->n * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return VPP_OK;
}

extern "C" vpp_status vpp_amr_cg_solve(vpp_amr a, const double* b, double* x, const vpp_cg_opts* o,
                                       vpp_cg_info* info, void* stream)
{
    if (!a || !b || !x || !o) return fail(VPP_ERR_INVALID_ARG, "null argument");
    VPP_ALIGNED(8, b, x);
    if (!(o->rtol >= 0.0) || !(o->atol >= 0.0) || o->max_iter < 0)
        return fail(VPP_ERR_INVALID_ARG, "CG options out of range");
    if (o->precision != VPP_FP64) return fail(VPP_ERR_UNSUPPORTED, "the refined-mesh solver runs in FP64");
    if (!a->phi_set) return fail(VPP_ERR_STATE, "vpp_amr_set_phi has not been called");
    DeviceGuard dg(a->desc.device);
    if (!a->w) {
        ReinitWork* w = new ReinitWork();
        const size_t n = (size_t)a->n;
        vpp_status st;
        if ((st = dev_alloc(&w->b, n, "amr cg b")) || (st = dev_alloc(&w->r, n, "amr cg r")) ||
            (st = dev_alloc(&w->p, n, "amr cg p")) || (st = dev_alloc(&w->q, n, "amr cg q")) ||
            (st = dev_alloc(&w->red, kRedDoubles, "amr cg partials")) ||
            (st = dev_alloc(&w->dot, kMaxRedBlocks, "amr cg dot partials")) || (st = dev_alloc(&w->rr, 1, "norm")) ||
            (st = dev_alloc(&w->st, 1, "amr cg state"))) {
            free_reinit(w);
            return st;
        }
        if (hipHostMalloc((void**)&w->hst, sizeof(CgState), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&w->hrr, sizeof(double), hipHostMallocDefault) != hipSuccess) {
            free_reinit(w);
            return fail(VPP_ERR_OUT_OF_MEMORY, "amr cg host mirrors");
        }
        a->w = w;
    }
    VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
    hipStream_t s = a->stream;
    ReinitWork& w = *a->w;
    const int64_t n = a->n;
    const int one[3] = {1, 1, 1};
    const SharedEnum none = shared_enum(a->args.mc, a->k, one);   // no shared nodes: q is used as it is
    const int gdot = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxRedBlocks, (n + 1023) / 1024));
    VPP_HIP(launch_amr_apply(a->k, a->args, a->phi, x, w.q, s));
    CgState* hs = w.hst;
    std::memset(hs, 0, sizeof(CgState));
    VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
    VPP_HIP(launch_cg_init<double>(w.st, w.red, b, w.q, w.r, w.p, a->inv64, n, s));
    VPP_HIP(hipMemcpyAsync(hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    vpp_cg_info inf{};
    inf.deflation_first_change = -1.0;
    const double r0 = std::sqrt(hs->rr_last), rz0 = hs->rz[0];
    const double thr = std::max(o->rtol * r0, o->atol);
    inf.rel_residual = r0 > 0 ? 1.0 : 0.0;
    bool iterate = true;
    if (!std::isfinite(r0) || !std::isfinite(rz0)) {
        inf.status = VPP_ERR_BREAKDOWN;
        iterate = false;
    } else if (r0 == 0.0 || r0 < o->atol) {
        inf.status = VPP_OK;
        iterate = false;
    } else if (o->max_iter == 0) {
        inf.status = VPP_ERR_NOT_CONVERGED;
        iterate = false;
    }
    if (iterate) {
        CgState init{};
        init.rz[0] = rz0;
        init.tol2 = thr * thr;
        init.max_iter = o->max_iter;
        *hs = init;
        VPP_HIP(hipMemcpyAsync(w.st, hs, sizeof(CgState), hipMemcpyHostToDevice, s));
        const int chunk = o->check_every > 0 ? o->check_every : 32;
        for (int done = 0; done < o->max_iter + chunk;) {
            for (int it = 0; it < chunk; ++it, ++done) {
                const int par = done & 1;
                VPP_HIP(launch_amr_apply(a->k, a->args, a->phi, w.p, w.q, s));
                VPP_HIP(launch_dot_partials(w.p, w.q, n, w.dot, gdot, s));
                VPP_HIP(launch_cg_assemble_update<double>(w.st, par, w.red, w.dot, gdot, a->args.mc, none, nullptr, 0,
                                                          w.r, w.q, a->inv64, n, s));
                VPP_HIP(launch_cg_pupdate<double>(w.st, par, w.red, x, w.r, w.p, a->inv64, n, s));
            }
            VPP_HIP(hipMemcpyAsync(hs, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            VPP_HIP(hipStreamSynchronize(s));
            if (hs->halt[0] || hs->halt[1]) break;
        }
        inf.iterations = hs->iters;
        inf.rel_residual = std::sqrt(hs->rr_last) / r0;
        if (hs->breakdown) inf.status = VPP_ERR_BREAKDOWN;
        else if (hs->rr_last < init.tol2) inf.status = VPP_OK;
        else inf.status = VPP_ERR_NOT_CONVERGED;
    }
    VPP_HIP(launch_amr_apply(a->k, a->args, a->phi, x, w.q, s));
    VPP_HIP(launch_residual(b, w.q, nullptr, n, w.red, w.rr, s));
    VPP_HIP(hipMemcpyAsync(w.hrr, w.rr, sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    inf.true_rel_residual = r0 > 0 ? std::sqrt(*w.hrr) / r0 : 0.0;
    if (info) *info = inf;
    if (inf.status == VPP_ERR_NOT_CONVERGED) return fail(VPP_ERR_NOT_CONVERGED, "CG did not converge");
    if (inf.status == VPP_ERR_BREAKDOWN) return fail(VPP_ERR_BREAKDOWN, "CG breakdown (p.Ap <= 0 or non-finite)");
    return VPP_OK;
}

extern "C" {

static void put_config(vpp_problem p, int prec, const LaunchCfg& c)
{
    if (prec == VPP_FP32) {
        p->cfg32 = c;
        set_tiles(p->m32, c);
    } else {
        p->cfg = c;
        set_tiles(p->m, c);
    }
}

vpp_status vpp_get_config_for(vpp_problem p, int32_t precision, vpp_kernel_config* cfg)
{
    if (!p || !cfg) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (precision != VPP_FP64 && precision != VPP_FP32)
        return fail(VPP_ERR_INVALID_ARG, "precision must be VPP_FP64 or VPP_FP32");
    const LaunchCfg& c = precision == VPP_FP32 ? p->cfg32 : p->cfg;
    cfg->variant = c.variant;
    for (int d = 0; d < 3; ++d) cfg->tile[d] = c.tile[d];
    return VPP_OK;
}

vpp_status vpp_set_config_for(vpp_problem p, int32_t precision, const vpp_kernel_config* cfg)
{
    if (!p || !cfg) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (precision != VPP_FP64 && precision != VPP_FP32)
        return fail(VPP_ERR_INVALID_ARG, "precision must be VPP_FP64 or VPP_FP32");
    LaunchCfg c{cfg->variant, {cfg->tile[0], cfg->tile[1], cfg->tile[2]}};
    if (!config_ok(p, c))
        return fail(VPP_ERR_UNSUPPORTED, p->m.mass != 0.0 ? "kernel configuration not available with the mass shift"
                                                          : "kernel configuration not available");
    DeviceGuard dg(p->desc.device);
    if (p->stream) VPP_HIP(hipStreamSynchronize(p->stream));
    put_config(p, precision, c);
    return ensure_apply_scratch(p);
}

vpp_status vpp_get_config(vpp_problem p, vpp_kernel_config* cfg) { return vpp_get_config_for(p, VPP_FP64, cfg); }

vpp_status vpp_set_config(vpp_problem p, const vpp_kernel_config* cfg)
{
    vpp_status s = vpp_set_config_for(p, VPP_FP64, cfg);
    if (s) return s;
    return vpp_set_config_for(p, VPP_FP32, cfg);
}

int32_t vpp_config_candidates(int32_t degree, vpp_kernel_config* out, int32_t cap)
{
    LaunchCfg tmp[64];
    const int n = list_apply_configs(degree, tmp, 64);
    for (int i = 0; i < n && i < cap && out; ++i) {
        out[i].variant = tmp[i].variant;
        for (int d = 0; d < 3; ++d) out[i].tile[d] = tmp[i].tile[d];
    }
    return n;
}

// Times every candidate configuration of one precision and keeps the fastest.
// Each timed apply follows a write of `flush` (larger than the last-level
// cache), so x, phi and y come from HBM as for applies on streaming data and
// for problems larger than the cache; without a flush buffer the applies run
// back to back.
static vpp_status tune_precision(vpp_problem p, int prec, const char* cache_path, double* flush, int64_t nflush)
{
    const bool mass = p->m.mass != 0.0;
    const std::string key = size_bucket_key(prec == VPP_FP32 ? (mass ? "apply32m/hbm" : "apply32/hbm")
                                                             : (mass ? "applym/hbm" : "apply/hbm"),
                                            p->k, p->N);
    LaunchCfg c;
    if (cache_lookup(cache_path, key, &c) && config_ok(p, c)) {
        put_config(p, prec, c);
        return ensure_apply_scratch(p);
    }
    vpp_status st;
    if ((st = ensure_work(p, prec == VPP_FP32))) return st;
    hipStream_t s = p->stream;
    CgWork& w = p->w;
    if (prec == VPP_FP32) VPP_HIP(launch_fill<float>(w.p32, p->N, 1.0f, s));
    else VPP_HIP(launch_fill<double>(w.x, p->N, 1.0, s));
    LaunchCfg cands[64];
    const int n = std::min(config_list(p, cands, 64), 64);
    constexpr int reps = 6;
    hipEvent_t ev[2 * reps] = {};
    for (int r = 0; r < 2 * reps && !st; ++r)
        if (hipEventCreate(&ev[r]) != hipSuccess) st = fail(VPP_ERR_HIP, "hipEventCreate failed");
    double best = 1e300;
    LaunchCfg best_cfg = prec == VPP_FP32 ? p->cfg32 : p->cfg;
    auto one = [&]() {
        return prec == VPP_FP32 ? do_apply32(p, w.p32, w.q32, nullptr, nullptr, s)
                                : do_apply64(p, w.x, w.q, nullptr, nullptr, s);
    };
    auto hip = [&](hipError_t e) {
        if (e != hipSuccess && !st) st = fail(VPP_ERR_HIP, hipGetErrorString(e));
        return st == VPP_OK;
    };
    for (int i = 0; i < n && !st; ++i) {
        put_config(p, prec, cands[i]);
        if ((st = ensure_apply_scratch(p))) break;
        if ((st = one())) break;
        for (int r = 0; r < reps && !st; ++r) {
            if (flush && !hip(launch_fill<double>(flush, nflush, (double)r, s))) break;
            if (!hip(hipEventRecord(ev[2 * r], s))) break;
            if ((st = one())) break;
            hip(hipEventRecord(ev[2 * r + 1], s));
        }
        if (st || !hip(hipEventSynchronize(ev[2 * reps - 1]))) break;
        double us = 0.0;
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            if (!hip(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]))) break;
            us += 1000.0 * ms / reps;
        }
        if (!st && us < best) {
            best = us;
            best_cfg = cands[i];
        }
    }
    for (int r = 0; r < 2 * reps; ++r)
        if (ev[r]) (void)hipEventDestroy(ev[r]);
    put_config(p, prec, best_cfg);
    if (st) return st;
    cache_store(cache_path, key, best_cfg, best);
    return ensure_apply_scratch(p);
}

vpp_status vpp_tune(vpp_problem p, const char* cache_path, void* stream)
{
    if (!p) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called");
    DeviceGuard dg(p->desc.device);
    VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
    // cache flush buffer: twice the 256 MB last-level cache (skipped if it
    // cannot be allocated)
    const int64_t nflush = (int64_t)64 << 20;
    double* flush = nullptr;
    if (hipMalloc((void**)&flush, (size_t)nflush * sizeof(double)) != hipSuccess) {
        flush = nullptr;
        (void)hipGetLastError();
    }
    vpp_status st = tune_precision(p, VPP_FP64, cache_path, flush, nflush);
    if (!st) st = tune_precision(p, VPP_FP32, cache_path, flush, nflush);
    if (flush) {
        (void)hipStreamSynchronize(p->stream);
        (void)hipFree(flush);
    }
    return st;
}

// ---------------------------------------------------------------------------
// Batches

static vpp_status batch_build_table(vpp_batch b)
{
    std::vector<BatchProblem> tab(b->probs.size());
    int item = 0, rhs = 0, dot = 0;
    int64_t part = 0;
    for (size_t i = 0; i < b->probs.size(); ++i) {
        MeshArgs m = b->probs[i]->m;
        set_tiles(m, b->cfg);
        tab[i].m = m;
        tab[i].phi = b->probs[i]->phi64;
        tab[i].tile_begin = item;
        tab[i].nrhs = b->nrhs[i];
        tab[i].rhs_begin = rhs;
        tab[i].part_begin = part;
        tab[i].nshared = shared_stride(m);
        tab[i].se = shared_enum(m, b->k, b->cfg.tile);
        tab[i].ntiles = tile_count(m);
        tab[i].dot_begin = dot;
        dot += tab[i].ntiles * b->nrhs[i];
        item += batch_items(b->k, tab[i].ntiles, b->nrhs[i]);
        rhs += b->nrhs[i];
        part += 8 * std::max<int64_t>(1, tab[i].nshared) * b->nrhs[i];
    }
    b->nitems = item;
    if ((size_t)part > b->part_n) {
        dev_free(b->d_part);
        b->part_n = 0;
        vpp_status st = dev_alloc(&b->d_part, (size_t)part, "batch partials");
        if (st) return st;
        b->part_n = (size_t)part;
    }
    VPP_HIP(hipMemcpy(b->d_probs, tab.data(), tab.size() * sizeof(BatchProblem), hipMemcpyHostToDevice));
    b->tab = tab;
    int per_cu = batch_blocks_per_cu(b->cfg, b->k);
    if (per_cu < 1) per_cu = 1;
    hipDeviceProp_t prop;
    VPP_HIP(hipGetDeviceProperties(&prop, b->device));
    b->nblocks = std::max(1, std::min(prop.multiProcessorCount * per_cu, b->nitems));
    return VPP_OK;
}

static int batch_any_mass(vpp_batch b)
{
    for (const auto& t : b->tab)
        if (t.m.mass != 0.0) return 1;
    return 0;
}

static vpp_status batch_build_graph(vpp_batch b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    hipGraph_t g = nullptr;
    VPP_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    BatchArgs ba{b->d_probs, (int)b->probs.size(), b->nitems, b->d_x, b->d_y, b->d_part, b->d_queue,
                 b->probs[0]->desc.heaviside, nullptr, 0, nullptr};
    ba.any_mass = batch_any_mass(b);
    hipError_t err = launch_batch_apply(b->cfg, b->k, ba, b->nblocks, b->total_rhs, false, b->stream);
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(VPP_ERR_HIP, std::string("batch graph capture: ") + hipGetErrorString(err));
    }
    VPP_HIP(e2);
    hipError_t e3 = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    VPP_HIP(e3);
    return VPP_OK;
}

static vpp_status batch_set_pointers(vpp_batch b, const double* const* x, double* const* y)
{
    bool same = !b->cur_x.empty();
    for (int i = 0; same && i < b->total_rhs; ++i) same = b->cur_x[i] == x[i] && b->cur_y[i] == y[i];
    if (same) return VPP_OK;
    b->cur_x.assign(x, x + b->total_rhs);
    b->cur_y.assign(y, y + b->total_rhs);
    VPP_HIP(hipMemcpy(b->d_x, x, b->total_rhs * sizeof(double*), hipMemcpyHostToDevice));
    VPP_HIP(hipMemcpy(b->d_y, y, b->total_rhs * sizeof(double*), hipMemcpyHostToDevice));
    return batch_build_graph(b);
}

static vpp_status batch_tune(vpp_batch b, const char* cache_path)
{
    const std::string key = size_bucket_key("batch", b->k, b->total_dofs);
    LaunchCfg c;
    if (cache_lookup(cache_path, key, &c) && batch_blocks_per_cu(c, b->k) > 0) {
        b->cfg = c;
        return batch_build_table(b);
    }
    // time every candidate on scratch vectors
    std::vector<double*> xs(b->total_rhs, nullptr), ys(b->total_rhs, nullptr);
    vpp_status st = VPP_OK;
    int r = 0;
    for (size_t i = 0; i < b->probs.size() && !st; ++i)
        for (int j = 0; j < b->nrhs[i] && !st; ++j, ++r) {
            if ((st = dev_alloc(&xs[r], b->probs[i]->N, "tune x")) ||
                (st = dev_alloc(&ys[r], b->probs[i]->N, "tune y")))
                break;
            if (launch_fill<double>(xs[r], b->probs[i]->N, 1.0, b->stream) != hipSuccess)
                st = fail(VPP_ERR_HIP, "fill");
        }
    LaunchCfg all[16], cands[16];
    const int na = std::min(list_batch_configs(b->k, all, 16), 16);
    int nc = 0;
    for (int i = 0; i < na; ++i)
        if (batch_blocks_per_cu(all[i], b->k) > 0) cands[nc++] = all[i];
    if (nc == 0) st = fail(VPP_ERR_UNSUPPORTED, "no batch kernel configuration for this degree");
    double best = 1e300;
    LaunchCfg best_cfg = nc ? cands[0] : LaunchCfg{4, {8, 8, 4}};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(VPP_ERR_HIP, "event");
    for (int i = 0; i < nc && !st; ++i) {
        b->cfg = cands[i];
        if ((st = batch_build_table(b))) break;
        b->cur_x.clear();
        if ((st = batch_set_pointers(b, xs.data(), ys.data()))) break;
        (void)hipGraphLaunch(b->graph, b->stream);
        (void)hipEventRecord(e0, b->stream);
        const int reps = 5;
        for (int k = 0; k < reps; ++k) (void)hipGraphLaunch(b->graph, b->stream);
        (void)hipEventRecord(e1, b->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = fail(VPP_ERR_HIP, "tuning run failed");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double us = 1000.0 * ms / reps;
        if (us < best) {
            best = us;
            best_cfg = cands[i];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->stream);
    for (auto* v : xs) dev_free(v);
    for (auto* v : ys) dev_free(v);
    b->cur_x.clear();
    b->cur_y.clear();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    if (st) return st;
    b->cfg = best_cfg;
    cache_store(cache_path, key, best_cfg, best);
    return batch_build_table(b);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched FP64 PCG.  A system (one (problem, rhs) pair) whose mesh has at
// least kLockstepMaxDofs unknowns fills the GPU on its own and is solved with
// the single-problem solver and its tuned kernels.  All other systems advance
// in lockstep, one iteration being the persistent batched apply (tile kernel
// with per-tile p.Ap partials) and the batched update and search-direction
// update; a system that has stopped is skipped by all three.  Each lockstep
// system's reductions have the workgroup count and summation order of a single
// solve on the batch's tiles.
constexpr int64_t kLockstepMaxDofs = int64_t(1) << 20;

static void batch_cg_free(vpp_batch b)
{
    if (b->cg_graph) (void)hipGraphExecDestroy(b->cg_graph);
    b->cg_graph = nullptr;
    b->cg_graph_iters = 0;
    dev_free(b->cg_probs);
    dev_free(b->cg_x); dev_free(b->cg_r); dev_free(b->cg_p); dev_free(b->cg_q);
    dev_free(b->cg_tx); dev_free(b->cg_tp); dev_free(b->cg_tq);
    dev_free(b->cg_st); dev_free(b->cg_red); dev_free(b->cg_dot); dev_free(b->cg_rr); dev_free(b->cg_sys);
    if (b->cg_hst) (void)hipHostFree(b->cg_hst);
    if (b->cg_hrr) (void)hipHostFree(b->cg_hrr);
    b->cg_hst = nullptr;
    b->cg_hrr = nullptr;
    b->cg_prob.clear();
    b->cg_index.clear();
    b->cg_nsys = 0;
}

static vpp_status batch_cg_setup(vpp_batch b)
{
    if (!b->cg_index.empty()) return VPP_OK;
    // the lockstep problems, renumbered: items, rhs and dot partials of the subset
    std::vector<BatchProblem> tab;
    int item = 0, rhs = 0, ndot = 0;
    b->cg_index.assign(b->total_rhs, -1);
    for (size_t i = 0, k = 0; i < b->probs.size(); k += b->nrhs[i], ++i) {
        if (b->probs[i]->N >= kLockstepMaxDofs) continue;
        BatchProblem P = b->tab[i];
        P.tile_begin = item;
        P.rhs_begin = rhs;
        P.dot_begin = ndot;
        for (int j = 0; j < b->nrhs[i]; ++j) b->cg_index[k + j] = rhs + j;
        item += batch_items(b->k, P.ntiles, P.nrhs);
        rhs += P.nrhs;
        ndot += P.ntiles * P.nrhs;
        tab.push_back(P);
        b->cg_prob.push_back((int)i);
    }
    const int S = rhs;
    b->cg_nsys = S;
    b->cg_nitems = item;
    if (S == 0) return VPP_OK;
    int per_cu = batch_blocks_per_cu(b->cfg, b->k);
    b->cg_nblocks = std::max(1, std::min(device_cu_count() * std::max(1, per_cu), item));
    b->cg_off.assign(S + 1, 0);
    for (size_t t = 0, sidx = 0; t < tab.size(); ++t)
        for (int j = 0; j < tab[t].nrhs; ++j, ++sidx)   // 512-byte aligned system vectors
            b->cg_off[sidx + 1] = b->cg_off[sidx] + ((b->probs[b->cg_prob[t]]->N + 63) & ~int64_t(63));
    const size_t nv = (size_t)b->cg_off[S];
    vpp_status st;
    if ((st = dev_alloc(&b->cg_probs, tab.size(), "batch cg table")) ||
        (st = dev_alloc(&b->cg_x, nv, "batch cg x")) || (st = dev_alloc(&b->cg_r, nv, "batch cg r")) ||
        (st = dev_alloc(&b->cg_p, nv, "batch cg p")) || (st = dev_alloc(&b->cg_q, nv, "batch cg q")) ||
        (st = dev_alloc(&b->cg_tx, S, "batch cg table")) || (st = dev_alloc(&b->cg_tp, S, "batch cg table")) ||
        (st = dev_alloc(&b->cg_tq, S, "batch cg table")) || (st = dev_alloc(&b->cg_st, S, "batch cg states")) ||
        (st = dev_alloc(&b->cg_red, (size_t)S * kRedDoubles, "batch cg partials")) ||
        (st = dev_alloc(&b->cg_dot, (size_t)std::max(1, ndot), "batch cg dot partials")) ||
        (st = dev_alloc(&b->cg_rr, S, "batch cg norms")) || (st = dev_alloc(&b->cg_sys, S, "batch cg table"))) {
        batch_cg_free(b);
        return st;
    }
    if (hipHostMalloc((void**)&b->cg_hst, S * sizeof(CgState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->cg_hrr, S * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        batch_cg_free(b);
        return fail(VPP_ERR_OUT_OF_MEMORY, "batch cg host mirrors");
    }
    std::vector<double*> tx(S), tp(S), tq(S);
    std::vector<CgSystem<double>> sys(S);
    int blk = 0;
    for (size_t t = 0, sidx = 0; t < tab.size(); ++t)
        for (int j = 0; j < tab[t].nrhs; ++j, ++sidx) {
            const BatchProblem& P = tab[t];
            const vpp_problem prob = b->probs[b->cg_prob[t]];
            const int64_t off = b->cg_off[sidx];
            tx[sidx] = b->cg_x + off;
            tp[sidx] = b->cg_p + off;
            tq[sidx] = b->cg_q + off;
            CgSystem<double>& y = sys[sidx];
            y.st = b->cg_st + sidx;
            y.red = b->cg_red + sidx * kRedDoubles;
            y.e = P.se;
            y.bcmask = P.m.bcmask;
            y.part = b->d_part + P.part_begin + (int64_t)j * 8 * P.nshared;
            y.stride = P.nshared;
            y.dot_part = b->cg_dot + P.dot_begin + j * P.ntiles;
            y.ndot = P.ntiles;
            y.x = tx[sidx];
            y.r = b->cg_r + off;
            y.p = tp[sidx];
            y.q = tq[sidx];
            y.invd = prob->inv64;
            y.n = prob->N;
            y.blk_begin = blk;
            y.nblk = cg_update_blocks(y.n);
            blk += y.nblk;
        }
    b->cg_blocks = blk;
    if (hipMemcpy(b->cg_probs, tab.data(), tab.size() * sizeof(BatchProblem), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cg_tx, tx.data(), S * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cg_tp, tp.data(), S * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cg_tq, tq.data(), S * sizeof(double*), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cg_sys, sys.data(), S * sizeof(CgSystem<double>), hipMemcpyHostToDevice) != hipSuccess) {
        batch_cg_free(b);
        return fail(VPP_ERR_HIP, "batch cg tables");
    }
    return VPP_OK;
}

// Record `iters` (even) lockstep PCG iterations into a graph.
static vpp_status batch_cg_graph(vpp_batch b, int iters)
{
    if (b->cg_graph && b->cg_graph_iters == iters) return VPP_OK;
    if (b->cg_graph) (void)hipGraphExecDestroy(b->cg_graph);
    b->cg_graph = nullptr;
    hipGraph_t g = nullptr;
    VPP_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int it = 0; it < iters && err == hipSuccess; ++it) {
        const int par = it & 1;
        BatchArgs ba{b->cg_probs, (int)b->cg_prob.size(), b->cg_nitems, b->cg_tp, b->cg_tq, b->d_part, b->d_queue,
                     b->probs[0]->desc.heaviside, b->cg_st, par, b->cg_dot};
        ba.any_mass = batch_any_mass(b);
        err = launch_batch_apply(b->cfg, b->k, ba, b->cg_nblocks, b->cg_nsys, true, b->stream);
        if (err == hipSuccess)
            err = launch_cg_batch_step(b->cg_sys, b->cg_nsys, b->cg_blocks, par, b->d_queue, b->stream);
    }
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(VPP_ERR_HIP, std::string("batch cg graph capture: ") + hipGetErrorString(err));
    }
    VPP_HIP(e2);
    hipError_t e3 = hipGraphInstantiate(&b->cg_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    VPP_HIP(e3);
    b->cg_graph_iters = iters;
    return VPP_OK;
}

// q = A x of every lockstep system (plain batched apply, assembly included).
static vpp_status batch_cg_apply_x(vpp_batch b)
{
    BatchArgs ba{b->cg_probs, (int)b->cg_prob.size(), b->cg_nitems, b->cg_tx, b->cg_tq, b->d_part, b->d_queue,
                 b->probs[0]->desc.heaviside, nullptr, 0, nullptr};
    ba.any_mass = batch_any_mass(b);
    VPP_HIP(launch_batch_apply(b->cfg, b->k, ba, b->cg_nblocks, b->cg_nsys, false, b->stream));
    return VPP_OK;
}

// Lockstep PCG of the systems k with cg_index[k] >= 0; rhs, x, info indexed by k.
static vpp_status batch_pcg64_lockstep(vpp_batch b, const double* const* rhs, double* const* x, const vpp_cg_opts& o,
                                       int chunk, std::vector<vpp_cg_info>& info)
{
    vpp_status st;
    const int S = b->cg_nsys;
    if (S == 0) return VPP_OK;
    if ((st = batch_cg_graph(b, chunk))) return st;
    hipStream_t s = b->stream;
    std::vector<int> sys_k(S);           // lockstep system -> caller's system index
    std::vector<int64_t> n(S);
    std::vector<const double*> inv(S);
    for (size_t i = 0, k = 0; i < b->probs.size(); ++i)
        for (int j = 0; j < b->nrhs[i]; ++j, ++k) {
            const int l = b->cg_index[k];
            if (l < 0) continue;
            sys_k[l] = (int)k;
            n[l] = b->probs[i]->N;
            inv[l] = b->probs[i]->inv64;
        }
    for (int l = 0; l < S; ++l)
        VPP_HIP(hipMemcpyAsync(b->cg_x + b->cg_off[l], x[sys_k[l]], n[l] * sizeof(double), hipMemcpyDeviceToDevice, s));
    if ((st = batch_cg_apply_x(b))) return st;
    CgState* hs = b->cg_hst;
    std::memset(hs, 0, S * sizeof(CgState));
    VPP_HIP(hipMemcpyAsync(b->cg_st, hs, S * sizeof(CgState), hipMemcpyHostToDevice, s));
    for (int l = 0; l < S; ++l) {
        const int64_t off = b->cg_off[l];
        VPP_HIP(launch_cg_init<double>(b->cg_st + l, b->cg_red + (size_t)l * kRedDoubles, rhs[sys_k[l]],
                                       b->cg_q + off, b->cg_r + off, b->cg_p + off, inv[l], n[l], s));
    }
    VPP_HIP(hipMemcpyAsync(hs, b->cg_st, S * sizeof(CgState), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    std::vector<double> r0(S), tol2(S);
    std::vector<bool> decided(S, true);
    for (int l = 0; l < S; ++l) {
        vpp_cg_info& inf = info[sys_k[l]];
        const double rr0 = hs[l].rr_last, rz0 = hs[l].rz[0];
        r0[l] = std::sqrt(rr0);
        const double thr = std::max(o.rtol * r0[l], o.atol);
        tol2[l] = thr * thr;
        inf = vpp_cg_info{};
        inf.deflation_first_change = -1.0;
        inf.rel_residual = r0[l] > 0 ? 1.0 : 0.0;
        CgState init{};
        init.rz[0] = rz0;
        init.tol2 = tol2[l];
        init.max_iter = o.max_iter;
        if (!std::isfinite(rr0) || !std::isfinite(rz0)) {
            inf.status = VPP_ERR_BREAKDOWN;
            init.breakdown = 1;
            init.halt[0] = 1;
        } else if (r0[l] == 0.0 || r0[l] < o.atol) {
            inf.status = VPP_OK;
            init.halt[0] = 1;   // converged before any iteration
        } else if (o.max_iter == 0) {
            inf.status = VPP_ERR_NOT_CONVERGED;
            init.halt[0] = 1;
        } else {
            decided[l] = false;
        }
        hs[l] = init;
    }
    VPP_HIP(hipMemcpyAsync(b->cg_st, hs, S * sizeof(CgState), hipMemcpyHostToDevice, s));
    const int max_launch = o.max_iter / chunk + 2;
    for (int launch = 0; launch < max_launch; ++launch) {
        bool all = true;
        for (int l = 0; l < S && all; ++l) all = hs[l].halt[0] || hs[l].halt[1];
        if (all) break;
        VPP_HIP(hipGraphLaunch(b->cg_graph, s));
        VPP_HIP(hipMemcpyAsync(hs, b->cg_st, S * sizeof(CgState), hipMemcpyDeviceToHost, s));
        VPP_HIP(hipStreamSynchronize(s));
    }
    for (int l = 0; l < S; ++l) {
        if (decided[l]) continue;
        vpp_cg_info& inf = info[sys_k[l]];
        inf.iterations = hs[l].iters;
        inf.rel_residual = std::sqrt(hs[l].rr_last) / r0[l];
        if (hs[l].breakdown) inf.status = VPP_ERR_BREAKDOWN;
        else if (hs[l].rr_last < tol2[l]) inf.status = VPP_OK;
        else inf.status = VPP_ERR_NOT_CONVERGED;
    }
    // true residuals ||b - A x|| in FP64, then the solutions back to the caller
    if ((st = batch_cg_apply_x(b))) return st;
    for (int l = 0; l < S; ++l) {
        const int64_t off = b->cg_off[l];
        VPP_HIP(launch_residual(rhs[sys_k[l]], b->cg_q + off, nullptr, n[l], b->cg_red + (size_t)l * kRedDoubles,
                                b->cg_rr + l, s));
        VPP_HIP(hipMemcpyAsync(x[sys_k[l]], b->cg_x + off, n[l] * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    VPP_HIP(hipMemcpyAsync(b->cg_hrr, b->cg_rr, S * sizeof(double), hipMemcpyDeviceToHost, s));
    VPP_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < S; ++l)
        info[sys_k[l]].true_rel_residual = r0[l] > 0 ? std::sqrt(b->cg_hrr[l]) / r0[l] : 0.0;
    return VPP_OK;
}

extern "C" {

vpp_status vpp_batch_create(const vpp_problem* probs, const int32_t* nrhs, int32_t nprob, const char* tune_cache,
                            vpp_batch* out)
{
    if (!probs || !nrhs || !out || nprob < 1) return fail(VPP_ERR_INVALID_ARG, "null argument or empty batch");
    *out = nullptr;
    const int k = probs[0] ? probs[0]->k : 0;
    const int dev = probs[0] ? probs[0]->desc.device : 0;
    for (int i = 0; i < nprob; ++i) {
        if (!probs[i]) return fail(VPP_ERR_INVALID_ARG, "null problem");
        if (probs[i]->k != k) return fail(VPP_ERR_UNSUPPORTED, "all problems of a batch must share the degree");
        if (probs[i]->desc.device != dev) return fail(VPP_ERR_UNSUPPORTED, "all problems must be on one device");
        if (probs[i]->desc.heaviside != probs[0]->desc.heaviside)
            return fail(VPP_ERR_UNSUPPORTED, "all problems of a batch must share the Heaviside law");
        if (arith_law(probs[i]->desc))
            return fail(VPP_ERR_UNSUPPORTED, "batches run the reciprocal density mean (Eq. rhoEff) only");
        if (!probs[i]->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called for every problem");
        if (nrhs[i] < 1) return fail(VPP_ERR_INVALID_ARG, "nrhs must be >= 1");
    }
    if (k != 2 && k != 3) return fail(VPP_ERR_UNSUPPORTED, "batched apply is available for degrees 2 and 3");
    DeviceGuard dg(dev);
    vpp_batch b = new vpp_batch_s();
    b->device = dev;
    b->k = k;
    b->probs.assign(probs, probs + nprob);
    b->nrhs.assign(nrhs, nrhs + nprob);
    for (int i = 0; i < nprob; ++i) {
        b->total_rhs += nrhs[i];
        b->total_dofs += probs[i]->N * nrhs[i];
    }
    b->cfg = LaunchCfg{4, {8, 4, 4}};
    vpp_status st;
    if ((st = dev_alloc(&b->d_probs, nprob, "batch table")) || (st = dev_alloc(&b->d_x, b->total_rhs, "batch x")) ||
        (st = dev_alloc(&b->d_y, b->total_rhs, "batch y")) || (st = dev_alloc(&b->d_queue, 1, "batch queue"))) {
        vpp_batch_destroy(b);
        return st;
    }
    // the work counter starts at zero; the assembly launch resets it after every pass
    if (hipMemset(b->d_queue, 0, sizeof(int)) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        vpp_batch_destroy(b);
        return fail(VPP_ERR_HIP, "batch set-up failed");
    }
    st = batch_tune(b, tune_cache);
    if (st) {
        vpp_batch_destroy(b);
        return st;
    }
    *out = b;
    return VPP_OK;
}

vpp_status vpp_batch_apply(vpp_batch b, const double* const* x, double* const* y, void* stream)
{
    if (!b || !x || !y) return fail(VPP_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < b->total_rhs; ++i) {
        if (!x[i] || !y[i]) return fail(VPP_ERR_INVALID_ARG, "null vector in batch");
        VPP_ALIGNED(8, x[i], y[i]);
        for (int j = 0; j < b->total_rhs; ++j)
            if ((const void*)x[i] == (const void*)y[j]) return fail(VPP_ERR_INVALID_ARG, "x and y must not alias");
    }
    DeviceGuard dg(b->device);
    // The pointer tables are refreshed synchronously, only when the caller's buffers change.
    bool changed = b->cur_x.empty() || !b->graph;
    for (int i = 0; !changed && i < b->total_rhs; ++i) changed = b->cur_x[i] != x[i] || b->cur_y[i] != y[i];
    if (changed) {
        VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
        VPP_HIP(hipStreamSynchronize(b->stream));
        vpp_status st = batch_set_pointers(b, x, y);
        if (st) return st;
    }
    VPP_HIP(hipGraphLaunch(b->graph, (hipStream_t)stream));
    return VPP_OK;
}

vpp_status vpp_batch_cg_solve(vpp_batch b, const double* const* rhs, double* const* x, const vpp_cg_opts* opts,
                              vpp_cg_info* info, void* stream)
{
    if (!b || !rhs || !x || !opts) return fail(VPP_ERR_INVALID_ARG, "null argument");
    if (!(opts->rtol >= 0.0) || !(opts->atol >= 0.0) || opts->max_iter < 0)
        return fail(VPP_ERR_INVALID_ARG, "tolerances must be >= 0 and max_iter >= 0");
    if (opts->precision != VPP_FP64 && opts->precision != VPP_MIXED)
        return fail(VPP_ERR_INVALID_ARG, "precision must be VPP_FP64 or VPP_MIXED");
    for (int i = 0; i < b->total_rhs; ++i)
        if (!rhs[i] || !x[i]) return fail(VPP_ERR_INVALID_ARG, "null vector in batch");
    for (int i = 0; i < b->total_rhs; ++i) VPP_ALIGNED(8, rhs[i], x[i]);
    for (auto* p : b->probs)
        if (!p->phi_set) return fail(VPP_ERR_STATE, "vpp_set_phi has not been called for every problem");
    DeviceGuard dg(b->device);
    std::vector<vpp_cg_info> inf(b->total_rhs);
    const bool fp64 = opts->precision == VPP_FP64;
    if (fp64) {
        int chunk = opts->check_every > 0 ? opts->check_every : 32;
        chunk = std::max(2, std::min(chunk, 512));
        chunk += chunk & 1;
        vpp_status st;
        if ((st = batch_cg_setup(b))) return st;
        VPP_HIP(hipStreamSynchronize((hipStream_t)stream));
        if ((st = batch_pcg64_lockstep(b, rhs, x, *opts, chunk, inf))) return st;
    }
    // systems solved one at a time: the large ones (FP64) or all (mixed
    // precision, each system with its own FP64 phases)
    for (size_t i = 0, r = 0; i < b->probs.size(); ++i)
        for (int j = 0; j < b->nrhs[i]; ++j, ++r) {
            if (fp64 && b->cg_index[r] >= 0) continue;
            vpp_status st = vpp_cg_solve(b->probs[i], rhs[r], x[r], opts, &inf[r], stream);
            if (st == VPP_ERR_HIP || st == VPP_ERR_OUT_OF_MEMORY || st == VPP_ERR_INVALID_ARG) return st;
        }
    vpp_status worst = VPP_OK;
    for (int r = 0; r < b->total_rhs; ++r) {
        if (info) info[r] = inf[r];
        if (inf[r].status != VPP_OK && worst == VPP_OK) worst = (vpp_status)inf[r].status;
    }
    if (worst != VPP_OK) return fail(worst, "at least one solve of the batch did not converge");
    return VPP_OK;
}

vpp_status vpp_batch_get_config(vpp_batch b, vpp_kernel_config* cfg)
{
    if (!b || !cfg) return fail(VPP_ERR_INVALID_ARG, "null argument");
    cfg->variant = b->cfg.variant;
    for (int d = 0; d < 3; ++d) cfg->tile[d] = b->cfg.tile[d];
    return VPP_OK;
}

vpp_status vpp_batch_destroy(vpp_batch b)
{
    if (!b) return VPP_OK;
    DeviceGuard dg(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    batch_cg_free(b);
    dev_free(b->d_probs); dev_free(b->d_x); dev_free(b->d_y); dev_free(b->d_part); dev_free(b->d_queue);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return VPP_OK;
}

}  // extern "C"

// Variant 6 (k = 3, FP64): one cell per wavefront, the 1D contractions of sum
// factorisation on the matrix cores.
//
// The 64 lanes of a wavefront hold the 4 x 4 x 4 values of one Q3 cell, lane
// l = x0 + 4 x1 + 16 x2 for three 2-bit fields that are, in some order, the
// three tensor indices of the cell.  v_mfma_f64_4x4x4f64 (four 4 x 4 x 4
// blocks) contracts over the field in lane bits 4-5:
//   B-form mfma(M, v, c): the values in the B operand, the matrix M in A; the
//       swept field stays in bits 4-5 and the layout is unchanged;
//   A-form mfma(v, M, c): the values in the A operand, M^T in B; the swept
//       field moves to bits 0-1 and the old bits-0-1 field to bits 4-5.
// Both forms take the same per-lane matrix entry M[l & 3][l >> 4] (A holds
// M[i][k] at lane i + 4 blk + 16 k, B holds M^T[k][j] = M[j][k] at lane
// j + 4 blk + 16 k, the result sits at lane j + 4 blk + 16 i), so a sweep is
// one instruction and the C operand accumulates for free.  The middle field
// reaches bits 4-5 through a lane permutation (ds_bpermute).  A cell's
// operator is 15 such contractions: 3 value sweeps of phi, 3 of u, a
// collocation derivative and its transpose per direction, 3 transposed value
// sweeps, and 8 permutations.
//
// A workgroup owns a tile of TX x TY x TZ cells (even extents) and has
// TX TY TZ / 16 wavefronts: the cell results go into the tile's node block in
// LDS in eight phases by cell parity, so cells of one phase share no node and
// the summation order is fixed; each wavefront takes two cells of every phase
// as two independent chains of contractions, and loads the next phase's phi
// and x before the barrier that ends the current one.  The block is then written like the
// other variants' blocks: nodes of this tile only to y, nodes on planes shared
// with neighbouring tiles as partials for the assembly kernel, Dirichlet nodes
// as identity rows.
#pragma once
#include "apply_impl.h"

namespace vpp {

// Value of lane `src` of the wavefront (ds_bpermute on both halves).
__device__ __forceinline__ double lane_pull(double v, int src)
{
    const int a = src << 2;
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Field permutations (involutions) of the lane index: swap the fields in bits
// 2-3 and 4-5, or in bits 0-1 and 4-5.
__device__ __forceinline__ int swap_fields12(int l) { return (l & 3) | (((l >> 4) & 3) << 2) | (((l >> 2) & 3) << 4); }
__device__ __forceinline__ int swap_fields02(int l) { return ((l >> 4) & 3) | (l & 12) | ((l & 3) << 4); }

__device__ __forceinline__ double mfma_b(double mat, double v, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(mat, v, c, 0, 0, 0);
}
__device__ __forceinline__ double mfma_a(double v, double mat, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(v, mat, c, 0, 0, 0);
}

// Per-lane matrix entries of the Q3 sweeps, M[l & 3][l >> 4].
struct Q3Mats {
    double S, ST, Dc, DcT, wref;   // wref: Gauss weight product at this lane in layout (q0 | q2 | q1)
};

__device__ __forceinline__ Q3Mats q3_mats(int l)
{
    constexpr Tables<3> t = make_tables<3>();
    const int r = l & 3, c = l >> 4;
    Q3Mats q;
    q.S = t.S[r][c];
    q.ST = t.S[c][r];
    q.Dc = t.Dc[r][c];
    q.DcT = t.Dc[c][r];
    q.wref = t.w[l & 3] * t.w[(l >> 2) & 3] * t.w[l >> 4];
    return q;
}

// Value sweeps of all three directions from the node layout (a0 | a1 | a2) to
// the Gauss-point layout (q0 | q2 | q1).
__device__ __forceinline__ double q3_forward(double v, const Q3Mats& q, int lane)
{
    v = mfma_a(v, q.S, 0.0);                       // sweeps a2 -> (q2 | a1 | a0)
    v = mfma_a(v, q.S, 0.0);                       // sweeps a0 -> (q0 | a1 | q2)
    v = lane_pull(v, swap_fields12(lane));         // -> (q0 | q2 | a1)
    return mfma_b(q.S, v, 0.0);                    // sweeps a1 -> (q0 | q2 | q1)
}

// Cell operator of one Q3 cell held by the wavefront: u (layout (a0|a1|a2),
// Dirichlet entries zeroed) -> A_e u in the same layout; cw = c' W at the
// Gauss points in layout (q0 | q2 | q1).
__device__ __forceinline__ double q3_cell_operator(const MeshArgs& m, double cw, double u, const Q3Mats& q,
                                                   int lane)
{
    const double uq = q3_forward(u, q, lane);      // (q0 | q2 | q1)
    // y direction (q1, bits 4-5)
    double g = mfma_b(q.Dc, uq, 0.0);
    double v = mfma_b(q.DcT, cw * m.rd[1] * g, 0.0);
    // x direction (q0, bits 0-1): to bits 4-5, A-form back to (q0 | q2 | q1)
    g = mfma_a(lane_pull(uq, swap_fields02(lane)), q.Dc, 0.0);
    v = mfma_a(lane_pull(cw * g, swap_fields02(lane)), q.DcT, v);
    // z direction (q2, bits 2-3): in layout (q0 | q1 | q2)
    const int s12 = swap_fields12(lane);
    g = mfma_b(q.Dc, lane_pull(uq, s12), 0.0);
    const double w = mfma_b(q.DcT, lane_pull(cw, s12) * m.rd[2] * g, 0.0);
    v += lane_pull(w, s12);
    // transposed value sweeps back to (a0 | a1 | a2)
    v = mfma_b(q.ST, v, 0.0);                      // q1 -> a1: (q0 | q2 | a1)
    v = lane_pull(v, swap_fields12(lane));         // -> (q0 | a1 | q2)
    v = mfma_a(v, q.ST, 0.0);                      // q2 -> a2: (a2 | a1 | q0)
    return mfma_a(v, q.ST, 0.0);                   // q0 -> a0: (a0 | a1 | a2)
}

template <typename T, int TX, int TY, int TZ, int HV, bool DOT>
__global__ void __launch_bounds__(64 * (TX * TY * TZ / 16)) apply_mfma_kernel(ApplyArgs<T> a)
{
    static_assert(std::is_same<T, double>::value, "variant 6 runs in FP64");
    static_assert(TX % 2 == 0 && TY % 2 == 0 && TZ % 2 == 0, "even tile extents: every parity phase has 2 NW cells");
    // NW wavefronts; each parity phase holds TX TY TZ / 8 = 2 NW cells, and
    // wavefront w takes cells w and w + NW of every phase as two independent
    // chains of contractions
    constexpr int NW = TX * TY * TZ / 16;
    constexpr int K = 3, BX = K * TX + 1, BY = K * TY + 1, BZ = K * TZ + 1, NB = BX * BY * BZ, NT = 64 * NW;
    constexpr int MX = TX / 2, MY = TY / 2;
    __shared__ double yb[NB];
    if (a.done && *a.done) return;
    const MeshArgs& m = a.m;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const TileCoord tc = tile_coord<K, TX, TY, TZ>(m, tile);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int a0 = lane & 3, a1 = (lane >> 2) & 3, a2 = lane >> 4;
    const Q3Mats q = q3_mats(lane);
    const int nx = m.nn[0], nxy = m.nn[0] * m.nn[1];
    const int64_t tile0 = uniform_i64(node_index(m, tc.n0[0], tc.n0[1], tc.n0[2]));
    const double* __restrict__ xt = a.x + tile0;
    const double* __restrict__ pt = a.phi + tile0;
    // cell (lx, ly, lz) of cell c of phase ph; false when it lies beyond the mesh
    auto cell_of = [&](int ph, int c, int& lx, int& ly, int& lz) {
        lx = (ph & 1) + 2 * (c % MX);
        ly = ((ph >> 1) & 1) + 2 * ((c / MX) % MY);
        lz = (ph >> 2) + 2 * (c / (MX * MY));
        return tc.t[0] * TX + lx < m.nc[0] && tc.t[1] * TY + ly < m.nc[1] && tc.t[2] * TZ + lz < m.nc[2];
    };
    auto load = [&](int ph, int c, double& ph_v, double& x_v) {
        int lx, ly, lz;
        if (!cell_of(ph, c, lx, ly, lz)) return;
        const unsigned off = (unsigned)((K * lx + a0) + nx * (K * ly + a1) + nxy * (K * lz + a2));
        ph_v = pt[off];
        x_v = xt[off];
    };
    for (int i = threadIdx.x; i < NB; i += NT) yb[i] = 0.0;
    double pn0 = 0.0, xn0 = 0.0, pn1 = 0.0, xn1 = 0.0;
    load(0, wave, pn0, xn0);
    load(0, wave + NW, pn1, xn1);
    __syncthreads();
#pragma unroll 1
    for (int ph = 0; ph < 8; ++ph) {
        const double pc0 = pn0, xc0 = xn0, pc1 = pn1, xc1 = xn1;
        if (ph < 7) {
            load(ph + 1, wave, pn0, xn0);
            load(ph + 1, wave + NW, pn1, xn1);
        }
        int lx0, ly0, lz0, lx1, ly1, lz1;
        const bool v0 = cell_of(ph, wave, lx0, ly0, lz0);
        const bool v1 = cell_of(ph, wave + NW, lx1, ly1, lz1);
        if (v0 || v1) {
            const bool d0 = is_dirichlet(m, tc.n0[0] + K * lx0 + a0, tc.n0[1] + K * ly0 + a1, tc.n0[2] + K * lz0 + a2);
            const bool d1 = is_dirichlet(m, tc.n0[0] + K * lx1 + a0, tc.n0[1] + K * ly1 + a1, tc.n0[2] + K * lz1 + a2);
            const double u0 = (v0 && !d0) ? xc0 : 0.0, u1 = (v1 && !d1) ? xc1 : 0.0;
            const double cw0 = coef_scaled<HV>(m, q3_forward(v0 ? pc0 : 0.0, q, lane)) * q.wref;
            const double cw1 = coef_scaled<HV>(m, q3_forward(v1 ? pc1 : 0.0, q, lane)) * q.wref;
            const double y0 = q3_cell_operator(m, cw0, u0, q, lane);
            const double y1 = q3_cell_operator(m, cw1, u1, q, lane);
            if (v0) yb[(K * lx0 + a0) + BX * ((K * ly0 + a1) + BY * (K * lz0 + a2))] += y0;
            if (v1) yb[(K * lx1 + a0) + BX * ((K * ly1 + a1) + BY * (K * lz1 + a2))] += y1;
        }
        __syncthreads();
    }
    // write-out of the node block
    const int e0 = tc.ext[0], e1 = tc.ext[1], e2 = tc.ext[2];
    const int t0 = tc.t[0], t1 = tc.t[1], t2 = tc.t[2];
    const unsigned nsh = (unsigned)a.nshared;
    double dsum = 0.0;
    for (int n = threadIdx.x; n < NB; n += NT) {
        const int c2 = n / (BX * BY), r = n - c2 * (BX * BY);
        const int c1 = r / BX, c0 = r - c1 * BX;
        if (c0 >= e0 || c1 >= e1 || c2 >= e2) continue;
        const int gi = tc.n0[0] + c0, gj = tc.n0[1] + c1, gl = tc.n0[2] + c2;
        const unsigned off = (unsigned)(c0 + nx * c1 + nxy * c2);
        const bool lo0 = c0 == 0 && t0 > 0, lo1 = c1 == 0 && t1 > 0, lo2 = c2 == 0 && t2 > 0;
        const bool hi0 = c0 == e0 - 1 && t0 < m.ntile[0] - 1, hi1 = c1 == e1 - 1 && t1 < m.ntile[1] - 1,
                   hi2 = c2 == e2 - 1 && t2 < m.ntile[2] - 1;
        if (is_dirichlet(m, gi, gj, gl)) {
            const double xv = xt[off];
            a.y[tile0 + off] = xv;
            if (DOT && !(lo0 || lo1 || lo2)) dsum += xv * xv;
            continue;
        }
        const double v = yb[n];
        if (lo0 || lo1 || lo2 || hi0 || hi1 || hi2) {
            int64_t fi;
            int rank;
            shared_from_tile(m, tc.t, lo0, lo1, lo2, hi0, hi1, hi2, gi, gj, gl, fi, rank);
            a.part[(unsigned)rank * nsh + (unsigned)fi] = v;
        } else {
            a.y[tile0 + off] = v;
        }
        if (DOT) dsum += xt[off] * v;
    }
    if constexpr (DOT) {
        const double s = block_sum<NT>(dsum);
        if (threadIdx.x == 0) a.dot_part[blockIdx.x] = s;
    }
}

}  // namespace vpp

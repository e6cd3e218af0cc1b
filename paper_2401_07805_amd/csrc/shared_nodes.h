// Enumeration of the nodes shared by several workgroup tiles and of their
// partial slots (host + device, so the index arithmetic is checked on the CPU).
#pragma once
#include <stdint.h>

#include "common.h"

namespace vpp {

// a / b for 0 <= a < 2^31 and 1 <= b < 2^20 through a double reciprocal (a few
// instructions instead of an integer division): (a + 0.5) / b lies at least
// 0.5 / b from an integer, and the product's rounding error is below
// 2^31 * 2^-52 < 0.5 / b, so truncation gives the exact quotient.
__host__ __device__ inline int qdiv(int a, int b, double inv_b)
{
    (void)b;
    return (int)(((double)a + 0.5) * inv_b);
}

// The r-th index in [0, n) that is not an interior tile boundary (multiples s,
// 2s, ..., (nt-1)s of the tile span s): the first group [0, s) has s entries,
// the middle groups ((g+1)s, (g+2)s) s-1 each, the last one runs to n-1.
// inv_s1 = 1 / (s - 1).
__host__ __device__ inline int nth_free(int r, int s, int nt, double inv_s1)
{
    if (r < s || nt <= 1) return r;
    const int rr = r - s;
    if (s > 1) {
        const int g = qdiv(rr, s - 1, inv_s1);
        if (g < nt - 2) return (g + 1) * s + 1 + (rr - g * (s - 1));
        return (nt - 1) * s + 1 + (rr - (nt - 2) * (s - 1));
    }
    return (nt - 1) * s + 1 + rr;
}

// Shared nodes, enumerated flat and without repetition:
//   family z: l on a z boundary plane                      (nbz * Ny * Nx)
//   family y: j on a y plane, l free                       (nby * (Nz - nbz) * Nx)
//   family x: i on an x plane, j and l free                (nbx * (Ny - nby) * (Nz - nbz))
struct SharedEnum {
    int s[3], nb[3], nn[3], nt[3];
    int64_t cz, cy, cx;
    double inv_s[3], inv_s1[3], inv_nn[3], inv_nb[3], inv_nyf;   // reciprocals for qdiv
};

__host__ __device__ inline SharedEnum shared_enum(const MeshArgs& m, int k, const int (&tile)[3])
{
    SharedEnum e;
    for (int d = 0; d < 3; ++d) {
        e.s[d] = k * tile[d];
        e.nt[d] = m.ntile[d];
        e.nb[d] = m.ntile[d] - 1;
        e.nn[d] = m.nn[d];
    }
    for (int d = 0; d < 3; ++d) {
        e.inv_s[d] = 1.0 / e.s[d];
        e.inv_s1[d] = e.s[d] > 1 ? 1.0 / (e.s[d] - 1) : 0.0;
        e.inv_nn[d] = 1.0 / e.nn[d];
        e.inv_nb[d] = e.nb[d] > 0 ? 1.0 / e.nb[d] : 0.0;
    }
    e.inv_nyf = 1.0 / (e.nn[1] - e.nb[1]);
    e.cz = (int64_t)e.nb[2] * e.nn[1] * e.nn[0];
    e.cy = (int64_t)e.nb[1] * (e.nn[2] - e.nb[2]) * e.nn[0];
    e.cx = (int64_t)e.nb[0] * (e.nn[1] - e.nb[1]) * (e.nn[2] - e.nb[2]);
    return e;
}

// Node (i, j, l) of enumeration position f (f < 2^31, every divisor < 2^20:
// checked by the host), with reciprocal divisions.
__host__ __device__ inline void shared_node(const SharedEnum& e, int64_t f64, int& i, int& j, int& l)
{
    int f = (int)f64;
    if (f < e.cz) {
        const int r = qdiv(f, e.nn[0], e.inv_nn[0]);
        i = f - r * e.nn[0];
        const int p = qdiv(r, e.nn[1], e.inv_nn[1]);
        j = r - p * e.nn[1];
        l = (p + 1) * e.s[2];
        return;
    }
    f -= (int)e.cz;
    if (f < e.cy) {
        const int r = qdiv(f, e.nn[0], e.inv_nn[0]);
        i = f - r * e.nn[0];
        const int lf = qdiv(r, e.nb[1], e.inv_nb[1]);
        j = (r - lf * e.nb[1] + 1) * e.s[1];
        l = nth_free(lf, e.s[2], e.nt[2], e.inv_s1[2]);
        return;
    }
    f -= (int)e.cy;
    const int r = qdiv(f, e.nb[0], e.inv_nb[0]);
    i = (f - r * e.nb[0] + 1) * e.s[0];
    const int ny = e.nn[1] - e.nb[1];
    const int lf = qdiv(r, ny, e.inv_nyf);
    j = nth_free(r - lf * ny, e.s[1], e.nt[1], e.inv_s1[1]);
    l = nth_free(lf, e.s[2], e.nt[2], e.inv_s1[2]);
}

// Number of tiles holding node (i, j, l) and this tile's rank among them (the
// order of shared_slots: z, y, x tile index ascending).  Along a direction where
// the node sits on an interior tile boundary there are two tiles, and the lower
// one (whose block holds the node on its top face) comes first.
__host__ __device__ inline void sharer_rank(const MeshArgs& m, int k, const int (&tile)[3], int i, int j, int l,
                                            const int (&t)[3], int& count, int& rank)
{
    const int idx[3] = {i, j, l};
    int nt[3], bit[3];
    for (int d = 0; d < 3; ++d) {
        const int span = k * tile[d];
        const int a = idx[d] / span;
        const bool sh = idx[d] == a * span && a > 0 && a < m.ntile[d];
        nt[d] = sh ? 2 : 1;
        bit[d] = (sh && t[d] == a) ? 1 : 0;
    }
    count = nt[0] * nt[1] * nt[2];
    rank = bit[0] + nt[0] * (bit[1] + nt[1] * bit[2]);
}

// Position of index v among the indices that are not interior tile boundaries
// (inverse of nth_free); v must not be a boundary.
__host__ __device__ inline int free_index(int v, int s, int nt)
{
    int a = v / s;
    if (a > nt - 1) a = nt - 1;
    return v - a;        // one boundary index below v per full span passed
}

// Position f of shared node (i, j, l) in the enumeration of shared_node.
__host__ __device__ inline int64_t shared_index(const SharedEnum& e, int i, int j, int l)
{
    const bool bz = l % e.s[2] == 0 && l / e.s[2] > 0 && l / e.s[2] < e.nt[2];
    if (bz) return i + (int64_t)e.nn[0] * (j + (int64_t)e.nn[1] * (l / e.s[2] - 1));
    const bool by = j % e.s[1] == 0 && j / e.s[1] > 0 && j / e.s[1] < e.nt[1];
    const int lf = free_index(l, e.s[2], e.nt[2]);
    if (by) return e.cz + i + (int64_t)e.nn[0] * ((j / e.s[1] - 1) + (int64_t)e.nb[1] * lf);
    const int jf = free_index(j, e.s[1], e.nt[1]);
    return e.cz + e.cy + (i / e.s[0] - 1) + (int64_t)e.nb[0] * (jf + (int64_t)(e.nn[1] - e.nb[1]) * lf);
}

// Node-space lookup used where a streaming kernel visits every node: whether
// global node g (< 2^31) is a shared node that is not a Dirichlet node (those
// are written directly as identity rows), and if so its enumeration position
// f (as shared_index) and the number of tiles holding it (as sharer_count).
// Reciprocal divisions only.  The part that depends on the row (j, l) alone is
// split off, so that consecutive nodes of a row share it.
struct SharedRow {
    int j, l, ay, lf, jf;
    bool by, bz, dir;   // on a y plane, on a z plane, Dirichlet row
};

__host__ __device__ inline SharedRow shared_row(const SharedEnum& e, int bcmask, int j, int l)
{
    SharedRow w;
    w.j = j;
    w.l = l;
    w.ay = qdiv(j, e.s[1], e.inv_s[1]);
    const int az = qdiv(l, e.s[2], e.inv_s[2]);
    w.by = j == w.ay * e.s[1] && w.ay > 0 && w.ay < e.nt[1];
    w.bz = l == az * e.s[2] && az > 0 && az < e.nt[2];
    w.dir = ((bcmask & 4) && j == 0) || ((bcmask & 8) && j == e.nn[1] - 1) || ((bcmask & 16) && l == 0) ||
            ((bcmask & 32) && l == e.nn[2] - 1);
    w.lf = l - (az < e.nt[2] - 1 ? az : e.nt[2] - 1);
    w.jf = j - (w.ay < e.nt[1] - 1 ? w.ay : e.nt[1] - 1);
    // on a z plane, lf is replaced by the plane index - 1 (see shared_in_row)
    if (w.bz) w.lf = az - 1;
    return w;
}

__host__ __device__ inline bool shared_in_row(const SharedEnum& e, int bcmask, const SharedRow& w, int i, int& f,
                                              int& count)
{
    const int ax = qdiv(i, e.s[0], e.inv_s[0]);
    const bool bx = i == ax * e.s[0] && ax > 0 && ax < e.nt[0];
    if (!(bx || w.by || w.bz)) return false;
    if (w.dir || ((bcmask & 1) && i == 0) || ((bcmask & 2) && i == e.nn[0] - 1)) return false;
    count = (bx ? 2 : 1) * (w.by ? 2 : 1) * (w.bz ? 2 : 1);
    if (w.bz)
        f = i + e.nn[0] * (w.j + e.nn[1] * w.lf);
    else if (w.by)
        f = (int)e.cz + i + e.nn[0] * ((w.ay - 1) + e.nb[1] * w.lf);
    else
        f = (int)(e.cz + e.cy) + (ax - 1) + e.nb[0] * (w.jf + (e.nn[1] - e.nb[1]) * w.lf);
    return true;
}

__host__ __device__ inline bool shared_lookup(const SharedEnum& e, int bcmask, int g, int& f, int& count)
{
    const int r = qdiv(g, e.nn[0], e.inv_nn[0]);
    const int l = qdiv(r, e.nn[1], e.inv_nn[1]);
    return shared_in_row(e, bcmask, shared_row(e, bcmask, r - l * e.nn[1], l), g - r * e.nn[0], f, count);
}

// Enumeration position and rank of node (gi, gj, gl) as seen from tile t, given
// on which faces of that tile's block it lies (lo*: bottom face with a tile
// below, hi*: top face with a tile above); at least one flag is set.  Needs no
// division: the plane index follows from the tile coordinate and, off a plane,
// the free index of a coordinate inside tile t is the coordinate minus t.
__host__ __device__ inline void shared_from_tile(const MeshArgs& m, const int (&t)[3], bool lo0, bool lo1, bool lo2,
                                                 bool hi0, bool hi1, bool hi2, int gi, int gj, int gl, int64_t& f,
                                                 int& rank)
{
    const bool s0 = lo0 || hi0, s1 = lo1 || hi1, s2 = lo2 || hi2;
    const int n0 = s0 ? 2 : 1, n1 = s1 ? 2 : 1;
    rank = (lo0 ? 1 : 0) + n0 * ((lo1 ? 1 : 0) + n1 * (lo2 ? 1 : 0));
    const int64_t nx = m.nn[0];
    const int nbx = m.ntile[0] - 1, nby = m.ntile[1] - 1, nbz = m.ntile[2] - 1;
    const int64_t cz = (int64_t)nbz * m.nn[1] * m.nn[0];
    const int64_t cy = (int64_t)nby * (m.nn[2] - nbz) * m.nn[0];
    if (s2) {
        const int zp = lo2 ? t[2] : t[2] + 1;
        f = gi + nx * (gj + (int64_t)m.nn[1] * (zp - 1));
    } else if (s1) {
        const int yp = lo1 ? t[1] : t[1] + 1;
        f = cz + gi + nx * ((yp - 1) + (int64_t)nby * (gl - t[2]));
    } else {
        const int xp = lo0 ? t[0] : t[0] + 1;
        f = cz + cy + (xp - 1) + (int64_t)nbx * ((gj - t[1]) + (int64_t)(m.nn[1] - nby) * (gl - t[2]));
    }
}

// Number of tiles holding shared node (i, j, l): 2 per direction in which it
// sits on an interior tile boundary.
__host__ __device__ inline int sharer_count(const SharedEnum& e, int i, int j, int l)
{
    const int idx[3] = {i, j, l};
    int n = 1;
    for (int d = 0; d < 3; ++d) {
        const int a = qdiv(idx[d], e.s[d], e.inv_s[d]);
        if (idx[d] == a * e.s[d] && a > 0 && a < e.nt[d]) n *= 2;
    }
    return n;
}

// Partial slots (tile * block size + local index) of node (i, j, l), in the
// order z, y, x tile index ascending; returns their number (1..8).  A node lies
// in two tiles along a direction when it sits on an interior tile boundary.
__host__ __device__ inline int shared_slots(const MeshArgs& m, int k, const int (&tile)[3], int i, int j, int l,
                                            int64_t (&slot)[8])
{
    const int idx[3] = {i, j, l};
    int t0[3], nt[3], l0[3], bdim[3];
    for (int d = 0; d < 3; ++d) {
        const int span = k * tile[d];
        bdim[d] = span + 1;
        const int a = idx[d] / span, r = idx[d] - a * span;
        if (r == 0 && a > 0 && a < m.ntile[d]) {
            t0[d] = a - 1;
            nt[d] = 2;
            l0[d] = span;           // top face of the lower tile
        } else {
            t0[d] = a < m.ntile[d] - 1 ? a : m.ntile[d] - 1;
            nt[d] = 1;
            l0[d] = idx[d] - span * t0[d];
        }
    }
    const int64_t bs = (int64_t)bdim[0] * bdim[1] * bdim[2];
    int n = 0;
    for (int c = 0; c < nt[2]; ++c)
        for (int b = 0; b < nt[1]; ++b)
            for (int a = 0; a < nt[0]; ++a) {
                const int tx = t0[0] + a, ty = t0[1] + b, tz = t0[2] + c;
                const int lx = a ? 0 : l0[0], ly = b ? 0 : l0[1], lz = c ? 0 : l0[2];
                const int64_t tid = tx + (int64_t)m.ntile[0] * (ty + (int64_t)m.ntile[1] * tz);
                slot[n++] = tid * bs + lx + bdim[0] * (ly + bdim[1] * lz);
            }
    return n;
}

}  // namespace vpp

// Device-side building blocks of the gfx950 MFM pass: cubic-spline kernel,
// minimum-image displacement, and the stackless walk over the implicit octree
// that the Morton-sorted particle order and the per-level cell tables define.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfm {

constexpr int kMaxLevels = 12;   // levels 0..kMaxLevels-1
constexpr int kWave = 64;

// Everything a kernel needs to walk the cell tables, passed by value.
struct TreeDesc {
    int bmax;                        // deepest level
    int ktot;                        // key bits at bmax
    int leaf;                        // stop descending at <= leaf particles
    int nact[kMaxLevels];            // axes refined at level l (0 at l = 0)
    int actmask[kMaxLevels];         // bit d set when axis d refines at level l
    int kbits[kMaxLevels];           // key-prefix bits of a level-l cell
    long long tab_off[kMaxLevels];   // offset of level l in the (start, end) table
    long long hmax_off[kMaxLevels];  // offset of level l in the hmax table (l < bmax)
    double cs[kMaxLevels][3];        // cell side per axis at level l
    double box[3];
    int periodic[3];
    int qbits[3];                    // quantisation bits per axis
};

// Run-time physics parameters shared by the pass kernels.
struct Phys {
    double gamma;
    double n_ngb;
    double beta;
    double cond_max;
    double box[3];
    int periodic[3];
    int h_maxit;
    int max_ngb;
};

// Device counters (all updated with atomics, read by the host after a sync).
struct Counters {
    unsigned long long list_entries;
    unsigned long long list_max;
    unsigned long long h_iters;
    unsigned long long h_iters_max;
    unsigned long long noconv;
    unsigned long long minimage;
    unsigned long long overflow;
    unsigned long long illcond;
    unsigned long long fallbacks;
    unsigned long long clamps;
    unsigned long long nonfinite;
    unsigned long long floors;
    unsigned long long first_bad;    // min index (init ~0ull)
    unsigned long long cond_bits;    // max of the positive double cond, as bits
    unsigned long long h_rounds_max; // most group scans a kernel-length solve needed
    unsigned long long h_fallback;   // particles solved by the per-particle kernel
};

// ---------------------------------------------------------------- kernel
// Cubic spline with support radius H: W = 8/(pi H^3) w(q), q = r/H,
// w = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1), 0 beyond.
template <typename T>
__device__ __forceinline__ T spline_w(T q) {
    if (q <= T(0.5)) return T(1) + q * q * (T(6) * q - T(6));
    if (q <= T(1)) {
        T t = T(1) - q;
        return T(2) * t * t * t;
    }
    return T(0);
}

// q * dw/dq
template <typename T>
__device__ __forceinline__ T spline_qdw(T q) {
    if (q <= T(0.5)) return q * q * (T(18) * q - T(12));
    if (q <= T(1)) {
        T t = T(1) - q;
        return T(-6) * q * t * t;
    }
    return T(0);
}

template <typename T>
__device__ __forceinline__ T kernel_norm(T H) {
    return T(2.5464790894703255) / (H * H * H);  // 8/pi / H^3
}

// x_j - x_i on one axis, moved to the nearest periodic image
__device__ __forceinline__ double min_image(double d, double L, int periodic) {
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

// distance along one axis from coordinate x to the interval [lo, hi)
__device__ __forceinline__ double axis_gap(double x, double lo, double hi, double L, int periodic) {
    if (x >= lo && x < hi) return 0.0;
    if (!periodic) return fmax(lo - x, x - hi);
    double g1 = lo - x;
    if (g1 < 0.0) g1 += L;
    double g2 = x - hi;
    if (g2 < 0.0) g2 += L;
    return fmin(g1, g2);
}

// ------------------------------------------------------ implicit octree walk
// Node = (level l, key prefix c, integer cell coordinates cx, cy, cz).
// A level-l cell holds the particles whose key starts with c: the sorted
// range tab[l][c] = [start, end).  `accept(l, c, cell_lo[3], cell_hi[3])`
// decides whether a non-empty node can hold a neighbour; `leaf(start, end)`
// scans a node's particles.  The walk visits nodes in Morton order without a
// stack: after a node it moves to the next sibling, climbing while the node
// is the last child of its parent.
template <typename Accept, typename Leaf>
__device__ __forceinline__ void tree_walk(const TreeDesc& td, const int2* __restrict__ tab,
                                          Accept&& accept, Leaf&& leaf) {
    int l = 0;
    unsigned long long c = 0;
    int cc[3] = {0, 0, 0};
    for (;;) {
        int2 se = tab[td.tab_off[l] + (long long)c];
        if (se.y > se.x) {
            double lo[3], hi[3];
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lo[d] = cc[d] * td.cs[l][d];
                hi[d] = lo[d] + td.cs[l][d];
            }
            if (accept(l, c, lo, hi)) {
                if (l == td.bmax || se.y - se.x <= td.leaf) {
                    leaf(se.x, se.y);
                } else {
                    // first child
                    l++;
                    int nb = td.nact[l];
                    c <<= nb;
                    int m = td.actmask[l];
#pragma unroll
                    for (int d = 0; d < 3; d++)
                        if (m & (1 << d)) cc[d] <<= 1;
                    continue;
                }
            }
        }
        // advance to the next sibling, climbing past last children
        for (;;) {
            if (l == 0) return;
            int nb = td.nact[l];
            unsigned k = (unsigned)(c & ((1ull << nb) - 1));
            if (k + 1 < (1u << nb)) {
                c++;
                k++;
                int m = td.actmask[l];
                int pos = nb;
#pragma unroll
                for (int d = 0; d < 3; d++)
                    if (m & (1 << d)) {
                        pos--;
                        cc[d] = (cc[d] & ~1) | ((k >> pos) & 1);
                    }
                break;
            }
            c >>= nb;
            int m = td.actmask[l];
#pragma unroll
            for (int d = 0; d < 3; d++)
                if (m & (1 << d)) cc[d] >>= 1;
            l--;
        }
    }
}

// squared distance from a point to a node box, with a relative pad so that a
// particle binned into a cell by rounding is never rejected by its bounds
__device__ __forceinline__ double node_dist2(const TreeDesc& td, const double xi[3],
                                             const double lo[3], const double hi[3]) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double pad = 1e-12 * td.box[d];
        double g = axis_gap(xi[d], lo[d] - pad, hi[d] + pad, td.box[d], td.periodic[d]);
        s += g * g;
    }
    return s;
}

// squared distance between a node box and a group box (both inside [0, box)),
// nearest periodic image per axis, padded like node_dist2
__device__ __forceinline__ double box_dist2(const TreeDesc& td, const double glo[3], const double ghi[3],
                                            const double lo[3], const double hi[3]) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double pad = 1e-12 * td.box[d];
        const double a = lo[d] - pad, b = hi[d] + pad;
        double g = fmax(0.0, fmax(a - ghi[d], glo[d] - b));
        if (td.periodic[d]) {
            const double L = td.box[d];
            g = fmin(g, fmax(0.0, fmax(a + L - ghi[d], glo[d] - b - L)));
            g = fmin(g, fmax(0.0, fmax(a - L - ghi[d], glo[d] - b + L)));
        }
        s += g * g;
    }
    return s;
}

// ------------------------------------------------- wave-cooperative group walk
// One wave (a block of 64 threads) walks the tree ONCE for its 64 Morton-
// consecutive particles, split into kSub sub-groups of 8 consecutive lanes,
// each with its own bounding box and search radius.  The walk goes level by
// level: the lanes test up to 64 children of the current frontier in parallel
// (one table load each) against every sub-group; a node carries the mask of
// sub-groups that can reach it, accepted inner nodes form the next frontier,
// accepted leaves become candidate ranges with their mask.  Pending ranges are
// handed to `chunk` in batches; a lane tests only candidates whose mask holds
// its own sub-group, so a sub-group with a large radius does not make the
// other 56 lanes test its far candidates.
constexpr int kSub = 8;         // sub-groups of 8 lanes per wave
constexpr int kFront = 128;     // frontier nodes per level (more are scanned as ranges)
constexpr int kRanges = 128;    // pending candidate ranges

struct SubGroups {
    double lo[kSub][3], hi[kSub][3];
    double R[kSub];             // < 0: sub-group inactive
};

struct GroupWalk {
    unsigned long long front[2][kFront];
    unsigned int fmask[2][kFront];
    int rs[kRanges], re[kRanges];
    unsigned int rm[kRanges];
    int pre[64];
};

// integer cell coordinates of the level-l cell with key prefix c
__device__ __forceinline__ void coords_of(const TreeDesc& td, int l, unsigned long long c, int cc[3]) {
    cc[0] = cc[1] = cc[2] = 0;
    for (int lev = l; lev >= 1; lev--) {
        const int m = td.actmask[lev];
        const int bit = l - lev;
        if (m & 4) {
            cc[2] |= (int)(c & 1) << bit;
            c >>= 1;
        }
        if (m & 2) {
            cc[1] |= (int)(c & 1) << bit;
            c >>= 1;
        }
        if (m & 1) {
            cc[0] |= (int)(c & 1) << bit;
            c >>= 1;
        }
    }
}

__device__ __forceinline__ unsigned long long lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// min / max over the 8 lanes of a sub-group
__device__ __forceinline__ double sub_min_d(double v) {
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double sub_max_d(double v) {
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Fill the sub-group boxes from the lanes' positions (inactive lanes pass
// act = false) and radii R (lanes that need no candidates pass R < 0).
__device__ __forceinline__ void set_subgroups(SubGroups& sg, bool act, const double xi[3], double R) {
    const int lane = threadIdx.x & 63;
    double lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        lo[d] = sub_min_d(act ? xi[d] : INFINITY);
        hi[d] = sub_max_d(act ? xi[d] : -INFINITY);
    }
    const double r = sub_max_d(act ? R : -1.0);
    __syncthreads();
    if ((lane & 7) == 0) {
        const int s = lane >> 3;
#pragma unroll
        for (int d = 0; d < 3; d++) {
            sg.lo[s][d] = lo[d];
            sg.hi[s][d] = hi[d];
        }
        sg.R[s] = r;
    }
    __syncthreads();
}

// sub-groups whose box lies within their radius (or within `rnode` when that
// is larger) of the node box [lo, hi); parent restricts the candidates
__device__ __forceinline__ unsigned int subgroup_hits(const TreeDesc& td, const SubGroups& sg, unsigned int parent,
                                                      const double lo[3], const double hi[3], double rnode) {
    unsigned int m = 0;
#pragma unroll
    for (int s = 0; s < kSub; s++) {
        if (!((parent >> s) & 1) || !(sg.R[s] >= 0.0)) continue;
        const double r = fmax(sg.R[s], rnode);
        if (box_dist2(td, sg.lo[s], sg.hi[s], lo, hi) < r * r) m |= 1u << s;
    }
    return m;
}

// Range of flattened position t in the current batch (pre[] = exclusive prefix
// of the batch's range lengths); returns the particle index, sets the range.
__device__ __forceinline__ int batch_candidate(const GroupWalk& g, int rs0, int nb, int t, int& k) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.pre[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    k = rs0 + lo;
    return g.rs[k] + (t - g.pre[lo]);
}

template <typename Chunk>
__device__ __forceinline__ void group_flush(GroupWalk& g, int nr, Chunk&& chunk) {
    const int lane = threadIdx.x & 63;
    for (int b = 0; b < nr; b += 64) {
        const int k = b + lane;
        const int len = k < nr ? g.re[k] - g.rs[k] : 0;
        int inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        const int total = __shfl(inc, 63, 64);
        const int nb = min(64, nr - b);
        __syncthreads();
        g.pre[lane] = inc - len;
        __syncthreads();
        chunk(b, nb, total);
    }
}

// accept(l, c, lo, hi, parent_mask) -> mask of sub-groups that need the node
template <typename Accept, typename Chunk>
__device__ __forceinline__ void group_walk(const TreeDesc& td, const int2* __restrict__ tab, int n, int leaf,
                                           GroupWalk& g, Accept&& accept, Chunk&& chunk) {
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = lanes_below();
    const unsigned int all = (1u << kSub) - 1;
    int nr = 0;
    int cur = 0, nf = 0;
    __syncthreads();
    if (n <= leaf) {
        if (lane == 0) {
            g.rs[0] = 0;
            g.re[0] = n;
            g.rm[0] = all;
        }
        nr = 1;
    } else {
        if (lane == 0) {
            g.front[0][0] = 0ull;
            g.fmask[0][0] = all;
        }
        nf = 1;
    }
    __syncthreads();
    for (int l = 0; l < td.bmax && nf > 0; l++) {
        const int nb = td.nact[l + 1];
        const int nch = nf << nb;
        int nf2 = 0;
        for (int base = 0; base < nch; base += 64) {
            const int t = base + lane;
            bool leaf_hit = false, inner_hit = false;
            int2 se = make_int2(0, 0);
            unsigned long long cchild = 0;
            unsigned int mk = 0;
            if (t < nch) {
                const unsigned long long cp = g.front[cur][t >> nb];
                const unsigned int pm = g.fmask[cur][t >> nb];
                cchild = (cp << nb) | (unsigned long long)(t & ((1 << nb) - 1));
                se = tab[td.tab_off[l + 1] + (long long)cchild];
                if (se.y > se.x) {
                    int cc[3];
                    coords_of(td, l + 1, cchild, cc);
                    double lo[3], hi[3];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        lo[d] = cc[d] * td.cs[l + 1][d];
                        hi[d] = lo[d] + td.cs[l + 1][d];
                    }
                    mk = accept(l + 1, cchild, lo, hi, pm);
                    if (mk) {
                        if (l + 1 == td.bmax || se.y - se.x <= leaf) leaf_hit = true;
                        else inner_hit = true;
                    }
                }
            }
            const unsigned long long mi = __ballot(inner_hit);
            if (inner_hit) {
                const int pos = nf2 + __popcll(mi & lt);
                if (pos < kFront) {
                    g.front[cur ^ 1][pos] = cchild;
                    g.fmask[cur ^ 1][pos] = mk;
                } else {
                    leaf_hit = true;   // frontier full: scan the whole node
                }
            }
            nf2 = min(kFront, nf2 + __popcll(mi));
            const unsigned long long ml = __ballot(leaf_hit);
            if (leaf_hit) {
                const int pos = nr + __popcll(ml & lt);
                g.rs[pos] = se.x;
                g.re[pos] = se.y;
                g.rm[pos] = mk;
            }
            nr += __popcll(ml);
            if (nr >= 64) {
                __syncthreads();
                group_flush(g, nr, chunk);
                nr = 0;
            }
        }
        __syncthreads();
        cur ^= 1;
        nf = nf2;
    }
    if (nr > 0) {
        __syncthreads();
        group_flush(g, nr, chunk);
    }
    __syncthreads();
}

// wave-wide min / max of doubles (all 64 lanes participate)
__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace mfm

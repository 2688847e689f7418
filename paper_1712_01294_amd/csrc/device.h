// Device-side building blocks of the gfx950 MFM pass: cubic-spline kernel,
// minimum-image displacement, and the wave-cooperative scans over the cell
// tables that the Morton-sorted particle order defines (one (start, end)
// range per cell of every level of an implicit octree).
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
    int actmask[kMaxLevels];         // bit d set when axis d refines at level l
    int kbits[kMaxLevels];           // key-prefix bits of a level-l cell
    long long tab_off[kMaxLevels];   // offset of level l in the (start, end) table
    double cs[kMaxLevels][3];        // cell side per axis at level l
    int ncell[kMaxLevels][3];        // cells per axis at level l (a power of two)
    unsigned long long mask[kMaxLevels][3];  // key-prefix bits of axis d at level l
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
    int limiter;          // 1: pairwise face limiter and condition-adaptive beta
    double beta_min, cond_lo, cond_hi;
};

// Device counters (all updated with atomics, read by the host after a sync).
// There are kCounterCopies copies, kCounterStride bytes apart; a block updates
// the copy of its blockIdx modulo the count, which spreads the atomics of a
// launch over as many cache lines (all on one line serialise in one L2
// channel), and the host combines the copies when it reads them.
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
    unsigned long long h_rounds3;    // particles that needed three or more scans
    unsigned long long gather_entries;  // sum of the gather-list lengths
    unsigned long long h_rescan;     // particles the rescanning kernel-length solver took
};
constexpr int kCounterCopies = 32;
constexpr int kCounterStride = 256;
static_assert(sizeof(Counters) <= kCounterStride, "counter copies overlap");

// the copy of the counters the calling block updates
__device__ __forceinline__ Counters* counter_copy(Counters* base) {
    return (Counters*)((char*)base + (blockIdx.x & (kCounterCopies - 1)) * kCounterStride);
}

// ---------------------------------------------------------------- kernel
// Cubic spline with support radius H: W = 8/(pi H^3) w(q), q = r/H,
// w = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1), 0 beyond.
// With t = max(1 - q, 0) and u = max(1/2 - q, 0) both pieces are one
// expression, w = 2 t^3 - 8 u^3 (expanding 2(1-q)^3 - (1-2q)^3 gives the inner
// piece), and q w'(q) = q (24 u^2 - 6 t^2): no selects or branches, so lanes
// with q on different pieces run the same instructions.
__device__ __forceinline__ double spline_pos(double a) { return fmax(a, 0.0); }
__device__ __forceinline__ float spline_pos(float a) { return fmaxf(a, 0.0f); }

template <typename T>
__device__ __forceinline__ T spline_w(T q) {
    const T t = spline_pos(T(1) - q);
    const T u = spline_pos(T(0.5) - q);
    return T(2) * (t * t) * t - T(8) * (u * u) * u;
}

// q * dw/dq
template <typename T>
__device__ __forceinline__ T spline_qdw(T q) {
    const T t = spline_pos(T(1) - q);
    const T u = spline_pos(T(0.5) - q);
    return q * (T(24) * (u * u) - T(6) * (t * t));
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

// ------------------------------------------------- wave-cooperative cell scan
// A group of lanes (Morton neighbours with similar trial radii) scans the union
// of their neighbourhoods together: the cells of one table level whose boxes
// come within Rq of the group's bounding box, on the finest level whose cells
// are at least kScanScale Rq wide.  Cells are taken 64 at a time, one per lane
// (key, table entry, periodic image); their particles are then staged 64 at a
// time in LDS with coalesced loads, already moved to the periodic image next to
// the group, and every lane tests each staged particle against its own sphere.
// The loop structure is the same for all lanes, so the wave never diverges on
// cell or particle counts and no lane waits on a dependent gather of its own.
// Cell keys come from per-axis cell coordinates deposited into the key bits of
// that axis (cells per axis are a power of two).
constexpr double kScanScale = 0.35;

// scatter the low bits of v into the set bits of mask (lowest first); bits of v
// beyond the mask's population are dropped, which reduces v modulo 2^popcount
__device__ __forceinline__ unsigned long long deposit_bits(unsigned v, unsigned long long mask) {
    unsigned long long r = 0;
    while (mask && v) {
        const unsigned long long low = mask & (~mask + 1);
        if (v & 1u) r |= low;
        v >>= 1;
        mask &= mask - 1;
    }
    return r;
}

// Sum of two deposited values modulo 2^popcount(mask): with the bits outside the
// mask set to one, carries run through them to the next mask bit.
__device__ __forceinline__ unsigned long long dilated_add(unsigned long long x, unsigned long long y,
                                                          unsigned long long mask) {
    return ((x | ~mask) + y) & mask;
}

// Difference of two deposited values modulo 2^popcount(mask): borrows run
// through the zero bits outside the mask.
__device__ __forceinline__ unsigned long long dilated_sub(unsigned long long x, unsigned long long y,
                                                          unsigned long long mask) {
    return (x - y) & mask;
}

// per-wave LDS of the cooperative scan
struct ScanLds {
    double4 cand[kWave];    // staged particles: image position, index bits in w
    int excl[kWave];        // exclusive prefix of the batch cells' particle counts
    int start[kWave];       // first particle of each batch cell
    double sh[3][kWave];    // periodic image shift of each batch cell
    unsigned long long key[3][kWave];   // key bits of cell coordinate a + t, t = 0..63, per axis
};

// order the LDS traffic of one wave (lanes read what other lanes wrote)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double sq_disp(const double4& q, const double xi[3], int wrap, const double box[3]) {
    double d0 = q.x - xi[0], d1 = q.y - xi[1], d2 = q.z - xi[2];
    if (wrap) {
        d0 = min_image(d0, box[0], wrap & 1);
        d1 = min_image(d1, box[1], wrap & 2);
        d2 = min_image(d2, box[2], wrap & 4);
    }
    return d0 * d0 + d1 * d1 + d2 * d2;
}

// Bit 63 - k of the mask is set when staged particle k lies inside the sphere,
// so the hit loop takes hits in staging order from the top bit down.  The tests
// go four at a time (a group shifted in below the previous ones); slots past nb
// hold a far-away point, so a group may run past nb.
template <bool kWrap>
__device__ __forceinline__ unsigned long long batch_mask(const ScanLds& S, int nb, const double xi[3], double R2,
                                                         int wrap, const double box[3]) {
    unsigned long long mk = 0;
    int k0 = 0;
    for (; k0 < nb; k0 += 4) {
        unsigned b = 0;
#pragma unroll
        for (int k = 0; k < 4; k++)
            b = (b << 1) + (sq_disp(S.cand[k0 + k], xi, kWrap ? wrap : 0, box) < R2 ? 1u : 0u);
        mk = (mk << 4) | b;
    }
    return k0 >= 64 ? mk : (k0 == 0 ? 0ull : mk << (64 - k0));
}

// Cell enumeration and staging shared by the cooperative scans: the cells of
// one table level within Rq of the box [bmin, bmax] (the finest level whose
// cells are at least scale Rq wide, kScanScale by default) are taken 64 at a
// time, one per lane (key, table entry, periodic image), and their particles
// are handed out 64 at a time, one per lane, with coalesced loads: chunk(q,
// valid, nb, wrap) runs on
// every lane for each such chunk, q being the lane's particle moved to the
// periodic image next to the box (index bits in q.w), valid whether the lane
// holds one, nb how many lanes do.  `wrap` has bit d set when the scan spans
// periodic axis d whole; displacements along such an axis must then take the
// minimum image themselves.  bmin, bmax and Rq must be uniform over the wave,
// with Rq below half of every periodic side.
template <typename Chunk>
__device__ __forceinline__ void scan_cells(const TreeDesc& td, const int2* __restrict__ tab,
                                           const double4* __restrict__ pos, ScanLds& S, int lane,
                                           const double bmin[3], const double bmax[3], double Rq, Chunk&& chunk,
                                           double scale = kScanScale) {
    int L = td.bmax;
    while (L > 0 && fmin(td.cs[L][0], fmin(td.cs[L][1], td.cs[L][2])) < scale * Rq) L--;
    L = __builtin_amdgcn_readfirstlane(L);
    int a[3], cnt[3], nc[3];
    int wrap = 0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double s = td.cs[L][d];
        nc[d] = td.ncell[L][d];
        int lo = (int)floor((bmin[d] - Rq) / s);
        int hi = (int)floor((bmax[d] + Rq) / s);
        if (td.periodic[d]) {
            if (hi - lo + 1 >= nc[d]) {
                lo = 0;
                hi = nc[d] - 1;
                wrap |= 1 << d;
            }
        } else {
            lo = max(lo, 0);
            hi = min(hi, nc[d] - 1);
        }
        a[d] = __builtin_amdgcn_readfirstlane(lo);
        cnt[d] = __builtin_amdgcn_readfirstlane(hi - lo + 1);
    }
    wrap = __builtin_amdgcn_readfirstlane(wrap);
    if (cnt[0] <= 0 || cnt[1] <= 0 || cnt[2] <= 0) return;
    const int ncells = cnt[0] * cnt[1] * cnt[2];
    // key bits of the range's cell coordinates (modulo the cells per axis) for
    // offsets 0..63 along each axis; a wider range deposits per lane
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int w = (a[d] + lane) & (nc[d] - 1);   // nc is a power of two
        S.key[d][lane] = deposit_bits((unsigned)w, td.mask[L][d]);
    }
    wave_lds_sync();
    // slack for the rounding of cell edges and of the keys' quantisation
    const double Rg = Rq * (1.0 + 1e-9) + 1e-12 * fmax(td.box[0], fmax(td.box[1], td.box[2]));
    const double Rg2 = Rg * Rg;
    const long long off = td.tab_off[L];
    // cell coordinates from the flat index through FP32 reciprocals (exact for
    // the few thousand cells a scan covers)
    const float inv2 = 1.0f / (float)cnt[2], inv1 = 1.0f / (float)cnt[1];
    for (int c0 = 0; c0 < ncells; c0 += kWave) {
        const int c = c0 + lane;
        int num = 0, st = 0;
        double sh[3] = {0.0, 0.0, 0.0};
        if (c < ncells) {
            const int t = (int)(((float)c + 0.5f) * inv2);
            const int tz = c - t * cnt[2];
            const int tx = (int)(((float)t + 0.5f) * inv1);
            const int ty = t - tx * cnt[1];
            const int u[3] = {a[0] + tx, a[1] + ty, a[2] + tz};
            double g2 = 0.0;
            unsigned long long key = 0;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                const double s = td.cs[L][d];
                const double clo = u[d] * s;
                const double g = (wrap >> d) & 1 ? 0.0 : fmax(0.0, fmax(clo - bmax[d], bmin[d] - (clo + s)));
                g2 += g * g;
                // unwrapped cell coordinates stay within one box side of [0, nc)
                int w = u[d];
                if (w < 0) {
                    w += nc[d];
                    sh[d] = -td.box[d];
                } else if (w >= nc[d]) {
                    w -= nc[d];
                    sh[d] = td.box[d];
                }
                key |= cnt[d] <= kWave ? S.key[d][u[d] - a[d]] : deposit_bits((unsigned)w, td.mask[L][d]);
            }
            if (g2 < Rg2) {
                const int2 se = tab[off + (long long)key];
                st = se.x;
                num = se.y - se.x;
            }
        }
        int incl = num;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int v = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += v;
        }
        const int total = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1, kWave));
        if (total == 0) continue;
        S.excl[lane] = incl - num;
        S.start[lane] = st;
        S.sh[0][lane] = sh[0];
        S.sh[1][lane] = sh[1];
        S.sh[2][lane] = sh[2];
        wave_lds_sync();
        for (int t0 = 0; t0 < total; t0 += kWave) {
            const int t = t0 + lane;
            // lanes past the end hold a far-away point that no sphere reaches
            double4 q = make_double4(1e30, 1e30, 1e30, __longlong_as_double(-1ll));
            if (t < total) {
                // the last batch cell whose prefix is <= t holds particle t
                int k = 0;
#pragma unroll
                for (int step = kWave / 2; step > 0; step >>= 1)
                    if (S.excl[k + step] <= t) k += step;
                const int j = S.start[k] + (t - S.excl[k]);
                const double4 p = pos[j];
                q = make_double4(p.x + S.sh[0][k], p.y + S.sh[1][k], p.z + S.sh[2][k],
                                 __longlong_as_double((long long)j));
            }
            chunk(q, t < total, min(kWave, total - t0), wrap);
        }
        wave_lds_sync();   // the next batch overwrites the cell data
    }
}

// Tests every particle of every cell within Rq of the box [bmin, bmax] against
// the calling lane's sphere |x - xi|^2 < R2 (lanes with sel false take no
// hits) and calls hit(j, r2) for each particle inside, in the order the cells
// are scanned.  Each chunk of 64 staged particles is put in LDS and first
// tested without branches into a 64-bit mask per lane, so the tests of
// neighbouring particles overlap; the lane then walks its set bits.
template <typename Hit>
__device__ __forceinline__ void group_scan(const TreeDesc& td, const int2* __restrict__ tab,
                                           const double4* __restrict__ pos, ScanLds& S, int lane,
                                           const double bmin[3], const double bmax[3], double Rq,
                                           const double xi[3], double R2, bool sel, Hit&& hit) {
    scan_cells(td, tab, pos, S, lane, bmin, bmax, Rq, [&](const double4& q, bool, int nb, int wrap) {
        S.cand[lane] = q;
        wave_lds_sync();
        unsigned long long mk = wrap ? batch_mask<true>(S, nb, xi, R2, wrap, td.box)
                                     : batch_mask<false>(S, nb, xi, R2, 0, td.box);
        if (!sel) mk = 0;
        while (mk) {
            const int k = __builtin_clzll(mk);
            mk &= ~(0x8000000000000000ull >> k);
            const double4 qk = S.cand[k];
            hit((int)__double_as_longlong(qk.w), sq_disp(qk, xi, wrap, td.box));
        }
        wave_lds_sync();
    });
}

// wave-wide sum of doubles in a fixed order (all 64 lanes participate)
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// a value known to be equal on all lanes, moved to scalar registers
__device__ __forceinline__ double uniform_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
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

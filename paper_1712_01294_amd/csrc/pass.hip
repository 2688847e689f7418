// The gfx950 MFM hydro pass: kernel length, flux lists, gradients, fluxes.
//
// One thread per (Morton-ordered) particle; blocks are remapped so that each
// XCD works on one contiguous run of particles and keeps its neighbours in
// its own L2.  The flux kernel evaluates every unordered pair on both of its
// particles with the lower index as the left state, so both copies are
// bitwise equal and the accumulated momentum and energy cancel exactly pair
// by pair; there are no atomics on outputs and results are deterministic.
#include <limits.h>
#include <math.h>

#include "device.h"
#include "kernels.h"

namespace mfm {

// blockIdx -> logical block so that XCD x (blocks x, x+8, ...) gets one contiguous range
__device__ __forceinline__ int xcd_block() {
    int G = gridDim.x, b = blockIdx.x;
    int x = b & 7, slot = b >> 3;
    int q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(v, o, 64);
        v = t > v ? t : v;
    }
    return v;
}

__device__ __forceinline__ void count_add(unsigned long long* c, unsigned long long v) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(c, v);
}

// the atomic is skipped when the counter already holds at least v (a stale
// read only costs an atomic that changes nothing)
__device__ __forceinline__ void count_max(unsigned long long* c, unsigned long long v) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0 && v && v > __atomic_load_n(c, __ATOMIC_RELAXED)) atomicMax(c, v);
}

__device__ __forceinline__ void flag_index(Counters* cnt, int i) {
    atomicMin(&cnt->first_bad, (unsigned long long)i);
}

__device__ __forceinline__ void displacement(const Phys& ph, const double xi[3], double xj0, double xj1,
                                             double xj2, double d[3]) {
    d[0] = min_image(xj0 - xi[0], ph.box[0], ph.periodic[0]);
    d[1] = min_image(xj1 - xi[1], ph.box[1], ph.periodic[1]);
    d[2] = min_image(xj2 - xi[2], ph.box[2], ph.periodic[2]);
}

// ------------------------------------------------------------ kernel length
// The root of (32/3) sum_j w(r_ij / H) = n_ngb is found per particle by
// safeguarded Newton iterations on the radii r_ij < hi of a bracket (lo, hi].
// A scan at a trial radius R collects the radii (rl) and indices (jl) within R
// into interleaved global lists (rl[k * n + i], coalesced across a wave); a
// lane whose R holds too few neighbours, or more than the list holds, adjusts R
// and scans again.  Scans are wave-cooperative: each pass takes the lanes whose
// trial radius is within a factor two of the largest one and lie close to the
// first of them, and scans their union once.  Particles the first round leaves
// without a bracket go to the per-particle list solver, one wave each, and the
// few it cannot finish to the rescanning solver.  After the root, the indices
// with r < H (self excluded) are compacted in place: the gather part of the
// flux list.

// Local density from the 3x3x3 blocks of cells around the particle's own cell:
// on the finest level l whose block holds at least kColdCount particles, and on
// level l + 1, whose block holds fewer.  log(count) is interpolated linearly in
// log(volume) between the two blocks to the volume that holds kColdCount
// particles; the guess is the radius holding n_ngb particles at that density.
// The interpolation removes most of the factor-of-8 steps between levels (on
// the clustered log-normal set the spread of log(H / guess) drops from 0.22 to
// 0.18 and the particles left without a bracket by the first scan from 17% to
// 11%).  A smaller kColdCount gives a more local estimate but a noisier one
// from particle to particle, which widens the cooperative scans (they reach the
// largest trial radius of the lanes they serve) by more than it saves.  Open
// sides shrink the blocks to the cells inside.  The search starts at the level
// where a block at the mean density would hold kColdCount particles and moves
// finer or coarser from there.
constexpr double kColdCount = 32.0;
struct BlockCount {
    double count;
    double vol;
};

__device__ BlockCount block_count(const TreeDesc& td, const int2* __restrict__ tab, const double xi[3], int l) {
    unsigned long long dil[3][3];   // deposited keys of coordinates c-1, c, c+1 per axis
    bool ok[3][3];
    int ncl[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int nc = td.ncell[l][d];
        const int c = min(nc - 1, max(0, (int)floor(xi[d] / td.cs[l][d])));
        // the neighbours c - 1 and c + 1 by dilated subtraction and addition of
        // the deposited 1 (wrapping modulo nc, which only periodic axes use)
        const unsigned long long m = td.mask[l][d];
        const unsigned long long one = m & (~m + 1);
        const unsigned long long dc = deposit_bits((unsigned)c, m);
        const unsigned long long dn[3] = {dilated_sub(dc, one, m), dc, dilated_add(dc, one, m)};
        ncl[d] = 0;
#pragma unroll
        for (int o = 0; o < 3; o++) {
            const int w = c + o - 1;
            bool in = true;
            if ((w < 0 || w >= nc) && !(td.periodic[d] && nc >= 3)) in = false;
            if (nc < 3 && o != 1) in = false;   // fewer than 3 cells: count each once
            ok[d][o] = in;
            ncl[d] += in;
            dil[d][o] = in ? dn[o] : 0ull;
        }
    }
    int cnt = 0;
    const long long off = td.tab_off[l];
#pragma unroll
    for (int ox = 0; ox < 3; ox++)
#pragma unroll
        for (int oy = 0; oy < 3; oy++)
#pragma unroll
            for (int oz = 0; oz < 3; oz++) {
                // cells outside an open side read cell 0 and count nothing
                const bool in = ok[0][ox] && ok[1][oy] && ok[2][oz];
                const int2 se = tab[off + (long long)(in ? (dil[0][ox] | dil[1][oy] | dil[2][oz]) : 0ull)];
                cnt += in ? se.y - se.x : 0;
            }
    return {(double)cnt, ncl[0] * td.cs[l][0] * ncl[1] * td.cs[l][1] * ncl[2] * td.cs[l][2]};
}

__device__ double cold_guess(const TreeDesc& td, const int2* __restrict__ tab, const double xi[3],
                             double n_ngb, long long n) {
    const double need = kColdCount;
    const double nbox = (double)n / (td.box[0] * td.box[1] * td.box[2]);
    int l = td.bmax;
    while (l > 0 && 27.0 * nbox * td.cs[l][0] * td.cs[l][1] * td.cs[l][2] < need) l--;
    BlockCount b = block_count(td, tab, xi, l);
    BlockCount f = {-1.0, 0.0};   // the finer block (count < need), once known
    if (b.count >= need) {
        while (l < td.bmax) {
            const BlockCount g = block_count(td, tab, xi, l + 1);
            if (g.count < need) {
                f = g;
                break;
            }
            b = g;
            l++;
        }
    } else {
        while (l > 0 && b.count < need) {
            f = b;
            b = block_count(td, tab, xi, --l);
        }
    }
    double vol = b.vol, count = fmax(b.count, 1.0);
    if (f.count >= 0.0 && b.count >= need && f.vol < b.vol) {
        // log count linear in log volume between the two blocks, at count = need
        const double lf = log(fmax(f.count, 0.5)), lb = log(b.count);
        const double t = (log(need) - lf) / (lb - lf);
        vol = exp(log(f.vol) + t * (log(b.vol) - log(f.vol)));
        count = need;
    }
    return cbrt(3.0 * n_ngb * vol / (4.0 * M_PI * count));
}

constexpr double kNewtonTail = 1e-9;   // last Newton step accepted without a check pass

// One safeguarded Newton update from the residual f and slope fp at Hc, inside
// the bracket (lo, hi]; true when Hc is final.  The sum is twice continuously
// differentiable in H (so is the spline), so Newton converges quadratically:
// after a step below kNewtonTail H the new iterate is within a small multiple
// of kNewtonTail^2 H (a few 1e-18 relative) of the root and is returned without
// another pass.  It is taken even at a bracket edge: an earlier iterate can
// land on the root and become lo or hi.
__device__ __forceinline__ bool newton_step(double f, double fp, double& lo, double& hi, double& Hc) {
    if (f == 0.0) return true;
    if (f < 0.0) lo = Hc;
    else hi = Hc;
    double Hn = Hc - f / fp;
    if (fabs(Hn - Hc) <= kNewtonTail * Hc) {
        Hc = fmin(hi, fmax(lo, Hn));
        return true;
    }
    if (!(Hn > lo && Hn <= hi)) Hn = 0.5 * (lo + hi);
    const double dH = fabs(Hn - Hc);
    Hc = Hn;
    return dH <= 1e-14 * Hc || !(hi - lo > 4e-16 * hi);
}

// safeguarded Newton on the m radii rl[k * n + i]; returns converged
__device__ bool newton_h(const double* __restrict__ rl, long long n, int i, int m, double n_ngb, int maxit,
                         double& lo, double& hi, double& Hc, unsigned long long& iters) {
    const double c32 = 32.0 / 3.0;
    for (int it = 0; it < maxit; it++) {
        iters++;
        const double iH = 1.0 / Hc;
        double s = 0.0, sq = 0.0;
#pragma unroll 8
        for (int k = 0; k < m; k++) {
            const double q = rl[(long long)k * n + i] * iH;
            s += spline_w(q);
            sq += spline_qdw(q);
        }
        if (newton_step(c32 * s - n_ngb, -c32 * sq * iH, lo, hi, Hc)) return true;
    }
    return false;
}

// Group scans per particle: particles the first round does not finish (no
// bracket yet, or more radii than the list holds) go to the per-particle solver,
// which is cheaper for them than further group passes over a sparse class.
constexpr int kScanRounds = 1;
constexpr double kColdPad = 1.05;   // first scan radius over a cold guess
constexpr double kWarmPad = 1.03;   // first scan radius over the previous H
constexpr double kStoreCold = 1.05;   // radii listed by a cold first scan, over the guess
// a scan pass takes the lanes with R >= kClassRatio Rref within kClassWindow Rref
// of the first of them on every axis (Rref: the largest trial radius pending).
// Fewer, wider classes pay down to a quarter: each pass scans the union once,
// and its narrow lanes' extra candidates cost less than passes of their own.
constexpr double kClassRatio = 0.25;
constexpr double kClassWindow = 2.0;

// Five waves per SIMD (96 VGPRs): the scan is latency-bound, and the extra wave
// outweighs the few loop-invariant values this budget spills to scratch.
// With HIER (hierarchical steps with active subsets) only the particles of
// mode 1 solve; the others keep their kernel length.  The cell tables may then
// be those of an earlier build: every scan reaches *pad further, the largest
// distance a particle has moved since.
constexpr int kSolveWaves = 5;
template <bool HIER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kSolveWaves))) void k_solve_h(PassArrays a, TreeDesc td, const int2* __restrict__ tab,
                                                  const double4* __restrict__ pos, Phys ph, Counters* cnt,
                                                  double* __restrict__ rl, int* __restrict__ jl,
                                                  int* __restrict__ gcount, int* __restrict__ counts,
                                                  int* __restrict__ fb_list, unsigned long long* __restrict__ fb_count,
                                                  const unsigned char* __restrict__ mode, const double* __restrict__ pad) {
    cnt = counter_copy(cnt);
    __shared__ ScanLds lds[256 / kWave];
    ScanLds& S = lds[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int i = xcd_block() * 256 + threadIdx.x;
    const bool act = i < a.n && (!HIER || mode[i] == kModeSolve);
    const long long n = a.n;
    const int cap = min(kRCap, ph.max_ngb);
    const double c32 = 32.0 / 3.0;
    double half = INFINITY;
    for (int d = 0; d < 3; d++)
        if (ph.periodic[d]) half = fmin(half, 0.5 * ph.box[d]);
    double xi[3] = {0.0, 0.0, 0.0};
    double guess = 0.0;
    bool warm = false;
    if (act) {
        const double4 pi = pos[i];
        xi[0] = pi.x;
        xi[1] = pi.y;
        xi[2] = pi.z;
        guess = a.H[i];
        warm = guess > 0.0;
        if (!warm) guess = cold_guess(td, tab, xi, ph.n_ngb, a.n);
    }
    // state 0: scanning, 1: bracketed with every radius below hi listed, 2: given up
    int state = act ? 0 : 2;
    double lo = 0.0, hi = INFINITY, top = INFINITY;   // top: smallest R whose list overflowed
    double R = (warm ? kWarmPad : kColdPad) * guess;
    double neff_hi = 0.0, fa = NAN;                   // residuals at the bracket ends
    int m = 0, rounds = 0;
    unsigned long long iters = 0;
    for (int pass = 0; pass < kScanRounds * kWave; pass++) {
        if (state == 0 && (rounds >= kScanRounds || !(R > lo))) state = 2;
        if (state == 0 && !(R < half)) {
            R = half * (1.0 - 1e-12);
            if (!(R > lo)) state = 2;   // the root lies beyond half a periodic side
        }
        const bool need = state == 0;
        if (__ballot(need) == 0) break;
        // this pass: lanes within 2x of the largest radius and within 2 Rref of the first such lane
        const double Rref = uniform_d(wave_max_d(need ? R : 0.0));
        const bool big = need && R >= kClassRatio * Rref;
        const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)__ballot(big)) - 1);
        const double xl0 = uniform_d(__shfl(xi[0], leader, kWave)), xl1 = uniform_d(__shfl(xi[1], leader, kWave)),
                     xl2 = uniform_d(__shfl(xi[2], leader, kWave));
        const double win = kClassWindow * Rref;
        const bool cls = big && fabs(xi[0] - xl0) <= win && fabs(xi[1] - xl1) <= win && fabs(xi[2] - xl2) <= win;
        const double Rq = uniform_d(wave_max_d(cls ? R : 0.0));
        double bmin[3], bmax[3];
        for (int d = 0; d < 3; d++) {
            bmin[d] = uniform_d(wave_min_d(cls ? xi[d] : INFINITY));
            bmax[d] = uniform_d(wave_max_d(cls ? xi[d] : -INFINITY));
        }
        const double R2 = R * R;
        // Weighted counts at R and at two trial lengths.  The first scan of a
        // cold start lists only the radii below kStoreCold times the guess (a
        // scan radius padded further brackets more roots in one scan; with the
        // default pads, equal to kStoreCold, every radius within R is listed),
        // with the trial lengths at the guess and at that limit; if the root lies
        // above the limit, the bracket is kept and one more scan lists them all.
        const bool part = !warm && rounds == 0 && kStoreCold > 0.0;
        const double Hg = R * (warm ? 1.0 / kWarmPad : 1.0 / kColdPad);
        const double Ht[2] = {part ? Hg : 0.97 * Hg, part ? kStoreCold * Hg : 1.03 * Hg};
        const double Sl = part ? Ht[1] : R;   // radii below Sl are listed
        const double iR = 1.0 / R, iT0 = 1.0 / Ht[0], iT1 = 1.0 / Ht[1];
        double sw = 0.0, st0 = 0.0, st1 = 0.0;
        if (cls) {
            rounds++;
            m = 0;
        }
        group_scan(td, tab, pos, S, lane, bmin, bmax, HIER ? Rq + *pad : Rq, xi, R2, cls, [&](int j, double r2) {
            const double r = sqrt(r2);
            if (r < Sl) {
                if (m < cap) {
                    rl[(long long)m * n + i] = r;
                    jl[(long long)m * n + i] = j;
                }
                m++;
            }
            sw += spline_w(r * iR);
            st0 += spline_w(r * iT0);
            st1 += spline_w(r * iT1);
        });
        if (cls) {
            const double neff = c32 * sw;
            if (neff < ph.n_ngb) {
                lo = R;
                if (hi < INFINITY) {
                    R = 0.5 * (lo + hi);
                } else {
                    // grow by the density estimate, at least 1.15x, at most 4x,
                    // and not past a radius known to overflow
                    const double g = 1.1 * cbrt(ph.n_ngb / fmax(neff, 1e-300));
                    R *= fmin(4.0, fmax(1.15, g));
                    if (top < INFINITY) R = fmin(R, 0.5 * (lo + top));
                }
            } else if (m > cap) {
                // bracketed, but too many radii to keep: rescan just above the estimated root
                hi = R;
                top = fmin(top, R);
                R = fmax(lo + 0.25 * (hi - lo), fmin(1.05 * R * cbrt(ph.n_ngb / neff), R * cbrt(0.8 * cap / m)));
                if (!(R < hi)) R = 0.5 * (lo + hi);
            } else {
                // every radius below R is listed: narrow the bracket with the trial counts
                // (summed in the same order as the Newton sums, so the signs agree)
                hi = R;
                neff_hi = neff;
                const double f0 = c32 * st0 - ph.n_ngb, f1 = c32 * st1 - ph.n_ngb;
                fa = NAN;
                if (Ht[1] < hi && Ht[1] > lo) {
                    if (f1 >= 0.0) hi = Ht[1], neff_hi = f1 + ph.n_ngb;
                    else lo = Ht[1], fa = f1;
                }
                if (Ht[0] < hi && Ht[0] > lo) {
                    if (f0 >= 0.0) hi = Ht[0], neff_hi = f0 + ph.n_ngb;
                    else lo = Ht[0], fa = f0;
                }
                if (hi > Sl) {
                    // the root lies above the listed radii: list them all up to hi
                    R = hi;
                } else {
                    state = 1;
                }
            }
        }
    }
    bool conv = false;
    double Hc = 0.0;
    if (state == 1) {
        // start from the secant of the bracket when both ends carry a residual,
        // else from the density scaling of the upper end
        const double fb = neff_hi - ph.n_ngb;
        if (fa < 0.0 && fb >= 0.0) Hc = lo + (hi - lo) * (-fa / (fb - fa));
        else Hc = (warm && guess > lo && guess < hi) ? guess : hi * cbrt(ph.n_ngb / neff_hi);
        if (!(Hc > lo && Hc <= hi)) Hc = 0.5 * (lo + hi);
        conv = newton_h(rl, n, i, m, ph.n_ngb, ph.h_maxit, lo, hi, Hc, iters);
    }
    if (state == 1 && conv) {
        double sum = 0.0;
        const double iH = 1.0 / Hc;
        int c = 0;
#pragma unroll 4
        for (int k = 0; k < m; k++) {
            const double r = rl[(long long)k * n + i];
            sum += spline_w(r * iH);
            const int j = jl[(long long)k * n + i];
            if (r < Hc && j != i) {
                jl[(long long)c * n + i] = j;
                c++;
            }
        }
        const double nk = kernel_norm(Hc) * sum;
        a.H[i] = Hc;
        a.nk[i] = nk;
        a.V[i] = 1.0 / nk;
        gcount[i] = c;
        counts[i] = c;
    } else if (act) {
        // hand over to the per-particle solver: the bracket and the next trial
        // radius, in the particle's own (now unused) radius slots 0-2
        const unsigned long long slot = atomicAdd(fb_count, 1ull);
        if (slot < (unsigned long long)a.n) fb_list[slot] = i;
        rl[i] = lo;
        rl[n + i] = hi;
        rl[2 * n + i] = R;
        a.H[i] = (hi < INFINITY) ? hi : (lo > 0.0 ? lo : guess);
    }
    const unsigned long long rr = (unsigned long long)rounds;
    count_add(&cnt->h_iters, iters + rr);
    count_max(&cnt->h_iters_max, iters + rr);
    count_max(&cnt->h_rounds_max, rr);
    count_add(&cnt->h_rounds3, rounds >= 3 ? 1ull : 0ull);
}

// Particles the group scan hands over, one wave each.  The wave scans the cells
// within a trial radius once and keeps every radius and index within it in
// registers (entry e on lane e mod 64, slot e / 64, scan order), narrows the
// bracket with the weighted count at that radius, and once the radius brackets
// the root with every radius kept, runs Newton on them with wave-wide sums in
// a fixed order.  Particles whose radii do not fit, or that find no bracket
// within kWaveScans scans, go on to the rescanning solver below.
constexpr int kWaveSlots = 3;   // entries per lane kept by the list solver (ra, rb, rc)
constexpr int kWaveScans = 16;
// At five waves per SIMD 5,120 waves are resident; 32,768 single-wave blocks
// (about 87 particles each on the clustered set) balance the end of the
// launch better than 16,384 (45.2 -> 44.5 ms for the solve stage).
constexpr int kWaveBlocks = 32768;   // waves of the list solver, striding over its particles
// a single sphere's scan enumerates its cells at a coarser level than a group's
constexpr double kWaveScanScale = 0.5;

// Five waves per SIMD: the list solver fits in 96 registers without spills,
// and the fifth wave hides more of its scans' load latency than four.
constexpr int kWaveSolveWaves = 5;
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kWaveSolveWaves))) void k_solve_h_wave(
                                                      PassArrays a, TreeDesc td, const int2* __restrict__ tab,
                                                      const double4* __restrict__ pos, Phys ph, Counters* cnt,
                                                      const int* __restrict__ fb_list,
                                                      const unsigned long long* __restrict__ fb_count,
                                                      const double* __restrict__ hand, int* __restrict__ jl,
                                                      int* __restrict__ gcount, int* __restrict__ counts,
                                                      int* __restrict__ fb2_list,
                                                      unsigned long long* __restrict__ fb2_count,
                                                      const double* __restrict__ pad) {
    cnt = counter_copy(cnt);
    __shared__ ScanLds S;
    const int lane = threadIdx.x;
    const unsigned long long nfb = min(*fb_count, (unsigned long long)a.n);
    const double pd = pad ? *pad : 0.0;
    if (blockIdx.x == 0 && lane == 0) cnt->h_fallback = *fb_count;
    const long long n = a.n;
    constexpr int kKeep = kWaveSlots * kWave;
    const double c32 = 32.0 / 3.0;
    double half = INFINITY;
    for (int d = 0; d < 3; d++)
        if (ph.periodic[d]) half = fmin(half, 0.5 * ph.box[d]);
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long iters = 0, iters_max = 0, over = 0, scans_max = 0, many = 0;
    for (unsigned long long t = blockIdx.x; t < nfb; t += gridDim.x) {
        const unsigned long long iters0 = iters;
        const int i = __builtin_amdgcn_readfirstlane(fb_list[t]);
        const double4 pi = pos[i];
        const double xi[3] = {uniform_d(pi.x), uniform_d(pi.y), uniform_d(pi.z)};
        double lo = uniform_d(hand[i]), hi = uniform_d(hand[n + i]), R = uniform_d(hand[2 * n + i]);
        if (!(R > lo)) R = (hi < INFINITY) ? hi : 1.3 * lo;
        // the kept entries of this lane: slots 0-2 (named, so they stay in registers)
        double ra = INFINITY, rb = INFINITY, rc = INFINITY;
        int ja = -1, jb = -1, jc = -1;
        int m = 0, scans = 0;
        double neff_hi = 0.0;
        bool bracketed = false;
        while (scans < kWaveScans) {
            if (!(R < half)) R = half * (1.0 - 1e-12);
            if (!(R > lo)) break;
            scans++;
            iters++;
            const double R2 = R * R, iR = 1.0 / R;
            double sw = 0.0;
            m = 0;
            ra = rb = rc = INFINITY;
            ja = jb = jc = -1;
            scan_cells(td, tab, pos, S, lane, xi, xi, R + pd, [&](const double4& q, bool valid, int, int wrap) {
                const double r2 = sq_disp(q, xi, wrap, td.box);
                const bool in = valid && r2 < R2;
                const double r = sqrt(r2);
                if (in) sw += spline_w(r * iR);
                // new entries m .. m + cin - 1 go to lanes (m + rank) mod 64; the
                // other lanes send to the remaining lanes, so every lane gets one value
                const unsigned long long b = __ballot(in);
                const int cin = __popcll(b);
                const int rank = in ? __popcll(b & below) : cin + __popcll(~b & below);
                const int dest = (m + rank) & (kWave - 1);
                const long long rbits = __double_as_longlong(r);
                const int rlo = __builtin_amdgcn_ds_permute(dest * 4, (int)rbits);
                const int rhi = __builtin_amdgcn_ds_permute(dest * 4, (int)(rbits >> 32));
                const int jv = __builtin_amdgcn_ds_permute(dest * 4, (int)__double_as_longlong(q.w));
                const int off = (lane - m) & (kWave - 1);
                if (off < cin) {
                    const int sl = (m + off) / kWave;
                    const double rv = __longlong_as_double(((long long)rhi << 32) | (unsigned)rlo);
                    ra = sl == 0 ? rv : ra;
                    ja = sl == 0 ? jv : ja;
                    rb = sl == 1 ? rv : rb;
                    jb = sl == 1 ? jv : jb;
                    rc = sl == 2 ? rv : rc;
                    jc = sl == 2 ? jv : jc;
                }
                m += cin;
            }, kWaveScanScale);
            sw = uniform_d(wave_sum_d(sw));
            const double neff = c32 * sw;
            if (m > kKeep) {
                // too many radii to keep; below n_ngb the root lies beyond them all
                if (neff < ph.n_ngb) break;
                hi = fmin(hi, R);
                R = fmax(lo + 0.25 * (hi - lo), fmin(1.05 * R * cbrt(ph.n_ngb / neff), R * cbrt(0.8 * kKeep / m)));
                if (!(R < hi)) R = 0.5 * (lo + hi);
            } else if (neff < ph.n_ngb) {
                lo = R;
                if (hi < INFINITY) {
                    R = hi;
                } else {
                    const double g = 1.1 * cbrt(ph.n_ngb / fmax(neff, 1e-300));
                    R *= fmin(4.0, fmax(1.15, g));
                }
            } else {
                hi = R;
                neff_hi = neff;
                bracketed = true;
                break;
            }
        }
        bool conv = false;
        double Hc = hi;
        if (bracketed) {
            Hc = hi * cbrt(ph.n_ngb / neff_hi);
            if (!(Hc > lo && Hc <= hi)) Hc = 0.5 * (lo + hi);
            for (int it = 0; it < ph.h_maxit; it++) {
                iters++;
                const double iH = 1.0 / Hc;
                double s = 0.0, sq = 0.0;
                const double rs[kWaveSlots] = {ra, rb, rc};
#pragma unroll
                for (int sl = 0; sl < kWaveSlots; sl++)
                    if (sl * kWave + lane < m) {
                        const double q = rs[sl] * iH;
                        s += spline_w(q);
                        sq += spline_qdw(q);
                    }
                s = uniform_d(wave_sum_d(s));
                sq = uniform_d(wave_sum_d(sq));
                if (newton_step(c32 * s - ph.n_ngb, -c32 * sq * iH, lo, hi, Hc)) {
                    conv = true;
                    break;
                }
            }
        }
        if (!conv) {
            // on to the rescanning solver, which grows a bracket from a.H
            if (lane == 0) {
                const unsigned long long slot = atomicAdd(fb2_count, 1ull);
                if (slot < (unsigned long long)a.n) fb2_list[slot] = i;
                a.H[i] = (hi < INFINITY) ? hi : R;
            }
            continue;
        }
        // gather list: every kept index with r < H but the particle itself, in scan order
        const double iH = 1.0 / Hc;
        double sum = 0.0;
        int c = 0;
        const double rs[kWaveSlots] = {ra, rb, rc};
        const int js[kWaveSlots] = {ja, jb, jc};
#pragma unroll
        for (int sl = 0; sl < kWaveSlots; sl++) {
            const bool have = sl * kWave + lane < m;
            if (have) sum += spline_w(rs[sl] * iH);
            const bool in = have && rs[sl] < Hc && js[sl] != i;
            const unsigned long long b = __ballot(in);
            const int slot = c + __popcll(b & below);
            if (in && slot < ph.max_ngb) jl[(long long)slot * n + i] = js[sl];
            c += __popcll(b);
        }
        sum = wave_sum_d(sum);
        if (c > ph.max_ngb) {
            c = ph.max_ngb;
            over = 1;
            if (lane == 0) flag_index(cnt, i);
        }
        if (lane == 0) {
            const double nk = kernel_norm(Hc) * sum;
            a.H[i] = Hc;
            a.nk[i] = nk;
            a.V[i] = 1.0 / nk;
            gcount[i] = c;
            counts[i] = c;
        }
        iters_max = max(iters_max, iters - iters0);
        scans_max = max(scans_max, (unsigned long long)scans);
        many += (1 + scans >= 3) ? 1ull : 0ull;
    }
    if (lane == 0) {
        if (iters) atomicAdd(&cnt->h_iters, iters);
        if (iters_max) atomicMax(&cnt->h_iters_max, iters_max);
        if (scans_max) atomicMax(&cnt->h_rounds_max, 1 + scans_max);
        if (many) atomicAdd(&cnt->h_rounds3, many);
        if (over) atomicAdd(&cnt->overflow, over);
    }
}

// Solve for the few particles the list solver handed on (no bracket within its
// scans, or more radii than it keeps): one wave per particle,
// every residual evaluation scans the cells within H again with the lanes
// splitting the particles, so there is no limit on the number of neighbours.
// The bracket grows from the handed-over H until it holds the root, then
// Newton with bisection safeguard; a last scan writes the gather list.
__global__ __launch_bounds__(64) void k_solve_h_fallback(PassArrays a, TreeDesc td, const int2* __restrict__ tab,
                                                          const double4* __restrict__ pos, Phys ph, Counters* cnt,
                                                          const int* __restrict__ fb_list,
                                                          const unsigned long long* __restrict__ fb_count,
                                                          int* __restrict__ jl, int* __restrict__ gcount,
                                                          int* __restrict__ counts, const double* __restrict__ pad) {
    cnt = counter_copy(cnt);
    __shared__ ScanLds S;
    const int lane = threadIdx.x;
    const double pd = pad ? *pad : 0.0;
    const unsigned long long nfb = min(*fb_count, (unsigned long long)a.n);
    if (blockIdx.x == 0 && lane == 0) cnt->h_rescan = *fb_count;
    const long long n = a.n;
    const double c32 = 32.0 / 3.0;
    double half = INFINITY;
    for (int d = 0; d < 3; d++)
        if (ph.periodic[d]) half = fmin(half, 0.5 * ph.box[d]);
    unsigned long long iters = 0, iters_max = 0, noconv = 0, noimg = 0, over = 0;
    for (unsigned long long t = blockIdx.x; t < nfb; t += gridDim.x) {
        const unsigned long long iters0 = iters;
        const int i = __builtin_amdgcn_readfirstlane(fb_list[t]);
        const double4 pi = pos[i];
        const double xi[3] = {uniform_d(pi.x), uniform_d(pi.y), uniform_d(pi.z)};
        // residual and slope at H, summing over r < H
        auto eval = [&](double H, double& f, double& fp, double& nk) {
            const double H2 = H * H, iH = 1.0 / H;
            double s = 0.0, sq = 0.0;
            scan_cells(td, tab, pos, S, lane, xi, xi, H + pd, [&](const double4& q, bool valid, int, int wrap) {
                const double r2 = sq_disp(q, xi, wrap, td.box);
                if (valid && r2 < H2) {
                    const double qq = sqrt(r2) * iH;
                    s += spline_w(qq);
                    sq += spline_qdw(qq);
                }
            });
            s = uniform_d(wave_sum_d(s));
            sq = uniform_d(wave_sum_d(sq));
            f = c32 * s - ph.n_ngb;
            fp = -c32 * sq * iH;
            nk = kernel_norm(H) * s;
        };
        double lo = 0.0, hi = a.H[i];
        hi = uniform_d(hi);
        double f, fp, nk;
        bool ok = false;
        for (int k = 0; k < 64; k++) {
            iters++;
            if (!(hi < half)) hi = half * (1.0 - 1e-12);
            eval(hi, f, fp, nk);
            if (f >= 0.0) {
                ok = true;
                break;
            }
            if (!(hi < half * (1.0 - 1e-13))) break;
            lo = hi;
            hi *= 1.3;
        }
        bool conv = false;
        double Hc = hi;
        if (ok) {
            Hc = 0.5 * (lo + hi);
            for (int it = 0; it < ph.h_maxit; it++) {
                iters++;
                eval(Hc, f, fp, nk);
                if (newton_step(f, fp, lo, hi, Hc)) {
                    conv = true;
                    break;
                }
            }
        }
        int c = 0;
        if (ok && conv) {
            eval(Hc, f, fp, nk);
            const double H2 = Hc * Hc;
            const int cap = ph.max_ngb;
            // every gather neighbour but the particle itself, in scan order
            scan_cells(td, tab, pos, S, lane, xi, xi, Hc + pd, [&](const double4& q, bool valid, int, int wrap) {
                const double r2 = sq_disp(q, xi, wrap, td.box);
                const int j = (int)__double_as_longlong(q.w);
                const bool in = valid && r2 < H2 && j != i && sqrt(r2) < Hc;
                const unsigned long long b = __ballot(in);
                const int slot = c + __popcll(b & ((1ull << lane) - 1ull));
                if (in && slot < cap) jl[(long long)slot * n + i] = j;
                c += __popcll(b);
            });
            if (c > cap) {
                c = cap;
                over = 1;
                if (lane == 0) flag_index(cnt, i);
            }
        } else {
            nk = 0.0;
            if (!ok) noimg = 1;
            else noconv = 1;
            if (lane == 0) flag_index(cnt, i);
        }
        if (lane == 0) {
            a.H[i] = Hc;
            a.nk[i] = nk;
            a.V[i] = 1.0 / nk;
            gcount[i] = c;
            counts[i] = c;
        }
        iters_max = max(iters_max, iters - iters0);
    }
    if (lane == 0) {
        if (iters) atomicAdd(&cnt->h_iters, iters);
        if (iters_max) atomicMax(&cnt->h_iters_max, iters_max);
        if (noconv) atomicAdd(&cnt->noconv, noconv);
        if (noimg) atomicAdd(&cnt->minimage, noimg);
        if (over) atomicAdd(&cnt->overflow, over);
    }
}

// Hierarchical steps with active subsets: a particle that keeps its kernel
// length and has an active particle within reach (mode kModeKept) lists its
// gather set r < H at the current positions with the scan and the distance
// test of the kernel-length solve, so that both particles of a pair decide on
// the same distance.  The lanes of a wave (Morton neighbours) scan together
// over the largest of their radii.
__global__ __launch_bounds__(256) void k_gather_kept(PassArrays a, TreeDesc td, const int2* __restrict__ tab,
                                                     const double4* __restrict__ pos, Phys ph,
                                                     const unsigned char* __restrict__ mode, const double* __restrict__ pad,
                                                     int* __restrict__ jl, int* __restrict__ gcount,
                                                     int* __restrict__ counts) {
    __shared__ ScanLds lds[256 / kWave];
    ScanLds& S = lds[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int i = xcd_block() * 256 + threadIdx.x;
    const bool sel = i < a.n && mode[i] == kModeKept;
    if (__ballot(sel) == 0) return;   // uniform over the wave
    const long long n = a.n;
    double xi[3] = {0.0, 0.0, 0.0};
    double H = 0.0;
    if (sel) {
        const double4 p = pos[i];
        xi[0] = p.x;
        xi[1] = p.y;
        xi[2] = p.z;
        H = a.H[i];
    }
    // scanned a little beyond H, so that no r < H is lost to the rounding of r^2
    const double Rs = H * (1.0 + 1e-9);
    const double Rq = uniform_d(wave_max_d(sel ? Rs : 0.0));
    double bmin[3], bmax[3];
    for (int d = 0; d < 3; d++) {
        bmin[d] = uniform_d(wave_min_d(sel ? xi[d] : INFINITY));
        bmax[d] = uniform_d(wave_max_d(sel ? xi[d] : -INFINITY));
    }
    const int cap = ph.max_ngb;
    int c = 0;
    group_scan(td, tab, pos, S, lane, bmin, bmax, Rq + *pad, xi, Rs * Rs, sel, [&](int j, double r2) {
        const double r = sqrt(r2);
        if (r < H && j != i) {
            if (c < cap) jl[(long long)c * n + i] = j;
            c++;
        }
    });
    if (sel) {
        gcount[i] = min(c, cap);
        counts[i] = c;   // beyond cap: an overflow, counted when the tails are sorted
    }
}

// --------------------------------------------------------------- flux lists
// The flux set r < max(H_i, H_j) is the gather set of i plus every j that has
// i in its gather set with r >= H_i.  The gradient kernel, which walks every
// gather list anyway, appends each such j to i's list (atomic slot); then each
// list sorts its appended tail by index so the list, and every sum over it, is
// deterministic.
constexpr int kTailNet = kTailBuf;   // tails up to this length are buffered and sorted in registers
static_assert(kTailNet % 4 == 0, "tail buffers are read as int4");

// bitonic sorting network on N registers (indices fixed at compile time)
template <int N>
__device__ __forceinline__ void bitonic_net(int* v) {
#pragma unroll
    for (int w = 2; w <= N; w <<= 1)
#pragma unroll
        for (int h = w >> 1; h > 0; h >>= 1)
#pragma unroll
            for (int k = 0; k < N; k++) {
                const int l = k ^ h;
                if (l > k) {
                    const int lo_v = min(v[k], v[l]), hi_v = max(v[k], v[l]);
                    const bool up = (k & w) == 0;
                    v[k] = up ? lo_v : hi_v;
                    v[l] = up ? hi_v : lo_v;
                }
            }
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// The tail of particle i (entries gcount[i] .. counts[i]-1 of its flux list,
// appended by other particles in no fixed order: the first kTailNet in i's
// contiguous tail buffer, the rest in the list) is sorted by index into the
// list, so every later sum over the list runs in one order.  A short tail is
// read from the buffer with vector loads, sorted in registers by a network
// sized to the wave's longest tail, and written through per-lane LDS columns
// a row at a time (the list is interleaved, list[k * n + i], and tails start
// at different rows), each store one coalesced row segment of the wave's
// columns.  Longer tails are ranked by the whole wave in LDS.
__global__ __launch_bounds__(256) void k_sort_tails(int n, int cap, const int* __restrict__ gcount,
                                                     int* __restrict__ counts, int* __restrict__ list,
                                                     const int* __restrict__ tails, Counters* cnt) {
    cnt = counter_copy(cnt);
    __shared__ int col[kTailNet][256];
    const int i = xcd_block() * 256 + threadIdx.x;
    unsigned long long c = 0, over = 0, gsum = 0;
    int g = 0, t = 0;
    if (i < n) {
        g = gcount[i];
        gsum = (unsigned long long)g;
        int e = counts[i];
        c = (unsigned long long)e;
        if (e > cap) {
            over = 1;
            flag_index(cnt, i);
            e = cap;
            counts[i] = cap;
        }
        t = e - g;
    }
    const bool net = t > 0 && t <= kTailNet;
    const int tmax = wave_max_i(net ? t : 0);
    if (tmax > 0) {
        int v[kTailNet];
        if (net) {
            const int4* tb = (const int4*)(tails + (long long)i * kTailNet);
#pragma unroll
            for (int q = 0; q < kTailNet / 4; q++) {
                const int4 x = tb[q];
                v[4 * q] = x.x;
                v[4 * q + 1] = x.y;
                v[4 * q + 2] = x.z;
                v[4 * q + 3] = x.w;
            }
        }
#pragma unroll
        for (int k = 0; k < kTailNet; k++) v[k] = net && k < t ? v[k] : INT_MAX;
        if (tmax <= 8) bitonic_net<8>(v);
        else if (tmax <= 16) bitonic_net<16>(v);
        else bitonic_net<kTailNet>(v);
#pragma unroll
        for (int k = 0; k < kTailNet; k++)
            if (k < t && net) col[k][threadIdx.x] = v[k];
        const int rlo = wave_min_i(net ? g : INT_MAX);
        const int rhi = wave_max_i(net ? g + t : INT_MIN);
        for (int r = rlo; r < rhi; r++)
            if (net && r >= g && r < g + t) list[(long long)r * n + i] = col[r - g][threadIdx.x];
    }
    // Long tails, one at a time per wave: the tail goes to a contiguous LDS
    // region of the wave, every lane ranks its entries against all of them (ties,
    // which a list does not hold, by position) and writes each entry to its slot.
    __syncthreads();   // every wave is done with the columns
    int* wb = &col[0][0] + (threadIdx.x >> 6) * (kTailNet * kWave);
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long lm = __ballot(t > kTailNet && t <= kTailNet * kWave);
    while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1;
        const int gs = __shfl(g, src, kWave), ts = __shfl(t, src, kWave), is = __shfl(i, src, kWave);
        for (int k = lane; k < ts; k += kWave)
            wb[k] = k < kTailNet ? tails[(long long)is * kTailNet + k] : list[(long long)(gs + k) * n + is];
        wave_lds_sync();
        for (int k = lane; k < ts; k += kWave) {
            const int v = wb[k];
            int rank = 0;
            for (int q = 0; q < ts; q++) {
                const int u = wb[q];
                rank += (u < v || (u == v && q < k)) ? 1 : 0;
            }
            list[(long long)(gs + rank) * n + is] = v;
        }
        wave_lds_sync();   // the next tail overwrites the region
    }
    if (t > kTailNet * kWave) {
        // beyond what the wave's LDS region holds: move the buffer in, then sort in place
        for (int k = 0; k < kTailNet; k++) list[(long long)(g + k) * n + i] = tails[(long long)i * kTailNet + k];
        for (int k = g + 1; k < g + t; k++) {
            const int v = list[(long long)k * n + i];
            int q = k - 1;
            while (q >= g && list[(long long)q * n + i] > v) {
                list[(long long)(q + 1) * n + i] = list[(long long)q * n + i];
                q--;
            }
            list[(long long)(q + 1) * n + i] = v;
        }
    }
    count_add(&cnt->list_entries, c);
    count_add(&cnt->gather_entries, gsum);
    count_max(&cnt->list_max, c);
    count_add(&cnt->overflow, over);
}

// ---------------------------------------------------------------- gradients
// Record of one particle for the flux kernel (32 slots, one or two cache lines):
// 0-2 x, y, z (FP64 record; the FP32 record holds the FP64 pressure in 0-1) | 3 1/H | 4 K = V^2 8/(pi H^3) | 5 rho | 6 P | 7-9 v | 10-15 B |
// 16-30 grad | 31 c.  With 1/H and K per particle a face needs no division for its kernel weights:
// V^2 W(r, H) = K w(r/H).
enum { R_X = 0, R_IH = 3, R_K = 4, R_RHO = 5, R_P = 6, R_V0 = 7, R_B = 10, R_G = 16, R_C = 31 };

// What the gradient kernel reads of a neighbour, packed into one 128-byte line
// per particle: (x, y, z, H), (rho, vx, vy, vz), (P, gather count, mode, -),
// unused; the mode (hierarchical steps with active subsets) is 0 without one.
__device__ __forceinline__ void pack_one(const PassArrays& a, const Phys& ph, const int* __restrict__ gcount,
                                         const unsigned char* __restrict__ mode, double4* __restrict__ prim, int i) {
    const double rho = a.m[i] * a.nk[i];
    prim[4 * (long long)i + 0] = make_double4(a.x[i], a.y[i], a.z[i], a.H[i]);
    prim[4 * (long long)i + 1] = make_double4(rho, a.vx[i], a.vy[i], a.vz[i]);
    prim[4 * (long long)i + 2] = make_double4((ph.gamma - 1.0) * rho * a.u[i], (double)gcount[i],
                                              mode ? (double)mode[i] : 0.0, 0.0);
}

__global__ void k_pack_prim(PassArrays a, Phys ph, const int* __restrict__ gcount,
                            const unsigned char* __restrict__ mode, double4* __restrict__ prim) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    pack_one(a, ph, gcount, mode, prim, i);
}

// A boundary with active subsets reads the records of the active particles'
// gather neighbours (their gradients) and of the active particles themselves
// (the kept particles' tail appends) only: each active particle packs its own
// and its gather neighbours' records.  A record packed by several of them gets
// the same values from each.  The others keep stale records, which no kernel
// of that boundary reads.
__global__ void k_pack_prim_active(PassArrays a, Phys ph, const int* __restrict__ gcount,
                                   const unsigned char* __restrict__ mode, const int* __restrict__ list,
                                   double4* __restrict__ prim) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n || mode[i] != kModeSolve) return;
    const long long n = a.n;
    pack_one(a, ph, gcount, mode, prim, i);
    const int cnum = gcount[i];
    for (int k = 0; k < cnum; k++) pack_one(a, ph, gcount, mode, prim, list[(long long)k * n + i]);
}

// i is outside j's gather set: the pair enters j's flux list as a tail entry
// (slots past the gather part, sorted afterwards); the first kTailNet go to
// j's contiguous tail buffer, so the appends to one particle share a cache
// line, the rest to the list itself
__device__ __forceinline__ void append_tail(int* __restrict__ counts, int* __restrict__ tails,
                                            int* __restrict__ list, int cap, long long n, int j, int jgather, int i) {
    const int slot = atomicAdd(&counts[j], 1);
    const int st = slot - jgather;
    if (st < kTailNet) tails[(long long)j * kTailNet + st] = i;
    else if (slot < cap) list[(long long)slot * n + j] = i;
}

// Four waves per SIMD (128 VGPRs, no spills): the kernel waits on the gathers
// of its neighbours' records, and a fourth wave hides more of that than the
// register budget it takes costs.
// With HIER (hierarchical steps with active subsets) only the particles of
// mode kModeSolve get new gradients; a kept particle with a gather list only
// appends itself to the lists of its active neighbours that do not reach it.
constexpr int kGradWaves = 4;
template <bool MIXED, bool HIER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kGradWaves))) void k_gradients(PassArrays a, Phys ph, const int* __restrict__ gcount,
                                                    int* __restrict__ counts, int* __restrict__ list, int* __restrict__ tails,
                                                    const double4* __restrict__ prim, void* __restrict__ recp,
                                                    Counters* cnt, const unsigned char* __restrict__ mode,
                                                    const long long* __restrict__ home) {
    cnt = counter_copy(cnt);
    const int i = xcd_block() * 256 + threadIdx.x;
    if (HIER && i < a.n && mode[i] == kModeKept) {
        const long long n = a.n;
        const double xi[3] = {a.x[i], a.y[i], a.z[i]};
        const int cnum = gcount[i];
        for (int k = 0; k < cnum; k++) {
            const int j = list[(long long)k * n + i];
            if (mode[j] != kModeSolve) continue;   // the pair is not due (and j's record may be stale)
            const double4 pj = prim[4 * (long long)j + 0];
            const double4 pg = prim[4 * (long long)j + 2];
            double d[3];
            displacement(ph, xi, pj.x, pj.y, pj.z, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(r < pj.w)) append_tail(counts, tails, list, ph.max_ngb, n, j, (int)pg.y, i);
        }
    }
    const bool act = i < a.n && (!HIER || mode[i] == kModeSolve);
    unsigned long long ill = 0, nonfin = 0, condbits = 0;
    if (act) {
        const long long n = a.n;
        const double xi[3] = {a.x[i], a.y[i], a.z[i]};
        const double Hi = a.H[i], Vi = a.V[i];
        const double rho_i = a.m[i] * a.nk[i];
        const double P_i = (ph.gamma - 1.0) * rho_i * a.u[i];
        const double phi_i[5] = {rho_i, a.vx[i], a.vy[i], a.vz[i], P_i};
        double E[6] = {0, 0, 0, 0, 0, 0};
        double S[15];
        double pmax[5], pmin[5];
#pragma unroll
        for (int k = 0; k < 15; k++) S[k] = 0.0;
#pragma unroll
        for (int f = 0; f < 5; f++) pmax[f] = pmin[f] = phi_i[f];
        double rmax = 0.0;
        const double norm = kernel_norm(Hi), iH = 1.0 / Hi;
        const float normf = (float)norm, iHf = (float)iH;
        const int cnum = gcount[i];
        const int cap = ph.max_ngb;
        // the next list entry is loaded one neighbour ahead, so the record
        // loads do not wait for their index
        int jn = cnum > 0 ? list[i] : 0;
        for (int k = 0; k < cnum; k++) {
            const int j = jn;
            if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
            const double4 pj = prim[4 * (long long)j + 0];
            const double4 qj = prim[4 * (long long)j + 1];
            const double2 pg = *(const double2*)&prim[4 * (long long)j + 2];
            const double Pj = pg.x;
            double d[3];
            displacement(ph, xi, pj.x, pj.y, pj.z, d);
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(r < pj.w)) append_tail(counts, tails, list, cap, n, j, (int)pg.y, i);
            const double phi_j[5] = {qj.x, qj.y, qj.z, qj.w, Pj};
            if (!MIXED) {
                const double psi = norm * spline_w(r * iH) * Vi;
                E[0] += d[0] * d[0] * psi;
                E[1] += d[0] * d[1] * psi;
                E[2] += d[0] * d[2] * psi;
                E[3] += d[1] * d[1] * psi;
                E[4] += d[1] * d[2] * psi;
                E[5] += d[2] * d[2] * psi;
#pragma unroll
                for (int f = 0; f < 5; f++) {
                    const double df = (phi_j[f] - phi_i[f]) * psi;
                    S[3 * f + 0] += df * d[0];
                    S[3 * f + 1] += df * d[1];
                    S[3 * f + 2] += df * d[2];
                }
            } else {
                // the pairwise kernel weight in FP32; the moments and sums in FP64, so
                // that E and the gradient sums share one set of weights and the
                // conditioning of E does not amplify per-product rounding
                const double psi = (double)(normf * spline_w((float)r * iHf)) * Vi;
                E[0] += d[0] * d[0] * psi;
                E[1] += d[0] * d[1] * psi;
                E[2] += d[0] * d[2] * psi;
                E[3] += d[1] * d[1] * psi;
                E[4] += d[1] * d[2] * psi;
                E[5] += d[2] * d[2] * psi;
#pragma unroll
                for (int f = 0; f < 5; f++) {
                    const double df = (phi_j[f] - phi_i[f]) * psi;
                    S[3 * f + 0] += df * d[0];
                    S[3 * f + 1] += df * d[1];
                    S[3 * f + 2] += df * d[2];
                }
            }
#pragma unroll
            for (int f = 0; f < 5; f++) {
                pmax[f] = fmax(pmax[f], phi_j[f]);
                pmin[f] = fmin(pmin[f], phi_j[f]);
            }
            rmax = fmax(rmax, r);
        }
        // B = E^-1 by cofactors (E symmetric: xx xy xz yy yz zz)
        const double c00 = E[3] * E[5] - E[4] * E[4];
        const double c01 = E[2] * E[4] - E[1] * E[5];
        const double c02 = E[1] * E[4] - E[2] * E[3];
        const double c11 = E[0] * E[5] - E[2] * E[2];
        const double c12 = E[1] * E[2] - E[0] * E[4];
        const double c22 = E[0] * E[3] - E[1] * E[1];
        const double det = E[0] * c00 + E[1] * c01 + E[2] * c02;
        const double idet = 1.0 / det;
        const double B[6] = {c00 * idet, c01 * idet, c02 * idet, c11 * idet, c12 * idet, c22 * idet};
        const double fe = E[0] * E[0] + E[3] * E[3] + E[5] * E[5] + 2.0 * (E[1] * E[1] + E[2] * E[2] + E[4] * E[4]);
        const double fb = B[0] * B[0] + B[3] * B[3] + B[5] * B[5] + 2.0 * (B[1] * B[1] + B[2] * B[2] + B[4] * B[4]);
        const double cond = sqrt(fe) * sqrt(fb);
        if (!(det > 0.0) || !(cond <= ph.cond_max)) {
            ill = 1;
            flag_index(cnt, i);
        }
        if (cond > 0.0) condbits = __double_as_longlong(cond);
        // the limiter constant: beta, or with the optional limiters (R24) beta moved
        // towards beta_min linearly in log10(cond) between cond_lo and cond_hi
        double beta = ph.beta;
        if (ph.limiter) {
            double t;
            if (cond <= ph.cond_lo) t = 0.0;
            else if (cond < ph.cond_hi) t = (log10(cond) - log10(ph.cond_lo)) / (log10(ph.cond_hi) - log10(ph.cond_lo));
            else t = 1.0;
            beta = ph.beta + (ph.beta_min - ph.beta) * t;
        }
        double g[15];
        double al[5];
        const double half = 0.5 * rmax;
#pragma unroll
        for (int f = 0; f < 5; f++) {
            const double* s = S + 3 * f;
            const double g0 = B[0] * s[0] + B[1] * s[1] + B[2] * s[2];
            const double g1 = B[1] * s[0] + B[3] * s[1] + B[4] * s[2];
            const double g2 = B[2] * s[0] + B[4] * s[1] + B[5] * s[2];
            double alpha;
            if (!MIXED) {
                const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
                alpha = 1.0;
                if (gn > 0.0) {
                    const double up = (pmax[f] - phi_i[f]) / (gn * half);
                    const double dn = (phi_i[f] - pmin[f]) / (gn * half);
                    alpha = fmin(1.0, beta * fmin(up, dn));
                }
            } else {
                const float h0 = (float)g0, h1 = (float)g1, h2 = (float)g2;
                const float gn = sqrtf(h0 * h0 + h1 * h1 + h2 * h2);
                float af = 1.0f;
                if (gn > 0.0f) {
                    const float hf = (float)half;
                    const float up = (float)(pmax[f] - phi_i[f]) / (gn * hf);
                    const float dn = (float)(phi_i[f] - pmin[f]) / (gn * hf);
                    af = fminf(1.0f, (float)beta * fminf(up, dn));
                }
                alpha = (double)af;
            }
            al[f] = alpha;
            g[3 * f + 0] = alpha * g0;
            g[3 * f + 1] = alpha * g1;
            g[3 * f + 2] = alpha * g2;
        }
        const long long io = HIER ? home[i] : i;   // column of B, grad and alpha
#pragma unroll
        for (int k = 0; k < 6; k++) a.B[k * n + io] = B[k];
#pragma unroll
        for (int k = 0; k < 15; k++) {
            a.grad[k * n + io] = g[k];
            if (!isfinite(g[k])) nonfin = 1;
        }
        if (a.alpha) {
#pragma unroll
            for (int f = 0; f < 5; f++) a.alpha[f * n + io] = al[f];
        }
        a.rho[i] = rho_i;
        a.P[i] = P_i;
        const double c_i = sqrt(ph.gamma * P_i / rho_i);
        if (!MIXED) {
            double* rec = (double*)recp + (long long)i * 32;
            double v[32];
            v[0] = xi[0];
            v[1] = xi[1];
            v[2] = xi[2];
            v[R_IH] = iH;
            v[R_K] = Vi * Vi * norm;
            v[R_RHO] = rho_i;
            v[R_P] = P_i;
            v[R_V0 + 0] = phi_i[1];
            v[R_V0 + 1] = phi_i[2];
            v[R_V0 + 2] = phi_i[3];
#pragma unroll
            for (int k = 0; k < 6; k++) v[R_B + k] = B[k];
#pragma unroll
            for (int k = 0; k < 15; k++) v[R_G + k] = g[k];
            v[R_C] = c_i;
            double2* r2 = (double2*)rec;
#pragma unroll
            for (int k = 0; k < 16; k++) r2[k] = make_double2(v[2 * k], v[2 * k + 1]);
        } else {
            float* rec = (float*)recp + (long long)i * 32;
            float v[32];
            // slots 0-1: the pressure in FP64 (its two halves), for the pressure
            // difference across a face; slot 2 unused
            const long long pbits = __double_as_longlong(P_i);
            v[0] = __int_as_float((int)(pbits & 0xffffffffll));
            v[1] = __int_as_float((int)(pbits >> 32));
            v[2] = 0.0f;
            v[R_IH] = (float)iH;
            v[R_K] = (float)(Vi * Vi * norm);
            v[R_RHO] = (float)rho_i;
            v[R_P] = (float)P_i;
            v[R_V0 + 0] = (float)phi_i[1];
            v[R_V0 + 1] = (float)phi_i[2];
            v[R_V0 + 2] = (float)phi_i[3];
#pragma unroll
            for (int k = 0; k < 6; k++) v[R_B + k] = (float)B[k];
#pragma unroll
            for (int k = 0; k < 15; k++) v[R_G + k] = (float)g[k];
            v[R_C] = (float)c_i;
            float4* r4 = (float4*)rec;
#pragma unroll
            for (int k = 0; k < 8; k++) r4[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        }
    }
    count_add(&cnt->illcond, ill);
    count_add(&cnt->nonfinite, nonfin);
    count_max(&cnt->cond_bits, condbits);
}

// Hierarchical steps with active subsets: the records of the particles that
// keep their kernel length and gradients and take part in a due pair (a flux
// list), from their kept H, V, n, B and limited gradients (B and grad at
// column home[i]) with the current position and predicted state, as the
// gradient kernel writes them.
__global__ void k_pack_rec_kept(PassArrays a, Phys ph, const unsigned char* __restrict__ mode,
                                const long long* __restrict__ home, const int* __restrict__ counts,
                                double* __restrict__ recp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n || mode[i] == kModeSolve || counts[i] == 0) return;
    const long long n = a.n;
    const long long h = home[i];
    const double Hi = a.H[i], Vi = a.V[i];
    const double rho_i = a.m[i] * a.nk[i];
    const double P_i = (ph.gamma - 1.0) * rho_i * a.u[i];
    double v[32];
    v[0] = a.x[i];
    v[1] = a.y[i];
    v[2] = a.z[i];
    v[R_IH] = 1.0 / Hi;
    v[R_K] = Vi * Vi * kernel_norm(Hi);
    v[R_RHO] = rho_i;
    v[R_P] = P_i;
    v[R_V0 + 0] = a.vx[i];
    v[R_V0 + 1] = a.vy[i];
    v[R_V0 + 2] = a.vz[i];
#pragma unroll
    for (int k = 0; k < 6; k++) v[R_B + k] = a.B[k * n + h];
#pragma unroll
    for (int k = 0; k < 15; k++) v[R_G + k] = a.grad[k * n + h];
    v[R_C] = sqrt(ph.gamma * P_i / rho_i);
    double2* r2 = (double2*)(recp + (long long)i * 32);
#pragma unroll
    for (int k = 0; k < 16; k++) r2[k] = make_double2(v[2 * k], v[2 * k + 1]);
}

// ------------------------------------------------------------------- fluxes
template <typename T>
struct PairOut {
    T Fm;
    T Fp[3];
    T FE;
    int fallback, clamp;
};

template <typename T>
__device__ __forceinline__ T tsqrt(T v);
template <>
__device__ __forceinline__ double tsqrt<double>(double v) { return sqrt(v); }
template <>
__device__ __forceinline__ float tsqrt<float>(float v) { return sqrtf(v); }

// One unordered pair, left state a (lower index), right state b, d = x_b - x_a.
// products and sums rounded one by one (contraction into fma is switched off
// here): the face sum is then the same bits whichever owner evaluates it
template <typename T>
__device__ __forceinline__ T mul_rn(T x, T y) {
#pragma clang fp contract(off)
    return x * y;
}
template <typename T>
__device__ __forceinline__ T add_rn(T x, T y) {
#pragma clang fp contract(off)
    return x + y;
}

// One unordered pair in canonical order (the lower index is the left state),
// evaluated by the owner `m` of one side with the record `o` of the other; mL
// says whether m is the left side, d = x_R - x_L is the canonical displacement
// and r its length.  Every per-side quantity is written with one expression
// for that side (left: +1/2, right: -1/2 along d), and the sum of the two
// face halves is commutative and unfused, so both owners produce the same
// bits; only the reconstructed face states are put in left/right order.
// MFV (the finite-volume form): the full HLLC flux through the face, which
// moves with w.  Only the side that the star-state selection picks is built:
// K is the left side when S* >= 0 (or S_L >= 0), else the right side, and the
// star correction S_K (U*_K - U_K) is added unless that side's outer wave has
// already passed the face.  In the face frame (primes) the side state is
// rho, v' = v - w, E = P/(gamma-1) + rho |v'|^2/2, with physical flux
// (rho u, rho u v' + P n, (E + P) u), u = v'.n; its star state scales by
// f = rho (S_K - u)/(S_K - S*) and takes the normal speed S*.  The lab-frame
// flux adds w times the mass flux to the momentum flux and
// w.F_mom' + |w|^2/2 F_mass to the energy flux.
template <typename T>
__device__ __forceinline__ void mfv_flux(const T qL[5], const T qR[5], const T w[3], const T nh[3], T uL, T uR,
                                         T SL, T SR, T Ss, T gamma, T Amag, PairOut<T>& out) {
    const bool left = (SL >= T(0)) || (Ss >= T(0));
    const bool star = left ? !(SL >= T(0)) : (SR >= T(0));
    T q[5];
#pragma unroll
    for (int f = 0; f < 5; f++) q[f] = left ? qL[f] : qR[f];
    const T u = left ? uL : uR;
    const T S = left ? SL : SR;
    const T rho = q[0], P = q[4];
    const T vp[3] = {q[1] - w[0], q[2] - w[1], q[3] - w[2]};
    const T E = P / (gamma - T(1)) + T(0.5) * rho * (vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]);
    T F[5];
    F[0] = rho * u;
#pragma unroll
    for (int c = 0; c < 3; c++) F[1 + c] = rho * vp[c] * u + P * nh[c];
    F[4] = (E + P) * u;
    if (star) {
        const T f = rho * (S - u) / (S - Ss);
        const T du = Ss - u;
        if (sizeof(T) == 8) {
            F[0] += S * (f - rho);
#pragma unroll
            for (int c = 0; c < 3; c++) F[1 + c] += S * (f * (vp[c] + du * nh[c]) - rho * vp[c]);
            F[4] += S * (f * (E / rho + du * (Ss + P / (rho * (S - u)))) - E);
        } else {
            // FP32: the same flux in the form S* U*_K + P*_K (0, n, S*), with the
            // side's star pressure P*_K = P + rho (S - u)(S* - u).  F_K +
            // S_K (U*_K - U_K) equals it identically (the star state satisfies the
            // jump conditions across S_K), but subtracts terms much larger than a
            // slow face's mass flux; this form has no such cancellation.
            const T Pst = P + rho * (S - u) * du;
            F[0] = f * Ss;
#pragma unroll
            for (int c = 0; c < 3; c++) F[1 + c] = f * (vp[c] + du * nh[c]) * Ss + Pst * nh[c];
            F[4] = (f * (E / rho + du * (Ss + P / (rho * (S - u)))) + Pst) * Ss;
        }
    }
    const T ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    out.Fm = F[0] * Amag;
#pragma unroll
    for (int c = 0; c < 3; c++) out.Fp[c] = (F[1 + c] + w[c] * F[0]) * Amag;
    out.FE = (F[4] + w[0] * F[1] + w[1] * F[2] + w[2] * F[3] + T(0.5) * ww * F[0]) * Amag;
}

// The optional pairwise limiter (R23) on one side's face value f, with pk that
// side's centre value and po the other's: on the other particle's side at most
// D/4 past the midpoint interpolant, on its own side at most D/2 outside the
// centre range [lo, hi] (D = hi - lo); a widened bound that would not keep the
// sign is lo / (1 + D / (2|lo|)) (hi likewise), taken here as
// lo |lo| / (|lo| + D/2).  That bound only matters where the value passes it,
// which v (|lo| + D/2) against lo |lo| decides without dividing, so the
// division runs only when a lane of the wave clamps there.  Each owner
// evaluates it with the same arguments for the same side, so both copies of a
// pair agree bit for bit.
__device__ __forceinline__ double lim_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float lim_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double lim_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float lim_max(float a, float b) { return fmaxf(a, b); }

// In t = s f, with s = +1 where the side's own value is the lower of the two
// and -1 where it is the higher, both cases read as the first one: t at most
// s mid + D/4 and at least s pk - D/2 (the sign flips are exact), so the bound
// is two min/max instructions.
// The same bound in the direct form, for the FP32 records (where the
// sign-flipped form measured slower: 18.0 against 22.1 ms on the clustered set).
template <typename T>
__device__ __forceinline__ T pair_limit_direct(T f, T pk, T po) {
    if (pk == po) return pk;
    const bool below = pk < po;   // the side's own value is the lower one
    const T lo = below ? pk : po, hi = below ? po : pk;
    const T D = hi - lo;
    const T mid = T(0.5) * (pk + po);
    const T e = below ? lo : hi;
    const T wide = below ? lo - T(0.5) * D : hi + T(0.5) * D;
    const T inner = below ? mid + T(0.25) * D : mid - T(0.25) * D;
    T v = below ? (f < inner ? f : inner) : (f > inner ? f : inner);
    if (wide * e > T(0)) return below ? (v > wide ? v : wide) : (v < wide ? v : wide);
    const T ae = e < T(0) ? -e : e;
    const T den = ae + T(0.5) * D, num = e * ae;
    const bool clamp = below ? v * den < num : v * den > num;
    if (__ballot(clamp)) {
        if (clamp) v = num / den;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T pair_limit(T f, T pk, T po) {
    if constexpr (sizeof(T) == 4) return pair_limit_direct(f, pk, po);
    const T s = pk < po ? T(1) : T(-1);
    const T D = pk < po ? po - pk : pk - po;
    const T spk = s * pk;
    const T t = lim_min(s * f, s * (T(0.5) * (pk + po)) + T(0.25) * D);
    const T wide = spk - T(0.5) * D;
    const bool keep = wide * spk > T(0);
    T r = keep ? lim_max(t, wide) : t;
    // the sign-keeping bound s b = spk |pk| / (|pk| + D/2): clamp where t is below it
    const T apk = pk < T(0) ? -pk : pk;
    const T den = apk + T(0.5) * D, num = spk * apk;
    const bool clamp = !keep && t * den < num;
    if (__ballot(clamp)) {
        if (clamp) r = num / den;
    }
    return pk == po ? pk : s * r;
}

template <typename T, bool MFV, bool LIM>
__device__ __forceinline__ PairOut<T> pair_flux(const T* __restrict__ m, const T* __restrict__ o, bool mL,
                                                const T d[3], T r, T gamma) {
    PairOut<T> out;
    out.Fm = out.Fp[0] = out.Fp[1] = out.Fp[2] = out.FE = T(0);
    out.fallback = out.clamp = 0;
    // face A = V_m^2 W_m B_m d + V_o^2 W_o B_o d (the kernel factor K = V^2 8/(pi H^3))
    const T km = m[R_K] * spline_w(r * m[R_IH]);
    const T ko = o[R_K] * spline_w(r * o[R_IH]);
    const T* Bm = m + R_B;
    const T* Bo = o + R_B;
    const T tm[3] = {Bm[0] * d[0] + Bm[1] * d[1] + Bm[2] * d[2], Bm[1] * d[0] + Bm[3] * d[1] + Bm[4] * d[2],
                     Bm[2] * d[0] + Bm[4] * d[1] + Bm[5] * d[2]};
    const T to[3] = {Bo[0] * d[0] + Bo[1] * d[1] + Bo[2] * d[2], Bo[1] * d[0] + Bo[3] * d[1] + Bo[4] * d[2],
                     Bo[2] * d[0] + Bo[4] * d[1] + Bo[5] * d[2]};
    T A[3];
#pragma unroll
    for (int c = 0; c < 3; c++) A[c] = add_rn(mul_rn(km, tm[c]), mul_rn(ko, to[c]));
    const T Amag = tsqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    if (!(Amag > T(0))) return out;
    const T iA = T(1) / Amag;
    const T nh[3] = {A[0] * iA, A[1] * iA, A[2] * iA};

    // midpoint reconstruction of rho, vx, vy, vz, P on each side
    const int slot[5] = {R_RHO, R_V0, R_V0 + 1, R_V0 + 2, R_P};
    const T sm = mL ? T(0.5) : T(-0.5);
    T qL[5], qR[5];
#pragma unroll
    for (int f = 0; f < 5; f++) {
        const T* gm = m + R_G + 3 * f;
        const T* go = o + R_G + 3 * f;
        T qm = m[slot[f]] + sm * (gm[0] * d[0] + gm[1] * d[1] + gm[2] * d[2]);
        T qo = o[slot[f]] + (-sm) * (go[0] * d[0] + go[1] * d[1] + go[2] * d[2]);
        if (LIM) {
            qm = pair_limit<T>(qm, m[slot[f]], o[slot[f]]);
            qo = pair_limit<T>(qo, o[slot[f]], m[slot[f]]);
        }
        qL[f] = mL ? qm : qo;
        qR[f] = mL ? qo : qm;
    }
    const bool first = !(qL[0] > T(0)) || !(qL[4] > T(0)) || !(qR[0] > T(0)) || !(qR[4] > T(0));
    if (first) {
#pragma unroll
        for (int f = 0; f < 5; f++) {
            qL[f] = mL ? m[slot[f]] : o[slot[f]];
            qR[f] = mL ? o[slot[f]] : m[slot[f]];
        }
        out.fallback = 1;
    }
    // pressure difference across the face, P_R - P_L.  With FP32 records the
    // centre pressures' difference is taken in FP64 first (each record carries
    // its pressure in FP64): in dense, slow gas that difference is a small part
    // of P, and rounding each face pressure to FP32 would swamp it (and with it
    // the contact speed S*); the FP32 reconstruction offsets are added after.
    T dPRL;
    if constexpr (sizeof(T) == 8) {
        dPRL = qR[4] - qL[4];
    } else {
        const double Pm = __longlong_as_double(((long long)__float_as_int(m[1]) << 32) |
                                               (unsigned)__float_as_int(m[0]));
        const double Po = __longlong_as_double(((long long)__float_as_int(o[1]) << 32) |
                                               (unsigned)__float_as_int(o[0]));
        const double dc = mL ? Po - Pm : Pm - Po;
        // the offsets as the reconstruction formed them: (face - centre) per side
        const T offL = first ? T(0) : qL[4] - (mL ? m[R_P] : o[R_P]);
        const T offR = first ? T(0) : qR[4] - (mL ? o[R_P] : m[R_P]);
        dPRL = (T)dc + (offR - offL);
    }
    // face frame: the mean of the two particle velocities (commutative)
    const T w[3] = {T(0.5) * (m[R_V0] + o[R_V0]), T(0.5) * (m[R_V0 + 1] + o[R_V0 + 1]),
                    T(0.5) * (m[R_V0 + 2] + o[R_V0 + 2])};
    const T uL = (qL[1] - w[0]) * nh[0] + (qL[2] - w[1]) * nh[1] + (qL[3] - w[2]) * nh[2];
    const T uR = (qR[1] - w[0]) * nh[0] + (qR[2] - w[1]) * nh[1] + (qR[3] - w[2]) * nh[2];
    const T rL = qL[0], pL = qL[4], rR = qR[0], pR = qR[4];
    const T cL = tsqrt(gamma * pL / rL), cR = tsqrt(gamma * pR / rR);
    const T SL = (uL - cL < uR - cR) ? uL - cL : uR - cR;
    const T SR = (uL + cL > uR + cR) ? uL + cL : uR + cR;
    const T mLf = rL * (SL - uL), mRf = rR * (SR - uR);
    const T Ss = (dPRL + mLf * uL - mRf * uR) / (mLf - mRf);
    if (MFV) {
        mfv_flux<T>(qL, qR, w, nh, uL, uR, SL, SR, Ss, gamma, Amag, out);
        return out;
    }
    T Ps = T(0.5) * (pL + pR + mLf * (Ss - uL) + mRf * (Ss - uR));
    if (Ps < T(0)) {
        Ps = T(0);
        out.clamp = 1;
    }
    const T wn = w[0] * nh[0] + w[1] * nh[1] + w[2] * nh[2];
#pragma unroll
    for (int c = 0; c < 3; c++) out.Fp[c] = Ps * A[c];
    out.FE = Ps * (Ss + wn) * Amag;
    return out;
}

template <typename T>
__device__ __forceinline__ void load_rec(const T* __restrict__ rec, long long i, T v[32]);
template <>
__device__ __forceinline__ void load_rec<double>(const double* __restrict__ rec, long long i, double v[32]) {
    const double2* p = (const double2*)(rec + i * 32);
#pragma unroll
    for (int k = 0; k < 16; k++) {
        double2 t = p[k];
        v[2 * k] = t.x;
        v[2 * k + 1] = t.y;
    }
}
template <>
__device__ __forceinline__ void load_rec<float>(const float* __restrict__ rec, long long i, float v[32]) {
    const float4* p = (const float4*)(rec + i * 32);
#pragma unroll
    for (int k = 0; k < 8; k++) {
        float4 t = p[k];
        v[4 * k] = t.x;
        v[4 * k + 1] = t.y;
        v[4 * k + 2] = t.z;
        v[4 * k + 3] = t.w;
    }
}

// Hierarchical steps (the levelled pass): a pair {i, j} has level max(bin_i,
// bin_j); only pairs of level >= lmin are evaluated, and each particle's sums
// per level go to lev[(l * 4 + c) * n + i] (c: dp x, y, z, dE) for the levels
// >= lmin, the others keeping their values.  The sums of levels bin_i ..
// bin_i + kLevWin - 1 (a particle's pairs are never coarser than its own bin)
// are kept in registers; finer levels are summed in place in lev.
constexpr int kLevWin = 4;
struct Levels {
    const long long* bin;
    int lmin, nlev;
    double* lev;
    const long long* home;   // column of lev per particle (null: the particle's index)
};

template <typename T, bool MFV, bool LIM, bool LEV = false>
__device__ __forceinline__ void fluxes_body(const PassArrays& a, const Phys& ph, const int* __restrict__ counts,
                                            const int* __restrict__ list, const T* __restrict__ rec,
                                            Counters* cnt, Levels lv = Levels{nullptr, 0, 0, nullptr, nullptr}) {
    cnt = counter_copy(cnt);
    const int i = xcd_block() * 256 + threadIdx.x;
    const bool act = i < a.n;
    unsigned long long nfall = 0, nclamp = 0, nonfin = 0;
    if (act) {
        const long long n = a.n;
        T ri[32];
        // in the levelled pass most particles of a partial boundary have no
        // list: their record is not read (its values only enter pairs)
        if (LEV && counts[i] == 0) {
#pragma unroll
            for (int q = 0; q < 32; q++) ri[q] = T(0);
        } else {
            load_rec<T>(rec, i, ri);
        }
        const double xi[3] = {a.x[i], a.y[i], a.z[i]};
        const double vi[3] = {(double)ri[R_V0], (double)ri[R_V0 + 1], (double)ri[R_V0 + 2]};
        const double ci = (double)ri[R_C];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        double accm = 0.0;
        double vs = 0.0;
        const T gam = (T)ph.gamma;
        const int cnum = counts[i];
        int bi = 0;
        long long li = i;
        double lacc[kLevWin][4];
        if (LEV) {
            bi = (int)lv.bin[i];
            if (lv.home) li = lv.home[i];
#pragma unroll
            for (int w = 0; w < kLevWin; w++)
#pragma unroll
                for (int c = 0; c < 4; c++) lacc[w][c] = 0.0;
            for (int l = max(lv.lmin, bi + kLevWin); l < lv.nlev; l++)
                for (int c = 0; c < 4; c++) lv.lev[((long long)l * 4 + c) * n + li] = 0.0;
        }
        // the next list entry is loaded one pair ahead, so the record loads of
        // a pair do not wait for its index
        int jn = cnum > 0 ? list[i] : 0;
        for (int k = 0; k < cnum; k++) {
            const int j = jn;
            if (k + 1 < cnum) jn = list[(long long)(k + 1) * n + i];
            int lj = 0;
            if (LEV) {
                // a pair that is not due costs its bin alone: no record, no flux,
                // no signal speed (the last boundary of a system step has every
                // pair due, so the signal speeds it leaves are complete); with
                // every level due the record load does not wait for the bin
                lj = max(bi, (int)lv.bin[j]);
                if (lv.lmin > 0 && lj < lv.lmin) continue;
            }
            T rj[32];
            load_rec<T>(rec, j, rj);
            double xj[3];
            if (sizeof(T) == 8) {
                xj[0] = (double)rj[0];
                xj[1] = (double)rj[1];
                xj[2] = (double)rj[2];
            } else {
                xj[0] = a.x[j];
                xj[1] = a.y[j];
                xj[2] = a.z[j];
            }
            double dij[3];
            displacement(ph, xi, xj[0], xj[1], xj[2], dij);   // x_j - x_i
            const double r = sqrt(dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2]);
            const bool iL = i < j;
            // signal speed over the flux neighbours (the due ones in the levelled pass)
            auto signal = [&]() {
                const double cj = (double)rj[R_C];
                const double proj = -((vi[0] - (double)rj[R_V0]) * dij[0] + (vi[1] - (double)rj[R_V0 + 1]) * dij[1] +
                                      (vi[2] - (double)rj[R_V0 + 2]) * dij[2]) / r;
                vs = fmax(vs, ci + cj - fmin(proj, 0.0));
            };
            // canonical displacement x_R - x_L: the minimum image commutes with
            // negation exactly, so both owners of the pair hold the same bits
            const double sg = iL ? 1.0 : -1.0;
            const T dT[3] = {(T)(sg * dij[0]), (T)(sg * dij[1]), (T)(sg * dij[2])};
            PairOut<T> o = pair_flux<T, MFV, LIM>(ri, rj, iL, dT, (T)r, gam);
            const double s = iL ? 1.0 : -1.0;
            if (MFV) accm -= s * (double)o.Fm;
            acc[0] -= s * (double)o.Fp[0];
            acc[1] -= s * (double)o.Fp[1];
            acc[2] -= s * (double)o.Fp[2];
            acc[3] -= s * (double)o.FE;
            nfall += o.fallback;
            nclamp += o.clamp;
            signal();
            if (LEV) {
                const double F[4] = {(double)o.Fp[0], (double)o.Fp[1], (double)o.Fp[2], (double)o.FE};
                const int w = lj - bi;
                if (w == 0) {   // both particles in one bin: most pairs
#pragma unroll
                    for (int c = 0; c < 4; c++) lacc[0][c] = lacc[0][c] - s * F[c];
                } else if (w < kLevWin) {
#pragma unroll
                    for (int q = 1; q < kLevWin; q++)
#pragma unroll
                        for (int c = 0; c < 4; c++) lacc[q][c] = (q == w) ? lacc[q][c] - s * F[c] : lacc[q][c];
                } else {
                    for (int c = 0; c < 4; c++) lv.lev[((long long)lj * 4 + c) * n + li] -= s * F[c];
                }
            }
        }
        if (LEV) {
#pragma unroll
            for (int w = 0; w < kLevWin; w++) {
                const int l = bi + w;
                if (l >= lv.lmin && l < lv.nlev)
#pragma unroll
                    for (int c = 0; c < 4; c++) lv.lev[((long long)l * 4 + c) * n + li] = lacc[w][c];
            }
            // due levels coarser than the particle's own bin hold no pair of it
            for (int l = lv.lmin; l < min(bi, lv.nlev); l++)
                for (int c = 0; c < 4; c++) lv.lev[((long long)l * 4 + c) * n + li] = 0.0;
        }
        a.dp[i] = acc[0];
        a.dp[n + i] = acc[1];
        a.dp[2 * n + i] = acc[2];
        a.dE[i] = acc[3];
        a.vsig[i] = vs;
        if (MFV) a.dm[i] = accm;
        if (!isfinite(acc[0]) || !isfinite(acc[1]) || !isfinite(acc[2]) || !isfinite(acc[3]) || !isfinite(accm)) {
            nonfin = 1;
            flag_index(cnt, i);
        }
    }
    count_add(&cnt->fallbacks, nfall);
    count_add(&cnt->clamps, nclamp);
    count_add(&cnt->nonfinite, nonfin);
}

// One kernel per record precision: each pair holds both records in registers.
// The FP32 form runs at four waves per SIMD.  The FP64 form runs at two: with
// the list index loaded a pair ahead, a third wave (a few spilled loop
// invariants, and twice the HBM traffic as more records compete for L2) no
// longer pays.
constexpr int kFlux64Waves = 2;
constexpr int kFluxMfvWaves = kFlux64Waves;
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFlux64Waves))) void k_fluxes_f64(PassArrays a, Phys ph, const int* __restrict__ counts,
                                                    const int* __restrict__ list, const double* __restrict__ rec,
                                                    Counters* cnt) {
    fluxes_body<double, false, LIM>(a, ph, counts, list, rec, cnt);
}

// The levelled pass of hierarchical steps (MFM, FP64 records).
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFlux64Waves))) void k_fluxes_levels(
    PassArrays a, Phys ph, const int* __restrict__ counts, const int* __restrict__ list,
    const double* __restrict__ rec, Counters* cnt, Levels lv) {
    fluxes_body<double, false, LIM, true>(a, ph, counts, list, rec, cnt, lv);
}

// The finite-volume form, FP64 records only, at two waves per SIMD like the
// FP64 form (at three its extra live values spill).
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFluxMfvWaves))) void k_fluxes_mfv(PassArrays a, Phys ph, const int* __restrict__ counts,
                                                    const int* __restrict__ list, const double* __restrict__ rec,
                                                    Counters* cnt) {
    fluxes_body<double, true, LIM>(a, ph, counts, list, rec, cnt);
}

constexpr int kFlux32Waves = 4;
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFlux32Waves)))
void k_fluxes_f32(PassArrays a, Phys ph, const int* __restrict__ counts, const int* __restrict__ list,
                  const float* __restrict__ rec, Counters* cnt) {
    fluxes_body<float, false, LIM>(a, ph, counts, list, rec, cnt);
}

// The finite-volume form on the FP32 records of the mixed form.
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFlux32Waves)))
void k_fluxes_mfv_f32(PassArrays a, Phys ph, const int* __restrict__ counts, const int* __restrict__ list,
                      const float* __restrict__ rec, Counters* cnt) {
    fluxes_body<float, true, LIM>(a, ph, counts, list, rec, cnt);
}

// ------------------------------------------------------------------ launchers
static int blocks_of(int n, int b) { return (n + b - 1) / b; }
constexpr int kFallbackWaves = 1024;

void launch_solve_h(const PassArrays& a, const TreeDesc& td, const int2* tab,
                    const double4* pos, const Phys& ph, Counters* cnt, double* rl, int* list, int* gcount,
                    int* counts, int* fb_list, unsigned long long* fb_count, int* fb2_list,
                    unsigned long long* fb2_count, hipEvent_t t0, hipEvent_t t1, hipStream_t s) {
    launch_fill_u64(1, fb_count, 0ull, s);
    launch_fill_u64(1, fb2_count, 0ull, s);
    if (t0) hipEventRecord(t0, s);
    k_solve_h<false><<<blocks_of(a.n, 256), 256, 0, s>>>(a, td, tab, pos, ph, cnt, rl, list, gcount, counts,
                                                         fb_list, fb_count, nullptr, nullptr);
    // one wave per handed-over particle, striding over the count left on the device
    k_solve_h_wave<<<kWaveBlocks, 64, 0, s>>>(a, td, tab, pos, ph, cnt, fb_list, fb_count, rl, list, gcount,
                                              counts, fb2_list, fb2_count, nullptr);
    k_solve_h_fallback<<<kFallbackWaves, 64, 0, s>>>(a, td, tab, pos, ph, cnt, fb2_list, fb2_count, list, gcount,
                                                     counts, nullptr);
    if (t1) hipEventRecord(t1, s);
}

void launch_gradients(const PassArrays& a, const Phys& ph, const int* gcount, int* counts, int* list, int* tails,
                      int mixed, double4* prim, void* rec, Counters* cnt, hipEvent_t t0, hipEvent_t t1,
                      hipStream_t s) {
    k_pack_prim<<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, gcount, nullptr, prim);
    if (t0) hipEventRecord(t0, s);
    if (mixed)
        k_gradients<true, false><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, gcount, counts, list, tails, prim, rec,
                                                                     cnt, nullptr, nullptr);
    else
        k_gradients<false, false><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, gcount, counts, list, tails, prim, rec,
                                                                      cnt, nullptr, nullptr);
    if (t1) hipEventRecord(t1, s);
    k_sort_tails<<<blocks_of(a.n, 256), 256, 0, s>>>(a.n, ph.max_ngb, gcount, counts, list, tails, cnt);
}

void launch_solve_h_active(const PassArrays& a, const TreeDesc& td, const int2* tab, const double4* pos,
                           const Phys& ph, Counters* cnt, const unsigned char* mode, const double* pad, double* rl,
                           int* list, int* gcount, int* counts, int* fb_list, unsigned long long* fb_count,
                           int* fb2_list, unsigned long long* fb2_count, hipStream_t s) {
    launch_fill_u64(1, fb_count, 0ull, s);
    launch_fill_u64(1, fb2_count, 0ull, s);
    k_solve_h<true><<<blocks_of(a.n, 256), 256, 0, s>>>(a, td, tab, pos, ph, cnt, rl, list, gcount, counts,
                                                        fb_list, fb_count, mode, pad);
    k_solve_h_wave<<<kWaveBlocks, 64, 0, s>>>(a, td, tab, pos, ph, cnt, fb_list, fb_count, rl, list, gcount,
                                              counts, fb2_list, fb2_count, pad);
    k_solve_h_fallback<<<kFallbackWaves, 64, 0, s>>>(a, td, tab, pos, ph, cnt, fb2_list, fb2_count, list, gcount,
                                                     counts, pad);
    k_gather_kept<<<blocks_of(a.n, 256), 256, 0, s>>>(a, td, tab, pos, ph, mode, pad, list, gcount, counts);
}

void launch_gradients_active(const PassArrays& a, const Phys& ph, const unsigned char* mode, const long long* home,
                             const int* gcount, int* counts, int* list, int* tails, double4* prim, void* rec,
                             Counters* cnt, hipStream_t s) {
    k_pack_prim_active<<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, gcount, mode, list, prim);
    k_gradients<false, true><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, gcount, counts, list, tails, prim, rec, cnt,
                                                                 mode, home);
    k_pack_rec_kept<<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, mode, home, counts, (double*)rec);
    k_sort_tails<<<blocks_of(a.n, 256), 256, 0, s>>>(a.n, ph.max_ngb, gcount, counts, list, tails, cnt);
}

template <bool LIM>
static void launch_fluxes_lim(const PassArrays& a, const Phys& ph, const int* counts, const int* list, int mixed,
                              int mfv, const void* rec, Counters* cnt, hipStream_t s) {
    if (mfv && mixed)
        k_fluxes_mfv_f32<LIM><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const float*)rec, cnt);
    else if (mfv)
        k_fluxes_mfv<LIM><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const double*)rec, cnt);
    else if (mixed)
        k_fluxes_f32<LIM><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const float*)rec, cnt);
    else
        k_fluxes_f64<LIM><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const double*)rec, cnt);
}

void launch_fluxes_levels(const PassArrays& a, const Phys& ph, const int* counts, const int* list, const void* rec,
                          Counters* cnt, const long long* bin, int lmin, int nlev, double* lev,
                          const long long* home, hipStream_t s) {
    const Levels lv{bin, lmin, nlev, lev, home};
    if (ph.limiter)
        k_fluxes_levels<true><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const double*)rec, cnt, lv);
    else
        k_fluxes_levels<false><<<blocks_of(a.n, 256), 256, 0, s>>>(a, ph, counts, list, (const double*)rec, cnt, lv);
}

void launch_fluxes(const PassArrays& a, const Phys& ph, const int* counts, const int* list, int mixed, int mfv,
                   const void* rec, Counters* cnt, hipStream_t s) {
    if (ph.limiter)
        launch_fluxes_lim<true>(a, ph, counts, list, mixed, mfv, rec, cnt, s);
    else
        launch_fluxes_lim<false>(a, ph, counts, list, mixed, mfv, rec, cnt, s);
}

}  // namespace mfm

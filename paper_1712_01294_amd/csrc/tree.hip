// Neighbour structure for the gfx950 MFM pass.
//
// Particles are ordered along a per-axis Morton curve and every level of the
// implicit octree is a table of sorted ranges, so a cell at any depth is one
// contiguous run of particles.  The build is: quantise positions -> keys,
// stable LSD radix sort (8-bit digits, wave-ballot ranking), reorder the
// particle arrays in place, fill (start, end) per occupied cell per level.
#include <stddef.h>

#include "device.h"
#include "kernels.h"

namespace mfm {

// ----------------------------------------------------------------- keys
__global__ void k_keys(int n, const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, TreeDesc td, unsigned long long* __restrict__ keys,
                       int* __restrict__ idx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* xs[3] = {x, y, z};
    unsigned q[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        double s = (double)(1u << td.qbits[d]) / td.box[d];
        double f = floor(xs[d][i] * s);
        long long v = (long long)f;
        long long top = (1ll << td.qbits[d]) - 1;
        if (!(f >= 0.0)) v = 0;  // also catches NaN
        if (v > top) v = top;
        q[d] = (unsigned)v;
    }
    unsigned long long key = 0;
    for (int l = 1; l <= td.bmax; l++) {
        int m = td.actmask[l];
#pragma unroll
        for (int d = 0; d < 3; d++)
            if (m & (1 << d)) key = (key << 1) | ((q[d] >> (td.bmax - l)) & 1u);
    }
    keys[i] = key;
    idx[i] = i;
}

// ---------------------------------------------------------- radix sort
// Tile = 4 waves x kRounds rounds x 64 lanes; element e of a tile belongs to
// wave e / (64 kRounds), round (e / 64) % kRounds, lane e % 64, so processing
// rounds in order inside each wave and waves in order inside the tile keeps
// the sort stable.
constexpr int kSortWaves = 4;
constexpr int kRounds = 8;
constexpr int kTile = kSortWaves * kRounds * 64;

__global__ __launch_bounds__(256) void k_radix_hist(int n, const unsigned long long* __restrict__ keys,
                                                     int shift, int nblocks, int* __restrict__ hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kTile;
    for (int t = threadIdx.x; t < kTile; t += 256) {
        int e = base + t;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(int n, const unsigned long long* __restrict__ kin,
                                                        const int* __restrict__ vin, int shift, int nblocks,
                                                        const int* __restrict__ offs,
                                                        unsigned long long* __restrict__ kout,
                                                        int* __restrict__ vout) {
    __shared__ int wc[kSortWaves][256];
    __shared__ int goff[256];
    int lane = threadIdx.x & 63;
    int w = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < kSortWaves * 256; t += 256) (&wc[0][0])[t] = 0;
    goff[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long kk[kRounds];
    int vv[kRounds], dg[kRounds], pos[kRounds];
    int base = blockIdx.x * kTile + w * (kRounds * 64);
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        int e = base + r * 64 + lane;
        bool valid = e < n;
        unsigned long long key = valid ? kin[e] : 0ull;
        int digit = (int)((key >> shift) & 255);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            unsigned long long bal = __ballot(valid && ((digit >> b) & 1));
            peers &= ((digit >> b) & 1) ? bal : ~bal;
        }
        int prior = valid ? wc[w][digit] : 0;
        __builtin_amdgcn_wave_barrier();
        int rank = __popcll(peers & lt);
        bool leader = valid && ((peers >> lane) >> 1) == 0;  // highest lane of its digit
        if (leader) wc[w][digit] = prior + rank + 1;
        __builtin_amdgcn_wave_barrier();
        kk[r] = key;
        vv[r] = valid ? vin[e] : 0;
        dg[r] = valid ? digit : -1;
        pos[r] = prior + rank;
    }
    __syncthreads();
    {
        int run = 0;
        for (int ww = 0; ww < kSortWaves; ww++) {
            int t = wc[ww][threadIdx.x];
            wc[ww][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRounds; r++) {
        if (dg[r] >= 0) {
            int o = goff[dg[r]] + wc[w][dg[r]] + pos[r];
            if (o >= 0 && o < n) {   // always true for a correct ranking; keeps a bug in bounds
                kout[o] = kk[r];
                vout[o] = vv[r];
            }
        }
    }
}

// ------------------------------------------------------- exclusive scan
constexpr int kScanItems = 4;
constexpr int kScanTile = 256 * kScanItems;

__global__ __launch_bounds__(256) void k_scan_tiles(int m, const int* __restrict__ in,
                                                     int* __restrict__ out, int* __restrict__ sums) {
    __shared__ int ws[4];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        tsum += v[k];
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = tsum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int wpre = 0;
    for (int k = 0; k < w; k++) wpre += ws[k];
    int run = wpre + inc - tsum;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) sums[blockIdx.x] = wpre + inc;
}

__global__ void k_scan_add(int m, int* __restrict__ out, const int* __restrict__ sums) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] += sums[i / kScanTile];
}

// exclusive scan of m ints; tmp must hold scan_tmp_ints(m) ints
long long scan_tmp_ints(long long m) {
    long long t = 0;
    while (m > 1) {
        m = (m + kScanTile - 1) / kScanTile;
        t += m;
    }
    return t + 1;
}

void exclusive_scan(int m, const int* in, int* out, int* tmp, hipStream_t s) {
    int nb = (m + kScanTile - 1) / kScanTile;
    int* sums = tmp;
    k_scan_tiles<<<nb, 256, 0, s>>>(m, in, out, sums);
    if (nb > 1) {
        exclusive_scan(nb, sums, sums, tmp + nb, s);
        k_scan_add<<<(m + 255) / 256, 256, 0, s>>>(m, out, sums);
    }
}

void radix_sort(int n, int bits, unsigned long long* keys, int* vals, unsigned long long* ktmp,
                int* vtmp, int* hist, int* scan_tmp, hipStream_t s) {
    int nblocks = (n + kTile - 1) / kTile;
    unsigned long long *ka = keys, *kb = ktmp;
    int *va = vals, *vb = vtmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        k_radix_hist<<<nblocks, 256, 0, s>>>(n, ka, shift, nblocks, hist);
        exclusive_scan(256 * nblocks, hist, hist, scan_tmp, s);
        k_radix_scatter<<<nblocks, 256, 0, s>>>(n, ka, va, shift, nblocks, hist, kb, vb);
        unsigned long long* t = ka;
        ka = kb;
        kb = t;
        int* tv = va;
        va = vb;
        vb = tv;
    }
    if (passes & 1) {
        hipMemcpyAsync(keys, ka, sizeof(unsigned long long) * n, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, va, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    }
}

// --------------------------------------------------- reorder in place
__global__ void k_gather_batch(int n, GatherBatch gb, const int* __restrict__ idx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int src = idx[i];
    if (src < 0 || src >= n) return;   // only reachable if the sort were wrong
    for (int a = 0; a < gb.count; a++) gb.dst[a][i] = gb.src[a][src];
}

__global__ void k_fill_u64(long long m, unsigned long long* __restrict__ p, unsigned long long v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < m; i += stride) p[i] = v;
}

// every counter word zero except first_bad of each copy, which starts at "none"
__global__ void k_reset_counters(unsigned long long* __restrict__ p) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int per = kCounterStride / 8;
    if (w >= kCounterCopies * per) return;
    p[w] = (w % per) == (int)(offsetof(Counters, first_bad) / 8) ? ~0ull : 0ull;
}

// dst[a][k] = src[a][k] for every array of the batch (8-byte elements)
__global__ void k_copy_batch(int n, GatherBatch gb) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    for (int a = 0; a < gb.count; a++) gb.dst[a][k] = gb.src[a][k];
}

// ----------------------------------------------------------- cell tables
__global__ void k_tables(int n, const unsigned long long* __restrict__ keys, TreeDesc td,
                         int2* __restrict__ tab) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    unsigned long long key = keys[k];
    if (key >> td.ktot) return;   // keys carry exactly ktot bits
    unsigned long long prev = k > 0 ? keys[k - 1] : 0;
    unsigned long long next = k + 1 < n ? keys[k + 1] : 0;
    for (int l = 0; l <= td.bmax; l++) {
        int sh = td.ktot - td.kbits[l];
        unsigned long long c = key >> sh;
        int* e = (int*)(tab + td.tab_off[l] + (long long)c);
        if (k == 0 || (prev >> sh) != c) e[0] = k;
        if (k == n - 1 || (next >> sh) != c) e[1] = k + 1;
    }
}

// Undo k_tables for the same sorted keys: the first particle of each cell
// clears that cell's entry on every level, so a build clears only the entries
// the last one wrote instead of the whole table.
__global__ void k_untables(int n, const unsigned long long* __restrict__ keys, TreeDesc td,
                           int2* __restrict__ tab) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    unsigned long long key = keys[k];
    if (key >> td.ktot) return;   // k_tables wrote nothing for it
    unsigned long long prev = k > 0 ? keys[k - 1] : 0;
    for (int l = 0; l <= td.bmax; l++) {
        int sh = td.ktot - td.kbits[l];
        unsigned long long c = key >> sh;
        if (k == 0 || (prev >> sh) != c) tab[td.tab_off[l] + (long long)c] = make_int2(0, 0);
    }
}

// positions packed per particle for the neighbour scans (one 32-byte load)
__global__ void k_pos4(int n, const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, double4* __restrict__ pos) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[i] = make_double4(x[i], y[i], z[i], 0.0);
}

void launch_keys(int n, const double* x, const double* y, const double* z, const TreeDesc& td,
                 unsigned long long* keys, int* idx, hipStream_t s) {
    k_keys<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, z, td, keys, idx);
}

void launch_gather(int n, const GatherBatch& gb, const int* idx, hipStream_t s) {
    k_gather_batch<<<(n + 255) / 256, 256, 0, s>>>(n, gb, idx);
}

void launch_reset_counters(Counters* c, hipStream_t s) {
    constexpr int words = kCounterCopies * kCounterStride / 8;
    k_reset_counters<<<(words + 255) / 256, 256, 0, s>>>((unsigned long long*)c);
}

void launch_copy_batch(int n, const GatherBatch& gb, hipStream_t s) {
    if (n <= 0 || gb.count <= 0) return;
    k_copy_batch<<<(n + 255) / 256, 256, 0, s>>>(n, gb);
}

void launch_fill_u64(long long m, unsigned long long* p, unsigned long long v, hipStream_t s) {
    if (m <= 0) return;
    long long blocks = (m + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_fill_u64<<<(int)blocks, 256, 0, s>>>(m, p, v);
}

void launch_tables(int n, const unsigned long long* keys, const TreeDesc& td, int2* tab, hipStream_t s) {
    k_tables<<<(n + 255) / 256, 256, 0, s>>>(n, keys, td, tab);
}

void launch_untables(int n, const unsigned long long* keys, const TreeDesc& td, int2* tab, hipStream_t s) {
    k_untables<<<(n + 255) / 256, 256, 0, s>>>(n, keys, td, tab);
}

void launch_pos4(int n, const double* x, const double* y, const double* z, double4* pos, hipStream_t s) {
    k_pos4<<<(n + 255) / 256, 256, 0, s>>>(n, x, y, z, pos);
}

}  // namespace mfm

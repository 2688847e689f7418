// C ABI of the gfx950 MFM hydro pass (declared in include/mfm.h).
#include <math.h>
#include <algorithm>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/mfm.h"
#include "device.h"
#include "kernels.h"
#include "order.h"

using namespace mfm;

// Optional per-kernel timing: HIP event pairs recorded around each launch of a
// pass kernel on the caller's stream, summed when the caller asks for them.
struct KernelClock {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, spare;
    double total_ms = 0.0;
    long long launches = 0;
};

struct mfm_ctx {
    mfm_params p;
    int64_t cap = 0;
    int device = 0;
    TreeDesc td;
    Phys ph;
    long long tab_len = 0;
    // tab holds exactly the cells of the first tab_keys_n sorted keys in
    // keys (-1: not known, so the next build clears the whole table)
    long long tab_keys_n = -1;
    unsigned long long *keys = nullptr, *ktmp = nullptr;
    int *idx = nullptr, *vtmp = nullptr, *hist = nullptr, *scan_tmp = nullptr;
    unsigned long long* gtmp = nullptr;   // kGatherMax x cap staging for in-place reordering
    int2* tab = nullptr;
    double4* pos = nullptr;               // packed positions of the current order
    double* rl = nullptr;                 // radii scratch of the kernel-length solve
    int *counts = nullptr, *gcount = nullptr, *list = nullptr;
    int* fb_list = nullptr;               // particles handed to the per-particle kernel-length solve
    unsigned long long* fb_count = nullptr;
    int* tails = nullptr;                 // per-particle tail buffers of the flux lists (kTailBuf slots)
    int* fb2_list = nullptr;              // particles the list solver hands to the rescanning one
    unsigned long long* fb2_count = nullptr;
    void* rec = nullptr;                  // 32 x 8 B per particle
    double4* prim = nullptr;              // 128 B per particle: what gradients read of a neighbour
    double *vp = nullptr, *up = nullptr, *Ehalf = nullptr;
    double* mp = nullptr;                 // predicted masses of the finite-volume step
    double *dt_part = nullptr, *dt_out = nullptr;
    Counters* cnt = nullptr;
    double* adj = nullptr;                // adjoint scratch, kAdjSlots x cap, allocated on first use
    double* lev = nullptr;                // per-level rates of hierarchical steps, 4 (kMaxBin+1) x cap, on first use
    int have_levels = 0, lev_nlev = 0;    // lev holds the rates of the current order, for lev_nlev levels
    unsigned char* hmode = nullptr;       // per-particle modes of active-subset sub-steps, on first use
    unsigned* hmarks = nullptr;           // one bit per cell-table entry: cells holding a due particle
    long long* hhome = nullptr;           // per particle: its column of the rates within a system step
    double* hmoved = nullptr;             // path length since the last build, per particle, and its largest
    int64_t n_tree = -1;
    int have_h = 0, have_grad = 0, have_flux = 0, rec_mixed = 0;
    hipStream_t last = nullptr;
    int timing = 0;
    KernelClock clk[3];                   // indexed by mfm_kernel
    char err[256] = {0};                  // last error message (a fixed buffer: no allocation on any path)
};

static void clock_drain(KernelClock& k) {
    for (auto& e : k.pending) {
        float ms = 0.0f;
        (void)hipEventSynchronize(e.second);
        (void)hipEventElapsedTime(&ms, e.first, e.second);
        k.total_ms += ms;
        k.launches++;
        k.spare.push_back(e);
    }
    k.pending.clear();
}

// event pair for the next launch of kernel k (both null when timing is off)
static std::pair<hipEvent_t, hipEvent_t> clock_take(mfm_ctx* c, int k) {
    if (!c->timing) return {nullptr, nullptr};
    KernelClock& kc = c->clk[k];
    if (kc.pending.size() >= 256) clock_drain(kc);
    std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
    if (!kc.spare.empty()) {
        e = kc.spare.back();
        kc.spare.pop_back();
    } else if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) {
        return {nullptr, nullptr};
    }
    kc.pending.push_back(e);
    return e;
}

static void clock_reset(mfm_ctx* c) {
    for (KernelClock& k : c->clk) {
        clock_drain(k);
        k.total_ms = 0.0;
        k.launches = 0;
    }
}

static mfm_status fail(mfm_ctx* c, mfm_status s, const char* m) {
    if (c) snprintf(c->err, sizeof c->err, "%s", m);
    return s;
}

static mfm_status hip_check(mfm_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return MFM_OK;
    if (c) snprintf(c->err, sizeof c->err, "%s: %s", what, hipGetErrorString(e));
    return MFM_E_HIP;
}

static mfm_status launched(mfm_ctx* c, const char* what) {
    return hip_check(c, hipGetLastError(), what);
}

static int ceil_log2(double v) {
    int b = 0;
    while ((double)(1ll << b) < v) b++;
    return b;
}

// Per-axis Morton layout: the longest axis gets bmax bits, shorter axes start
// refining once the cells along the longest axis are no longer than them.
static void setup_tree(mfm_ctx* c) {
    TreeDesc& td = c->td;
    memset(&td, 0, sizeof(td));
    int bmax = c->p.tree_levels;
    if (bmax <= 0) bmax = ceil_log2(cbrt((double)c->cap)) + 2;   // ~1/64 particle per finest cell
    if (bmax < 2) bmax = 2;
    if (bmax > kMaxLevels - 1) bmax = kMaxLevels - 1;
    double Lmax = fmax(c->p.box[0], fmax(c->p.box[1], c->p.box[2]));
    for (int d = 0; d < 3; d++) {
        int drop = (int)lround(log2(Lmax / c->p.box[d]));
        int q = bmax - (drop > 0 ? drop : 0);
        td.qbits[d] = q > 0 ? q : 0;
        td.box[d] = c->p.box[d];
        td.periodic[d] = c->p.periodic[d];
    }
    td.bmax = bmax;
    long long off = 0;
    int k = 0;
    for (int l = 0; l <= bmax; l++) {
        int m = 0, nb = 0;
        for (int d = 0; d < 3; d++)
            if (l >= 1 && l > bmax - td.qbits[d]) {
                m |= 1 << d;
                nb++;
            }
        k += nb;
        td.actmask[l] = m;
        td.kbits[l] = k;
        td.tab_off[l] = off;
        off += 1ll << k;
        for (int d = 0; d < 3; d++) {
            int act = l - (bmax - td.qbits[d]);
            if (act < 0) act = 0;
            td.cs[l][d] = c->p.box[d] / (double)(1ll << act);
            td.ncell[l][d] = 1 << act;
        }
        // bit positions of each axis in the level-l key prefix: bits appended
        // level by level, axes x, y, z in that order, the last one lowest
        int pos = k;
        for (int lev = 1; lev <= l; lev++)
            for (int d = 0; d < 3; d++)
                if (td.actmask[lev] & (1 << d)) {
                    pos--;
                    td.mask[l][d] |= 1ull << pos;
                }
    }
    td.ktot = k;
    c->tab_len = off;
}

// mfm_create's parameter checks (see include/mfm.h)
static bool params_valid(const mfm_params& p) {
    if (!(p.gamma > 1.0) || !(p.n_ngb > 32.0 / 3.0) || !(p.beta > 0.0) || !(p.cond_max > 0.0)) return false;
    for (int d = 0; d < 3; d++)
        if (!(p.box[d] > 0.0) || (p.periodic[d] != 0 && p.periodic[d] != 1)) return false;
    if (p.precision != MFM_FP64 && p.precision != MFM_MIXED) return false;
    if (p.scheme != MFM_SCHEME_MFM && p.scheme != MFM_SCHEME_MFV) return false;
    if (p.limiter != 0 && p.limiter != 1) return false;
    if (p.limiter && (!(p.beta_min > 0.0) || !(p.cond_lo > 0.0) || !(p.cond_hi > p.cond_lo))) return false;
    return true;
}

// parameters, device-side physics and the cell-table layout of a context
static void init_params(mfm_ctx* c, const mfm_params& p) {
    c->p = p;
    c->ph.gamma = p.gamma;
    c->ph.n_ngb = p.n_ngb;
    c->ph.beta = p.beta;
    c->ph.cond_max = p.cond_max;
    for (int d = 0; d < 3; d++) {
        c->ph.box[d] = p.box[d];
        c->ph.periodic[d] = p.periodic[d];
    }
    c->ph.h_maxit = p.h_maxit > 0 ? p.h_maxit : 64;
    c->ph.max_ngb = p.max_ngb > 0 ? p.max_ngb : 256;
    c->ph.limiter = p.limiter;
    c->ph.beta_min = p.beta_min;
    c->ph.cond_lo = p.cond_lo;
    c->ph.cond_hi = p.cond_hi;
    setup_tree(c);
}

extern "C" {

const char* mfm_status_str(mfm_status s) {
    // a C caller may pass any int: copy the bits out rather than load an
    // enum value outside the enumeration's range
    static_assert(sizeof(mfm_status) == sizeof(int), "mfm_status is an int");
    int v;
    memcpy(&v, &s, sizeof v);
    switch (v) {
        case MFM_OK: return "ok";
        case MFM_E_INVALID: return "invalid argument";
        case MFM_E_HIP: return "HIP runtime error";
        case MFM_E_NOCONV: return "kernel length did not converge";
        case MFM_E_ILLCOND: return "ill-conditioned gradient matrix";
        case MFM_E_MINIMAGE: return "kernel length reached half a periodic box side";
        case MFM_E_CAPACITY: return "capacity exceeded";
        case MFM_E_NONFINITE: return "non-finite result";
        case MFM_E_STATE: return "call order violated";
    }
    return "unknown status";
}

const char* mfm_last_error(const mfm_ctx* c) { return c ? c->err : "null context"; }

int32_t mfm_max_ngb(const mfm_ctx* c) { return c ? c->ph.max_ngb : 0; }

void mfm_destroy(mfm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (KernelClock& k : c->clk) {
        clock_drain(k);
        for (auto& e : k.spare) {
            hipEventDestroy(e.first);
            hipEventDestroy(e.second);
        }
    }
    void* bufs[] = {c->keys, c->ktmp, c->idx, c->vtmp, c->hist, c->scan_tmp, c->gtmp, c->tab, c->pos, c->rl,
                    c->counts, c->gcount, c->list, c->fb_list, c->fb_count, c->fb2_list, c->fb2_count, c->tails, c->rec, c->prim, c->vp, c->up, c->Ehalf, c->mp, c->dt_part, c->dt_out, c->cnt, c->adj, c->lev,
                    c->hmode, c->hmarks, c->hhome, c->hmoved};
    for (void* b : bufs)
        if (b) hipFree(b);
    delete c;
}

mfm_status mfm_create(const mfm_params* params, int64_t capacity, mfm_ctx** out) {
    if (!out) return MFM_E_INVALID;
    *out = nullptr;
    if (!params || !params_valid(*params)) return MFM_E_INVALID;
    if (capacity < 1 || capacity > (1ll << 30)) return MFM_E_INVALID;
    mfm_ctx* c = new mfm_ctx();
    c->cap = capacity;
    (void)hipGetDevice(&c->device);
    init_params(c, *params);
    const long long n = capacity;
    const int nblocks = (int)((n + 2047) / 2048);
    const long long hist_len = 256ll * nblocks;
    mfm_status st = MFM_OK;
    auto alloc = [&](void** ptr, size_t bytes, const char* what) {
        if (st != MFM_OK) return;
        st = hip_check(c, hipMalloc(ptr, bytes < 16 ? 16 : bytes), what);
    };
    alloc((void**)&c->keys, sizeof(unsigned long long) * n, "keys");
    alloc((void**)&c->ktmp, sizeof(unsigned long long) * n, "keys tmp");
    alloc((void**)&c->idx, sizeof(int) * n, "idx");
    alloc((void**)&c->vtmp, sizeof(int) * n, "idx tmp");
    alloc((void**)&c->hist, sizeof(int) * hist_len, "hist");
    alloc((void**)&c->scan_tmp, sizeof(int) * scan_tmp_ints(hist_len > n ? hist_len : n), "scan tmp");
    alloc((void**)&c->gtmp, sizeof(unsigned long long) * n * kGatherMax, "gather staging");
    alloc((void**)&c->tab, sizeof(int2) * c->tab_len, "cell tables");
    alloc((void**)&c->pos, sizeof(double4) * n, "packed positions");
    alloc((void**)&c->rl, sizeof(double) * n * kRCap, "radius lists");
    alloc((void**)&c->counts, sizeof(int) * n, "list counts");
    alloc((void**)&c->gcount, sizeof(int) * n, "gather counts");
    alloc((void**)&c->list, sizeof(int) * n * c->ph.max_ngb, "flux lists");
    alloc((void**)&c->fb_list, sizeof(int) * n, "fallback list");
    alloc((void**)&c->fb_count, sizeof(unsigned long long), "fallback count");
    alloc((void**)&c->fb2_list, sizeof(int) * n, "second fallback list");
    alloc((void**)&c->tails, sizeof(int) * (size_t)kTailBuf * n, "tail buffers");
    alloc((void**)&c->fb2_count, sizeof(unsigned long long), "second fallback count");
    alloc((void**)&c->rec, sizeof(double) * 32 * n, "records");
    alloc((void**)&c->prim, sizeof(double4) * 4 * n, "neighbour records");
    alloc((void**)&c->vp, sizeof(double) * 3 * n, "predicted v");
    alloc((void**)&c->up, sizeof(double) * n, "predicted u");
    alloc((void**)&c->Ehalf, sizeof(double) * n, "half-step energy");
    if (params->scheme == MFM_SCHEME_MFV) alloc((void**)&c->mp, sizeof(double) * n, "predicted masses");
    alloc((void**)&c->dt_part, sizeof(double) * 1024, "dt partials");
    alloc((void**)&c->dt_out, sizeof(double) * 2, "dt");
    alloc((void**)&c->cnt, (size_t)kCounterCopies * kCounterStride, "counters");
    if (st != MFM_OK) {
        fprintf(stderr, "mfm_create: %s\n", c->err);
        mfm_destroy(c);
        return st;
    }
    *out = c;
    return MFM_OK;
}

static void reset_counters(mfm_ctx* c, hipStream_t s) { launch_reset_counters(c->cnt, s); }

static mfm_status check_particles(mfm_ctx* c, const mfm_particles* p) {
    if (!c) return MFM_E_INVALID;
    if (!p) return fail(c, MFM_E_INVALID, "null particle struct");
    if (p->n < 1) return fail(c, MFM_E_INVALID, "n must be >= 1");
    if (p->n > c->cap) return fail(c, MFM_E_CAPACITY, "n exceeds the context capacity");
    if (!p->x || !p->y || !p->z || !p->m || !p->vx || !p->vy || !p->vz || !p->u || !p->H)
        return fail(c, MFM_E_INVALID, "x, y, z, m, vx, vy, vz, u and H are required");
    return MFM_OK;
}

static PassArrays arrays_of(const mfm_particles* p) {
    PassArrays a;
    a.n = (int)p->n;
    a.x = p->x;
    a.y = p->y;
    a.z = p->z;
    a.m = p->m;
    a.vx = p->vx;
    a.vy = p->vy;
    a.vz = p->vz;
    a.u = p->u;
    a.H = p->H;
    a.nk = p->nk;
    a.V = p->V;
    a.B = p->B;
    a.rho = p->rho;
    a.P = p->P;
    a.grad = p->grad;
    a.alpha = p->alpha;
    a.dp = p->dp;
    a.dE = p->dE;
    a.vsig = p->vsig;
    a.dm = p->dm;
    return a;
}

// order by key and reorder `extra` arrays too (step scratch)
static mfm_status build(mfm_ctx* c, mfm_particles* p, hipStream_t s, double* const* extra, int nextra) {
    const int n = (int)p->n;
    (void)hipSetDevice(c->device);
    // clear the last build's cells while its sorted keys are still there
    if (c->tab_keys_n > 0) launch_untables((int)c->tab_keys_n, c->keys, c->td, c->tab, s);
    else launch_fill_u64(c->tab_len, (unsigned long long*)c->tab, 0ull, s);
    c->tab_keys_n = -1;
    launch_keys(n, p->x, p->y, p->z, c->td, c->keys, c->idx, s);
    radix_sort(n, c->td.ktot, c->keys, c->idx, c->ktmp, c->vtmp, c->hist, c->scan_tmp, s);
    // each batch: one launch copies its arrays to the staging, one gathers them back in key order
    GatherBatch gb, cb;
    gb.count = cb.count = 0;
    auto flush = [&]() {
        launch_copy_batch(n, cb, s);
        launch_gather(n, gb, c->idx, s);
        gb.count = cb.count = 0;
    };
    auto add = [&](void* ptr) {
        if (!ptr) return;
        if (gb.count == kGatherMax) flush();   // staging full: reorder this batch, then reuse the staging
        unsigned long long* stage = c->gtmp + (long long)gb.count * n;
        cb.src[cb.count] = (const unsigned long long*)ptr;
        cb.dst[cb.count] = stage;
        cb.count++;
        gb.src[gb.count] = stage;
        gb.dst[gb.count] = (unsigned long long*)ptr;
        gb.count++;
    };
    add(p->x);
    add(p->y);
    add(p->z);
    add(p->m);
    add(p->vx);
    add(p->vy);
    add(p->vz);
    add(p->u);
    add(p->H);
    if (p->dp) {
        add(p->dp);
        add(p->dp + n);
        add(p->dp + 2 * (long long)n);
    }
    add(p->dE);
    add(p->vsig);
    add(p->dm);
    add(p->id);
    for (int k = 0; k < nextra; k++) add(extra[k]);
    flush();
    launch_tables(n, c->keys, c->td, c->tab, s);
    launch_pos4(n, p->x, p->y, p->z, c->pos, s);
    c->n_tree = n;
    c->have_h = c->have_grad = c->have_flux = 0;
    c->last = s;
    mfm_status st = launched(c, "build_neighbours");
    if (!st) c->tab_keys_n = n;
    return st;
}

mfm_status mfm_build_neighbours(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    return build(c, p, (hipStream_t)stream, nullptr, 0);
}

// The particles back in the order they were given in: particle k moves to
// position id[k] in every array that is set, after a device check (one
// synchronisation) that id is a permutation of 0 .. n-1.  The context's cell
// tables, lists and per-level rates belong to the old order afterwards.
mfm_status mfm_unpermute(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    if (!p->id) return fail(c, MFM_E_INVALID, "id is required to restore the input order");
    const int n = (int)p->n;
    hipStream_t s = (hipStream_t)stream;
    (void)hipSetDevice(c->device);
    launch_fill_u64(1, c->fb_count, 0ull, s);
    launch_check_perm(n, (const long long*)p->id, c->vtmp, c->fb_count, s);
    unsigned long long bad = 0;
    st = hip_check(c, hipMemcpyAsync(&bad, c->fb_count, sizeof bad, hipMemcpyDeviceToHost, s), "id check");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "id check");
    if (st) return st;
    if (bad) return fail(c, MFM_E_INVALID, "id is not a permutation of 0 .. n-1");
    launch_narrow_ids(n, (const long long*)p->id, c->idx, s);
    // each batch: one launch copies its arrays to the staging, one scatters them back
    GatherBatch sb, cb;
    sb.count = cb.count = 0;
    auto flush = [&]() {
        launch_copy_batch(n, cb, s);
        launch_unpermute(n, sb, c->idx, s);
        sb.count = cb.count = 0;
    };
    auto add = [&](void* ptr, int rows) {
        if (!ptr) return;
        for (int r = 0; r < rows; r++) {
            if (sb.count == kGatherMax) flush();
            unsigned long long* stage = c->gtmp + (long long)sb.count * n;
            cb.src[cb.count] = (const unsigned long long*)ptr + (long long)r * n;
            cb.dst[cb.count] = stage;
            cb.count++;
            sb.src[sb.count] = stage;
            sb.dst[sb.count] = (unsigned long long*)ptr + (long long)r * n;
            sb.count++;
        }
    };
    add(p->x, 1);
    add(p->y, 1);
    add(p->z, 1);
    add(p->m, 1);
    add(p->vx, 1);
    add(p->vy, 1);
    add(p->vz, 1);
    add(p->u, 1);
    add(p->H, 1);
    add(p->nk, 1);
    add(p->V, 1);
    add(p->B, 6);
    add(p->rho, 1);
    add(p->P, 1);
    add(p->grad, 15);
    add(p->alpha, 5);
    add(p->dp, 3);
    add(p->dE, 1);
    add(p->vsig, 1);
    add(p->dm, 1);
    add(p->id, 1);
    flush();
    c->n_tree = -1;
    c->have_h = c->have_grad = c->have_flux = 0;
    c->have_levels = 0;
    c->last = s;
    return launched(c, "unpermute");
}

static mfm_status do_solve_h(mfm_ctx* c, mfm_particles* p, hipStream_t s) {
    if (!p->nk || !p->V) return fail(c, MFM_E_INVALID, "nk and V are required");
    if (c->n_tree != p->n) return fail(c, MFM_E_STATE, "mfm_build_neighbours must run on these particles first");
    PassArrays a = arrays_of(p);
    const auto ev = clock_take(c, MFM_KERNEL_SOLVE_H);
    launch_solve_h(a, c->td, c->tab, c->pos, c->ph, c->cnt, c->rl, c->list, c->gcount, c->counts,
                   c->fb_list, c->fb_count, c->fb2_list, c->fb2_count, ev.first, ev.second, s);
    c->have_h = 1;
    c->have_grad = c->have_flux = 0;
    c->have_levels = 0;
    c->last = s;
    return launched(c, "solve_h");
}

static mfm_status do_gradients(mfm_ctx* c, mfm_particles* p, hipStream_t s) {
    if (!p->B || !p->rho || !p->P || !p->grad || !p->nk || !p->V)
        return fail(c, MFM_E_INVALID, "B, rho, P, grad, nk and V are required");
    if (!c->have_h || c->n_tree != p->n) return fail(c, MFM_E_STATE, "mfm_solve_h must run first");
    PassArrays a = arrays_of(p);
    c->rec_mixed = c->p.precision == MFM_MIXED;
    c->have_flux = 0;
    const auto ev = clock_take(c, MFM_KERNEL_GRADIENTS);
    launch_gradients(a, c->ph, c->gcount, c->counts, c->list, c->tails, c->rec_mixed, c->prim, c->rec, c->cnt, ev.first,
                     ev.second, s);
    c->have_grad = 1;
    c->last = s;
    return launched(c, "gradients");
}

static mfm_status do_fluxes(mfm_ctx* c, mfm_particles* p, hipStream_t s) {
    if (!p->dp || !p->dE || !p->vsig) return fail(c, MFM_E_INVALID, "dp, dE and vsig are required");
    const int mfv = c->p.scheme == MFM_SCHEME_MFV;
    if (mfv && !p->dm) return fail(c, MFM_E_INVALID, "the finite-volume scheme needs dm");
    if (!c->have_grad || c->n_tree != p->n) return fail(c, MFM_E_STATE, "mfm_gradients must run first");
    PassArrays a = arrays_of(p);
    const auto ev = clock_take(c, MFM_KERNEL_FLUXES);
    if (ev.first) hipEventRecord(ev.first, s);
    launch_fluxes(a, c->ph, c->counts, c->list, c->rec_mixed, mfv, c->rec, c->cnt, s);
    if (ev.second) hipEventRecord(ev.second, s);
    c->have_flux = 1;
    c->last = s;
    return launched(c, "hydro_fluxes");
}

mfm_status mfm_solve_h(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    (void)hipSetDevice(c->device);
    reset_counters(c, (hipStream_t)stream);
    return do_solve_h(c, p, (hipStream_t)stream);
}

mfm_status mfm_gradients(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    (void)hipSetDevice(c->device);
    return do_gradients(c, p, (hipStream_t)stream);
}

mfm_status mfm_hydro_fluxes(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    (void)hipSetDevice(c->device);
    return do_fluxes(c, p, (hipStream_t)stream);
}

mfm_status mfm_hydro_pass(mfm_ctx* c, mfm_particles* p, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    (void)hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (c->p.scheme == MFM_SCHEME_MFV && !p->dm) return fail(c, MFM_E_INVALID, "the finite-volume scheme needs dm");
    reset_counters(c, s);
    if ((st = do_solve_h(c, p, s))) return st;
    if ((st = do_gradients(c, p, s))) return st;
    return do_fluxes(c, p, s);
}

// One step's tape (caller-owned device memory): in the step's own order, after
// its reorder, kTapeD doubles per particle (component-major, [slot * n + i]),
// then the step's permutation, the list counts, the gather counts and the flux
// lists ([k * n + i], max_ngb slots).
enum { T_X = 0, T_M = 3, T_V1 = 4, T_EH = 7, T_VP = 8, T_UP = 11, T_DP = 12, T_DE = 15, T_H = 16, T_NK = 17,
       T_V = 18, T_B = 19, T_RHO = 25, T_P = 26, T_GRAD = 27, kTapeD = 42 };

static long long tape_bytes(const mfm_ctx* c, long long n) {
    return (long long)sizeof(double) * kTapeD * n + (long long)sizeof(int) * (3 + (long long)c->ph.max_ngb) * n;
}

struct TapeView {
    double* d;
    int *idx, *counts, *gcount, *list;
};

static TapeView tape_view(void* t, long long n) {
    TapeView v;
    v.d = (double*)t;
    int* ib = (int*)(v.d + (long long)kTapeD * n);
    v.idx = ib;
    v.counts = ib + n;
    v.gcount = ib + 2 * n;
    v.list = ib + 3 * n;
    return v;
}

// after the step's pass, before its closing kick: the state, the predicted
// state, the pass outputs, the permutation and the lists, into the tape
static mfm_status write_tape(mfm_ctx* c, const mfm_particles* p, void* tape, hipStream_t s) {
    const long long n = p->n;
    TapeView t = tape_view(tape, n);
    GatherBatch cb;
    cb.count = 0;
    auto cp = [&](int slot, const double* src) {
        if (cb.count == kGatherMax) {
            launch_copy_batch((int)n, cb, s);
            cb.count = 0;
        }
        cb.src[cb.count] = (const unsigned long long*)src;
        cb.dst[cb.count] = (unsigned long long*)(t.d + (long long)slot * n);
        cb.count++;
    };
    cp(T_X, p->x);
    cp(T_X + 1, p->y);
    cp(T_X + 2, p->z);
    cp(T_M, p->m);
    cp(T_V1, p->vx);
    cp(T_V1 + 1, p->vy);
    cp(T_V1 + 2, p->vz);
    cp(T_EH, c->Ehalf);
    for (int k = 0; k < 3; k++) cp(T_VP + k, c->vp + k * n);
    cp(T_UP, c->up);
    for (int k = 0; k < 3; k++) cp(T_DP + k, p->dp + k * n);
    cp(T_DE, p->dE);
    cp(T_H, p->H);
    cp(T_NK, p->nk);
    cp(T_V, p->V);
    for (int k = 0; k < 6; k++) cp(T_B + k, p->B + k * n);
    cp(T_RHO, p->rho);
    cp(T_P, p->P);
    for (int k = 0; k < 15; k++) cp(T_GRAD + k, p->grad + k * n);
    launch_copy_batch((int)n, cb, s);
    mfm_status st;
    if ((st = hip_check(c, hipMemcpyAsync(t.idx, c->idx, sizeof(int) * n, hipMemcpyDeviceToDevice, s), "tape idx")))
        return st;
    if ((st = hip_check(c, hipMemcpyAsync(t.counts, c->counts, sizeof(int) * n, hipMemcpyDeviceToDevice, s),
                        "tape counts")))
        return st;
    if ((st = hip_check(c, hipMemcpyAsync(t.gcount, c->gcount, sizeof(int) * n, hipMemcpyDeviceToDevice, s),
                        "tape gather counts")))
        return st;
    launch_copy_lists((int)n, c->counts, c->list, t.list, s);
    return MFM_OK;
}

static mfm_status do_step(mfm_ctx* c, mfm_particles* p, double dt, double* dt_used, void* tape, void* stream);

mfm_status mfm_step(mfm_ctx* c, mfm_particles* p, double dt, double* dt_used, void* stream) {
    return do_step(c, p, dt, dt_used, nullptr, stream);
}

extern "C" int64_t mfm_tape_bytes(const mfm_ctx* c) { return c ? (int64_t)tape_bytes(c, c->cap) : -1; }

extern "C" mfm_status mfm_step_taped(mfm_ctx* c, mfm_particles* p, double dt, void* tape, void* stream) {
    if (!c) return MFM_E_INVALID;
    if (!tape) return fail(c, MFM_E_INVALID, "null tape");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, MFM_E_INVALID, "a taped step needs a fixed dt > 0");
    if (c->p.scheme != MFM_SCHEME_MFM || c->p.limiter)
        return fail(c, MFM_E_INVALID, "the adjoints cover the MFM scheme with the per-particle limiter only");
    return do_step(c, p, dt, nullptr, tape, stream);
}

static mfm_status do_step(mfm_ctx* c, mfm_particles* p, double dt, double* dt_used, void* tape, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    const int mfv = c->p.scheme == MFM_SCHEME_MFV;
    if (!p->dp || !p->dE || !p->vsig || !p->nk || !p->V || !p->B || !p->rho || !p->P || !p->grad || (mfv && !p->dm))
        return fail(c, MFM_E_INVALID, "mfm_step needs every pass output array");
    if (!c->have_flux || c->n_tree != p->n)
        return fail(c, MFM_E_STATE, "mfm_step needs a pass on the current state (mfm_hydro_pass)");
    (void)hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)p->n;
    if (!(dt > 0.0)) {
        const int parts = dt_min_parts(n);
        launch_dt_min(n, p->H, p->vsig, c->dt_part, parts, c->dt_out, s);
        double h = 0.0;
        if ((st = hip_check(c, hipMemcpyAsync(&h, c->dt_out, sizeof(double), hipMemcpyDeviceToHost, s), "dt copy")))
            return st;
        if ((st = hip_check(c, hipStreamSynchronize(s), "dt sync"))) return st;
        dt = c->p.cfl * h;
        if (!(dt > 0.0) || !isfinite(dt)) return fail(c, MFM_E_NONFINITE, "Courant step is not positive and finite");
    }
    if (dt_used) *dt_used = dt;
    reset_counters(c, s);
    PassArrays a = arrays_of(p);
    if (mfv)
        launch_kick_drift_mfv(a, c->ph, dt, c->p.u_floor, c->vp, c->up, c->Ehalf, c->mp, s);
    else
        launch_kick_drift(a, c->ph, dt, c->p.u_floor, c->vp, c->up, c->Ehalf, s);
    double* extra[6] = {c->vp, c->vp + n, c->vp + 2 * (long long)n, c->up, c->Ehalf, c->mp};
    if ((st = build(c, p, s, extra, mfv ? 6 : 5))) return st;
    // pass on the predicted state (with the predicted masses in the finite-volume form)
    mfm_particles q = *p;
    q.vx = c->vp;
    q.vy = c->vp + n;
    q.vz = c->vp + 2 * (long long)n;
    q.u = c->up;
    if (mfv) q.m = c->mp;
    if ((st = do_solve_h(c, &q, s))) return st;
    if ((st = do_gradients(c, &q, s))) return st;
    if ((st = do_fluxes(c, &q, s))) return st;
    if (tape && (st = write_tape(c, p, tape, s))) return st;
    a = arrays_of(p);
    if (mfv)
        launch_kick2_mfv(a, dt, c->p.u_floor, c->Ehalf, p->u, c->cnt, s);
    else
        launch_kick2(a, dt, c->p.u_floor, c->Ehalf, p->u, c->cnt, s);
    c->last = s;
    return launched(c, "step");
}

mfm_status mfm_set_kernel_timing(mfm_ctx* c, int enable) {
    if (!c) return MFM_E_INVALID;
    (void)hipSetDevice(c->device);
    clock_reset(c);
    c->timing = enable ? 1 : 0;
    return MFM_OK;
}

mfm_status mfm_kernel_time(mfm_ctx* c, int kernel, double* total_ms, int64_t* launches) {
    if (!c || kernel < 0 || kernel > 2 || !total_ms || !launches) return fail(c, MFM_E_INVALID, "bad kernel timing query");
    (void)hipSetDevice(c->device);
    clock_drain(c->clk[kernel]);
    *total_ms = c->clk[kernel].total_ms;
    *launches = c->clk[kernel].launches;
    return MFM_OK;
}

mfm_status mfm_get_counters(mfm_ctx* c, mfm_counters* out) {
    if (!c || !out) return MFM_E_INVALID;
    (void)hipSetDevice(c->device);
    mfm_status st;
    if ((st = hip_check(c, hipStreamSynchronize(c->last), "sync"))) return st;
    // combine the per-block-group copies: sums, maxima and the smallest index
    unsigned char raw[kCounterCopies * kCounterStride];
    if ((st = hip_check(c, hipMemcpy(raw, c->cnt, sizeof(raw), hipMemcpyDeviceToHost), "counter copy"))) return st;
    Counters h;
    memcpy(&h, raw, sizeof(h));
    for (int k = 1; k < kCounterCopies; k++) {
        Counters o;
        memcpy(&o, raw + (size_t)k * kCounterStride, sizeof(o));
        h.list_entries += o.list_entries;
        h.list_max = std::max(h.list_max, o.list_max);
        h.h_iters += o.h_iters;
        h.h_iters_max = std::max(h.h_iters_max, o.h_iters_max);
        h.noconv += o.noconv;
        h.minimage += o.minimage;
        h.overflow += o.overflow;
        h.illcond += o.illcond;
        h.fallbacks += o.fallbacks;
        h.clamps += o.clamps;
        h.nonfinite += o.nonfinite;
        h.floors += o.floors;
        h.first_bad = std::min(h.first_bad, o.first_bad);
        h.cond_bits = std::max(h.cond_bits, o.cond_bits);   // positive doubles order as their bits
        h.h_rounds_max = std::max(h.h_rounds_max, o.h_rounds_max);
        h.h_fallback += o.h_fallback;
        h.h_rounds3 += o.h_rounds3;
        h.gather_entries += o.gather_entries;
        h.h_rescan += o.h_rescan;
    }
    static_assert(sizeof(Counters) == 19 * 8, "combine every counter field");
    out->list_entries = (int64_t)h.list_entries;
    out->pairs = (int64_t)(h.list_entries / 2);
    out->list_max = (int64_t)h.list_max;
    out->h_iters = (int64_t)h.h_iters;
    out->h_iters_max = (int64_t)h.h_iters_max;
    out->noconv = (int64_t)h.noconv;
    out->minimage = (int64_t)h.minimage;
    out->overflow = (int64_t)h.overflow;
    out->illcond = (int64_t)h.illcond;
    out->fallbacks = (int64_t)h.fallbacks;
    out->clamps = (int64_t)h.clamps;
    out->nonfinite = (int64_t)h.nonfinite;
    out->floors = (int64_t)h.floors;
    out->first_bad = h.first_bad == ~0ull ? -1 : (int64_t)h.first_bad;
    double cm;
    memcpy(&cm, &h.cond_bits, sizeof(cm));
    out->cond_max_seen = cm;
    out->h_rounds_max = (int64_t)h.h_rounds_max;
    out->h_fallback = (int64_t)h.h_fallback;
    out->h_rounds3 = (int64_t)h.h_rounds3;
    out->gather_entries = (int64_t)h.gather_entries;
    out->h_rescan = (int64_t)h.h_rescan;
    return MFM_OK;
}

// the status that a set of device counters stands for (mfm_check's precedence)
static mfm_status status_of(mfm_ctx* c, const mfm_counters& k) {
    char buf[160];
    if (k.noconv) {
        snprintf(buf, sizeof buf, "%lld particles without a converged kernel length (first %lld)",
                 (long long)k.noconv, (long long)k.first_bad);
        return fail(c, MFM_E_NOCONV, buf);
    }
    if (k.minimage) {
        snprintf(buf, sizeof buf, "%lld kernel lengths reached half a periodic side (first %lld)",
                 (long long)k.minimage, (long long)k.first_bad);
        return fail(c, MFM_E_MINIMAGE, buf);
    }
    if (k.overflow) {
        snprintf(buf, sizeof buf, "%lld flux lists exceeded max_ngb=%d (longest %lld)", (long long)k.overflow,
                 c->ph.max_ngb, (long long)k.list_max);
        return fail(c, MFM_E_CAPACITY, buf);
    }
    if (k.nonfinite) {
        snprintf(buf, sizeof buf, "%lld non-finite outputs (first %lld)", (long long)k.nonfinite,
                 (long long)k.first_bad);
        return fail(c, MFM_E_NONFINITE, buf);
    }
    if (k.illcond) {
        snprintf(buf, sizeof buf, "%lld ill-conditioned gradient matrices (first %lld)", (long long)k.illcond,
                 (long long)k.first_bad);
        return fail(c, MFM_E_ILLCOND, buf);
    }
    return MFM_OK;
}

mfm_status mfm_check(mfm_ctx* c) {
    mfm_counters k;
    mfm_status st = mfm_get_counters(c, &k);
    if (st) return st;
    return status_of(c, k);
}

mfm_status mfm_copy_flux_lists(mfm_ctx* c, int32_t* counts, int32_t* list, void* stream) {
    if (!c || !counts || !list) return MFM_E_INVALID;
    if (!c->have_grad) return fail(c, MFM_E_STATE, "no flux lists yet (they are complete after mfm_gradients)");
    (void)hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    const long long n = c->n_tree;
    mfm_status st;
    if ((st = hip_check(c, hipMemcpyAsync(counts, c->counts, sizeof(int) * n, hipMemcpyDeviceToDevice, s),
                        "copy counts")))
        return st;
    return hip_check(c, hipMemcpyAsync(list, c->list, sizeof(int) * n * c->ph.max_ngb, hipMemcpyDeviceToDevice, s),
                     "copy lists");
}

}  // extern "C"

// ------------------------------------------------------------------ adjoints

static mfm_status ensure_adj(mfm_ctx* c) {
    if (c->adj) return MFM_OK;
    return hip_check(c, hipMalloc((void**)&c->adj, sizeof(double) * kAdjSlots * c->cap), "adjoint scratch");
}

extern "C" mfm_status mfm_hydro_pass_adjoint(mfm_ctx* c, const mfm_particles* p, const double* adj_dp,
                                             const double* adj_dE, double* adj_x, double* adj_v, double* adj_u,
                                             void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    if (c->p.scheme != MFM_SCHEME_MFM || c->p.limiter)
        return fail(c, MFM_E_INVALID, "the adjoints cover the MFM scheme with the per-particle limiter only");
    if (!adj_dp || !adj_dE || !adj_x || !adj_v || !adj_u) return fail(c, MFM_E_INVALID, "null adjoint array");
    if (!p->nk || !p->V || !p->B || !p->rho || !p->P || !p->grad)
        return fail(c, MFM_E_INVALID, "the pass adjoint needs the forward outputs nk, V, B, rho, P, grad");
    if (!c->have_grad || !c->have_flux || c->n_tree != p->n)
        return fail(c, MFM_E_STATE, "the pass adjoint needs the pass of this state on this context");
    (void)hipSetDevice(c->device);
    if ((st = ensure_adj(c))) return st;
    hipStream_t s = (hipStream_t)stream;
    PassArrays a = arrays_of(p);
    launch_pass_adjoint(a, c->ph, c->counts, c->gcount, c->list, adj_dp, adj_dE, c->adj, adj_x, adj_v, adj_u, s);
    c->last = s;
    return launched(c, "hydro_pass_adjoint");
}

// The reverse of one step (part two and three of the step adjoint): from the
// adjoints of the state after the step to those of the checkpoint, given the
// step's pass arrays q (predicted state and pass outputs, in the step's
// order), its state after the first kick v1, its half-step energy, its flux
// lists and its permutation idx (step order -> checkpoint order).
static void reverse_step(mfm_ctx* c, const mfm_particles* q, const double* v1x, const double* v1y,
                         const double* v1z, const double* Ehalf, const int* counts, const int* gcount,
                         const int* list, const int* idx, const mfm_particles* ck, double dt, double* adj_x,
                         double* adj_v, double* adj_u, double* adj_dp, double* adj_dE, hipStream_t s) {
    const long long n = ck->n;
    double* A = c->adj;
    double* lxF = A + 28 * n;
    double* lvp = A + 31 * n;
    double* lup = A + 34 * n;
    double* lp2 = A + 35 * n;
    double* le2 = A + 38 * n;
    double* lv1 = A + 39 * n;
    double* lE1 = A + 42 * n;
    double* olx = A + 43 * n;
    double* olv = A + 46 * n;
    double* olu = A + 49 * n;
    double* olp = A + 50 * n;
    double* ole = A + 53 * n;
    double* olE0 = A + 54 * n;
    double* lE0 = A + 55 * n;
    launch_step_rev1((int)n, q->m, v1x, v1y, v1z, Ehalf, q->dp, q->dE, dt, c->p.u_floor, adj_x, adj_v, adj_u, adj_dp,
                     adj_dE, lp2, le2, lv1, lE1, s);
    PassArrays qa = arrays_of(q);
    launch_pass_adjoint(qa, c->ph, counts, gcount, list, lp2, le2, A, lxF, lvp, lup, s);
    launch_step_rev2((int)n, q->m, q->vx, q->u, dt, c->p.u_floor, adj_x, lxF, lvp, lup, lv1, lE1, olx, olv, olu, olp,
                     ole, olE0, s);
    GatherBatch gb;
    gb.count = 0;
    auto add = [&](const double* src, double* dst) {
        gb.src[gb.count] = (const unsigned long long*)src;
        gb.dst[gb.count] = (unsigned long long*)dst;
        gb.count++;
    };
    for (int k = 0; k < 3; k++) {
        add(olx + k * n, adj_x + k * n);
        add(olv + k * n, adj_v + k * n);
        add(olp + k * n, adj_dp + k * n);
    }
    add(olu, adj_u);
    add(ole, adj_dE);
    add(olE0, lE0);
    launch_unpermute((int)n, gb, idx, s);
    launch_step_rev3((int)n, ck->m, ck->vx, ck->vy, ck->vz, lE0, adj_v, s);
}

extern "C" mfm_status mfm_step_adjoint(mfm_ctx* c, const mfm_particles* ck, mfm_particles* w, double dt,
                                       double* adj_x, double* adj_v, double* adj_u, double* adj_dp, double* adj_dE,
                                       void* stream) {
    mfm_status st = check_particles(c, ck);
    if (st) return st;
    if (c->p.scheme != MFM_SCHEME_MFM || c->p.limiter)
        return fail(c, MFM_E_INVALID, "the adjoints cover the MFM scheme with the per-particle limiter only");
    if ((st = check_particles(c, w))) return st;
    if (w->n != ck->n) return fail(c, MFM_E_INVALID, "checkpoint and work sets differ in size");
    if (!(dt > 0.0)) return fail(c, MFM_E_INVALID, "the step adjoint needs a fixed dt > 0");
    if (!ck->dp || !ck->dE) return fail(c, MFM_E_INVALID, "the checkpoint needs dp and dE of its state");
    if (!w->dp || !w->dE || !w->vsig || !w->nk || !w->V || !w->B || !w->rho || !w->P || !w->grad)
        return fail(c, MFM_E_INVALID, "the work set needs every pass output array");
    if (!adj_x || !adj_v || !adj_u || !adj_dp || !adj_dE) return fail(c, MFM_E_INVALID, "null adjoint array");
    (void)hipSetDevice(c->device);
    if ((st = ensure_adj(c))) return st;
    hipStream_t s = (hipStream_t)stream;
    const long long n = ck->n;
    // 1. forward recompute of the step from the checkpoint, on the work set
    // (the checkpoint's arrays copied in one launch)
    {
        GatherBatch cb;
        cb.count = 0;
        auto cp = [&](void* dst, const void* src) {
            cb.src[cb.count] = (const unsigned long long*)src;
            cb.dst[cb.count] = (unsigned long long*)dst;
            cb.count++;
        };
        cp(w->x, ck->x);
        cp(w->y, ck->y);
        cp(w->z, ck->z);
        cp(w->m, ck->m);
        cp(w->vx, ck->vx);
        cp(w->vy, ck->vy);
        cp(w->vz, ck->vz);
        cp(w->u, ck->u);
        cp(w->H, ck->H);
        for (int k = 0; k < 3; k++) cp(w->dp + k * n, ck->dp + k * n);
        cp(w->dE, ck->dE);
        if (w->id && ck->id) cp(w->id, ck->id);
        launch_copy_batch((int)n, cb, s);
    }
    reset_counters(c, s);
    PassArrays a = arrays_of(w);
    launch_kick_drift(a, c->ph, dt, c->p.u_floor, c->vp, c->up, c->Ehalf, s);
    double* extra[5] = {c->vp, c->vp + n, c->vp + 2 * n, c->up, c->Ehalf};
    if ((st = build(c, w, s, extra, 5))) return st;
    mfm_particles q = *w;
    q.vx = c->vp;
    q.vy = c->vp + n;
    q.vz = c->vp + 2 * n;
    q.u = c->up;
    if ((st = do_solve_h(c, &q, s))) return st;
    if ((st = do_gradients(c, &q, s))) return st;
    if ((st = do_fluxes(c, &q, s))) return st;
    // 2. reverse, in the recomputed order; 3. back to the checkpoint's order
    reverse_step(c, &q, w->vx, w->vy, w->vz, c->Ehalf, c->counts, c->gcount, c->list, c->idx, ck, dt, adj_x, adj_v,
                 adj_u, adj_dp, adj_dE, s);
    c->last = s;
    return launched(c, "step_adjoint");
}

// The step's reverse from its tape: the same kernels as mfm_step_adjoint's
// part two and three, on the taped arrays instead of a recomputed step.
extern "C" mfm_status mfm_step_adjoint_taped(mfm_ctx* c, const mfm_particles* ck, const void* tape, double dt,
                                             double* adj_x, double* adj_v, double* adj_u, double* adj_dp,
                                             double* adj_dE, void* stream) {
    mfm_status st = check_particles(c, ck);
    if (st) return st;
    if (c->p.scheme != MFM_SCHEME_MFM || c->p.limiter)
        return fail(c, MFM_E_INVALID, "the adjoints cover the MFM scheme with the per-particle limiter only");
    if (!tape) return fail(c, MFM_E_INVALID, "null tape");
    if (!(dt > 0.0)) return fail(c, MFM_E_INVALID, "the step adjoint needs a fixed dt > 0");
    if (!adj_x || !adj_v || !adj_u || !adj_dp || !adj_dE) return fail(c, MFM_E_INVALID, "null adjoint array");
    (void)hipSetDevice(c->device);
    if ((st = ensure_adj(c))) return st;
    hipStream_t s = (hipStream_t)stream;
    const long long n = ck->n;
    TapeView t = tape_view(const_cast<void*>(tape), n);
    double* d = t.d;
    auto col = [&](int slot) { return d + (long long)slot * n; };
    mfm_particles q;
    memset(&q, 0, sizeof q);
    q.n = n;
    q.x = col(T_X);
    q.y = col(T_X + 1);
    q.z = col(T_X + 2);
    q.m = col(T_M);
    q.vx = col(T_VP);
    q.vy = col(T_VP + 1);
    q.vz = col(T_VP + 2);
    q.u = col(T_UP);
    q.H = col(T_H);
    q.nk = col(T_NK);
    q.V = col(T_V);
    q.B = col(T_B);
    q.rho = col(T_RHO);
    q.P = col(T_P);
    q.grad = col(T_GRAD);
    q.dp = col(T_DP);
    q.dE = col(T_DE);
    reverse_step(c, &q, col(T_V1), col(T_V1 + 1), col(T_V1 + 2), col(T_EH), t.counts, t.gcount, t.list, t.idx, ck,
                 dt, adj_x, adj_v, adj_u, adj_dp, adj_dE, s);
    c->last = s;
    return launched(c, "step_adjoint_taped");
}

// ------------------------------------------------------------ hierarchical steps
static mfm_status do_fluxes_levels(mfm_ctx* c, mfm_particles* p, const long long* bins, int lmin, int nlev,
                                   const long long* home, hipStream_t s) {
    if (!c->have_grad || c->n_tree != p->n) return fail(c, MFM_E_STATE, "mfm_gradients must run first");
    PassArrays a = arrays_of(p);
    launch_fluxes_levels(a, c->ph, c->counts, c->list, c->rec, c->cnt, bins, lmin, nlev, c->lev, home, s);
    c->have_flux = 1;
    c->last = s;
    return launched(c, "hydro_fluxes (levels)");
}

// Largest path length since the last build, in finest cells, up to which a
// partial boundary of a hierarchical step keeps the cell tables.
constexpr double kSkinCells = 0.5;

// A sub-step boundary's pass with active subsets (reading R26): kernel
// lengths and gradients of the due particles only, the others keeping theirs.
static mfm_status do_pass_active(mfm_ctx* c, mfm_particles* q, const long long* bins, int lmin, int nlev,
                                 hipStream_t s) {
    const long long n = q->n;
    PassArrays a = arrays_of(q);
    launch_hier_modes((int)n, q->x, q->y, q->z, q->H, bins, lmin, c->td, c->tab_len, c->hmarks, c->hmode,
                      c->gcount, c->counts, s);
    launch_solve_h_active(a, c->td, c->tab, c->pos, c->ph, c->cnt, c->hmode, c->hmoved + n, c->rl, c->list,
                          c->gcount, c->counts, c->fb_list, c->fb_count, c->fb2_list, c->fb2_count, s);
    launch_gradients_active(a, c->ph, c->hmode, c->hhome, c->gcount, c->counts, c->list, c->tails, c->prim, c->rec,
                            c->cnt, s);
    c->have_h = c->have_grad = 1;
    c->rec_mixed = 0;
    c->last = s;
    if (mfm_status st = launched(c, "hydro_pass (active subsets)")) return st;
    mfm_status st = do_fluxes_levels(c, q, bins, lmin, nlev, c->hhome, s);
    // the lists and packed records now hold the due subset only: no later
    // call may take them for those of a whole pass
    c->have_h = c->have_grad = c->have_flux = 0;
    return st;
}

// The one host synchronisation of a hierarchical step: whether every bin lies in
// 0 .. max_bin and whether the last gradient pass on the context ran on these
// particles as they stand (same order, positions and kernel lengths, bit for
// bit, checked on the device against its packed neighbour records; then the
// kernel lengths, densities, volumes and gather lists of that pass hold for
// them).
struct HierChecks {
    bool bins_ok, unmoved;
};
static mfm_status hier_checks(mfm_ctx* c, const mfm_particles* p, const long long* bins, int max_bin,
                              hipStream_t s, HierChecks* out) {
    const bool can_reuse = c->have_grad && c->n_tree == p->n;
    launch_fill_u64(1, c->fb_count, 0ull, s);
    launch_check_bins((int)p->n, bins, max_bin, c->fb_count, s);
    if (can_reuse) launch_same_positions((int)p->n, p->x, p->y, p->z, p->H, c->prim, c->fb_count, s);
    unsigned long long flags = 0;
    mfm_status st = hip_check(c, hipMemcpyAsync(&flags, c->fb_count, sizeof flags, hipMemcpyDeviceToHost, s),
                              "hierarchical step checks");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "hierarchical step checks");
    if (st) return st;
    out->bins_ok = !(flags & 1ull);
    out->unmoved = can_reuse && !(flags & 2ull);
    return MFM_OK;
}

extern "C" mfm_status mfm_step_hier(mfm_ctx* c, mfm_particles* p, int64_t* bins, int32_t max_bin, double T,
                                    int32_t flags, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    if (c->p.scheme != MFM_SCHEME_MFM || c->p.precision != MFM_FP64)
        return fail(c, MFM_E_INVALID, "hierarchical steps cover the MFM scheme in FP64");
    if (!bins) return fail(c, MFM_E_INVALID, "bins is required");
    if (max_bin < 0 || max_bin > kMaxBin) return fail(c, MFM_E_INVALID, "max_bin must lie in 0 .. 7");
    if (!(T > 0.0) || !isfinite(T)) return fail(c, MFM_E_INVALID, "T must be positive and finite");
    if (!p->dp || !p->dE || !p->vsig || !p->nk || !p->V || !p->B || !p->rho || !p->P || !p->grad)
        return fail(c, MFM_E_INVALID, "hierarchical steps need every pass output array");
    if (flags & ~(MFM_HIER_REBIN | MFM_HIER_ACTIVE)) return fail(c, MFM_E_INVALID, "unknown hierarchical step flag");
    const bool rebin = flags & MFM_HIER_REBIN, active = flags & MFM_HIER_ACTIVE;
    (void)hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    const long long n = p->n;
    if (!c->lev && (st = hip_check(c, hipMalloc((void**)&c->lev, sizeof(double) * 4 * (kMaxBin + 1) * c->cap),
                                   "level rates")))
        return st;
    if (active && !c->hmode) {
        if ((st = hip_check(c, hipMalloc((void**)&c->hmode, c->cap), "sub-step modes"))) return st;
        if ((st = hip_check(c, hipMalloc((void**)&c->hmarks, 8 * ((c->tab_len + 63) / 64)), "cell marks")))
            return st;
        if ((st = hip_check(c, hipMalloc((void**)&c->hmoved, sizeof(double) * (c->cap + 1)), "moved distances")))
            return st;
    }
    if (!c->hhome && (st = hip_check(c, hipMalloc((void**)&c->hhome, sizeof(long long) * c->cap), "home columns")))
        return st;
    const int nlev = max_bin + 1;
    long long* b = (long long*)bins;
    HierChecks chk;
    if ((st = hier_checks(c, p, b, max_bin, s, &chk))) return st;
    if (!chk.bins_ok) return fail(c, MFM_E_INVALID, "bins outside 0 .. max_bin");
    reset_counters(c, s);
    if (rebin || !c->have_levels || c->lev_nlev != nlev || c->n_tree != p->n) {
        // the per-level rates of the current state, every level due; when the
        // particles have not moved since the last pass (as after a hierarchical
        // step, whose last boundary passes over every particle), that pass's
        // kernel lengths, densities, volumes and gather lists still hold, and
        // only the gradients and the fluxes are evaluated again
        if (chk.unmoved) {
            launch_reset_counts((int)n, c->gcount, c->counts, s);
        } else {
            double* e1[1] = {(double*)b};
            if ((st = build(c, p, s, e1, 1))) return st;
            if ((st = do_solve_h(c, p, s))) return st;
        }
        if ((st = do_gradients(c, p, s))) return st;
        if ((st = do_fluxes_levels(c, p, b, 0, nlev, nullptr, s))) return st;
    } else if (!c->have_flux) {
        return fail(c, MFM_E_STATE, "hierarchical steps continue from a hierarchical step on this state");
    }
    const int K = 1 << max_bin;
    const double delta = T / (double)K;
    launch_hier_begin((int)n, p->m, p->vx, p->vy, p->vz, p->u, c->Ehalf, c->lev, nlev, T, s);
    // Within the system step a particle's per-level rates (and, with active
    // subsets, its kept gradient matrix and limited gradients) stay in the column
    // where it stood at the start, home[i]; each sub-step's reorder carries the
    // particle state, E, the bins and home (with active subsets also the kept n
    // and V), but not the pass outputs and u, which are written anew, nor the
    // predicted state, which is predicted after the reorder.
    //
    // With active subsets a boundary with lmin > 0 keeps the cell tables and
    // the particle order of the last build, as long as no particle has moved
    // more than kSkinCells of the finest cell since (one synchronised read per
    // such boundary): the particles drift without being wrapped into the box,
    // their packed positions are refreshed, and every scan reaches further by
    // the largest path length since that build (moved[n]).  The boundaries with
    // every level due build anew.
    launch_iota((int)n, c->hhome, s);
    if (active) launch_fill_u64(n + 1, (unsigned long long*)c->hmoved, 0ull, s);
    mfm_particles pb = *p;
    pb.dp = pb.dE = pb.vsig = pb.u = pb.dm = nullptr;
    for (int k = 1; k <= K; k++) {
        const int tz = __builtin_ctz((unsigned)k);
        const int lmin = max_bin - tz > 0 ? max_bin - tz : 0;
        bool rebuild = !(active && lmin > 0);
        launch_hier_drift(arrays_of(p), c->ph, delta, rebuild ? 1 : 0, rebuild ? nullptr : c->hmoved, s);
        if (!rebuild) {
            // keep the tables while no particle has moved half of the finest
            // cell since the build (the scans reach that much further); else
            // wrap the positions and build anew
            double moved = 0.0;
            if ((st = hip_check(c, hipMemcpyAsync(&moved, c->hmoved + n, sizeof moved, hipMemcpyDeviceToHost, s),
                                "moved distance")))
                return st;
            if ((st = hip_check(c, hipStreamSynchronize(s), "moved distance"))) return st;
            const double finest = std::min(c->td.cs[c->td.bmax][0], std::min(c->td.cs[c->td.bmax][1],
                                                                               c->td.cs[c->td.bmax][2]));
            if (!(moved <= kSkinCells * finest)) {
                rebuild = true;
                launch_hier_drift(arrays_of(p), c->ph, 0.0, 1, nullptr, s);   // wraps only
            }
        }
        if (rebuild) {
            double* extra[5] = {c->Ehalf, (double*)b, (double*)c->hhome, p->nk, p->V};
            if ((st = build(c, &pb, s, extra, active ? 5 : 3))) return st;
            if (active) launch_fill_u64(n + 1, (unsigned long long*)c->hmoved, 0ull, s);
        } else {
            launch_pos4((int)n, p->x, p->y, p->z, c->pos, s);
        }
        launch_hier_predict((int)n, p->m, p->vx, p->vy, p->vz, c->Ehalf, c->lev, c->hhome, lmin, nlev, T,
                            c->p.u_floor, c->vp, c->up, s);
        // the last boundary rewrites every level, in the current order
        if (lmin == 0) launch_iota((int)n, c->hhome, s);
        mfm_particles q = *p;
        q.vx = c->vp;
        q.vy = c->vp + n;
        q.vz = c->vp + 2 * n;
        q.u = c->up;
        if (active && lmin > 0) {
            if ((st = do_pass_active(c, &q, b, lmin, nlev, s))) return st;
        } else {
            if ((st = do_solve_h(c, &q, s))) return st;
            if ((st = do_gradients(c, &q, s))) return st;
            if ((st = do_fluxes_levels(c, &q, b, lmin, nlev, c->hhome, s))) return st;
        }
        launch_hier_kick((int)n, p->m, p->vx, p->vy, p->vz, c->Ehalf, c->lev, c->hhome, lmin, nlev, T,
                         k < K ? 2 : 1, s);
    }
    launch_hier_finish((int)n, p->m, p->vx, p->vy, p->vz, c->Ehalf, c->p.u_floor, p->u, c->cnt, s);
    c->have_levels = 1;
    c->lev_nlev = nlev;
    c->last = s;
    return launched(c, "step_hier");
}

// The neighbour time-step limiter on the last pass's flux lists, in sweeps
// until no bin changes (one synchronisation each; a bin rises at most max_bin
// times, so at most max_bin + 1 sweeps).
extern "C" mfm_status mfm_limit_bins(mfm_ctx* c, const mfm_particles* p, int64_t* bins, int32_t max_bin,
                                     int64_t* raised, void* stream) {
    mfm_status st = check_particles(c, p);
    if (st) return st;
    if (!bins) return fail(c, MFM_E_INVALID, "bins is required");
    if (max_bin < 0 || max_bin > kMaxBin) return fail(c, MFM_E_INVALID, "max_bin must lie in 0 .. 7");
    if (!c->have_grad || c->n_tree != p->n)
        return fail(c, MFM_E_STATE, "no flux lists of these particles (a pass must run first)");
    (void)hipSetDevice(c->device);
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)p->n;
    long long* next = (long long*)c->ktmp;
    unsigned long long word = 0, total = 0;
    launch_fill_u64(1, c->fb_count, 0ull, s);
    launch_check_bins(n, (const long long*)bins, max_bin, c->fb_count, s);
    for (int sweep = 0; sweep <= max_bin + 1; sweep++) {
        if ((st = hip_check(c, hipMemcpyAsync(&word, c->fb_count, sizeof word, hipMemcpyDeviceToHost, s),
                            "limiter count")))
            return st;
        if ((st = hip_check(c, hipStreamSynchronize(s), "limiter count"))) return st;
        if (sweep == 0) {
            if (word & 1ull) return fail(c, MFM_E_INVALID, "a bin lies outside 0 .. max_bin");
        } else {
            total += word;
            if (word == 0) break;
        }
        launch_fill_u64(1, c->fb_count, 0ull, s);
        launch_limit_bins(n, c->ph.max_ngb, c->counts, c->list, (const long long*)bins, next, c->fb_count, s);
        if ((st = hip_check(c, hipMemcpyAsync(bins, next, sizeof(long long) * n, hipMemcpyDeviceToDevice, s),
                            "limited bins")))
            return st;
    }
    if (raised) *raised = (int64_t)total;
    c->last = s;
    return launched(c, "limit_bins");
}

extern "C" mfm_status mfm_copy_levels(mfm_ctx* c, double* out, void* stream) {
    if (!c || !out) return MFM_E_INVALID;
    if (!c->have_levels || !c->lev) return fail(c, MFM_E_STATE, "no per-level rates (run mfm_step_hier first)");
    (void)hipSetDevice(c->device);
    const long long n = c->n_tree;
    return hip_check(c, hipMemcpyAsync(out, c->lev, sizeof(double) * 4 * c->lev_nlev * n, hipMemcpyDeviceToDevice,
                                       (hipStream_t)stream),
                     "copy levels");
}

// ------------------------------------------------- whole pass without allocation
// mfm_hydro_pass_noalloc runs mfm_build_neighbours + mfm_hydro_pass for up to
// kNoAllocMaxN particles with every scratch buffer carved from `scratch`, a
// file-scope device array that each GPU holds from the library's load until
// the process ends.  Host code reaches that array only through the address
// hipGetSymbolAddress returns for it on each device (kept in g_noalloc_ptr).
namespace {

constexpr long long kNoAllocMaxN = 8192;   // particles per call
constexpr int kNoAllocMaxNgb = 256;        // flux-list slots per particle
constexpr int kNoAllocLevels = 6;          // deepest cell-table level
constexpr int kNoAllocDevices = 64;
// cells of levels 0..kNoAllocLevels of the implicit octree when every axis refines at every level
constexpr long long kNoAllocTab = ((1ll << (3 * (kNoAllocLevels + 1))) - 1) / 7;
constexpr long long kNoAllocScanInts = kNoAllocMaxN + 1024;   // bound on scan_tmp_ints(max(hist, n))

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// every scratch buffer of one pass, in carving order (bytes)
constexpr long long N_ = kNoAllocMaxN;
constexpr size_t kNoAllocSizes[] = {
    8 * N_,                                   // keys
    8 * N_,                                   // ktmp
    4 * N_,                                   // idx
    4 * N_,                                   // vtmp
    4 * 256 * ((N_ + 2047) / 2048),           // hist
    4 * kNoAllocScanInts,                     // scan_tmp
    8 * N_ * kGatherMax,                      // gtmp
    8 * kNoAllocTab,                          // tab
    32 * N_,                                  // pos
    8 * N_ * kRCap,                           // rl
    4 * N_,                                   // counts
    4 * N_,                                   // gcount
    4 * N_ * kNoAllocMaxNgb,                  // list
    4 * N_,                                   // fb_list
    8,                                        // fb_count
    4 * N_,                                   // fb2_list
    8,                                        // fb2_count
    4 * (size_t)kTailBuf * N_,                // tails
    8 * 32 * N_,                              // rec
    32 * 4 * N_,                              // prim
    (size_t)kCounterCopies * kCounterStride,  // cnt
};
constexpr size_t noalloc_total() {
    size_t t = 0;
    for (size_t b : kNoAllocSizes) t += align256(b);
    return t;
}
constexpr size_t kNoAllocBytes = noalloc_total();   // about 27 MB
static_assert(kNoAllocBytes < (32u << 20), "the no-allocation scratch stays modest");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_noalloc_mutex;
void* g_noalloc_ptr[kNoAllocDevices];   // device address of `scratch` on each device
mfm_ctx g_noalloc_ctx[kNoAllocDevices]; // host-side context whose buffers point into it

// point every scratch buffer of c into the array at base
void noalloc_carve(mfm_ctx* c, unsigned char* base) {
    void** dst[] = {(void**)&c->keys, (void**)&c->ktmp, (void**)&c->idx, (void**)&c->vtmp, (void**)&c->hist,
                    (void**)&c->scan_tmp, (void**)&c->gtmp, (void**)&c->tab, (void**)&c->pos, (void**)&c->rl,
                    (void**)&c->counts, (void**)&c->gcount, (void**)&c->list, (void**)&c->fb_list,
                    (void**)&c->fb_count, (void**)&c->fb2_list, (void**)&c->fb2_count, (void**)&c->tails,
                    (void**)&c->rec, (void**)&c->prim, (void**)&c->cnt};
    static_assert(sizeof(dst) / sizeof(dst[0]) == sizeof(kNoAllocSizes) / sizeof(kNoAllocSizes[0]),
                  "one size per carved buffer");
    size_t off = 0;
    for (size_t k = 0; k < sizeof(kNoAllocSizes) / sizeof(kNoAllocSizes[0]); k++) {
        *dst[k] = base + off;
        off += align256(kNoAllocSizes[k]);
    }
}

}  // namespace

extern "C" mfm_status mfm_hydro_pass_noalloc(const mfm_params* params, mfm_particles* p, mfm_counters* counters,
                                             void* stream) {
    if (!params || !params_valid(*params)) return MFM_E_INVALID;
    if (params->max_ngb > kNoAllocMaxNgb || params->tree_levels > kNoAllocLevels) return MFM_E_INVALID;
    if (!p || p->n < 1) return MFM_E_INVALID;
    if (p->n > kNoAllocMaxN) return MFM_E_CAPACITY;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return MFM_E_HIP;
    mfm_ctx* c = &g_noalloc_ctx[dev];
    {
        // set-up, once per device with that device current: the device address of the array
        std::lock_guard<std::mutex> lock(g_noalloc_mutex);
        if (!g_noalloc_ptr[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MFM_E_HIP;
            g_noalloc_ptr[dev] = ptr;
        }
    }
    mfm_params q = *params;
    q.max_ngb = q.max_ngb > 0 ? q.max_ngb : kNoAllocMaxNgb;
    q.tree_levels = q.tree_levels > 0 ? q.tree_levels : kNoAllocLevels;
    c->cap = kNoAllocMaxN;
    c->device = dev;
    c->timing = 0;
    c->adj = nullptr;
    c->vp = c->up = c->Ehalf = c->mp = c->dt_part = c->dt_out = nullptr;
    init_params(c, q);
    if (c->tab_len > kNoAllocTab || scan_tmp_ints(std::max(256ll * ((p->n + 2047) / 2048), (long long)p->n)) >
                                        kNoAllocScanInts)
        return fail(c, MFM_E_CAPACITY, "cell tables or scan scratch exceed the no-allocation scratch");
    noalloc_carve(c, (unsigned char*)g_noalloc_ptr[dev]);
    c->tab_keys_n = -1;   // the shared array may hold another call's tables
    c->n_tree = -1;
    c->have_h = c->have_grad = c->have_flux = 0;
    c->err[0] = 0;
    mfm_status st = check_particles(c, p);
    if (st) return st;
    if (!p->nk || !p->V || !p->B || !p->rho || !p->P || !p->grad || !p->dp || !p->dE || !p->vsig)
        return fail(c, MFM_E_INVALID, "every pass output array is required");
    if (q.scheme == MFM_SCHEME_MFV && !p->dm) return fail(c, MFM_E_INVALID, "the finite-volume scheme needs dm");
    hipStream_t s = (hipStream_t)stream;
    if ((st = build(c, p, s, nullptr, 0))) return st;
    reset_counters(c, s);
    if ((st = do_solve_h(c, p, s))) return st;
    if ((st = do_gradients(c, p, s))) return st;
    if ((st = do_fluxes(c, p, s))) return st;
    if (!counters) return MFM_OK;
    if ((st = mfm_get_counters(c, counters))) return st;
    return status_of(c, *counters);
}

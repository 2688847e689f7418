// Host sanitizer driver for the library's argument, capacity and error
// handling (test infrastructure).  Linked against a build of libmfm whose host
// code carries AddressSanitizer and UndefinedBehaviorSanitizer (device code
// untouched) by tests/test_host_sanitizers.py.  Every call here must return
// before any kernel launch: particle structs hold null arrays or a count the
// checks refuse.  Without a GPU, mfm_create's first allocation fails and the
// error path (a partly built context destroyed) is what runs; with one, the
// context is created and the per-call checks run against it.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mfm.h"

static int failures = 0;

static void expect(const char* what, mfm_status got, mfm_status want) {
    const bool ok = got == want;
    printf("%-58s %-16s %s\n", what, mfm_status_str(got), ok ? "ok" : "UNEXPECTED");
    if (!ok) failures++;
}

static mfm_params valid_params() {
    mfm_params p;
    memset(&p, 0, sizeof p);
    p.gamma = 5.0 / 3.0;
    p.n_ngb = 32.0;
    p.cfl = 0.25;
    p.box[0] = p.box[1] = p.box[2] = 1.0;
    p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    p.beta = 1.0;
    p.cond_max = 1e6;
    return p;
}

int main() {
    for (int s = 1; s >= -9; s--) printf("status %d: %s\n", s, mfm_status_str((mfm_status)s));
    printf("last error of a null context: %s\n", mfm_last_error(nullptr));
    mfm_destroy(nullptr);

    mfm_ctx* ctx = nullptr;
    mfm_params p = valid_params();
    expect("create: null out", mfm_create(&p, 16, nullptr), MFM_E_INVALID);
    expect("create: null params", mfm_create(nullptr, 16, &ctx), MFM_E_INVALID);
    struct Bad {
        const char* what;
        void (*spoil)(mfm_params&);
    } bad[] = {
        {"create: gamma = 1", [](mfm_params& q) { q.gamma = 1.0; }},
        {"create: gamma NaN", [](mfm_params& q) { q.gamma = NAN; }},
        {"create: n_ngb below the self count", [](mfm_params& q) { q.n_ngb = 10.0; }},
        {"create: box side 0", [](mfm_params& q) { q.box[1] = 0.0; }},
        {"create: beta 0", [](mfm_params& q) { q.beta = 0.0; }},
        {"create: precision 7", [](mfm_params& q) { q.precision = 7; }},
        {"create: scheme 5", [](mfm_params& q) { q.scheme = 5; }},
        {"create: limiter 3", [](mfm_params& q) { q.limiter = 3; }},
        {"create: limiter with cond_hi <= cond_lo", [](mfm_params& q) {
             q.limiter = 1;
             q.beta_min = 0.5;
             q.cond_lo = 10.0;
             q.cond_hi = 10.0;
         }},
    };
    for (auto& b : bad) {
        mfm_params q = valid_params();
        b.spoil(q);
        ctx = reinterpret_cast<mfm_ctx*>(0x1);
        expect(b.what, mfm_create(&q, 16, &ctx), MFM_E_INVALID);
        if (ctx != nullptr) {
            printf("create left a non-null context on failure\n");
            failures++;
        }
    }
    expect("create: capacity 0", mfm_create(&p, 0, &ctx), MFM_E_INVALID);
    expect("create: capacity 2^31", mfm_create(&p, (int64_t)1 << 31, &ctx), MFM_E_INVALID);

    mfm_particles none;
    memset(&none, 0, sizeof none);
    mfm_counters cnt;
    expect("build_neighbours: null context", mfm_build_neighbours(nullptr, &none, nullptr), MFM_E_INVALID);
    expect("solve_h: null context", mfm_solve_h(nullptr, &none, nullptr), MFM_E_INVALID);
    expect("unpermute: null context", mfm_unpermute(nullptr, &none, nullptr), MFM_E_INVALID);
    expect("limit_bins: null context", mfm_limit_bins(nullptr, &none, nullptr, 3, nullptr, nullptr), MFM_E_INVALID);
    expect("hydro_pass: null context", mfm_hydro_pass(nullptr, &none, nullptr), MFM_E_INVALID);
    expect("get_counters: null context", mfm_get_counters(nullptr, &cnt), MFM_E_INVALID);
    if (mfm_tape_bytes(nullptr) != -1) {
        printf("tape_bytes of a null context is not -1\n");
        failures++;
    }
    expect("step_taped: null context", mfm_step_taped(nullptr, &none, 1e-3, nullptr, nullptr), MFM_E_INVALID);
    expect("step_adjoint_taped: null context",
           mfm_step_adjoint_taped(nullptr, &none, nullptr, 1e-3, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr),
           MFM_E_INVALID);
    expect("noalloc: null params", mfm_hydro_pass_noalloc(nullptr, &none, nullptr, nullptr), MFM_E_INVALID);
    mfm_params q = valid_params();
    q.gamma = 0.5;
    expect("noalloc: bad params", mfm_hydro_pass_noalloc(&q, &none, nullptr, nullptr), MFM_E_INVALID);
    expect("noalloc: n = 0", mfm_hydro_pass_noalloc(&p, &none, nullptr, nullptr), MFM_E_INVALID);
    none.n = 1 << 20;
    expect("noalloc: n past its limit", mfm_hydro_pass_noalloc(&p, &none, nullptr, nullptr), MFM_E_CAPACITY);
    none.n = 0;

    const mfm_status st = mfm_create(&p, 1000, &ctx);
    printf("create with valid parameters: %s\n", mfm_status_str(st));
    if (st == MFM_OK) {
        expect("build_neighbours: null particles", mfm_build_neighbours(ctx, nullptr, nullptr), MFM_E_INVALID);
        expect("build_neighbours: n = 0", mfm_build_neighbours(ctx, &none, nullptr), MFM_E_INVALID);
        none.n = 1001;
        expect("build_neighbours: n past capacity", mfm_build_neighbours(ctx, &none, nullptr), MFM_E_CAPACITY);
        none.n = 10;
        expect("build_neighbours: null arrays", mfm_build_neighbours(ctx, &none, nullptr), MFM_E_INVALID);
        expect("solve_h: null arrays", mfm_solve_h(ctx, &none, nullptr), MFM_E_INVALID);
        expect("unpermute: null arrays", mfm_unpermute(ctx, &none, nullptr), MFM_E_INVALID);
        expect("limit_bins: null arrays", mfm_limit_bins(ctx, &none, nullptr, 3, nullptr, nullptr), MFM_E_INVALID);
        {
            // every required array set (never read: the call stops at the missing id)
            double dummy[10] = {0};
            mfm_particles q = none;
            q.x = q.y = q.z = q.m = q.vx = q.vy = q.vz = q.u = q.H = dummy;
            q.id = nullptr;
            expect("unpermute: null id", mfm_unpermute(ctx, &q, nullptr), MFM_E_INVALID);
        }
        expect("step: null arrays", mfm_step(ctx, &none, 1e-3, nullptr, nullptr), MFM_E_INVALID);
        int64_t bins[1] = {0};
        expect("step_hier: null arrays", mfm_step_hier(ctx, &none, bins, 1, 1e-3, 1, nullptr), MFM_E_INVALID);
        expect("step_taped: null tape", mfm_step_taped(ctx, &none, 1e-3, nullptr, nullptr), MFM_E_INVALID);
        expect("step_taped: dt <= 0", mfm_step_taped(ctx, &none, 0.0, bins, nullptr), MFM_E_INVALID);
        printf("last error: %s\n", mfm_last_error(ctx));
        mfm_destroy(ctx);
    } else if (st != MFM_E_HIP) {
        printf("create with valid parameters gave neither OK nor a HIP error\n");
        failures++;
    }
    printf("%d unexpected results\n", failures);
    return failures ? 1 : 0;
}

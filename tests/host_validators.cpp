// Host-side checks of the C ABI's pure-host validators, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code only
// (tests/test_host_sanitizers.py).  No GPU is touched: only the validators,
// the workspace sizing, the checkpoint plan and the status strings run, on
// good, bad and extreme arguments.  Exit status 0 = every status as expected.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <limits>
#include <vector>

#include "ptyr.h"

static int failures = 0;

static void expect(const char* what, int got, int want) {
    if (got != want) {
        printf("FAIL %s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

static ptyr_geom base() {
    ptyr_geom g;
    memset(&g, 0, sizeof g);
    g.N = 128; g.M = 6; g.S = 12; g.H = 640; g.W = 640; g.B_max = 64;
    g.dx = 0.15; g.lambda = 0.0197; g.loss_kind = PTYR_LOSS_GAUSSIAN; g.loss_p = 0.5;
    g.wave_budget_bytes = (size_t)64 * 6 * 24 * 128 * 128 * 8;
    g.n_scan = 16384;
    return g;
}

int main() {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    ptyr_geom g = base();
    expect("base", ptyr_check_geom(&g), PTYR_OK);
    expect("null geometry", ptyr_check_geom(nullptr), PTYR_E_ARG);
    if (ptyr_workspace_bytes(&g) == 0) { printf("FAIL workspace of the base geometry is 0\n"); ++failures; }

    struct Case { const char* name; void (*edit)(ptyr_geom&); int want; };
    const Case cases[] = {
        {"N=64", [](ptyr_geom& x) { x.N = 64; }, PTYR_OK},
        {"N=96", [](ptyr_geom& x) { x.N = 96; }, PTYR_E_ARG},
        {"N=-128", [](ptyr_geom& x) { x.N = -128; }, PTYR_E_ARG},
        {"M=0", [](ptyr_geom& x) { x.M = 0; }, PTYR_E_ARG},
        {"M=INT_MAX", [](ptyr_geom& x) { x.M = 2147483647; }, PTYR_E_ARG},
        {"B_max*M huge", [](ptyr_geom& x) { x.B_max = 1 << 20; x.M = 1 << 12; }, PTYR_E_ARG},
        {"n_obj=64, M*B at the limit", [](ptyr_geom& x) { x.n_obj = 64; x.B_max = 1024; x.M = 16; }, PTYR_OK},
        {"n_obj=65", [](ptyr_geom& x) { x.n_obj = 65; }, PTYR_E_ARG},
        {"S=0", [](ptyr_geom& x) { x.S = 0; }, PTYR_E_ARG},
        {"H<N", [](ptyr_geom& x) { x.H = 127; }, PTYR_E_ARG},
        {"H, W = INT_MAX", [](ptyr_geom& x) { x.H = x.W = 2147483647; }, PTYR_E_ARG},
        {"object of 2^40 elements", [](ptyr_geom& x) { x.S = 16; x.H = x.W = 1 << 18; }, PTYR_OK},
        {"object above 2^40 elements", [](ptyr_geom& x) { x.S = 17; x.H = x.W = 1 << 18; }, PTYR_E_ARG},
        {"dx NaN", [](ptyr_geom& x) { x.dx = std::numeric_limits<double>::quiet_NaN(); }, PTYR_E_ARG},
        {"lambda -inf", [](ptyr_geom& x) { x.lambda = -std::numeric_limits<double>::infinity(); }, PTYR_E_ARG},
        {"loss kind 2", [](ptyr_geom& x) { x.loss_kind = 2; }, PTYR_E_ARG},
        {"loss p inf", [](ptyr_geom& x) { x.loss_p = std::numeric_limits<double>::infinity(); }, PTYR_E_ARG},
        {"unknown flag", [](ptyr_geom& x) { x.flags = 0x100u; }, PTYR_E_ARG},
        {"n_scan < 0", [](ptyr_geom& x) { x.n_scan = -1; }, PTYR_E_ARG},
        {"sparse_w NaN", [](ptyr_geom& x) { x.sparse_w = std::numeric_limits<double>::quiet_NaN(); }, PTYR_E_ARG},
        {"pacbed_w < 0", [](ptyr_geom& x) { x.pacbed_w = -1.0; }, PTYR_E_ARG},
        {"Eq. 9 weights", [](ptyr_geom& x) { x.w_gaussian = 0.5; x.w_poisson = 2.0; }, PTYR_OK},
        {"w_poisson inf", [](ptyr_geom& x) { x.w_poisson = std::numeric_limits<double>::infinity(); }, PTYR_E_ARG},
        {"p_gaussian < 0", [](ptyr_geom& x) { x.p_gaussian = -0.5; }, PTYR_E_ARG},
        {"N=256 all waves", [](ptyr_geom& x) { x.N = 256; x.H = x.W = 1024; x.B_max = 16; x.M = 8; x.S = 30;
                                               x.wave_budget_bytes = (size_t)16 * 8 * 60 * 256 * 256 * 8; }, PTYR_OK},
        {"N=256 small budget", [](ptyr_geom& x) { x.N = 256; x.H = x.W = 1024; x.wave_budget_bytes = 0; },
         PTYR_E_ARG},
    };
    for (const Case& c : cases) {
        ptyr_geom x = base();
        c.edit(x);
        expect(c.name, ptyr_check_geom(&x), c.want);
        const size_t ws = ptyr_workspace_bytes(&x);
        if ((c.want == PTYR_OK) != (ws > 0)) {
            printf("FAIL %s: workspace %zu\n", c.name, ws);
            ++failures;
        }
        int stride = -1;
        expect(c.name, ptyr_checkpoint_plan(&x, &stride), c.want);
        if (c.want == PTYR_OK && (stride < 1 || stride > x.S + 1)) {
            printf("FAIL %s: stride %d\n", c.name, stride);
            ++failures;
        }
    }
    // the checkpoint plan over every budget from nothing to all waves
    for (size_t waves = 0; waves <= 2 * 12 + 1; ++waves) {
        ptyr_geom x = base();
        x.wave_budget_bytes = waves * (size_t)64 * 6 * 128 * 128 * 8;
        int stride = 0;
        expect("budget", ptyr_checkpoint_plan(&x, &stride), PTYR_OK);
        const int want1 = waves >= 24;
        if ((stride == 1) != want1) { printf("FAIL budget %zu waves: stride %d\n", waves, stride); ++failures; }
    }
    expect("plan null stride", ptyr_checkpoint_plan(&g, nullptr), PTYR_E_ARG);

    // positions: inside, on the edges, outside, non-finite, huge
    ptyr_geom p = base();
    p.N = 64; p.H = p.W = 128; p.B_max = 4;
    const float ok[] = {64.f, 64.f, 32.f, 96.f, 32.f, 32.f, 96.f, 96.f};
    expect("positions inside", ptyr_check_args(&p, 4, ok), PTYR_OK);
    expect("B = 0", ptyr_check_args(&p, 0, ok), PTYR_E_ARG);
    expect("B > B_max", ptyr_check_args(&p, 5, nullptr), PTYR_E_ARG);
    expect("B < 0", ptyr_check_args(&p, -3, nullptr), PTYR_E_ARG);
    const float bad[][2] = {{31.4f, 64.f}, {64.f, 96.6f}, {NAN, 64.f}, {64.f, INFINITY}, {1e30f, 64.f},
                            {-1e30f, 64.f}, {64.f, -2147483648.f}};
    for (const auto& b : bad) expect("position outside", ptyr_check_args(&p, 1, b), PTYR_E_BOUNDS);
    const float tie[] = {32.5f, 95.5f};     // half to even: 32 and 96 -> corners 0 and 64
    expect("rounding ties", ptyr_check_args(&p, 1, tie), PTYR_OK);
    std::vector<float> many(2 * 4, 64.f);
    expect("vector positions", ptyr_check_args(&p, 4, many.data()), PTYR_OK);

    for (int s = 0; s <= 7; ++s)          // every value the enum can hold, unknown ones included
        if (!ptyr_status_str((ptyr_status)s)) { printf("FAIL status string %d\n", s); ++failures; }
    (void)nan;
    (void)inf;
    if (failures) return 1;
    printf("OK\n");
    return 0;
}

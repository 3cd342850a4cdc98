// Host-only driver for the sanitizer build (test infrastructure): builds
// seeded pseudo-random circuits through the C ABI and asks for the planned
// and generated passes of every one of them at several tile shapes, so that
// AddressSanitizer and UndefinedBehaviorSanitizer watch the planner, the op
// merger, the deferred-factor algebra and the source generator.  Needs no
// GPU (nothing is launched).  Exit status 0 when every call succeeds.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "qstate.h"

namespace {

uint64_t g_state = 0x243f6a8885a308d3ull;
double urand()
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}
int irand(int n) { return (int)(urand() * n) % n; }

// a random 2x2 unitary e^{i a} [[cos t e^{i b}, sin t e^{i c}], [-sin t e^{-i c}, cos t e^{-i b}]]
void unitary(qs_cplx u[4])
{
    const double a = 6.283 * urand(), b = 6.283 * urand(), c = 6.283 * urand(), t = 1.5707 * urand();
    const double ct = cos(t), st = sin(t);
    auto e = [](double x, double m) { return qs_cplx{m * cos(x), m * sin(x)}; };
    u[0] = e(a + b, ct);
    u[1] = e(a + c, st);
    u[2] = e(a - c + M_PI, st);
    u[3] = e(a - b, ct);
}

int fail(const char* what)
{
    fprintf(stderr, "%s failed: %s\n", what, qs_last_error());
    return 1;
}

int add_random_ops(qs_circuit c, int n, int count, bool channels)
{
    for (int i = 0; i < count; ++i) {
        const int kind = irand(channels ? 5 : 4);
        int qs[4];
        const int k = irand(4);
        for (int j = 0; j <= k; ++j) {
            bool again;
            do {
                qs[j] = irand(n);
                again = false;
                for (int m = 0; m < j; ++m) again = again || qs[m] == qs[j];
            } while (again);
        }
        qs_status s = QS_OK;
        if (kind <= 1) {
            qs_cplx u[4];
            unitary(u);
            s = qs_circuit_add_unitary(c, qs, k, qs[k], u);
        } else if (kind == 2) {
            s = qs_circuit_add_not(c, qs, k, qs[k]);
        } else if (kind == 3) {
            s = qs_circuit_add_phase(c, qs, k + 1, 6.283 * urand());
        } else {
            s = qs_circuit_add_channel(c, irand(3), qs[0], 0.01 * urand());
        }
        if (s) return fail("add op");
    }
    return 0;
}

int add_layered(qs_circuit c, int n, int depth)
{
    for (int l = 0; l < depth; ++l) {
        for (int q = 0; q < n; ++q) {
            qs_cplx u[4];
            unitary(u);
            if (qs_circuit_add_unitary(c, nullptr, 0, q, u)) return fail("add unitary");
        }
        for (int q = l % 2; q + 1 < n; q += 2)
            if (qs_circuit_add_not(c, &q, 1, q + 1)) return fail("add not");
        int p[4] = {irand(n), -1, -1, -1};
        for (int j = 1; j < 4; ++j) {
            bool again;
            do {
                p[j] = irand(n);
                again = false;
                for (int m = 0; m < j; ++m) again = again || p[m] == p[j];
            } while (again);
        }
        if (qs_circuit_add_phase(c, p, 4, 6.283 * urand())) return fail("add phase");
    }
    return 0;
}

// every pass's source and kernel data
int generate_all(qs_circuit c, int n, int kind, int prec, int K, int TB, int L)
{
    int npass = 0;
    size_t len = 0;
    if (qs_circuit_source(c, n, kind, prec, K, TB, 0, L, 0, nullptr, 0, &len, &npass)) return fail("source");
    for (int p = 0; p < npass; ++p) {
        std::vector<char> src;
        if (qs_circuit_source(c, n, kind, prec, K, TB, 0, L, p, nullptr, 0, &len, nullptr)) return fail("source len");
        src.resize(len + 1);
        if (qs_circuit_source(c, n, kind, prec, K, TB, 0, L, p, src.data(), src.size(), &len, nullptr))
            return fail("source text");
        size_t m = 0;
        if (qs_circuit_pass_data(c, n, kind, prec, K, TB, 0, L, p, nullptr, 0, &m, nullptr)) return fail("data len");
        std::vector<double> d(m + 1);
        if (qs_circuit_pass_data(c, n, kind, prec, K, TB, 0, L, p, d.data(), m, &m, nullptr)) return fail("data");
    }
    printf("n=%d kind=%d prec=%d tile=(%d,%d,%d): %d passes\n", n, kind, prec, K, TB, L, npass);
    return 0;
}

}  // namespace

int main()
{
    struct Shape {
        int K, TB, L;
    };
    const Shape sv_shapes[] = {{12, 8, 4}, {11, 8, 4}};
    for (int trial = 0; trial < 2; ++trial) {
        qs_circuit c = nullptr;
        if (qs_circuit_create(&c)) return fail("create");
        const int n = 16 + 3 * trial;
        if (add_layered(c, n, 3)) return 1;
        if (add_random_ops(c, n, 40, false)) return 1;
        const Shape& s = sv_shapes[trial];
        if (generate_all(c, n, QS_STATEVEC, trial == 0 ? QS_C128 : QS_C64, s.K, s.TB, s.L)) return 1;
        qs_circuit_destroy(c);
    }
    {
        qs_circuit c = nullptr;
        if (qs_circuit_create(&c)) return fail("create");
        const int N = 7;
        if (add_layered(c, N, 2)) return 1;
        if (add_random_ops(c, N, 30, true)) return 1;
        if (generate_all(c, N, QS_DENSITY, QS_C128, 12, 8, 4)) return 1;
        qs_circuit_destroy(c);
    }
    std::vector<double> draws(1000);
    if (qs_philox_draws(7, 3, 5, 1000, draws.data())) return fail("draws");
    printf("ok\n");
    return 0;
}

// Host-side checks of the C ABI built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code: every entry point that does
// no device work (grids, panel coefficients, footprint estimate, default
// options, version) with valid and invalid arguments, and the argument
// checks of the device entry points that refuse before touching a device.
// Exits non-zero on the first wrong result; the sanitizers abort on the
// first memory or undefined-behaviour error.
#include "ite.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int fails = 0;
#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

int main() {
    CHECK(std::strstr(ite_version(), "gfx950") != nullptr);
    ite_step_opts o;
    ite_default_opts(&o);
    CHECK(o.krylov_dim == 10 && o.max_cycles == 1 && o.nsweeps == 1 && o.gl_nodes == 2);
    ite_default_opts(nullptr);

    // geometric grid: exact size query, then fill; refused parameters
    int n = 0;
    CHECK(ite_loggrid(0.01, 1000.0, 1.3, nullptr, 0, &n) == ITE_EINVAL && n == 46);
    std::vector<double> g(n);
    CHECK(ite_loggrid(0.01, 1000.0, 1.3, g.data(), n, &n) == ITE_OK && n == 46);
    CHECK(g[0] == 0.0 && g[1] == 0.01 && g[n - 1] == 1000.0);
    for (int k = 1; k < n; ++k) CHECK(g[k] > g[k - 1]);
    CHECK(ite_loggrid(0.0, 1.0, 1.5, g.data(), n, &n) == ITE_EINVAL);
    CHECK(ite_loggrid(1.0, 0.5, 1.5, g.data(), n, &n) == ITE_EINVAL);
    CHECK(ite_loggrid(0.1, 1.0, 1.0, g.data(), n, &n) == ITE_EINVAL);
    CHECK(ite_loggrid(NAN, 1.0, 2.0, g.data(), n, &n) == ITE_EINVAL);

    // panel grid: P n + 1 points, too small a buffer refused
    int np = 0;
    std::vector<double> pg(14 * 4 + 1);
    CHECK(ite_panel_grid(64.0, 14, 4, pg.data(), (int)pg.size(), &np) == ITE_OK && np == 57);
    CHECK(pg[0] == 0.0 && std::fabs(pg[np - 1] - 64.0) < 1e-12);
    CHECK(ite_panel_grid(64.0, 14, 4, pg.data(), 10, &np) != ITE_OK);
    CHECK(ite_panel_grid(-1.0, 14, 4, pg.data(), (int)pg.size(), &np) == ITE_EINVAL);

    // Gauss-Legendre coefficients: weights sum to 1, quadrature of t^k exact
    // up to degree 2p - 1, rows of A integrate 1 to c_i, r_inf = (-1)^p
    for (int p = 1; p <= 7; ++p) {
        std::vector<double> c(p), b(p), A((size_t)p * p), w(p);
        double r = 0.0;
        CHECK(ite_gl_coefficients(p, c.data(), b.data(), A.data(), w.data(), &r) == ITE_OK);
        for (int k = 0; k < 2 * p; ++k) {
            double q = 0.0;
            for (int i = 0; i < p; ++i) q += b[i] * std::pow(c[i], k);
            CHECK(std::fabs(q - 1.0 / (k + 1)) < 1e-14);
        }
        for (int i = 0; i < p; ++i) {
            double s = 0.0;
            for (int j = 0; j < p; ++j) s += A[(size_t)i * p + j];
            CHECK(std::fabs(s - c[i]) < 1e-13);
        }
        CHECK(std::fabs(r - (p % 2 ? -1.0 : 1.0)) < 1e-11);
    }
    {
        double buf[64], r = 0.0;
        CHECK(ite_gl_coefficients(0, buf, buf, buf, buf, &r) == ITE_EINVAL);
        CHECK(ite_gl_coefficients(8, buf, buf, buf, buf, &r) == ITE_EINVAL);
        CHECK(ite_gl_coefficients(2, nullptr, buf, buf, buf, &r) == ITE_EINVAL);
    }

    // admission footprint: grows with the bond dimension, refuses bad input
    {
        std::vector<int> d(64, 2), w(65, 5);
        w[0] = w[64] = 1;
        const double f256 = ite_request_footprint(64, d.data(), w.data(), 256, 10);
        const double f512 = ite_request_footprint(64, d.data(), w.data(), 512, 10);
        CHECK(f256 > 0.0 && f512 > f256);
        CHECK(ite_request_footprint(1, d.data(), w.data(), 256, 10) < 0.0);
        CHECK(ite_request_footprint(64, nullptr, w.data(), 256, 10) < 0.0);
    }

    // device entry points refuse NULL handles before any device work
    ite_step_report rep;
    CHECK(ite_imag_step(nullptr, nullptr, 0.1, &o, &rep) == ITE_EINVAL);
    CHECK(ite_measure_energy(nullptr, nullptr, nullptr) == ITE_EINVAL);
    CHECK(ite_mps_overlap(nullptr, nullptr, nullptr) == ITE_EINVAL);
    CHECK(ite_mps_norm(nullptr, nullptr) == ITE_EINVAL);
    CHECK(ite_mpo_apply(nullptr, nullptr, 8, 0.0, 0.0, nullptr, nullptr) == ITE_EINVAL);
    CHECK(ite_evolve_loggrid(nullptr, nullptr, 0.01, 1.0, 1.3, &o, nullptr, 0, nullptr) == ITE_EINVAL);
    CHECK(ite_ctx_create(0, nullptr, nullptr, nullptr) == ITE_EINVAL);
    CHECK(std::strlen(ite_last_error(nullptr)) > 0);

    if (fails) {
        std::fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    std::printf("host ABI checks passed\n");
    return 0;
}

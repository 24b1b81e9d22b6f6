// Host-only driver that runs every entry point of the CPU oracle on small
// seeded states under AddressSanitizer and UndefinedBehaviorSanitizer
// (built and run by tests/test_oracle_sanitizers.py): every boundary type
// on every side, both orders, the three fluxes, the friction laws, rain
// fields, a hyetograph and Green-Ampt, the forward-mode tangent and the
// gauge run.  Any out-of-bounds access, use of uninitialised heap memory
// found by the sanitizers, or undefined arithmetic aborts the run; the
// driver itself checks that every result is finite.
#include "../oracle/swe_oracle.cpp"

#include <cstdio>
#include <cstdlib>

namespace {

// 64-bit linear congruential generator (Knuth's MMIX constants)
struct Lcg {
    uint64_t s;
    double uniform() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) * (1.0 / 9007199254740992.0);
    }
};

int failures = 0;

void expect_finite(const char* what, const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) {
            std::printf("non-finite value in %s\n", what);
            ++failures;
            return;
        }
}

void one_case(int nx, int ny, const int bc[4], int order, int flux, int law, bool fields,
              uint64_t seed) {
    Lcg r{seed};
    const size_t n = (size_t)nx * ny;
    std::vector<double> h(n), qx(n), qy(n), z(n), fric(n), vinf(n, 0.0), w(n), ks(n), psi(n),
        dth(n);
    for (size_t s = 0; s < n; ++s) {
        z[s] = r.uniform() + 0.02 * (double)(s % nx);
        h[s] = r.uniform() < 0.3 ? 0.0 : 2.0 * r.uniform();
        qx[s] = h[s] > 0.0 ? h[s] * (4.0 * r.uniform() - 2.0) : 0.0;
        qy[s] = h[s] > 0.0 ? h[s] * (4.0 * r.uniform() - 2.0) : 0.0;
        fric[s] = 0.02 + 0.02 * r.uniform();
        w[s] = 0.5 + r.uniform();
        ks[s] = 1e-6 * (0.5 + r.uniform());
        psi[s] = 0.05 * (0.5 + r.uniform());
        dth[s] = 0.3 * (0.5 + r.uniform());
    }
    const double rain_t[3] = {0.0, 0.5, 1.5};
    const double rain_r[3] = {3e-5, 0.0, 1e-5};
    orc_params p;
    std::memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.dx = 0.8; p.dy = 1.3; p.g = 9.81;
    p.cfl = order == 1 ? 1.0 : 0.5; p.dt_max = 0.5; p.h_eps = 1e-12;
    for (int k = 0; k < 4; ++k) {
        p.bc[k] = bc[k];
        p.bc_h[k] = 0.3 + 0.4 * k;
        p.bc_q[k] = 0.2 * k;
    }
    p.fric_law = law; p.fric_coef = law == 2 ? 0.1 : 0.03;
    p.rain = 1e-5; p.infil_on = 1; p.ks = 1e-6; p.psi = 0.05; p.dtheta = 0.3;
    p.order = order; p.flux = flux;
    if (fields) {
        p.rain_n = 3; p.rain_t = rain_t; p.rain_r = rain_r; p.rain_w = w.data();
        p.ks_f = ks.data(); p.psi_f = psi.data(); p.dtheta_f = dth.data();
    }
    // single rate
    std::vector<double> ph(n), pqx(n), pqy(n);
    double amax[2];
    orc_rate(&p, h.data(), qx.data(), qy.data(), z.data(), ph.data(), pqx.data(), pqy.data(),
             amax);
    expect_finite("rate", ph);
    // a run with its dt log
    std::vector<double> h1 = h, qx1 = qx, qy1 = qy, dts(12, 0.0);
    double t = 0.0;
    int32_t done = 0;
    int rc = orc_run(&p, h1.data(), qx1.data(), qy1.data(), z.data(),
                     law ? fric.data() : nullptr, vinf.data(), &t, 2.0, 12, dts.data(), &done);
    if (rc < 0) {
        std::printf("orc_run failed rc=%d (%dx%d order %d flux %d)\n", rc, nx, ny, order, flux);
        ++failures;
    }
    expect_finite("run h", h1);
    expect_finite("run qx", qx1);
    // tangent and gauge runs on the second-order HLL scheme with friction
    if (order == 2 && flux == 0 && law != 0 && done > 0) {
        const int32_t gauges[3] = {0, (int32_t)(n / 2), (int32_t)(n - 1)};
        std::vector<double> obs((size_t)done * 3, 0.1), dfric(n, 1e-3);
        double loss = 0.0, dloss = 0.0;
        orc_tangent_run(&p, h.data(), qx.data(), qy.data(), z.data(), fric.data(),
                        dfric.data(), done, dts.data(), gauges, 3, 1, obs.data(), &loss,
                        &dloss);
        if (!std::isfinite(loss) || !std::isfinite(dloss)) {
            std::printf("tangent run not finite\n");
            ++failures;
        }
        std::vector<double> h2 = h, qx2 = qx, qy2 = qy, out((size_t)done * 3);
        orc_gauge_run(&p, h2.data(), qx2.data(), qy2.data(), z.data(), fric.data(), done,
                      dts.data(), gauges, 3, 1, out.data());
        expect_finite("gauges", out);
    }
}

}  // namespace

int main() {
    const int shapes[4][2] = {{2, 2}, {7, 5}, {3, 9}, {37, 29}};
    const int mixes[5][4] = {{0, 0, 0, 0}, {1, 1, 1, 1}, {2, 3, 4, 1}, {3, 2, 0, 4}, {4, 0, 2, 3}};
    uint64_t seed = 1;
    for (const auto& sh : shapes)
        for (const auto& bc : mixes)
            for (int order = 1; order <= 2; ++order)
                for (int flux = 0; flux <= 2; ++flux)
                    for (int law = 0; law <= 2; ++law)
                        one_case(sh[0], sh[1], bc, order, flux, law, (seed & 1) != 0, seed++);
    // face, MUSCL and minmod helpers on a few states, one side dry
    double out[6];
    for (int flux = 0; flux <= 2; ++flux) {
        orc_face(9.81, 1.0, 0.1, 0.5, -0.2, 0.0, 0.3, 0.0, 0.0, out, flux);
        orc_face(9.81, 0.7, 0.0, -3.0, 1.0, 1.2, 0.0, 2.0, 0.5, out, flux);
    }
    double a[4] = {1.0, 0.1, 0.2, 1.1}, c[4] = {0.5, -0.3, 0.1, 0.6}, b[4] = {0.0, 0.0, 0.0, 0.0},
           rec[8];
    orc_muscl(a, c, b, 1e-12, rec);
    (void)orc_minmod(-1.0, 2.0);
    std::printf("sanitized oracle run: %d failures\n", failures);
    return failures ? 1 : 0;
}

// Host build of the per-sample arithmetic that the kernels run (gl_device.h:
// set constants, classification, quartic, boundary walk, quadrature), for the
// CPU tests.  The host build takes IEEE division and square root where the
// device takes the hardware estimates; everything else is the same source.
//
//   gl_host_check math           largest errors of the own sine/cosine, the
//                                arctangent and the angle reduction against
//                                the C library, and the largest reduced angle
//   gl_host_check flux P T O     P: float64 params [10][n] (parameter-major),
//                                T: float64 times [n] (one per set),
//                                O: float64 instantaneous fluxes [n];
//                                prints the number of ellipse arcs the arc
//                                rule accepted at its last level unconverged
//   gl_host_check snap N P T O   the same samples by the paper's integrator
//                                (FP32 snap + Simpson, N nodes)
//   gl_host_check ell P T O      general ellipsoids: P float64 [13][n], the
//                                per-sample shadow of locked sets from
//                                lock_at; prints the unconverged arc count
//   gl_host_check guesses Q O    first iterates of the quartic solver: Q
//                                float64 coefficients [n][5] (a0..a4), O
//                                float64 [n][5]: the real root of q' when it
//                                has one (else NaN), then the four Ferrari
//                                guesses for the roots of q (NaN where none)
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "gl_device.h"

static std::vector<double> read_all(const char* path)
{
    std::vector<double> v;
    FILE* f = std::fopen(path, "rb");
    if (!f) return v;
    double x;
    while (std::fread(&x, sizeof(x), 1, f) == 1) v.push_back(x);
    std::fclose(f);
    return v;
}

int main(int argc, char** argv)
{
    if (argc >= 2 && std::strcmp(argv[1], "math") == 0) {
        std::mt19937_64 rng(7);
        std::uniform_real_distribution<double> ua(-M_PI, M_PI), uy(-3.0, 3.0);
        double es = 0.0, ec = 0.0, ea = 0.0, ew = 0.0, rw = 0.0;
        for (int i = 0; i < 2000000; ++i) {
            const double a = ua(rng);
            double s, c;
            gl::sincos_pi(a, s, c);
            es = std::fmax(es, std::fabs(s - std::sin(a)));
            ec = std::fmax(ec, std::fabs(c - std::cos(a)));
            const double y = uy(rng), x = uy(rng);
            ea = std::fmax(ea, std::fabs(gl::atan2_d(y, x) - std::atan2(y, x)));
            const double w = 40.0 * ua(rng);
            ew = std::fmax(ew, std::fabs(std::remainder(gl::wrap_pi(w) - w, 2.0 * M_PI)));
            rw = std::fmax(rw, std::fabs(gl::wrap_pi(w)));
        }
        // edge arguments of the arctangent
        const double ys[] = {0.0, -0.0, 1.0, -1.0, 0.0, 1e-300, 1.0};
        const double xs[] = {0.0, 1.0, 0.0, 0.0, -1.0, -1.0, 1.0};
        for (int i = 0; i < 7; ++i) ea = std::fmax(ea, std::fabs(gl::atan2_d(ys[i], xs[i]) - std::atan2(ys[i], xs[i])));
        std::printf("%.6e %.6e %.6e %.6e %.17g\n", es, ec, ea, ew, rw);
        return 0;
    }
    if (argc == 5 && std::strcmp(argv[1], "flux") == 0) {
        const std::vector<double> p = read_all(argv[2]), t = read_all(argv[3]);
        const size_t n = t.size();
        if (n == 0 || p.size() != 10 * n) return 2;
        std::vector<double> out(n);
        gl::NoCensus nc;
        for (size_t s = 0; s < n; ++s) {
            double q[10];
            for (int i = 0; i < 10; ++i) q[i] = p[(size_t)i * n + s];
            gl::SetConst c;
            out[s] = gl::make_set_const(q, 0.0, 1, c) ? gl::flux_instant(c, t[s], nullptr, nc) : std::nan("");
        }
        std::printf("%d\n", nc.unconv);
        FILE* f = std::fopen(argv[4], "wb");
        if (!f) return 3;
        const bool ok = std::fwrite(out.data(), sizeof(double), n, f) == n;
        std::fclose(f);
        return ok ? 0 : 4;
    }
    if (argc == 6 && std::strcmp(argv[1], "snap") == 0) {
        // the paper's integrator (FP32 snap + Simpson) with N nodes
        const int nodes = std::atoi(argv[2]);
        const std::vector<double> p = read_all(argv[3]), t = read_all(argv[4]);
        const size_t n = t.size();
        if (n == 0 || p.size() != 10 * n || nodes < 2 || nodes % 2) return 2;
        std::vector<double> out(n);
        for (size_t s = 0; s < n; ++s) {
            double q[10];
            for (int i = 0; i < 10; ++i) q[i] = p[(size_t)i * n + s];
            gl::SetConst c;
            out[s] = gl::make_set_const(q, 0.0, 1, c) ? (double)gl::flux_snap(c, t[s], nodes) : std::nan("");
        }
        FILE* f = std::fopen(argv[5], "wb");
        if (!f) return 3;
        const bool ok = std::fwrite(out.data(), sizeof(double), n, f) == n;
        std::fclose(f);
        return ok ? 0 : 4;
    }
    if (argc == 5 && std::strcmp(argv[1], "ell") == 0) {
        const std::vector<double> p = read_all(argv[2]), t = read_all(argv[3]);
        const size_t n = t.size();
        const int np = gl::kEllParams;
        if (n == 0 || p.size() != (size_t)np * n) return 2;
        std::vector<double> out(n);
        gl::NoCensus nc;
        for (size_t s = 0; s < n; ++s) {
            double q[gl::kEllParams];
            for (int i = 0; i < np; ++i) q[i] = p[(size_t)i * n + s];
            gl::SetConst c;
            if (!gl::make_set_const_ell(q, 0.0, 1, c)) {
                out[s] = std::nan("");
                continue;
            }
            if (c.locked) {
                gl::SetConst l;
                gl::lock_at(c, t[s], l);
                out[s] = gl::flux_instant(l, t[s], nullptr, nc);
            } else {
                out[s] = gl::flux_instant(c, t[s], nullptr, nc);
            }
        }
        std::printf("%d\n", nc.unconv);
        FILE* f = std::fopen(argv[4], "wb");
        if (!f) return 3;
        const bool ok = std::fwrite(out.data(), sizeof(double), n, f) == n;
        std::fclose(f);
        return ok ? 0 : 4;
    }
    if (argc == 4 && std::strcmp(argv[1], "guesses") == 0) {
        const std::vector<double> q = read_all(argv[2]);
        if (q.empty() || q.size() % 5) return 2;
        const size_t n = q.size() / 5;
        std::vector<double> out(5 * n);
        for (size_t i = 0; i < n; ++i) {
            const gl::Poly4 p{q[5 * i], q[5 * i + 1], q[5 * i + 2], q[5 * i + 3], q[5 * i + 4]};
            out[5 * i] = gl::cubic_one_root(p);
            float g[4];
            gl::quartic_guesses(p, g);
            for (int k = 0; k < 4; ++k) out[5 * i + 1 + k] = (double)g[k];
        }
        FILE* f = std::fopen(argv[3], "wb");
        if (!f) return 3;
        const bool ok = std::fwrite(out.data(), sizeof(double), out.size(), f) == out.size();
        std::fclose(f);
        return ok ? 0 : 4;
    }
    std::fprintf(stderr, "usage: gl_host_check math | flux params times out | snap nodes params times out | "
                         "ell params times out | guesses coeffs out\n");
    return 1;
}

// Host-side set-up of one instance (see host_setup.h).
//
// Compact scheme (Sec. 2.1 and Appendix of the paper): five operator
// families share the "denominator" stencil d0 on 5 points; an operator term
// L(g) at row n is sum_j dL[n][j] g(r_{sigma_n + j}) and stands for
// sum_j d0[n][j] (L g)(r_{sigma_n + j}).  Centred rows get d0 and d4s from
// exactness of D D_* D D_* on degrees 0..8 plus sum(d0) = 1; the two rows next
// to each wall use d0 = e_n; d1, d2, d2s then follow from exactness on
// degrees 0..4.  Everything is computed in long double on O(1)-scaled
// monomials x = (r - r_n)/h and rounded once.
#include "host_setup.h"

#include <algorithm>
#include <cmath>
#include <sstream>

namespace tc {

namespace {

using ld = long double;

// Gaussian elimination with partial pivoting, n <= 10, in place.
bool solve_dense(int n, ld a[10][10], ld b[10]) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabsl(a[i][k]) > fabsl(a[p][k])) p = i;
        if (a[p][k] == 0.0L) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) { ld t = a[k][j]; a[k][j] = a[p][j]; a[p][j] = t; }
            ld t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            ld f = a[i][k] / a[k][k];
            if (f == 0.0L) continue;
            for (int j = k; j < n; ++j) a[i][j] -= f * a[k][j];
            b[i] -= f * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        ld s = b[i];
        for (int j = i + 1; j < n; ++j) s -= a[i][j] * b[j];
        b[i] = s / a[i][i];
    }
    return true;
}

// h^k d^k/dr^k of x^p at x.
ld dmono(ld x, int p, int k) {
    if (k > p) return 0.0L;
    ld f = 1.0L;
    for (int i = 0; i < k; ++i) f *= (ld)(p - i);
    ld xp = 1.0L;
    for (int i = 0; i < p - k; ++i) xp *= x;
    return f * xp;
}

// h^order (L x^p) at x, with q = h / r at that point.
ld scaled_op(int fam, ld x, ld q, int p) {
    ld d0 = dmono(x, p, 0), d1 = dmono(x, p, 1), d2 = dmono(x, p, 2);
    switch (fam) {
        case F_D1: return d1;
        case F_D2: return d2;
        case F_D2S: return d2 + q * d1 - q * q * d0;
        case F_D4S: {
            ld d3 = dmono(x, p, 3), d4 = dmono(x, p, 4);
            return d4 + 2 * q * d3 - 3 * q * q * d2 + 3 * q * q * q * d1 - 3 * q * q * q * q * d0;
        }
    }
    return d0;
}

int order_of(int fam) {
    switch (fam) {
        case F_D1: return 1;
        case F_D2: case F_D2S: return 2;
        case F_D4S: return 4;
    }
    return 0;
}

bool is_smooth_size(int n) {
    if (n < 4 || n > MAX_FFT) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

}  // namespace

bool make_plan(int n, FftPlan& p) {
    p = FftPlan{};
    p.n = n;
    int m = n;
    while (m > 1) {
        int r = (m % 4 == 0) ? 4 : (m % 3 == 0) ? 3 : (m % 2 == 0) ? 2 : 0;
        if (r == 0 || p.npass == MAX_RADICES) return false;
        p.radix[p.npass++] = r;
        m /= r;
    }
    return true;
}

int build_setup(const tc_geometry& g, Setup& s, std::string& err) {
    std::ostringstream e;
    auto fin = [](double x) { return std::isfinite(x); };
    if (!(fin(g.radius_ratio) && g.radius_ratio > 0.0 && g.radius_ratio < 1.0))
        e << "radius_ratio must lie in (0, 1); ";
    if (!(fin(g.gap) && g.gap > 0.0)) e << "gap must be > 0; ";
    if (!(fin(g.re) && g.re > 0.0)) e << "re must be > 0; ";
    if (!fin(g.re_outer)) e << "re_outer must be finite; ";
    if (!(fin(g.dt) && g.dt > 0.0)) e << "dt must be > 0; ";
    if (g.nr < 7) e << "nr must be >= 7; ";
    if (g.nr > 4097) e << "nr must be <= 4097; ";
    if (!is_smooth_size(g.ntheta)) e << "ntheta must be 2^a 3^b in [4, 1536]; ";
    if (!is_smooth_size(g.nz) || (g.nz % 2)) e << "nz must be even, 2^a 3^b in [4, 1536]; ";
    if (!(fin(g.theta_period) && g.theta_period >= 0.0)) e << "theta_period must be >= 0; ";
    if (!(fin(g.lz) && g.lz >= 0.0)) e << "lz must be >= 0; ";
    if (!(fin(g.stretch) && g.stretch >= 0.0 && g.stretch <= 10.0)) e << "stretch must lie in [0, 10]; ";
    if (g.precision != TC_PREC_FP64 && g.precision != TC_PREC_MIXED) e << "unknown precision; ";
    if (g.flags & ~(TC_FLAG_LINEAR | TC_FLAG_DRYRUN | TC_FLAG_GENERIC_FFT)) e << "unknown flags; ";
    if (e.str().empty()) {
        // the theta kernel keeps three rows of length ntheta in LDS (64 KiB per block)
        const size_t csize = g.precision == TC_PREC_MIXED ? 8 : 16;
        if ((size_t)3 * g.ntheta * csize > 65536) e << "ntheta too large for this precision (3 ntheta complex values must fit 64 KiB); ";
    }
    if (!e.str().empty()) {
        err = e.str();
        return TC_EINVAL;
    }

    s = Setup{};
    s.g = g;
    s.nr = g.nr;
    s.ntheta = g.ntheta;
    s.nz = g.nz;
    s.kt = (g.ntheta - 1) / 3;
    s.kz = (g.nz - 1) / 3;
    s.nj = s.kt + 1;
    s.nl = 2 * s.kz + 1;
    const double d = g.gap;
    s.ri = d * g.radius_ratio / (1.0 - g.radius_ratio);
    s.ro = d / (1.0 - g.radius_ratio);
    s.nu = d / g.re;
    s.w_outer = g.re_outer / g.re;
    const double rc = 0.5 * (s.ri + s.ro);
    s.theta = g.theta_period > 0 ? g.theta_period : std::fmin(2.0 * M_PI, 5.0 * M_PI * d / rc);
    s.lz = g.lz > 0 ? g.lz : 2.5 * d;

    // radial grid: r_n = R_i + d (1 + T(xi_n)) / 2, walls exact
    const int nr = s.nr;
    s.r.resize(nr);
    for (int n = 0; n < nr; ++n) {
        double xi = -1.0 + 2.0 * n / (nr - 1);
        double t = g.stretch > 0 ? std::tanh(g.stretch * xi) / std::tanh(g.stretch) : xi;
        s.r[n] = s.ri + d * (1.0 + t) / 2.0;
    }
    s.r[0] = s.ri;
    s.r[nr - 1] = s.ro;
    for (int n = 1; n < nr; ++n)
        if (!(s.r[n] > s.r[n - 1])) {
            err = "radial grid is not strictly increasing (stretch too strong for nr)";
            return TC_EINVAL;
        }

    // compact coefficients
    s.sigma.resize(nr);
    s.coef.assign((size_t)N_FAMILIES * nr * 5, 0.0);
    for (int n = 0; n < nr; ++n) {
        int sg = n - 2;
        if (sg < 0) sg = 0;
        if (sg > nr - 5) sg = nr - 5;
        s.sigma[n] = sg;
        ld h = ((ld)s.r[sg + 4] - (ld)s.r[sg]) / 4.0L;
        ld x[5], q[5];
        for (int j = 0; j < 5; ++j) {
            x[j] = ((ld)s.r[sg + j] - (ld)s.r[n]) / h;
            q[j] = h / (ld)s.r[sg + j];
        }
        ld d0[5] = {0, 0, 0, 0, 0};
        ld d4[5];
        if (sg == n - 2) {
            ld a[10][10], b[10];
            for (int p = 0; p < 9; ++p) {
                for (int j = 0; j < 5; ++j) {
                    a[p][j] = -scaled_op(F_D4S, x[j], q[j], p);
                    a[p][5 + j] = dmono(x[j], p, 0);
                }
                b[p] = 0.0L;
            }
            for (int j = 0; j < 10; ++j) a[9][j] = j < 5 ? 1.0L : 0.0L;
            b[9] = 1.0L;
            if (!solve_dense(10, a, b)) {
                err = "singular compact-coefficient system";
                return TC_EINVAL;
            }
            for (int j = 0; j < 5; ++j) { d0[j] = b[j]; d4[j] = b[5 + j]; }
        } else {
            d0[n - sg] = 1.0L;
            ld a[10][10], b[10];
            for (int p = 0; p < 5; ++p) {
                for (int j = 0; j < 5; ++j) a[p][j] = dmono(x[j], p, 0);
                b[p] = scaled_op(F_D4S, x[n - sg], q[n - sg], p);
            }
            if (!solve_dense(5, a, b)) {
                err = "singular compact-coefficient system";
                return TC_EINVAL;
            }
            for (int j = 0; j < 5; ++j) d4[j] = b[j];
        }
        for (int j = 0; j < 5; ++j) {
            s.coef[(F_D0 * nr + n) * 5 + j] = (double)d0[j];
            s.coef[(F_D4S * nr + n) * 5 + j] = (double)(d4[j] / (h * h * h * h));
        }
        for (int fam : {F_D1, F_D2, F_D2S}) {
            ld a[10][10], b[10];
            for (int p = 0; p < 5; ++p) {
                ld acc = 0.0L;
                for (int j = 0; j < 5; ++j) {
                    a[p][j] = dmono(x[j], p, 0);
                    acc += d0[j] * scaled_op(fam, x[j], q[j], p);
                }
                b[p] = acc;
            }
            if (!solve_dense(5, a, b)) {
                err = "singular compact-coefficient system";
                return TC_EINVAL;
            }
            ld hk = 1.0L;
            for (int i = 0; i < order_of(fam); ++i) hk *= h;
            for (int j = 0; j < 5; ++j) s.coef[(fam * nr + n) * 5 + j] = (double)(b[j] / hk);
        }
    }

    // LU of the centred block of d0 (rows/columns 2..nr-3), no pivoting
    s.blu.assign((size_t)nr * 5, 0.0);
    {
        std::vector<ld> u0(nr, 0), u1(nr, 0), u2(nr, 0);
        for (int n = 2; n <= nr - 3; ++n) {
            ld row[5];
            for (int j = 0; j < 5; ++j) {
                int col = n - 2 + j;
                row[j] = (col >= 2 && col <= nr - 3) ? (ld)s.c(F_D0, n, j) : 0.0L;
            }
            ld l2 = 0, l1 = 0;
            ld c = row[1], dd = row[2], a = row[3];
            if (n - 2 >= 2) {
                l2 = row[0] / u0[n - 2];
                c -= l2 * u1[n - 2];
                dd -= l2 * u2[n - 2];
            }
            if (n - 1 >= 2) {
                l1 = c / u0[n - 1];
                dd -= l1 * u1[n - 1];
                a -= l1 * u2[n - 1];
            }
            if (dd == 0.0L) {
                err = "singular compact denominator";
                return TC_EINVAL;
            }
            u0[n] = dd;
            u1[n] = a;
            u2[n] = row[4];
            double* o = &s.blu[(size_t)n * 5];
            o[0] = (double)l2;
            o[1] = (double)l1;
            o[2] = (double)(1.0L / dd);
            o[3] = (double)a;
            o[4] = (double)row[4];
        }
    }

    // Segmented sweeps: the centred block (rows 2..nr-3) is cut into
    // dv_nseg segments of dv_seg rows (8 of 4, 8 or 16; 16 segments of 8
    // rows measured slower).  Inside segment [s0, s1) the
    // forward recurrence y_n = r_n - l1_n y_{n-1} - l2_n y_{n-2} is the
    // particular solution from zero carry-in plus y_{s0-1} hf1 + y_{s0-2} hf2,
    // the backward one x_n = (y_n - u1_n x_{n+1} - u2_n x_{n+2}) / u0_n the
    // particular solution plus x_{s1} hb1 + x_{s1+1} hb2.
    {
        const int nc = nr - 4;
        int L = 0, S = 0;
        if (nc <= 32) {
            L = 4;
            S = 8;
        } else if (nc <= 64) {
            L = 8;
            S = 8;
        } else if (nc <= 128) {
            L = 16;
            S = 8;
        }
        s.dv_seg = L;
        s.dv_nseg = S;
        s.dvh.assign((size_t)4 * nr, 0.0);
        if (s.dv_seg) {
            for (int seg = 0; seg < S; ++seg) {
                const int s0 = 2 + seg * L, s1 = std::min(s0 + L, nr - 2);
                for (int which = 0; which < 2; ++which) {
                    ld a1 = which == 0 ? 1.0L : 0.0L, a2 = which == 0 ? 0.0L : 1.0L;  // y_{n-1}, y_{n-2}
                    for (int n = s0; n < s1; ++n) {
                        const ld h = -(ld)s.blu[(size_t)n * 5 + 1] * a1 - (ld)s.blu[(size_t)n * 5 + 0] * a2;
                        s.dvh[(size_t)which * nr + n] = (double)h;
                        a2 = a1;
                        a1 = h;
                    }
                    ld b1 = which == 0 ? 1.0L : 0.0L, b2 = which == 0 ? 0.0L : 1.0L;  // x_{n+1}, x_{n+2}
                    for (int n = s1 - 1; n >= s0; --n) {
                        const double* o = &s.blu[(size_t)n * 5];
                        const ld x = (-(ld)o[3] * b1 - (ld)o[4] * b2) * (ld)o[2];
                        s.dvh[(size_t)(2 + which) * nr + n] = (double)x;
                        b2 = b1;
                        b1 = x;
                    }
                }
            }
        }
    }

    // wavenumbers
    s.m.resize(s.nj);
    for (int j = 0; j < s.nj; ++j) s.m[j] = 2.0 * M_PI * j / s.theta;
    s.alpha.resize(s.nl);
    for (int l = -s.kz; l <= s.kz; ++l) s.alpha[l + s.kz] = 2.0 * M_PI * l / s.lz;

    // FFT tables
    auto twid = [](int n, std::vector<double>& t) {
        t.resize(2 * (size_t)n);
        const ld two_pi = 6.283185307179586476925286766559005768L;
        for (int k = 0; k < n; ++k) {
            ld a = two_pi * (ld)k / (ld)n;
            t[2 * k] = (double)cosl(a);
            t[2 * k + 1] = (double)sinl(a);
        }
    };
    twid(s.ntheta, s.tw_theta);
    twid(s.nz, s.tw_z);
    if (!make_plan(s.ntheta, s.plan_theta) || !make_plan(s.nz, s.plan_z)) {
        err = "unsupported transform length";
        return TC_EINVAL;
    }
    return TC_OK;
}

}  // namespace tc

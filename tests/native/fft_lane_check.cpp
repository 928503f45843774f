// Host check of the lane FFT (paper_0711_1429_amd/csrc/fft_lane.h): every
// lane runs on its own host thread and the block barrier is a std::barrier,
// so the LDS exchanges are reproduced exactly.  Compared with a direct DFT in
// long double.  Prints one line per case and exits non-zero on failure.
#include <barrier>
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_0711_1429_amd/csrc/fft_lane.h"

using namespace tc;

struct HostSync {
    std::barrier<>* b;
    void operator()() const { b->arrive_and_wait(); }
};

template <int N, int SIGN, bool OUT_REGS>
double run_case(unsigned seed) {
    using P = lane::Plan<N>;
    std::vector<C<double>> in(N), buf(N), out(N);
    std::vector<double> tw(2 * N);
    const long double pi2 = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < N; ++k) {
        tw[2 * k] = (double)cosl(pi2 * k / N);
        tw[2 * k + 1] = (double)sinl(pi2 * k / N);
    }
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    for (auto& z : in) z = {nd(rng), nd(rng)};
    std::vector<C<double>> twp(lane::tw_size<N>() + 1);
    lane::fill_twiddles<double, N>(twp.data(), tw.data(), 0, 1);
    std::barrier<> bar(P::TL);
    HostSync sync{&bar};
    std::vector<std::thread> th;
    for (int g = 0; g < P::TL; ++g) {
        th.emplace_back([&, g] {
            C<double> x[P::P];
            for (int k = 0; k < P::P; ++k) x[k] = in[g + k * P::TL];
            lane::fft<double, N, SIGN, OUT_REGS>(buf.data(), x, g, twp.data(), sync);
            if (OUT_REGS)
                for (int s = 0; s < P::P; ++s) out[g + P::TL * lane::last_slot_to_m<N>(s)] = x[s];
        });
    }
    for (auto& t : th) t.join();
    if (!OUT_REGS)
        for (int k = 0; k < N; ++k) out[k] = buf[lane::swz<double, N>(k)];
    double err = 0, scale = 0;
    for (int k = 0; k < N; ++k) {
        std::complex<long double> s = 0;
        for (int n = 0; n < N; ++n) {
            long double a = SIGN * pi2 * (long double)((long long)n * k % N) / N;
            s += std::complex<long double>(in[n].x, in[n].y) * std::complex<long double>(cosl(a), sinl(a));
        }
        err = std::fmax(err, (double)std::abs(s - std::complex<long double>(out[k].x, out[k].y)));
        scale = std::fmax(scale, (double)std::abs(s));
    }
    return err / scale;
}

template <int N>
bool check() {
    static_assert(lane::supported(N), "unsupported size");
    double e[4] = {run_case<N, 1, true>(1), run_case<N, -1, true>(2), run_case<N, 1, false>(3),
                   run_case<N, -1, false>(4)};
    double m = 0;
    for (double x : e) m = std::fmax(m, x);
    std::printf("N=%4d lanes=%2d P=%2d passes=%d max_rel_err=%.3e\n", N, lane::Plan<N>::TL, lane::Plan<N>::P,
                lane::Plan<N>::NPASS, m);
    return m < 1e-14;
}

int main() {
    bool ok = true;
    ok &= check<8>();
    ok &= check<12>();
    ok &= check<16>();
    ok &= check<24>();
    ok &= check<32>();
    ok &= check<48>();
    ok &= check<64>();
    ok &= check<96>();
    ok &= check<128>();
    ok &= check<192>();
    ok &= check<256>();
    ok &= check<384>();
    ok &= check<512>();
    ok &= check<768>();
    std::printf(ok ? "ALL OK\n" : "FAILED\n");
    return ok ? 0 : 1;
}

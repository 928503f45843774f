// Compile-time-sized Stockham FFT in which every lane owns P points.
//
// A transform of length N is processed by Tl = N / P lanes (Tl a power of two
// and at most 64, so one transform never spans two wavefronts).  The first
// pass has radix P; every later pass has a radix R dividing P, so in every
// pass each lane computes exactly P / R butterflies of radix R and no lane is
// idle.  Between passes the values go through an LDS buffer of N points per
// transform; the caller provides the synchronisation functor (a block barrier
// on the device, a thread barrier in the host test).
//
// Register layout: during a pass of radix R a lane holds x[t * R + k],
// butterfly t (index jb = g + t * Tl) element k.  The first pass reads
// position g + k * Tl; the last pass leaves position g + Tl * (t + k * K)
// (K = P / R_last) in x[t * R + k].
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace tc {
namespace lane {

template <typename T>
__host__ __device__ __forceinline__ C<T> add(C<T> a, C<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ C<T> sub(C<T> a, C<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ C<T> mul(C<T> a, C<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by (sign * i)
template <typename T, int SIGN>
__host__ __device__ __forceinline__ C<T> mul_si(C<T> a) {
    return SIGN > 0 ? C<T>{-a.y, a.x} : C<T>{a.y, -a.x};
}

// Radix-R DFT in registers with exponent SIGN * 2 pi i / R (R = 2, 3, 4, 6, 8, 12).
template <typename T, int R, int SIGN>
__host__ __device__ __forceinline__ void dft(C<T>* x);

template <typename T, int SIGN>
__host__ __device__ __forceinline__ void dft2(C<T>& a, C<T>& b) {
    C<T> s = add(a, b), d = sub(a, b);
    a = s;
    b = d;
}

template <typename T, int SIGN>
__host__ __device__ __forceinline__ void dft3(C<T>& a, C<T>& b, C<T>& c) {
    const T h = (T)0.866025403784438646763723170752936183L;  // sqrt(3)/2
    C<T> t1 = add(b, c), t2 = sub(b, c);
    C<T> m = {a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
    C<T> n = mul_si<T, SIGN>(C<T>{h * t2.x, h * t2.y});
    a = add(a, t1);
    b = add(m, n);
    c = sub(m, n);
}

template <typename T, int SIGN>
__host__ __device__ __forceinline__ void dft4(C<T>& a, C<T>& b, C<T>& c, C<T>& d) {
    C<T> s0 = add(a, c), d0 = sub(a, c);
    C<T> s1 = add(b, d), d1 = mul_si<T, SIGN>(sub(b, d));
    a = add(s0, s1);
    c = sub(s0, s1);
    b = add(d0, d1);
    d = sub(d0, d1);
}

template <typename T, int R, int SIGN>
__host__ __device__ __forceinline__ void dft(C<T>* x) {
    if constexpr (R == 2) {
        dft2<T, SIGN>(x[0], x[1]);
    } else if constexpr (R == 3) {
        dft3<T, SIGN>(x[0], x[1], x[2]);
    } else if constexpr (R == 4) {
        dft4<T, SIGN>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 6) {
        // 6 = 3 x 2: x[n1 + 2 n2] -> X[k2 + 3 k1]
        C<T> a0 = x[0], a1 = x[2], a2 = x[4];  // n1 = 0
        C<T> b0 = x[1], b1 = x[3], b2 = x[5];  // n1 = 1
        dft3<T, SIGN>(a0, a1, a2);
        dft3<T, SIGN>(b0, b1, b2);
        // twiddle w6^(n1 k2), n1 = 1: k2 = 1 -> w6, k2 = 2 -> w6^2
        const T h = (T)0.866025403784438646763723170752936183L;
        const C<T> w1 = {(T)0.5, SIGN > 0 ? h : -h};
        const C<T> w2 = {(T)-0.5, SIGN > 0 ? h : -h};
        b1 = mul(b1, w1);
        b2 = mul(b2, w2);
        dft2<T, SIGN>(a0, b0);
        dft2<T, SIGN>(a1, b1);
        dft2<T, SIGN>(a2, b2);
        x[0] = a0; x[3] = b0;
        x[1] = a1; x[4] = b1;
        x[2] = a2; x[5] = b2;
    } else if constexpr (R == 8) {
        // 8 = 2 x 4: x[n1 + 2 n2] (n2 = 0..3) -> X[k2 + 4 k1]
        C<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
        C<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
        dft4<T, SIGN>(e0, e1, e2, e3);
        dft4<T, SIGN>(o0, o1, o2, o3);
        const T s = (T)0.707106781186547524400844362104849039L;
        o1 = mul(o1, C<T>{s, SIGN > 0 ? s : -s});
        o2 = mul_si<T, SIGN>(o2);
        o3 = mul(o3, C<T>{-s, SIGN > 0 ? s : -s});
        dft2<T, SIGN>(e0, o0);
        dft2<T, SIGN>(e1, o1);
        dft2<T, SIGN>(e2, o2);
        dft2<T, SIGN>(e3, o3);
        x[0] = e0; x[4] = o0;
        x[1] = e1; x[5] = o1;
        x[2] = e2; x[6] = o2;
        x[3] = e3; x[7] = o3;
    } else if constexpr (R == 12) {
        // 12 = 4 x 3: x[n1 + 4 n2] (n1 = 0..3, n2 = 0..2) -> X[k2 + 3 k1]
        C<T> a[4][3];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            a[n1][0] = x[n1];
            a[n1][1] = x[n1 + 4];
            a[n1][2] = x[n1 + 8];
            dft3<T, SIGN>(a[n1][0], a[n1][1], a[n1][2]);
        }
        // twiddles w12^(n1 k2)
        const T h = (T)0.866025403784438646763723170752936183L;
        const T sg = SIGN > 0 ? (T)1 : (T)-1;
        const C<T> w1 = {h, sg * (T)0.5};        // w12^1
        const C<T> w2 = {(T)0.5, sg * h};        // w12^2
        const C<T> w4 = {(T)-0.5, sg * h};       // w12^4
        const C<T> w6 = {(T)-1, (T)0};           // w12^6
        a[1][1] = mul(a[1][1], w1);
        a[1][2] = mul(a[1][2], w2);
        a[2][1] = mul(a[2][1], w2);
        a[2][2] = mul(a[2][2], w4);
        a[3][1] = mul_si<T, SIGN>(a[3][1]);      // w12^3 = sign i
        a[3][2] = mul(a[3][2], w6);
#pragma unroll
        for (int k2 = 0; k2 < 3; ++k2) {
            dft4<T, SIGN>(a[0][k2], a[1][k2], a[2][k2], a[3][k2]);
            x[k2] = a[0][k2];
            x[k2 + 3] = a[1][k2];
            x[k2 + 6] = a[2][k2];
            x[k2 + 9] = a[3][k2];
        }
    }
}

// ------------------------------------------------------------------ plan
struct Radices {
    int n;
    int r[10];
};

constexpr int points_per_lane(int N) { return N % 3 == 0 ? 12 : (N >= 64 ? 8 : 4); }

constexpr Radices radices(int N) {
    Radices x{};
    const int P = points_per_lane(N);
    x.n = 0;
    x.r[x.n++] = P;
    int m = N / P;
    while (m > 1) {
        int best = 1;
        for (int d = P; d >= 2; --d)
            if (P % d == 0 && m % d == 0) {
                best = d;
                break;
            }
        if (best == 1) return Radices{0, {}};
        x.r[x.n++] = best;
        m /= best;
    }
    return x;
}

constexpr int ns_before(int N, int pass) {
    Radices r = radices(N);
    int ns = 1;
    for (int i = 0; i < pass; ++i) ns *= r.r[i];
    return ns;
}

constexpr bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Sizes the lane FFT supports: N = 2^a * 3^b with b <= 1, lanes per
// transform a power of two in [1, 64], and a full radix plan.
constexpr bool supported(int N) {
    if (N < 8) return false;
    int m = N;
    while (m % 2 == 0) m /= 2;
    if (m != 1 && m != 3) return false;
    const int P = points_per_lane(N);
    if (N % P) return false;
    const int tl = N / P;
    return is_pow2(tl) && tl <= 64 && radices(N).n > 0;
}

template <int N>
struct Plan {
    static constexpr int P = points_per_lane(N);
    static constexpr int TL = N / P;
    static constexpr Radices rad = radices(N);
    static constexpr int NPASS = rad.n;
    static constexpr int RLAST = rad.r[rad.n - 1];
    static constexpr int KLAST = P / RLAST;
};

// Position held in register m after the last pass (m = t + k K as
// described above) is g + TL * m: the map from the last pass's (t, k)
// register slot to m.
template <int N>
__host__ __device__ constexpr int last_slot_to_m(int slot) {
    return slot / Plan<N>::RLAST + (slot % Plan<N>::RLAST) * Plan<N>::KLAST;
}

// LDS address of transform element e.  For N >= 64 the low four bits of e
// are XOR-ed with bits 3..6: a bijection inside each aligned block of 16
// elements that spreads the strided stores of the Stockham passes over
// distinct LDS banks.  Complex floats of the 12-points-per-lane lengths are
// stored in natural order instead, which measured faster for them.
template <typename T, int N>
__host__ __device__ __forceinline__ int swz(int e) {
    if constexpr (N >= 64 && N % 16 == 0 && !(sizeof(T) == 4 && points_per_lane(N) == 12)) {
        return e ^ ((e >> 3) & 15);
    } else {
        return e;
    }
}

// ------------------------------------------------------------------ twiddles
// Pass p > 0 multiplies element k of butterfly jb by w^(k * (jb mod NS_p) *
// STEP_p) with w = exp(+-2 pi i / N).  The per-pass table holds
// w^(jm * STEP_p) for jm < NS_p at offset tw_offset(N, p), so the lanes of a
// pass read consecutive entries; the powers k = 2.. are formed by
// multiplication.
constexpr int tw_offset(int N, int pass) {
    int off = 0;
    for (int q = 1; q < pass; ++q) off += ns_before(N, q);
    return off;
}

template <int N>
constexpr int tw_size() { return tw_offset(N, Plan<N>::NPASS); }

// Fill the per-pass table from a full table of exp(+2 pi i e / N) (2N reals).
// Each thread first loads its first entry of every pass (at a clamped index
// where the pass has fewer entries than threads), then stores them, so those
// loads are in flight together; entries beyond the first round follow.
template <typename T, int N, int PASS, typename TwPtr>
__host__ __device__ __forceinline__ void fill_first(C<T>* first, TwPtr tw_full, int tid) {
    if constexpr (PASS < Plan<N>::NPASS) {
        constexpr int NS = ns_before(N, PASS);
        constexpr int STEP = N / (NS * radices(N).r[PASS]);
        const int e = (tid < NS ? tid : NS - 1) * STEP;
        first[PASS] = C<T>{tw_full[2 * e], tw_full[2 * e + 1]};
        fill_first<T, N, PASS + 1>(first, tw_full, tid);
    }
}
template <typename T, int N, int PASS, typename TwPtr>
__host__ __device__ __forceinline__ void fill_pass(C<T>* twp, const C<T>* first, TwPtr tw_full, int tid, int nthreads) {
    if constexpr (PASS < Plan<N>::NPASS) {
        constexpr int NS = ns_before(N, PASS);
        constexpr int STEP = N / (NS * radices(N).r[PASS]);
        constexpr int OFF = tw_offset(N, PASS);
        if (tid < NS) twp[OFF + tid] = first[PASS];
        for (int jm = tid + nthreads; jm < NS; jm += nthreads) {
            const int e = jm * STEP;
            twp[OFF + jm] = C<T>{tw_full[2 * e], tw_full[2 * e + 1]};
        }
        fill_pass<T, N, PASS + 1>(twp, first, tw_full, tid, nthreads);
    }
}

// tw_full: any pointer-like to T (a device kernel passes a global-address-space pointer)
template <typename T, int N, typename TwPtr>
__host__ __device__ __forceinline__ void fill_twiddles(C<T>* twp, TwPtr tw_full, int tid, int nthreads) {
    C<T> first[Plan<N>::NPASS > 1 ? Plan<N>::NPASS : 1];
    fill_first<T, N, 1>(first, tw_full, tid);
    fill_pass<T, N, 1>(twp, first, tw_full, tid, nthreads);
}

// ------------------------------------------------------------------ passes
template <typename T, int N, int PASS, int SIGN>
__host__ __device__ __forceinline__ void butterflies(C<T>* x, int g, const C<T>* twp) {
    constexpr Radices rad = radices(N);
    constexpr int R = rad.r[PASS];
    constexpr int NS = ns_before(N, PASS);
    constexpr int TL = Plan<N>::TL;
    constexpr int K = Plan<N>::P / R;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        if constexpr (NS > 1) {
            const int jb = g + t * TL;
            const int jm = jb % NS;
            constexpr int OFF = tw_offset(N, PASS);
            C<T> w1 = twp[OFF + jm];
            if (SIGN < 0) w1.y = -w1.y;
            C<T> wk = w1;
#pragma unroll
            for (int k = 1; k < R; ++k) {
                x[t * R + k] = mul(x[t * R + k], wk);
                if (k + 1 < R) wk = mul(wk, w1);
            }
        }
        dft<T, R, SIGN>(x + t * R);
    }
}

// Read the inputs of pass PASS (> 0) from the transform's LDS region.
template <typename T, int N, int PASS>
__host__ __device__ __forceinline__ void load_pass(const C<T>* buf, C<T>* x, int g) {
    constexpr Radices rad = radices(N);
    constexpr int R = rad.r[PASS];
    constexpr int TL = Plan<N>::TL;
    constexpr int K = Plan<N>::P / R;
#pragma unroll
    for (int t = 0; t < K; ++t)
#pragma unroll
        for (int k = 0; k < R; ++k) x[t * R + k] = buf[swz<T, N>(g + t * TL + k * (N / R))];
}

// Write the outputs of pass PASS to the transform's LDS region (natural
// Stockham positions).
template <typename T, int N, int PASS>
__host__ __device__ __forceinline__ void store_pass(C<T>* buf, const C<T>* x, int g) {
    constexpr Radices rad = radices(N);
    constexpr int R = rad.r[PASS];
    constexpr int NS = ns_before(N, PASS);
    constexpr int TL = Plan<N>::TL;
    constexpr int K = Plan<N>::P / R;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int jb = g + t * TL;
        const int idx = (jb / NS) * NS * R + jb % NS;
#pragma unroll
        for (int k = 0; k < R; ++k) buf[swz<T, N>(idx + k * NS)] = x[t * R + k];
    }
}

// Runs passes PASS.. with x holding the inputs of pass PASS.  When
// OUT_REGS, the last pass's outputs stay in x (layout above); otherwise they
// are written to buf, element e at swz<T, N>(e).  SYNC() is called between every LDS
// write and read (and between a read and the next overwrite of buf).
template <typename T, int N, int PASS, int SIGN, bool OUT_REGS, typename Sync>
__host__ __device__ __forceinline__ void run_passes(C<T>* buf, C<T>* x, int g, const C<T>* tw, const Sync& sync) {
    constexpr int NP = Plan<N>::NPASS;
    if constexpr (PASS < NP) {
        butterflies<T, N, PASS, SIGN>(x, g, tw);
        if constexpr (PASS + 1 < NP) {
            store_pass<T, N, PASS>(buf, x, g);
            sync();
            load_pass<T, N, PASS + 1>(buf, x, g);
            sync();
            run_passes<T, N, PASS + 1, SIGN, OUT_REGS>(buf, x, g, tw, sync);
        } else if constexpr (!OUT_REGS) {
            store_pass<T, N, PASS>(buf, x, g);
        }
    }
}

// Full transform: x[k] holds position g + k * TL on entry; tw is the per-pass
// twiddle table filled by fill_twiddles.
template <typename T, int N, int SIGN, bool OUT_REGS, typename Sync>
__host__ __device__ __forceinline__ void fft(C<T>* buf, C<T>* x, int g, const C<T>* tw, const Sync& sync) {
    run_passes<T, N, 0, SIGN, OUT_REGS>(buf, x, g, tw, sync);
}

}  // namespace lane
}  // namespace tc

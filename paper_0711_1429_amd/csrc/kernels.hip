// HIP kernels (gfx950) of one RK3 / Crank--Nicolson substep of the
// Taylor--Couette DNS (Pirro & Quadrio; Sec. 2.1 and Appendix).
//
// Spectral fields are [r][j][l + K_z] complex (plane-major), so every radial
// sweep reads consecutive modes with consecutive lanes.  Per substep:
//
//   k_dv     velocity recovery, radial part: D v from the compact derivative
//            (d0 D v = d1 v, pentadiagonal, one mode per lane).
//   k_zinv   u, v, w per (r, j-column block): recovery of u and w from
//            (v, eta, D v) in FP64, zero-padded inverse z FFT in LDS, written
//            transposed as [field][r][z][j].
//   k_theta  per (r, z-pair): the two real theta rows of each field packed
//            as one complex row, inverse FFT, the six products, forward FFT,
//            unpacked and truncated to j <= K_theta: [product][r][z][j].
//   k_zfwd   per (r, j-column block): forward z FFT, truncation to |l| <= K_z
//            and the 1/(N_theta N_z) normalisation: [product][r][j][l].
//   k_rhs    one (r, mode) per lane: the explicit terms N = nu E + NL of
//            eq. (final-v) / eq. (final-eta) (and of the mean flow) from
//            5-point compact stencils, and the Runge--Kutta right-hand side.
//   k_solve  one (|l|, j) pair and one equation per lane: assembles the real
//            pentadiagonal Crank--Nicolson matrix on the fly (boundary rows
//            folded) and eliminates both +l and -l right-hand sides.
//
// The FFT stages are templated on the storage type (double, or float for the
// mixed-precision path); recovery, the radial stages and reductions are FP64.
#include <cmath>
#include <mutex>

#include "fft_lane.h"
#include "fft_xlane.h"
#include "kernels.h"

namespace tc {

const char* const kKernelNames[K_COUNT] = {
    "radial_derivative", "zfft_inverse", "theta_rows_products", "zfft_forward",
    "radial_rhs",        "radial_solve", "stats_energy",        "finite_check"};

namespace {

constexpr int NT = 256;             // threads of the FFT and stencil kernels
constexpr int ZELEMS = 3072;        // max complex elements per z-FFT block
constexpr int TELEMS = 3 * MAX_FFT; // max complex elements per theta block
constexpr int SOLVE_NT = 64;        // lanes per block of the radial solve
constexpr int RED_NT = 256;         // lanes per block of the reductions

using cd = C<double>;

template <typename T>
__device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C<T> cscale(C<T> a, T s) { return {a.x * s, a.y * s}; }
// i * z
__device__ __forceinline__ cd ci(cd z) { return {-z.y, z.x}; }
__device__ __forceinline__ cd cfma(double s, cd a, cd acc) { return {acc.x + s * a.x, acc.y + s * a.y}; }

template <typename T>
__device__ __forceinline__ C<T> twid(const T* tw, int t, int sign) {
    C<T> w = {tw[2 * t], tw[2 * t + 1]};
    if (sign < 0) w.y = -w.y;
    return w;
}

// In-register DFT of radix R with exponent sign * 2 pi i / R.
template <typename T, int R>
__device__ __forceinline__ void dft(C<T>* x, int sign) {
    if constexpr (R == 2) {
        C<T> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T h = (T)0.86602540378443864676;  // sqrt(3)/2
        C<T> t1 = cadd(x[1], x[2]);
        C<T> t2 = csub(x[1], x[2]);
        C<T> m = {x[0].x - (T)0.5 * t1.x, x[0].y - (T)0.5 * t1.y};
        T s = sign > 0 ? h : -h;
        C<T> n = {-s * t2.y, s * t2.x};  // s i t2
        x[0] = cadd(x[0], t1);
        x[1] = cadd(m, n);
        x[2] = csub(m, n);
    } else {  // R == 4
        C<T> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        C<T> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        C<T> id = sign > 0 ? C<T>{-d.y, d.x} : C<T>{d.y, -d.x};  // sign i d
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, id);
        x[3] = csub(b, id);
    }
}

// One Stockham autosort pass of radix R over ncols columns of length N held
// in LDS as buf[col * N + i].  Inputs are read into registers, the block
// synchronises, outputs are written back in place.
template <typename T, int R, int MAXB>
__device__ __forceinline__ void fft_pass(C<T>* buf, int ncols, int N, int Ns, int sign, const T* tw) {
    const int tid = threadIdx.x;
    const int nbf = N / R;
    const int total = ncols * nbf;
    const int step = N / (Ns * R);
    C<T> y[MAXB][R];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        const int b = tid + t * NT;
        if (b < total) {
            const int col = b / nbf;
            const int jb = b - col * nbf;
            const C<T>* base = buf + col * N;
            C<T> x[R];
#pragma unroll
            for (int k = 0; k < R; ++k) x[k] = base[jb + k * nbf];
            const int jm = jb % Ns;
#pragma unroll
            for (int k = 1; k < R; ++k) x[k] = cmul(x[k], twid(tw, jm * k * step, sign));
            dft<T, R>(x, sign);
#pragma unroll
            for (int k = 0; k < R; ++k) y[t][k] = x[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        const int b = tid + t * NT;
        if (b < total) {
            const int col = b / nbf;
            const int jb = b - col * nbf;
            const int jm = jb % Ns;
            C<T>* base = buf + col * N;
            const int idx = (jb / Ns) * Ns * R + jm;
#pragma unroll
            for (int k = 0; k < R; ++k) base[idx + k * Ns] = y[t][k];
        }
    }
    __syncthreads();
}

// Complete FFT of ncols columns (ncols * N <= ELEMS) in LDS; the caller has
// synchronised after filling buf.  Ends synchronised.
template <typename T, int ELEMS>
__device__ void fft_lds(C<T>* buf, int ncols, const FftPlanDev& p, int sign, const T* tw) {
    int ns = 1;
    for (int i = 0; i < p.npass; ++i) {
        const int r = p.radix[i];
        if (r == 4)
            fft_pass<T, 4, (ELEMS + 4 * NT - 1) / (4 * NT)>(buf, ncols, p.n, ns, sign, tw);
        else if (r == 3)
            fft_pass<T, 3, (ELEMS + 3 * NT - 1) / (3 * NT)>(buf, ncols, p.n, ns, sign, tw);
        else
            fft_pass<T, 2, (ELEMS + 2 * NT - 1) / (2 * NT)>(buf, ncols, p.n, ns, sign, tw);
        ns *= r;
    }
}

template <typename T>
__device__ __forceinline__ const T* tw_z(const DevGeom& g);
template <>
__device__ __forceinline__ const double* tw_z<double>(const DevGeom& g) { return g.tw_z; }
template <>
__device__ __forceinline__ const float* tw_z<float>(const DevGeom& g) { return g.tw_z_f; }
template <typename T>
__device__ __forceinline__ const T* tw_t(const DevGeom& g);
template <>
__device__ __forceinline__ const double* tw_t<double>(const DevGeom& g) { return g.tw_theta; }
template <>
__device__ __forceinline__ const float* tw_t<float>(const DevGeom& g) { return g.tw_theta_f; }

// Wavenumber coefficients at radius R: k^2, a = 1/k^2 and its analytic
// r-derivatives a1, a2, a3 (s = alpha^2 R^2 + m^2, a = R^2 / s).
struct Wn {
    double k2, a, a1, a2, a3;
};
__device__ __forceinline__ Wn wavecoef(double m, double al, double R) {
    const double m2 = m * m, aR2 = al * al * R * R;
    const double s = aR2 + m2;
    const double is = 1.0 / s;
    Wn w;
    w.k2 = s / (R * R);
    w.a = R * R * is;
    w.a1 = 2.0 * m2 * R * is * is;
    w.a2 = 2.0 * m2 * (m2 - 3.0 * aR2) * is * is * is;
    w.a3 = -24.0 * m2 * al * al * R * (m2 - aR2) * is * is * is * is;
    return w;
}

// a = 1/k^2 = R^2 / (alpha^2 R^2 + m^2) of mode (m, alpha) at radius R.  Here
// and in recover the multiply-adds are written as fused ones, so that every
// kernel (and every tile shape of one) rounds them alike rather than as the
// compiler's contraction of each instance happens to pair them.
__device__ __forceinline__ double inv_k2(double R, double m, double al) {
    return R * R / fma(al * al * R, R, m * m);
}

// u, w from v, eta and D v (continuity and the definition of eta):
// u = (i alpha D_* v - (i m / R) eta) a,  w = ((i m / R) D_* v + i alpha eta) a.
__device__ __forceinline__ void recover(cd v, cd eta, cd dv, double R, double m, double al, double a,
                                        cd& u, cd& w) {
    const cd ds = {dv.x + v.x / R, dv.y + v.y / R};
    const double mr = m / R;
    u.x = fma(mr, eta.y, -(al * ds.y)) * a;
    u.y = fma(al, ds.x, -(mr * eta.x)) * a;
    w.x = fma(-mr, ds.y, -(al * eta.y)) * a;
    w.y = fma(mr, ds.x, al * eta.x) * a;
}

// ---------------------------------------------------------------- k_dv
// Rows are processed in chunks of DV_CH whose loads are issued together, so
// one memory latency is paid per chunk rather than per row.
constexpr int DV_CH = 8;

__global__ __launch_bounds__(NT) void k_dv(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const cd* __restrict__ v = b.v;
    cd* __restrict__ dv = b.dv;
    const int mode = blockIdx.x * NT + threadIdx.x;
    if (mode >= g.P) return;
    const int nr = g.nr;
    const size_t P = g.P;
    const double* d0 = g.coef;
    const double* d1 = g.coef + (size_t)1 * nr * 5;
    if (mode == g.mean) {
        for (int n = 0; n < nr; ++n) dv[n * P + mode] = cd{0.0, 0.0};
        return;
    }
    cd e1 = {0.0, 0.0}, el = {0.0, 0.0};
    for (int j = 0; j < 5; ++j) {
        e1 = cfma(d1[1 * 5 + j], v[(size_t)(g.sigma[1] + j) * P + mode], e1);
        el = cfma(d1[(nr - 2) * 5 + j], v[(size_t)(g.sigma[nr - 2] + j) * P + mode], el);
    }
    dv[mode] = cd{0.0, 0.0};
    dv[1 * P + mode] = e1;
    dv[(size_t)(nr - 2) * P + mode] = el;
    dv[(size_t)(nr - 1) * P + mode] = cd{0.0, 0.0};
    // rolling window w[0..3] = v[n-2 .. n+1]; v[n+2] arrives from the chunk
    cd w0 = v[0 * P + mode], w1 = v[1 * P + mode], w2 = v[2 * P + mode], w3 = v[3 * P + mode];
    cd y1 = {0.0, 0.0}, y2 = {0.0, 0.0};
    for (int n0 = 2; n0 <= nr - 3; n0 += DV_CH) {
        cd vin[DV_CH];
#pragma unroll
        for (int c = 0; c < DV_CH; ++c) {
            const int m = n0 + c + 2;
            vin[c] = m <= nr - 1 ? v[(size_t)m * P + mode] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int c = 0; c < DV_CH; ++c) {
            const int n = n0 + c;
            if (n > nr - 3) break;
            const cd w4 = vin[c];
            const double* k1 = d1 + n * 5;
            const double* k0 = d0 + n * 5;
            cd rhs = cfma(k1[0], w0, cfma(k1[1], w1, cfma(k1[2], w2, cfma(k1[3], w3, cfma(k1[4], w4, cd{0, 0})))));
            // known D v at rows 1 and nr-2 move to the right-hand side
            if (n - 2 <= 1 && n + 2 >= 1) rhs = cfma(-k0[1 - (n - 2)], e1, rhs);
            if (n - 2 <= nr - 2 && n + 2 >= nr - 2) rhs = cfma(-k0[nr - 2 - (n - 2)], el, rhs);
            const double* L = g.blu + n * 5;
            const cd y = cfma(-L[0], y2, cfma(-L[1], y1, rhs));
            dv[(size_t)n * P + mode] = y;
            y2 = y1;
            y1 = y;
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = w4;
        }
    }
    cd x1 = {0.0, 0.0}, x2 = {0.0, 0.0};
    for (int n0 = nr - 3; n0 >= 2; n0 -= DV_CH) {
        cd yin[DV_CH];
#pragma unroll
        for (int c = 0; c < DV_CH; ++c) {
            const int n = n0 - c;
            yin[c] = n >= 2 ? dv[(size_t)n * P + mode] : cd{0.0, 0.0};
        }
#pragma unroll
        for (int c = 0; c < DV_CH; ++c) {
            const int n = n0 - c;
            if (n < 2) break;
            const double* L = g.blu + n * 5;
            const cd t = cfma(-L[4], x2, cfma(-L[3], x1, yin[c]));
            const cd x = {t.x * L[2], t.y * L[2]};
            dv[(size_t)n * P + mode] = x;
            x2 = x1;
            x1 = x;
        }
    }
}

// D v with the d0 system swept in DV_SEGMENTS segments of L rows of the
// centred block (rows 2..nr-3).  Wavefront w of a block owns segment w of the
// same 64 modes (one lane per mode), so a mode's segments meet in LDS.  Each
// lane forms its rows' right-hand sides d1 v from a register window of v,
// runs the forward recurrence from zero carry-in, and adds the carried-in
// values times the segment responses (host table dvh) once the chain of
// segment end values has been resolved through LDS; the back substitution
// goes the same way in the other direction.  v is read once (plus a 4-row
// halo per segment), D v written once, and all rows of a mode are in flight
// together.  The mean slot of v is zero, so it needs no branch.
template <int L, int DV_SEGMENTS>
__global__ __launch_bounds__(64 * DV_SEGMENTS) void k_dv_seg(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const auto* __restrict__ v = glb(b.v);
    auto* __restrict__ dv = glb(b.dv);
    // segment end values: forward sweep (xc) and back substitution (xb) in
    // separate arrays, so the second exchange needs no barrier before it
    __shared__ cd xc[DV_SEGMENTS][2][64];
    __shared__ cd xb[DV_SEGMENTS][2][64];
    if ((int)blockIdx.x * 64 >= g.P) return;  // past this instance's modes (whole block)
    const int seg = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x & 63;
    const int nr = g.nr;
    const size_t P = g.P;
    const int m0 = blockIdx.x * 64 + lane;
    const bool act = m0 < g.P;
    const size_t mode = act ? m0 : g.P - 1;  // idle lanes read a valid column
    const int s0 = 2 + seg * L;
    const int len = max(0, min(s0 + L, nr - 2) - s0);
    const auto* __restrict__ d0 = glb(g.coef);
    const auto* __restrict__ d1 = glb(g.coef) + (size_t)nr * 5;
    const auto* __restrict__ blu = glb(g.blu);
    const auto* __restrict__ hf1 = glb(g.dvh);
    const auto* __restrict__ hf2 = glb(g.dvh) + nr;
    const auto* __restrict__ hb1 = glb(g.dvh) + 2 * nr;
    const auto* __restrict__ hb2 = glb(g.dvh) + 3 * nr;
    cd p[L];
#pragma unroll
    for (int i = 0; i < L; ++i) p[i] = cd{0, 0};
    cd e1 = {0, 0}, el = {0, 0};  // D v at rows 1 and nr-2 (explicit rows)
    if (len > 0) {
        cd w[L + 4];  // v at rows s0-2 .. s0+L+1 (clamped to the grid)
#pragma unroll
        for (int t = 0; t < L + 4; ++t) w[t] = v[(size_t)min(s0 - 2 + t, nr - 1) * P + mode];
        if (seg == 0)
#pragma unroll
            for (int j = 0; j < 5; ++j) e1 = cfma(d1[1 * 5 + j], w[j], e1);
        if (s0 + len > nr - 4)
#pragma unroll
            for (int j = 0; j < 5; ++j) el = cfma(d1[(size_t)(nr - 2) * 5 + j], v[(size_t)(nr - 5 + j) * P + mode], el);
        cd y1 = {0, 0}, y2 = {0, 0};
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int n = s0 + i;
            if (i < len) {
                const auto* k1 = d1 + (size_t)n * 5;
                cd rhs = cfma(k1[0], w[i], cfma(k1[1], w[i + 1], cfma(k1[2], w[i + 2],
                         cfma(k1[3], w[i + 3], cfma(k1[4], w[i + 4], cd{0, 0})))));
                // the known D v at rows 1 and nr-2 move to the right-hand side
                if (n <= 3) rhs = cfma(-d0[(size_t)n * 5 + (3 - n)], e1, rhs);
                if (n >= nr - 4) rhs = cfma(-d0[(size_t)n * 5 + (nr - n)], el, rhs);
                const cd y = cfma(-blu[(size_t)n * 5 + 0], y2, cfma(-blu[(size_t)n * 5 + 1], y1, rhs));
                p[i] = y;
                y2 = y1;
                y1 = y;
            }
        }
    }
    // forward carries: segment t's end values (y_{t1-1}, y_{t1-2}) with zero carry-in
    xc[seg][0][lane] = p[L - 1];
    xc[seg][1][lane] = p[L - 2];
    __syncthreads();
    cd c1 = {0, 0}, c2 = {0, 0};  // y_{s0-1}, y_{s0-2}: every earlier segment is full
    for (int t = 0; t < (len > 0 ? seg : 0); ++t) {
        const int te = 2 + (t + 1) * L - 1;
        const cd n1 = cfma(hf1[te], c1, cfma(hf2[te], c2, xc[t][0][lane]));
        const cd n2 = cfma(hf1[te - 1], c1, cfma(hf2[te - 1], c2, xc[t][1][lane]));
        c1 = n1;
        c2 = n2;
    }
#pragma unroll
    for (int i = 0; i < L; ++i)
        if (i < len) p[i] = cfma(hf1[s0 + i], c1, cfma(hf2[s0 + i], c2, p[i]));
    {
        cd q1 = {0, 0}, q2 = {0, 0};
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            if (i < len) {
                const auto* o = blu + (size_t)(s0 + i) * 5;
                const cd t = cfma(-o[4], q2, cfma(-o[3], q1, p[i]));
                const cd q = {t.x * o[2], t.y * o[2]};
                p[i] = q;
                q2 = q1;
                q1 = q;
            }
        }
    }
    // backward carries: (x_{t0}, x_{t0+1}) of segment t with zero carry-in
    xb[seg][0][lane] = p[0];
    xb[seg][1][lane] = p[1];
    __syncthreads();
    cd d1c = {0, 0}, d2c = {0, 0};  // x_{s1}, x_{s1+1}; zero beyond the last non-empty segment
    if (!act || len == 0) return;
    for (int t = DV_SEGMENTS - 1; t > seg; --t) {
        const int t0 = 2 + t * L;
        if (t0 >= nr - 2) continue;  // empty segment: carries pass through
        const cd n1 = cfma(hb1[t0], d1c, cfma(hb2[t0], d2c, xb[t][0][lane]));
        const cd n2 = cfma(hb1[t0 + 1], d1c, cfma(hb2[t0 + 1], d2c, xb[t][1][lane]));
        d1c = n1;
        d2c = n2;
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
        if (i < len) {
            const int n = s0 + i;
            dv[(size_t)n * P + mode] = cfma(hb1[n], d1c, cfma(hb2[n], d2c, p[i]));
        }
    }
    if (seg == 0) {
        dv[mode] = cd{0, 0};
        dv[P + mode] = e1;
    }
    if (s0 + len == nr - 2) {
        dv[(size_t)(nr - 2) * P + mode] = el;
        dv[(size_t)(nr - 1) * P + mode] = cd{0, 0};
    }
}

// ---------------------------------------------------------------- k_zinv
template <typename T>
__global__ __launch_bounds__(NT) void k_zinv(const InstDev* __restrict__ I, int jb) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const cd* __restrict__ v = b.v;
    const cd* __restrict__ eta = b.eta;
    const cd* __restrict__ dv = b.dv;
    const double* __restrict__ umean = b.umean;
    const double* __restrict__ wmean = b.wmean;
    C<T>* __restrict__ zb = (C<T>*)b.zb;
    extern __shared__ __align__(16) char smem_raw[];
    C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
    const int r = blockIdx.y;
    const int j0 = blockIdx.x * jb;
    const int nz = g.nz, kz = g.kz, nl = g.nl, nj = g.nj;
    const int ncols = min(jb, nj - j0);
    const double R = g.r[r];
    const size_t P = g.P;
    const T* tw = tw_z<T>(g);
    for (int f = 0; f < 3; ++f) {
        for (int idx = threadIdx.x; idx < ncols * nz; idx += NT) {
            const int col = idx / nz;
            const int q = idx - col * nz;
            const int l = q <= kz ? q : q - nz;
            C<T> val = {(T)0, (T)0};
            if (l >= -kz) {
                const int j = j0 + col;
                const size_t e = (size_t)r * P + (size_t)j * nl + (l + kz);
                if (j == 0 && l == 0) {
                    if (f == 0) val.x = (T)umean[r];
                    if (f == 2) val.x = (T)wmean[r];
                } else if (f == 1) {
                    val = C<T>{(T)v[e].x, (T)v[e].y};
                } else {
                    const double m = g.m[j], al = g.alpha[l + kz];
                    const double a = inv_k2(R, m, al);
                    cd u, w;
                    recover(v[e], eta[e], dv[e], R, m, al, a, u, w);
                    const cd s = f == 0 ? u : w;
                    val = C<T>{(T)s.x, (T)s.y};
                }
            }
            buf[col * nz + q] = val;
        }
        __syncthreads();
        fft_lds<T, ZELEMS>(buf, ncols, g.plan_z, +1, tw);
        C<T>* out = zb + ((size_t)f * g.nr + r) * nz * nj;
        for (int idx = threadIdx.x; idx < ncols * nz; idx += NT) {
            const int z = idx / ncols;
            const int col = idx - z * ncols;
            out[(size_t)z * nj + j0 + col] = buf[col * nz + z];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- k_theta
template <typename T>
__device__ __forceinline__ C<T> pmul(C<T> a, C<T> b) { return {a.x * b.x, a.y * b.y}; }

// Unpack the forward transforms of packed row pairs and write j = 0..K_theta
// of rows z0 and z0 + 1 of the products f0..f0+2.
template <typename T>
__device__ __forceinline__ void theta_write(const DevGeom& g, const C<T>* buf, C<T>* pb, int r, int z0, int f0) {
    const int N = g.ntheta, nj = g.nj;
    for (int idx = threadIdx.x; idx < 3 * nj; idx += NT) {
        const int f = idx / nj;
        const int j = idx - f * nj;
        const C<T> h = buf[f * N + j];
        const C<T> hm = buf[f * N + (j == 0 ? 0 : N - j)];
        const C<T> p0 = {(T)0.5 * (h.x + hm.x), (T)0.5 * (h.y - hm.y)};
        const C<T> p1 = {(T)0.5 * (h.y + hm.y), (T)0.5 * (hm.x - h.x)};
        C<T>* out = pb + (((size_t)(f0 + f) * g.nr + r) * g.nz + z0) * nj;
        out[j] = p0;
        out[nj + j] = p1;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_theta(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const C<T>* __restrict__ zb = (const C<T>*)b.zb;
    C<T>* __restrict__ pb = (C<T>*)b.pb;
    extern __shared__ __align__(16) char smem_raw[];
    C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
    const int r = blockIdx.y;
    const int z0 = 2 * blockIdx.x;
    const int N = g.ntheta, kt = g.kt, nj = g.nj, nz = g.nz;
    const T* tw = tw_t<T>(g);
    for (int idx = threadIdx.x; idx < 3 * N; idx += NT) {
        const int f = idx / N;
        const int p = idx - f * N;
        const C<T>* row0 = zb + (((size_t)f * g.nr + r) * nz + z0) * nj;
        const C<T>* row1 = row0 + nj;
        C<T> h = {(T)0, (T)0};
        if (p <= kt) {
            C<T> a = row0[p], b = row1[p];
            if (p == 0) {
                a.y = (T)0;
                b.y = (T)0;
            }
            h = C<T>{a.x - b.y, a.y + b.x};
        } else if (p >= N - kt) {
            const int jj = N - p;
            const C<T> a = row0[jj], b = row1[jj];
            // conj(a) + i conj(b)
            h = C<T>{a.x + b.y, b.x - a.y};
        }
        buf[f * N + p] = h;
    }
    __syncthreads();
    fft_lds<T, TELEMS>(buf, 3, g.plan_theta, +1, tw);

    constexpr int MAXP = MAX_FFT / NT;
    C<T> keep[MAXP][3];
#pragma unroll
    for (int t = 0; t < MAXP; ++t) {
        const int p = threadIdx.x + t * NT;
        if (p < N) {
            const C<T> u = buf[p], vv = buf[N + p], w = buf[2 * N + p];
            buf[p] = pmul(u, u);
            buf[N + p] = pmul(u, vv);
            buf[2 * N + p] = pmul(u, w);
            keep[t][0] = pmul(vv, vv);
            keep[t][1] = pmul(vv, w);
            keep[t][2] = pmul(w, w);
        }
    }
    __syncthreads();
    fft_lds<T, TELEMS>(buf, 3, g.plan_theta, -1, tw);
    theta_write<T>(g, buf, pb, r, z0, 0);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXP; ++t) {
        const int p = threadIdx.x + t * NT;
        if (p < N) {
            buf[p] = keep[t][0];
            buf[N + p] = keep[t][1];
            buf[2 * N + p] = keep[t][2];
        }
    }
    __syncthreads();
    fft_lds<T, TELEMS>(buf, 3, g.plan_theta, -1, tw);
    theta_write<T>(g, buf, pb, r, z0, 3);
}

// ---------------------------------------------------------------- k_zfwd
template <typename T>
__global__ __launch_bounds__(NT) void k_zfwd(const InstDev* __restrict__ I, int jb) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const C<T>* __restrict__ pb = (const C<T>*)b.pb;
    C<T>* __restrict__ ps = (C<T>*)b.ps;
    extern __shared__ __align__(16) char smem_raw[];
    C<T>* buf = reinterpret_cast<C<T>*>(smem_raw);
    const int r = blockIdx.y;
    const int j0 = blockIdx.x * jb;
    const int nz = g.nz, kz = g.kz, nl = g.nl, nj = g.nj;
    const int ncols = min(jb, nj - j0);
    const size_t P = g.P;
    const T scale = (T)(1.0 / ((double)g.ntheta * (double)g.nz));
    const T* tw = tw_z<T>(g);
    for (int f = 0; f < 6; ++f) {
        const C<T>* in = pb + ((size_t)f * g.nr + r) * nz * nj;
        for (int idx = threadIdx.x; idx < ncols * nz; idx += NT) {
            const int z = idx / ncols;
            const int col = idx - z * ncols;
            buf[col * nz + z] = in[(size_t)z * nj + j0 + col];
        }
        __syncthreads();
        fft_lds<T, ZELEMS>(buf, ncols, g.plan_z, -1, tw);
        C<T>* out = ps + (size_t)f * g.nr * P + (size_t)r * P;
        for (int idx = threadIdx.x; idx < ncols * nl; idx += NT) {
            const int col = idx / nl;
            const int li = idx - col * nl;
            const int l = li - kz;
            const int q = l < 0 ? l + nz : l;
            out[(size_t)(j0 + col) * nl + li] = cscale(buf[col * nz + q], scale);
        }
        __syncthreads();
    }
}

// Index of the precomputed unpivoted LU factors of the Crank--Nicolson
// systems: for substep k and equation e (0: v or the mean u, 1: eta or the
// mean w), the fields {l2, l1, 1/u0, u1, u2} of every row and mode pair.
__device__ __forceinline__ size_t lu_index(const DevGeom& g, int k, int eqn, int field, int i, int pair) {
    return ((((size_t)k * 2 + eqn) * 5 + field) * g.nr + i) * g.npairs + pair;
}

// ---------------------------------------------------------------- k_rhs
// One lane per (mode, chunk of rr consecutive rows of 2..nr-3, the rows
// whose 5-point stencils are centred).  The lane walks the chunk's rr + 4
// stencil points in increasing r, forms the per-point operands of every
// compact family once, and scatters them into the accumulators of the five
// rows whose stencil contains the point.  Row cc of the chunk lives in
// accumulator slot (cc + pad) mod 5: its first point assigns the slot, its
// fifth finishes it and the row is written at once, so five rows of
// accumulators are live.  The point loop is unrolled by the slot period only,
// which keeps the kernel small enough for the instruction cache; when the
// rr + 4 points are not whole periods the walk starts pad < 5 points early.
// Slots of rows outside the chunk collect values that are never written.  Every chunk is full length: the last one is shifted down to end at
// row nr-3 and may recompute rows of its neighbour, writing bit-identical
// values (the kernel reads nothing it writes).  The first chunk also writes
// the off-centre eta row 1 and the zero row 0, the last chunk the eta row
// nr-2 and the zero row nr-1.  Lanes are laid out chunk-major over the mode
// count rounded up to whole wavefronts, so the chunk is wave-uniform and
// coefficient and grid reads are scalar.  The mean (0,0) mode's rows are
// independent of each other and are done by the blocks with blockIdx.y = 1,
// one lane per row.
//
// The explicit-term registers N alternate between two buffers: substep 0
// writes n[0] (its rho is zero, so nothing is read), substep 1 reads n[0]
// and writes n[1], substep 2 reads n[1] and writes nothing (the next
// substep 0 does not read it).

// mean (0,0) mode: mean axial and azimuthal momentum, one row
template <typename TP, int K>
__device__ __forceinline__ void rhs_mean_row(const DevGeom& g, const DevBuf& b, const TC_GLOBAL C<TP>* __restrict__ ps,
                                             const StepCoef& sc, int n) {
    const size_t P = g.P;
    const int nr = g.nr;
    const int mode = g.mean;
    const size_t gid = (size_t)n * P + mode;
    const size_t S = (size_t)nr * P;
    const double bdt = sc.beta * g.dt * g.nu;
    cd rv = {0.0, 0.0}, re = {0.0, 0.0};
    cd fnu = {0.0, 0.0}, fnw = {0.0, 0.0};
    if (n >= 1 && n <= nr - 2) {
        const int s = g.sigma[n];
        const double* d0 = g.coef + ((size_t)0 * nr + n) * 5;
        const double* d1 = g.coef + ((size_t)1 * nr + n) * 5;
        const double* d2s = g.coef + ((size_t)3 * nr + n) * 5;
        double iu = 0, iw = 0, fu = 0, fw = 0;
        for (int jj = 0; jj < 5; ++jj) {
            const int m = s + jj;
            const double R = g.r[m];
            const double um = b.umean[m], wm = b.wmean[m];
            const double uv = (double)ps[1 * S + (size_t)m * P + mode].x;
            const double vw = (double)ps[4 * S + (size_t)m * P + mode].x;
            iu += d0[jj] * (um + bdt * um / (R * R)) + d2s[jj] * (bdt * um);
            iw += d0[jj] * wm + d2s[jj] * (bdt * wm);
            fu -= d1[jj] * uv + d0[jj] * (uv / R);
            fw -= d1[jj] * vw + d0[jj] * (2.0 * vw / R);
        }
        double pu = 0.0, pw = 0.0;
        if (K > 0) {
            pu = b.nmean[((size_t)(K - 1) * 2 + 0) * nr + n];
            pw = b.nmean[((size_t)(K - 1) * 2 + 1) * nr + n];
        }
        rv.x = iu + g.dt * (sc.gamma * fu + sc.rho * pu);
        re.x = iw + g.dt * (sc.gamma * fw + sc.rho * pw);
        fnu.x = fu;
        fnw.x = fw;
    }
    if (K < 2) {  // the mean flow's explicit terms stay FP64 in both precisions
        b.nmean[((size_t)K * 2 + 0) * nr + n] = fnu.x;
        b.nmean[((size_t)K * 2 + 1) * nr + n] = fnw.x;
    }
    b.rv[gid] = rv;
    b.re[gid] = re;
}

template <typename TP>
struct RhsPoint {
    cd v, eta, dv;
    C<TP> UU, UV, UW, VV, VW, WW;
};

template <typename TP>
__device__ __forceinline__ void rhs_load(const TC_GLOBAL cd* __restrict__ v, const TC_GLOBAL cd* __restrict__ eta,
                                         const TC_GLOBAL cd* __restrict__ dv, const TC_GLOBAL C<TP>* __restrict__ ps,
                                         size_t S, size_t e,
                                         RhsPoint<TP>& p) {
    p.v = v[e];
    p.eta = eta[e];
    p.dv = dv[e];
    p.UU = ps[e];
    p.UV = ps[S + e];
    p.UW = ps[2 * S + e];
    p.VV = ps[3 * S + e];
    p.VW = ps[4 * S + e];
    p.WW = ps[5 * S + e];
}

// per-point operands of eq. (final-v) and eq. (final-eta): the weights of
// each compact family in the explicit half of the Crank--Nicolson operator,
// and the nonlinear-plus-explicit-viscous vectors multiplied by d0, d1, d2, d2s
struct RhsOps {
    cd v, eta, ne0, ne1, nv0, nv1, nv2, nv2s;
    double ke0, kv0, kv1, kv2s, kv4s;
};

template <typename TP>
__device__ __forceinline__ RhsOps rhs_ops(const RhsPoint<TP>& p, double R, double mm, double al, double nu,
                                          double bdt) {
    const cd UU = {(double)p.UU.x, (double)p.UU.y}, UV = {(double)p.UV.x, (double)p.UV.y};
    const cd UW = {(double)p.UW.x, (double)p.UW.y}, VV = {(double)p.VV.x, (double)p.VV.y};
    const cd VW = {(double)p.VW.x, (double)p.VW.y}, WW = {(double)p.WW.x, (double)p.WW.y};
    const Wn wc = wavecoef(mm, al, R);
    cd u, w;
    recover(p.v, p.eta, p.dv, R, mm, al, wc.a, u, w);
    const double iR = 1.0 / R, iR2 = iR * iR, iR3 = iR2 * iR;
    const cd iu = ci(u), iUV = ci(UV), iVW = ci(VW), iw = ci(w);
    RhsOps o;
    o.v = p.v;
    o.eta = p.eta;
    // eta equation (eq. (final-eta)): implicit d0, d2s; explicit d0, d1
    o.ke0 = 1.0 - bdt * wc.k2;
    cd ne0 = cfma(4.0 * nu * mm * iR3, iu, cd{0, 0});
    ne0 = cfma(2.0 * nu * mm * al * iR2, p.v, ne0);
    ne0 = cfma(mm * al * iR, UU, ne0);
    ne0 = cfma(-2.0 * mm * iR2, iUV, ne0);
    ne0 = cfma(mm * mm * iR2 - al * al, UW, ne0);
    ne0 = cfma(-al * mm * iR, WW, ne0);
    o.ne0 = cfma(2.0 * al * iR, iVW, ne0);
    cd ne1 = cfma(2.0 * nu * mm * iR2, iu, cd{0, 0});
    ne1 = cfma(-mm * iR, iUV, ne1);
    o.ne1 = cfma(al, iVW, ne1);
    // v equation (eq. (final-v)): implicit d0, d1, d2s, d4s; explicit d0, d1, d2, d2s
    const cd c = {-al * u.y - mm * iR * w.y, al * u.x + mm * iR * w.x};  // i alpha u + i (m/R) w
    o.kv0 = 1.0 - bdt * wc.k2;
    o.kv1 = wc.a1 + bdt * (wc.a2 * iR + wc.a3 - wc.a1 * iR2 - 2.0 * mm * mm * wc.a * iR3);
    o.kv2s = -wc.a + bdt * (2.0 - 2.0 * wc.a1 * iR);
    o.kv4s = -bdt * wc.a;
    cd nv0 = cfma(-2.0 * nu * mm * iR2, iw, cd{0, 0});
    nv0 = cfma(-al, iUV, nv0);
    nv0 = cfma(-mm * iR, iVW, nv0);
    nv0 = cfma(-iR, VV, nv0);
    o.nv0 = cfma(iR, WW, nv0);
    cd nv1 = cfma(2.0 * nu * mm * (wc.a * iR3 - wc.a1 * iR2), iw, cd{0, 0});
    nv1 = cfma(al * wc.a1, iUV, nv1);
    nv1 = cfma(mm * (wc.a1 * iR - 3.0 * wc.a * iR2), iVW, nv1);
    nv1 = cfma(wc.a * al * al, UU, nv1);
    nv1 = cfma(wc.a * 2.0 * al * mm * iR, UW, nv1);
    nv1 = cfma(wc.a * mm * mm * iR2, WW, nv1);
    o.nv1 = cfma(-1.0, VV, nv1);
    cd nv2 = cfma(2.0 * nu * mm * wc.a * iR2, iw, cd{0, 0});
    o.nv2 = cfma(-mm * wc.a * iR, iVW, nv2);
    cd nv2s = cfma(-3.0 * nu * wc.a1, c, cd{0, 0});
    o.nv2s = cfma(-al * wc.a, iUV, nv2s);
    return o;
}

struct RhsAcc {
    cd Iv, Nv, Ie, Ne;
};

// eta row: co points at the coefficient of stencil point jj of the row
__device__ __forceinline__ void rhs_acc_eta(RhsAcc& A, const RhsOps& o, const TC_CONST double* co, size_t fs,
                                            double bdt) {
    const double c0 = co[0], c1 = co[fs], c2s = co[3 * fs];
    A.Ie = cfma(c0 * o.ke0 + c2s * bdt, o.eta, A.Ie);
    A.Ne = cfma(c0, o.ne0, cfma(c1, o.ne1, A.Ne));
}

__device__ __forceinline__ void rhs_acc_both(RhsAcc& A, const RhsOps& o, const TC_CONST double* co, size_t fs,
                                             double bdt) {
    const double c0 = co[0], c1 = co[fs], c2 = co[2 * fs], c2s = co[3 * fs], c4s = co[4 * fs];
    A.Ie = cfma(c0 * o.ke0 + c2s * bdt, o.eta, A.Ie);
    A.Ne = cfma(c0, o.ne0, cfma(c1, o.ne1, A.Ne));
    A.Iv = cfma(c0 * o.kv0 + c1 * o.kv1 + c2s * o.kv2s + c4s * o.kv4s, o.v, A.Iv);
    A.Nv = cfma(c0, o.nv0, cfma(c1, o.nv1, cfma(c2, o.nv2, cfma(c2s, o.nv2s, A.Nv))));
}

template <typename TP>
__device__ __forceinline__ C<TP> narrow(cd z) { return C<TP>{(TP)z.x, (TP)z.y}; }
template <typename TP>
__device__ __forceinline__ cd widen(C<TP> z) { return cd{(double)z.x, (double)z.y}; }

// right-hand side of one row: (M + beta dt nu L) q + dt (gamma N + rho N_prev),
// r for v (zero on the wall-derivative rows, vrow false) and q for eta
template <int K>
__device__ __forceinline__ void rhs_values(const RhsAcc& A, bool vrow, cd pv, cd pe, double dt, const StepCoef& sc,
                                           cd& r, cd& q) {
    r = cd{0, 0};
    if (vrow) r = cfma(dt * sc.gamma, A.Nv, K > 0 ? cfma(dt * sc.rho, pv, A.Iv) : A.Iv);
    q = cfma(dt * sc.gamma, A.Ne, K > 0 ? cfma(dt * sc.rho, pe, A.Ie) : A.Ie);
}

// the explicit terms of one row into the N registers of the next substep
template <typename TP, int K>
__device__ __forceinline__ void n_store(TC_GLOBAL C<TP>* __restrict__ nv, TC_GLOBAL C<TP>* __restrict__ ne, size_t gid,
                                        bool vrow, const RhsAcc& A) {
    if (K < 2) {
        nv[gid] = narrow<TP>(vrow ? A.Nv : cd{0, 0});
        ne[gid] = narrow<TP>(A.Ne);
    }
}

template <typename TP, int K>
__device__ __forceinline__ void rhs_store(TC_GLOBAL C<TP>* __restrict__ nv, TC_GLOBAL C<TP>* __restrict__ ne,
                                          TC_GLOBAL cd* __restrict__ rv, TC_GLOBAL cd* __restrict__ re, size_t gid, bool vrow, const RhsAcc& A, cd pv,
                                          cd pe, double dt, const StepCoef& sc) {
    cd r, q;
    rhs_values<K>(A, vrow, pv, pe, dt, sc, r, q);
    n_store<TP, K>(nv, ne, gid, vrow, A);
    rv[gid] = r;
    re[gid] = q;
}

// The forward elimination of the Crank--Nicolson systems of v and eta run
// along a column as its right-hand-side rows complete (rows in increasing
// order): y_n = r_n - l1_n y_{n-1} - l2_n y_{n-2} with the precomputed factors
// of the lane's pair, row 1 folded with the raw row 2 and row nr-2 with the
// raw row nr-3 first (the same folds the solve would apply).  rv / re then
// hold y and the solve only substitutes back.
struct FwdState {
    cd y1v, y2v, y1e, y2e;  // y_{n-1}, y_{n-2} of v and eta
    cd rv_raw, re_raw;      // the last raw right-hand sides (row nr-3 when the walk ends)
    double lv2, lv1, le2, le1;  // factors of the next row to complete
};
struct FwdArgs {
    const TC_GLOBAL double* __restrict__ lv;  // l2 of eqn v at row 0 of the lane's pair (l1: + lfs)
    const TC_GLOBAL double* __restrict__ le;  // the same for eta
    size_t lfs, lrs;                          // field and row strides of the factor table
    double f0v, f0e, f1v, f1e;                // fold factors of rows 1 and nr-2
};
__device__ __forceinline__ void fwd_fetch(FwdState& F, const FwdArgs& fa, int n) {
    const size_t o = (size_t)max(n, 0) * fa.lrs;
    F.lv2 = fa.lv[o];
    F.lv1 = fa.lv[fa.lfs + o];
    F.le2 = fa.le[o];
    F.le1 = fa.le[fa.lfs + o];
}
// row n's raw (r, q) -> y, written to rv / re at gid
__device__ __forceinline__ void fwd_row(FwdState& F, TC_GLOBAL cd* __restrict__ rv, TC_GLOBAL cd* __restrict__ re,
                                        size_t gid, cd r, cd q, double lv2, double lv1, double le2, double le1) {
    const cd yv = cfma(-lv2, F.y2v, cfma(-lv1, F.y1v, r));
    const cd ye = cfma(-le2, F.y2e, cfma(-le1, F.y1e, q));
    rv[gid] = yv;
    re[gid] = ye;
    F.y2v = F.y1v;
    F.y1v = yv;
    F.y2e = F.y1e;
    F.y1e = ye;
    F.rv_raw = r;
    F.re_raw = q;
}

template <typename TP, int K>
__device__ __forceinline__ void rhs_zero_row(TC_GLOBAL C<TP>* __restrict__ nv, TC_GLOBAL C<TP>* __restrict__ ne,
                                             TC_GLOBAL cd* __restrict__ rv, TC_GLOBAL cd* __restrict__ re, size_t gid) {
    if (K < 2) {
        nv[gid] = C<TP>{(TP)0, (TP)0};
        ne[gid] = C<TP>{(TP)0, (TP)0};
    }
    rv[gid] = cd{0, 0};
    re[gid] = cd{0, 0};
}

// An empty asm statement that takes the accumulators as read-write register
// operands: it pins each accumulation where it is written.  Without it the
// compiler sinks the accumulations towards the (later, sometimes
// conditional) stores and keeps several stencil points' operands live
// instead of one row's accumulator.
__device__ __forceinline__ void pin_eta(RhsAcc& A) {
    asm volatile("" : "+v"(A.Ie.x), "+v"(A.Ie.y), "+v"(A.Ne.x), "+v"(A.Ne.y));
}
__device__ __forceinline__ void pin_both(RhsAcc& A) {
    asm volatile("" : "+v"(A.Ie.x), "+v"(A.Ie.y), "+v"(A.Ne.x), "+v"(A.Ne.y), "+v"(A.Iv.x), "+v"(A.Iv.y),
                 "+v"(A.Nv.x), "+v"(A.Nv.y));
}

// The lane body.  All pointers are restrict-qualified arguments, so loads of
// the next stencil point may be scheduled above the stores of finished rows;
// a scheduling barrier closes every point, so the compiler neither hoists
// further loads nor interleaves points (either would take the register count
// above two waves per SIMD).
template <typename TP, int K, bool FWD>
__device__ __forceinline__ void rhs_lane(const TC_GLOBAL cd* __restrict__ v, const TC_GLOBAL cd* __restrict__ eta,
                                         const TC_GLOBAL cd* __restrict__ dv, const TC_GLOBAL C<TP>* __restrict__ ps,
                                         const TC_GLOBAL C<TP>* __restrict__ pnv,
                                         const TC_GLOBAL C<TP>* __restrict__ pne, TC_GLOBAL C<TP>* __restrict__ nnv,
                                         TC_GLOBAL C<TP>* __restrict__ nne, TC_GLOBAL cd* __restrict__ rv,
                                         TC_GLOBAL cd* __restrict__ re, const TC_CONST double* __restrict__ coef,
                                         const TC_CONST double* __restrict__ r, int nr, int P, int mode, int n0, int rr,
                                         bool first, bool last, double mm, double al, double nu, double dt,
                                         const StepCoef& sc, const FwdArgs& fa) {
    const size_t S = (size_t)nr * P;
    const size_t fs = (size_t)nr * 5;
    const double bdt = sc.beta * dt * nu;
    const int T = rr + 4;             // stencil points of the chunk
    const int pad = (5 - T % 5) % 5;  // leading points that bring the walk to whole periods
    RhsAcc A[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) A[q] = RhsAcc{{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    RhsAcc W1 = {{0, 0}, {0, 0}, {0, 0}, {0, 0}}, W2 = W1;  // eta rows 1 and nr-2
    RhsPoint<TP> nxt;
    rhs_load<TP>(v, eta, dv, ps, S, (size_t)max(n0 - 2 - pad, 0) * P + mode, nxt);
    cd pv = {0, 0}, pe = {0, 0};
    FwdState F = {};
    cd p1 = {0, 0};  // N_prev of eta at row 1 (FWD: row 1 is eliminated with row 2)
    if constexpr (FWD) {
        if (K > 0) p1 = widen<TP>(pne[(size_t)P + mode]);
        fwd_fetch(F, fa, n0 - 4 - pad);
    }
    // point mi = base + q - pad; the pad leading points (mi < 0, rows read
    // clamped to the grid) only feed accumulators of rows before the chunk,
    // which are never written, so row cc sits in slot (cc + pad) mod 5
    for (int base = 0; base < T + pad; base += 5) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int mi = base + q - pad;
            const int m = n0 - 2 + mi;  // <= n0 + rr + 1 <= nr - 1
            const RhsPoint<TP> cur = nxt;
            rhs_load<TP>(v, eta, dv, ps, S, (size_t)min(max(m + 1, 0), nr - 1) * P + mode, nxt);
            // N_prev of the row finished at the next point (clamped row
            // index: the first three points read a row that is not used)
            cd npv = {0, 0}, npe = {0, 0};
            if (K > 0) {
                const size_t gid = (size_t)max(n0 + mi - 3, 0) * P + mode;
                npv = widen<TP>(pnv[gid]);
                npe = widen<TP>(pne[gid]);
            }
            // factors of the row finished now (fetched one point earlier) and of the next
            const double lv2 = F.lv2, lv1 = F.lv1, le2 = F.le2, le1 = F.le1;
            if constexpr (FWD) fwd_fetch(F, fa, n0 + mi - 3);
            const RhsOps o = rhs_ops<TP>(cur, r[max(m, 0)], mm, al, nu, bdt);
#pragma unroll
            for (int jj = 0; jj < 5; ++jj) {
                // row cc = mi - jj in slot (q - jj) mod 5; coefficient rows
                // of rows outside the chunk are clamped into the table
                const int slot = (q - jj + 5) % 5;
                const int n = min(max(n0 + mi - jj, 0), nr - 1);
                if (jj == 0) A[slot] = RhsAcc{{0, 0}, {0, 0}, {0, 0}, {0, 0}};
                rhs_acc_both(A[slot], o, coef + (size_t)n * 5 + jj, fs, bdt);
                pin_both(A[slot]);
            }
            if (mi >= 0 && mi < 5) {  // sigma_1 = 0: points 0..4 of the first chunk
                rhs_acc_eta(W1, o, coef + 1 * 5 + mi, fs, bdt);
                pin_eta(W1);
            }
            if (mi >= T - 5) {  // sigma_{nr-2} = nr - 5: the last five points of the last chunk
                rhs_acc_eta(W2, o, coef + (size_t)(nr - 2) * 5 + (mi - (T - 5)), fs, bdt);
                pin_eta(W2);
            }
            if (mi >= 4) {  // row mi - 4 is complete
                const size_t gid = (size_t)(n0 + mi - 4) * P + mode;
                if constexpr (!FWD) {
                    rhs_store<TP, K>(nnv, nne, rv, re, gid, true, A[(q + 1) % 5], pv, pe, dt, sc);
                } else {
                    cd r, qe;
                    rhs_values<K>(A[(q + 1) % 5], true, pv, pe, dt, sc, r, qe);
                    n_store<TP, K>(nnv, nne, gid, true, A[(q + 1) % 5]);
                    if (mi == 4) {  // row 2; row 1 (points 0..4, all in) first, folded with it
                        cd r1, q1;
                        rhs_values<K>(W1, false, cd{0, 0}, p1, dt, sc, r1, q1);
                        n_store<TP, K>(nnv, nne, (size_t)P + mode, false, W1);
                        F.y1v = cfma(-fa.f0v, r, r1);
                        F.y1e = cfma(-fa.f0e, qe, q1);
                        rv[(size_t)P + mode] = F.y1v;
                        re[(size_t)P + mode] = F.y1e;
                    }
                    fwd_row(F, rv, re, gid, r, qe, lv2, lv1, le2, le1);
                }
            }
            pv = npv;
            pe = npe;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if (first) {
        if constexpr (!FWD) {
            if (K > 0) p1 = widen<TP>(pne[(size_t)P + mode]);
            rhs_store<TP, K>(nnv, nne, rv, re, (size_t)P + mode, false, W1, cd{0, 0}, p1, dt, sc);
        }
        rhs_zero_row<TP, K>(nnv, nne, rv, re, (size_t)mode);
    }
    if (last) {
        cd p2 = {0, 0};
        if (K > 0) p2 = widen<TP>(pne[(size_t)(nr - 2) * P + mode]);
        if constexpr (!FWD) {
            rhs_store<TP, K>(nnv, nne, rv, re, (size_t)(nr - 2) * P + mode, false, W2, cd{0, 0}, p2, dt, sc);
        } else {  // row nr-2, folded with the raw row nr-3
            cd r2, q2;
            rhs_values<K>(W2, false, cd{0, 0}, p2, dt, sc, r2, q2);
            n_store<TP, K>(nnv, nne, (size_t)(nr - 2) * P + mode, false, W2);
            r2 = cfma(-fa.f1v, F.rv_raw, r2);
            q2 = cfma(-fa.f1e, F.re_raw, q2);
            fwd_fetch(F, fa, nr - 2);
            fwd_row(F, rv, re, (size_t)(nr - 2) * P + mode, r2, q2, F.lv2, F.lv1, F.le2, F.le1);
        }
        rhs_zero_row<TP, K>(nnv, nne, rv, re, (size_t)(nr - 1) * P + mode);
    }
}

// FWD for the mean (0,0) mode, whose rows the mean blocks form one lane per
// row: once they are all written, one lane runs the elimination of the two
// mean-profile systems (wall values moved to the right-hand side, rows 1 and
// nr-2 folded) down the column.
template <int K>
__device__ void mean_forward(const DevGeom& g, const DevBuf& b) {
    const int nr = g.nr;
    const size_t P = g.P;
    const int mode = g.mean;
    for (int eqn = 0; eqn < 2; ++eqn) {
        cd* col = eqn == 0 ? b.rv : b.re;
        const double* mw = b.mwall + ((size_t)K * 2 + eqn) * nr;
        const double* lub = b.lu + lu_index(g, K, eqn, 0, 0, 0);  // pair 0 holds the mean systems
        const size_t lfs = (size_t)nr * g.npairs;
        const double f0 = b.fold[(((size_t)K * 2 + eqn) * 2 + 0) * g.npairs];
        const double f1 = b.fold[(((size_t)K * 2 + eqn) * 2 + 1) * g.npairs];
        auto raw = [&](int n) {
            cd r = col[(size_t)n * P + mode];
            r.x -= mw[n];
            return r;
        };
        cd p1 = {0, 0}, p2 = {0, 0}, keep = {0, 0};
        for (int n = 1; n <= nr - 2; ++n) {
            cd rn = raw(n);
            if (n == 1) rn = cfma(-f0, raw(2), rn);
            if (n == nr - 2) rn = cfma(-f1, keep, rn);
            if (n == nr - 3) keep = rn;
            const double l2 = lub[(size_t)n * g.npairs], l1 = lub[lfs + (size_t)n * g.npairs];
            const cd yn = cfma(-l2, p2, cfma(-l1, p1, rn));
            col[(size_t)n * P + mode] = yn;
            p2 = p1;
            p1 = yn;
        }
    }
}

// rows per chunk (1 <= rr <= nr - 4).  Large FP64 launches take one chunk
// per column.  Otherwise the default takes rr + 4 a multiple of 5 (no
// leading points): the longest such chunk up to RHS_MAX_ROWS re-reads the
// least halo; small launches (a few hundred wavefronts) take shorter chunks,
// trading halo re-reads for wavefronts in flight.
constexpr int RHS_MAX_ROWS = 21;
constexpr int RHS_MIN_WAVES = 4096;
constexpr long long RHS_ONE_CHUNK_WAVES = 1000;

template <typename TP, int K, bool FWD>
__global__ __launch_bounds__(NT) void k_rhs(const InstDev* __restrict__ I, StepCoef sc) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const int rr = g.rhs_rr;
    const auto* __restrict__ ps = glb((const C<TP>*)b.ps);
    if (blockIdx.y == 1) {  // the mean (0,0) mode: one lane per row
        const int n = blockIdx.x * NT + threadIdx.x;
        if (n < g.nr) rhs_mean_row<TP, K>(g, b, ps, sc, n);
        if constexpr (FWD) {  // every row is in block 0 (nr <= NT)
            __syncthreads();
            if (blockIdx.x == 0 && threadIdx.x == 0) mean_forward<K>(g, b);
        }
        return;
    }
    const int P = g.P;
    const int Pp = (P + 63) & ~63;
    const int nr = g.nr;
    const int nchunk = (nr - 4 + rr - 1) / rr;
    const int gid0 = blockIdx.x * NT + threadIdx.x;
    const int chunk = __builtin_amdgcn_readfirstlane(gid0 / Pp);
    const int mode = gid0 - chunk * Pp;
    if (chunk >= nchunk || mode >= P) return;
    const int n0 = min(2 + chunk * rr, nr - 2 - rr);
    const bool first = chunk == 0, last = chunk == nchunk - 1;
    if (mode == g.mean) return;  // done by the blockIdx.y == 1 blocks
    const int j = mode / g.nl;
    const int li = mode - j * g.nl;
    using CT = C<TP>;
    FwdArgs fa = {};
    if constexpr (FWD) {
        const int lp = li >= g.kz ? li - g.kz : g.kz - li;
        const int pair = j * (g.kz + 1) + lp;
        fa.lv = glb(b.lu) + lu_index(g, K, 0, 0, 0, pair);
        fa.le = glb(b.lu) + lu_index(g, K, 1, 0, 0, pair);
        fa.lfs = (size_t)g.nr * g.npairs;
        fa.lrs = (size_t)g.npairs;
        const auto* fold = glb(b.fold);
        fa.f0v = fold[(((size_t)K * 2 + 0) * 2 + 0) * g.npairs + pair];
        fa.f1v = fold[(((size_t)K * 2 + 0) * 2 + 1) * g.npairs + pair];
        fa.f0e = fold[(((size_t)K * 2 + 1) * 2 + 0) * g.npairs + pair];
        fa.f1e = fold[(((size_t)K * 2 + 1) * 2 + 1) * g.npairs + pair];
    }
    rhs_lane<TP, K, FWD>(glb(b.v), glb(b.eta), glb(b.dv), ps, glb(K > 0 ? (const CT*)b.nv[K > 0 ? K - 1 : 0] : nullptr),
                    glb(K > 0 ? (const CT*)b.neta[K > 0 ? K - 1 : 0] : nullptr),
                    glb(K < 2 ? (CT*)b.nv[K < 2 ? K : 0] : nullptr), glb(K < 2 ? (CT*)b.neta[K < 2 ? K : 0] : nullptr),
                    glb(b.rv), glb(b.re), cst(g.coef), cst(g.r), nr, P, mode, n0, rr, first, last, glb(g.m)[j],
                    glb(g.alpha)[li], g.nu, g.dt, sc, fa);
}

// ---------------------------------------------------------------- k_solve
enum { SYS_V = 0, SYS_ETA = 1, SYS_UMEAN = 2, SYS_WMEAN = 3 };

// Row i (1..nr-2) of the Crank--Nicolson matrix M - beta dt nu L in the
// unknowns 1..nr-2: E[3 + k] is the entry of column i + k (k = -3..3); the
// wall columns 0 and nr-1 are returned separately in w0, wn.
__device__ __forceinline__ void lhs_row(const DevGeom& g, int sys, double mm, double al, double bdt, int i,
                                        double E[7], double& w0, double& wn) {
    const int nr = g.nr;
#pragma unroll
    for (int k = 0; k < 7; ++k) E[k] = 0.0;
    w0 = wn = 0.0;
    if (sys == SYS_V && (i == 1 || i == nr - 2)) {
        // v wall-derivative rows: sum_j d1[wall][j] v_{sigma+j} = 0
        const int wall = i == 1 ? 0 : nr - 1;
        const int s = g.sigma[wall];
        const double* d1 = g.coef + ((size_t)1 * nr + wall) * 5;
        for (int jj = 0; jj < 5; ++jj) {
            const int col = s + jj;
            if (col == 0) w0 += d1[jj];
            else if (col == nr - 1) wn += d1[jj];
            else E[col - i + 3] += d1[jj];
        }
        return;
    }
    const int s = g.sigma[i];
    const double* d0 = g.coef + ((size_t)0 * nr + i) * 5;
    const double* d1 = g.coef + ((size_t)1 * nr + i) * 5;
    const double* d2s = g.coef + ((size_t)3 * nr + i) * 5;
    const double* d4s = g.coef + ((size_t)4 * nr + i) * 5;
    for (int jj = 0; jj < 5; ++jj) {
        const int col = s + jj;
        const double R = g.r[col];
        double cf;
        if (sys == SYS_V) {
            const Wn wc = wavecoef(mm, al, R);
            const double iR = 1.0 / R;
            cf = d0[jj] * (1.0 + bdt * wc.k2)
               + d1[jj] * (wc.a1 - bdt * (wc.a2 * iR + wc.a3 - wc.a1 * iR * iR - 2.0 * mm * mm * wc.a * iR * iR * iR))
               + d2s[jj] * (-wc.a - bdt * (2.0 - 2.0 * wc.a1 * iR))
               + d4s[jj] * (bdt * wc.a);
        } else if (sys == SYS_ETA) {
            const double k2 = (al * al * R * R + mm * mm) / (R * R);
            cf = d0[jj] * (1.0 + bdt * k2) - d2s[jj] * bdt;
        } else if (sys == SYS_UMEAN) {
            cf = d0[jj] * (1.0 - bdt / (R * R)) - d2s[jj] * bdt;
        } else {
            cf = d0[jj] - d2s[jj] * bdt;
        }
        if (col == 0) w0 += cf;
        else if (col == nr - 1) wn += cf;
        else E[col - i + 3] += cf;
    }
}

// Rows are read in chunks of SV_CH ahead of the substitutions so that one
// memory latency is paid per chunk.
constexpr int SV_CH = 8;

// ------------------------------------------------ precomputed elimination
// The Crank--Nicolson matrices depend only on the mode pair, the equation and
// the substep (through beta_k dt nu), not on the state: their unpivoted LU
// factors are computed once per context (lu_index, with the explicit terms
// above); fold holds the two boundary-row folding factors.

__global__ __launch_bounds__(SOLVE_NT) void k_factor(DevGeom g, DevBuf b, StepCoef sc, int k) {
    const int pair = blockIdx.x * SOLVE_NT + threadIdx.x;
    if (pair >= g.npairs) return;
    const int eqn = blockIdx.y;
    const int nr = g.nr, kz = g.kz;
    const int j = pair / (kz + 1);
    const int lp = pair - j * (kz + 1);
    const bool mean = (j == 0 && lp == 0);
    const int sys = mean ? (eqn == 0 ? SYS_UMEAN : SYS_WMEAN) : (eqn == 0 ? SYS_V : SYS_ETA);
    const double q0 = sys == SYS_WMEAN ? 1.0 : 0.0;
    const double qn = sys == SYS_WMEAN ? g.w_outer : 0.0;
    const double mm = g.m[j], al = g.alpha[kz + lp];
    const double bdt = sc.beta * g.dt * g.nu;
    double id1 = 0, s11 = 0, s21 = 0, id2 = 0, s12 = 0, s22 = 0;
    double G[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 1; i <= nr - 2; ++i) {
        double E[7], w0, wn;
        lhs_row(g, sys, mm, al, bdt, i, E, w0, wn);
        // the known wall values of the mean profiles move to the right-hand side
        if (mean) b.mwall[((size_t)k * 2 + eqn) * nr + i] = w0 * q0 + wn * qn;
        if (i == 1) {
            double F[7], f0, fn;
            lhs_row(g, sys, mm, al, bdt, 2, F, f0, fn);
            const double f = E[6] / F[5];
            E[3] -= f * F[2];
            E[4] -= f * F[3];
            E[5] -= f * F[4];
            E[6] = 0.0;
            b.fold[(((size_t)k * 2 + eqn) * 2 + 0) * g.npairs + pair] = f;
        }
        if (i == nr - 2) {
            const double f = E[0] / G[1];
            E[1] -= f * G[2];
            E[2] -= f * G[3];
            E[3] -= f * G[4];
            E[0] = 0.0;
            b.fold[(((size_t)k * 2 + eqn) * 2 + 1) * g.npairs + pair] = f;
        }
        if (i == nr - 3) {
#pragma unroll
            for (int q = 0; q < 7; ++q) G[q] = E[q];
        }
        double l2 = 0.0, l1 = 0.0;
        if (i >= 3) {
            l2 = E[1] * id2;
            E[2] -= l2 * s12;
            E[3] -= l2 * s22;
        }
        if (i >= 2) {
            l1 = E[2] * id1;
            E[3] -= l1 * s11;
            E[4] -= l1 * s21;
        }
        const double id = 1.0 / E[3];
        b.lu[lu_index(g, k, eqn, 0, i, pair)] = l2;
        b.lu[lu_index(g, k, eqn, 1, i, pair)] = l1;
        b.lu[lu_index(g, k, eqn, 2, i, pair)] = id;
        b.lu[lu_index(g, k, eqn, 3, i, pair)] = E[4];
        b.lu[lu_index(g, k, eqn, 4, i, pair)] = E[5];
        id2 = id1; s12 = s11; s22 = s21;
        id1 = id;  s11 = E[4]; s21 = E[5];
    }
}

// Forward and back substitution with the precomputed factors of substep k,
// one (|l|, j) pair and one equation per lane; the (0,0) pair solves the
// mean axial (equation 0) and azimuthal (equation 1) profiles.
__global__ __launch_bounds__(SOLVE_NT) void k_solve_lu(const InstDev* __restrict__ I, int k) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const int pair = blockIdx.x * SOLVE_NT + threadIdx.x;
    if (pair >= g.npairs) return;
    const int eqn = blockIdx.y;
    const int nr = g.nr, kz = g.kz, nl = g.nl;
    const size_t P = g.P;
    const int j = pair / (kz + 1);
    const int lp = pair - j * (kz + 1);
    const bool mean = (j == 0 && lp == 0);  // mean axial (eqn 0) / azimuthal (eqn 1) profile
    const double* mwall = b.mwall + ((size_t)k * 2 + eqn) * nr;
    const int modeA = j * nl + kz + lp;
    const int modeB = j * nl + kz - lp;
    const bool mirror = (j == 0 && lp > 0);  // -l is written as the conjugate of +l
    const bool two = lp > 0 && !mirror;
    cd* rhs = eqn == 0 ? b.rv : b.re;
    cd* out = eqn == 0 ? b.v : b.eta;
    const double ftop = b.fold[(((size_t)k * 2 + eqn) * 2 + 0) * g.npairs + pair];
    const double fbot = b.fold[(((size_t)k * 2 + eqn) * 2 + 1) * g.npairs + pair];
    cd yA1 = {0, 0}, yA2 = {0, 0}, yB1 = {0, 0}, yB2 = {0, 0};
    cd gA = {0, 0}, gB = {0, 0};
    for (int i0 = 1; i0 <= nr - 2; i0 += SV_CH) {
        cd rAc[SV_CH], rBc[SV_CH];
        double l2c[SV_CH], l1c[SV_CH];
#pragma unroll
        for (int c = 0; c < SV_CH; ++c) {
            const int i = i0 + c;
            const bool ok = i <= nr - 2;
            rAc[c] = ok ? rhs[(size_t)i * P + modeA] : cd{0, 0};
            rBc[c] = (ok && two) ? rhs[(size_t)i * P + modeB] : cd{0, 0};
            l2c[c] = ok ? b.lu[lu_index(g, k, eqn, 0, i, pair)] : 0.0;
            l1c[c] = ok ? b.lu[lu_index(g, k, eqn, 1, i, pair)] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < SV_CH; ++c) {
            const int i = i0 + c;
            if (i > nr - 2) break;
            cd rA = rAc[c], rB = rBc[c];
            if (mean) rA.x -= mwall[i];
            if (i == nr - 3) {
                gA = rA;
                gB = rB;
            }
            if (i == 1) {
                cd r2A = rhs[(size_t)2 * P + modeA];
                const cd r2B = two ? rhs[(size_t)2 * P + modeB] : cd{0, 0};
                if (mean) r2A.x -= mwall[2];
                rA = cfma(-ftop, r2A, rA);
                rB = cfma(-ftop, r2B, rB);
            }
            if (i == nr - 2) {
                rA = cfma(-fbot, gA, rA);
                rB = cfma(-fbot, gB, rB);
            }
            rA = cfma(-l2c[c], yA2, cfma(-l1c[c], yA1, rA));
            rB = cfma(-l2c[c], yB2, cfma(-l1c[c], yB1, rB));
            rhs[(size_t)i * P + modeA] = rA;
            if (two) rhs[(size_t)i * P + modeB] = rB;
            yA2 = yA1; yA1 = rA;
            yB2 = yB1; yB1 = rB;
        }
    }
    cd xA1 = {0, 0}, xA2 = {0, 0}, xB1 = {0, 0}, xB2 = {0, 0};
    for (int i0 = nr - 2; i0 >= 1; i0 -= SV_CH) {
        double idc[SV_CH], s1c[SV_CH], s2c[SV_CH];
        cd yAc[SV_CH], yBc[SV_CH];
#pragma unroll
        for (int c = 0; c < SV_CH; ++c) {
            const int i = i0 - c;
            const bool ok = i >= 1;
            idc[c] = ok ? b.lu[lu_index(g, k, eqn, 2, i, pair)] : 0.0;
            s1c[c] = ok ? b.lu[lu_index(g, k, eqn, 3, i, pair)] : 0.0;
            s2c[c] = ok ? b.lu[lu_index(g, k, eqn, 4, i, pair)] : 0.0;
            yAc[c] = ok ? rhs[(size_t)i * P + modeA] : cd{0, 0};
            yBc[c] = (ok && two) ? rhs[(size_t)i * P + modeB] : cd{0, 0};
        }
#pragma unroll
        for (int c = 0; c < SV_CH; ++c) {
            const int i = i0 - c;
            if (i < 1) break;
            const cd tA = cfma(-s2c[c], xA2, cfma(-s1c[c], xA1, yAc[c]));
            const cd xA = {tA.x * idc[c], tA.y * idc[c]};
            if (mean) {
                (eqn == 0 ? b.umean : b.wmean)[i] = xA.x;
            } else {
                out[(size_t)i * P + modeA] = xA;
                if (mirror) out[(size_t)i * P + modeB] = cd{xA.x, -xA.y};
            }
            xA2 = xA1;
            xA1 = xA;
            if (two) {
                const cd tB = cfma(-s2c[c], xB2, cfma(-s1c[c], xB1, yBc[c]));
                const cd xB = {tB.x * idc[c], tB.y * idc[c]};
                out[(size_t)i * P + modeB] = xB;
                xB2 = xB1;
                xB1 = xB;
            }
        }
    }
    if (mean) {
        double* mo = eqn == 0 ? b.umean : b.wmean;
        mo[0] = eqn == 0 ? 0.0 : 1.0;
        mo[nr - 1] = eqn == 0 ? 0.0 : g.w_outer;
        return;
    }
    out[modeA] = cd{0, 0};
    out[(size_t)(nr - 1) * P + modeA] = cd{0, 0};
    if (two || mirror) {
        out[modeB] = cd{0, 0};
        out[(size_t)(nr - 1) * P + modeB] = cd{0, 0};
    }
}

// The same substitutions with each column's rows 1..nr-2 cut into
// SV_SEGMENTS segments of L rows, one wavefront per segment and one lane per
// mode (the -l columns of j = 0 are written by their +l lanes as conjugates).
// Each lane runs the forward recurrence y_n = r_n - l1_n y_{n-1} - l2_n y_{n-2}
// over its rows from zero carry-in, together with the two real responses to
// unit carried-in values (from the same l1, l2), publishes the end values and
// responses in LDS, resolves its true carry-in along the chain of earlier
// segments and corrects its rows; the back substitution runs the same way
// from the last segment down.  Every right-hand side, factor and output is
// read or written once, and all rows of a column are in flight together.
//
// Lane layout.  Unpaired: lane i of block x takes mode 64 x + i of the plane.
// Paired: block x takes the pairs (j, |l|) with |l| in 32 q .. 32 q + 31 of
// one j (x = j * groups + q, groups = ceil((K_z + 1) / 32)); lane i < 32 takes
// +|l| and lane 32 + i takes -|l| of the same pair, so the two lanes read the
// pair's factors at the same address in the same instruction and each factor
// is fetched once instead of once per sign of l.
__device__ __forceinline__ int solve_pair_groups(int kz) { return (kz + 32) / 32; }

//
// BACK: the explicit-term kernel has already run the forward elimination
// (with the boundary-row folds and the mean wall terms) along each column and
// left y in rv / re; only the back substitution runs here.
template <int L, int SV_SEGMENTS, bool PAIRED, bool BACK>
__global__ __launch_bounds__(64 * SV_SEGMENTS) void k_solve_seg(const InstDev* __restrict__ I, int k) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    // end values and end responses of each segment, forward sweep (xc, hx)
    // and back substitution (xb, hb) in separate arrays, so the second
    // exchange needs no barrier before it
    constexpr int FS = BACK ? 1 : SV_SEGMENTS;
    __shared__ cd xc[FS][2][64];
    __shared__ double hx[FS][4][64];
    __shared__ cd xb[SV_SEGMENTS][2][64];
    __shared__ double hb[SV_SEGMENTS][4][64];
    const int seg = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x & 63;
    const int eqn = blockIdx.y;
    const int nr = g.nr, kz = g.kz, nl = g.nl;
    const size_t P = g.P;
    int mode, j, l;
    bool inside;  // the lane's mode exists (else it reads a valid one and idles)
    if constexpr (PAIRED) {
        const int groups = solve_pair_groups(kz);
        if ((int)blockIdx.x >= g.nj * groups) return;  // past this instance's pairs (whole block)
        j = (int)blockIdx.x / groups;
        const int lq = ((int)blockIdx.x - j * groups) * 32 + (lane & 31);
        const bool neg = lane >= 32;
        inside = lq <= kz && !(neg && lq == 0);
        const int lc = min(lq, kz);
        l = neg ? -lc : lc;
        mode = j * nl + kz + l;
    } else {
        if ((int)blockIdx.x * 64 >= g.P) return;  // past this instance's modes (whole block)
        const int m0 = blockIdx.x * 64 + lane;
        inside = m0 < g.P;
        mode = min(m0, g.P - 1);
        j = mode / nl;
        l = mode - j * nl - kz;
    }
    const int lp = l < 0 ? -l : l;
    const int pair = j * (kz + 1) + lp;
    const bool mean = (j == 0 && l == 0);
    // lanes past the last mode, and the -l columns of j = 0, only take part in
    // the barriers
    const bool act = inside && !(j == 0 && l < 0);
    const bool mirror = (j == 0 && l > 0);
    const int s0 = 1 + seg * L;
    const int len = max(0, min(s0 + L, nr - 1) - s0);
    const auto* __restrict__ rhs = glb(eqn == 0 ? b.rv : b.re);
    auto* __restrict__ out = glb(eqn == 0 ? b.v : b.eta);
    const auto* __restrict__ mwall = glb(b.mwall) + ((size_t)k * 2 + eqn) * nr;
    const auto* __restrict__ lu = glb(b.lu);
    const auto* __restrict__ fold = glb(b.fold);
    const size_t fstride = (size_t)nr * g.npairs;  // between the five factor fields
    const auto* __restrict__ lub = lu + lu_index(g, k, eqn, 0, 0, pair);
    auto raw = [&](int n) {  // right-hand side of row n before elimination
        cd r = rhs[(size_t)n * P + mode];
        if (mean) r.x -= mwall[n];
        return r;
    };
    cd y[L];
    double h1[L], h2[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        y[i] = cd{0, 0};
        h1[i] = 0.0;
        h2[i] = 0.0;
    }
    if constexpr (BACK) {
#pragma unroll
        for (int i = 0; i < L; ++i)
            if (i < len) y[i] = rhs[(size_t)(s0 + i) * P + mode];
    }
    if (!BACK && len > 0) {
        cd r[L];
#pragma unroll
        for (int i = 0; i < L; ++i) r[i] = raw(min(s0 + i, nr - 2));
        if (s0 == 1) r[0] = cfma(-fold[(((size_t)k * 2 + eqn) * 2 + 0) * g.npairs + pair], raw(2), r[0]);
        cd p1 = {0, 0}, p2 = {0, 0};
        double a1 = 1.0, a2 = 0.0, c1 = 0.0, c2 = 1.0;  // responses to y_{s0-1} and y_{s0-2}
#pragma unroll
        for (int i = 0; i < L; ++i) {
            if (i < len) {
                const int n = s0 + i;
                cd rn = r[i];
                if (n == nr - 2) rn = cfma(-fold[(((size_t)k * 2 + eqn) * 2 + 1) * g.npairs + pair], raw(nr - 3), rn);
                const double l2 = lub[(size_t)n * g.npairs], l1 = lub[fstride + (size_t)n * g.npairs];
                const cd yn = cfma(-l2, p2, cfma(-l1, p1, rn));
                const double an = -l1 * a1 - l2 * a2, cn = -l1 * c1 - l2 * c2;
                y[i] = yn;
                h1[i] = an;
                h2[i] = cn;
                p2 = p1;
                p1 = yn;
                a2 = a1;
                a1 = an;
                c2 = c1;
                c1 = cn;
            }
        }
    }
    if constexpr (!BACK) {
    xc[seg][0][lane] = y[L - 1];
    xc[seg][1][lane] = y[L - 2];
    hx[seg][0][lane] = h1[L - 1];
    hx[seg][1][lane] = h2[L - 1];
    hx[seg][2][lane] = h1[L - 2];
    hx[seg][3][lane] = h2[L - 2];
    __syncthreads();
    {
        cd c1 = {0, 0}, c2 = {0, 0};  // y_{s0-1}, y_{s0-2}; every earlier segment is full
        for (int t = 0; t < (len > 0 ? seg : 0); ++t) {
            const cd n1 = cfma(hx[t][0][lane], c1, cfma(hx[t][1][lane], c2, xc[t][0][lane]));
            const cd n2 = cfma(hx[t][2][lane], c1, cfma(hx[t][3][lane], c2, xc[t][1][lane]));
            c1 = n1;
            c2 = n2;
        }
#pragma unroll
        for (int i = 0; i < L; ++i)
            if (i < len) y[i] = cfma(h1[i], c1, cfma(h2[i], c2, y[i]));
    }
    }
    // back substitution from zero carry-in, with the responses to x_{s1}, x_{s1+1}
    {
        cd q1 = {0, 0}, q2 = {0, 0};
        double a1 = 1.0, a2 = 0.0, c1 = 0.0, c2 = 1.0;
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            if (i < len) {
                const size_t o = (size_t)(s0 + i) * g.npairs;
                const double id = lub[2 * fstride + o], u1 = lub[3 * fstride + o], u2 = lub[4 * fstride + o];
                const cd t = cfma(-u2, q2, cfma(-u1, q1, y[i]));
                const cd q = {t.x * id, t.y * id};
                const double an = (-u1 * a1 - u2 * a2) * id, cn = (-u1 * c1 - u2 * c2) * id;
                y[i] = q;
                h1[i] = an;
                h2[i] = cn;
                q2 = q1;
                q1 = q;
                a2 = a1;
                a1 = an;
                c2 = c1;
                c1 = cn;
            }
        }
    }
    // (x_{s0}, x_{s0+1}) from zero carry-in; for a one-row segment x_{s0+1} is
    // the carried-in x_{s1} itself, which is zero for the last segment
    xb[seg][0][lane] = y[0];
    xb[seg][1][lane] = y[1];
    hb[seg][0][lane] = h1[0];
    hb[seg][1][lane] = h2[0];
    hb[seg][2][lane] = h1[1];
    hb[seg][3][lane] = h2[1];
    __syncthreads();
    if (!act || len == 0) return;
    cd d1 = {0, 0}, d2 = {0, 0};  // x_{s1}, x_{s1+1}: zero beyond the last non-empty segment
    for (int t = SV_SEGMENTS - 1; t > seg; --t) {
        if (1 + t * L >= nr - 1) continue;  // empty segment
        const cd n1 = cfma(hb[t][0][lane], d1, cfma(hb[t][1][lane], d2, xb[t][0][lane]));
        const cd n2 = cfma(hb[t][2][lane], d1, cfma(hb[t][3][lane], d2, xb[t][1][lane]));
        d1 = n1;
        d2 = n2;
    }
    auto* mo = glb(eqn == 0 ? b.umean : b.wmean);
#pragma unroll
    for (int i = 0; i < L; ++i) {
        if (i < len) {
            const int n = s0 + i;
            const cd x = cfma(h1[i], d1, cfma(h2[i], d2, y[i]));
            if (mean) {
                mo[n] = x.x;
            } else {
                out[(size_t)n * P + mode] = x;
                if (mirror) out[(size_t)n * P + (mode - 2 * l)] = cd{x.x, -x.y};
            }
        }
    }
    // wall rows
    const bool first = s0 == 1, last = s0 + len == nr - 1;
    if (mean) {
        if (first) mo[0] = eqn == 0 ? 0.0 : 1.0;
        if (last) mo[nr - 1] = eqn == 0 ? 0.0 : g.w_outer;
    } else {
        if (first) {
            out[mode] = cd{0, 0};
            if (mirror) out[mode - 2 * l] = cd{0, 0};
        }
        if (last) {
            out[(size_t)(nr - 1) * P + mode] = cd{0, 0};
            if (mirror) out[(size_t)(nr - 1) * P + (mode - 2 * l)] = cd{0, 0};
        }
    }
}

// ---------------------------------------------------------------- reductions
// Volume-weighted energy density c_j (|u|^2 + |v|^2 + |w|^2) w_n r_n over
// all (r, mode), block partial sums in a fixed order; also counts non-finite
// state values.
__global__ __launch_bounds__(RED_NT) void k_energy(DevGeom g, DevBuf b) {
    __shared__ double se[RED_NT], sp[RED_NT];
    __shared__ int sf[RED_NT];
    const size_t P = g.P;
    const size_t total = (size_t)g.nr * P;
    double e = 0, ep = 0;
    int bad = 0;
    for (size_t gid = (size_t)blockIdx.x * RED_NT + threadIdx.x; gid < total; gid += (size_t)gridDim.x * RED_NT) {
        const int n = (int)(gid / P);
        const int mode = (int)(gid - (size_t)n * P);
        const int j = mode / g.nl;
        const int li = mode - j * g.nl;
        const double R = g.r[n];
        const double cj = j == 0 ? 1.0 : 2.0;
        const cd v = b.v[gid], eta = b.eta[gid];
        if (!(isfinite(v.x) && isfinite(v.y) && isfinite(eta.x) && isfinite(eta.y))) bad = 1;
        double d;
        if (mode == g.mean) {
            const double um = b.umean[n], wm = b.wmean[n];
            if (!(isfinite(um) && isfinite(wm))) bad = 1;
            d = um * um + wm * wm;
            e += g.wr[n] * d;
        } else {
            const double mm = g.m[j], al = g.alpha[li];
            const double a = inv_k2(R, mm, al);
            cd u, w;
            recover(v, eta, b.dv[gid], R, mm, al, a, u, w);
            d = cj * (u.x * u.x + u.y * u.y + v.x * v.x + v.y * v.y + w.x * w.x + w.y * w.y);
            e += g.wr[n] * d;
            ep += g.wr[n] * d;
        }
    }
    se[threadIdx.x] = e;
    sp[threadIdx.x] = ep;
    sf[threadIdx.x] = bad;
    __syncthreads();
    for (int h = RED_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            sp[threadIdx.x] += sp[threadIdx.x + h];
            sf[threadIdx.x] |= sf[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        b.partial[2 * blockIdx.x] = se[0];
        b.partial[2 * blockIdx.x + 1] = sp[0];
        b.flags[blockIdx.x] = sf[0];
    }
}

// Radial profiles (Sec. 5): at node n, the mean profiles and the plane
// averages of the fluctuations' products, by Parseval over the stored half
// spectrum without the (0,0) mode (c_0 = 1, c_{j>0} = 2): <u'u'>, <v'v'>,
// <w'w'> and <v'w'>.  One block per node, sums in a fixed order; out is
// [6][nr]: u_mean, w_mean, uu, vv, ww, vw.
__global__ __launch_bounds__(RED_NT) void k_profiles(DevGeom g, DevBuf b, double* __restrict__ out) {
    __shared__ double sa[4][RED_NT];
    const int n = blockIdx.x;
    const size_t P = g.P;
    const double R = g.r[n];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int mode = threadIdx.x; mode < g.P; mode += RED_NT) {
        if (mode == g.mean) continue;
        const int j = mode / g.nl;
        const int li = mode - j * g.nl;
        const size_t gid = (size_t)n * P + mode;
        const double cj = j == 0 ? 1.0 : 2.0;
        const double mm = g.m[j], al = g.alpha[li];
        const double a = inv_k2(R, mm, al);
        const cd v = b.v[gid];
        cd u, w;
        recover(v, b.eta[gid], b.dv[gid], R, mm, al, a, u, w);
        acc[0] += cj * (u.x * u.x + u.y * u.y);
        acc[1] += cj * (v.x * v.x + v.y * v.y);
        acc[2] += cj * (w.x * w.x + w.y * w.y);
        acc[3] += cj * (v.x * w.x + v.y * w.y);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sa[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = RED_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < 4; ++k) sa[k][threadIdx.x] += sa[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[n] = b.umean[n];
        out[g.nr + n] = b.wmean[n];
#pragma unroll
        for (int k = 0; k < 4; ++k) out[(size_t)(2 + k) * g.nr + n] = sa[k][0];
    }
}

// Sums the partials in a fixed order and evaluates the wall shear
// g = |D w - w / r| at both walls from the one-sided compact rows.
__global__ __launch_bounds__(RED_NT) void k_stats_final(DevGeom g, DevBuf b, int nblocks) {
    __shared__ double se[RED_NT], sp[RED_NT];
    __shared__ int sf[RED_NT];
    double e = 0, ep = 0;
    int bad = 0;
    for (int i = threadIdx.x; i < nblocks; i += RED_NT) {
        e += b.partial[2 * i];
        ep += b.partial[2 * i + 1];
        bad |= b.flags[i];
    }
    se[threadIdx.x] = e;
    sp[threadIdx.x] = ep;
    sf[threadIdx.x] = bad;
    __syncthreads();
    for (int h = RED_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            sp[threadIdx.x] += sp[threadIdx.x + h];
            sf[threadIdx.x] |= sf[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int nr = g.nr;
        const double* d1 = g.coef + (size_t)1 * nr * 5;
        double dwi = 0, dwo = 0;
        for (int jj = 0; jj < 5; ++jj) {
            dwi += d1[0 * 5 + jj] * b.wmean[g.sigma[0] + jj];
            dwo += d1[(nr - 1) * 5 + jj] * b.wmean[g.sigma[nr - 1] + jj];
        }
        b.stats[0] = fabs(dwi - b.wmean[0] / g.r[0]);
        b.stats[1] = fabs(dwo - b.wmean[nr - 1] / g.r[nr - 1]);
        b.stats[2] = se[0];
        b.stats[3] = sp[0];
        b.stats[4] = (double)sf[0];
    }
}

__global__ __launch_bounds__(RED_NT) void k_finite(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    __shared__ int sf[RED_NT];
    const size_t total = (size_t)g.nr * g.P;
    int bad = 0;
    for (size_t i = (size_t)blockIdx.x * RED_NT + threadIdx.x; i < total; i += (size_t)gridDim.x * RED_NT) {
        const cd v = b.v[i], e = b.eta[i];
        if (!(isfinite(v.x) && isfinite(v.y) && isfinite(e.x) && isfinite(e.y))) bad = 1;
    }
    for (int i = blockIdx.x * RED_NT + threadIdx.x; i < g.nr; i += gridDim.x * RED_NT)
        if (!(isfinite(b.umean[i]) && isfinite(b.wmean[i]))) bad = 1;
    sf[threadIdx.x] = bad;
    __syncthreads();
    for (int h = RED_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sf[threadIdx.x] |= sf[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.flags[blockIdx.x] = sf[0];
}

__global__ __launch_bounds__(RED_NT) void k_flags_final(const InstDev* __restrict__ I, int nblocks) {
    const DevBuf b = I[blockIdx.z].b;
    __shared__ int sf[RED_NT];
    int bad = 0;
    for (int i = threadIdx.x; i < nblocks; i += RED_NT) bad |= b.flags[i];
    sf[threadIdx.x] = bad;
    __syncthreads();
    for (int h = RED_NT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) sf[threadIdx.x] |= sf[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) b.stats[5] = (double)sf[0];
}

// ===================================================== lane-FFT fast path
// Compile-time transform lengths (see fft_lane.h); the generic kernels above
// serve every other length.

struct DevSync {
    __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

// j-columns per block of the z kernels: 3072 complex doubles or 6144
// complex floats per tile (48 KiB of LDS), at most 16 columns
constexpr int zlane_cols(int N, int esize) {
    const int c = (esize == 8 ? 6144 : 3072) / N;
    return c < 1 ? 1 : (c > 16 ? 16 : c);
}

// Column pitch of the z kernels' LDS tiles: the transposes read or write one
// element per column for consecutive columns, so the pitch is offset from N
// by 16 / JB elements, which puts the JB columns of a group of 16 lanes in
// distinct element slots (and so spreads them over the banks).
constexpr int zlane_pitch_jb(int N, int jb) { return N + ((16 % jb) == 0 ? 16 / jb : 1); }
constexpr int zlane_pitch(int N, int esize) { return zlane_pitch_jb(N, zlane_cols(N, esize)); }

// Tile-shape variants the autotuner may pick for a launch group: the z
// kernels at half or twice the default columns per block (at most 32
// columns, 1024 threads and 160 KB of LDS per block), the theta kernel at 1,
// 2 or 4 wavefronts per block.  Code 0 is the default shape.
constexpr int zlane_variant_cols(int N, int esize, int code) {
    const int d = zlane_cols(N, esize);
    const int jb = code == 1 ? d / 2 : (code == 2 ? d * 2 : d);
    return jb < 1 ? 1 : jb;
}
template <typename T, int N>
constexpr bool zlane_variant_ok(int code) {
    if (code < 0 || code > 2) return false;
    const int jb = zlane_variant_cols(N, (int)sizeof(C<T>), code);
    if (code == 1 && zlane_cols(N, (int)sizeof(C<T>)) < 2) return false;
    return jb <= 32 && jb * lane::Plan<N>::TL <= 1024 &&
           (long long)jb * zlane_pitch_jb(N, jb) * (long long)sizeof(C<T>) + (lane::tw_size<N>() + 1) * (long long)sizeof(C<T>) <=
               160 * 1024;
}

// The value v of lane src of this wavefront (ds_bpermute: the LDS crossbar,
// no LDS memory).  Every lane of the wavefront must be active.
__device__ __forceinline__ int lane_read_b32(int v, int src) { return __builtin_amdgcn_ds_bpermute(src * 4, v); }
__device__ __forceinline__ C<double> lane_read(C<double> v, int src) {
    const unsigned long long x = __builtin_bit_cast(unsigned long long, v.x);
    const unsigned long long y = __builtin_bit_cast(unsigned long long, v.y);
    const unsigned long long xl = (unsigned)lane_read_b32((int)(unsigned)x, src);
    const unsigned long long xh = (unsigned)lane_read_b32((int)(unsigned)(x >> 32), src);
    const unsigned long long yl = (unsigned)lane_read_b32((int)(unsigned)y, src);
    const unsigned long long yh = (unsigned)lane_read_b32((int)(unsigned)(y >> 32), src);
    return C<double>{__builtin_bit_cast(double, xl | (xh << 32)), __builtin_bit_cast(double, yl | (yh << 32))};
}
__device__ __forceinline__ C<float> lane_read(C<float> v, int src) {
    const int x = lane_read_b32(__builtin_bit_cast(int, v.x), src);
    const int y = lane_read_b32(__builtin_bit_cast(int, v.y), src);
    return C<float>{__builtin_bit_cast(float, x), __builtin_bit_cast(float, y)};
}

// The block of a plane's column groups that runs block x: with the groups
// paired so that x and x + 8 (which the dispatcher sends to the same XCD, and
// so the same L2) take adjacent groups.  A complex-float group of fewer than
// 16 columns covers part of each 128-byte line of a z row; paired, two such
// parts are fetched through one L2.  Identity unless gx is a multiple of 16.
__device__ __forceinline__ int xcd_pair(int x, int gx) {
    if (gx % 16) return x;
    return (x & ~15) + 2 * (x & 7) + ((x >> 3) & 1);
}

// Wavefront-scope ordering of LDS accesses: a wavefront's LDS instructions
// execute in order, so a fence that keeps the compiler from moving them
// across this point is all that lanes of one wavefront need to exchange data.
struct WaveSync {
    __device__ __forceinline__ void operator()() const {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// register slot that holds position g + TL m after a transform kept in
// registers (inverse of last_slot_to_m)
template <int N>
__host__ __device__ constexpr int m_to_last_slot(int m) {
    for (int s = 0; s < lane::Plan<N>::P; ++s)
        if (lane::last_slot_to_m<N>(s) == m) return s;
    return 0;
}

// wavefronts per block of the theta kernel with w loaded into registers
// (measured best: 1 in FP64, so that every wavefront starts and ends on its
// own, 2 in FP32)
template <typename T>
constexpr int theta_waves() { return sizeof(T) == 8 ? 1 : 2; }

// theta rows: each wavefront owns W = 64 / TL packed row pairs (z0, z0 + 1)
// and does everything for them.  It loads u, v and w, inverse-transforms them
// in turn (the results stay in registers, in the same slot order for all
// three), forms each of the six products pointwise in registers and
// forward-transforms it.  The wavefronts of a block share only the twiddle
// table, so no block-wide barrier follows it.  XM selects the transform:
// 0 the Stockham passes through the wavefront's own LDS region (fft_lane.h);
// for N = 768 (fft_xlane.h) 1 every exchange between lanes in registers, 2
// the highest lane digit swapped in registers and the two lower ones through
// a small LDS buffer, 3 as 2 with the rows of w fetched into LDS by the
// memory unit (16-byte LDS-DMA loads) while u and v are transformed, so that
// they arrive without registers held for them.
template <typename T, int N, int WV, int XM>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(2))) void k_theta_wave(
    const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const auto* __restrict__ zb = glb((const C<T>*)b.zb);
    auto* __restrict__ pb = glb((C<T>*)b.pb);
    using PL = lane::Plan<N>;
    constexpr int TL = PL::TL, P = PL::P, W = 64 / TL;
    constexpr bool XL = XM != 0, LOW_LDS = XM >= 2, WDMA = XM == 3;
    static_assert(!XL || (N == xlane::N && TL == 64), "the register-exchange transform is 768 points per wavefront");
    __shared__ C<T> lds[XM == 0 ? WV * W * N : (LOW_LDS ? WV * xlane::XBUF : 1)];
    // K_theta = (N - 1) / 3 is fixed by N, so which of the kept band, the zero
    // band and the mirrored band a register slot covers is known at compile
    // time for every slot but one or two
    constexpr int KT = (N - 1) / 3, NJ = KT + 1;
    // w's two z rows per wavefront, in whole 1 KB DMA pieces (64 lanes x 16 bytes)
    constexpr int WBYTES = 2 * NJ * (int)sizeof(C<T>);
    constexpr int WPIECES = (WBYTES + 1023) / 1024, WSTRIDE = WPIECES * 1024 / (int)sizeof(C<T>);
    __shared__ __attribute__((aligned(16))) C<T> wl[WDMA ? WV * WSTRIDE : 1];
    __shared__ C<T> twl[XL ? xlane::NTW : lane::tw_size<N>() + 1];  // twiddles
    if ((int)blockIdx.y >= g.nr || (int)blockIdx.x * WV * W >= g.nz / 2) return;  // whole block
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lw = threadIdx.x & 63;
    const int grp = lw / TL;
    const int gl = lw - grp * TL;
    const int rp = (blockIdx.x * WV + wv) * W + grp;
    const int nz = g.nz, nr = g.nr;
    const bool active = rp < nz / 2;
    const int r = blockIdx.y;
    const int z0 = 2 * rp;
    const xlane::LaneBits lbits(lw);
    // slot of position gl + TL m after a transform that leaves natural order
    auto slot = [](int m) { return XL ? m : m_to_last_slot<N>(m); };
    auto inverse = [&](C<T>* x) {
        if constexpr (XL) xlane::inverse<T, LOW_LDS>(x, twl, lds + wv * xlane::XBUF, lw, lbits, WaveSync());
        else lane::fft<T, N, +1, true>(lds + (wv * W + grp) * N, x, gl, twl, WaveSync());
    };
    auto forward = [&](C<T>* x) {
        if constexpr (XL) xlane::forward<T, LOW_LDS>(x, twl, lds + wv * xlane::XBUF, lw, lbits, WaveSync());
        else lane::fft<T, N, -1, true>(lds + (wv * W + grp) * N, x, gl, twl, WaveSync());
    };
    // the z-spectral rows of field fl packed into the complex sequence of the
    // two real rows (z0, z0 + 1)
    // get0(p), get1(p): mode p of rows z0 and z0 + 1.  Every load is issued
    // before any value is combined (a slot that covers part of a band loads
    // at a valid index in every lane and selects afterwards), so the loads of
    // a field are in flight together instead of one slot's after another's.
    auto fetch = [&](auto get0, auto get1, C<T>* a, C<T>* c) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int p = gl + k * TL;
            const bool low_all = k * TL + TL - 1 <= KT, low_none = k * TL > KT;
            const bool high_all = k * TL >= N - KT, high_none = k * TL + TL - 1 < N - KT;
            if (low_none && high_none) continue;
            const bool lo = low_all || (!low_none && p <= KT);
            const bool hi = high_all || (!high_none && p >= N - KT);
            const unsigned idx = lo ? (unsigned)p : (hi ? (unsigned)(N - p) : 0u);
            a[k] = get0(idx);
            c[k] = get1(idx);
        }
    };
    auto combine = [&](const C<T>* a, const C<T>* c, C<T>* x) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int p = gl + k * TL;
            const bool low_all = k * TL + TL - 1 <= KT, low_none = k * TL > KT;
            const bool high_all = k * TL >= N - KT, high_none = k * TL + TL - 1 < N - KT;
            C<T> h = {(T)0, (T)0};
            if (!(low_none && high_none)) {
                const bool lo = low_all || (!low_none && p <= KT);
                const bool hi = high_all || (!high_none && p >= N - KT);
                C<T> ak = a[k], ck = c[k];
                if (k == 0 && p == 0) {
                    ak.y = (T)0;
                    ck.y = (T)0;
                }
                // selected component by component: a select between the two
                // complex values as whole objects is compiled as a choice of
                // address between two stack copies, in scratch memory
                const T hlx = ak.x - ck.y, hly = ak.y + ck.x, hhx = ak.x + ck.y, hhy = ck.x - ak.y;
                h.x = lo ? hlx : (hi ? hhx : (T)0);
                h.y = lo ? hly : (hi ? hhy : (T)0);
                if (!active) h = C<T>{(T)0, (T)0};
            }
            x[k] = h;
        }
    };
    // a row pair past the plane's end (a wavefront with no work) reads the
    // plane's first pair and discards it, so the loads need no branch
    const int z0c = active ? z0 : 0;
    auto row_pair = [&](int fl) {
        const auto* row0 = zb + (((size_t)fl * nr + r) * nz + z0c) * NJ;
        if constexpr (W == 1) row0 = uniform(row0);  // one row pair per wavefront
        return row0;
    };
    auto fetch_field = [&](int fl, C<T>* a, C<T>* c) {
        const auto* row0 = row_pair(fl);
        const auto* row1 = row0 + NJ;
        fetch([&](unsigned p) { return at(row0, p); }, [&](unsigned p) { return at(row1, p); }, a, c);
    };
    // forward-transform product x (slot order of the inverse transforms) and
    // write its two z rows.  The transform's outputs stay in registers: lane
    // gl holds positions gl + TL m, and the mirrored position N - j of its
    // output j = gl + TL q sits in lane TL - gl at m = P - 1 - q (lane 0
    // holds its own, at m = P - q), read across lanes.
    constexpr int QN = (NJ + TL - 1) / TL;
    static_assert(QN <= P, "kept outputs per lane");
    const int partner = grp * TL + ((TL - gl) & (TL - 1));
    auto product_out = [&](int prod, const C<T>* a, const C<T>* c) {
        C<T> x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = pmul(a[slot(k)], c[slot(k)]);
        forward(x);
        C<T> hm[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const C<T> got = lane_read(x[slot(P - 1 - q)], partner);
            hm[q] = gl == 0 ? x[slot((P - q) % P)] : got;
        }
        if (active) {
            auto* out = pb + (((size_t)prod * nr + r) * nz + z0) * NJ;
            if constexpr (W == 1) out = uniform(out);  // one row pair per wavefront
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const int j = gl + q * TL;
                if ((q + 1) * TL <= NJ || j < NJ) {
                    const C<T> h = x[slot(q)];
                    at(out, (unsigned)j) = C<T>{(T)0.5 * (h.x + hm[q].x), (T)0.5 * (h.y - hm[q].y)};
                    at(out, (unsigned)(NJ + j)) = C<T>{(T)0.5 * (h.y + hm[q].y), (T)0.5 * (hm[q].x - h.x)};
                }
            }
        }
    };
    // u and v first, w after the three products that need only u and v, so
    // that at most three transform-sized register sets are live at a time
    C<T> u[P], v[P], w[P];
    if constexpr (XL) {
        if (threadIdx.x < 64) xlane::fill_twiddles<T>(twl, glb(tw_t<T>(g)), lw);
    } else {
        lane::fill_twiddles<T, N>(twl, glb(tw_t<T>(g)), threadIdx.x, 64 * WV);
    }
    {
        // the loads of u and v, all in flight together
        C<T> au[P], cu[P], av[P], cv[P];
        fetch_field(0, au, cu);
        fetch_field(1, av, cv);
        combine(au, cu, u);
        combine(av, cv, v);
    }
    __syncthreads();  // twiddle table complete
    C<T>* const wrow = wl + wv * WSTRIDE;
    if constexpr (WDMA) {
        // issued right after u's and v's loads.  The compiler waits for them
        // (vmcnt) before the first read of wl; its wait counts do not tell
        // DMA loads from ordinary ones, so the wait for u and v covers them
        // too: w arrives in the same round trip, without registers held
        static_assert(W == 1 && WBYTES <= WPIECES * 1024, "w rows per wavefront");
        if (active) {
            const auto* src = (const TC_GLOBAL char*)row_pair(2);
#pragma unroll
            for (int q = 0; q < WPIECES; ++q) {
                const int off = q * 1024 + lw * 16;
                if (off < WBYTES)
                    __builtin_amdgcn_global_load_lds((const void*)(src + off),
                                                     (__attribute__((address_space(3))) void*)(wrow + q * (1024 / (int)sizeof(C<T>))),
                                                     16, 0, 0);
            }
        }
    }
    inverse(u);
    inverse(v);
    product_out(0, u, u);
    product_out(1, u, v);
    product_out(3, v, v);
    // after vv: loading w into registers earlier keeps a fourth register set live
    {
        C<T> aw[P], cw[P];
        if constexpr (WDMA) fetch([&](unsigned p) { return wrow[p]; }, [&](unsigned p) { return wrow[NJ + p]; }, aw, cw);
        else fetch_field(2, aw, cw);
        combine(aw, cw, w);
    }
    inverse(w);
    product_out(2, u, w);
    product_out(4, v, w);
    product_out(5, w, w);
}

// inverse z transform of u, v, w for JB j-columns of one plane; v, eta and
// D v are read once per element.
template <typename T, int N, int JBV>
__global__ __launch_bounds__(JBV * lane::Plan<N>::TL) void k_zinv_lane(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const auto* __restrict__ v = glb(b.v);
    const auto* __restrict__ eta = glb(b.eta);
    const auto* __restrict__ dv = glb(b.dv);
    const auto* __restrict__ umean = glb(b.umean);
    const auto* __restrict__ wmean = glb(b.wmean);
    auto* __restrict__ zb = glb((C<T>*)b.zb);
    using PL = lane::Plan<N>;
    constexpr int TL = PL::TL, P = PL::P, JB = JBV, NTH = JB * TL, PITCH = zlane_pitch_jb(N, JB);
    __shared__ C<T> lds[JB * PITCH];
    const int c = threadIdx.x / TL;
    const int gl = threadIdx.x - c * TL;
    const int r = blockIdx.y;
    const int j0 = (sizeof(T) == 4 ? xcd_pair(blockIdx.x, gridDim.x) : (int)blockIdx.x) * JB;
    if (r >= g.nr || j0 >= g.nj) return;  // past this instance's extents (whole block)
    const int nj = g.nj;
    // K_z = (N - 1) / 3 is fixed by N: which of the kept band, the zero band
    // and the mirrored band a register slot covers is known at compile time
    // for every slot but one or two
    constexpr int KZ = (N - 1) / 3, NL = 2 * KZ + 1;
    const int ncols = min(JB, nj - j0);
    const int j = j0 + c;
    const bool active = c < ncols;
    const double R = cst(g.r)[r];
    const size_t Pm = g.P;
    const auto* tw = glb(tw_z<T>(g));
    // a column's transform lives in TL lanes of one wavefront, so its LDS
    // exchanges need only wavefront-scope ordering; the block barriers below
    // guard the twiddle table and the transposed write-out, which cross columns
    const WaveSync sync;
    __shared__ C<T> twl[lane::tw_size<N>() + 1];
    C<T> X[3][P];
    const int jc = active ? j : j0;  // a lane past the tile reads its block's first column
    const double mm = glb(g.m)[jc];
    const auto* vr = v + (size_t)r * Pm;  // plane r
    const auto* er = eta + (size_t)r * Pm;
    const auto* dr = dv + (size_t)r * Pm;
    // slot k's band, its l (0 in the zero band: a valid mode, read and dropped)
    // and the element's offset in the plane
    auto band = [&](int k, bool& low, bool& high, int& l) {
        const int q = gl + k * TL;
        const bool low_all = k * TL + TL - 1 <= KZ, low_none = k * TL > KZ;
        const bool high_all = k * TL >= N - KZ, high_none = k * TL + TL - 1 < N - KZ;
        low = low_all || (!low_none && q <= KZ);
        high = !low && (high_all || (!high_none && q >= N - KZ));
        l = low ? q : (high ? q - N : 0);
    };
    auto zero_band = [&](int k) { return k * TL > KZ && k * TL + TL - 1 < N - KZ; };
    // slot k of u, v, w from the loaded v, eta, D v and alpha of its mode
    auto slot = [&](int k, cd lv, cd le, cd ld, double al, double um, double wm) {
        bool low, high;
        int l;
        band(k, low, high, l);
        C<T> xu = {(T)0, (T)0}, xv = xu, xw = xu;
        const double a = inv_k2(R, mm, al);
        cd u, w;
        recover(lv, le, ld, R, mm, al, a, u, w);
        if (j == 0 && l == 0) {  // the mean mode: a is not finite there, and not used
            xu = C<T>{(T)um, (T)0};
            xw = C<T>{(T)wm, (T)0};
        } else {
            xu = C<T>{(T)u.x, (T)u.y};
            xv = C<T>{(T)lv.x, (T)lv.y};
            xw = C<T>{(T)w.x, (T)w.y};
        }
        if (!(active && (low || high))) xu = xv = xw = C<T>{(T)0, (T)0};
        X[0][k] = xu;
        X[1][k] = xv;
        X[2][k] = xw;
    };
    auto load = [&](int k, cd& lv, cd& le, cd& ld, double& al) {
        bool low, high;
        int l;
        band(k, low, high, l);
        const unsigned e = (unsigned)(jc * NL + (l + KZ));
        al = glb(g.alpha)[l + KZ];
        lv = at(vr, e);
        le = at(er, e);
        ld = at(dr, e);
    };
    if constexpr (sizeof(T) == 8 || N <= 128) {
        // FP64 (two waves per SIMD), and the short FP32 transforms: every
        // load of the lane, then the twiddle table's, are issued before any
        // value is combined, so they are in flight together instead of one
        // slot's after another's
        cd lv[P], le[P], ld[P];
        double lal[P];
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (!zero_band(k)) load(k, lv[k], le[k], ld[k], lal[k]);
        const double um = umean[r], wm = wmean[r];
        lane::fill_twiddles<T, N>(twl, tw, threadIdx.x, NTH);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (zero_band(k)) {
                X[0][k] = X[1][k] = X[2][k] = C<T>{(T)0, (T)0};
                continue;
            }
            slot(k, lv[k], le[k], ld[k], lal[k], um, wm);
        }
    } else {
        // FP32 at 192 points and more (four waves per SIMD, which hide the
        // latency of one slot's loads at a time; holding every slot's would
        // cost the fourth wave)
        lane::fill_twiddles<T, N>(twl, tw, threadIdx.x, NTH);
        const double um = umean[r], wm = wmean[r];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (zero_band(k)) {
                X[0][k] = X[1][k] = X[2][k] = C<T>{(T)0, (T)0};
                continue;
            }
            cd lv, le, ld;
            double al;
            load(k, lv, le, ld, al);
            slot(k, lv, le, ld, al, um, wm);
        }
    }
    // transposed write-out: tile element e of this lane is idx = threadIdx.x +
    // e NTH, row z = idx / ncols and column cc = idx mod ncols, at these
    // offsets in the plane and in LDS (-1: past the tile)
    int goff[P], loff[P];
    {
        const bool full = ncols == JB;  // every block but an instance's last
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const int idx = threadIdx.x + e * NTH;
            const int z = full ? idx / JB : idx / ncols;
            const int cc = idx - z * (full ? JB : ncols);
            const bool ok = idx < ncols * N;
            goff[e] = ok ? z * nj + j0 + cc : -1;
            loff[e] = ok ? cc * PITCH + z : -1;
        }
    }
    __syncthreads();  // twiddles in place
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        lane::fft<T, N, +1, true>(lds + c * PITCH, X[f], gl, twl, sync);
#pragma unroll
        for (int q = 0; q < P; ++q) lds[c * PITCH + gl + TL * lane::last_slot_to_m<N>(q)] = X[f][q];
        __syncthreads();
        auto* out = uniform(zb + ((size_t)f * g.nr + r) * N * nj);
#pragma unroll
        for (int e = 0; e < P; ++e)
            if (goff[e] >= 0) at(out, (unsigned)goff[e]) = lds[loff[e]];
        __syncthreads();
    }
}

// forward z transform of the six products for JB j-columns of one plane,
// truncation to |l| <= K_z and normalisation.
template <typename T, int N, int JBV>
__global__ __launch_bounds__(JBV * lane::Plan<N>::TL) void k_zfwd_lane(const InstDev* __restrict__ I) {
    const DevGeom g = I[blockIdx.z].g;
    const DevBuf b = I[blockIdx.z].b;
    const auto* __restrict__ pb = glb((const C<T>*)b.pb);
    auto* __restrict__ ps = glb((C<T>*)b.ps);
    using PL = lane::Plan<N>;
    constexpr int TL = PL::TL, P = PL::P, JB = JBV, NTH = JB * TL, PITCH = zlane_pitch_jb(N, JB);
    __shared__ C<T> lds[JB * PITCH];
    const int c = threadIdx.x / TL;
    const int gl = threadIdx.x - c * TL;
    const int r = blockIdx.y;
    const int j0 = (sizeof(T) == 4 ? xcd_pair(blockIdx.x, gridDim.x) : (int)blockIdx.x) * JB;
    if (r >= g.nr || j0 >= g.nj) return;  // past this instance's extents (whole block)
    const int nj = g.nj;
    constexpr int KZ = (N - 1) / 3, NL = 2 * KZ + 1;  // K_z is fixed by N
    const int ncols = min(JB, nj - j0);
    const bool active = c < ncols;
    const size_t Pm = g.P;
    const T scale = (T)(1.0 / ((double)g.ntheta * (double)N));
    const auto* tw = glb(tw_z<T>(g));
    // as in k_zinv_lane: wavefront-scope ordering inside a column's transform,
    // block barriers around the transposed load, which crosses columns
    const WaveSync sync;
    __shared__ C<T> twl[lane::tw_size<N>() + 1];
    lane::fill_twiddles<T, N>(twl, tw, threadIdx.x, NTH);
    // tile element e of this lane is idx = threadIdx.x + e NTH, row z =
    // idx / ncols and column cc = idx mod ncols, the same for every product:
    // its offset in the plane and in LDS are formed once (-1: past the tile)
    int goff[P], loff[P];
    {
        const bool full = ncols == JB;  // every block but an instance's last
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const int idx = threadIdx.x + e * NTH;
            const int z = full ? idx / JB : idx / ncols;
            const int cc = idx - z * (full ? JB : ncols);
            const bool ok = idx < ncols * N;
            goff[e] = ok ? z * nj + j0 + cc : -1;
            loff[e] = ok ? cc * PITCH + z : -1;
        }
    }
    // the next product's tile (P values per lane) is fetched into registers
    // while the current one is transformed
    C<T> nxt[P];
    auto fetch = [&](int f) {
        const auto* in = uniform(pb + ((size_t)f * g.nr + r) * N * nj);
        // past the tile the load repeats the plane's first element (in
        // bounds) and the value is never stored (loff < 0 exactly where
        // goff < 0), so the raw values are kept and the loads stay in flight
#pragma unroll
        for (int e = 0; e < P; ++e) nxt[e] = at(in, (unsigned)max(goff[e], 0));
    };
    fetch(0);
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
#pragma unroll
        for (int e = 0; e < P; ++e)
            if (loff[e] >= 0) lds[loff[e]] = nxt[e];
        __syncthreads();  // also completes the twiddle table on the first pass
        if (f < 5) fetch(f + 1);
        C<T> x[P];
#pragma unroll
        for (int k = 0; k < P; ++k) x[k] = active ? lds[c * PITCH + gl + k * TL] : C<T>{(T)0, (T)0};
        sync();
        lane::fft<T, N, -1, true>(lds + c * PITCH, x, gl, twl, sync);
        if constexpr (sizeof(T) == 8) {
            // Loads and stores share one wait counter: once this product's
            // stores are issued, waiting for the next tile would wait for
            // them too.  The next tile is therefore required here, after the
            // transform and before the stores: an empty statement that takes
            // its registers as inputs (it reads and writes no memory, and as
            // a volatile statement it stays between the transform and the
            // stores).
#pragma unroll
            for (int e = 0; e < P; ++e) asm volatile("" : : "v"(nxt[e].x), "v"(nxt[e].y));
        }
        if (active) {
            auto* out = uniform(ps + (size_t)f * g.nr * Pm + (size_t)r * Pm);  // plane r of product f
#pragma unroll
            for (int s = 0; s < P; ++s) {
                const int q = gl + TL * lane::last_slot_to_m<N>(s);
                const int l = q <= KZ ? q : q - N;
                if (l >= -KZ) at(out, (unsigned)((j0 + c) * NL + l + KZ)) = cscale(x[s], scale);
            }
        }
        __syncthreads();  // every column read before the next transposed load
    }
}

// Spectral u and w of every mode (mean profiles in the (0,0) slot).
__global__ __launch_bounds__(NT) void k_velocity(DevGeom g, DevBuf b, cd* __restrict__ uo, cd* __restrict__ wo) {
    const size_t gid = (size_t)blockIdx.x * NT + threadIdx.x;
    const size_t P = g.P;
    if (gid >= (size_t)g.nr * P) return;
    const int n = (int)(gid / P);
    const int mode = (int)(gid - (size_t)n * P);
    if (mode == g.mean) {
        uo[gid] = cd{b.umean[n], 0.0};
        wo[gid] = cd{b.wmean[n], 0.0};
        return;
    }
    const int j = mode / g.nl;
    const int li = mode - j * g.nl;
    const double R = g.r[n], mm = g.m[j], al = g.alpha[li];
    const double a = inv_k2(R, mm, al);
    cd u, w;
    recover(b.v[gid], b.eta[gid], b.dv[gid], R, mm, al, a, u, w);
    uo[gid] = u;
    wo[gid] = w;
}

}  // namespace

int zcols_per_block(int nz, int nj) {
    int jb = ZELEMS / nz;
    if (jb < 1) jb = 1;
    if (jb > nj) jb = nj;
    return jb;
}

int reduction_blocks(const DevGeom& g) {
    const size_t total = (size_t)g.nr * g.P;
    size_t nb = (total + RED_NT - 1) / RED_NT;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

void launch_dv(const Batch& B, hipStream_t s) {
    const DevGeom& g = B.g;
    const dim3 gseg((g.P + 63) / 64, 1, B.count);
    switch (g.dv_nseg * 100 + g.dv_seg) {
        case 804: hipLaunchKernelGGL((k_dv_seg<4, 8>), gseg, dim3(64 * 8), 0, s, B.inst); return;
        case 808: hipLaunchKernelGGL((k_dv_seg<8, 8>), gseg, dim3(64 * 8), 0, s, B.inst); return;
        case 816: hipLaunchKernelGGL((k_dv_seg<16, 8>), gseg, dim3(64 * 8), 0, s, B.inst); return;
    }
    dim3 grid((g.P + NT - 1) / NT, 1, B.count);
    hipLaunchKernelGGL(k_dv, grid, dim3(NT), 0, s, B.inst);
}

#define TC_LANE_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768)

template <typename T, int N, int CODE>
void zinv_lane_v(const Batch& B, hipStream_t s) {
    if constexpr (zlane_variant_ok<T, N>(CODE)) {
        constexpr int JB = zlane_variant_cols(N, sizeof(C<T>), CODE);
        dim3 grid((B.g.nj + JB - 1) / JB, B.g.nr, B.count);
        hipLaunchKernelGGL((k_zinv_lane<T, N, JB>), grid, dim3(JB * lane::Plan<N>::TL), 0, s, B.inst);
    }
}
template <typename T, int N>
void zinv_lane(const Batch& B, hipStream_t s) {
    const int code = zlane_variant_ok<T, N>(B.g.tile_zinv) ? B.g.tile_zinv : 0;
    if (code == 1) zinv_lane_v<T, N, 1>(B, s);
    else if (code == 2) zinv_lane_v<T, N, 2>(B, s);
    else zinv_lane_v<T, N, 0>(B, s);
}
template <typename T, int N, int CODE>
void zfwd_lane_v(const Batch& B, hipStream_t s) {
    if constexpr (zlane_variant_ok<T, N>(CODE)) {
        constexpr int JB = zlane_variant_cols(N, sizeof(C<T>), CODE);
        dim3 grid((B.g.nj + JB - 1) / JB, B.g.nr, B.count);
        hipLaunchKernelGGL((k_zfwd_lane<T, N, JB>), grid, dim3(JB * lane::Plan<N>::TL), 0, s, B.inst);
    }
}
template <typename T, int N>
void zfwd_lane(const Batch& B, hipStream_t s) {
    const int code = zlane_variant_ok<T, N>(B.g.tile_zfwd) ? B.g.tile_zfwd : 0;
    if (code == 1) zfwd_lane_v<T, N, 1>(B, s);
    else if (code == 2) zfwd_lane_v<T, N, 2>(B, s);
    else zfwd_lane_v<T, N, 0>(B, s);
}
template <typename T, int N, int WV, int XM>
void theta_lane_v(const Batch& B, hipStream_t s) {
    constexpr int RB = (64 / lane::Plan<N>::TL) * WV;  // row pairs per block
    dim3 grid((B.g.nz / 2 + RB - 1) / RB, B.g.nr, B.count);
    hipLaunchKernelGGL((k_theta_wave<T, N, WV, XM>), grid, dim3(64 * WV), 0, s, B.inst);
}
// the transform of the theta kernel: the lane-digit swaps (fft_xlane.h)
// wherever one wavefront holds one transform of 12 points per lane, with w
// loaded into registers in FP64 and fetched into LDS by DMA in FP32 (measured
// best: in FP32 the DMA form keeps four waves per SIMD, in FP64 both forms
// run two and the register form is 1 % faster)
template <typename T, int N>
constexpr int theta_xm() { return N == xlane::N ? (sizeof(T) == 4 ? 3 : 2) : 0; }
// the other form of w's fetch, and the wavefronts per block of each (the
// DMA form needs at least two per block in FP64 for two waves per SIMD
// within the LDS, four in FP32)
template <typename T, int N>
constexpr int theta_xm_alt() { return theta_xm<T, N>() == 3 ? 2 : 3; }
template <typename T, int XM>
constexpr int theta_waves_for() { return XM == 3 ? (sizeof(T) == 8 ? 2 : 4) : theta_waves<T>(); }
// theta tile code: 0 the default wavefronts per block, 1, 2 or 4 explicitly
// (codes 1, 2, 3); where the lane-digit transform is the default, code 4 runs
// the Stockham transform and code 5 the transform with every swap in
// registers, and code 6 the lane-digit transform with the other form of w's
// fetch, each at its default wavefronts
template <typename T, int N>
void theta_lane(const Batch& B, hipStream_t s) {
    constexpr int XM = theta_xm<T, N>();
    switch (B.g.tile_theta) {
        case 1: theta_lane_v<T, N, 1, XM>(B, s); return;
        case 2: theta_lane_v<T, N, 2, XM>(B, s); return;
        case 3: theta_lane_v<T, N, 4, XM>(B, s); return;
        case 4:
        case 5:
        case 6:
            if constexpr (XM != 0) {
                constexpr int XA = theta_xm_alt<T, N>();
                if (B.g.tile_theta == 4) theta_lane_v<T, N, theta_waves<T>(), 0>(B, s);
                else if (B.g.tile_theta == 5) theta_lane_v<T, N, theta_waves<T>(), 1>(B, s);
                else theta_lane_v<T, N, theta_waves_for<T, XA>(), XA>(B, s);
                return;
            }
            break;
    }
    theta_lane_v<T, N, theta_waves_for<T, XM>(), XM>(B, s);
}

template <typename T>
bool zinv_fast(const Batch& B, hipStream_t s) {
    // the lane kernels take K_z = (nz - 1) / 3 as a compile-time constant
    if (B.g.kz != (B.g.nz - 1) / 3 || B.g.nl != 2 * B.g.kz + 1) return false;
    switch (B.g.nz) {
#define TC_CASE(N) case N: zinv_lane<T, N>(B, s); return true;
        TC_LANE_SIZES(TC_CASE)
#undef TC_CASE
    }
    return false;
}
template <typename T>
bool zfwd_fast(const Batch& B, hipStream_t s) {
    if (B.g.kz != (B.g.nz - 1) / 3 || B.g.nl != 2 * B.g.kz + 1) return false;
    switch (B.g.nz) {
#define TC_CASE(N) case N: zfwd_lane<T, N>(B, s); return true;
        TC_LANE_SIZES(TC_CASE)
#undef TC_CASE
    }
    return false;
}
template <typename T>
bool theta_fast(const Batch& B, hipStream_t s) {
    // the lane kernel takes K_theta = (ntheta - 1) / 3 as a compile-time constant
    if (B.g.kt != (B.g.ntheta - 1) / 3 || B.g.nj != B.g.kt + 1) return false;
    switch (B.g.ntheta) {
#define TC_CASE(N) case N: theta_lane<T, N>(B, s); return true;
        TC_LANE_SIZES(TC_CASE)
#undef TC_CASE
    }
    return false;
}

bool lane_length(int n) {
    switch (n) {
#define TC_CASE(N) case N: return true;
        TC_LANE_SIZES(TC_CASE)
#undef TC_CASE
    }
    return false;
}

template <typename T>
bool tile_ok_t(int stage, int n, int code) {
    if (stage == ST_THETA) return lane_length(n) && ((code >= 0 && code <= 3) || (code <= 6 && n == xlane::N));
    switch (n) {
#define TC_CASE(N) case N: return zlane_variant_ok<T, N>(code);
        TC_LANE_SIZES(TC_CASE)
#undef TC_CASE
    }
    return false;
}

bool tile_variant_ok(int stage, const DevGeom& g, bool fp32, int code) {
    if (g.generic_fft) return code == 0;
    if (stage == ST_ZINV || stage == ST_ZFWD) {
        if (!lane_length(g.nz) || g.kz != (g.nz - 1) / 3) return code == 0;
        return fp32 ? tile_ok_t<float>(stage, g.nz, code) : tile_ok_t<double>(stage, g.nz, code);
    }
    if (stage == ST_THETA) {
        if (!lane_length(g.ntheta) || g.kt != (g.ntheta - 1) / 3) return code == 0;
        return fp32 ? tile_ok_t<float>(stage, g.ntheta, code) : tile_ok_t<double>(stage, g.ntheta, code);
    }
    return false;
}

long long stage_key(int stage, const DevGeom& g) {
    // run-time-length transforms launch per exact shape
    const long long shape = (1LL << 40) | ((long long)g.nr << 24) | ((long long)g.ntheta << 12) | g.nz;
    switch (stage) {
        case ST_DV: return g.dv_nseg * 100 + g.dv_seg;
        case ST_ZINV:
        case ST_ZFWD: return (!g.generic_fft && lane_length(g.nz)) ? g.nz : shape;
        case ST_THETA: return (!g.generic_fft && lane_length(g.ntheta)) ? g.ntheta : shape;
        case ST_RHS: return 0;
        case ST_SOLVE: return g.solve_seg;
    }
    return shape;
}

void launch_zinv(const Batch& B, bool fp32, hipStream_t s) {
    const DevGeom& g = B.g;
    if (!g.generic_fft && (fp32 ? zinv_fast<float>(B, s) : zinv_fast<double>(B, s))) return;
    const int jb = zcols_per_block(g.nz, g.nj);
    dim3 grid((g.nj + jb - 1) / jb, g.nr, B.count);
    if (fp32)
        hipLaunchKernelGGL(k_zinv<float>, grid, dim3(NT), (size_t)jb * g.nz * sizeof(C<float>), s, B.inst, jb);
    else
        hipLaunchKernelGGL(k_zinv<double>, grid, dim3(NT), (size_t)jb * g.nz * sizeof(C<double>), s, B.inst, jb);
}

void launch_theta(const Batch& B, bool fp32, hipStream_t s) {
    const DevGeom& g = B.g;
    if (!g.generic_fft && (fp32 ? theta_fast<float>(B, s) : theta_fast<double>(B, s))) return;
    dim3 grid(g.nz / 2, g.nr, B.count);
    if (fp32)
        hipLaunchKernelGGL(k_theta<float>, grid, dim3(NT), (size_t)3 * g.ntheta * sizeof(C<float>), s, B.inst);
    else
        hipLaunchKernelGGL(k_theta<double>, grid, dim3(NT), (size_t)3 * g.ntheta * sizeof(C<double>), s, B.inst);
}

void launch_zfwd(const Batch& B, bool fp32, hipStream_t s) {
    const DevGeom& g = B.g;
    if (!g.generic_fft && (fp32 ? zfwd_fast<float>(B, s) : zfwd_fast<double>(B, s))) return;
    const int jb = zcols_per_block(g.nz, g.nj);
    dim3 grid((g.nj + jb - 1) / jb, g.nr, B.count);
    if (fp32)
        hipLaunchKernelGGL(k_zfwd<float>, grid, dim3(NT), (size_t)jb * g.nz * sizeof(C<float>), s, B.inst, jb);
    else
        hipLaunchKernelGGL(k_zfwd<double>, grid, dim3(NT), (size_t)jb * g.nz * sizeof(C<double>), s, B.inst, jb);
}

bool rhs_fwd_ok(const DevGeom& g) {
    // whole columns per lane, the mean rows in one block, a segmented solve
    return g.rhs_rr >= g.nr - 4 && g.nr <= NT && g.solve_seg != 0;
}

int rhs_rows(int nr, int P, long long waves_per_chunk_row, bool fp32) {
    // FP64 launches with a thousand or more wavefronts per chunk row walk each
    // column in one chunk (no halo; measured fastest at 129 x 65280 modes)
    if (!fp32 && waves_per_chunk_row >= RHS_ONE_CHUNK_WAVES) return nr - 4;
    const int cap = min(nr - 4, RHS_MAX_ROWS);
    int rr = cap - ((cap - 1) % 5);
    (void)P;
    while (rr > 6 && (long long)((nr - 4 + rr - 1) / rr) * waves_per_chunk_row < RHS_MIN_WAVES) rr -= 5;
    return rr;
}

// B.g carries the largest nr and P and the smallest chunk of the batch, so the
// grid covers every member; lanes past a member's chunks or modes return.
template <typename TP>
void launch_rhs_t(const Batch& B, const StepCoef& c, int k, hipStream_t s) {
    const DevGeom& g = B.g;
    const int rr = g.rhs_rr;
    const size_t total = (size_t)((g.nr - 4 + rr - 1) / rr) * ((g.P + 63) & ~63);
    // grid.y = 1: the mean rows (ceil(nr / NT) of those blocks do work)
    const unsigned gx = (unsigned)std::max((total + NT - 1) / NT, (size_t)(g.nr + NT - 1) / NT);
    dim3 grid(gx, 2, B.count);
    if (g.rhs_fwd) {
        if (k == 0) hipLaunchKernelGGL((k_rhs<TP, 0, true>), grid, dim3(NT), 0, s, B.inst, c);
        else if (k == 1) hipLaunchKernelGGL((k_rhs<TP, 1, true>), grid, dim3(NT), 0, s, B.inst, c);
        else hipLaunchKernelGGL((k_rhs<TP, 2, true>), grid, dim3(NT), 0, s, B.inst, c);
        return;
    }
    if (k == 0) hipLaunchKernelGGL((k_rhs<TP, 0, false>), grid, dim3(NT), 0, s, B.inst, c);
    else if (k == 1) hipLaunchKernelGGL((k_rhs<TP, 1, false>), grid, dim3(NT), 0, s, B.inst, c);
    else hipLaunchKernelGGL((k_rhs<TP, 2, false>), grid, dim3(NT), 0, s, B.inst, c);
}

void launch_rhs(const Batch& B, bool fp32, const StepCoef& c, int k, hipStream_t s) {
    if (fp32)
        launch_rhs_t<float>(B, c, k, s);
    else
        launch_rhs_t<double>(B, c, k, s);
}

void launch_factor(const DevGeom& g, const DevBuf& b, const StepCoef& c, int k, hipStream_t s) {
    dim3 grid((g.npairs + SOLVE_NT - 1) / SOLVE_NT, 2);
    hipLaunchKernelGGL(k_factor, grid, dim3(SOLVE_NT), 0, s, g, b, c, k);
}

// Segments of the segmented solve: 8 segments of L rows (L = 4 or 8), or 16
// segments of 8 rows for up to 128 unknowns (at most 123 VGPRs per lane);
// 0 above that (sequential kernel).  Code 100 * segments + L, plus
// SOLVE_PAIRED for the paired lane layout.  The default is one lane per mode:
// on 129 x 65280 modes the paired layout reads half the factor bytes but
// measured 2 % slower (the second read of a pair's factors comes from cache);
// the autotuner has both.
constexpr int SOLVE_PAIRED = 10000;

int solve_segment_rows(int nr, int kz) {
    (void)kz;
    const int nu = nr - 2;
    if (nu <= 8 * 4) return 804;
    if (nu <= 8 * 8) return 808;
    if (nu <= 16 * 8) return 1608;
    return 0;
}

bool solve_shape_fits(int code, int nr) {
    const int base = code % SOLVE_PAIRED;
    if (code < 0 || code / SOLVE_PAIRED > 1) return false;
    if (base != 804 && base != 808 && base != 1608) return false;
    return (base / 100) * (base % 100) >= nr - 2;
}

// the segmented solve of shape B.g.solve_seg; false when the shape is not one
template <bool BACK>
static bool launch_solve_seg(const Batch& B, int k, hipStream_t s) {
    // grid.y selects the equation, grid.z the instance
    const dim3 gseg((B.g.P + 63) / 64, 2, B.count);
    // paired: B.g carries the largest nj and the largest K_z of the group
    const dim3 gpair(B.g.nj * ((B.g.kz + 32) / 32), 2, B.count);
    switch (B.g.solve_seg) {
        case 804: hipLaunchKernelGGL((k_solve_seg<4, 8, false, BACK>), gseg, dim3(64 * 8), 0, s, B.inst, k); return true;
        case 808: hipLaunchKernelGGL((k_solve_seg<8, 8, false, BACK>), gseg, dim3(64 * 8), 0, s, B.inst, k); return true;
        case 1608:
            hipLaunchKernelGGL((k_solve_seg<8, 16, false, BACK>), gseg, dim3(64 * 16), 0, s, B.inst, k);
            return true;
        case SOLVE_PAIRED + 804:
            hipLaunchKernelGGL((k_solve_seg<4, 8, true, BACK>), gpair, dim3(64 * 8), 0, s, B.inst, k);
            return true;
        case SOLVE_PAIRED + 808:
            hipLaunchKernelGGL((k_solve_seg<8, 8, true, BACK>), gpair, dim3(64 * 8), 0, s, B.inst, k);
            return true;
        case SOLVE_PAIRED + 1608:
            hipLaunchKernelGGL((k_solve_seg<8, 16, true, BACK>), gpair, dim3(64 * 16), 0, s, B.inst, k);
            return true;
    }
    return false;
}

void launch_solve(const Batch& B, int k, hipStream_t s) {
    if (B.g.rhs_fwd ? launch_solve_seg<true>(B, k, s) : launch_solve_seg<false>(B, k, s)) return;
    dim3 grid((B.g.npairs + SOLVE_NT - 1) / SOLVE_NT, 2, B.count);
    hipLaunchKernelGGL(k_solve_lu, grid, dim3(SOLVE_NT), 0, s, B.inst, k);
}

void launch_velocity(const DevGeom& g, const DevBuf& b, C<double>* u, C<double>* w, hipStream_t s) {
    const size_t total = (size_t)g.nr * g.P;
    hipLaunchKernelGGL(k_velocity, dim3((unsigned)((total + NT - 1) / NT)), dim3(NT), 0, s, g, b, u, w);
}

void launch_profiles(const DevGeom& g, const DevBuf& b, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_profiles, dim3(g.nr), dim3(RED_NT), 0, s, g, b, out);
}

void launch_stats(const DevGeom& g, const DevBuf& b, hipStream_t s) {
    const int nb = reduction_blocks(g);
    hipLaunchKernelGGL(k_energy, dim3(nb), dim3(RED_NT), 0, s, g, b);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(RED_NT), 0, s, g, b, nb);
}

// ------------------------------------------------ statistics without allocation
// The reduction partials, flags and results of the statistics kernels in a
// file-scope device array, for callers that cannot allocate device memory
// (tc_stats_noalloc).  Every GPU the library runs on holds its own copy until
// the process ends; its device address is looked up once per device, with
// that device current, and host code uses only that address (the array's
// name in host code is a host-side stand-in).  Layout, in doubles: partials
// [2][kNoallocBlocks], flags [kNoallocBlocks] ints, results [16].  Every call
// overwrites what it reads (each reduction block writes its own partial and
// flag), so nothing needs clearing; calls that overlap on one GPU share the
// array and race.
constexpr int kNoallocBlocks = 1024;
constexpr size_t kScratchDoubles = 2 * (size_t)kNoallocBlocks + kNoallocBlocks / 2 + 16;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

int noalloc_max_blocks() { return kNoallocBlocks; }

const double* launch_stats_noalloc(int device, const DevGeom& g, const DevBuf& b, hipStream_t s) {
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (device >= 0 && device < kMaxDevices) base = g_scratch_ptr[device];
    }
    const int nb = reduction_blocks(g);
    if (!base || nb > kNoallocBlocks) return nullptr;
    DevBuf t = b;
    t.partial = base;
    t.flags = reinterpret_cast<int*>(base + 2 * (size_t)kNoallocBlocks);
    t.stats = base + 2 * (size_t)kNoallocBlocks + kNoallocBlocks / 2;
    t.partial_n = kNoallocBlocks;
    launch_stats(g, t, s);
    return t.stats;
}

// non-finite flag of every instance of a shape class into its stats[5]
void launch_finite(const Batch& B, hipStream_t s) {
    const int nb = reduction_blocks(B.g);
    hipLaunchKernelGGL(k_finite, dim3(nb, 1, B.count), dim3(RED_NT), 0, s, B.inst);
    hipLaunchKernelGGL(k_flags_final, dim3(1, 1, B.count), dim3(RED_NT), 0, s, B.inst, nb);
}

}  // namespace tc

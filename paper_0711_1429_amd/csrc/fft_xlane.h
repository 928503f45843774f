// 768-point transform held by one wavefront whose exchanges between lanes
// are swaps of a 2-bit digit of the lane index with two bits of the register
// slot index: the highest digit in registers (permlane swaps across rows of 16
// lanes), the two lower digits either in registers too (DPP moves inside
// rows) or through a small LDS buffer (LOW_LDS, what the theta kernel uses).
//
// Lane g (0..63) holds 12 complex points in slots s = 4 grp + q (grp = 0..2,
// q = 0..3).  Write g = c + 4 d + 16 h with the 2-bit digits c, d, h.
//
// Transform with exponent +2 pi i / 768 ("inverse"):
//   input   slot s of lane g = X[g + 64 s]           (natural order)
//   P0      12-point DFT over the slots, then slot n1 times w^(n1 g)
//           (w = exp(2 pi i / 768))
//   P1      swap lane digit h with the slot digit q, 4-point DFTs over q,
//           slot digit a times w64^(a (c + 4 d))
//   P2      swap lane digit d with q, 4-point DFTs, slot digit a times
//           w16^(a c)
//   P3      swap lane digit c with q, 4-point DFTs
//   output  slot 4 grp + f of lane c + 4 d + 16 h holds position
//           4 grp + h + 12 d + 48 c + 192 f  (a fixed permutation, "pi order")
// This is the Cooley--Tukey split 768 = 12 x 64 with n = n1 + 12 n2,
// k = g + 64 s, and the 64-point DFT over the lane index taken as three
// radix-4 stages, each after bringing one 2-bit lane digit into the slots.
//
// Transform with exponent -2 pi i / 768 ("forward"): the same stages in
// reverse order with conjugate twiddles; it takes pi order and returns
// natural order (slot s of lane g = X[g + 64 s]).  Pointwise products of two
// fields in pi order are products of the same physical points, so the
// physical-space work between the two transforms never needs natural order.
//
// A digit swap exchanges two lane bits with the two low slot bits, one bit at
// a time: for a pair of slots (A, B) differing in slot bit b and a lane bit
// l, a lane whose bit l is 0 keeps A and receives its partner's A into B, a
// lane whose bit l is 1 keeps B and receives its partner's B into A (the 2 x 2
// transpose of (lane bit, slot bit)).  Lane bits 4 and 5 use
// v_permlane16_swap / v_permlane32_swap, which perform exactly this exchange
// on a pair of registers; lane bits 0..3 send the selected word with one DPP
// move (quad_perm for bits 0 and 1, row_ror for bits 2 and 3).
//
// With LOW_LDS the swaps of lane digits c and d go through a small LDS buffer
// instead (one group of four slots at a time: each lane writes its four
// slots, then reads the four values of its new slots), so only the swap of h
// is done in registers; the selects a DPP exchange needs cost more VALU time
// than the LDS round trip they replace.
//
// Twiddles come from an LDS table: w^(n1 g) for n1 = 1..11 as 11 rows of 64
// lanes (each lane reads its own column), then w64^(a m) for m = g mod 16 and
// w16^(a m) for m = g mod 4 (a = 1..3) as rows of 16 and 4 entries.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lane.h"

namespace tc {
namespace xlane {

constexpr int N = 768;
constexpr int P = 12;
constexpr int TW1 = 11 * 64;       // offset of the w64 rows in the twiddle table
constexpr int TW2 = TW1 + 3 * 16;  // offset of the w16 rows
constexpr int NTW = TW2 + 3 * 4;   // twiddle table entries
// LDS buffer of one wavefront for the LOW_LDS swaps: four slot rows, padded
// so that the reads of each swap hit distinct banks
constexpr int XPITCH0 = 65, XPITCH2 = 68;
constexpr int XBUF = 4 * XPITCH2;

template <typename T>
struct Words {
    unsigned w[sizeof(C<T>) / 4];
};

// the lane's bits 0..3 (which side of each DPP exchange it is on)
struct LaneBits {
    bool b[4];
    __device__ __forceinline__ explicit LaneBits(int g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (g >> i) & 1;
    }
};

// One 32-bit word of slots A (slot bit 0) and B (slot bit 1) exchanged
// between lanes that differ in lane bit LB.
template <int LB>
__device__ __forceinline__ void swap_word(unsigned& a, unsigned& b, bool bit) {
    if constexpr (LB == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else if constexpr (LB == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const unsigned t = bit ? a : b;  // what this lane sends
        unsigned lo, hi;                 // the partner's word, for lanes with bit l clear / set
        if constexpr (LB == 0) {
            lo = hi = __builtin_amdgcn_mov_dpp(t, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
        } else if constexpr (LB == 1) {
            lo = hi = __builtin_amdgcn_mov_dpp(t, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
        } else if constexpr (LB == 3) {
            lo = hi = __builtin_amdgcn_mov_dpp(t, 0x128, 0xF, 0xF, false);  // row_ror:8
        } else {
            lo = __builtin_amdgcn_mov_dpp(t, 0x12C, 0xF, 0xF, false);  // row_ror:12, from lane + 4
            hi = __builtin_amdgcn_mov_dpp(t, 0x124, 0xF, 0xF, false);  // row_ror:4, from lane - 4
        }
        a = bit ? hi : a;
        b = bit ? b : lo;
    }
}

// exchange lane bit LB with slot bit SB for every pair of slots
template <typename T, int LB, int SB>
__device__ __forceinline__ void bit_swap(C<T>* x, const LaneBits& lb) {
    const bool bit = LB < 4 ? lb.b[LB < 4 ? LB : 0] : false;
#pragma unroll
    for (int s = 0; s < P; ++s) {
        if ((s >> SB) & 1) continue;
        Words<T> a = __builtin_bit_cast(Words<T>, x[s]);
        Words<T> b = __builtin_bit_cast(Words<T>, x[s | (1 << SB)]);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(C<T>) / 4); ++i) swap_word<LB>(a.w[i], b.w[i], bit);
        x[s] = __builtin_bit_cast(C<T>, a);
        x[s | (1 << SB)] = __builtin_bit_cast(C<T>, b);
    }
}

// swap the 2-bit lane digit at bit D with the slot digit q
template <typename T, int D>
__device__ __forceinline__ void digit_swap(C<T>* x, const LaneBits& lb) {
    bit_swap<T, D, 0>(x, lb);
    bit_swap<T, D + 1, 1>(x, lb);
}

template <typename T, int SIGN>
__device__ __forceinline__ void radix4_groups(C<T>* x) {
#pragma unroll
    for (int grp = 0; grp < 3; ++grp) lane::dft4<T, SIGN>(x[4 * grp], x[4 * grp + 1], x[4 * grp + 2], x[4 * grp + 3]);
}

// x * w (CONJ false) or x * conj(w) (CONJ true)
template <typename T, bool CONJ>
__device__ __forceinline__ C<T> twiddle(C<T> x, C<T> w) {
    if constexpr (CONJ) return C<T>{x.x * w.x + x.y * w.y, x.y * w.x - x.x * w.y};
    return lane::mul(x, w);
}

// slot digit a = 1..3 of every group times entry a - 1 of the table rows at
// OFF (rows of M entries, indexed by g mod M)
template <typename T, bool CONJ, int OFF, int M>
__device__ __forceinline__ void twiddle_groups(C<T>* x, const C<T>* tw, int g) {
#pragma unroll
    for (int a = 1; a < 4; ++a) {
        const C<T> w = tw[OFF + (a - 1) * M + (g & (M - 1))];
#pragma unroll
        for (int grp = 0; grp < 3; ++grp) x[4 * grp + a] = twiddle<T, CONJ>(x[4 * grp + a], w);
    }
}

// Fill the twiddle table from the full table of exp(+2 pi i e / 768) (2 N
// reals); lane g writes column g of the w^(n1 g) rows and entry g of the
// shorter rows.
template <typename T, typename TwPtr>
__device__ __forceinline__ void fill_twiddles(C<T>* tw, TwPtr full, int g) {
    // every lane loads all its entries (the short tables at a clamped index)
    // before any is stored, so the loads are in flight together
    auto get = [&](int e) { return C<T>{full[2 * e], full[2 * e + 1]}; };
    C<T> t0[P - 1], t1[3], t2[3];
#pragma unroll
    for (int n1 = 1; n1 < P; ++n1) t0[n1 - 1] = get((n1 * g) % N);
#pragma unroll
    for (int a = 1; a < 4; ++a) {
        t1[a - 1] = get(12 * a * (g & 15));
        t2[a - 1] = get(48 * a * (g & 3));
    }
#pragma unroll
    for (int n1 = 1; n1 < P; ++n1) tw[(n1 - 1) * 64 + g] = t0[n1 - 1];
    if (g < 16)
#pragma unroll
        for (int a = 1; a < 4; ++a) tw[TW1 + (a - 1) * 16 + g] = t1[a - 1];
    if (g < 4)
#pragma unroll
        for (int a = 1; a < 4; ++a) tw[TW2 + (a - 1) * 4 + g] = t2[a - 1];
}

// The swap of the lane digit at bit D (0 or 2) with the slot digit through
// the wavefront's LDS buffer, one group of four slots at a time.  SYNC orders
// the buffer's writes and reads (the LDS accesses of one wavefront execute in
// order, so the next group may overwrite what the last one read).
template <typename T, int D, typename Sync>
__device__ __forceinline__ void lds_digit_swap(C<T>* x, C<T>* buf, int g, const Sync& sync) {
    constexpr int PITCH = D == 0 ? XPITCH0 : XPITCH2;
    const int mine = (g >> D) & 3;
    const int rest = g & ~(3 << D);
#pragma unroll
    for (int grp = 0; grp < 3; ++grp) {
#pragma unroll
        for (int q = 0; q < 4; ++q) buf[q * PITCH + g] = x[4 * grp + q];
        sync();
#pragma unroll
        for (int t = 0; t < 4; ++t) x[4 * grp + t] = buf[mine * PITCH + (rest | (t << D))];
        sync();
    }
}

template <typename T, int D, bool LOW_LDS, typename Sync>
__device__ __forceinline__ void swap_digit(C<T>* x, C<T>* buf, int g, const LaneBits& lb, const Sync& sync) {
    if constexpr (LOW_LDS && D < 4) lds_digit_swap<T, D>(x, buf, g, sync);
    else digit_swap<T, D>(x, lb);
}

// exponent +2 pi i / N: natural order in, pi order out
template <typename T, bool LOW_LDS, typename Sync>
__device__ __forceinline__ void inverse(C<T>* x, const C<T>* tw, C<T>* buf, int g, const LaneBits& lb,
                                        const Sync& sync) {
    lane::dft<T, 12, +1>(x);
#pragma unroll
    for (int n1 = 1; n1 < P; ++n1) x[n1] = twiddle<T, false>(x[n1], tw[(n1 - 1) * 64 + g]);
    swap_digit<T, 4, LOW_LDS>(x, buf, g, lb, sync);
    radix4_groups<T, +1>(x);
    twiddle_groups<T, false, TW1, 16>(x, tw, g);
    swap_digit<T, 2, LOW_LDS>(x, buf, g, lb, sync);
    radix4_groups<T, +1>(x);
    twiddle_groups<T, false, TW2, 4>(x, tw, g);
    swap_digit<T, 0, LOW_LDS>(x, buf, g, lb, sync);
    radix4_groups<T, +1>(x);
}

// exponent -2 pi i / N: pi order in, natural order out
template <typename T, bool LOW_LDS, typename Sync>
__device__ __forceinline__ void forward(C<T>* x, const C<T>* tw, C<T>* buf, int g, const LaneBits& lb,
                                        const Sync& sync) {
    radix4_groups<T, -1>(x);
    twiddle_groups<T, true, TW2, 4>(x, tw, g);
    swap_digit<T, 0, LOW_LDS>(x, buf, g, lb, sync);
    radix4_groups<T, -1>(x);
    swap_digit<T, 2, LOW_LDS>(x, buf, g, lb, sync);
    twiddle_groups<T, true, TW1, 16>(x, tw, g);
    radix4_groups<T, -1>(x);
    swap_digit<T, 4, LOW_LDS>(x, buf, g, lb, sync);
#pragma unroll
    for (int n1 = 1; n1 < P; ++n1) x[n1] = twiddle<T, true>(x[n1], tw[(n1 - 1) * 64 + g]);
    lane::dft<T, 12, -1>(x);
}

}  // namespace xlane
}  // namespace tc

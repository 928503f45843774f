// Host-side set-up of one Taylor--Couette instance: validated geometry,
// radial grid, compact finite-difference coefficients, the LU factors of the
// shared compact "denominator" d0, wavenumbers and FFT plans.  Plain C++,
// no HIP: everything here runs once per context on the CPU in extended
// precision and is rounded to double for the device.
#pragma once

#include <string>
#include <vector>

#include "../../include/tc.h"

namespace tc {

enum Family { F_D0 = 0, F_D1 = 1, F_D2 = 2, F_D2S = 3, F_D4S = 4, N_FAMILIES = 5 };

constexpr int MAX_RADICES = 12;
constexpr int MAX_FFT = 1536;

struct FftPlan {
    int n = 0;
    int npass = 0;
    int radix[MAX_RADICES] = {};
};

// Everything the device needs about one instance, computed on the host.
struct Setup {
    tc_geometry g{};
    int nr = 0, ntheta = 0, nz = 0;
    int kt = 0, kz = 0, nj = 0, nl = 0;
    double ri = 0, ro = 0, nu = 0, theta = 0, lz = 0, w_outer = 0;
    std::vector<double> r;            // [nr]
    std::vector<int> sigma;           // [nr] stencil start
    std::vector<double> coef;         // [N_FAMILIES][nr][5]
    // LU of the centred block (rows 2..nr-3) of d0, unpivoted, per row:
    // {l2, l1, 1/u0, u1, u2}
    std::vector<double> blu;          // [nr][5]
    // Segmented sweeps of the same system (dv_nseg segments of dv_seg rows of
    // the centred block; dv_seg = 0 when the block has more than 128 rows): the
    // responses of the forward and backward recurrences inside each segment
    // to unit values carried in from the neighbouring segment,
    // [4][nr] = {forward from y_{s0-1}, forward from y_{s0-2},
    //            backward from x_{s1}, backward from x_{s1+1}}.
    int dv_seg = 0;
    int dv_nseg = 0;
    std::vector<double> dvh;          // [4][nr]
    std::vector<double> m;            // [nj]   m_j
    std::vector<double> alpha;        // [nl]   alpha_l, l = -kz..kz
    std::vector<double> tw_theta;     // [2*ntheta] exp(+2 pi i k / ntheta)
    std::vector<double> tw_z;         // [2*nz]
    FftPlan plan_theta, plan_z;

    double c(int fam, int n, int j) const { return coef[(fam * nr + n) * 5 + j]; }
};


// Validate g and fill s.  Returns TC_OK or TC_EINVAL with a message in err.
int build_setup(const tc_geometry& g, Setup& s, std::string& err);

// Factor n into radices 4, 3, 2 (in that preference).  Returns false when n
// has another prime factor.
bool make_plan(int n, FftPlan& p);

}  // namespace tc

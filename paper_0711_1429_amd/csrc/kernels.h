// Device-side data of one instance and the launchers of the substep kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "host_setup.h"

namespace tc {

template <typename T>
struct C {
    T x, y;
};

// The same pointer in the global address space.  Every buffer the kernels
// touch outside LDS is global memory, but pointers read from the instance
// descriptors are generic, and loads and stores through generic pointers
// compile to flat instructions, which count against the LDS wait counter as
// well and so make every LDS wait also wait for outstanding memory traffic.
// TC_GLOBAL qualifies such pointers in signatures.  (The host pass, which
// only parses device code, keeps generic pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TC_GLOBAL __attribute__((address_space(1)))
#else
#define TC_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ TC_GLOBAL T* glb(T* p) {
    return (TC_GLOBAL T*)p;
}

// base[i] with a 32-bit element offset (the byte offset must stay below
// 4 GiB): with a wave-uniform base the access compiles to a scalar base plus
// a 32-bit lane offset instead of a 64-bit address per lane.
template <typename T>
__device__ __forceinline__ TC_GLOBAL T& at(TC_GLOBAL T* base, unsigned i) {
    return *(TC_GLOBAL T*)((TC_GLOBAL char*)base + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const TC_GLOBAL T& at(const TC_GLOBAL T* base, unsigned i) {
    return *(const TC_GLOBAL T*)((const TC_GLOBAL char*)base + i * (unsigned)sizeof(T));
}

// p, the same in every lane, held in scalar registers (so that the compiler
// keeps it as the scalar base of the accesses through it)
template <typename T>
__device__ __forceinline__ T* uniform(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
#else
    return p;
#endif
}

// A table that no kernel writes, in the constant address space: reads of it
// at wave-uniform addresses compile to scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define TC_CONST __attribute__((address_space(4)))
#else
#define TC_CONST
#endif
template <typename T>
__device__ __forceinline__ const TC_CONST T* cst(const T* p) {
    return (const TC_CONST T*)p;
}

struct FftPlanDev {
    int n;
    int npass;
    int radix[MAX_RADICES];
};

// Read-only per-instance tables on the device, passed by value to kernels.
struct DevGeom {
    int nr, nj, nl, kt, kz, ntheta, nz;
    int P;            // nj * nl modes per radial plane
    int mean;         // index of the (0,0) mode within a plane (= kz)
    int npairs;       // nj * (kz + 1)
    double nu, w_outer, dt;
    const double* r;        // [nr]
    const int* sigma;       // [nr]
    const double* coef;     // [5][nr][5]
    const double* blu;      // [nr][5]
    const double* dvh;      // [4][nr] segment responses of the d0 sweeps
    int dv_seg;             // rows per segment of the segmented D v kernel, 0: sequential kernel
    int dv_nseg;            // segments of the segmented D v kernel
    int rhs_rr;             // rows per chunk of the RHS kernel
    int solve_seg;          // segment shape of the radial solve (100 * segments + rows, + 10000 for
                            // the paired lane layout), 0: sequential
    const double* m;        // [nj]
    const double* alpha;    // [nl]
    const double* tw_theta; // [ntheta] complex
    const double* tw_z;     // [nz] complex
    const float* tw_theta_f;
    const float* tw_z_f;
    const double* wr;       // [nr] trapezoid weight * r
    FftPlanDev plan_theta, plan_z;
    int generic_fft;        // 1: run-time-length FFT kernels even for compiled lengths
    int tile_zinv;          // tile shape of the fixed-length z kernels: 0 default columns per
    int tile_zfwd;          //   block, 1 half, 2 twice (when that shape is compiled)
    int tile_theta;         // theta kernel wavefronts per block: 0 default, 1, 2, 3 for 1, 2, 4;
                            //   at N_theta = 768 also 4 (Stockham transform), 5 (register exchanges)
    int linear;             // 1: no products (the transform stages are not launched)
    int rhs_fwd;            // 1: the explicit-term kernel (one chunk per column) also runs the
                            //   solve's forward elimination; the segmented solve only substitutes back
};

// Coefficients of one substep of the low-storage RK3 / Crank--Nicolson
// scheme (the time step and viscosity are per instance, in DevGeom).
struct StepCoef {
    double gamma;    // weight of N^{k-1}
    double rho;      // weight of N^{k-2}
    double beta;     // Crank--Nicolson weight
};

// Device buffers of one instance.  c128 arrays are [nr][nj][nl].
struct DevBuf {
    C<double>* v;
    C<double>* eta;
    void* nv[2];       // explicit-term registers of v, alternating by substep (mean slot
                       // unused); complex of the transform precision
    void* neta[2];     // the same for eta (mean slot unused)
    double* nmean;     // [2][2][nr] explicit terms of the mean axial and azimuthal
                       // profiles, alternating like nv/neta; FP64 in both precisions
    C<double>* dv;     // radial derivative of v
    C<double>* rv;     // right-hand side / forward-elimination values of v
    C<double>* re;     // the same for eta
    double* umean;
    double* wmean;
    void* zb;          // [3][nr][nz][nj]  after the inverse z transform (T)
    void* pb;          // [6][nr][nz][nj]  products after the forward theta transform (T)
    void* ps;          // [6][nr][nj][nl]  product spectra (T)
    double* lu;        // [3][2][5][nr][npairs] precomputed LU factors per substep
    double* fold;      // [3][2][2][npairs] boundary-row folding factors
    double* mwall;     // [3][2][nr] wall terms of the mean-profile right-hand sides
    double* partial;   // reduction partials
    int* flags;        // reduction flags
    double* stats;     // [16] statistics
    int partial_n;     // capacity of partial (doubles) / flags (ints)
};

// One instance's tables and buffers, as the batched kernels read them from
// device memory (blockIdx.z selects the instance).
struct InstDev {
    DevGeom g;
    DevBuf b;
};

// Instances that share (N_r, N_theta, N_z) and the transform path run in one
// launch per kernel: inst points to `count` consecutive InstDev in device
// memory; g is a host copy of any member's tables (launch shapes only).
struct Batch {
    const InstDev* inst;
    int count;
    DevGeom g;
};

enum KernelId {
    K_DV = 0,
    K_ZINV,
    K_THETA,
    K_ZFWD,
    K_RHS,
    K_SOLVE,
    K_ENERGY,
    K_FINITE,
    K_COUNT
};

extern const char* const kKernelNames[K_COUNT];

void launch_dv(const Batch& B, hipStream_t s);
void launch_zinv(const Batch& B, bool fp32, hipStream_t s);
void launch_theta(const Batch& B, bool fp32, hipStream_t s);
void launch_zfwd(const Batch& B, bool fp32, hipStream_t s);
void launch_rhs(const Batch& B, bool fp32, const StepCoef& c, int k, hipStream_t s);

// Step stages and their launch-group keys: instances whose keys agree share
// one launch of the stage's kernel (same compile-time variant); the grid then
// covers the largest member and every block checks its own instance's
// extents.  A Batch passed to a launcher carries those largest extents.
enum Stage { ST_DV, ST_ZINV, ST_THETA, ST_ZFWD, ST_RHS, ST_SOLVE, ST_COUNT };
long long stage_key(int stage, const DevGeom& g);
// rows per chunk of the RHS kernel for an instance launched with `waves`
// wavefronts per chunk row in total
int rhs_rows(int nr, int P, long long waves_per_chunk_row, bool fp32);
// whether the explicit-term launch of g can also run the solve's forward
// elimination (DevGeom::rhs_fwd): one chunk per column, N_r at most one block
// of mean rows, a segmented solve
bool rhs_fwd_ok(const DevGeom& g);
// the default segment shape and lane layout of the radial solve, and whether
// shape `code` is compiled and covers nr - 2 unknowns
int solve_segment_rows(int nr, int kz);
bool solve_shape_fits(int code, int nr);
// whether tile code `code` of a transform stage (ST_ZINV, ST_THETA, ST_ZFWD)
// is compiled for the group's transform length and precision
bool tile_variant_ok(int stage, const DevGeom& g, bool fp32, int code);
// precomputed LU factors of substep k (run once per context and k)
void launch_factor(const DevGeom& g, const DevBuf& b, const StepCoef& c, int k, hipStream_t s);
void launch_solve(const Batch& B, int k, hipStream_t s);
// spectral u, w of the current state (needs b.dv up to date)
void launch_velocity(const DevGeom& g, const DevBuf& b, C<double>* u, C<double>* w, hipStream_t s);
// energy reductions + finite check + statistics into b.stats
void launch_stats(const DevGeom& g, const DevBuf& b, hipStream_t s);
// radial profiles [6][nr] (mean u, mean w, <u'u'>, <v'v'>, <w'w'>, <v'w'>) into device memory out
void launch_profiles(const DevGeom& g, const DevBuf& b, double* out, hipStream_t s);
// The statistics with their reduction scratch in the library's file-scope
// device array instead of b.partial / b.flags / b.stats.  noalloc_scratch_init
// looks up that array's address on `device` (which must be current) once;
// launch_stats_noalloc returns the device address of the 5 results, or null
// when the device was not initialised or the grid needs more reduction blocks
// than the array holds.
hipError_t noalloc_scratch_init(int device);
int noalloc_max_blocks();
const double* launch_stats_noalloc(int device, const DevGeom& g, const DevBuf& b, hipStream_t s);
// finite check of the state into b.flags[0]
void launch_finite(const Batch& B, hipStream_t s);

// Launch-shape helpers shared by the host code (buffer sizing).
int zcols_per_block(int nz, int nj);
int reduction_blocks(const DevGeom& g);

}  // namespace tc

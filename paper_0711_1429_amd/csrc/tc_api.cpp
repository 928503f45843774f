// C ABI of libtc.so (declared in include/tc.h): contexts, device memory,
// field I/O with validation, the substep sequence and statistics.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tc.h"
#include "host_setup.h"
#include "kernels.h"

using namespace tc;

namespace {

// Low-storage RK3 coefficients (reading of Sec. 2.1 / Sec. 3.1: the paper
// names a 3-substep Runge--Kutta scheme with Crank--Nicolson viscous terms
// but prints no coefficients): gamma, rho and the Crank--Nicolson weight
// beta = (gamma + rho) / 2 of each substep.
constexpr double kGamma[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double kRho[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

struct Instance {
    Setup s;
    DevGeom g{};
    DevBuf b{};
    std::vector<void*> allocs;
    double time = 0.0;
    long long steps = 0;
    int red_blocks = 1;
    const InstDev* self = nullptr;  // this instance's entry in the array of all instances
};

// Instances of the same shape (the non-finite check runs per shape).
struct ShapeClass {
    DevGeom g{};
    std::vector<int> members;
    InstDev* dev = nullptr;
};

// Instances that share one launch of a step stage's kernel (equal stage key);
// g holds the largest extents of the members (see stage_key).
struct LaunchGroup {
    long long key = 0;
    DevGeom g{};
    std::vector<int> members;
    InstDev* dev = nullptr;
};

struct TimedLaunch {
    int id;
    hipEvent_t start, stop;
};

}  // namespace

// a side stream of the step graph and the event that joins it back
struct Branch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};
constexpr int kMaxBranches = 16;

struct tc_ctx {
    std::vector<Instance> inst;
    std::vector<Branch> branch;         // step-graph branches (several shape classes)
    hipEvent_t fork = nullptr;
    std::vector<ShapeClass> classes;
    std::vector<LaunchGroup> groups[ST_COUNT];
    InstDev* all_dev = nullptr;         // descriptors of all instances, in order
    std::vector<void*> allocs;          // class arrays
    double* hflags = nullptr;           // pinned: one non-finite flag per instance
    bool use_graphs = true;
    bool rhs_elimination = true;        // forward elimination in the explicit-term kernel where it fits
    hipGraphExec_t step_graph = nullptr;  // one full step of every instance
    hipStream_t graph_stream = nullptr;
    bool dryrun = false;
    bool fp32 = false;
    hipStream_t own = nullptr;
    hipStream_t stream = nullptr;
    int device = -1;                    // HIP device the context was created on
    std::string err;
    bool timing = false;
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> pool;
    double ms[K_COUNT] = {};
    long long calls[K_COUNT] = {};
};

namespace {

thread_local std::string g_create_error;

int fail(tc_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(tc_ctx* c, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? TC_ENOMEM : TC_EDEVICE, m);
}

#define HIPCHK(ctx, call)                                  \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

hipEvent_t take_event(tc_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs fn() (which launches kernel `id` on c->stream), bracketed by events
// when timing is on.
template <typename F>
void timed(tc_ctx* c, int id, F fn) {
    if (!c->timing) {
        fn();
        return;
    }
    TimedLaunch t{id, take_event(c), take_event(c)};
    if (t.start) (void)hipEventRecord(t.start, c->stream);
    fn();
    if (t.stop) (void)hipEventRecord(t.stop, c->stream);
    c->pending.push_back(t);
}

void collect_timing(tc_ctx* c) {
    if (c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& t : c->pending) {
        float ms = 0.0f;
        if (t.start && t.stop && hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
            c->ms[t.id] += ms;
            c->calls[t.id] += 1;
        }
        if (t.start) c->pool.push_back(t.start);
        if (t.stop) c->pool.push_back(t.stop);
    }
    c->pending.clear();
}

int check_launch(tc_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, what);
    return TC_OK;
}

StepCoef step_coef(int k) {
    StepCoef sc;
    sc.gamma = kGamma[k];
    sc.rho = kRho[k];
    sc.beta = 0.5 * (kGamma[k] + kRho[k]);
    return sc;
}

template <typename T>
int dev_alloc(tc_ctx* c, Instance& in, T** p, size_t count) {
    void* q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
    in.allocs.push_back(q);
    *p = static_cast<T*>(q);
    return TC_OK;
}

template <typename T>
int upload(tc_ctx* c, Instance& in, const T** p, const std::vector<T>& host) {
    T* d = nullptr;
    int rc = dev_alloc(c, in, &d, host.size());
    if (rc) return rc;
    HIPCHK(c, hipMemcpy(d, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
    *p = d;
    return TC_OK;
}

int alloc_instance(tc_ctx* c, Instance& in) {
    const Setup& s = in.s;
    DevGeom& g = in.g;
    g.nr = s.nr;
    g.nj = s.nj;
    g.nl = s.nl;
    g.kt = s.kt;
    g.kz = s.kz;
    g.ntheta = s.ntheta;
    g.nz = s.nz;
    g.P = s.nj * s.nl;
    g.mean = s.kz;
    g.npairs = s.nj * (s.kz + 1);
    g.nu = s.nu;
    g.w_outer = s.w_outer;
    g.dt = s.g.dt;
    auto plan = [](const FftPlan& p) {
        FftPlanDev d{};
        d.n = p.n;
        d.npass = p.npass;
        for (int i = 0; i < MAX_RADICES; ++i) d.radix[i] = p.radix[i];
        return d;
    };
    g.generic_fft = (s.g.flags & TC_FLAG_GENERIC_FFT) ? 1 : 0;
    g.linear = (s.g.flags & TC_FLAG_LINEAR) ? 1 : 0;
    g.plan_theta = plan(s.plan_theta);
    g.plan_z = plan(s.plan_z);

    std::vector<double> wr(s.nr);
    for (int n = 0; n < s.nr; ++n) {
        double w = n == 0 ? 0.5 * (s.r[1] - s.r[0])
                 : n == s.nr - 1 ? 0.5 * (s.r[n] - s.r[n - 1])
                 : 0.5 * (s.r[n + 1] - s.r[n - 1]);
        wr[n] = w * s.r[n];
    }
    std::vector<float> twt(s.tw_theta.begin(), s.tw_theta.end());
    std::vector<float> twz(s.tw_z.begin(), s.tw_z.end());
    int rc;
    if ((rc = upload(c, in, &g.r, s.r))) return rc;
    if ((rc = upload(c, in, &g.sigma, s.sigma))) return rc;
    if ((rc = upload(c, in, &g.coef, s.coef))) return rc;
    if ((rc = upload(c, in, &g.blu, s.blu))) return rc;
    if ((rc = upload(c, in, &g.dvh, s.dvh))) return rc;
    g.dv_seg = s.dv_seg;
    g.solve_seg = solve_segment_rows(s.nr, s.kz);
    g.dv_nseg = s.dv_nseg;
    if ((rc = upload(c, in, &g.m, s.m))) return rc;
    if ((rc = upload(c, in, &g.alpha, s.alpha))) return rc;
    if ((rc = upload(c, in, &g.tw_theta, s.tw_theta))) return rc;
    if ((rc = upload(c, in, &g.tw_z, s.tw_z))) return rc;
    if ((rc = upload(c, in, &g.tw_theta_f, twt))) return rc;
    if ((rc = upload(c, in, &g.tw_z_f, twz))) return rc;
    if ((rc = upload(c, in, &g.wr, wr))) return rc;

    const size_t S = (size_t)s.nr * g.P;
    const size_t Q = (size_t)s.nr * s.nz * s.nj;
    const size_t cz = c->fp32 ? sizeof(C<float>) : sizeof(C<double>);
    DevBuf& b = in.b;
    C<double>** c128[] = {&b.v, &b.eta, &b.dv, &b.rv, &b.re};
    for (auto p : c128)
        if ((rc = dev_alloc(c, in, p, S))) return rc;
    // the N registers hold the explicit terms of the previous substep at the
    // precision of the products they are formed from
    char* nreg = nullptr;
    if ((rc = dev_alloc(c, in, &nreg, 4 * S * cz))) return rc;
    HIPCHK(c, hipMemset(nreg, 0, 4 * S * cz));
    for (int q = 0; q < 2; ++q) {
        b.nv[q] = nreg + (size_t)(2 * q) * S * cz;
        b.neta[q] = nreg + (size_t)(2 * q + 1) * S * cz;
    }
    if ((rc = dev_alloc(c, in, &b.nmean, (size_t)4 * s.nr))) return rc;
    HIPCHK(c, hipMemset(b.nmean, 0, (size_t)4 * s.nr * sizeof(double)));
    if ((rc = dev_alloc(c, in, &b.umean, s.nr))) return rc;
    if ((rc = dev_alloc(c, in, &b.wmean, s.nr))) return rc;
    char* raw = nullptr;
    if ((rc = dev_alloc(c, in, &raw, 3 * Q * cz))) return rc;
    b.zb = raw;
    if ((rc = dev_alloc(c, in, &raw, 6 * Q * cz))) return rc;
    b.pb = raw;
    if ((rc = dev_alloc(c, in, &raw, 6 * S * cz))) return rc;
    b.ps = raw;
    HIPCHK(c, hipMemset(b.ps, 0, 6 * S * cz));  // stays zero for TC_FLAG_LINEAR
    if ((rc = dev_alloc(c, in, &b.lu, (size_t)3 * 2 * 5 * s.nr * g.npairs))) return rc;
    if ((rc = dev_alloc(c, in, &b.fold, (size_t)3 * 2 * 2 * g.npairs))) return rc;
    if ((rc = dev_alloc(c, in, &b.mwall, (size_t)3 * 2 * s.nr))) return rc;
    in.red_blocks = reduction_blocks(g);
    b.partial_n = in.red_blocks;
    if ((rc = dev_alloc(c, in, &b.partial, (size_t)2 * in.red_blocks))) return rc;
    if ((rc = dev_alloc(c, in, &b.flags, (size_t)in.red_blocks))) return rc;
    if ((rc = dev_alloc(c, in, &b.stats, 16))) return rc;
    for (auto p : c128) HIPCHK(c, hipMemset(*p, 0, S * sizeof(C<double>)));
    HIPCHK(c, hipMemset(b.umean, 0, s.nr * sizeof(double)));
    HIPCHK(c, hipMemset(b.wmean, 0, s.nr * sizeof(double)));
    HIPCHK(c, hipMemset(b.lu, 0, (size_t)3 * 2 * 5 * s.nr * g.npairs * sizeof(double)));
    HIPCHK(c, hipMemset(b.fold, 0, (size_t)3 * 2 * 2 * g.npairs * sizeof(double)));
    HIPCHK(c, hipMemset(b.mwall, 0, (size_t)3 * 2 * s.nr * sizeof(double)));
    for (int k = 0; k < 3; ++k) launch_factor(g, b, step_coef(k), k, c->stream);
    if (int e = check_launch(c, "factor launch")) return e;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TC_OK;
}

void free_instance(Instance& in) {
    for (void* p : in.allocs) (void)hipFree(p);
    in.allocs.clear();
}

Instance* get_inst(tc_ctx* c, int i) {
    if (!c || i < 0 || i >= (int)c->inst.size()) return nullptr;
    return &c->inst[i];
}

int need_device(tc_ctx* c) {
    if (c->dryrun) return fail(c, TC_EINVAL, "context was created with TC_FLAG_DRYRUN (host only)");
    return TC_OK;
}

Batch batch_of(const ShapeClass& cl) { return Batch{cl.dev, (int)cl.members.size(), cl.g}; }
Batch batch_of(const LaunchGroup& gr) { return Batch{gr.dev, (int)gr.members.size(), gr.g}; }
Batch batch_of(const Instance& in) { return Batch{in.self, 1, in.g}; }

// Stage st of substep k for one launch group on stream s.
void group_stage(tc_ctx* c, int st, const LaunchGroup& gr, int k, hipStream_t s) {
    const Batch B = batch_of(gr);
    switch (st) {
        case ST_DV: timed(c, K_DV, [&] { launch_dv(B, s); }); break;
        case ST_ZINV: timed(c, K_ZINV, [&] { launch_zinv(B, c->fp32, s); }); break;
        case ST_THETA: timed(c, K_THETA, [&] { launch_theta(B, c->fp32, s); }); break;
        case ST_ZFWD: timed(c, K_ZFWD, [&] { launch_zfwd(B, c->fp32, s); }); break;
        case ST_RHS: timed(c, K_RHS, [&] { launch_rhs(B, c->fp32, step_coef(k), k, s); }); break;
        case ST_SOLVE: timed(c, K_SOLVE, [&] { launch_solve(B, k, s); }); break;
    }
}

// roctx range names of the substeps (a profiler shows each substep's
// launches under its range; host-side markers, nothing is added to the stream)
const char* const kSubstepRange[3] = {"tc substep 1", "tc substep 2", "tc substep 3"};

int run_substep(tc_ctx* c, int k) {
    roctxRangePushA(kSubstepRange[k]);
    for (int st = 0; st < ST_COUNT; ++st)
        for (auto& gr : c->groups[st]) group_stage(c, st, gr, k, c->stream);
    roctxRangePop();
    return check_launch(c, "substep launch");
}

int products_only(tc_ctx* c, Instance& in) {
    hipStream_t s = c->stream;
    const Batch B = batch_of(in);
    launch_dv(B, s);
    if (in.g.linear) return check_launch(c, "product launch");  // products stay zero
    launch_zinv(B, c->fp32, s);
    launch_theta(B, c->fp32, s);
    launch_zfwd(B, c->fp32, s);
    return check_launch(c, "product launch");
}

int upload_descriptors(tc_ctx* c);

// Group instances by launch shape and upload the per-class instance arrays.
int build_classes(tc_ctx* c) {
    for (int i = 0; i < (int)c->inst.size(); ++i) {
        const DevGeom& g = c->inst[i].g;
        ShapeClass* found = nullptr;
        for (auto& cl : c->classes)
            if (cl.g.nr == g.nr && cl.g.ntheta == g.ntheta && cl.g.nz == g.nz && cl.g.generic_fft == g.generic_fft)
                found = &cl;
        if (!found) {
            c->classes.push_back(ShapeClass{});
            found = &c->classes.back();
            found->g = g;
        }
        found->members.push_back(i);
    }
    // RHS chunk length per instance, from the wavefronts of one launch over all instances
    long long rhs_waves = 0;
    for (auto& in : c->inst) rhs_waves += (in.g.P + 63) / 64;
    for (auto& in : c->inst) in.g.rhs_rr = rhs_rows(in.g.nr, in.g.P, rhs_waves, c->fp32);
    // launch groups per stage, keyed by stage_key; extents are the members' largest
    for (int st = 0; st < ST_COUNT; ++st) {
        auto& G = c->groups[st];
        for (int i = 0; i < (int)c->inst.size(); ++i) {
            const DevGeom& g = c->inst[i].g;
            if (g.linear && (st == ST_ZINV || st == ST_THETA || st == ST_ZFWD)) continue;
            const long long key = stage_key(st, g);
            LaunchGroup* found = nullptr;
            for (auto& gr : G)
                if (gr.key == key) found = &gr;
            if (!found) {
                G.push_back(LaunchGroup{});
                found = &G.back();
                found->key = key;
                found->g = g;
            }
            DevGeom& m = found->g;
            m.nr = std::max(m.nr, g.nr);
            m.nj = std::max(m.nj, g.nj);
            m.P = std::max(m.P, g.P);
            m.npairs = std::max(m.npairs, g.npairs);
            if (st == ST_SOLVE) m.kz = std::max(m.kz, g.kz);  // the paired grid covers every member
            m.rhs_rr = std::min(m.rhs_rr, g.rhs_rr);
            if (st == ST_THETA) m.nz = std::max(m.nz, g.nz);
            found->members.push_back(i);
        }
    }
    // device descriptor arrays: one per launch group, one per shape class, and
    // one of all instances (the single-instance launches)
    auto alloc_array = [&](size_t n, InstDev** out) -> int {
        void* q = nullptr;
        if (hipMalloc(&q, n * sizeof(InstDev)) != hipSuccess) return fail(c, TC_ENOMEM, "hipMalloc of descriptors");
        c->allocs.push_back(q);
        *out = static_cast<InstDev*>(q);
        return TC_OK;
    };
    for (int st = 0; st < ST_COUNT; ++st)
        for (auto& gr : c->groups[st])
            if (int rc = alloc_array(gr.members.size(), &gr.dev)) return rc;
    for (auto& cl : c->classes)
        if (int rc = alloc_array(cl.members.size(), &cl.dev)) return rc;
    if (int rc = alloc_array(c->inst.size(), &c->all_dev)) return rc;
    for (size_t i = 0; i < c->inst.size(); ++i) c->inst[i].self = c->all_dev + i;
    return upload_descriptors(c);
}

// DevGeom::rhs_fwd of every instance and launch group from the current launch
// parameters: on for a context of one instance whose explicit-term launch
// takes whole columns and whose solve is segmented (rhs_fwd_ok).
static void refresh_rhs_fwd(tc_ctx* c) {
    const bool one = c->inst.size() == 1;
    for (auto& in : c->inst) in.g.rhs_fwd = (c->rhs_elimination && one && rhs_fwd_ok(in.g)) ? 1 : 0;
    for (int st = 0; st < ST_COUNT; ++st)
        for (auto& gr : c->groups[st]) {
            int f = 1;
            for (int i : gr.members) f = f && c->inst[i].g.rhs_fwd;
            gr.g.rhs_fwd = f;
        }
}

// Copy every instance's current DevGeom/DevBuf into the device descriptor
// arrays (after a change of a per-instance launch parameter).
int upload_descriptors(tc_ctx* c) {
    refresh_rhs_fwd(c);
    auto put = [&](const std::vector<int>& members, InstDev* dev) {
        std::vector<InstDev> host(members.size());
        for (size_t q = 0; q < members.size(); ++q) host[q] = InstDev{c->inst[members[q]].g, c->inst[members[q]].b};
        return hipMemcpy(dev, host.data(), host.size() * sizeof(InstDev), hipMemcpyHostToDevice);
    };
    for (int st = 0; st < ST_COUNT; ++st)
        for (auto& gr : c->groups[st]) HIPCHK(c, put(gr.members, gr.dev));
    for (auto& cl : c->classes) {
        cl.g = c->inst[cl.members[0]].g;
        HIPCHK(c, put(cl.members, cl.dev));
    }
    std::vector<int> all(c->inst.size());
    for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
    HIPCHK(c, put(all, c->all_dev));
    return TC_OK;
}

void drop_graph(tc_ctx* c) {
    if (c->step_graph) (void)hipGraphExecDestroy(c->step_graph);
    c->step_graph = nullptr;
    c->graph_stream = nullptr;
}

// Capture one full step (3 substeps of every instance) into a graph on the
// current stream.  A stage with several launch groups forks them onto side
// streams and joins them back before the next stage (the groups of a stage
// share no memory), so they run concurrently on replay.  The captured work
// has no memset or host callback nodes.
int capture_step(tc_ctx* c) {
    drop_graph(c);
    int maxg = 1;
    for (int st = 0; st < ST_COUNT; ++st) maxg = std::max(maxg, (int)c->groups[st].size());
    const int nbranch = maxg > 1 ? std::min(maxg, kMaxBranches) : 0;
    while ((int)c->branch.size() < nbranch) {
        Branch br;
        if (hipStreamCreateWithFlags(&br.stream, hipStreamNonBlocking) != hipSuccess)
            return fail(c, TC_EDEVICE, "hipStreamCreate for a graph branch failed");
        if (hipEventCreateWithFlags(&br.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(br.stream);
            return fail(c, TC_EDEVICE, "hipEventCreate for a graph branch failed");
        }
        c->branch.push_back(br);
    }
    if (nbranch && !c->fork) HIPCHK(c, hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
    hipGraph_t graph = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = TC_OK;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        for (int st = 0; st < ST_COUNT && e == hipSuccess; ++st) {
            const auto& G = c->groups[st];
            if (G.size() == 1 || nbranch == 0) {
                for (const auto& gr : G) group_stage(c, st, gr, k, c->stream);
                continue;
            }
            const int nb = std::min((int)G.size(), nbranch);
            e = hipEventRecord(c->fork, c->stream);
            for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(c->branch[b].stream, c->fork, 0);
            for (size_t q = 0; q < G.size() && e == hipSuccess; ++q) group_stage(c, st, G[q], k, c->branch[q % nb].stream);
            for (int b = 0; b < nb && e == hipSuccess; ++b) {
                e = hipEventRecord(c->branch[b].done, c->branch[b].stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->branch[b].done, 0);
            }
        }
    }
    if (e != hipSuccess) rc = hip_fail(c, e, "graph branch fork/join");
    else rc = check_launch(c, "substep launch");
    e = hipStreamEndCapture(c->stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->step_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->step_graph = nullptr;
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    c->graph_stream = c->stream;
    return TC_OK;
}

// Host checks of loaded fields (see tc_load_fields in tc.h).
int validate_fields(tc_ctx* c, const Instance& in, const double* v, const double* eta, const double* um,
                    const double* wm) {
    const Setup& s = in.s;
    const size_t P = (size_t)s.nj * s.nl;
    const size_t S = (size_t)s.nr * P;
    for (size_t i = 0; i < 2 * S; ++i)
        if (!std::isfinite(v[i]) || !std::isfinite(eta[i])) return fail(c, TC_ENONFINITE, "non-finite v or eta");
    for (int n = 0; n < s.nr; ++n)
        if (!std::isfinite(um[n]) || !std::isfinite(wm[n]))
            return fail(c, TC_ENONFINITE, "non-finite mean profile");
    for (int wall : {0, s.nr - 1})
        for (size_t i = 0; i < 2 * P; ++i)
            if (v[2 * wall * P + i] != 0.0 || eta[2 * wall * P + i] != 0.0)
                return fail(c, TC_ESHAPE, "v and eta must vanish at the walls");
    const int kz = s.kz;
    for (int n = 0; n < s.nr; ++n) {
        const size_t base = 2 * ((size_t)n * P);
        const size_t mean = base + 2 * (size_t)kz;
        if (v[mean] != 0.0 || v[mean + 1] != 0.0 || eta[mean] != 0.0 || eta[mean + 1] != 0.0)
            return fail(c, TC_ESHAPE, "the (0,0) slots of v and eta must be zero (mean flow is separate)");
        for (int l = 1; l <= kz; ++l) {
            const size_t p = base + 2 * (size_t)(kz + l), q = base + 2 * (size_t)(kz - l);
            if (v[p] != v[q] || v[p + 1] != -v[q + 1] || eta[p] != eta[q] || eta[p + 1] != -eta[q + 1])
                return fail(c, TC_ESHAPE, "the j = 0 column must be Hermitian: f[0][-l] = conj(f[0][l])");
        }
    }
    if (um[0] != 0.0 || um[s.nr - 1] != 0.0) return fail(c, TC_ESHAPE, "u_mean must vanish at both walls");
    if (wm[0] != 1.0 || wm[s.nr - 1] != s.w_outer)
        return fail(c, TC_ESHAPE, "w_mean must equal 1 at the inner wall and re_outer/re at the outer wall");
    return TC_OK;
}

}  // namespace

extern "C" {

int tc_abi_version(void) { return TC_ABI_VERSION; }

int tc_create(const tc_geometry* g, int n_instances, tc_ctx** out) {
    g_create_error.clear();
    if (!g || !out) return fail(nullptr, TC_EINVAL, "null argument");
    if (n_instances < 1 || n_instances > 4096) return fail(nullptr, TC_EINVAL, "n_instances must be in [1, 4096]");
    tc_ctx* c = new (std::nothrow) tc_ctx();
    if (!c) return fail(nullptr, TC_ENOMEM, "host allocation failed");
    c->dryrun = (g[0].flags & TC_FLAG_DRYRUN) != 0;
    c->fp32 = g[0].precision == TC_PREC_MIXED;
    c->inst.resize(n_instances);
    for (int i = 0; i < n_instances; ++i) {
        std::string err;
        if (g[i].precision != g[0].precision || (g[i].flags & TC_FLAG_DRYRUN) != (g[0].flags & TC_FLAG_DRYRUN)) {
            delete c;
            return fail(nullptr, TC_EINVAL, "all instances must share precision and flags");
        }
        int rc = build_setup(g[i], c->inst[i].s, err);
        if (rc) {
            delete c;
            return fail(nullptr, rc, "instance " + std::to_string(i) + ": " + err);
        }
    }
    if (!c->dryrun) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
            delete c;
            return fail(nullptr, TC_EDEVICE, "no HIP device");
        }
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            delete c;
            return fail(nullptr, TC_EDEVICE, "cannot query the HIP device");
        }
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            delete c;
            return fail(nullptr, TC_EDEVICE, std::string("libtc.so is built for gfx950, device is ") + prop.gcnArchName);
        }
        c->device = dev;
        // the static reduction scratch of tc_stats_noalloc: its address on this device
        if (hipError_t e = noalloc_scratch_init(dev); e != hipSuccess) {
            delete c;
            return fail(nullptr, TC_EDEVICE, std::string("static scratch lookup failed: ") + hipGetErrorString(e));
        }
        if (hipStreamCreate(&c->own) != hipSuccess) {
            delete c;
            return fail(nullptr, TC_EDEVICE, "hipStreamCreate failed");
        }
        c->stream = c->own;
        int rc = TC_OK;
        for (auto& in : c->inst)
            if ((rc = alloc_instance(c, in))) break;
        if (!rc) rc = build_classes(c);
        if (!rc && hipHostMalloc((void**)&c->hflags, sizeof(double) * n_instances) != hipSuccess)
            rc = fail(c, TC_ENOMEM, "hipHostMalloc of the flag buffer failed");
        if (rc) {
            std::string m = c->err;
            for (auto& x : c->inst) free_instance(x);
            for (void* p : c->allocs) (void)hipFree(p);
            if (c->hflags) (void)hipHostFree(c->hflags);
            (void)hipStreamDestroy(c->own);
            delete c;
            return fail(nullptr, rc, m);
        }
    }
    *out = c;
    return TC_OK;
}

int tc_destroy(tc_ctx* c) {
    if (!c) return TC_OK;
    if (!c->dryrun) {
        (void)hipStreamSynchronize(c->stream);
        drop_graph(c);
        for (auto& br : c->branch) {
            (void)hipEventDestroy(br.done);
            (void)hipStreamDestroy(br.stream);
        }
        if (c->fork) (void)hipEventDestroy(c->fork);
        for (auto& in : c->inst) free_instance(in);
        for (void* p : c->allocs) (void)hipFree(p);
        if (c->hflags) (void)hipHostFree(c->hflags);
        for (auto& t : c->pending) {
            if (t.start) (void)hipEventDestroy(t.start);
            if (t.stop) (void)hipEventDestroy(t.stop);
        }
        for (auto e : c->pool) (void)hipEventDestroy(e);
        if (c->own) (void)hipStreamDestroy(c->own);
    }
    delete c;
    return TC_OK;
}

int tc_set_stream(tc_ctx* c, void* stream) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    collect_timing(c);
    (void)hipStreamSynchronize(c->stream);
    c->stream = stream ? static_cast<hipStream_t>(stream) : c->own;
    drop_graph(c);
    return TC_OK;
}

int tc_mode_shape(const tc_ctx* cc, int inst, int* nr, int* nj, int* nl) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (nr) *nr = in->s.nr;
    if (nj) *nj = in->s.nj;
    if (nl) *nl = in->s.nl;
    return TC_OK;
}

int tc_grid(const tc_ctx* cc, int inst, double* r) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in || !r) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    std::memcpy(r, in->s.r.data(), in->s.nr * sizeof(double));
    return TC_OK;
}

int tc_load_fields(tc_ctx* c, int inst, const double* v, const double* eta, const double* um, const double* wm) {
    Instance* in = get_inst(c, inst);
    if (!in || !v || !eta || !um || !wm) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (int rc = validate_fields(c, *in, v, eta, um, wm)) return rc;
    const size_t S = (size_t)in->s.nr * in->g.P;
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(in->b.v, v, S * 16, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(in->b.eta, eta, S * 16, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(in->b.umean, um, in->s.nr * 8, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(in->b.wmean, wm, in->s.nr * 8, hipMemcpyHostToDevice, s));
    const size_t cz = c->fp32 ? sizeof(C<float>) : sizeof(C<double>);
    for (int q = 0; q < 2; ++q) {
        HIPCHK(c, hipMemsetAsync(in->b.nv[q], 0, S * cz, s));
        HIPCHK(c, hipMemsetAsync(in->b.neta[q], 0, S * cz, s));
    }
    HIPCHK(c, hipMemsetAsync(in->b.nmean, 0, (size_t)4 * in->s.nr * sizeof(double), s));
    HIPCHK(c, hipStreamSynchronize(s));
    in->time = 0.0;
    in->steps = 0;
    return TC_OK;
}

int tc_get_fields(tc_ctx* c, int inst, double* v, double* eta, double* um, double* wm) {
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    const size_t S = (size_t)in->s.nr * in->g.P;
    hipStream_t s = c->stream;
    if (v) HIPCHK(c, hipMemcpyAsync(v, in->b.v, S * 16, hipMemcpyDeviceToHost, s));
    if (eta) HIPCHK(c, hipMemcpyAsync(eta, in->b.eta, S * 16, hipMemcpyDeviceToHost, s));
    if (um) HIPCHK(c, hipMemcpyAsync(um, in->b.umean, in->s.nr * 8, hipMemcpyDeviceToHost, s));
    if (wm) HIPCHK(c, hipMemcpyAsync(wm, in->b.wmean, in->s.nr * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return TC_OK;
}

static int finite_check(tc_ctx* c) {
    // one launch pair per shape class; every instance's flag lands in pinned
    // host memory, with one wait for all
    const int n = (int)c->inst.size();
    for (auto& cl : c->classes) timed(c, K_FINITE, [&] { launch_finite(batch_of(cl), c->stream); });
    if (int rc = check_launch(c, "finite check")) return rc;
    for (int i = 0; i < n; ++i)
        HIPCHK(c, hipMemcpyAsync(c->hflags + i, c->inst[i].b.stats + 5, sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n; ++i)
        if (c->hflags[i] != 0.0)
            return fail(c, TC_ENONFINITE, "non-finite values in the state of instance " + std::to_string(i));
    return TC_OK;
}

int tc_step(tc_ctx* c, int nsteps) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (nsteps < 0) return fail(c, TC_EINVAL, "nsteps must be >= 0");
    // graphs replay whole steps; per-kernel timing needs the eager launches
    const bool graph = c->use_graphs && !c->timing && nsteps > 0;
    if (graph && (!c->step_graph || c->graph_stream != c->stream))
        if (int rc = capture_step(c)) return rc;
    for (int it = 0; it < nsteps; ++it) {
        if (graph) {
            roctxRangePushA("tc step (graph replay)");
            const hipError_t e = hipGraphLaunch(c->step_graph, c->stream);
            roctxRangePop();
            HIPCHK(c, e);
        } else {
            for (int k = 0; k < 3; ++k)
                if (int rc = run_substep(c, k)) return rc;
        }
        for (auto& in : c->inst) {
            in.time += in.s.g.dt;
            in.steps += 1;
        }
    }
    if (int rc = finite_check(c)) return rc;
    return TC_OK;
}

int tc_substep(tc_ctx* c, int k) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (k < 1 || k > 3) return fail(c, TC_EINVAL, "substep index must be 1, 2 or 3");
    if (int rc = run_substep(c, k - 1)) return rc;
    return finite_check(c);
}

int tc_velocity(tc_ctx* c, int inst, double* u, double* w) {
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    const size_t S = (size_t)in->s.nr * in->g.P;
    launch_dv(batch_of(*in), c->stream);
    // rv / re are scratch between substeps
    launch_velocity(in->g, in->b, in->b.rv, in->b.re, c->stream);
    if (int rc = check_launch(c, "velocity")) return rc;
    if (u) HIPCHK(c, hipMemcpyAsync(u, in->b.rv, S * 16, hipMemcpyDeviceToHost, c->stream));
    if (w) HIPCHK(c, hipMemcpyAsync(w, in->b.re, S * 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TC_OK;
}

int tc_products(tc_ctx* c, int inst, double* prod) {
    Instance* in = get_inst(c, inst);
    if (!in || !prod) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (int rc = products_only(c, *in)) return rc;
    const size_t S = (size_t)in->s.nr * in->g.P;
    if (c->fp32) {
        std::vector<float> tmp(12 * S);
        HIPCHK(c, hipMemcpyAsync(tmp.data(), in->b.ps, 12 * S * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < 12 * S; ++i) prod[i] = tmp[i];
    } else {
        HIPCHK(c, hipMemcpyAsync(prod, in->b.ps, 12 * S * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return TC_OK;
}

int tc_profiles(tc_ctx* c, int inst, double* out) {
    Instance* in = get_inst(c, inst);
    if (!in || !out) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    launch_dv(batch_of(*in), c->stream);
    // rv is scratch between substeps; 6 nr doubles fit in its 2 nr P
    double* dev = reinterpret_cast<double*>(in->b.rv);
    launch_profiles(in->g, in->b, dev, c->stream);
    if (int rc = check_launch(c, "profiles")) return rc;
    HIPCHK(c, hipMemcpyAsync(out, dev, (size_t)6 * in->s.nr * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return TC_OK;
}

namespace {

// The statistics of instance `in` from the 5 reduction results st (wall
// shear g at both walls, energy sums with and without the mean, non-finite
// flag).
void fill_stats(const Instance* in, const double st[5], tc_stats_t* out) {
    const Setup& s = in->s;
    double vol = 0.0;
    for (int n = 0; n < s.nr; ++n) {
        double w = n == 0 ? 0.5 * (s.r[1] - s.r[0])
                 : n == s.nr - 1 ? 0.5 * (s.r[n] - s.r[n - 1])
                 : 0.5 * (s.r[n + 1] - s.r[n - 1]);
        vol += w * s.r[n];
    }
    const double gi = st[0], go = st[1];
    out->time = in->time;
    out->torque_in = 2.0 * M_PI * s.ri * gi;
    out->torque_out = 2.0 * M_PI * s.ro * s.ro * go / s.ri;
    out->tau_in = s.nu * gi;
    out->tau_out = s.nu * go;
    out->retau_in = std::sqrt(out->tau_in) * 0.5 * s.g.gap / s.nu;
    out->retau_out = std::sqrt(out->tau_out) * 0.5 * s.g.gap / s.nu;
    out->energy = st[2] / (2.0 * vol);
    out->energy_pert = st[3] / (2.0 * vol);
    out->steps = in->steps;
    out->nonfinite = st[4] != 0.0;
}

}  // namespace

int tc_stats(tc_ctx* c, int inst, tc_stats_t* out) {
    Instance* in = get_inst(c, inst);
    if (!in || !out) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    timed(c, K_DV, [&] { launch_dv(batch_of(*in), c->stream); });
    timed(c, K_ENERGY, [&] { launch_stats(in->g, in->b, c->stream); });
    if (int rc = check_launch(c, "stats")) return rc;
    double st[5];
    HIPCHK(c, hipMemcpyAsync(st, in->b.stats, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_stats(in, st, out);
    return TC_OK;
}

int tc_stats_noalloc(tc_ctx* c, int inst, tc_stats_t* out) {
    Instance* in = get_inst(c, inst);
    if (!in || !out) return c ? fail(c, TC_EINVAL, "bad instance index or null pointer") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (reduction_blocks(in->g) > noalloc_max_blocks())
        return fail(c, TC_EINVAL, "the grid needs " + std::to_string(reduction_blocks(in->g)) +
                                      " reduction blocks; the static scratch holds " +
                                      std::to_string(noalloc_max_blocks()));
    int cur = -1;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != c->device) return fail(c, TC_EINVAL, "the context's device is not the current HIP device");
    launch_dv(batch_of(*in), c->stream);
    const double* res = launch_stats_noalloc(c->device, in->g, in->b, c->stream);
    if (!res) return fail(c, TC_EDEVICE, "static scratch not initialised on this device");
    if (int rc = check_launch(c, "stats (static scratch)")) return rc;
    double st[5];
    HIPCHK(c, hipMemcpyAsync(st, res, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_stats(in, st, out);
    return TC_OK;
}

int tc_timing(tc_ctx* c, int enable) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    collect_timing(c);
    if (enable) {
        for (int i = 0; i < K_COUNT; ++i) {
            c->ms[i] = 0.0;
            c->calls[i] = 0;
        }
    }
    c->timing = enable != 0;
    return TC_OK;
}

int tc_kernel_times(tc_ctx* c, double* ms, long long* calls, int n) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    collect_timing(c);
    for (int i = 0; i < n && i < K_COUNT; ++i) {
        if (ms) ms[i] = c->ms[i];
        if (calls) calls[i] = c->calls[i];
    }
    return TC_OK;
}

int tc_set_rhs_elimination(tc_ctx* c, int enable) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    (void)hipStreamSynchronize(c->stream);
    c->rhs_elimination = enable != 0;
    drop_graph(c);
    return upload_descriptors(c);
}

int tc_use_graphs(tc_ctx* c, int enable) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    (void)hipStreamSynchronize(c->stream);
    c->use_graphs = enable != 0;
    drop_graph(c);
    return TC_OK;
}

namespace {

// Mean duration (ms) of `reps` launches of stage st for group gr, substep k.
int time_stage(tc_ctx* c, int st, const LaunchGroup& gr, int k, int reps, hipEvent_t e0, hipEvent_t e1,
               double* ms) {
    const Batch B = batch_of(gr);
    auto launch = [&] {
        switch (st) {
            case ST_RHS: launch_rhs(B, c->fp32, step_coef(k), k, c->stream); break;
            case ST_SOLVE: launch_solve(B, k, c->stream); break;
            case ST_ZINV: launch_zinv(B, c->fp32, c->stream); break;
            case ST_THETA: launch_theta(B, c->fp32, c->stream); break;
            case ST_ZFWD: launch_zfwd(B, c->fp32, c->stream); break;
        }
    };
    launch();  // warm
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) launch();
    HIPCHK(c, hipEventRecord(e1, c->stream));
    if (int rc = check_launch(c, "autotune launch")) return rc;
    HIPCHK(c, hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    return TC_OK;
}

}  // namespace

int tc_autotune(tc_ctx* c, int repeats) {
    if (!c) return TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    if (repeats < 1 || repeats > 1000) return fail(c, TC_EINVAL, "repeats must be in [1, 1000]");
    collect_timing(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    const bool was_timing = c->timing;
    c->timing = false;
    // candidates are timed with the plain explicit-term and solve kernels
    const bool was_elim = c->rhs_elimination;
    c->rhs_elimination = false;
    // snapshot the state and the N registers; the tuning runs one substep to
    // fill every intermediate and then re-launches idempotent stages
    std::vector<void*> snap;
    auto cleanup = [&] {
        for (void* p : snap) (void)hipFree(p);
        c->timing = was_timing;
        c->rhs_elimination = was_elim;
    };
    struct Copy {
        void* dst;
        const void* src;
        size_t bytes;
    };
    std::vector<Copy> saved;
    const size_t cz = c->fp32 ? sizeof(C<float>) : sizeof(C<double>);
    for (auto& in : c->inst) {
        const size_t S = (size_t)in.s.nr * in.g.P;
        const std::pair<void*, size_t> parts[] = {{in.b.v, S * 16}, {in.b.eta, S * 16},
                                                  {in.b.umean, in.s.nr * 8ul}, {in.b.wmean, in.s.nr * 8ul},
                                                  {in.b.nv[0], S * cz}, {in.b.neta[0], S * cz},
                                                  {in.b.nv[1], S * cz}, {in.b.neta[1], S * cz},
                                                  {in.b.nmean, in.s.nr * 32ul}};
        for (auto& pr : parts) {
            void* q = nullptr;
            if (hipMalloc(&q, pr.second) != hipSuccess) {
                cleanup();
                return fail(c, TC_ENOMEM, "autotune: no memory for the state snapshot");
            }
            snap.push_back(q);
            saved.push_back(Copy{q, pr.first, pr.second});
            if (hipMemcpyAsync(q, pr.first, pr.second, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
                cleanup();
                return fail(c, TC_EDEVICE, "autotune: snapshot copy failed");
            }
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TC_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(c, TC_EDEVICE, "hipEventCreate");
    const int k = 1;  // a substep that reads and writes the N registers
    if (!rc) rc = run_substep(c, k);
    // RHS chunks per column, per launch group: with n chunks every member takes
    // rr = ceil((nr - 4) / n) rows per chunk (the last chunk overlaps its
    // neighbour by less than n rows); the group's grid is sized by the
    // largest nr and the smallest rr, and lanes past a member's chunks return
    for (auto& gr : c->groups[ST_RHS]) {
        if (rc) break;
        std::vector<int> best_rr;
        double best = 1e30;
        // candidates: n chunks per member (n > 0), or -n rows for every member
        for (int cand : {1, 2, 3, 4, 5, 6, 8, 10, -21, -16, -11, -6}) {
            std::vector<int> rr;
            int rr_min = 1 << 30;
            bool ok = true;
            for (int i : gr.members) {
                const int rows = c->inst[i].g.nr - 4;
                rr.push_back(cand > 0 ? (rows + cand - 1) / cand : -cand);
                ok = ok && rr.back() <= rows;
                rr_min = std::min(rr_min, rr.back());
            }
            if (!ok) continue;
            for (size_t m = 0; m < gr.members.size(); ++m) c->inst[gr.members[m]].g.rhs_rr = rr[m];
            gr.g.rhs_rr = rr_min;
            if ((rc = upload_descriptors(c))) break;
            double ms = 0;
            if ((rc = time_stage(c, ST_RHS, gr, k, repeats, e0, e1, &ms))) break;
            if (ms < best) {
                best = ms;
                best_rr = rr;
            }
        }
        if (rc) break;
        int rr_min = 1 << 30;
        for (size_t m = 0; m < gr.members.size(); ++m) {
            c->inst[gr.members[m]].g.rhs_rr = best_rr[m];
            rr_min = std::min(rr_min, best_rr[m]);
        }
        gr.g.rhs_rr = rr_min;
    }
    // segment shape of the radial solve, per launch group
    for (auto& gr : c->groups[ST_SOLVE]) {
        if (rc || gr.g.solve_seg == 0) continue;
        int best_code = gr.g.solve_seg;
        double best = 1e30;
        for (int code : {804, 808, 1608, 10804, 10808, 11608}) {
            if (!solve_shape_fits(code, gr.g.nr)) continue;
            gr.g.solve_seg = code;
            double ms = 0;
            if ((rc = time_stage(c, ST_SOLVE, gr, k, repeats, e0, e1, &ms))) break;
            if (ms < best) {
                best = ms;
                best_code = code;
            }
        }
        gr.g.solve_seg = best_code;
        for (int i : gr.members) c->inst[i].g.solve_seg = best_code;
    }
    // tile shapes of the transform stages, per launch group (the stages read
    // only the state and the previous stage's output, so they can be
    // relaunched at will; the arithmetic of every element is the same)
    for (int st : {ST_ZINV, ST_THETA, ST_ZFWD}) {
        for (auto& gr : c->groups[st]) {
            if (rc) break;
            int& field = st == ST_ZINV ? gr.g.tile_zinv : (st == ST_THETA ? gr.g.tile_theta : gr.g.tile_zfwd);
            int best_code = field;
            double best = 1e30;
            // (theta code 6, the other form of w's fetch, changes at most the
            // rounding, as the solve's segment shapes do; codes 4 and 5 are
            // other transforms and not candidates)
            for (int code : {0, 1, 2, 3, 6}) {
                if (code == 6 && st != ST_THETA) continue;
                if (!tile_variant_ok(st, gr.g, c->fp32, code)) continue;
                field = code;
                double ms = 0;
                if ((rc = time_stage(c, st, gr, k, repeats, e0, e1, &ms))) break;
                if (ms < best) {
                    best = ms;
                    best_code = code;
                }
            }
            field = best_code;
            for (int i : gr.members) {
                DevGeom& mg = c->inst[i].g;
                (st == ST_ZINV ? mg.tile_zinv : (st == ST_THETA ? mg.tile_theta : mg.tile_zfwd)) = best_code;
            }
        }
    }
    c->rhs_elimination = was_elim;
    if (!rc) rc = upload_descriptors(c);
    // restore the state
    for (auto& cp : saved)
        if (!rc && hipMemcpyAsync(const_cast<void*>(cp.src), cp.dst, cp.bytes, hipMemcpyDeviceToDevice, c->stream) !=
                       hipSuccess)
            rc = fail(c, TC_EDEVICE, "autotune: restore copy failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess && !rc) rc = fail(c, TC_EDEVICE, "autotune: synchronise");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    cleanup();
    return rc;
}

int tc_set_rhs_rows(tc_ctx* c, int inst, int rows) {
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (rows < 1 || rows > in->g.nr - 4) return fail(c, TC_EINVAL, "rows per chunk must be in [1, nr - 4]");
    if (int rc = need_device(c)) return rc;
    in->g.rhs_rr = rows;
    // the launch group's grid covers its members with the smallest chunk
    for (auto& gr : c->groups[ST_RHS]) {
        bool member = false;
        int rr_min = 1 << 30;
        for (int i : gr.members) {
            member = member || i == inst;
            rr_min = std::min(rr_min, c->inst[i].g.rhs_rr);
        }
        if (member) gr.g.rhs_rr = rr_min;
    }
    drop_graph(c);
    return upload_descriptors(c);
}

int tc_tuning(const tc_ctx* cc, int inst, int* rhs_rows_out, int* solve_shape_out) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (rhs_rows_out) *rhs_rows_out = in->g.rhs_rr;
    if (solve_shape_out) *solve_shape_out = in->g.solve_seg;
    return TC_OK;
}

namespace {

// The launch group of stage st that holds instance inst.
LaunchGroup* group_of(tc_ctx* c, int st, int inst) {
    for (auto& gr : c->groups[st])
        for (int i : gr.members)
            if (i == inst) return &gr;
    return nullptr;
}

}  // namespace

int tc_set_solve_shape(tc_ctx* c, int inst, int code) {
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    LaunchGroup* gr = group_of(c, ST_SOLVE, inst);
    if (!gr || gr->g.solve_seg == 0) return fail(c, TC_EINVAL, "this instance's solve is not segmented");
    for (int i : gr->members)
        if (!solve_shape_fits(code, c->inst[i].g.nr))
            return fail(c, TC_EINVAL, "solve shape " + std::to_string(code) + " does not fit instance " +
                                          std::to_string(i));
    gr->g.solve_seg = code;
    for (int i : gr->members) c->inst[i].g.solve_seg = code;
    drop_graph(c);
    return upload_descriptors(c);
}

int tc_set_tiles(tc_ctx* c, int inst, int zinv, int theta, int zfwd) {
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (int rc = need_device(c)) return rc;
    const int want[3] = {zinv, theta, zfwd};
    const int stages[3] = {ST_ZINV, ST_THETA, ST_ZFWD};
    for (int q = 0; q < 3; ++q) {
        LaunchGroup* gr = group_of(c, stages[q], inst);
        if (gr && !tile_variant_ok(stages[q], gr->g, c->fp32, want[q]))
            return fail(c, TC_EINVAL, "tile code " + std::to_string(want[q]) + " is not compiled for this stage");
        if (!gr && want[q] != 0) return fail(c, TC_EINVAL, "this instance has no transform stages");
    }
    for (int q = 0; q < 3; ++q) {
        LaunchGroup* gr = group_of(c, stages[q], inst);
        if (!gr) continue;
        auto field = [&](DevGeom& g) -> int& {
            return q == 0 ? g.tile_zinv : (q == 1 ? g.tile_theta : g.tile_zfwd);
        };
        field(gr->g) = want[q];
        for (int i : gr->members) field(c->inst[i].g) = want[q];
    }
    drop_graph(c);
    return upload_descriptors(c);
}

int tc_tiles(const tc_ctx* cc, int inst, int* zinv, int* theta, int* zfwd) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (zinv) *zinv = in->g.tile_zinv;
    if (theta) *theta = in->g.tile_theta;
    if (zfwd) *zfwd = in->g.tile_zfwd;
    return TC_OK;
}

int tc_kernel_count(void) { return K_COUNT; }

const char* tc_kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kKernelNames[id] : ""; }

double tc_kernel_bytes(const tc_ctx* cc, int inst, int id) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in) return 0.0;
    const double S = (double)in->s.nr * in->s.nj * in->s.nl;  // spectral points
    const double Q = (double)in->s.nr * in->s.nz * in->s.nj;  // mixed-space points
    const double t = c->fp32 ? 8.0 : 16.0;                    // complex size on the FFT side
    switch (id) {
        case K_DV: return 32.0 * S;                           // read v, write D v
        case K_ZINV: return 48.0 * S + 3.0 * t * Q;           // read v, eta, D v; write 3 fields
        case K_THETA: return 3.0 * t * Q + 6.0 * t * Q;       // read 3 fields; write 6 products
        case K_ZFWD: return 6.0 * t * Q + 6.0 * t * S;        // read 6; write 6 spectra
        case K_RHS:  // read v, eta, D v and 6 spectra, write the RHS of v and eta; the
                     // N registers (2 complex of the transform precision) are read by
                     // substeps 2, 3 and written by 1, 2 (the average over a step is given);
                     // with the forward elimination also the l2, l1 fields of both equations
            return (48.0 + 6.0 * t + 2.0 * t * 2.0 / 3.0 + 2.0 * t * 2.0 / 3.0 + 32.0) * S +
                   (in->g.rhs_fwd ? 32.0 * in->s.nr * in->s.nj * (in->s.kz + 1.0) : 0.0);
        case K_SOLVE:  // read RHS and the 5 LU fields of both equations (3 after the
                       // forward elimination in the explicit-term kernel), write v, eta
            return 32.0 * S + (in->g.rhs_fwd ? 48.0 : 80.0) * in->s.nr * in->s.nj * (in->s.kz + 1.0) + 32.0 * S;
        case K_ENERGY: return 48.0 * S;
        case K_FINITE: return 32.0 * S;
    }
    return 0.0;
}

int tc_coefficients(const tc_ctx* cc, int inst, double* coef, int* sigma) {
    tc_ctx* c = const_cast<tc_ctx*>(cc);
    Instance* in = get_inst(c, inst);
    if (!in) return c ? fail(c, TC_EINVAL, "bad instance index") : TC_EINVAL;
    if (coef) std::memcpy(coef, in->s.coef.data(), in->s.coef.size() * sizeof(double));
    if (sigma) std::memcpy(sigma, in->s.sigma.data(), in->s.sigma.size() * sizeof(int));
    return TC_OK;
}

const char* tc_last_error(const tc_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

}  // extern "C"

// C ABI of libteuk (declared and documented in include/teuk.h).
//
// A single-instance handle is a batch of one: both forms build the same
// per-instance descriptors and launch the same step kernel, so batched and
// single-instance results are bitwise identical by construction.
#include "teuk.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dispatch.hpp"

namespace {

thread_local std::string g_err;

constexpr size_t kMaxRowsLds = 40 * 1024;
constexpr unsigned long long kMaxPlaneDoubles = 1ull << 32;
constexpr int kMaxObserverPoints = 1024;
constexpr double kMaxObserverDoubles = 268435456.0;   // 2^28 doubles (2 GiB) of records

// Scratch of teuk_coefficients_noalloc: a device array each GPU holds from
// the library's load until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is handed to kernels and copies.
constexpr size_t kScratchDoubles = (size_t)1 << 20;      // 8 MiB per device
__device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};


int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? TEUK_ENOMEM : TEUK_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

int scratch_on_current_device(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TEUK_ENOTSUP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(TEUK_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return TEUK_OK;
}

int validate(int s, int m, double a_over_M, const teuk_grid *g, int prec) {
    (void)m;
    if (!g) return fail(TEUK_EINVAL, "grid is NULL");
    if (s < -2 || s > 2) return fail(TEUK_EINVAL, "spin weight s must satisfy |s| <= 2");
    if (!(std::fabs(a_over_M) < 1.0)) return fail(TEUK_EINVAL, "|a/M| must be < 1");
    if (g->n_theta < 5) return fail(TEUK_EINVAL, "n_theta must be >= 5 (ghost rows reflect up to 5 rows)");
    if (g->n_theta > 256) return fail(TEUK_ENOTSUP, "n_theta > 256 is not supported by this build");
    if (g->n_r < 3) return fail(TEUK_EINVAL, "n_r must be >= 3");
    if (!(g->rstar_min < g->rstar_max) || !std::isfinite(g->rstar_min) || !std::isfinite(g->rstar_max))
        return fail(TEUK_EINVAL, "need finite rstar_min < rstar_max");
    if (!(g->cfl > 0.0) || !std::isfinite(g->cfl)) return fail(TEUK_EINVAL, "cfl must be > 0");
    if (g->angular_order != 10 && g->angular_order != 2)
        return fail(TEUK_EINVAL, "angular_order must be 10 or 2");
    if (prec != TEUK_FP64 && prec != TEUK_DD && prec != TEUK_QD)
        return fail(TEUK_EINVAL, "precision must be 1 (FP64), 2 (double-double) or 4 (quad-double)");
    // The step kernels address a plane (one word of one component) with
    // 32-bit offsets; the largest array, the eight coefficient components of
    // `prec` words each, must stay below 2^32 doubles.
    if (8ull * (unsigned long long)prec * (unsigned long long)g->n_r * (unsigned long long)g->n_theta >= kMaxPlaneDoubles)
        return fail(TEUK_ENOTSUP, "grid too large: 8 * words * n_r * n_theta must be below 2^32");
    if (g->mass == 0.0) {
        if (a_over_M != 0.0 || !(g->rstar_min > 0.0))
            return fail(TEUK_EINVAL, "flat-space mode (mass 0) needs a/M = 0 and rstar_min > 0");
    } else if (g->mass != 1.0) {
        return fail(TEUK_EINVAL, "mass must be 1.0 (or 0.0 for the flat-space test mode)");
    }
    return TEUK_OK;
}

// Coefficient source of the double-double wide sweep (lwk::wide_launch
// cmode): 0 stored planes loaded in the stage, 3 the same planes requested
// one phase ahead (bitwise equal to 0), 4 rebuilt per point from
// double-double radial rows.  TEUK_DD_COEF=0|3|4 overrides the default.
int dd_cmode_default() {
    const char *v = std::getenv("TEUK_DD_COEF");
    if (v && (v[0] == '0' || v[0] == '3' || v[0] == '4') && v[1] == 0) return v[0] - '0';
    return 0;
}

struct Instance {
    int s = 0, m = 0, words = 1, reach = 5;
    double a_over_M = 0.0;
    teuk_grid g{};
    double *u[2] = {nullptr, nullptr};
    double *ch = nullptr, *cf = nullptr, *wt = nullptr;
    int onfly = 0;                                   // FP64: per-point coefficients from rows
    int injected = 0;                                // coefficients set by teuk_set_coefficients: planes only
    double *rf = nullptr, *rh = nullptr, *trig = nullptr;
    double hdt[lwk::kMaxWords] = {}, dt[lwk::kMaxWords] = {};
    double dt_lead = 0.0;
    int cur = 0;            // buffer holding the current fields
    long steps = 0;
    size_t plane() const { return (size_t)g.n_r * g.n_theta; }
    size_t hplane() const { return (size_t)(g.n_r - 1) * g.n_theta; }
};

struct Batch {
    int words = 1;
    std::vector<Instance> inst;
    int seg_req = 8;         // requested r* nodes per work item
    int segcols = 8;         // in use: seg_req, shortened where the FP64 radial rows exceed their LDS share
    int nt = 64;
    int nt_req = 0;          // requested block size (0 = default for the sweep)
    int sweep_req = -1;      // requested sweep (TEUK_SWEEP_*; -1 = default for the precision)
    int sweep = 0;           // sweep in use
    int cmode = 0;           // wide sweep: coefficient mode (see lwk::wide_launch)
    int tm = 0;              // wide sweep: unrolled iteration count (0 = loop)
    int fuse = 1;            // time steps per launch (wide sweep)
    bool no_scalar_rows = std::getenv("TEUK_NO_SCALAR_ROWS") != nullptr;   // diagnostics: force LDS rows
    int dd_cmode = dd_cmode_default();         // dd wide sweep: coefficient source (see dd_cmode_default)
    size_t lds = 0;          // dynamic LDS bytes per block of the step kernel
    lwk::InstDev *d_inst = nullptr;
    lwk::WorkItem *d_items = nullptr;
    int nitems = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    int sticky = TEUK_OK;
    int graph_steps = 0;
    // captured step loops, one per state buffer the replay starts from
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    long graph_replays = 0;
    // host round trip of the state after every step (measurement mode)
    double *host_state = nullptr;
    // observer time series of instance 0 (see teuk_set_observer)
    int obs_n = 0, obs_every = 0;
    long obs_cap = 0;
    int *obs_idx = nullptr;          // device: plane index i * n_theta + j per point
    double *obs_ring = nullptr;      // device: obs_cap records of 1 + 2 W obs_n doubles
    long long *obs_ctr = nullptr;    // device: steps since set_initial, records written, next step due
    // slab sweep (lw_slab_kernel): columns per lane, segments, exchange buffers,
    // flags and error word, and the tag of the last step launched
    int slab_r = 0, slab_nseg = 0;
    double *slab_x = nullptr;
    unsigned long long *slab_flags = nullptr;
    int *slab_err = nullptr;
    long long slab_base = 0;
    bool slab_fault = false;         // TEUK_FAULT=slab-abort: every wait of every launch gives up
    bool slab_coop = std::getenv("TEUK_SLAB_COOPERATIVE") != nullptr;   // cooperative launches
};

void free_slab(Batch &b) {
    hipFree(b.slab_x);
    hipFree(b.slab_flags);
    hipFree(b.slab_err);
    b.slab_x = nullptr;
    b.slab_flags = nullptr;
    b.slab_err = nullptr;
    b.slab_r = b.slab_nseg = 0;
    b.slab_base = 0;
}

void drop_graph(Batch &b) {
    for (int p = 0; p < 2; ++p) {
        if (b.gexec[p]) hipGraphExecDestroy(b.gexec[p]);
        if (b.graph[p]) hipGraphDestroy(b.graph[p]);
        b.gexec[p] = nullptr;
        b.graph[p] = nullptr;
    }
}

void free_observer(Batch &b) {
    hipFree(b.obs_idx);
    hipFree(b.obs_ring);
    hipFree(b.obs_ctr);
    b.obs_idx = nullptr;
    b.obs_ring = nullptr;
    b.obs_ctr = nullptr;
    b.obs_n = b.obs_every = 0;
    b.obs_cap = 0;
}

void free_batch(Batch &b) {
    if (b.stream) hipStreamSynchronize(b.stream);
    drop_graph(b);
    for (auto &I : b.inst) {
        hipFree(I.u[0]);
        hipFree(I.u[1]);
        hipFree(I.ch);
        hipFree(I.cf);
        hipFree(I.wt);
        hipFree(I.rf);
        hipFree(I.rh);
        hipFree(I.trig);
        I.u[0] = I.u[1] = I.ch = I.cf = I.wt = I.rf = I.rh = I.trig = nullptr;
    }
    hipFree(b.d_inst);
    hipFree(b.d_items);
    b.d_inst = nullptr;
    b.d_items = nullptr;
    free_observer(b);
    free_slab(b);
    if (b.host_state) hipHostFree(b.host_state);
    b.host_state = nullptr;
    if (b.own_stream) hipStreamDestroy(b.own_stream);
    b.own_stream = nullptr;
}

hipError_t coef_pass(int words, lwk::CoefJob &job, hipStream_t st) {
    switch (words) {
        case 1: return lwk::coef_pass_f64(job, st);
        case 2: return lwk::coef_pass_dd(job, st);
        default: return lwk::coef_pass_qd(job, st);
    }
}

// columns per lane and iteration of a wide sweep
int wide_run(int sweep) { return sweep == TEUK_SWEEP_WIDE2 ? 2 : 1; }

hipError_t step_launch(const Batch &b, int parity, int ns) {
    bool onfly = true;
    for (auto &I : b.inst) onfly = onfly && I.onfly;
    if (b.words == 1 && !onfly) {
        for (auto &I : b.inst)
            if (I.onfly) return hipErrorInvalidValue;   // mixed modes are not produced by the API
    }
    if (b.sweep != TEUK_SWEEP_SEGMENT) {
        const int run = wide_run(b.sweep);
        // one instance: the launch arguments carry its geometry and state
        // pointers and the kernel derives its segment from the block index
        // (same order as the work list), so no load precedes the state loads
        lwk::WideArgs one{};
        const lwk::WideArgs *onep = nullptr;
        if (b.inst.size() == 1) {
            const Instance &I = b.inst[0];
            one = {I.u[parity], I.u[parity ^ 1], I.g.n_r, I.g.n_theta, b.segcols, 0};
            onep = &one;
        }
        switch (b.words) {
            case 1:
                return lwk::wide_f64(b.nt, run, b.cmode, b.tm, ns, b.lds, onep, b.d_inst, b.d_items, b.nitems, parity,
                                     b.stream, false);
            case 2:
                return lwk::wide_dd(b.nt, run, b.cmode, b.tm, ns, b.lds, onep, b.d_inst, b.d_items, b.nitems, parity,
                                    b.stream, false);
            default:
                return lwk::wide_qd(b.nt, run, 0, b.tm, ns, b.lds, onep, b.d_inst, b.d_items, b.nitems, parity,
                                    b.stream, false);
        }
    }
    if (ns != 1) return hipErrorInvalidValue;         // the segment sweep takes one step per launch
    switch (b.words) {
        case 1: return lwk::step_f64(b.nt, b.segcols, onfly, b.lds, b.d_inst, b.d_items, b.nitems, parity, b.stream);
        case 2: return lwk::step_dd(b.nt, b.segcols, false, b.lds, b.d_inst, b.d_items, b.nitems, parity, b.stream);
        default: return lwk::step_qd(b.nt, b.segcols, false, b.lds, b.d_inst, b.d_items, b.nitems, parity, b.stream);
    }
}

int default_sweep(int words) { (void)words; return TEUK_SWEEP_WIDE; }
int max_wide_block(int words) { return words == 1 ? 1024 : (words == 2 ? 512 : 256); }

size_t wide_lds(const Batch &b, int nt) {
    size_t need = 0;
    for (auto &I : b.inst) {
        size_t x = 0;
        const int run = wide_run(b.sweep);
        switch (b.words) {
            case 1: x = lwk::wide_xchg_bytes<double>(nt, I.g.n_theta, run); break;
            case 2: x = lwk::wide_xchg_bytes<lwk::dd>(nt, I.g.n_theta, run); break;
            default: x = lwk::wide_xchg_bytes<lwk::qd>(nt, I.g.n_theta, run); break;
        }
        if (b.cmode == 1) x += lwk::wide_rows_bytes(b.segcols + 2 * b.fuse);
        need = std::max(need, x);
    }
    return need;
}

int device_lds_limit() {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lim <= 0)
        lim = 64 * 1024;
    return lim;
}

// XCD-aware order of one instance's work items (positions first..first+n-1
// of the list, i.e. blocks first.. of the launch).  The GPU hands block b to
// XCD b mod kXcds; the blocks one XCD receives get consecutive segments, so a
// column two neighbouring segments both read is fetched through one L2.
constexpr int kXcds = 8;   // the kernels' lwk::xcd_segment computes the same order for one instance
void xcd_order(std::vector<lwk::WorkItem> &items, size_t first, size_t n) {
    const std::vector<lwk::WorkItem> src(items.begin() + first, items.begin() + first + n);
    size_t cnt[kXcds] = {}, base[kXcds] = {}, seen[kXcds] = {};
    for (size_t l = 0; l < n; ++l) cnt[(first + l) % kXcds]++;
    size_t acc = 0;
    for (int q = 0; q < kXcds; ++q) {
        const size_t x = (first + q) % kXcds;
        base[x] = acc;
        acc += cnt[x];
    }
    for (size_t l = 0; l < n; ++l) {
        const size_t x = (first + l) % kXcds;
        items[first + l] = src[base[x] + seen[x]++];
    }
}

// Columns the wide-sweep work item [c0, c1) of a grid of nr nodes holds with
// ns steps per launch: ns neighbours on each side (fewer at the domain
// boundaries) and, when it reaches the right boundary with ns > 1, ns padding
// columns past it (the step kernel computes the same count).
int wide_cols(int c0, int c1, int nr, int ns) {
    const int a = std::max(c0 - ns, 0), e = std::min(c1 - 1 + ns, nr - 1);
    return e - a + 1 + ((ns > 1 && e == nr - 1) ? ns : 0);
}

// Plan of the slab sweep into the copy b (see build_worklist): block, segment
// length, LDS, residency of every block, and zeroed exchange buffers, flags
// and error word (allocated here; build_worklist hands them to the handle or
// frees them).
int plan_slab(const Batch &h, Batch &b) {
    if (b.inst.size() != 1) return fail(TEUK_ENOTSUP, "the slab sweep advances a single instance");
    const Instance &I = b.inst[0];
    // (every precision: FP64, double-double, quad-double)
    if (b.words == 1 && (!I.onfly || I.injected))
        return fail(TEUK_ENOTSUP, "the FP64 slab sweep needs per-point coefficients (not stored or injected planes)");
    const int nth = I.g.n_theta, nr = I.g.n_r;
    if (nth != 64 && nth != 128 && nth != 256) return fail(TEUK_ENOTSUP, "the slab sweep is built for n_theta 64, 128 and 256");
    if (b.fuse != 1)
        return fail(TEUK_EINVAL, "the slab sweep runs a call's steps in one launch: steps per launch must be 1");
    // default block: 4 n_theta threads (four groups)
    const int nt = b.nt_req ? b.nt_req : 4 * nth;
    if (nt < 256 || nt < nth || nt % nth != 0)
        return fail(TEUK_EINVAL, "slab sweep: block must be 256, 512 or 1024 threads and a multiple of n_theta");
    const int G = nt / nth;
    int dev = 0, cus = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e != hipSuccess) return hip_fail(e, "slab sweep: device attributes");
    if (h.slab_coop && !coop) return fail(TEUK_ENOTSUP, "slab sweep: the device does not launch cooperatively");
    // the requested segment length; with the default block, one that does not
    // fit is replaced by the shortest that does (1, 2 or 4 columns per lane;
    // multiword 1 or 2)
    const int max_r = b.words == 1 ? 4 : 2;
    std::vector<int> segs{b.seg_req};
    if (!b.nt_req)
        for (int r = 1; r <= max_r; r *= 2) segs.push_back(G * r);
    int seg = 0, r = 0, nseg = 0;
    size_t lds = 0;
    std::string why;
    int why_rc = TEUK_OK;
    for (int cand : segs) {
        const int rc_ = cand / G;
        if (cand % G != 0 || (rc_ != 1 && rc_ != 2 && rc_ != 4) || rc_ > max_r) {
            if (why.empty()) {
                why = b.words == 1 ? "slab sweep: segcols must be 1, 2 or 4 times block / n_theta"
                                   : "multiword slab sweep: segcols must be 1 or 2 times block / n_theta";
                why_rc = TEUK_EINVAL;
            }
            continue;
        }
        const size_t l = lwk::slab_lds_bytes(nt, nth, rc_, b.words);
        if (l > (size_t)device_lds_limit()) {
            if (why.empty()) {
                why = "slab sweep: launch shape needs more LDS than the device has";
                why_rc = TEUK_EINVAL;
            }
            continue;
        }
        int per_cu = 0;
        e = b.words == 1   ? lwk::slab_f64(nt, nth, rc_, 1, l, nullptr, 0, nullptr, &per_cu)
            : b.words == 2 ? lwk::slab_dd(nt, nth, rc_, 1, l, nullptr, 0, nullptr, &per_cu)
                           : lwk::slab_qd(nt, nth, rc_, 1, l, nullptr, 0, nullptr, &per_cu);
        if (e != hipSuccess) return hip_fail(e, "slab sweep: occupancy");
        const int ns = (nr + cand - 1) / cand;
        if ((long)per_cu * cus < ns) {
            if (why.empty()) {
                why = "slab sweep: " + std::to_string(ns) + " segments of " + std::to_string(cand) +
                      " nodes, but the device holds " + std::to_string((long)per_cu * cus) +
                      " such blocks at once (use longer segments)";
                why_rc = TEUK_ENOTSUP;
            }
            continue;
        }
        seg = cand;
        r = rc_;
        nseg = ns;
        lds = l;
        break;
    }
    if (!seg) return fail(why_rc, why);
    const size_t nx = 2 * 2 * (size_t)nseg * 6 * b.words * nth, nf = (size_t)nseg * 2 * (nth / 64) * lwk::kSlabFlagPad;
    e = hipMalloc((void **)&b.slab_x, nx * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&b.slab_flags, nf * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void **)&b.slab_err, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(b.slab_x, 0, nx * sizeof(double), h.stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.slab_flags, 0, nf * sizeof(unsigned long long), h.stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.slab_err, 0, sizeof(int), h.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h.stream);
    if (e != hipSuccess) {
        free_slab(b);
        return hip_fail(e, "slab sweep: exchange buffers");
    }
    b.nt = nt;
    b.segcols = seg;
    b.lds = lds;
    b.cmode = b.words == 1 ? 2 : 0;
    b.tm = 0;
    b.slab_r = r;
    b.slab_nseg = nseg;
    return TEUK_OK;
}

// (Re)build the launch plan, the descriptors and the work list from the
// requests (sweep, segment length, block, steps per launch) and the
// instances; all instances must share `cur`.  Transactional: the plan is
// worked out on a copy `b` of the requests and new device arrays are filled
// before anything of the handle `h` changes, so on failure `h` keeps its
// previous plan and arrays and stays usable.
int build_worklist(Batch &h) {
    Batch b;
    b.words = h.words;
    b.inst = h.inst;
    b.seg_req = h.seg_req;
    b.segcols = h.seg_req;
    b.nt_req = h.nt_req;
    b.sweep_req = h.sweep_req;
    b.fuse = h.fuse;
    b.no_scalar_rows = h.no_scalar_rows;
    b.dd_cmode = h.dd_cmode;
    int maxnth = 0;
    for (auto &I : b.inst) maxnth = std::max(maxnth, I.g.n_theta);
    b.sweep = b.sweep_req >= 0 ? b.sweep_req : default_sweep(b.words);
    b.lds = 0;
    if (b.sweep == TEUK_SWEEP_SLAB) {
        if (int rc = plan_slab(h, b)) return rc;
    } else if (b.sweep != TEUK_SWEEP_SEGMENT) {
        // FP64 per-point coefficients: radial rows by scalar loads when every
        // wavefront lies in one theta column (n_theta a multiple of 64), else
        // staged in LDS
        bool onfly = b.words == 1, wave_cols = true;
        for (auto &I : b.inst) {
            onfly = onfly && I.onfly;
            wave_cols = wave_cols && I.g.n_theta % 64 == 0;
        }
        bool injected = false;
        for (auto &I : b.inst) injected = injected || I.injected;
        // (injected coefficients exist only as planes: no per-point rebuild)
        const int dd_mode = (b.dd_cmode == 4 && injected) ? 0 : b.dd_cmode;
        b.cmode = !onfly ? (b.words == 2 ? dd_mode : 0) : (wave_cols && !b.no_scalar_rows ? 2 : 1);
        // FP64 radial rows of a segment stay within kMaxRowsLds
        while (b.segcols > 1 && lwk::wide_rows_bytes(b.segcols + 2 * b.fuse) > kMaxRowsLds) b.segcols -= 1;
        const size_t lim = (size_t)device_lds_limit();
        if (b.nt_req) {
            if (b.nt_req > max_wide_block(b.words)) return fail(TEUK_EINVAL, "block too large for this precision");
            b.nt = b.nt_req;
            b.lds = wide_lds(b, b.nt);
            if (b.lds > lim) return fail(TEUK_EINVAL, "launch shape needs more LDS than the device has");
        } else {
            // about four theta columns per block, fewer if LDS runs short (the
            // default shape stays within the 64 KiB every launch gets)
            const size_t cap = std::min<size_t>(lim, 64 * 1024);
            int nt = 64;
            while (nt < 4 * maxnth && nt < max_wide_block(b.words)) nt *= 2;
            while (nt / 2 >= maxnth && wide_lds(b, nt) > cap) nt /= 2;
            b.nt = nt;
            b.lds = wide_lds(b, nt);
            if (b.lds > 64 * 1024 && b.sweep_req < 0) {
                // default sweep only: wide slots for this n_theta and precision
                // would need more than 64 KiB of LDS; the segment sweep does not
                b.sweep = TEUK_SWEEP_SEGMENT;
                b.lds = 0;
            } else if (b.lds > lim) {
                return fail(TEUK_EINVAL, "n_theta too large for the device's LDS");
            }
        }
    }
    if (b.sweep == TEUK_SWEEP_SLAB) {
        // planned above
    } else if (b.sweep != TEUK_SWEEP_SEGMENT) {
        // iterations a work item needs: its columns over the columns a block takes per iteration
        // (fused steps read fuse columns on each side, plus fuse columns
        // past the right domain boundary)
        int ti = 0;
        for (auto &I : b.inst) {
            const int nr = I.g.n_r, per = (b.nt / I.g.n_theta) * wide_run(b.sweep);
            for (int c0 = 0; c0 < nr; c0 += b.segcols) {
                const int K = wide_cols(c0, std::min(c0 + b.segcols, nr), nr, b.fuse);
                ti = std::max(ti, (K + per - 1) / per);
            }
        }
        b.tm = ti <= 4 ? ti : 0;
        if (b.fuse > 1) {
            const int run = wide_run(b.sweep);
            const int max_tm = b.words == 1 ? (run == 1 ? 4 : 3) : 2;
            const bool ok = b.tm >= 1 && b.tm <= max_tm && b.nt >= 128 && b.nt <= 512 &&
                            ((b.words == 2 && run == 1) || (b.words == 1 && b.cmode > 0));
            if (!ok)
                return fail(TEUK_EINVAL, "fused steps need blocks of 128-512 threads and either dd with runs of "
                                         "one column and at most two iterations per step, or FP64 per-point "
                                         "coefficients with at most four iterations (runs of one column) or "
                                         "three (runs of two): segcols + 2 * fuse columns (+ fuse past the "
                                         "right boundary) within iterations * run * block / n_theta");
        }
        if (b.lds > 64 * 1024) {
            const int run = wide_run(b.sweep);
            // both the one-instance and the work-list form
            const lwk::WideArgs one{};
            hipError_t e = hipSuccess;
            for (const lwk::WideArgs *o : {&one, (const lwk::WideArgs *)nullptr}) {
                if (e != hipSuccess) break;
                for (int ns : {1, b.fuse}) {
                    if (e != hipSuccess) break;
                    e = b.words == 1
                            ? lwk::wide_f64(b.nt, run, b.cmode, b.tm, ns, b.lds, o, nullptr, nullptr, 0, 0, nullptr, true)
                        : b.words == 2 ? lwk::wide_dd(b.nt, run, b.cmode, b.tm, ns, b.lds, o, nullptr, nullptr, 0, 0, nullptr, true)
                                       : lwk::wide_qd(b.nt, run, 0, b.tm, ns, b.lds, o, nullptr, nullptr, 0, 0, nullptr, true);
                }
            }
            if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(dynamic LDS)");
        }
    } else {
        if (b.fuse > 1) return fail(TEUK_EINVAL, "the segment sweep takes one step per launch");
        b.nt = maxnth <= 64 ? 64 : (maxnth <= 128 ? 128 : 256);
        if (b.nt_req > b.nt) b.nt = b.nt_req;
        if (b.nt > 256) return fail(TEUK_EINVAL, "the segment sweep takes blocks of at most 256 threads");
        // FP64 per-point mode stages the radial rows of a block in LDS: keep that
        // within kMaxRowsLds by shortening the segments if needed
        for (;;) {
            size_t need = 0;
            for (auto &I : b.inst)
                if (I.onfly) need = std::max(need, lwk::rows_lds_bytes(b.nt, I.g.n_theta, b.segcols));
            if (need <= kMaxRowsLds || b.segcols == 1) {
                b.lds = need;
                break;
            }
            b.segcols -= 1;
        }
    }
    std::vector<lwk::InstDev> hd(b.inst.size());
    std::vector<lwk::WorkItem> items;
    // largest instances first
    std::vector<int> order(b.inst.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return b.inst[x].plane() > b.inst[y].plane();
    });
    for (size_t k = 0; k < b.inst.size(); ++k) {
        const Instance &I = b.inst[k];
        lwk::InstDev &D = hd[k];
        D.nr = I.g.n_r;
        D.nth = I.g.n_theta;
        D.reach = I.reach;
        D.segcols = b.segcols;
        const int G = b.sweep != TEUK_SWEEP_SEGMENT ? 1 : b.nt / D.nth;   // wide: one segment per block
        const int nseg = (D.nr + b.segcols - 1) / b.segcols;
        D.groups = (nseg + G - 1) / G;
        D.words = I.words;
        D.u[0] = I.u[0];
        D.u[1] = I.u[1];
        D.ch = I.ch;
        D.cf = I.cf;
        D.wt = I.wt;
        D.onfly = I.onfly;
        D.rf = I.rf;
        D.rh = I.rh;
        D.trig = I.trig;
        std::memcpy(D.hdt, I.hdt, sizeof D.hdt);
        std::memcpy(D.dt, I.dt, sizeof D.dt);
    }
    for (int k : order) {
        const size_t first = items.size();
        for (int gi = 0; gi < hd[k].groups; ++gi) items.push_back({k, gi});
        xcd_order(items, first, items.size() - first);
    }
    lwk::InstDev *d_inst = nullptr;
    lwk::WorkItem *d_items = nullptr;
    hipError_t e = hipMalloc((void **)&d_inst, hd.size() * sizeof(lwk::InstDev));
    if (e == hipSuccess) e = hipMalloc((void **)&d_items, std::max<size_t>(1, items.size()) * sizeof(lwk::WorkItem));
    if (e == hipSuccess) e = hipMemcpy(d_inst, hd.data(), hd.size() * sizeof(lwk::InstDev), hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(d_items, items.data(), items.size() * sizeof(lwk::WorkItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(d_inst);
        hipFree(d_items);
        free_slab(b);
        return hip_fail(e, "descriptors and work list");
    }
    // commit (the previous arrays are no longer referenced by queued work:
    // every caller has waited for the handle's stream, or nothing was queued)
    hipFree(h.d_inst);
    hipFree(h.d_items);
    h.d_inst = d_inst;
    h.d_items = d_items;
    h.nitems = (int)items.size();
    h.sweep = b.sweep;
    h.segcols = b.segcols;
    h.nt = b.nt;
    h.cmode = b.cmode;
    h.tm = b.tm;
    h.lds = b.lds;
    free_slab(h);
    h.slab_r = b.slab_r;
    h.slab_nseg = b.slab_nseg;
    h.slab_x = b.slab_x;
    h.slab_flags = b.slab_flags;
    h.slab_err = b.slab_err;
    h.slab_base = 0;
    drop_graph(h);
    return TEUK_OK;
}

int create_batch(Batch &b, int n, const int *s, const int *m, const double *a, const teuk_grid *g,
                 int prec) {
    if (n < 1) return fail(TEUK_EINVAL, "batch size must be >= 1");
    for (int k = 0; k < n; ++k) {
        int rc = validate(s[k], m[k], a[k], &g[k], prec);
        if (rc != TEUK_OK) return rc;
    }
    if (const char *f = std::getenv("TEUK_FAULT")) {
        if (std::strcmp(f, "alloc") == 0) return fail(TEUK_ENOMEM, "allocation failure injected by TEUK_FAULT=alloc");
        b.slab_fault = std::strcmp(f, "slab-abort") == 0;
    }
    b.words = prec;
    hipError_t e = hipStreamCreateWithFlags(&b.own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    b.stream = b.own_stream;
    b.inst.resize(n);
    const int W = prec;
    for (int k = 0; k < n; ++k) {
        Instance &I = b.inst[k];
        I.s = s[k];
        I.m = m[k];
        I.a_over_M = a[k];
        I.g = g[k];
        I.words = W;
        I.reach = g[k].angular_order / 2;
        const size_t st_bytes = 4 * (size_t)W * I.plane() * sizeof(double);
        const size_t cf_bytes = 8 * (size_t)W * I.plane() * sizeof(double);
        const size_t ch_bytes = 8 * (size_t)W * I.hplane() * sizeof(double);
        const size_t wt_bytes = (size_t)(2 * I.reach + 1) * W * g[k].n_theta * sizeof(double);
        I.onfly = (W == 1);
        const bool rows_mp = (W == 2);               // double-double: radial rows for the per-point mode
        if ((e = hipMalloc((void **)&I.u[0], st_bytes)) != hipSuccess ||
            (e = hipMalloc((void **)&I.u[1], st_bytes)) != hipSuccess ||
            (e = hipMalloc((void **)&I.wt, wt_bytes)) != hipSuccess)
            return hip_fail(e, "hipMalloc(instance arrays)");
        if (I.onfly) {
            if ((e = hipMalloc((void **)&I.rf, (size_t)lwk::kRadRow * g[k].n_r * sizeof(double))) != hipSuccess ||
                (e = hipMalloc((void **)&I.rh, (size_t)lwk::kRadRow * (g[k].n_r - 1) * sizeof(double))) != hipSuccess ||
                (e = hipMalloc((void **)&I.trig, 2 * (size_t)g[k].n_theta * sizeof(double))) != hipSuccess)
                return hip_fail(e, "hipMalloc(coefficient rows)");
        } else if ((e = hipMalloc((void **)&I.cf, cf_bytes)) != hipSuccess ||
                   (e = hipMalloc((void **)&I.ch, ch_bytes)) != hipSuccess) {
            return hip_fail(e, "hipMalloc(coefficient planes)");
        }
        if (rows_mp &&
            ((e = hipMalloc((void **)&I.rf, (size_t)lwk::kRadRow * W * g[k].n_r * sizeof(double))) != hipSuccess ||
             (e = hipMalloc((void **)&I.rh, (size_t)lwk::kRadRow * W * (g[k].n_r - 1) * sizeof(double))) != hipSuccess ||
             (e = hipMalloc((void **)&I.trig, 2 * (size_t)W * g[k].n_theta * sizeof(double))) != hipSuccess))
            return hip_fail(e, "hipMalloc(coefficient rows)");
        if ((e = hipMemsetAsync(I.u[0], 0, st_bytes, b.stream)) != hipSuccess ||
            (e = hipMemsetAsync(I.u[1], 0, st_bytes, b.stream)) != hipSuccess)
            return hip_fail(e, "hipMemset(state)");
        lwk::CoefJob J{};
        J.s = I.s;
        J.m = I.m;
        J.nr = g[k].n_r;
        J.nth = g[k].n_theta;
        J.reach = I.reach;
        J.a_over_M = a[k];
        J.mass = g[k].mass;
        J.rstar_min = g[k].rstar_min;
        J.rstar_max = g[k].rstar_max;
        J.cfl = g[k].cfl;
        J.ch = I.ch;
        J.cf = I.cf;
        J.wt = I.wt;
        J.onfly = I.onfly;
        J.rows_mp = rows_mp;
        J.rf = I.rf;
        J.rh = I.rh;
        J.trig = I.trig;
        if ((e = coef_pass(W, J, b.stream)) != hipSuccess) return hip_fail(e, "coefficient pass");
        std::memcpy(I.hdt, J.hdt, sizeof I.hdt);
        std::memcpy(I.dt, J.dt, sizeof I.dt);
        I.dt_lead = J.dt_lead;
    }
    if ((e = hipStreamSynchronize(b.stream)) != hipSuccess) return hip_fail(e, "coefficient pass (sync)");
    return build_worklist(b);
}

int slab_check(Batch &b);

int check_ok(Batch &b) {
    if (b.sticky != TEUK_OK) return fail(b.sticky, "handle is in a failed state after an earlier device error");
    return TEUK_OK;
}

// Wait for the handle's queued work (before its launch shape or stream
// changes); a device error found here puts the handle in the failed state.
int quiesce(Batch &b) {
    if (int rc = check_ok(b)) return rc;
    if (!b.stream) return TEUK_OK;
    const hipError_t e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "stream synchronize");
    }
    return slab_check(b);
}

// host interchange [j][i][w]  <->  device planar [w][i][j]
int upload_field(Batch &b, Instance &I, int comp, const double *src, int buf) {
    const int W = I.words, nr = I.g.n_r, nth = I.g.n_theta;
    std::vector<double> tmp((size_t)W * I.plane());
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nr; ++i) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            if (i != 0 && i != nr - 1)
                for (int w = 0; w < W; ++w) v[w] = src[((size_t)j * nr + i) * W + w];
            // renormalise to a non-overlapping expansion (the kernels assume one)
            if (W == 2) {
                lwk::two_sum(v[0], v[1], v[0], v[1]);
            } else if (W == 4) {
                const lwk::qd q = lwk::qd_renorm(v[0], v[1], v[2], v[3], 0.0);
                v[0] = q.x0; v[1] = q.x1; v[2] = q.x2; v[3] = q.x3;
            }
            for (int w = 0; w < W; ++w) tmp[(size_t)w * I.plane() + (size_t)i * nth + j] = v[w];
        }
    hipError_t e = hipMemcpyAsync(I.u[buf] + (size_t)comp * W * I.plane(), tmp.data(),
                                  tmp.size() * sizeof(double), hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) return hip_fail(e, "upload");
    return TEUK_OK;
}

int download_planes(Batch &b, const double *dsrc, int nplanes_w, int nr, int nth, int W, double *out) {
    // dsrc holds W planes of nr x nth (theta fastest); out is [nth][nr][W]
    std::vector<double> tmp((size_t)W * nr * nth);
    hipError_t e = hipStreamSynchronize(b.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(tmp.data(), dsrc, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "download");
    }
    if (int rc = slab_check(b)) return rc;
    (void)nplanes_w;
    const size_t plane = (size_t)nr * nth;
    for (int j = 0; j < nth; ++j)
        for (int i = 0; i < nr; ++i)
            for (int w = 0; w < W; ++w)
                out[((size_t)j * nr + i) * W + w] = tmp[(size_t)w * plane + (size_t)i * nth + j];
    return TEUK_OK;
}

// Observer counters (see observer_record_kernel) for a run now at `step`:
// the next record is due at the next multiple of `every`; `clear` also drops
// the records held.
int reset_observer(Batch &b, long step, bool clear) {
    if (b.obs_n <= 0) return TEUK_OK;
    long long c[3];
    hipError_t e = hipStreamSynchronize(b.stream);
    if (e == hipSuccess) e = hipMemcpy(c, b.obs_ctr, sizeof c, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        c[0] = step;
        if (clear) c[1] = 0;
        c[2] = (step / b.obs_every + 1) * (long long)b.obs_every;
        e = hipMemcpy(b.obs_ctr, c, sizeof c, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "observer counters");
    }
    return TEUK_OK;
}

int set_initial(Batch &b, int k, const double *pr, const double *pim, const double *qr, const double *qim) {
    if (int rc = check_ok(b)) return rc;
    if (k < 0 || k >= (int)b.inst.size()) return fail(TEUK_EINVAL, "instance index out of range");
    if (!pr || !pim || !qr || !qim) return fail(TEUK_EINVAL, "field pointer is NULL");
    Instance &I = b.inst[k];
    // all instances of a batch step together: keep them on the same buffer
    int buf = I.cur;
    const double *src[4] = {pr, pim, qr, qim};
    // refuse non-finite values before anything is uploaded (radial boundary
    // nodes are overwritten with zero and not checked)
    const size_t nv = (size_t)I.words * I.plane();
    for (int c = 0; c < 4; ++c)
        for (size_t q = 0; q < nv; ++q) {
            const size_t i = (q / I.words) % (size_t)I.g.n_r;
            if (i != 0 && i != (size_t)I.g.n_r - 1 && !std::isfinite(src[c][q]))
                return fail(TEUK_ENONFINITE, "initial field " + std::to_string(c) + " holds Inf or NaN");
        }
    for (int c = 0; c < 4; ++c)
        if (int rc = upload_field(b, I, c, src[c], buf)) return rc;
    I.steps = 0;
    if (k == 0) return reset_observer(b, 0, true);
    return TEUK_OK;
}

// Observer record after a launch that advanced `ns` steps and left its
// fields in u (one block; see teuk_set_observer).  ctr[0] = steps since
// set_initial, ctr[1] = records written, ctr[2] = step at which the next
// record is due.  Every thread reads the counters before the barrier and
// thread 0 writes them after it; launches on one stream run in order, so
// the next launch sees the new values (also inside a captured graph).
__global__ void observer_record_kernel(const double *__restrict__ u, unsigned long long plane, int W, int npts,
                                       const int *__restrict__ idx, int every, long long cap, double *ring,
                                       long long *ctr, int ns) {
    const long long step = ctr[0] + ns, nrec = ctr[1], due = ctr[2];
    const bool rec = step >= due;
    if (rec) {
        const int len = 2 * W * npts;
        double *r = ring + (size_t)(nrec % cap) * (size_t)(1 + len);
        if (threadIdx.x == 0) r[0] = (double)step;
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            const int p = q / (2 * W), c = (q / W) % 2, w = q % W;
            r[1 + q] = u[((size_t)c * W + w) * plane + (size_t)idx[p]];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ctr[0] = step;
        if (rec) {
            ctr[1] = nrec + 1;
            ctr[2] = (step / every + 1) * every;
        }
    }
}

// Polls of one slab wait before it gives up: 2^21 polls (each a load that
// may miss to memory, then s_sleep 2) take of the order of a second, against
// microseconds for a step.
constexpr long long kSlabSpin = 1ll << 21;
// Steps of one slab launch at most (a longer call takes several launches).
constexpr long kSlabMaxSteps = 4096;

// One slab launch of `ns` steps from buffer `parity` into the other buffer.
hipError_t slab_launch(Batch &b, int parity, int ns) {
    const Instance &I = b.inst[0];
    lwk::SlabArgs a{};
    a.uin = I.u[parity];
    a.uout = I.u[parity ^ 1];
    a.rf = I.rf;
    a.rh = I.rh;
    a.trig = I.trig;
    a.wt = I.wt;
    a.ch = I.ch;
    a.cf = I.cf;
    a.xbuf = b.slab_x;
    a.flags = b.slab_flags;
    a.err = b.slab_err;
    a.base = b.slab_base;
    a.spin = kSlabSpin;
    a.nr = I.g.n_r;
    a.nth = I.g.n_theta;
    a.nseg = b.slab_nseg;
    a.reach = I.reach;
    a.nsteps = ns;
    std::memcpy(a.hdt, I.hdt, sizeof a.hdt);
    std::memcpy(a.dt, I.dt, sizeof a.dt);
    hipError_t e = hipSuccess;
    if (b.slab_fault) e = hipMemsetD32Async((hipDeviceptr_t)b.slab_err, 1, 1, b.stream);
    const int mode = b.slab_coop ? 2 : 0;
    if (e == hipSuccess)
        e = b.words == 1   ? lwk::slab_f64(b.nt, I.g.n_theta, b.slab_r, mode, b.lds, &a, b.slab_nseg, b.stream, nullptr)
            : b.words == 2 ? lwk::slab_dd(b.nt, I.g.n_theta, b.slab_r, mode, b.lds, &a, b.slab_nseg, b.stream, nullptr)
                           : lwk::slab_qd(b.nt, I.g.n_theta, b.slab_r, mode, b.lds, &a, b.slab_nseg, b.stream, nullptr);
    b.slab_base += ns;
    return e;
}

// After the handle's stream has drained: a slab launch whose wait gave up
// puts the handle in the failed state.
int slab_check(Batch &b) {
    if (!b.slab_err) return TEUK_OK;
    int v = 0;
    const hipError_t e = hipMemcpy(&v, b.slab_err, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "slab error word");
    }
    if (v) {
        b.sticky = TEUK_EDEVICE;
        return fail(TEUK_EDEVICE, "slab sweep: a wait for a neighbouring block gave up; the kernel ended early and "
                                  "the fields are not valid");
    }
    return TEUK_OK;
}

// one step-kernel launch of `ns` steps from buffer `parity`, then the
// observer record if one is set
hipError_t launch_step(Batch &b, int parity, int ns) {
    hipError_t e = b.sweep == TEUK_SWEEP_SLAB ? slab_launch(b, parity, ns) : step_launch(b, parity, ns);
    if (e == hipSuccess && b.obs_n > 0) {
        const Instance &I = b.inst[0];
        observer_record_kernel<<<1, 256, 0, b.stream>>>(I.u[parity ^ 1], (unsigned long long)I.plane(), b.words,
                                                        b.obs_n, b.obs_idx, b.obs_every, (long long)b.obs_cap,
                                                        b.obs_ring, b.obs_ctr, ns);
        e = hipGetLastError();
    }
    return e;
}

// launches of a captured step loop: about graph_steps / fuse, at least one
// (the slab sweep runs a call's steps in one launch and takes no graph)
int graph_launches(const Batch &b) {
    return b.graph_steps > 0 && b.sweep != TEUK_SWEEP_SLAB ? std::max(1, b.graph_steps / b.fuse) : 0;
}

// capture the step loop that starts from state buffer `par`
hipError_t capture_graph(Batch &b, int par) {
    const int nl = graph_launches(b);
    hipError_t e = hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int q = 0; q < nl && e == hipSuccess; ++q) e = launch_step(b, (par + q) & 1, b.fuse);
    const hipError_t e2 = hipStreamEndCapture(b.stream, &b.graph[par]);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b.gexec[par], b.graph[par], nullptr, nullptr, 0);
    return e;
}

// Host round trip (measurement mode): the state of every instance goes to
// host memory and back after each step, as a design that keeps the fields on
// the host and offloads the step would move them.
hipError_t round_trip(const Batch &b, int buf) {
    hipError_t e = hipSuccess;
    for (const Instance &I : b.inst) {
        const size_t bytes = 4 * (size_t)I.words * I.plane() * sizeof(double);
        if (e == hipSuccess) e = hipMemcpyAsync(b.host_state, I.u[buf], bytes, hipMemcpyDeviceToHost, b.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(I.u[buf], b.host_state, bytes, hipMemcpyHostToDevice, b.stream);
    }
    return e;
}

int do_steps(Batch &b, long n) {
    if (int rc = check_ok(b)) return rc;
    if (n < 0) return fail(TEUK_EINVAL, "step count must be >= 0");
    int cur = b.inst[0].cur;
    long left = n;
    hipError_t e = hipSuccess;
    // a launch advances `fuse` steps (the remainder goes one step per launch);
    // a captured graph holds graph_launches(b) launches, and one graph is kept
    // per state buffer a replay can start from
    const int F = b.fuse;
    if (b.sweep == TEUK_SWEEP_SLAB && !b.host_state) {
        // launches of up to kSlabMaxSteps steps, cut where an observer record
        // falls due
        while (left > 0 && e == hipSuccess) {
            long k = std::min(left, kSlabMaxSteps);
            if (b.obs_n > 0) {
                const long st = b.inst[0].steps + (n - left);
                k = std::min(k, (st / b.obs_every + 1) * (long)b.obs_every - st);
            }
            e = launch_step(b, cur, (int)k);
            cur ^= 1;
            left -= k;
        }
    } else if (b.host_state) {
        for (; left > 0 && e == hipSuccess; --left) {
            e = launch_step(b, cur, 1);
            cur ^= 1;
            if (e == hipSuccess) e = round_trip(b, cur);
        }
    } else {
        const int gl = graph_launches(b);
        const long gsteps = (long)gl * F;
        while (gl > 0 && left >= gsteps && e == hipSuccess) {
            if (!b.gexec[cur]) {
                e = capture_graph(b, cur);
                if (e != hipSuccess) {
                    b.sticky = TEUK_EDEVICE;
                    drop_graph(b);
                    return hip_fail(e, "graph capture");
                }
            }
            e = hipGraphLaunch(b.gexec[cur], b.stream);
            ++b.graph_replays;
            left -= gsteps;
            cur = (cur + gl) & 1;
        }
        for (; left >= F && e == hipSuccess; left -= F) {
            e = launch_step(b, cur, F);
            cur ^= 1;
        }
        for (; left > 0 && e == hipSuccess; --left) {
            e = launch_step(b, cur, 1);
            cur ^= 1;
        }
    }
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "step launch");
    }
    for (auto &I : b.inst) {
        I.cur = cur;
        I.steps += n;
    }
    return TEUK_OK;
}

// capture the step loops of both starting buffers now (no steps run)
int prepare_graph(Batch &b) {
    if (int rc = check_ok(b)) return rc;
    if (graph_launches(b) <= 0 || b.host_state) return TEUK_OK;
    for (int par = 0; par < 2; ++par) {
        hipError_t e = b.gexec[par] ? hipSuccess : capture_graph(b, par);
        // move the executable graph to the device now, so that its first
        // replay does not pay for it
        if (e == hipSuccess) e = hipGraphUpload(b.gexec[par], b.stream);
        if (e != hipSuccess) {
            b.sticky = TEUK_EDEVICE;
            drop_graph(b);
            return hip_fail(e, "graph capture");
        }
    }
    const hipError_t e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "graph upload");
    }
    return TEUK_OK;
}

int read_field(Batch &b, int k, int f, double *out) {
    if (int rc = check_ok(b)) return rc;
    if (k < 0 || k >= (int)b.inst.size()) return fail(TEUK_EINVAL, "instance index out of range");
    if (f < 0 || f > 3 || !out) return fail(TEUK_EINVAL, "bad field or NULL output");
    Instance &I = b.inst[k];
    return download_planes(b, I.u[I.cur] + (size_t)f * I.words * I.plane(), 1, I.g.n_r, I.g.n_theta, I.words, out);
}

int set_stream(Batch &b, void *st) {
    if (int rc = quiesce(b)) return rc;
    b.stream = st ? (hipStream_t)st : b.own_stream;
    drop_graph(b);
    return TEUK_OK;
}

}  // namespace

struct teuk {
    Batch b;
};
struct teuk_batch {
    Batch b;
};

extern "C" {

int teuk_abi_version(void) { return TEUK_ABI_VERSION; }
const char *teuk_build_info(void) { return "libteuk gfx950 fp64/dd/qd lax-wendroff"; }
const char *teuk_last_error(void) { return g_err.c_str(); }

int teuk_validate(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec) {
    return validate(s, m, a_over_M, grid, (int)prec);
}

int teuk_create(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec, teuk_t **out) {
    if (!out) return fail(TEUK_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(s, m, a_over_M, grid, (int)prec);
    if (rc != TEUK_OK) return rc;
    teuk_t *h = new (std::nothrow) teuk_t;
    if (!h) return fail(TEUK_ENOMEM, "host allocation");
    rc = create_batch(h->b, 1, &s, &m, &a_over_M, grid, (int)prec);
    if (rc != TEUK_OK) {
        free_batch(h->b);
        delete h;
        return rc;
    }
    *out = h;
    return TEUK_OK;
}

int teuk_destroy(teuk_t *h) {
    if (!h) return TEUK_OK;
    free_batch(h->b);
    delete h;
    return TEUK_OK;
}

int teuk_set_initial(teuk_t *h, const double *a, const double *b, const double *c, const double *d) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_initial(h->b, 0, a, b, c, d);
}
int teuk_step(teuk_t *h, long n) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return do_steps(h->b, n);
}
int teuk_read_field(teuk_t *h, teuk_field f, double *out) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return read_field(h->b, 0, (int)f, out);
}
double teuk_dt(const teuk_t *h) { return h ? h->b.inst[0].dt_lead : 0.0; }
long teuk_steps_done(const teuk_t *h) { return h ? h->b.inst[0].steps : -1; }
int teuk_words(const teuk_t *h) { return h ? h->b.words : 0; }
int teuk_set_step_index(teuk_t *h, long n) {
    if (!h || n < 0) return fail(TEUK_EINVAL, "bad handle or step index");
    if (int rc = check_ok(h->b)) return rc;
    h->b.inst[0].steps = n;
    return reset_observer(h->b, n, false);
}
int teuk_set_stream(teuk_t *h, void *st) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_stream(h->b, st);
}
int teuk_use_graph(teuk_t *h, int k) {
    if (!h || k < 0) return fail(TEUK_EINVAL, "bad handle or graph length");
    drop_graph(h->b);
    h->b.graph_steps = k;
    return TEUK_OK;
}
static int set_launch(Batch &b, int segcols, int block);
int teuk_set_tile(teuk_t *h, int segcols) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_launch(h->b, segcols, h->b.nt_req);
}

static int set_launch(Batch &b, int segcols, int block) {
    if (segcols < 1 || (block != 0 && block != 64 && block != 128 && block != 256 && block != 512 && block != 1024))
        return fail(TEUK_EINVAL, "segcols must be >= 1 and block one of 0, 64, 128, 256, 512, 1024");
    int maxnth = 0;
    for (auto &I : b.inst) maxnth = std::max(maxnth, I.g.n_theta);
    if (block != 0 && block < maxnth) return fail(TEUK_EINVAL, "block must be >= n_theta");
    if (int rc = quiesce(b)) return rc;
    const int old_seg = b.seg_req, old_nt = b.nt_req;
    b.seg_req = segcols;
    b.nt_req = block;
    const int rc = build_worklist(b);
    if (rc != TEUK_OK) {
        // the handle keeps its previous plan (build_worklist changes nothing
        // on failure); restore the requests that plan was built from
        b.seg_req = old_seg;
        b.nt_req = old_nt;
    }
    return rc;
}

static int set_sweep(Batch &b, int sweep) {
    if (sweep != -1 && sweep != TEUK_SWEEP_SEGMENT && sweep != TEUK_SWEEP_WIDE && sweep != TEUK_SWEEP_WIDE2 &&
        sweep != TEUK_SWEEP_SLAB)
        return fail(TEUK_EINVAL, "sweep must be -1 (default), 0 (segment), 1 (wide), 2 (wide, runs of two) or 3 (slab)");
    if (sweep == TEUK_SWEEP_WIDE2 && b.words != 1)
        return fail(TEUK_ENOTSUP, "the wide sweep with runs of two columns is built for FP64 only");
    if (int rc = quiesce(b)) return rc;
    const int old = b.sweep_req, old_nt = b.nt_req;
    b.sweep_req = sweep;
    b.nt_req = 0;
    const int rc = build_worklist(b);
    if (rc != TEUK_OK) {
        b.sweep_req = old;
        b.nt_req = old_nt;
    }
    return rc;
}

int teuk_set_sweep(teuk_t *h, int sweep) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_sweep(h->b, sweep);
}
int teuk_batch_set_sweep(teuk_batch_t *b, int sweep) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_sweep(b->b, sweep);
}
int teuk_get_sweep(const teuk_t *h) { return h ? h->b.sweep : TEUK_EINVAL; }

static int set_fuse(Batch &b, int ns) {
    if (ns != 1 && ns != 2 && ns != 4) return fail(TEUK_EINVAL, "steps per launch must be 1, 2 or 4");
    if (int rc = quiesce(b)) return rc;
    const int old = b.fuse;
    b.fuse = ns;
    const int rc = build_worklist(b);
    if (rc != TEUK_OK) b.fuse = old;
    return rc;
}
int teuk_set_fuse(teuk_t *h, int steps_per_launch) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_fuse(h->b, steps_per_launch);
}
int teuk_batch_set_fuse(teuk_batch_t *b, int steps_per_launch) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_fuse(b->b, steps_per_launch);
}

int teuk_set_launch(teuk_t *h, int segcols, int block) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_launch(h->b, segcols, block);
}
int teuk_batch_set_launch(teuk_batch_t *b, int segcols, int block) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_launch(b->b, segcols, block);
}

int teuk_check_finite(teuk_t *h, int *ok) {
    if (!h || !ok) return fail(TEUK_EINVAL, "NULL argument");
    Instance &I = h->b.inst[0];
    std::vector<double> tmp((size_t)I.words * I.plane());
    *ok = 1;
    for (int f = 0; f < 4; ++f) {
        int rc = read_field(h->b, 0, f, tmp.data());
        if (rc) return rc;
        for (double v : tmp)
            if (!std::isfinite(v)) *ok = 0;
    }
    return *ok ? TEUK_OK : fail(TEUK_ENONFINITE, "a field holds Inf or NaN");
}

int teuk_get_coefficients(teuk_t *h, int which, double *out) {
    if (!h || !out || which < 0 || which > 2) return fail(TEUK_EINVAL, "bad arguments");
    Batch &b = h->b;
    Instance &I = b.inst[0];
    const int W = I.words, nth = I.g.n_theta;
    if (which == 2) {
        const int taps = 2 * I.reach + 1;
        for (int k = 0; k < taps; ++k) {
            // one "row" of nth entries per tap: reuse the plane download with nr = 1
            int rc = download_planes(b, I.wt + (size_t)k * W * nth, 1, 1, nth, W, out + (size_t)k * nth * W);
            if (rc) return rc;
        }
        return TEUK_OK;
    }
    const int nr = which == 0 ? I.g.n_r - 1 : I.g.n_r;
    const double *src = which == 0 ? I.ch : I.cf;
    double *tmp = nullptr;
    if (I.onfly) {
        // FP64 kernels rebuild the coefficients per point: materialise them with the same routine
        const size_t np = 8 * ((size_t)I.g.n_r + (I.g.n_r - 1)) * nth;
        hipError_t e = hipMalloc((void **)&tmp, np * sizeof(double));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(coefficient planes)");
        double *cf = tmp, *ch = tmp + 8 * (size_t)I.g.n_r * nth;
        e = lwk::fp64_planes(I.g.n_r, nth, I.rf, I.rh, I.trig, cf, ch, b.stream);
        if (e != hipSuccess) {
            hipFree(tmp);
            return hip_fail(e, "coefficient planes");
        }
        src = which == 0 ? ch : cf;
    }
    const size_t plane = (size_t)nr * nth;
    int rc = TEUK_OK;
    for (int c = 0; c < 8 && rc == TEUK_OK; ++c)
        rc = download_planes(b, src + (size_t)c * W * plane, 1, nr, nth, W, out + (size_t)c * plane * W);
    if (tmp) {
        const hipError_t e = hipStreamSynchronize(b.stream);
        const hipError_t e2 = hipFree(tmp);
        if (rc == TEUK_OK && e != hipSuccess) rc = hip_fail(e, "stream synchronize");
        if (rc == TEUK_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipFree");
    }
    return rc;
}

int teuk_set_coefficients(teuk_t *h, int which, const double *in) {
    if (!h || !in || which < 0 || which > 1) return fail(TEUK_EINVAL, "bad arguments");
    Batch &b = h->b;
    if (int rc = quiesce(b)) return rc;
    Instance &I = b.inst[0];
    const int W = I.words, nth = I.g.n_theta;
    if (I.onfly) {
        // switch this instance to stored planes, seeded from its own per-point
        // coefficients.  Stored planes have no fused form: a handle set to
        // several steps per launch falls back to one.  Nothing of the handle
        // changes unless the new plan is in place.
        double *cf = nullptr, *ch = nullptr;
        hipError_t e = hipMalloc((void **)&cf, 8 * (size_t)I.g.n_r * nth * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&ch, 8 * (size_t)(I.g.n_r - 1) * nth * sizeof(double));
        if (e == hipSuccess) e = lwk::fp64_planes(I.g.n_r, nth, I.rf, I.rh, I.trig, cf, ch, b.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
        if (e != hipSuccess) {
            hipFree(cf);
            hipFree(ch);
            return hip_fail(e, "coefficient planes");
        }
        I.cf = cf;
        I.ch = ch;
        I.onfly = 0;
        const int old_fuse = b.fuse, old_sweep = b.sweep_req, old_nt = b.nt_req;
        int rc = build_worklist(b);
        if (rc != TEUK_OK && b.sweep_req == TEUK_SWEEP_SLAB) {
            // the slab sweep needs per-point coefficients: back to the default
            b.sweep_req = -1;
            b.nt_req = 0;
            rc = build_worklist(b);
        }
        if (rc != TEUK_OK && b.fuse > 1) {
            b.fuse = 1;
            rc = build_worklist(b);
        }
        if (rc != TEUK_OK) {
            b.fuse = old_fuse;
            b.sweep_req = old_sweep;
            b.nt_req = old_nt;
            I.onfly = 1;
            I.cf = I.ch = nullptr;
            hipFree(cf);
            hipFree(ch);
            return rc;
        }
    }
    if (!I.injected) {
        // the step must read the planes from now on (the per-point modes
        // would ignore them)
        I.injected = 1;
        if (int rc = build_worklist(b)) {
            I.injected = 0;
            return rc;
        }
    }
    const int nr = which == 0 ? I.g.n_r - 1 : I.g.n_r;
    double *dst = which == 0 ? I.ch : I.cf;
    const size_t plane = (size_t)nr * nth;
    std::vector<double> tmp((size_t)W * plane);
    for (int c = 0; c < 8; ++c) {
        for (int j = 0; j < nth; ++j)
            for (int i = 0; i < nr; ++i)
                for (int w = 0; w < W; ++w)
                    tmp[(size_t)w * plane + (size_t)i * nth + j] = in[(size_t)c * plane * W + ((size_t)j * nr + i) * W + w];
        hipError_t e = hipMemcpyAsync(dst + (size_t)c * W * plane, tmp.data(), tmp.size() * sizeof(double),
                                      hipMemcpyHostToDevice, b.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
        if (e != hipSuccess) {
            b.sticky = TEUK_EDEVICE;     // the planes are partly overwritten
            return hip_fail(e, "set coefficients");
        }
    }
    return TEUK_OK;
}

// ---------------------------------------------------------------- batched
int teuk_batch_create(int n, const int *s, const int *m, const double *a, const teuk_grid *grids,
                      teuk_precision prec, teuk_batch_t **out) {
    if (!out || !s || !m || !a || !grids) return fail(TEUK_EINVAL, "NULL argument");
    *out = nullptr;
    teuk_batch_t *b = new (std::nothrow) teuk_batch_t;
    if (!b) return fail(TEUK_ENOMEM, "host allocation");
    int rc = create_batch(b->b, n, s, m, a, grids, (int)prec);
    if (rc != TEUK_OK) {
        free_batch(b->b);
        delete b;
        return rc;
    }
    *out = b;
    return TEUK_OK;
}
int teuk_batch_destroy(teuk_batch_t *b) {
    if (!b) return TEUK_OK;
    free_batch(b->b);
    delete b;
    return TEUK_OK;
}
int teuk_batch_set_initial(teuk_batch_t *b, int k, const double *p, const double *q, const double *r,
                           const double *t) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_initial(b->b, k, p, q, r, t);
}
int teuk_batch_step(teuk_batch_t *b, long n) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return do_steps(b->b, n);
}
int teuk_batch_read_field(teuk_batch_t *b, int k, teuk_field f, double *out) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return read_field(b->b, k, (int)f, out);
}
int teuk_batch_set_stream(teuk_batch_t *b, void *st) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_stream(b->b, st);
}
int teuk_batch_size(const teuk_batch_t *b) { return b ? (int)b->b.inst.size() : 0; }
double teuk_batch_dt(const teuk_batch_t *b, int k) {
    return (b && k >= 0 && k < (int)b->b.inst.size()) ? b->b.inst[k].dt_lead : 0.0;
}
int teuk_batch_set_tile(teuk_batch_t *b, int segcols) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_launch(b->b, segcols, b->b.nt_req);
}
int teuk_batch_use_graph(teuk_batch_t *b, int k) {
    if (!b || k < 0) return fail(TEUK_EINVAL, "bad handle or graph length");
    drop_graph(b->b);
    b->b.graph_steps = k;
    return TEUK_OK;
}

int teuk_prepare_graph(teuk_t *h) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return prepare_graph(h->b);
}
int teuk_batch_prepare_graph(teuk_batch_t *b) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return prepare_graph(b->b);
}
long teuk_graph_replays(const teuk_t *h) { return h ? h->b.graph_replays : -1; }
long teuk_batch_graph_replays(const teuk_batch_t *b) { return b ? b->b.graph_replays : -1; }

static int set_round_trip(Batch &b, int on) {
    if (int rc = quiesce(b)) return rc;
    if (!on) {
        if (b.host_state) hipHostFree(b.host_state);
        b.host_state = nullptr;
        return TEUK_OK;
    }
    if (b.host_state) return TEUK_OK;
    size_t bytes = 0;
    for (const Instance &I : b.inst) bytes = std::max(bytes, 4 * (size_t)I.words * I.plane() * sizeof(double));
    const hipError_t e = hipHostMalloc((void **)&b.host_state, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        b.host_state = nullptr;
        return hip_fail(e, "hipHostMalloc(round-trip buffer)");
    }
    drop_graph(b);
    return TEUK_OK;
}
int teuk_set_host_round_trip(teuk_t *h, int on) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    return set_round_trip(h->b, on);
}
int teuk_batch_set_host_round_trip(teuk_batch_t *b, int on) {
    if (!b) return fail(TEUK_EINVAL, "handle is NULL");
    return set_round_trip(b->b, on);
}

int teuk_set_observer(teuk_t *h, int n_points, const int *i, const int *j, int every, long capacity) {
    if (!h) return fail(TEUK_EINVAL, "handle is NULL");
    Batch &b = h->b;
    const Instance &I = b.inst[0];
    if (n_points < 0 || n_points > kMaxObserverPoints)
        return fail(TEUK_EINVAL, "n_points must be 0..1024");
    if (n_points > 0) {
        if (!i || !j) return fail(TEUK_EINVAL, "point index array is NULL");
        for (int p = 0; p < n_points; ++p)
            if (i[p] < 0 || i[p] >= I.g.n_r || j[p] < 0 || j[p] >= I.g.n_theta)
                return fail(TEUK_EINVAL, "observer point outside the grid");
        if (every < 1) return fail(TEUK_EINVAL, "every must be >= 1");
        const double doubles = (double)capacity * (1.0 + 2.0 * b.words * n_points);
        if (capacity < 1 || doubles > kMaxObserverDoubles)
            return fail(TEUK_EINVAL, "capacity must be >= 1 and hold at most 2^28 doubles of records");
    }
    if (int rc = quiesce(b)) return rc;
    free_observer(b);
    drop_graph(b);
    if (n_points == 0) return TEUK_OK;
    std::vector<int> idx(n_points);
    for (int p = 0; p < n_points; ++p) idx[p] = i[p] * I.g.n_theta + j[p];
    const size_t rec = 1 + 2 * (size_t)b.words * n_points;
    hipError_t e = hipMalloc((void **)&b.obs_idx, n_points * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&b.obs_ring, (size_t)capacity * rec * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&b.obs_ctr, 3 * sizeof(long long));
    if (e == hipSuccess) e = hipMemcpy(b.obs_idx, idx.data(), n_points * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_observer(b);
        return hip_fail(e, "observer buffers");
    }
    b.obs_n = n_points;
    b.obs_every = every;
    b.obs_cap = capacity;
    return reset_observer(b, I.steps, true);
}

int teuk_read_observer(teuk_t *h, long max_records, double *out, long *n_out, long *n_total) {
    if (!h || max_records < 0 || (max_records > 0 && !out)) return fail(TEUK_EINVAL, "bad arguments");
    Batch &b = h->b;
    if (int rc = check_ok(b)) return rc;
    if (b.obs_n <= 0) return fail(TEUK_EINVAL, "no observer is set");
    long long c[3] = {0, 0, 0};
    hipError_t e = hipStreamSynchronize(b.stream);
    if (e == hipSuccess) {
        // records of a slab launch that ended early are not valid
        if (int rc = slab_check(b)) return rc;
        e = hipMemcpy(c, b.obs_ctr, sizeof c, hipMemcpyDeviceToHost);
    }
    const size_t rec = 1 + 2 * (size_t)b.words * b.obs_n;
    const long held = (long)std::min<long long>(c[1], b.obs_cap);
    const long n = std::min(held, max_records);
    // the n most recent records, oldest first: records c[1]-n .. c[1]-1, which
    // sit in ring slots q0 .. q0+n-1 (mod capacity): at most two copies
    if (e == hipSuccess && n > 0) {
        const long long q0 = (c[1] - n) % b.obs_cap;
        const long first = (long)std::min<long long>(n, b.obs_cap - q0);
        e = hipMemcpy(out, b.obs_ring + (size_t)q0 * rec, (size_t)first * rec * sizeof(double), hipMemcpyDeviceToHost);
        if (e == hipSuccess && first < n)
            e = hipMemcpy(out + (size_t)first * rec, b.obs_ring, (size_t)(n - first) * rec * sizeof(double),
                          hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) {
        b.sticky = TEUK_EDEVICE;
        return hip_fail(e, "read observer");
    }
    if (n_out) *n_out = n;
    if (n_total) *n_total = (long)c[1];
    return TEUK_OK;
}

// ---- allocation-free coefficient pass (teuk_coefficients_noalloc)
int teuk_coefficients_noalloc(int s, int m, double a_over_M, const teuk_grid *grid, teuk_precision prec,
                              double *d_ch, double *d_cf, double *d_wt, void *stream) {
    int rc = validate(s, m, a_over_M, grid, (int)prec);
    if (rc != TEUK_OK) return rc;
    if (!d_ch || !d_cf || !d_wt) return fail(TEUK_EINVAL, "output pointer is NULL");
    const int W = (int)prec;
    const size_t need = lwk::coef_scratch_doubles(W, grid->n_r, grid->n_theta, W == 1);
    if (need > kScratchDoubles)
        return fail(TEUK_EINVAL, "grid needs " + std::to_string(need) + " doubles of scratch; the library holds " +
                                     std::to_string(kScratchDoubles));
    double *scr = nullptr;
    if ((rc = scratch_on_current_device(&scr)) != TEUK_OK) return rc;
    lwk::CoefJob J{};
    J.s = s;
    J.m = m;
    J.nr = grid->n_r;
    J.nth = grid->n_theta;
    J.reach = grid->angular_order / 2;
    J.a_over_M = a_over_M;
    J.mass = grid->mass;
    J.rstar_min = grid->rstar_min;
    J.rstar_max = grid->rstar_max;
    J.cfl = grid->cfl;
    J.ch = d_ch;
    J.cf = d_cf;
    J.wt = d_wt;
    J.onfly = 0;
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = W == 1 ? lwk::coef_pass_into_f64(J, scr, true, st)
                 : W == 2 ? lwk::coef_pass_into_dd(J, scr, st)
                          : lwk::coef_pass_into_qd(J, scr, st);
    if (e != hipSuccess) return hip_fail(e, "coefficient pass");
    return TEUK_OK;
}

}  // extern "C"

// lbm_sc.hip -- host side of the C ABI declared in include/lbm_sc.h.
//
// Owns validation, the batched plan (flattened tile list over instances of
// any size, per-instance device table), the step loop with its QoI window,
// HIP-graph replay of step pairs, the block-size autotuner and the calls
// into the kernels of kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "lbm_sc.h"
#include "kernels.h"
#include "quadrature.h"

using namespace lbmsc;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Clears n words with a kernel: entry points that a caller may capture into
// a graph record no memset nodes.
__global__ __launch_bounds__(256) void k_clear_i32(int32_t *__restrict__ p, int32_t n)
{
    const int32_t e = blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (e < n) p[e] = 0;
}

hipError_t clear_i32(int32_t *p, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

int64_t ncells_of(const lbm_domain *d) { return (int64_t)d->nx * d->ny * d->nz; }

int64_t stride_of(int64_t ncells)
{
    // an odd number of 256-byte blocks per population plane, so the 19 planes
    // do not all start on the same HBM channel
    int64_t blocks = (ncells + 63) / 64;
    if ((blocks & 1) == 0) blocks += 1;
    return blocks * 64;
}

int check_domain(const lbm_domain *d)
{
    if (!d) return fail(LBM_E_INVALID, "domain is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(LBM_E_INVALID, "non-positive box size");
    const int64_t n = ncells_of(d);
    // kernels address a population array with 32-bit byte offsets
    if (n > (int64_t)INT32_MAX || 19 * stride_of(n) >= ((int64_t)1 << 30))
        return fail(LBM_E_INVALID, "box of %lld cells exceeds the 32-bit byte-offset range", (long long)n);
    const int *f = d->face;
    for (int k = 0; k < 6; ++k)
        if (f[k] < LBM_WALL || f[k] > LBM_PERIODIC) return fail(LBM_E_INVALID, "face %d has unknown kind %d", k, f[k]);
    for (int a = 0; a < 3; ++a)
        if ((f[2 * a] == LBM_PERIODIC) != (f[2 * a + 1] == LBM_PERIODIC))
            return fail(LBM_E_INVALID, "periodic faces must come in pairs (axis %d)", a);
    if (!(f[0] == LBM_WALL || f[0] == LBM_INLET || f[0] == LBM_PERIODIC))
        return fail(LBM_E_INVALID, "-x face must be WALL, INLET or PERIODIC");
    if (!(f[1] == LBM_WALL || f[1] == LBM_OUTLET || f[1] == LBM_PERIODIC))
        return fail(LBM_E_INVALID, "+x face must be WALL, OUTLET or PERIODIC");
    if (f[2] == LBM_INLET || f[2] == LBM_OUTLET || f[2] == LBM_FREESLIP || f[3] == LBM_INLET ||
        f[3] == LBM_OUTLET || f[3] == LBM_FREESLIP)
        return fail(LBM_E_INVALID, "y faces must be WALL or PERIODIC");
    if (!(f[4] == LBM_WALL || f[4] == LBM_PERIODIC)) return fail(LBM_E_INVALID, "-z face must be WALL or PERIODIC");
    if (!(f[5] == LBM_WALL || f[5] == LBM_FREESLIP || f[5] == LBM_PERIODIC))
        return fail(LBM_E_INVALID, "+z face must be WALL, FREESLIP or PERIODIC");
    if (f[1] == LBM_OUTLET && (d->nx & 1))
        return fail(LBM_E_INVALID, "an outlet needs an even nx (got %d)", d->nx);
    if (f[1] == LBM_OUTLET && d->nx < 2) return fail(LBM_E_INVALID, "an outlet needs nx >= 2");
    return LBM_OK;
}

Box box_of(const lbm_domain *d)
{
    Box b;
    b.nx = d->nx;
    b.ny = d->ny;
    b.nz = d->nz;
    for (int k = 0; k < 6; ++k) b.face[k] = d->face[k];
    return b;
}

struct GeoPtrs {
    uint8_t *flags;
    uint32_t *smask;
    int32_t *probes;
};

GeoPtrs geo_ptrs(const void *base, const lbm_domain *d)
{
    const int64_t n = ncells_of(d);
    char *b = (char *)base;
    GeoPtrs p;
    p.flags = (uint8_t *)b;
    p.smask = (uint32_t *)(b + align256(n));
    p.probes = (int32_t *)(b + align256(n) + align256(4 * n));
    return p;
}

int check_device()
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBM_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
    return LBM_OK;
}

// Device scratch of lbm_adjoint_step_inplace_noalloc: the instance tables
// of buffer pointers and the per-tile gradient partials of one adjoint step.
// One copy per device, resident until the process ends.  Host code never
// uses the array's name as an address: the device address of each device's
// copy is taken once with hipGetSymbolAddress (scratch_ptr).
constexpr size_t SCRATCH_BYTES = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with the device current).
int scratch_ptr(unsigned char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_E_UNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_E_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_dev[dev];
    return LBM_OK;
}

}  // namespace

struct lbm_plan {
    int n_inst = 0;
    int model = 0;
    Variant v{256, 1, 1, 0};
    std::vector<lbm_instance> inst;
    std::vector<Geo> geo_h;
    Geo *geo_d = nullptr;
    int32_t *tiles_d = nullptr;
    uint64_t *tinfo_d = nullptr;  // per tile: all-solid lines and wavefront classes (launch_tile_info)
    int32_t n_tiles = 0;
    int32_t *health_d = nullptr;
    int64_t step = 0;
    int64_t avg_begin = 0, avg_end = 0;
    int pending = 0;             // states accumulated in the FP32 partials since the last flush
    int flush_every = 64;
    int64_t steady_from = 0;     // from this step on every instance's inflow is constant in time
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    int graph_pairs = 8;
    // instance blocks for the memory-side cache: consecutive instances whose
    // state fits block_bytes; plain stretches advance one block at a time
    // (used when there are two blocks or more and every instance fits)
    // 224 MiB: about 92 % of the 256 MB cache (blocks of 255 MB already run
    // 12 % slower per step than blocks of 223 MB)
    int64_t block_bytes = int64_t(224) << 20;
    std::vector<std::pair<int32_t, int32_t>> blocks;   // tile ranges [begin, end)
    std::vector<hipGraphExec_t> bexec;
    std::map<std::vector<uintptr_t>, void *> tables;
    double *gpart_d = nullptr;   // per-tile adjoint gradient partials [gpart_tiles][3]
    int32_t gpart_tiles = 0;
};

namespace {

// Instance blocks (see lbm_plan::block_bytes): the state one step touches
// per instance is its populations and per-cell flags and solid-link masks.
int build_blocks(lbm_plan *p)
{
    for (auto e : p->bexec) HIPCHK(hipGraphExecDestroy(e));
    p->bexec.clear();
    p->blocks.clear();
    if (p->block_bytes <= 0) return LBM_OK;
    std::vector<std::pair<int32_t, int32_t>> b;
    int64_t used = 0;
    for (int i = 0; i < p->n_inst; ++i) {
        const Geo &g = p->geo_h[i];
        const int64_t bytes = (int64_t)Q * 4 * g.qs + 5 * (int64_t)g.ncells;
        if (bytes > p->block_bytes) return LBM_OK;          // an instance alone overflows the cache
        const int32_t t0 = g.tile0;
        const int32_t t1 = i + 1 < p->n_inst ? p->geo_h[i + 1].tile0 : p->n_tiles;
        if (b.empty() || used + bytes > p->block_bytes) {
            b.push_back({t0, t1});
            used = 0;
        } else {
            b.back().second = t1;
        }
        used += bytes;
    }
    if (b.size() >= 2) p->blocks = b;
    return LBM_OK;
}

int build_tiles(lbm_plan *p)
{
    std::vector<int32_t> tiles;
    for (int i = 0; i < p->n_inst; ++i) {
        Geo &g = p->geo_h[i];
        g.tile0 = (int32_t)tiles.size();
        const int64_t nt = (g.ncells + p->v.tile() - 1) / p->v.tile();
        if ((int64_t)tiles.size() + nt > (int64_t)INT32_MAX / 2) return fail(LBM_E_INVALID, "too many tiles");
        for (int64_t t = 0; t < nt; ++t) tiles.push_back(i);
    }
    if (p->tiles_d) HIPCHK(hipFree(p->tiles_d));
    p->tiles_d = nullptr;
    p->n_tiles = (int32_t)tiles.size();
    HIPCHK(hipMalloc(&p->tiles_d, sizeof(int32_t) * std::max<size_t>(1, tiles.size())));
    HIPCHK(hipMemcpy(p->tiles_d, tiles.data(), sizeof(int32_t) * tiles.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->geo_d, p->geo_h.data(), sizeof(Geo) * p->n_inst, hipMemcpyHostToDevice));
    // the flags may still be in flight on the caller's geometry stream
    if (p->tinfo_d) HIPCHK(hipFree(p->tinfo_d));
    p->tinfo_d = nullptr;
    HIPCHK(hipMalloc(&p->tinfo_d, 2 * sizeof(uint64_t) * std::max<size_t>(1, tiles.size())));
    HIPCHK(hipDeviceSynchronize());
    if (launch_tile_info(p->v.tile(), p->geo_d, p->tiles_d, p->n_tiles, p->tinfo_d, nullptr))
        return fail(LBM_E_HIP, "tile-info launch failed");
    HIPCHK(hipDeviceSynchronize());
    if (p->gexec) {
        HIPCHK(hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
    }
    return build_blocks(p);
}

void set_theta(Geo &g, const lbm_instance &in)
{
    g.inflow = in.inflow;
    g.speed = in.theta[0];
    g.phi = in.theta[1];
    g.cphi = std::cos(in.theta[1]);
    g.sphi = std::sin(in.theta[1]);
    g.z0 = in.theta[2];
    g.series = nullptr;
    g.series_len = g.hour_steps = g.blend_steps = 0;
    g.inv_log_h = g.dlog_h = 0.0f;
    if (in.inflow == LBM_INFLOW_SERIES) {
        g.series = in.series_dev;
        g.series_len = in.series_len;
        g.hour_steps = in.hour_steps;
        g.blend_steps = in.blend_steps;
        const double H = in.ref_height, z0 = in.theta[2];
        g.inv_log_h = (float)(1.0 / std::log((H + z0) / z0));
        g.dlog_h = (float)(1.0 / (H + z0) - 1.0 / z0);
    }
}

// parameters of an instance's inflow that the kernels rely on
int check_inflow(const lbm_instance &in, const float theta[3])
{
    if (in.inflow == LBM_INFLOW_LOGLAW && !(theta[2] > 0.0f)) return fail(LBM_E_INVALID, "z0 must be positive");
    if (in.inflow != LBM_INFLOW_SERIES) return LBM_OK;
    if (!(theta[2] > 0.0f)) return fail(LBM_E_INVALID, "z0 must be positive");
    if (!in.series_dev || in.series_len < 1 || in.hour_steps < 1 || in.blend_steps < 0 ||
        in.blend_steps > in.hour_steps || !(in.ref_height > 0.0f))
        return fail(LBM_E_INVALID, "series inflow: need a series, series_len >= 1, hour_steps >= 1, "
                                   "0 <= blend_steps <= hour_steps and ref_height > 0");
    return LBM_OK;
}

// device copy of a host array of pointers, cached by content
template <class T>
int table_of(lbm_plan *p, const T *host, T **out)
{
    std::vector<uintptr_t> key(p->n_inst);
    for (int i = 0; i < p->n_inst; ++i) key[i] = (uintptr_t)host[i];
    auto it = p->tables.find(key);
    if (it != p->tables.end()) {
        *out = (T *)it->second;
        return LBM_OK;
    }
    if (p->tables.size() >= 64) {
        HIPCHK(hipDeviceSynchronize());
        for (auto &kv : p->tables) HIPCHK(hipFree(kv.second));
        p->tables.clear();
    }
    void *d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(uintptr_t) * p->n_inst));
    HIPCHK(hipMemcpy(d, key.data(), sizeof(uintptr_t) * p->n_inst, hipMemcpyHostToDevice));
    p->tables[key] = d;
    *out = (T *)d;
    return LBM_OK;
}

bool step_accumulates(const lbm_plan *p, int64_t n) { return p->avg_begin < n && n < p->avg_end; }

int flush(lbm_plan *p, hipStream_t s)
{
    if (launch_flush(p->v.tile(), p->geo_d, p->tiles_d, p->n_tiles, s)) return fail(LBM_E_HIP, "flush launch failed");
    p->pending = 0;
    return LBM_OK;
}

int ensure_graph(lbm_plan *p)
{
    if (p->gexec) return LBM_OK;
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    StepArgs a{};
    a.step = (p->steady_from + 1) / 2 * 2 + 2;
    a.tinfo = p->tinfo_d;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < p->graph_pairs; ++k) {
        launch_step(p->v, p->model, 0, p->geo_d, p->tiles_d, p->n_tiles, a, p->health_d, cap);
        launch_step(p->v, p->model, 1, p->geo_d, p->tiles_d, p->n_tiles, a, p->health_d, cap);
    }
    hipGraph_t g;
    HIPCHK(hipStreamEndCapture(cap, &g));
    HIPCHK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
    HIPCHK(hipStreamDestroy(cap));
    return LBM_OK;
}

int ensure_block_graphs(lbm_plan *p)
{
    if (!p->bexec.empty()) return LBM_OK;
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    for (auto &bl : p->blocks) {
        StepArgs a{};
        a.step = (p->steady_from + 1) / 2 * 2 + 2;
        a.tinfo = p->tinfo_d;
        a.tile_base = bl.first;
        HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < p->graph_pairs; ++k) {
            launch_step(p->v, p->model, 0, p->geo_d, p->tiles_d, bl.second, a, p->health_d, cap);
            launch_step(p->v, p->model, 1, p->geo_d, p->tiles_d, bl.second, a, p->health_d, cap);
        }
        hipGraph_t g;
        HIPCHK(hipStreamEndCapture(cap, &g));
        hipGraphExec_t e;
        HIPCHK(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(g));
        p->bexec.push_back(e);
    }
    HIPCHK(hipStreamDestroy(cap));
    return LBM_OK;
}

bool pair_plain(const lbm_plan *p, int64_t n)
{
    for (int64_t m = n; m < n + 2; ++m) {
        if (m < p->steady_from) return false;
        if (p->avg_end > p->avg_begin && m >= p->avg_begin && m < p->avg_end + 1) return false;
    }
    return true;
}

// kind > 0 records the state of every step; qoi: the steps also add to the
// QoI sums (a forward run that records), else recording leaves them alone
// (the adjoint sweep's segment re-runs)
int run_steps(lbm_plan *p, int32_t n_steps, int32_t kind, float *const *rec_d, int32_t n_slots, hipStream_t s,
              bool qoi = false)
{
    const bool sums = kind == 0 || qoi;
    int32_t left = n_steps;
    while (left > 0) {
        const int64_t n = p->step;
        // replay captured pairs over stretches without ramp, QoI or recording
        if (p->use_graph && kind == 0 && (n & 1) == 0 && left >= 2 * p->graph_pairs) {
            bool plain = true;
            for (int k = 0; k < p->graph_pairs && plain; ++k) plain = pair_plain(p, n + 2 * k);
            if (plain && !p->blocks.empty()) {
                // the whole plain stretch one instance block at a time: the
                // steps of a stretch do not depend on the step index, so each
                // instance takes them in order while its state stays in the
                // memory-side cache
                int64_t pairs = 0;
                while (2 * (pairs + 1) <= left && pair_plain(p, n + 2 * pairs)) ++pairs;
                pairs -= pairs % p->graph_pairs;
                int r = ensure_block_graphs(p);
                if (r) return r;
                for (auto e : p->bexec)
                    for (int64_t k = 0; k < pairs; k += p->graph_pairs) HIPCHK(hipGraphLaunch(e, s));
                p->step += 2 * pairs;
                left -= (int32_t)(2 * pairs);
                continue;
            }
            if (plain) {
                int r = ensure_graph(p);
                if (r) return r;
                HIPCHK(hipGraphLaunch(p->gexec, s));
                p->step += 2 * p->graph_pairs;
                left -= 2 * p->graph_pairs;
                continue;
            }
        }
        if (!p->blocks.empty()) {
            // ramp, blend and window steps, and every step of a recording
            // run, one instance block at a time too, in chunks of steps with
            // per-step arguments: a chunk ends where the QoI accumulation
            // starts or stops, at the window's last state (captured
            // batch-wide), where the steady inflow begins, after the states
            // the FP32 partials may hold before the (batch-wide) flush, so
            // the sums keep their order, and, in runs that do not record,
            // past the steady inflow's start at the next even step (plain
            // stretches take the graphs above).  Records are per instance
            // (slot n % n_slots), so each instance writes the same records
            // in the same order as in the batched order.
            const bool acc = sums && step_accumulates(p, n);
            const bool window = sums && p->avg_end > p->avg_begin;
            int32_t chunk = 0;
            for (; chunk < left; ++chunk) {
                const int64_t m = n + chunk;
                if ((sums && step_accumulates(p, m)) != acc) break;
                if (n < p->steady_from && m >= p->steady_from) break;
                if (acc && p->pending + chunk >= p->flush_every) break;
                if (chunk > 0 && window && m == p->avg_end) break;
                if (kind == 0 && chunk > 0 && !acc && m >= p->steady_from && (m & 1) == 0) break;
            }
            if (chunk >= 2) {
                for (auto &bl : p->blocks) {
                    for (int32_t k = 0; k < chunk; ++k) {
                        StepArgs a{};
                        a.step = n + k;
                        a.tinfo = p->tinfo_d;
                        a.accumulate = acc ? 1 : 0;
                        a.record = kind;
                        a.rec = rec_d;
                        a.rec_slot = kind ? (int32_t)((n + k) % n_slots) : 0;
                        a.tile_base = bl.first;
                        if (launch_step(p->v, p->model, (int)((n + k) & 1), p->geo_d, p->tiles_d, bl.second, a,
                                        p->health_d, s))
                            return fail(LBM_E_HIP, "step launch failed: %s", hipGetErrorString(hipGetLastError()));
                    }
                }
                p->step = n + chunk;
                left -= chunk;
                if (acc) p->pending += chunk;
                if (window && p->step == p->avg_end && p->step > p->avg_begin) {
                    if (launch_capture(p->v.tile(), (int)(p->step & 1), p->geo_d, p->tiles_d, p->n_tiles, p->step,
                                       p->health_d, s))
                        return fail(LBM_E_HIP, "capture launch failed");
                    ++p->pending;
                    int r = flush(p, s);
                    if (r) return r;
                } else if (p->pending >= p->flush_every) {
                    int r = flush(p, s);
                    if (r) return r;
                }
                continue;
            }
        }
        StepArgs a{};
        a.step = n;
        a.tinfo = p->tinfo_d;
        a.accumulate = (sums && step_accumulates(p, n)) ? 1 : 0;
        a.record = kind;
        a.rec = rec_d;
        a.rec_slot = kind ? (n % n_slots) : 0;
        if (launch_step(p->v, p->model, (int)(n & 1), p->geo_d, p->tiles_d, p->n_tiles, a, p->health_d, s))
            return fail(LBM_E_HIP, "step launch failed: %s", hipGetErrorString(hipGetLastError()));
        p->step = n + 1;
        --left;
        if (a.accumulate) ++p->pending;
        if (sums && p->avg_end > p->avg_begin && p->step == p->avg_end && p->step > p->avg_begin) {
            // the last state of the window is never collided inside the window
            if (launch_capture(p->v.tile(), (int)(p->step & 1), p->geo_d, p->tiles_d, p->n_tiles, p->step,
                               p->health_d, s))
                return fail(LBM_E_HIP, "capture launch failed");
            ++p->pending;
            int r = flush(p, s);
            if (r) return r;
        } else if (p->pending >= p->flush_every) {
            int r = flush(p, s);
            if (r) return r;
        }
    }
    return LBM_OK;
}

int check_plan(const lbm_plan *p)
{
    if (!p) return fail(LBM_E_INVALID, "plan is NULL");
    return LBM_OK;
}

std::string tune_key(const lbm_plan *p)
{
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    std::vector<std::string> dims;
    for (auto &in : p->inst) {
        char b[64];
        snprintf(b, sizeof b, "%dx%dx%d", in.dom.nx, in.dom.ny, in.dom.nz);
        dims.push_back(b);
    }
    std::sort(dims.begin(), dims.end());
    std::ostringstream os;
    // the build stamp keeps results of an older kernel build from being reused
    os << std::string(prop.gcnArchName).substr(0, 6) << "|" << __DATE__ << " " << __TIME__ << "|m" << p->model
       << "|n" << p->n_inst << "|b" << p->blocks.size();
    // run-length encoded multiset of box sizes
    for (size_t i = 0; i < dims.size();) {
        size_t j = i;
        while (j < dims.size() && dims[j] == dims[i]) ++j;
        os << "|" << dims[i] << "*" << (j - i);
        i = j;
    }
    return os.str();
}

std::string tune_path()
{
    const char *e = std::getenv("LBMSC_TUNE_CACHE");
    if (e && *e) return e;
    const char *h = std::getenv("HOME");
    return std::string(h ? h : ".") + "/.cache/lbmsc_tune.json";
}

std::map<std::string, int> read_tune_cache()
{
    std::map<std::string, int> m;
    std::ifstream in(tune_path());
    if (!in) return m;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    for (;;) {
        size_t a = t.find('"', pos);
        if (a == std::string::npos) break;
        size_t b = t.find('"', a + 1);
        if (b == std::string::npos) break;
        size_t c = t.find(':', b);
        if (c == std::string::npos) break;
        m[t.substr(a + 1, b - a - 1)] = std::atoi(t.c_str() + c + 1);
        pos = c + 1;
    }
    return m;
}

void write_tune_cache(const std::map<std::string, int> &m)
{
    const std::string path = tune_path();
    // create the missing directories of the path one by one (no shell)
    for (size_t slash = path.find('/', 1); slash != std::string::npos; slash = path.find('/', slash + 1)) {
        struct stat st;
        const std::string dir = path.substr(0, slash);
        if (stat(dir.c_str(), &st) == 0) {
            if (!S_ISDIR(st.st_mode)) return;
            continue;
        }
        if (mkdir(dir.c_str(), 0755) != 0 && stat(dir.c_str(), &st) != 0) return;
    }
    std::ofstream out(path + ".tmp");
    out << "{\n";
    size_t k = 0;
    for (auto &kv : m) out << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
    out << "}\n";
    out.close();
    std::rename((path + ".tmp").c_str(), path.c_str());
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }
const char *lbm_version(void) { return "lbmsc 1.0 (gfx950, D3Q19 AA in-place, BGK/Smagorinsky, adjoint)"; }

int lbm_quadrature(int32_t kind, int32_t level, int32_t dim, double *nodes_host, double *weights_host, int32_t cap,
                   int32_t *n_out)
{
    std::vector<double> x, w;
    if (kind == LBM_QUAD_GAUSS_LEGENDRE) {
        if (dim != 1) return fail(LBM_E_INVALID, "Gauss-Legendre rules are one-dimensional");
        if (level < 1 || level > 256) return fail(LBM_E_INVALID, "Gauss-Legendre point count %d out of range", level);
        if (!gauss_legendre(level, x, w)) return fail(LBM_E_INVALID, "Gauss-Legendre eigen-solve failed");
    } else if (kind == LBM_QUAD_SMOLYAK_CC) {
        if (!smolyak_cc(level, dim, x, w)) return fail(LBM_E_INVALID, "Smolyak level %d dim %d not supported", level, dim);
    } else if (kind == LBM_QUAD_GAUSS_HERMITE) {
        if (level < 1 || level > 256) return fail(LBM_E_INVALID, "Gauss-Hermite point count %d out of range", level);
        if (!tensor_gauss_hermite(level, dim, x, w))
            return fail(LBM_E_INVALID, "Gauss-Hermite rule with %d points in %d dimensions not supported", level, dim);
    } else {
        return fail(LBM_E_INVALID, "unknown quadrature kind %d", kind);
    }
    const int32_t n = (int32_t)w.size();
    if (n_out) *n_out = n;
    if (!nodes_host && !weights_host) return LBM_OK;
    if (!nodes_host || !weights_host) return fail(LBM_E_INVALID, "nodes and weights must both be given");
    if (cap < n) return fail(LBM_E_INVALID, "capacity %d < %d nodes", cap, n);
    std::memcpy(nodes_host, x.data(), sizeof(double) * x.size());
    std::memcpy(weights_host, w.data(), sizeof(double) * w.size());
    return LBM_OK;
}

int lbm_gpc_basis(const double *nodes_host, const double *weights_host, int32_t n_nodes, int32_t dim,
                  int32_t order, double *phi_out, int32_t *alpha_out, int32_t cap, int32_t *n_basis)
{
    if (dim < 1 || dim > 8 || order < 0 || order > 16 || n_nodes < 0)
        return fail(LBM_E_INVALID, "gPC basis: need 1 <= dim <= 8, 0 <= order <= 16, n_nodes >= 0");
    std::vector<int> alpha;
    gpc_multi_indices(dim, order, alpha);
    const int32_t P = (int32_t)(alpha.size() / dim);
    if (n_basis) *n_basis = P;
    if (!phi_out) return LBM_OK;
    if (!nodes_host || !alpha_out) return fail(LBM_E_INVALID, "gPC basis: nodes and alpha output needed");
    if (cap < n_nodes) return fail(LBM_E_INVALID, "gPC basis: capacity %d < %d nodes", cap, n_nodes);
    std::vector<double> phi;
    gpc_basis(nodes_host, n_nodes, dim, alpha, phi);
    // projection weights of the coefficients c_p = sum_j a_j Q_j Phi_p(Z^(j))
    if (weights_host)
        for (int32_t j = 0; j < n_nodes; ++j)
            for (int32_t k = 0; k < P; ++k) phi[(size_t)j * P + k] *= weights_host[j];
    std::memcpy(phi_out, phi.data(), sizeof(double) * phi.size());
    for (size_t k = 0; k < alpha.size(); ++k) alpha_out[k] = alpha[k];
    return LBM_OK;
}

int lbm_gpc_coefficients(const float *q_dev, const double *wphi_dev, int32_t n_nodes, int32_t n_basis,
                         int64_t n_elems, double *coef_dev, double *var_dev, double *band_dev, hipStream_t s)
{
    if (n_nodes < 1 || n_basis < 1 || n_basis > 64 || n_elems < 0)
        return fail(LBM_E_INVALID, "gPC coefficients: need n_nodes >= 1, 1 <= n_basis <= 64, n_elems >= 0");
    if (n_elems == 0) return LBM_OK;
    if (!q_dev || !wphi_dev || !coef_dev) return fail(LBM_E_INVALID, "gPC coefficients: NULL buffer");
    int r = check_device();
    if (r) return r;
    if (launch_gpc(q_dev, wphi_dev, n_nodes, n_basis, n_elems, coef_dev, var_dev, band_dev, s))
        return fail(LBM_E_HIP, "gPC launch failed: %s", hipGetErrorString(hipGetLastError()));
    return LBM_OK;
}

int lbm_node_params(const double *xi_host, int32_t dim, double base, double rel, double angle_deg, double z0,
                    float theta_out[3])
{
    if (!xi_host || !theta_out || dim < 1) return fail(LBM_E_INVALID, "bad arguments to lbm_node_params");
    theta_out[0] = (float)(base * (1.0 + rel * xi_host[0]));
    theta_out[1] = dim > 1 ? (float)(angle_deg * xi_host[1] * M_PI / 180.0) : 0.0f;
    theta_out[2] = (float)z0;
    return LBM_OK;
}

int64_t lbm_geometry_bytes(const lbm_domain *dom, int32_t n_probes)
{
    if (check_domain(dom) || n_probes < 0) return -1;
    const int64_t n = ncells_of(dom);
    return align256(n) + align256(4 * n) + align256(4 * (int64_t)std::max(1, n_probes));
}

int64_t lbm_population_stride(const lbm_domain *dom)
{
    if (check_domain(dom)) return -1;
    return stride_of(ncells_of(dom));
}

// A fluid cell takes all of its solid links by one rule (the per-cell
// FL_MANTLE bit), so none may border a building and the mantle region at
// once.  Walks the fluid neighbours of every building cell.
static int check_mantle_contact(const lbm_domain *dom, const uint8_t *solid)
{
    const int nx = dom->nx, ny = dom->ny, nz = dom->nz;
    const bool px = dom->face[0] == LBM_PERIODIC, py = dom->face[2] == LBM_PERIODIC, pz = dom->face[4] == LBM_PERIODIC;
    auto at = [&](int x, int y, int z, bool &in) -> uint8_t {
        if (px) x = wrap1(x, nx);
        if (py) y = wrap1(y, ny);
        if (pz) z = wrap1(z, nz);
        in = x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
        return in ? solid[((int64_t)z * ny + y) * nx + x] : (uint8_t)CELL_FLUID;
    };
    bool any_mantle = false;
    for (int64_t c = 0, n = (int64_t)nx * ny * nz; c < n && !any_mantle; ++c) any_mantle = solid[c] == CELL_MANTLE;
    if (!any_mantle) return LBM_OK;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (solid[((int64_t)z * ny + y) * nx + x] != CELL_BUILDING) continue;
                for (int i = 1; i < Q; ++i) {
                    // fluid cell f = b + c_i sees b as its neighbour f - c_i
                    int fx = x + cx(i), fy = y + cy(i), fz = z + cz(i);
                    bool in;
                    if (at(fx, fy, fz, in) != CELL_FLUID || !in) continue;
                    if (px) fx = wrap1(fx, nx);
                    if (py) fy = wrap1(fy, ny);
                    if (pz) fz = wrap1(fz, nz);
                    for (int j = 1; j < Q; ++j)
                        if (at(fx - cx(j), fy - cy(j), fz - cz(j), in) == CELL_MANTLE)
                            return fail(LBM_E_INVALID, "fluid cell (%d,%d,%d) borders a building and the mantle", fx,
                                        fy, fz);
                }
            }
    return LBM_OK;
}

int lbm_init_geometry(const lbm_domain *dom, const uint8_t *solid_host, const int32_t *probe_host, int32_t n_probes,
                      void *geom_dev, float *f_dev, hipStream_t stream)
{
    int r = check_domain(dom);
    if (r) return r;
    if (!solid_host || !geom_dev || !f_dev) return fail(LBM_E_INVALID, "NULL buffer");
    if (n_probes < 0 || (n_probes > 0 && !probe_host)) return fail(LBM_E_INVALID, "bad probe list");
    r = check_device();
    if (r) return r;
    const int64_t n = ncells_of(dom);
    const int nx = dom->nx, ny = dom->ny, nz = dom->nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const uint8_t kind = solid_host[((int64_t)z * ny + y) * nx + x];
                if (kind == CELL_FLUID) continue;
                if (kind > CELL_MANTLE)
                    return fail(LBM_E_INVALID, "cell (%d,%d,%d): mask code %d (0 fluid, 1 building, 2 mantle)", x, y,
                                z, (int)kind);
                if (dom->face[5] == LBM_FREESLIP && z == nz - 1 && kind == CELL_BUILDING)
                    return fail(LBM_E_INVALID, "building cell (%d,%d,%d) in the layer under a free-slip sky", x, y, z);
                if (dom->face[1] == LBM_OUTLET && x >= nx - 2)
                    return fail(LBM_E_INVALID, "solid cell (%d,%d,%d) in the last two columns before an outlet", x, y, z);
            }
    r = check_mantle_contact(dom, solid_host);
    if (r) return r;
    for (int32_t k = 0; k < n_probes; ++k) {
        const int32_t c = probe_host[k];
        if (c < 0 || c >= n) return fail(LBM_E_INVALID, "probe %d outside the box", k);
        if (k > 0 && c <= probe_host[k - 1]) return fail(LBM_E_INVALID, "probe cells must be strictly increasing");
        if (solid_host[c]) return fail(LBM_E_INVALID, "probe %d sits in a solid cell", k);
    }
    const int64_t qs = stride_of(n);
    GeoPtrs gp = geo_ptrs(geom_dev, dom);
    HIPCHK(hipStreamSynchronize(stream));
    if (n_probes > 0) HIPCHK(hipMemcpy(gp.probes, probe_host, sizeof(int32_t) * n_probes, hipMemcpyHostToDevice));
    // stage the solid mask in the last population plane (cleared right after)
    uint8_t *stage = (uint8_t *)(f_dev + 18 * qs);
    HIPCHK(hipMemcpy(stage, solid_host, (size_t)n, hipMemcpyHostToDevice));
    if (launch_init_geometry(box_of(dom), stage, gp.flags, gp.smask, gp.probes, n_probes, stream))
        return fail(LBM_E_HIP, "geometry kernel launch failed");
    HIPCHK(hipMemsetAsync(f_dev, 0, sizeof(float) * 19 * (size_t)qs, stream));
    return LBM_OK;
}

int lbm_plan_create(const lbm_instance *inst, int32_t n_inst, const lbm_plan_opts *opts, lbm_plan **plan_out)
{
    if (!inst || n_inst < 1 || !plan_out) return fail(LBM_E_INVALID, "bad plan arguments");
    *plan_out = nullptr;
    int r = check_device();
    if (r) return r;
    Variant v{256, 1, 1, 0};
    if (opts && opts->block) v.bs = opts->block;
    if (opts && opts->cells_per_thread) v.cpt = opts->cells_per_thread;
    if (opts && opts->block) v.nt = opts->nontemporal;
    if (opts && opts->block) v.xcd = opts->xcd_order;
    if (!variant_ok(v))
        return fail(LBM_E_INVALID, "launch shape: block must be 64, 128, 256 or 512, cells per thread 1, 2 or 4, "
                                   "non-temporal mask 0..3, XCD order 0 or 1");
    lbm_plan *p = new lbm_plan();
    p->n_inst = n_inst;
    p->v = v;
    p->inst.assign(inst, inst + n_inst);
    p->model = inst[0].model;
    if (opts) {
        p->avg_begin = opts->avg_begin;
        p->avg_end = opts->avg_end;
        p->use_graph = opts->use_graph != 0;
    }
    p->geo_h.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const lbm_instance &in = inst[i];
        r = check_domain(&in.dom);
        if (!r && (!in.geom_dev || !in.f_dev)) r = fail(LBM_E_INVALID, "instance %d: NULL buffer", i);
        if (!r && in.model != p->model) r = fail(LBM_E_INVALID, "instance %d: all instances of a plan share one model", i);
        if (!r && in.model != LBM_BGK && in.model != LBM_SMAGORINSKY && in.model != LBM_RR3)
            r = fail(LBM_E_INVALID, "instance %d: unknown model", i);
        if (!r && !(in.tau0 > 0.5f)) r = fail(LBM_E_INVALID, "instance %d: tau0 must exceed 1/2 (got %g)", i, in.tau0);
        if (!r && !(in.cs >= 0.0f)) r = fail(LBM_E_INVALID, "instance %d: negative Smagorinsky constant", i);
        if (!r && in.inflow != LBM_INFLOW_UNIFORM && in.inflow != LBM_INFLOW_LOGLAW &&
            in.inflow != LBM_INFLOW_SERIES)
            r = fail(LBM_E_INVALID, "instance %d: unknown inflow kind", i);
        if (!r) r = check_inflow(in, in.theta);
        if (!r && in.inflow == LBM_INFLOW_LOGLAW && !(in.theta[2] > 0.0f))
            r = fail(LBM_E_INVALID, "instance %d: log-law roughness z0 must be positive", i);
        if (!r && ((in.qoi_part_dev == nullptr) != (in.qoi_sum_dev == nullptr)))
            r = fail(LBM_E_INVALID, "instance %d: QoI partial and sum buffers go together", i);
        if (!r && in.n_probes < 0) r = fail(LBM_E_INVALID, "instance %d: negative probe count", i);
        if (r) {
            delete p;
            return r;
        }
        Geo &g = p->geo_h[i];
        std::memset(&g, 0, sizeof g);
        const int64_t n = ncells_of(&in.dom);
        GeoPtrs gp = geo_ptrs(in.geom_dev, &in.dom);
        g.f = in.f_dev;
        g.flags = gp.flags;
        g.smask = gp.smask;
        g.probes = gp.probes;
        g.qpart = in.qoi_part_dev;
        g.qsum = in.qoi_sum_dev;
        g.psum = in.probe_sum_dev;
        g.qs = stride_of(n);
        g.ncells = (int32_t)n;
        g.n_probes = in.n_probes;
        g.box = box_of(&in.dom);
        g.offy = in.dom.nx;
        g.offz = in.dom.nx * in.dom.ny;
        g.dx = make_fastdiv((uint32_t)in.dom.nx);
        g.dxy = make_fastdiv((uint32_t)(in.dom.nx * in.dom.ny));
        g.tau0 = in.tau0;
        g.kcs = in.model != LBM_BGK ? (float)(18.0 * std::sqrt(2.0) * in.cs * in.cs) : 0.0f;
        g.ramp = in.ramp;
        set_theta(g, in);
        // the inflow is time-dependent during the ramp and, for a measured
        // series, until the blend into its last hour has ended
        int64_t steady = in.ramp;
        if (in.inflow == LBM_INFLOW_SERIES)
            steady += (int64_t)(in.series_len - 1) * in.hour_steps + in.blend_steps;
        p->steady_from = std::max(p->steady_from, steady);
    }
    if (hipMalloc(&p->geo_d, sizeof(Geo) * n_inst) != hipSuccess ||
        hipMalloc(&p->health_d, sizeof(int32_t) * n_inst) != hipSuccess ||
        hipMemset(p->health_d, 0, sizeof(int32_t) * n_inst) != hipSuccess) {
        lbm_plan_destroy(p);
        return fail(LBM_E_HIP, "plan allocation failed");
    }
    r = build_tiles(p);
    if (r) {
        lbm_plan_destroy(p);
        return r;
    }
    *plan_out = p;
    return LBM_OK;
}

void lbm_plan_destroy(lbm_plan *p)
{
    if (!p) return;
    (void)hipDeviceSynchronize();
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    for (auto e : p->bexec) (void)hipGraphExecDestroy(e);
    for (auto &kv : p->tables) (void)hipFree(kv.second);
    if (p->geo_d) (void)hipFree(p->geo_d);
    if (p->tiles_d) (void)hipFree(p->tiles_d);
    if (p->tinfo_d) (void)hipFree(p->tinfo_d);
    if (p->health_d) (void)hipFree(p->health_d);
    if (p->gpart_d) (void)hipFree(p->gpart_d);
    delete p;
}

int64_t lbm_plan_step(const lbm_plan *p) { return p ? p->step : -1; }

int lbm_plan_set_cache_block(lbm_plan *p, int64_t bytes)
{
    int r = check_plan(p);
    if (r) return r;
    if (bytes < 0) return fail(LBM_E_INVALID, "negative cache block size");
    HIPCHK(hipDeviceSynchronize());                 // block graphs may still be in flight
    p->block_bytes = bytes;
    return build_blocks(p);
}

int32_t lbm_plan_cache_blocks(const lbm_plan *p) { return p ? (int32_t)p->blocks.size() : -1; }

int lbm_plan_set_step(lbm_plan *p, int64_t step)
{
    int r = check_plan(p);
    if (r) return r;
    if (step < 0 || (step & 1)) return fail(LBM_E_INVALID, "the step counter can only be set to an even step");
    p->step = step;
    p->pending = 0;
    return LBM_OK;
}

int lbm_plan_set_theta(lbm_plan *p, int32_t i, const float theta[3])
{
    int r = check_plan(p);
    if (r) return r;
    if (i < 0 || i >= p->n_inst || !theta) return fail(LBM_E_INVALID, "bad instance index or theta");
    r = check_inflow(p->inst[i], theta);
    if (r) return r;
    for (int k = 0; k < 3; ++k) p->inst[i].theta[k] = theta[k];
    set_theta(p->geo_h[i], p->inst[i]);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(p->geo_d + i, &p->geo_h[i], sizeof(Geo), hipMemcpyHostToDevice));
    return LBM_OK;
}

int lbm_plan_reset_qoi(lbm_plan *p, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    for (int i = 0; i < p->n_inst; ++i)
        if (launch_zero_qoi(p->geo_h[i], s)) return fail(LBM_E_HIP, "zero launch failed");
    HIPCHK(clear_i32(p->health_d, p->n_inst, s));
    p->pending = 0;
    return LBM_OK;
}

int lbm_sync(lbm_plan *p, hipStream_t s)
{
    (void)p;
    HIPCHK(hipStreamSynchronize(s));
    return LBM_OK;
}

int lbm_check_health(lbm_plan *p, hipStream_t s, int32_t *bad_inst)
{
    int r = check_plan(p);
    if (r) return r;
    std::vector<int32_t> h(p->n_inst);
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(h.data(), p->health_d, sizeof(int32_t) * p->n_inst, hipMemcpyDeviceToHost));
    for (int i = 0; i < p->n_inst; ++i)
        if (h[i]) {
            if (bad_inst) *bad_inst = i;
            return fail(LBM_E_UNSTABLE, "instance %d became unstable (rho <= 0 or not finite)", i);
        }
    if (bad_inst) *bad_inst = -1;
    return LBM_OK;
}

int lbm_collide_stream(lbm_plan *p, int32_t n_steps, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (n_steps < 0) return fail(LBM_E_INVALID, "negative step count");
    return run_steps(p, n_steps, 0, nullptr, 1, s);
}

namespace {

int collide_stream_record(lbm_plan *p, int32_t n_steps, int32_t kind, float *const *rec_host, int32_t n_slots,
                          bool qoi, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (n_steps < 0 || n_slots < 1 || !rec_host) return fail(LBM_E_INVALID, "bad record arguments");
    if (kind < 1 || kind > 3)
        return fail(LBM_E_INVALID, "record kind must be 1 (rho,u), 2 (populations) or 3 (regularised state)");
    if (kind == 3 && p->model != LBM_RR3) return fail(LBM_E_INVALID, "record kind 3 is for the regularised model");
    for (int i = 0; i < p->n_inst; ++i)
        if (!rec_host[i]) return fail(LBM_E_INVALID, "instance %d: NULL record buffer", i);
    float **rec_d = nullptr;
    r = table_of(p, (float *const *)rec_host, &rec_d);
    if (r) return r;
    return run_steps(p, n_steps, kind, rec_d, n_slots, s, qoi);
}

}  // namespace

int lbm_collide_stream_record(lbm_plan *p, int32_t n_steps, int32_t kind, float *const *rec_host, int32_t n_slots,
                              hipStream_t s)
{
    return collide_stream_record(p, n_steps, kind, rec_host, n_slots, false, s);
}

int lbm_collide_stream_record_qoi(lbm_plan *p, int32_t n_steps, int32_t kind, float *const *rec_host,
                                  int32_t n_slots, hipStream_t s)
{
    return collide_stream_record(p, n_steps, kind, rec_host, n_slots, true, s);
}

int lbm_read_fields(lbm_plan *p, int32_t i, float *out_dev, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (i < 0 || i >= p->n_inst || !out_dev) return fail(LBM_E_INVALID, "bad instance index or output");
    if (launch_fields((int)(p->step & 1), p->geo_d, i, p->geo_h[i], p->step, out_dev, 0, s))
        return fail(LBM_E_HIP, "fields launch failed");
    return LBM_OK;
}

int lbm_read_populations(lbm_plan *p, int32_t i, float *out_dev, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (i < 0 || i >= p->n_inst || !out_dev) return fail(LBM_E_INVALID, "bad instance index or output");
    if (launch_fields((int)(p->step & 1), p->geo_d, i, p->geo_h[i], p->step, out_dev, 1, s))
        return fail(LBM_E_HIP, "populations launch failed");
    return LBM_OK;
}

int lbm_qoi_average(lbm_plan *p, int32_t i, float *out_dev, float *probe_out_dev, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (i < 0 || i >= p->n_inst) return fail(LBM_E_INVALID, "bad instance index");
    const int64_t cnt = p->avg_end - p->avg_begin;
    if (cnt <= 0) return fail(LBM_E_INVALID, "the plan has no QoI window");
    const Geo &g = p->geo_h[i];
    if (out_dev && !g.qsum) return fail(LBM_E_INVALID, "instance %d has no QoI sums", i);
    if (probe_out_dev && !g.psum) return fail(LBM_E_INVALID, "instance %d has no probe sums", i);
    Geo gg = g;
    if (!out_dev) gg.qsum = nullptr;
    if (!probe_out_dev) gg.n_probes = 0;
    if (launch_average(gg, 1.0 / (double)cnt, out_dev, probe_out_dev, s)) return fail(LBM_E_HIP, "average launch failed");
    return LBM_OK;
}

int lbm_sc_moments(const float *q_dev, const double *w_host, int32_t n_nodes, int64_t n_elems, double *mean_dev,
                   double *var_dev, unsigned long long *n_negative_dev, hipStream_t stream)
{
    if (!w_host) return fail(LBM_E_INVALID, "NULL weights");
    if (n_nodes < 1 || n_nodes > 256) return fail(LBM_E_INVALID, "node count %d outside [1, 256]", n_nodes);
    if (n_elems < 0) return fail(LBM_E_INVALID, "negative element count");
    double sw = 0.0;
    for (int j = 0; j < n_nodes; ++j) sw += w_host[j];
    if (std::fabs(sw - 1.0) > 1e-12) return fail(LBM_E_INVALID, "weights sum to %.17g, not 1", sw);
    if (n_elems == 0) return LBM_OK;
    if (!q_dev || !mean_dev || !var_dev) return fail(LBM_E_INVALID, "NULL buffer");
    if (launch_moments(q_dev, w_host, n_nodes, n_elems, mean_dev, var_dev, n_negative_dev, stream))
        return fail(LBM_E_HIP, "moments launch failed");
    return LBM_OK;
}

namespace {

// mode 0: two buffers (natural layout); mode 1 / 2: one buffer in place
int adjoint_step(lbm_plan *p, int64_t step, float *const *lam_in_host, float *const *lam_out_host,
                 float *const *rec_host, int32_t kind, int32_t n_slots, const double *const *pw_host,
                 double *dJdtheta_dev, int mode, bool noalloc, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (!lam_in_host || !lam_out_host || !rec_host || !pw_host || !dJdtheta_dev || n_slots < 1 || step < 0)
        return fail(LBM_E_INVALID, "bad adjoint arguments");
    if (kind < 1 || kind > 3) return fail(LBM_E_INVALID, "record kind must be 1, 2 or 3");
    if (p->model == LBM_SMAGORINSKY && kind != 2)
        return fail(LBM_E_INVALID, "the Smagorinsky adjoint needs recorded populations (kind 2)");
    if (p->model == LBM_RR3 && kind == 1)
        return fail(LBM_E_INVALID, "the regularised adjoint needs recorded populations or its state (kind 2 or 3)");
    if (p->model == LBM_BGK && kind == 3) return fail(LBM_E_INVALID, "record kind 3 is for the regularised model");
    for (int i = 0; i < p->n_inst; ++i)
        if (!lam_in_host[i] || !lam_out_host[i] || !rec_host[i] || (mode == 0 && lam_in_host[i] == lam_out_host[i]))
            return fail(LBM_E_INVALID, "instance %d: missing or aliased adjoint buffers", i);
    AdjArgs a{};
    double *part = nullptr;
    if (noalloc) {
        // tables and partials in the device scratch array: [lam][rec][pw][partials]
        const size_t tab = (size_t)align256(8 * (int64_t)p->n_inst);
        const size_t need = 3 * tab + sizeof(double) * 3 * (size_t)p->n_tiles;
        if (need > SCRATCH_BYTES)
            return fail(LBM_E_INVALID,
                        "the allocation-free adjoint step needs %zu bytes of scratch for %d instances and %d tiles; "
                        "the limit is %zu",
                        need, p->n_inst, p->n_tiles, SCRATCH_BYTES);
        unsigned char *sp = nullptr;
        r = scratch_ptr(&sp);
        if (r) return r;
        HIPCHK(hipMemcpyAsync(sp, lam_out_host, 8 * (size_t)p->n_inst, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(sp + tab, rec_host, 8 * (size_t)p->n_inst, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(sp + 2 * tab, pw_host, 8 * (size_t)p->n_inst, hipMemcpyHostToDevice, s));
        a.lam_in = a.lam_out = (float *const *)sp;
        a.rec = (float *const *)(sp + tab);
        a.pw = (const double *const *)(sp + 2 * tab);
        part = (double *)(sp + 3 * tab);
    } else {
        r = table_of(p, (float *const *)lam_in_host, (float ***)&a.lam_in);
        if (!r) r = table_of(p, (float *const *)lam_out_host, (float ***)&a.lam_out);
        if (!r) r = table_of(p, (float *const *)rec_host, (float ***)&a.rec);
        if (!r) r = table_of(p, (const double *const *)pw_host, (const double ***)&a.pw);
        if (r) return r;
    }
    a.step = step;
    a.model = p->model;
    a.record = kind;
    a.rec_slot = step % n_slots;
    a.in_window = (p->avg_begin < step && step <= p->avg_end) ? 1 : 0;
    a.inv_count = p->avg_end > p->avg_begin ? 1.0 / (double)(p->avg_end - p->avg_begin) : 0.0;
    a.grad = dJdtheta_dev;
    if (!noalloc) {
        if (p->gpart_tiles < p->n_tiles) {
            if (p->gpart_d) HIPCHK(hipFree(p->gpart_d));
            p->gpart_d = nullptr;
            p->gpart_tiles = 0;
            HIPCHK(hipMalloc(&p->gpart_d, sizeof(double) * 3 * (size_t)p->n_tiles));
            p->gpart_tiles = p->n_tiles;
        }
        part = p->gpart_d;
    }
    // every tile writes its partial, so the buffer needs no clearing
    a.part = part;
    a.tinfo = p->tinfo_d;
    // the adjoint keeps more live state per cell than a step: it runs one
    // cell per thread over the same tiles (whole tile per workgroup, up to
    // 512 threads), which holds more wavefronts per SIMD in flight
    Variant va = p->v;
    va.bs = std::min(p->v.tile(), 512);
    va.cpt = p->v.tile() / va.bs;
    if (launch_adjoint(va, p->geo_d, p->tiles_d, p->n_tiles, a, mode, s) ||
        launch_grad_reduce(p->v.tile(), p->geo_h.data(), p->n_inst, p->geo_d, part, dJdtheta_dev, s))
        return fail(LBM_E_HIP, "adjoint launch failed: %s", hipGetErrorString(hipGetLastError()));
    return LBM_OK;
}

}  // namespace

int lbm_adjoint_step(lbm_plan *p, int64_t step, float *const *lam_in_host, float *const *lam_out_host,
                     float *const *rec_host, int32_t kind, int32_t n_slots, const double *const *pw_host,
                     double *dJdtheta_dev, hipStream_t s)
{
    return adjoint_step(p, step, lam_in_host, lam_out_host, rec_host, kind, n_slots, pw_host, dJdtheta_dev, 0, false,
                        s);
}

int lbm_adjoint_step_inplace(lbm_plan *p, int64_t step, float *const *lam_host, float *const *rec_host,
                             int32_t kind, int32_t n_slots, const double *const *pw_host, double *dJdtheta_dev,
                             hipStream_t s)
{
    return adjoint_step(p, step, lam_host, lam_host, rec_host, kind, n_slots, pw_host, dJdtheta_dev,
                        (step & 1) ? 1 : 2, false, s);
}

int lbm_adjoint_step_inplace_noalloc(lbm_plan *p, int64_t step, float *const *lam_host, float *const *rec_host,
                                     int32_t kind, int32_t n_slots, const double *const *pw_host,
                                     double *dJdtheta_dev, hipStream_t s)
{
    return adjoint_step(p, step, lam_host, lam_host, rec_host, kind, n_slots, pw_host, dJdtheta_dev,
                        (step & 1) ? 1 : 2, true, s);
}

int lbm_adjoint_init(lbm_plan *p, float *const *lam_out_host, const double *const *pw_host, hipStream_t s)
{
    int r = check_plan(p);
    if (r) return r;
    if (!lam_out_host || !pw_host) return fail(LBM_E_INVALID, "bad adjoint arguments");
    if (p->step & 1) return fail(LBM_E_INVALID, "the adjoint starts from an even step");
    for (int i = 0; i < p->n_inst; ++i)
        if (!lam_out_host[i]) return fail(LBM_E_INVALID, "instance %d: NULL adjoint buffer", i);
    AdjArgs a{};
    r = table_of(p, (float *const *)lam_out_host, (float ***)&a.lam_out);
    if (!r) r = table_of(p, (const double *const *)pw_host, (const double ***)&a.pw);
    if (r) return r;
    a.step = p->step;
    a.model = p->model;
    a.in_window = (p->avg_begin < p->step && p->step <= p->avg_end) ? 1 : 0;
    a.inv_count = p->avg_end > p->avg_begin ? 1.0 / (double)(p->avg_end - p->avg_begin) : 0.0;
    if (launch_adjoint_init(p->v.tile(), p->geo_d, p->tiles_d, p->n_tiles, a, s))
        return fail(LBM_E_HIP, "adjoint init launch failed");
    return LBM_OK;
}

int lbm_plan_variant(const lbm_plan *p, int32_t variant_out[4])
{
    if (!p || !variant_out) return fail(LBM_E_INVALID, "bad arguments");
    variant_out[0] = p->v.bs;
    variant_out[1] = p->v.cpt;
    variant_out[2] = p->v.nt;
    variant_out[3] = p->v.xcd;
    return LBM_OK;
}

int lbm_plan_autotune(lbm_plan *p, hipStream_t s, int32_t variant_out[4])
{
    int r = check_plan(p);
    if (r) return r;
    if (p->step & 1) return fail(LBM_E_INVALID, "autotune from an even step");
    const std::string key = tune_key(p);
    std::map<std::string, int> cache = read_tune_cache();
    auto it = cache.find(key);
    Variant best{0, 0, 0, 0};
    auto decode = [](int code) {
        return Variant{code & 0xffff, (code >> 16) & 0xf, (code >> 20) & 0xf, (code >> 24) & 0xf};
    };
    auto encode = [](const Variant &v) { return v.bs | (v.cpt << 16) | (v.nt << 20) | (v.xcd << 24); };
    if (it != cache.end() && variant_ok(decode(it->second))) {
        best = decode(it->second);
    } else {
        // save the populations, time step pairs for every launch shape, restore
        std::vector<size_t> bytes(p->n_inst);
        size_t total = 0;
        for (int i = 0; i < p->n_inst; ++i) total += (bytes[i] = sizeof(float) * 19 * (size_t)p->geo_h[i].qs);
        char *save = nullptr;
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipMalloc(&save, total));
        size_t off = 0;
        for (int i = 0; i < p->n_inst; ++i) {
            HIPCHK(hipMemcpyAsync(save + off, p->geo_h[i].f, bytes[i], hipMemcpyDeviceToDevice, s));
            off += bytes[i];
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const Variant saved = p->v;
        // time `pairs` step pairs (after two untimed ones) of shape v, in the
        // order plain stretches run: the whole batch per step, or with
        // instance blocks each block through its own pairs in turn (the
        // times of the blocks summed)
        auto time_pairs = [&](const Variant &v, int pairs, float &ms) -> int {
            p->v = v;
            int rc = build_tiles(p);
            if (rc) return rc;
            std::vector<std::pair<int32_t, int32_t>> ranges = p->blocks;
            if (ranges.empty()) ranges.push_back({0, p->n_tiles});
            StepArgs a{};
            a.step = p->steady_from + 2;
            a.tinfo = p->tinfo_d;
            ms = 0.f;
            for (const auto &rg : ranges) {
                a.tile_base = rg.first;
                for (int w = 0; w < 2 + pairs; ++w) {
                    if (w == 2) HIPCHK(hipEventRecord(e0, s));
                    launch_step(v, p->model, 0, p->geo_d, p->tiles_d, rg.second, a, p->health_d, s);
                    launch_step(v, p->model, 1, p->geo_d, p->tiles_d, rg.second, a, p->health_d, s);
                }
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                ms += t;
            }
            return 0;
        };
        // coarse pass over every shape, then the six fastest re-timed three
        // times each (interleaved) and ranked by their best time
        std::vector<std::pair<float, Variant>> coarse;
        for (int bs : {64, 128, 256, 512})
            for (int cpt : {1, 2, 4})
                for (int nt : {0, 1, 2, 3})
                    for (int xcd : {0, 1}) {
                        const Variant v{bs, cpt, nt, xcd};
                        float ms = 0.f;
                        if (!r) r = time_pairs(v, 4, ms);
                        coarse.push_back({ms, v});
                    }
        std::stable_sort(coarse.begin(), coarse.end(),
                         [](const std::pair<float, Variant> &x, const std::pair<float, Variant> &y) {
                             return x.first < y.first;
                         });
        const size_t n_fine = std::min<size_t>(6, coarse.size());
        std::vector<float> fine(n_fine, 1e30f);
        for (int rep = 0; rep < 3 && !r; ++rep)
            for (size_t k = 0; k < n_fine && !r; ++k) {
                float ms = 0.f;
                r = time_pairs(coarse[k].second, 8, ms);
                fine[k] = std::min(fine[k], ms);
            }
        float best_ms = 1e30f;
        for (size_t k = 0; k < n_fine; ++k)
            if (fine[k] < best_ms) {
                best_ms = fine[k];
                best = coarse[k].second;
            }
        if (!best.bs) best = saved;
        off = 0;
        for (int i = 0; i < p->n_inst; ++i) {
            HIPCHK(hipMemcpyAsync(p->geo_h[i].f, save + off, bytes[i], hipMemcpyDeviceToDevice, s));
            off += bytes[i];
        }
        HIPCHK(clear_i32(p->health_d, p->n_inst, s));
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(hipFree(save));
        HIPCHK(hipEventDestroy(e0));
        HIPCHK(hipEventDestroy(e1));
        if (r) return r;
        cache[key] = encode(best);
        write_tune_cache(cache);
    }
    p->v = best;
    r = build_tiles(p);
    if (r) return r;
    return lbm_plan_variant(p, variant_out);
}

}  // extern "C"

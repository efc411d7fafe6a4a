// lhf_batch.hip -- many independent vortex systems evaluated by one executable
// HIP graph, with a per-system octree depth chosen by a measured cost model.
//
// Systems that share a depth share one plan: their Morton keys carry the system
// index, so one sort, one tree build and one launch per phase and level cover all
// of them (no interaction list crosses systems).  Each group plan gathers the
// coordinates of its systems once at creation and afterwards indexes the caller's
// arrays directly (its permutation is rewritten to global element indices), so an
// execute needs no gather or scatter of its own.  The executes of all groups are
// captured once into a graph with one branch per group (up to four concurrent
// streams) and replayed by every later execute with the same array pointers.
//
// Depth selection follows the cost model of the paper's complexity analysis
// (Sec. 4.1, eqs. fmm2-fmm3): work = (far-field cost per box) x (boxes) + (near-field
// cost per pair) x (pairs), with both unit costs measured on the device by
// lhf_autotune, subject to the accuracy constraint of the core split (the leaf side
// must be wide enough that the singular far kernel is within tol of the Gaussian
// core, eq. vem1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "lhf_internal.h"

struct lhf_batch {
    lhf_desc desc;
    int nsys = 0;
    int64_t n = 0;
    std::vector<int32_t> sys_depth;
    std::vector<lhf_plan *> group;          // one plan per distinct depth, most costly first
    std::vector<double> group_cost;
    std::vector<hipStream_t> lanes;         // concurrent branches of the captured graph
    hipStream_t cap = nullptr;              // capture stream
    std::vector<hipEvent_t> ev;             // [0]: fork, [1 + k]: join of lane k
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_omega = nullptr;          // arrays the captured graph reads and writes
    void *g_v = nullptr, *g_s = nullptr;
    int warn = 0;
};

namespace lhf {

// K(r; a) of eq. vem1
static double core_kernel(double r, double a)
{
    return erf(r / (a * sqrt(2.0))) - sqrt(2.0 / M_PI) * (r / a) * exp(-r * r / (2.0 * a * a));
}

// expected non-empty boxes of level l for n uniform points in the cube
static double exp_boxes(int64_t n, int l)
{
    const double cells = ldexp(1.0, 3 * l);
    return cells * -expm1((double)n * log1p(-1.0 / cells));
}

// expected ordered near-field pairs (distinct elements in the same or adjacent
// leaves) for n uniform points at depth d: per axis a point's neighbourhood
// covers (3m - 2)/m^2 of the side on average, m = 2^d
static double exp_pairs(int64_t n, int d)
{
    const double m = ldexp(1.0, d);
    const double f = (3.0 * m - 2.0) / (m * m);
    return (double)n * (double)(n - 1) * f * f * f;
}

static double model_cost(const lhf_tune *t, int64_t n, int d)
{
    double boxes = 0.0;
    for (int l = 2; l <= d; l++) boxes += exp_boxes(n, l);
    return t->t_box_ns * boxes + t->t_pair_ns * exp_pairs(n, d);
}

static bool core_ok(double len, double a, double tol, int d)
{
    return !(a > 0.0) || 1.0 - core_kernel(len / ldexp(1.0, d), a) <= tol;
}

template <typename T>
__global__ void k_gather_rows(int64_t n, const T *__restrict__ x, const int32_t *__restrict__ gidx,
                              T *__restrict__ xg)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = gidx[i];
    xg[3 * i] = x[3 * o];
    xg[3 * i + 1] = x[3 * o + 1];
    xg[3 * i + 2] = x[3 * o + 2];
}

__global__ void k_remap(int64_t n, int32_t *__restrict__ perm, const int32_t *__restrict__ gidx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[i] = gidx[perm[i]];
}

static void batch_drop_graph(lhf_batch *B)
{
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->g_omega = nullptr;
    B->g_v = B->g_s = nullptr;
}

static void batch_free(lhf_batch *B)
{
    if (!B) return;
    batch_drop_graph(B);
    for (lhf_plan *P : B->group) plan_free(P);
    for (hipStream_t s : B->lanes) (void)hipStreamDestroy(s);
    if (B->cap) (void)hipStreamDestroy(B->cap);
    for (hipEvent_t e : B->ev) (void)hipEventDestroy(e);
    delete B;
}

// one plan over the systems 'sys' (ascending), all at depth d
static lhf_status group_plan(lhf_batch *B, const std::vector<int> &sys, int d, const int64_t *off, const void *x,
                             const double *lo, const double *len, const double *a, hipStream_t st, lhf_plan **out)
{
    const int ns = (int)sys.size();
    std::vector<int64_t> loff(ns + 1, 0);
    std::vector<double> glo(3 * (size_t)ns), glen(ns), ga(ns);
    for (int k = 0; k < ns; k++) {
        const int s = sys[k];
        loff[k + 1] = loff[k] + (off[s + 1] - off[s]);
        for (int c = 0; c < 3; c++) glo[3 * k + c] = lo[3 * s + c];
        glen[k] = len[s];
        ga[k] = a[s];
    }
    const int64_t ng = loff[ns];
    lhf_desc dd = B->desc;
    dd.depth = d;
    if (ng == 0) return arg_error("internal: empty depth group");
    if (ns == B->nsys) {
        // every system in one group: the caller's arrays are already in place
        return plan_new(out, &dd, ns, loff.data(), x, glo.data(), glen.data(), ga.data(), st);
    }
    std::vector<int32_t> gidx((size_t)ng);
    for (int k = 0; k < ns; k++)
        for (int64_t i = 0; i < off[sys[k] + 1] - off[sys[k]]; i++) gidx[loff[k] + i] = (int32_t)(off[sys[k]] + i);
    const size_t ts = B->desc.precision == LHF_FP64 ? 8 : 4;
    int32_t *dg = nullptr;
    void *xg = nullptr;
    hipError_t e = dev_malloc(&dg, sizeof(int32_t) * ng);
    if (e == hipSuccess) e = dev_malloc(&xg, ts * 3 * ng);
    if (e == hipSuccess) e = hipMemcpyAsync(dg, gidx.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const unsigned nb = (unsigned)((ng + 255) / 256);
        if (ts == 8)
            hipLaunchKernelGGL(k_gather_rows<double>, dim3(nb), dim3(256), 0, st, ng, (const double *)x, dg,
                               (double *)xg);
        else
            hipLaunchKernelGGL(k_gather_rows<float>, dim3(nb), dim3(256), 0, st, ng, (const float *)x, dg,
                               (float *)xg);
        e = hipGetLastError();
    }
    lhf_status rs = LHF_OK;
    if (e == hipSuccess) {
        rs = plan_new(out, &dd, ns, loff.data(), xg, glo.data(), glen.data(), ga.data(), st);
        if (rs >= 0) {
            hipLaunchKernelGGL(k_remap, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, ng, (*out)->perm, dg);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(st);
        }
    }
    if (dg) (void)dev_free(dg);
    if (xg) (void)dev_free(xg);
    if (e != hipSuccess) {
        if (*out) plan_free(*out);
        *out = nullptr;
        return hip_fail(e, "batch group construction");
    }
    return rs;
}

static lhf_status batch_capture(lhf_batch *B, const void *omega, void *v, void *s)
{
    batch_drop_graph(B);
    const int K = (int)B->lanes.size();
    LHF_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    lhf_status rs = LHF_OK;
    hipError_t e = hipEventRecord(B->ev[0], B->cap);
    for (int k = 0; k < K && e == hipSuccess; k++) e = hipStreamWaitEvent(B->lanes[k], B->ev[0], 0);
    for (size_t g = 0; g < B->group.size() && e == hipSuccess && rs >= 0; g++)
        {
            lhf_io io;
            memset(&io, 0, sizeof(io));
            io.omega = omega;
            io.v = v;
            io.s = s;
            io.what = 3;
            rs = execute_impl(B->group[g], &io, B->lanes[g % K]);
        }
    for (int k = 0; k < K && e == hipSuccess; k++) {
        e = hipEventRecord(B->ev[1 + k], B->lanes[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(B->cap, B->ev[1 + k], 0);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(B->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess || rs < 0) {
        if (g) (void)hipGraphDestroy(g);
        if (rs < 0) return rs;
        return hip_fail(e != hipSuccess ? e : e2, "batch graph capture");
    }
    B->graph = g;
    e = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        batch_drop_graph(B);
        return hip_fail(e, "hipGraphInstantiate");
    }
    B->g_omega = omega;
    B->g_v = v;
    B->g_s = s;
    return LHF_OK;
}

// unit costs of the cost model, measured on the current device
static lhf_status measure_tune(int32_t p, int32_t precision, hipStream_t st, lhf_tune *out)
{
    const int64_t n = (int64_t)1 << 17;
    const size_t ts = precision == LHF_FP64 ? 8 : 4;
    // uniform points and strengths from splitmix64 (fixed seed)
    std::vector<double> hx(3 * n), hw(3 * n);
    uint64_t z = 0x5eed5eed5eedull;
    auto next = [&]() {
        z += 0x9e3779b97f4a7c15ull;
        uint64_t r = z;
        r = (r ^ (r >> 30)) * 0xbf58476d1ce4e5b9ull;
        r = (r ^ (r >> 27)) * 0x94d049bb133111ebull;
        r ^= r >> 31;
        return (double)(r >> 11) * 0x1.0p-53;
    };
    for (int64_t i = 0; i < 3 * n; i++) hx[i] = next();
    for (int64_t i = 0; i < 3 * n; i++) hw[i] = next() - 0.5;
    std::vector<float> fx, fw;
    const void *px = hx.data(), *pw = hw.data();
    if (ts == 4) {
        fx.assign(hx.begin(), hx.end());
        fw.assign(hw.begin(), hw.end());
        px = fx.data();
        pw = fw.data();
    }
    void *dx = nullptr, *dw = nullptr, *dv = nullptr, *ds = nullptr;
    hipError_t e = dev_malloc(&dx, ts * 3 * n);
    if (e == hipSuccess) e = dev_malloc(&dw, ts * 3 * n);
    if (e == hipSuccess) e = dev_malloc(&dv, ts * 3 * n);
    if (e == hipSuccess) e = dev_malloc(&ds, ts * 3 * n);
    if (e == hipSuccess) e = hipMemcpyAsync(dx, px, ts * 3 * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dw, pw, ts * 3 * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    lhf_status rs = e == hipSuccess ? LHF_OK : hip_fail(e, "autotune buffers");
    double far_ns_per_box = 0.0, near_ns_per_pair = 0.0;
    // far-field unit cost from depth 5 (far work dominates), near-field from depth 3
    const int depths[2] = {5, 3};
    for (int k = 0; k < 2 && rs >= 0; k++) {
        lhf_desc d;
        lhf_desc_default(&d);
        d.p = p;
        d.precision = precision;
        d.depth = depths[k];
        d.flags = LHF_SINGULAR;
        lhf_plan *P = nullptr;
        rs = lhf_plan_create(&P, &d, n, dx, 0.0, st);
        if (rs < 0) break;
        for (int w = 0; w < 2 && rs >= 0; w++) rs = lhf_execute(P, dw, dv, ds, nullptr, st);
        if (rs >= 0) rs = lhf_profile_begin(P, 3);
        for (int w = 0; w < 3 && rs >= 0; w++) rs = lhf_execute(P, dw, dv, ds, nullptr, st);
        double ph[LHF_NPHASE];
        int32_t ne = 0;
        if (rs >= 0) rs = lhf_profile_end(P, ph, &ne);
        lhf_stats S;
        if (rs >= 0) rs = lhf_plan_stats(P, &S);
        if (rs >= 0 && ne > 0) {
            double boxes = 0.0;
            for (int l = 2; l <= d.depth; l++) boxes += (double)S.boxes[l];
            const double far_ms = (ph[1] + ph[2] + ph[3] + ph[4]) / ne;
            const double near_ms = ph[5] / ne;
            if (k == 0) far_ns_per_box = 1e6 * far_ms / std::max(boxes, 1.0);
            else near_ns_per_pair = 1e6 * near_ms / std::max((double)S.n_p2p_pairs, 1.0);
        }
        lhf_status dr = lhf_plan_destroy(P);
        if (rs >= 0 && dr < 0) rs = dr;
    }
    (void)hipStreamSynchronize(st);
    for (void *b : {dx, dw, dv, ds})
        if (b) (void)dev_free(b);
    if (rs < 0) return rs;
    out->p = p;
    out->precision = precision;
    out->t_box_ns = far_ns_per_box;
    out->t_pair_ns = near_ns_per_pair;
    return LHF_OK;
}

static std::string tune_key(int32_t p, int32_t precision)
{
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    return arch + "/" + (precision == LHF_FP64 ? "fp64" : "fp32") + "/p" + std::to_string(p);
}

struct TuneEntry {
    std::string key;
    double t_box, t_pair;
};

// cache file: a JSON array with one object per line
//   [
//    {"key": "gfx950/fp32/p10", "t_box_ns": 123.4, "t_pair_ns": 0.0123},
//   ]
static std::vector<TuneEntry> read_cache(const char *path)
{
    std::vector<TuneEntry> v;
    FILE *f = fopen(path, "r");
    if (!f) return v;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        char key[128];
        double a = 0, b = 0;
        if (sscanf(line, " {\"key\": \"%127[^\"]\", \"t_box_ns\": %lf, \"t_pair_ns\": %lf}", key, &a, &b) == 3)
            v.push_back({key, a, b});
    }
    fclose(f);
    return v;
}

static bool write_cache(const char *path, const std::vector<TuneEntry> &v)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "[\n");
    for (size_t i = 0; i < v.size(); i++)
        fprintf(f, " {\"key\": \"%s\", \"t_box_ns\": %.9g, \"t_pair_ns\": %.9g}%s\n", v[i].key.c_str(), v[i].t_box,
                v[i].t_pair, i + 1 < v.size() ? "," : "");
    fprintf(f, "]\n");
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace lhf

using namespace lhf;

extern "C" {

void lhf_tune_default(int32_t p, int32_t precision, lhf_tune *t)
{
    if (!t) return;
    // unit costs measured with this library on MI355X (uniform cubes, FP32 at p = 10,
    // FP64 at p = 12), scaled to other p by the p^3 work of a rotation-based M2L
    const double q = (double)p * p * p;
    t->p = p;
    t->precision = precision;
    t->t_box_ns = precision == LHF_FP64 ? 430.0 * q / 1728.0 : 330.0 * q / 1000.0;
    t->t_pair_ns = precision == LHF_FP64 ? 0.012 : 0.0042;
}

lhf_status lhf_autotune(int32_t p, int32_t precision, const char *cache_path, lhf_tune *out, void *stream)
{
    if (!out) return arg_error("out is NULL");
    if (precision != LHF_FP64 && precision != LHF_FP32) return arg_error("unknown precision");
    if (p < 1 || p > (precision == LHF_FP64 ? MAXP : 16)) return arg_error("p out of range");
    const std::string key = tune_key(p, precision);
    std::vector<TuneEntry> cache;
    if (cache_path && cache_path[0]) {
        cache = read_cache(cache_path);
        for (const TuneEntry &c : cache)
            if (c.key == key) {
                out->p = p;
                out->precision = precision;
                out->t_box_ns = c.t_box;
                out->t_pair_ns = c.t_pair;
                return LHF_OK;
            }
    }
    lhf_status rs = measure_tune(p, precision, (hipStream_t)stream, out);
    if (rs < 0) return rs;
    if (cache_path && cache_path[0]) {
        cache.push_back({key, out->t_box_ns, out->t_pair_ns});
        if (!write_cache(cache_path, cache)) {
            set_error(std::string("could not write the autotune cache ") + cache_path);
            return LHF_ERR_ARG;
        }
    }
    return LHF_OK;
}

lhf_status lhf_choose_depth(const lhf_tune *t, int64_t n, double len, double a, double tol, int32_t *depth)
{
    if (!t || !depth) return arg_error("tune and depth must be non-NULL");
    if (n < 0) return arg_error("n must be >= 0");
    if (!(len > 0.0) || !isfinite(len) || !(a >= 0.0) || !isfinite(a) || !(tol > 0.0))
        return arg_error("len > 0, a >= 0 and tol > 0 must be finite");
    if (!(t->t_box_ns > 0.0) || !(t->t_pair_ns > 0.0)) return arg_error("unit costs must be > 0");
    int best = 2;
    double best_c = INFINITY;
    bool any = false;
    for (int d = 2; d <= 8; d++) {
        if (!core_ok(len, a, tol, d)) continue;
        const double c = model_cost(t, n, d);
        if (!any || c < best_c) {
            best = d;
            best_c = c;
        }
        any = true;
    }
    *depth = best;
    return any ? LHF_OK : LHF_WARN_CORE_SPLIT;
}

lhf_status lhf_batch_create(lhf_batch **out, const lhf_desc *d, int32_t n_systems, const int64_t *sys_offsets,
                            const void *x, const double *sys_lo, const double *sys_len, const double *sys_a,
                            const int32_t *sys_depth, const lhf_tune *tune, void *stream)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (!d) return arg_error("desc is NULL");
    if (n_systems < 1) return arg_error("n_systems must be >= 1");
    if (!sys_offsets || !sys_lo || !sys_len || !sys_a || !x) return arg_error("arrays must be non-NULL");
    if (sys_offsets[0] != 0) return arg_error("sys_offsets[0] must be 0");
    for (int s = 0; s < n_systems; s++) {
        if (sys_offsets[s + 1] < sys_offsets[s]) return arg_error("sys_offsets must be non-decreasing");
        if (!(sys_len[s] > 0.0) || !isfinite(sys_len[s]) || !(sys_a[s] >= 0.0) || !isfinite(sys_a[s]))
            return arg_error("cube sides must be > 0 and core radii >= 0, all finite");
        if (sys_depth && (sys_depth[s] < 2 || sys_depth[s] > MAXDEPTH)) return arg_error("sys_depth out of 2..10");
    }
    const int64_t n = sys_offsets[n_systems];
    if (n < 1) return arg_error("the systems hold no elements");
    if (n > (int64_t)0x7fffffff) return arg_error("total n must fit in int32");
    lhf_tune tdef;
    if (!tune) {
        lhf_tune_default(d->p, d->precision, &tdef);
        tune = &tdef;
    }
    lhf_batch *B = new lhf_batch();
    B->desc = *d;
    B->nsys = n_systems;
    B->n = n;
    B->sys_depth.resize(n_systems);
    // depth of each system, then one group per depth (empty systems join any group)
    std::vector<std::vector<int>> by_depth(MAXDEPTH + 1);
    std::vector<double> cost(MAXDEPTH + 1, 0.0);
    for (int s = 0; s < n_systems; s++) {
        const int64_t ns = sys_offsets[s + 1] - sys_offsets[s];
        int32_t dep = 0;
        if (sys_depth) dep = sys_depth[s];
        else {
            const double as = (d->flags & LHF_SINGULAR) ? 0.0 : sys_a[s];
            lhf_status cs = lhf_choose_depth(tune, ns, sys_len[s], as, d->tol, &dep);
            if (cs < 0) {
                batch_free(B);
                return cs;
            }
        }
        B->sys_depth[s] = dep;
        by_depth[dep].push_back(s);
        cost[dep] += model_cost(tune, ns, dep);
    }
    std::vector<int> order;
    for (int dep = 2; dep <= MAXDEPTH; dep++)
        if (!by_depth[dep].empty()) {
            int64_t cnt = 0;
            for (int s : by_depth[dep]) cnt += sys_offsets[s + 1] - sys_offsets[s];
            if (cnt > 0) order.push_back(dep);
        }
    // a group with no elements folds into the first non-empty one
    for (int dep = 2; dep <= MAXDEPTH; dep++) {
        if (by_depth[dep].empty() || std::find(order.begin(), order.end(), dep) != order.end()) continue;
        for (int s : by_depth[dep]) {
            by_depth[order[0]].push_back(s);
            B->sys_depth[s] = order[0];
        }
        by_depth[dep].clear();
    }
    std::sort(order.begin(), order.end(), [&](int u, int w) { return cost[u] > cost[w]; });
    hipStream_t st = (hipStream_t)stream;
    lhf_status rs = LHF_OK;
    for (int dep : order) {
        std::vector<int> sys = by_depth[dep];
        std::sort(sys.begin(), sys.end());
        lhf_plan *P = nullptr;
        lhf_status gs = group_plan(B, sys, dep, sys_offsets, x, sys_lo, sys_len, sys_a, st, &P);
        if (gs < 0) {
            batch_free(B);
            return gs;
        }
        if (gs > 0) rs = gs;
        B->group.push_back(P);
        B->group_cost.push_back(cost[dep]);
    }
    const int K = std::min<int>(4, (int)B->group.size());
    B->ev.resize(1 + K, nullptr);
    hipError_t e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
    for (int k = 0; k < K && e == hipSuccess; k++) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) B->lanes.push_back(s);
    }
    for (int k = 0; k <= K && e == hipSuccess; k++) e = hipEventCreateWithFlags(&B->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_free(B);
        return hip_fail(e, "batch streams");
    }
    B->warn = rs;
    *out = B;
    return rs;
}

lhf_status lhf_batch_execute(lhf_batch *B, const void *omega, void *v, void *s, int32_t use_graph, void *stream)
{
    if (!B) return arg_error("batch is NULL");
    if (!omega || !v || !s) return arg_error("omega, v and s must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) {
        for (lhf_plan *P : B->group) {
            lhf_io io;
            memset(&io, 0, sizeof(io));
            io.omega = omega;
            io.v = v;
            io.s = s;
            io.what = 3;
            lhf_status rs = execute_impl(P, &io, st);
            if (rs < 0) return rs;
        }
        return LHF_OK;
    }
    if (!B->exec || B->g_omega != omega || B->g_v != v || B->g_s != s) {
        lhf_status rs = batch_capture(B, omega, v, s);
        if (rs < 0) return rs;
    }
    LHF_HIP(hipGraphLaunch(B->exec, st));
    return LHF_OK;
}

lhf_status lhf_batch_info(const lhf_batch *B, int32_t *n_groups, int32_t *sys_depth, lhf_stats *total)
{
    if (!B) return arg_error("batch is NULL");
    if (n_groups) *n_groups = (int32_t)B->group.size();
    if (sys_depth)
        for (int s = 0; s < B->nsys; s++) sys_depth[s] = B->sys_depth[s];
    if (total) {
        memset(total, 0, sizeof(*total));
        total->n = B->n;
        total->p = B->desc.p;
        for (lhf_plan *P : B->group) {
            lhf_stats S;
            lhf_status rs = lhf_plan_stats(P, &S);
            if (rs < 0) return rs;
            total->depth = std::max(total->depth, S.depth);
            for (int l = 0; l <= S.depth; l++) total->boxes[l] += S.boxes[l];
            total->n_m2l += S.n_m2l;
            total->n_m2m += S.n_m2m;
            total->n_l2l += S.n_l2l;
            total->n_p2p_pairs += S.n_p2p_pairs;
            total->n_theta_classes = std::max(total->n_theta_classes, S.n_theta_classes);
        }
    }
    return LHF_OK;
}

lhf_status lhf_batch_destroy(lhf_batch *B)
{
    if (!B) return LHF_OK;
    hipError_t e = hipSuccess;
    for (hipStream_t s : B->lanes) {
        hipError_t e1 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e1;
    }
    for (lhf_plan *P : B->group) {
        hipError_t e1 = hipStreamSynchronize(P->stream);
        if (e == hipSuccess) e = e1;
    }
    batch_free(B);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return LHF_OK;
}

}  // extern "C"

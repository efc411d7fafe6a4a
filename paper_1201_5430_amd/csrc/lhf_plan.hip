// lhf_plan.hip -- plan construction and the C ABI of liblhfmm.
//
// Plan = the paper's "FMM set" stage (Sec. 4, table of modifications: data
// structure and translation precomputation, unchanged from the scalar FMM):
//   1. integer coordinates and Morton keys (FP64), stable radix sort
//   2. non-empty boxes of every level, parent / child links
//   3. interaction lists: V (M2L, children of the parent's neighbours that are
//      not adjacent, <= 189 per box) and U (adjacent leaves, near field)
//   4. operator tables in FP64 on the device: rotation matrices per polar
//      angle class, z phases per direction, coaxial M2L coefficients
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <math.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <numeric>
#include <string>
#include <vector>

#include "lhf_internal.h"

namespace lhf {

lhf_status execute_impl(lhf_plan *P, const lhf_io *io, hipStream_t st);
lhf_status autotune_impl(lhf_plan *P, const void *omega, int *ns, int *ts, hipStream_t st);
int m2l_quarter_max_ns(int p);
bool m2l_tile_supported(int precision, int p);
void dmap_build(const lhf_plan *Pl, int level, hipStream_t st);
bool wpad_build(lhf_plan *Pl, hipStream_t st);
bool m2l_mfma_supported(int precision, int p);
bool m2l_half_supported(int precision, int p);
bool whalf_build(lhf_plan *Pl, hipStream_t st);
bool mmhalf_build(lhf_plan *Pl, hipStream_t st);
bool wmfma_build(lhf_plan *Pl, hipStream_t st);

bool m2l_tile_owned(int precision, int p);
bool m2l_half_owned(int precision, int p);
bool m2l_quarter_supported(int precision, int p);
bool wquarter_build(lhf_plan *Pl, hipStream_t st);
bool mm_half_supported(int precision, int p);
bool mm_quarter_supported(int precision, int p);
bool m2l_qmfma_supported(int precision, int p);
int m2l_qmfma_max_ns(int p);
bool qmfma_build(lhf_plan *Pl, hipStream_t st);
bool mmquarter_build(lhf_plan *Pl, hipStream_t st);

// ---- device memory cache -----------------------------------------------------------------
namespace {
struct MemCache {
    std::mutex mu;
    std::map<std::pair<size_t, int>, std::vector<void *>> idle;  // (bytes, device) -> free blocks
    std::unordered_map<void *, std::pair<size_t, int>> live;     // block -> (bytes, device)
    size_t idle_bytes = 0;
};
MemCache &mem_cache()
{
    static MemCache *m = new MemCache();  // lives as long as the process
    return *m;
}
bool mem_cache_on()
{
    static const bool on = getenv("LHF_NO_MEMCACHE") == nullptr;
    return on;
}
// idle bytes kept at most (LHF_MEMCACHE_GB, default 16 GiB of the 288 GB)
size_t mem_cache_cap()
{
    static const size_t cap = [] {
        const char *e = getenv("LHF_MEMCACHE_GB");
        const double gb = e ? atof(e) : 16.0;
        return (size_t)(std::max(0.0, gb) * 1073741824.0);
    }();
    return cap;
}
size_t round_block(size_t b)
{
    const size_t small = 512, large = (size_t)2 << 20;
    b = std::max<size_t>(b, 1);
    return b < ((size_t)1 << 20) ? (b + small - 1) / small * small : (b + large - 1) / large * large;
}
// release idle blocks (of one device, or of all with dev < 0), largest first, until at most keep
// bytes stay idle: a later reallocation costs one call per block whatever its size, so the cap
// is met with the fewest blocks given back, and the many small blocks of small plans stay
void mem_trim_locked(MemCache &m, int dev, size_t keep)
{
    for (auto it = m.idle.end(); it != m.idle.begin() && m.idle_bytes > keep;) {
        --it;
        if (dev >= 0 && it->first.second != dev) continue;
        while (!it->second.empty() && m.idle_bytes > keep) {
            (void)hipFree(it->second.back());
            it->second.pop_back();
            m.idle_bytes -= it->first.first;
        }
        if (it->second.empty()) it = m.idle.erase(it);
    }
}
}  // namespace

// ---- allocation-free evaluation: a bump arena over a fixed device array ----------------------
// While a thread runs lhf_evaluate_noalloc, every device block of its plan (and every temporary
// of the plan's construction) is carved from that call's arena instead of hipMalloc; freeing
// such a block is a no-op.  The arena's memory is the file-scope array 'scratch' below.
namespace {
struct Arena {
    char *base = nullptr;
    size_t cap = 0, off = 0;
    size_t need = 0;       // bytes the plan asked for when the arena ran out (0: it did not)
};
thread_local Arena *t_arena = nullptr;
}  // namespace

hipError_t dev_malloc_raw(void **p, size_t bytes)
{
    if (t_arena) {
        const size_t at = (t_arena->off + 255) & ~(size_t)255;
        if (at + bytes > t_arena->cap) {
            t_arena->need = at + bytes;
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
        *p = t_arena->base + at;
        t_arena->off = at + bytes;
        return hipSuccess;
    }
    if (!mem_cache_on()) return hipMalloc(p, bytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t rb = round_block(bytes);
    MemCache &m = mem_cache();
    {
        std::lock_guard<std::mutex> lk(m.mu);
        auto it = m.idle.find({rb, dev});
        if (it != m.idle.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            m.idle_bytes -= rb;
            m.live[*p] = {rb, dev};
            return hipSuccess;
        }
    }
    e = hipMalloc(p, rb);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> lk(m.mu);
        mem_trim_locked(m, dev, 0);
        e = hipMalloc(p, rb);
    }
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(m.mu);
        m.live[*p] = {rb, dev};
    }
    return e;
}

hipError_t dev_free(void *p)
{
    if (!p) return hipSuccess;
    if (t_arena && (char *)p >= t_arena->base && (char *)p < t_arena->base + t_arena->cap) return hipSuccess;
    if (!mem_cache_on()) return hipFree(p);
    MemCache &m = mem_cache();
    std::lock_guard<std::mutex> lk(m.mu);
    auto it = m.live.find(p);
    if (it == m.live.end()) return hipFree(p);
    const auto key = it->second;
    m.live.erase(it);
    m.idle[key].push_back(p);
    m.idle_bytes += key.first;
    if (m.idle_bytes > mem_cache_cap()) mem_trim_locked(m, -1, mem_cache_cap());
    return hipSuccess;
}

static thread_local std::string g_err = "no error";

void set_error(const std::string &msg) { g_err = msg; }

lhf_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string("HIP error ") + hipGetErrorString(e) + " in " + what);
    return LHF_ERR_HIP;
}

lhf_status arg_error(const std::string &msg)
{
    set_error(msg);
    return LHF_ERR_ARG;
}

// ---------------------------------------------------------------------------
// tree kernels
// ---------------------------------------------------------------------------
__device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
__device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// flags: [0] = element outside its cube, [1] = non-finite coordinate.
// System s of element i: sys_off[s] <= i < sys_off[s+1]; its cube is sys_geo[4s..4s+3] =
// (lo0, lo1, lo2, L).  The key is (s << 3 depth) | Morton(q >> (21 - depth)).
template <typename T>
__global__ void k_keys(int64_t n, const T *__restrict__ x, int nsys, const int64_t *__restrict__ sys_off,
                       const double *__restrict__ sys_geo, int depth, uint64_t *__restrict__ key,
                       int32_t *__restrict__ idx, int32_t *__restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo_s = 0, hi_s = nsys - 1;  // last s with sys_off[s] <= i
    while (lo_s < hi_s) {
        const int mid = (lo_s + hi_s + 1) >> 1;
        if (sys_off[mid] <= i) lo_s = mid;
        else hi_s = mid - 1;
    }
    const int s = lo_s;
    const double *g = sys_geo + 4 * s;
    const double scale = (double)(1u << QBITS) / g[3];
    uint32_t q[3];
    const double qmax = (double)((1u << QBITS) - 1u);
    for (int d = 0; d < 3; d++) {
        const double xv = (double)x[3 * i + d];
        if (!isfinite(xv)) {
            atomicOr(&flags[1], 1);
            q[d] = 0;
            continue;
        }
        const double t = (xv - g[d]) * scale;  // one rounding each: no contraction possible
        if (t < 0.0 || t > (double)(1u << QBITS)) atomicOr(&flags[0], 1);
        double f = floor(t);
        f = fmin(fmax(f, 0.0), qmax);
        q[d] = (uint32_t)f;
    }
    const int sh = QBITS - depth;
    key[i] = ((uint64_t)s << (3 * depth)) | spread3(q[0] >> sh) | (spread3(q[1] >> sh) << 1) |
             (spread3(q[2] >> sh) << 2);
    idx[i] = (int32_t)i;
}

template <typename T>
__global__ void k_gather_x(int64_t n, const T *__restrict__ x, const int32_t *__restrict__ perm, T *__restrict__ xs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    xs[i] = x[3 * o];
    xs[n + i] = x[3 * o + 1];
    xs[2 * n + i] = x[3 * o + 2];
}

__global__ void k_level_flags(int64_t n, const uint64_t *__restrict__ skey, int sh, int32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (skey[i] >> sh) != (skey[i - 1] >> sh)) ? 1 : 0;
}

// id: inclusive scan of flags (1-based box id per element)
__global__ void k_level_fill(int64_t n, const uint64_t *__restrict__ skey, int sh, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ id, uint64_t *__restrict__ key, int32_t *__restrict__ start,
                             int32_t *__restrict__ eleaf, int64_t *__restrict__ nb_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = id[i] - 1;
    if (flag[i]) {
        key[b] = skey[i] >> sh;
        start[b] = (int32_t)i;
    }
    if (eleaf) eleaf[i] = b;
    if (i == n - 1) *nb_out = id[i];
}

__global__ void k_counts(int64_t nb, int64_t n, const int32_t *__restrict__ start, int32_t *__restrict__ count)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    count[b] = (int32_t)((b + 1 < nb ? (int64_t)start[b + 1] : n) - start[b]);
}

__device__ inline int64_t lower_bound_u64(const uint64_t *a, int64_t len, uint64_t k)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ inline int64_t find_u64(const uint64_t *a, int64_t len, uint64_t k)
{
    int64_t i = lower_bound_u64(a, len, k);
    return (i < len && a[i] == k) ? i : -1;
}

struct LevelTab {
    int64_t off[MAXDEPTH + 2];
    int64_t nb[MAXDEPTH + 2];
};

// parent / children links for all boxes
__global__ void k_links(int64_t nbox, int depth, LevelTab lt, const uint64_t *__restrict__ bkey,
                        int32_t *__restrict__ parent, int32_t *__restrict__ child0, int32_t *__restrict__ nchild)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int l = 0;
    while (l < depth && b >= lt.off[l + 1]) l++;
    const uint64_t k = bkey[b];
    if (l == 0) parent[b] = -1;
    else parent[b] = (int32_t)(lt.off[l - 1] + find_u64(bkey + lt.off[l - 1], lt.nb[l - 1], k >> 3));
    if (l == depth) {
        child0[b] = -1;
        nchild[b] = 0;
    } else {
        const uint64_t *ck = bkey + lt.off[l + 1];
        int64_t f = lower_bound_u64(ck, lt.nb[l + 1], k << 3);
        int64_t e = lower_bound_u64(ck, lt.nb[l + 1], (k << 3) + 8);
        child0[b] = (int32_t)(lt.off[l + 1] + f);
        nchild[b] = (int32_t)(e - f);
    }
}

// V-list of every box at levels >= 2 (fixed stride VMAX), for the generic per-box M2L (the
// batched kernels derive the lists from the dense box maps themselves)
__global__ void k_vlist(int64_t off, int64_t nb, int level, const uint64_t *__restrict__ bkey,
                        int32_t *__restrict__ vcount, int32_t *__restrict__ vsrc, int16_t *__restrict__ vdir)
{
    const int64_t bl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bl >= nb) return;
    const int64_t b = off + bl;
    const uint64_t kfull = bkey[b];
    const uint64_t sys = kfull >> (3 * level), k = kfull & ((1ull << (3 * level)) - 1);
    const int ix = (int)compact3(k), iy = (int)compact3(k >> 1), iz = (int)compact3(k >> 2);
    const int px = ix >> 1, py = iy >> 1, pz = iz >> 1;
    const int side = 1 << level;
    const uint64_t *lk = bkey + off;
    int cnt = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++)
                for (int c = 0; c < 8; c++) {
                    const int cx = 2 * (px + dx) + (c & 1), cy = 2 * (py + dy) + ((c >> 1) & 1),
                              cz = 2 * (pz + dz) + ((c >> 2) & 1);
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= side || cy >= side || cz >= side) continue;
                    const int ex = ix - cx, ey = iy - cy, ez = iz - cz;
                    if (abs(ex) <= 1 && abs(ey) <= 1 && abs(ez) <= 1) continue;
                    const uint64_t ck = (sys << (3 * level)) | spread3((uint32_t)cx) | (spread3((uint32_t)cy) << 1) |
                                        (spread3((uint32_t)cz) << 2);
                    const int64_t j = find_u64(lk, nb, ck);
                    if (j < 0) continue;
                    if (vsrc) {
                        vsrc[b * VMAX + cnt] = (int32_t)(off + j);
                        vdir[b * VMAX + cnt] = (int16_t)((ex + 3) + 7 * (ey + 3) + 49 * (ez + 3));  // t = c_T - c_S
                    }
                    cnt++;
                }
    vcount[b] = cnt;
}

// V-list counts from the dense box map of the level (batched-M2L plans, which build the maps
// anyway): the same walk as k_vlist with one map lookup per candidate instead of a search
__global__ void k_vcount_map(int64_t off, int64_t nb, int level, const uint64_t *__restrict__ bkey,
                             const int32_t *__restrict__ dmap, int32_t *__restrict__ vcount)
{
    const int64_t bl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bl >= nb) return;
    const int64_t b = off + bl;
    const uint64_t kfull = bkey[b];
    const uint64_t sys = kfull >> (3 * level), k = kfull & ((1ull << (3 * level)) - 1);
    const int ix = (int)compact3(k), iy = (int)compact3(k >> 1), iz = (int)compact3(k >> 2);
    const int px = ix >> 1, py = iy >> 1, pz = iz >> 1;
    const int side = 1 << level;
    const int32_t *map = dmap + (size_t)sys * side * side * side;
    int cnt = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++)
                for (int c = 0; c < 8; c++) {
                    const int cx = 2 * (px + dx) + (c & 1), cy = 2 * (py + dy) + ((c >> 1) & 1),
                              cz = 2 * (pz + dz) + ((c >> 2) & 1);
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= side || cy >= side || cz >= side) continue;
                    if (abs(ix - cx) <= 1 && abs(iy - cy) <= 1 && abs(iz - cz) <= 1) continue;
                    cnt += map[((size_t)cz * side + cy) * side + cx] >= 0;
                }
    vcount[b] = cnt;
}

// U-list (adjacent leaves incl. self) of every leaf, 27 slots
__global__ void k_ulist(int64_t off, int64_t nb, int level, const uint64_t *__restrict__ bkey,
                        const int32_t *__restrict__ bcount, int32_t *__restrict__ ulist, int64_t *__restrict__ npairs)
{
    const int64_t bl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bl >= nb) return;
    const uint64_t kfull = bkey[off + bl];
    const uint64_t sys = kfull >> (3 * level), k = kfull & ((1ull << (3 * level)) - 1);
    const int ix = (int)compact3(k), iy = (int)compact3(k >> 1), iz = (int)compact3(k >> 2);
    const int side = 1 << level;
    const uint64_t *lk = bkey + off;
    int q = 0;
    int64_t src = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int cx = ix + dx, cy = iy + dy, cz = iz + dz;
                int32_t val = -1;
                if (cx >= 0 && cy >= 0 && cz >= 0 && cx < side && cy < side && cz < side) {
                    const uint64_t ck = (sys << (3 * level)) | spread3((uint32_t)cx) | (spread3((uint32_t)cy) << 1) |
                                        (spread3((uint32_t)cz) << 2);
                    const int64_t j = find_u64(lk, nb, ck);
                    if (j >= 0) {
                        val = (int32_t)(off + j);
                        src += bcount[off + j];
                    }
                }
                ulist[bl * 27 + q++] = val;
            }
    const int64_t me = bcount[off + bl];
    atomicAdd((unsigned long long *)npairs, (unsigned long long)(me * src - me));
}

__global__ void k_sum_i32(int64_t n, const int32_t *__restrict__ a, int64_t *__restrict__ out)
{
    __shared__ int64_t sh[256];
    int64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)out, (unsigned long long)sh[0]);
}

__global__ void k_add_i32(int64_t n, int32_t *__restrict__ a, int32_t add)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += add;
}

// ---------------------------------------------------------------------------
// adaptive tree.  A box belongs to the tree iff it is a root or its parent holds
// more than maxleaf elements; it is a leaf iff it belongs and holds at most maxleaf
// elements or sits on the deepest level D.  Built from the full set of non-empty
// boxes of every level (the uniform levels of the sorted keys).
// ---------------------------------------------------------------------------

// keep flag of each non-empty box of level l (cap entries, nb[l] of them valid);
// leaves are counted per level
__global__ void k_akeep(int64_t cap, int l, int D, int64_t maxleaf, int64_t n, const int64_t *__restrict__ dnb,
                        const uint64_t *__restrict__ key, const int32_t *__restrict__ start,
                        const uint64_t *__restrict__ pkey, const int32_t *__restrict__ pstart,
                        int32_t *__restrict__ flag, int64_t *__restrict__ nleaf)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cap) return;
    const int64_t nb = dnb[l];
    if (b >= nb) {
        flag[b] = 0;
        return;
    }
    const int64_t cnt = (b + 1 < nb ? (int64_t)start[b + 1] : n) - start[b];
    int keep = 1;
    if (l > 0) {
        const int64_t pnb = dnb[l - 1];
        const int64_t pb = find_u64(pkey, pnb, key[b] >> 3);
        const int64_t pcnt = (pb + 1 < pnb ? (int64_t)pstart[pb + 1] : n) - pstart[pb];
        keep = pcnt > maxleaf;
    }
    flag[b] = keep;
    if (keep && (cnt <= maxleaf || l == D)) atomicAdd((unsigned long long *)(nleaf + l), 1ull);
}

__global__ void k_last_i32(int64_t len, const int32_t *__restrict__ a, int64_t *__restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = len > 0 ? (int64_t)a[len - 1] : 0;
}

// kept boxes of level l into the global box arrays (kid: inclusive scan of the keep flags)
__global__ void k_acompact(int64_t cap, int l, int64_t n, const int64_t *__restrict__ dnb,
                           const int32_t *__restrict__ kid, const uint64_t *__restrict__ key,
                           const int32_t *__restrict__ start, uint64_t *__restrict__ okey,
                           int32_t *__restrict__ ostart, int32_t *__restrict__ ocount)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cap) return;
    const int64_t nb = dnb[l];
    if (b >= nb) return;
    const int prev = b > 0 ? kid[b - 1] : 0;
    if (kid[b] == prev) return;
    okey[prev] = key[b];
    ostart[prev] = start[b];
    ocount[prev] = (int32_t)((b + 1 < nb ? (int64_t)start[b + 1] : n) - start[b]);
}

// level of every box, and head[first element of each leaf] = leaf box
__global__ void k_blev(int64_t nbox, int D, LevelTab lt, int64_t maxleaf, const int32_t *__restrict__ bstart,
                       const int32_t *__restrict__ bcount, int8_t *__restrict__ blev, int32_t *__restrict__ head)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int l = 0;
    while (l < D && b >= lt.off[l + 1]) l++;
    blev[b] = (int8_t)l;
    if (bcount[b] <= maxleaf || l == D) head[bstart[b]] = (int32_t)b;
}

// leaf list in element order (pos: inclusive scan of the head flags)
__global__ void k_leaf_list(int64_t n, const int32_t *__restrict__ head, const int32_t *__restrict__ pos,
                            int32_t *__restrict__ leaves)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && head[i] >= 0) leaves[pos[i] - 1] = head[i];
}

__global__ void k_fill_i32(int64_t n, int32_t *__restrict__ a, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_is_head(int64_t n, const int32_t *__restrict__ head, int32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = head[i] >= 0 ? 1 : 0;
}

// eleaf[i] = position of the leaf holding sorted element i (one block per leaf)
__global__ void k_leaf_fill(int64_t nleaf, const int32_t *__restrict__ leaves, const int32_t *__restrict__ bstart,
                            const int32_t *__restrict__ bcount, int32_t *__restrict__ eleaf)
{
    const int64_t t = blockIdx.x;
    if (t >= nleaf) return;
    const int b = leaves[t];
    const int s0 = bstart[b], c = bcount[b];
    for (int e = threadIdx.x; e < c; e += blockDim.x) eleaf[s0 + e] = (int32_t)t;
}

__device__ inline void box_ijk(uint64_t key, int l, uint32_t c[3])
{
    const uint64_t k = key & ((1ull << (3 * l)) - 1);
    c[0] = compact3(k);
    c[1] = compact3(k >> 1);
    c[2] = compact3(k >> 2);
}

// closed boxes (l1, c1), (l2, c2) touch or overlap; coordinates on the grid of level D
__device__ inline bool boxes_touch(int l1, const uint32_t c1[3], int l2, const uint32_t c2[3], int D)
{
    for (int d = 0; d < 3; d++) {
        const uint32_t lo1 = c1[d] << (D - l1), hi1 = (c1[d] + 1) << (D - l1);
        const uint32_t lo2 = c2[d] << (D - l2), hi2 = (c2[d] + 1) << (D - l2);
        if (lo1 > hi2 || lo2 > hi1) return false;
    }
    return true;
}

// Near-field source list of every leaf b (level lb), after Carrier, Greengard & Rokhlin:
//   U: b, same-level leaves adjacent to b, finer leaves adjacent to b below its colleagues,
//      coarser adjacent leaves (colleagues of b's ancestors) -- smoothed kernel;
//   W: boxes below a colleague of b whose parent touches b but which do not -- singular;
//   X: coarser leaves that are colleagues of an ancestor of b but do not touch b -- singular
//      (these are exactly the leaves C with b or one of its ancestors in W(C)).
// The finer boxes are found by a depth-first walk from each non-leaf colleague that
// descends only into boxes touching b.  PASS 0 counts entries and element pairs;
// PASS 1 writes the entries at the scanned offsets.  With wxexp, W boxes of levels >= 2 and
// the X entries of a leaf of level >= 2 go to the second list (box << 1 | is_x) instead:
// M2P of the W box's multipole at b's elements, P2L of the X leaf's elements into b's local
// expansion (every X entry qualifies: b or an ancestor of level >= 2 lies in the W-list of q).
template <int PASS>
__global__ void k_adlist(int64_t nleaf, int D, LevelTab lt, const int32_t *__restrict__ leaves,
                         const int8_t *__restrict__ blev, const uint64_t *__restrict__ bkey,
                         const int32_t *__restrict__ bcount, const int32_t *__restrict__ bchild0,
                         const int32_t *__restrict__ bnchild, int32_t *__restrict__ cnt_or_start,
                         int32_t *__restrict__ ent, int64_t *__restrict__ pairs, int32_t *__restrict__ flags,
                         int wxexp, int32_t *__restrict__ wcnt_or_start, int32_t *__restrict__ went)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nleaf) return;
    const int b = leaves[t];
    const int lb = blev[b];
    const uint64_t kb = bkey[b];
    const uint64_t sys = kb >> (3 * lb);
    uint32_t cb[3];
    box_ijk(kb, lb, cb);
    const int64_t nb_el = bcount[b];
    int64_t pu = 0, pw = 0, pm2p = 0, pp2l = 0;
    int nent = 0, nwx = 0;
    const int base = PASS ? cnt_or_start[t] : 0;
    const int wbase = (PASS && wxexp) ? wcnt_or_start[t] : 0;
    // sing: 0 = U, 1 = W, 2 = X
    auto emit = [&](int q, int kind) {
        const int64_t c = bcount[q];
        const bool byexp = wxexp && ((kind == 1 && blev[q] >= 2) || (kind == 2 && lb >= 2));
        if (byexp) {
            if (kind == 1) pm2p += nb_el;
            else pp2l += c;
            if (PASS) went[wbase + nwx] = (q << 1) | (kind == 2);
            nwx++;
            return;
        }
        const int sing = kind != 0;
        if (sing) pw += nb_el * c;
        else pu += nb_el * c;
        if (PASS) ent[base + nent] = (q << 1) | sing;
        nent++;
    };
    auto find_box = [&](int l, const int32_t c[3]) -> int {
        const int side = 1 << l;
        if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= side || c[1] >= side || c[2] >= side) return -1;
        const uint64_t k = (sys << (3 * l)) | spread3((uint32_t)c[0]) | (spread3((uint32_t)c[1]) << 1) |
                           (spread3((uint32_t)c[2]) << 2);
        const int64_t j = find_u64(bkey + lt.off[l], lt.nb[l], k);
        return j < 0 ? -1 : (int)(lt.off[l] + j);
    };
    // same level: b itself, leaf colleagues, and the walk below non-leaf colleagues
    constexpr int STK = 64;
    int stq[STK];
    int8_t stl[STK];
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int32_t c[3] = {(int32_t)cb[0] + dx, (int32_t)cb[1] + dy, (int32_t)cb[2] + dz};
                const int q = find_box(lb, c);
                if (q < 0) continue;
                if (q == b || bnchild[q] == 0) {
                    emit(q, 0);
                    continue;
                }
                int sp = 0;
                stq[sp] = q;
                stl[sp++] = (int8_t)lb;
                while (sp > 0) {
                    sp--;
                    const int node = stq[sp], ln = stl[sp];
                    const int c0 = bchild0[node], nc = bnchild[node];
                    for (int k = 0; k < nc; k++) {
                        const int ch = c0 + k;
                        uint32_t cc[3];
                        box_ijk(bkey[ch], ln + 1, cc);
                        if (!boxes_touch(ln + 1, cc, lb, cb, D)) {
                            emit(ch, 1);  // W
                        } else if (bnchild[ch] == 0) {
                            emit(ch, 0);
                        } else if (sp < STK) {
                            stq[sp] = ch;
                            stl[sp++] = (int8_t)(ln + 1);
                        } else {
                            atomicOr(&flags[2], 1);  // walk deeper than the stack: reported as an error
                        }
                    }
                }
            }
    // coarser leaves: colleagues of the ancestors
    for (int l = lb - 1; l >= 1; l--) {
        const int sh = lb - l;
        const int32_t ca[3] = {(int32_t)(cb[0] >> sh), (int32_t)(cb[1] >> sh), (int32_t)(cb[2] >> sh)};
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    const int32_t c[3] = {ca[0] + dx, ca[1] + dy, ca[2] + dz};
                    const int q = find_box(l, c);
                    if (q < 0 || bnchild[q] != 0) continue;
                    const uint32_t cq[3] = {(uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]};
                    emit(q, boxes_touch(l, cq, lb, cb, D) ? 0 : 2);  // U or X
                }
    }
    if (!PASS) {
        cnt_or_start[t] = nent;
        if (wxexp) wcnt_or_start[t] = nwx;
        atomicAdd((unsigned long long *)&pairs[1], (unsigned long long)(pu - nb_el));
        atomicAdd((unsigned long long *)&pairs[2], (unsigned long long)pw);
        atomicAdd((unsigned long long *)&pairs[4], (unsigned long long)pm2p);
        atomicAdd((unsigned long long *)&pairs[5], (unsigned long long)pp2l);
    }
}

// ---------------------------------------------------------------------------
// operator tables (FP64 arithmetic on the device)
// ---------------------------------------------------------------------------

// Rotation about the y axis by theta.  In the orthonormal basis
// Yh_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m| e^{i m phi}, F(R_y(theta) r) = exp(-theta G) F
// with G the matrix of D_{r x e_y} (eq. drt4 with t = e_y, rescaled): a real
// skew-symmetric tridiagonal matrix.  U = exp(-theta G) is computed by a
// Taylor series on theta/2^s followed by s squarings.  The forward / backward
// matrices of the scaled bar coefficients follow by diagonal rescaling:
//   R basis: Hb_mm' = U_mm' N_m'/N_m,   S basis: Hb_mm' = (-1)^(m+m') U_mm' N_m/N_m',
// N_m = sqrt((n-|m|)!(n+|m|)!), and U(-theta) = U(theta)^T.  They are stored
// split into the block acting on real parts and the block acting on imaginary parts:
//   Re: W_m'm = Hb_0m' (m=0),  Hb_mm' + Hb_-m,m' (m>0);   Im: W_m'm = Hb_mm' - Hb_-m,m'.
__device__ inline double gen_entry(int n, int m, int mp)
{
    // G[m][mp], nonzero for mp = m +- 1
    if (mp == m - 1) {
        if (m >= 1) return 0.5 * sqrt((double)(n + m) * (double)(n - m + 1));
        if (m == 0) return -0.5 * sqrt((double)n * (double)(n + 1));
        return -0.5 * sqrt((double)(n - m + 1) * (double)(n + m));
    }
    if (mp == m + 1) {
        if (m >= 1) return -0.5 * sqrt((double)(n - m) * (double)(n + m + 1));
        if (m == 0) return -0.5 * sqrt((double)n * (double)(n + 1));
        return 0.5 * sqrt((double)(n + m + 1) * (double)(n - m));
    }
    return 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_rot(int p, const double *__restrict__ theta, T *__restrict__ out)
{
    extern __shared__ double sd[];
    const int cls = blockIdx.x, n = blockIdx.y;
    const int D = 2 * n + 1, DD = D * D;
    double *E = sd, *Tm = E + DD, *Tmp = Tm + DD;
    double *fct = Tmp + DD;  // factorials 0..2n
    const int tid = threadIdx.x;
    const double th = theta[cls];
    for (int i = tid; i <= 2 * n; i += blockDim.x) {
        double f = 1.0;
        for (int k = 2; k <= i; k++) f *= (double)k;
        fct[i] = f;
    }
    // scaling: |theta| (n+1) / 2^s <= 1
    int s = 0;
    double sc = fabs(th) * (double)(n + 1);
    while (sc > 1.0) {
        sc *= 0.5;
        s++;
    }
    const double alpha = -th / (double)(1ull << s);  // A = alpha G
    for (int idx = tid; idx < DD; idx += blockDim.x) {
        const int i = idx / D, j = idx % D;
        E[idx] = (i == j) ? 1.0 : 0.0;
        Tm[idx] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 1; k <= 30; k++) {
        // Tmp = Tm * A / k  (A tridiagonal, zero diagonal)
        for (int idx = tid; idx < DD; idx += blockDim.x) {
            const int i = idx / D, j = idx % D;
            const int mj = j - n;
            double acc = 0.0;
            if (j - 1 >= 0) acc += Tm[i * D + j - 1] * alpha * gen_entry(n, mj - 1, mj);
            if (j + 1 < D) acc += Tm[i * D + j + 1] * alpha * gen_entry(n, mj + 1, mj);
            Tmp[idx] = acc / (double)k;
        }
        __syncthreads();
        for (int idx = tid; idx < DD; idx += blockDim.x) {
            Tm[idx] = Tmp[idx];
            E[idx] += Tmp[idx];
        }
        __syncthreads();
    }
    for (int q = 0; q < s; q++) {
        for (int idx = tid; idx < DD; idx += blockDim.x) {
            const int i = idx / D, j = idx % D;
            double acc = 0.0;
            for (int k = 0; k < D; k++) acc += E[i * D + k] * E[k * D + j];
            Tmp[idx] = acc;
        }
        __syncthreads();
        for (int idx = tid; idx < DD; idx += blockDim.x) E[idx] = Tmp[idx];
        __syncthreads();
    }
    // E = U(theta), indices (m+n, m'+n)
    const int RS = rot_set_size(p);
    const int boff = rot_block_off(n);
    auto Nm = [&](int m) { return sqrt(fct[n - abs(m)] * fct[n + abs(m)]); };
    for (int kind = 0; kind < ROT_NKIND; kind++) {
        T *W = out + ((size_t)cls * ROT_NKIND + kind) * RS + boff;
        const bool back = (kind == ROT_S_BACK || kind == ROT_R_BACK);
        const bool sbasis = (kind == ROT_S_FWD || kind == ROT_S_BACK);
        auto Hb = [&](int m, int mp) {
            const double u = back ? E[(mp + n) * D + (m + n)] : E[(m + n) * D + (mp + n)];
            if (sbasis) return (((m + mp) & 1) ? -1.0 : 1.0) * u * Nm(m) / Nm(mp);
            return u * Nm(mp) / Nm(m);
        };
        for (int idx = tid; idx < (n + 1) * (n + 1) + n * n; idx += blockDim.x) {
            double val;
            if (idx < (n + 1) * (n + 1)) {
                const int mp = idx / (n + 1), m = idx % (n + 1);
                val = (m == 0) ? Hb(0, mp) : Hb(m, mp) + Hb(-m, mp);
            } else {
                const int j = idx - (n + 1) * (n + 1);
                const int mp = j / n + 1, m = j % n + 1;
                val = Hb(m, mp) - Hb(-m, mp);
            }
            W[idx] = (T)val;
        }
    }
}

__device__ inline void dir_vector(int dir, int &dx, int &dy, int &dz)
{
    if (dir < NDIR_M2L) {
        dx = dir % 7 - 3;
        dy = (dir / 7) % 7 - 3;
        dz = dir / 49 - 3;
    } else {
        const int oct = (dir - NDIR_M2L) & 7;
        const int bx = oct & 1, by = (oct >> 1) & 1, bz = (oct >> 2) & 1;
        const int sg = (dir - NDIR_M2L) < 8 ? 1 : -1;  // child->parent: (1-2b); parent->child: -(1-2b)
        dx = sg * (1 - 2 * bx);
        dy = sg * (1 - 2 * by);
        dz = sg * (1 - 2 * bz);
    }
}

template <typename T>
__global__ void k_zph(int p, T *__restrict__ zph)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NDIR * p) return;
    const int dir = i / p, m = i % p;
    int dx, dy, dz;
    dir_vector(dir, dx, dy, dz);
    const double ph = (dx == 0 && dy == 0) ? 0.0 : atan2((double)dy, (double)dx);
    double sn, cs;
    sincos((double)m * ph, &sn, &cs);
    zph[(size_t)dir * 2 * p + m] = (T)cs;
    zph[(size_t)dir * 2 * p + p + m] = (T)sn;
}

// M2L coaxial (S|R) Hankel vector per squared offset length: k!/tau^(k+1), tau = |d| (units of h)
template <typename T>
__global__ void k_coax(int p, T *__restrict__ coax)
{
    const int d2 = blockIdx.x * blockDim.x + threadIdx.x;
    if (d2 >= 28) return;
    const int len = 2 * p + 2;
    if (d2 == 0) {
        for (int k = 0; k < len; k++) coax[k] = (T)0;
        return;
    }
    const double tau = sqrt((double)d2);
    double c = 1.0 / tau;
    for (int k = 0; k < len; k++) {
        coax[d2 * len + k] = (T)c;
        c *= (double)(k + 1) / tau;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int64_t igcd(int64_t a, int64_t b)
{
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// polar-angle classes of all directions: two integer vectors share a class iff
// dz1/|d1| = dz2/|d2| (compared exactly on sign(dz) and the reduced fraction dz^2/|d|^2)
static void theta_classes(std::vector<int16_t> &cls, std::vector<double> &theta)
{
    std::map<std::pair<int, std::pair<int64_t, int64_t>>, int> ids;
    cls.assign(NDIR, 0);
    theta.clear();
    for (int dir = 0; dir < NDIR; dir++) {
        int dx, dy, dz;
        if (dir < NDIR_M2L) {
            dx = dir % 7 - 3;
            dy = (dir / 7) % 7 - 3;
            dz = dir / 49 - 3;
        } else {
            const int oct = (dir - NDIR_M2L) & 7;
            const int sg = (dir - NDIR_M2L) < 8 ? 1 : -1;
            dx = sg * (1 - 2 * (oct & 1));
            dy = sg * (1 - 2 * ((oct >> 1) & 1));
            dz = sg * (1 - 2 * ((oct >> 2) & 1));
        }
        const int64_t n2 = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
        if (n2 == 0) {
            cls[dir] = 0;
            continue;
        }
        int64_t num = (int64_t)dz * dz, den = n2;
        int64_t g = igcd(num, den);
        if (g) {
            num /= g;
            den /= g;
        }
        const int sgn = dz > 0 ? 1 : (dz < 0 ? -1 : 0);
        auto key = std::make_pair(sgn, std::make_pair(num, den));
        auto it = ids.find(key);
        if (it == ids.end()) {
            int id = (int)theta.size();
            ids[key] = id;
            theta.push_back(acos((double)dz / sqrt((double)n2)));
            cls[dir] = (int16_t)id;
        } else {
            cls[dir] = (int16_t)it->second;
        }
    }
}

// Static M2L schedule of one sibling group: for each child position c and each
// of its 189 interaction offsets d (children of the parent's neighbours, not
// adjacent to the child), the entry (c, code(d)) with d = c_T - c_S, grouped
// by the polar-angle class of d.
static lhf_status build_schedule(lhf_plan *P, const std::vector<int16_t> &cls, int ntheta, hipStream_t st)
{
    std::vector<std::vector<std::pair<int16_t, int16_t>>> by(ntheta);
    for (int c = 0; c < 8; c++) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        for (int pz = -1; pz <= 1; pz++)
            for (int py = -1; py <= 1; py++)
                for (int px = -1; px <= 1; px++)
                    for (int ch = 0; ch < 8; ch++) {
                        const int sx = 2 * px + (ch & 1), sy = 2 * py + ((ch >> 1) & 1), sz = 2 * pz + ((ch >> 2) & 1);
                        const int dx = cx - sx, dy = cy - sy, dz = cz - sz;  // t = c_T - c_S (units of h)
                        if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
                        const int code = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
                        by[cls[code]].push_back({(int16_t)c, (int16_t)code});
                    }
    }
    // within a class, entries go round-robin over the child positions so that
    // consecutive translations (one wavefront's batch) have distinct targets
    std::vector<int16_t> start, ec, ed, cth;
    for (int k = 0; k < ntheta; k++) {
        if (by[k].empty()) continue;
        start.push_back((int16_t)ec.size());
        cth.push_back((int16_t)k);
        std::vector<std::vector<int16_t>> perc(8);
        for (auto &e : by[k]) perc[e.first].push_back(e.second);
        size_t left = by[k].size();
        for (size_t r = 0; left > 0; r++)
            for (int c = 0; c < 8; c++)
                if (r < perc[c].size()) {
                    ec.push_back((int16_t)c);
                    ed.push_back(perc[c][r]);
                    left--;
                }
    }
    start.push_back((int16_t)ec.size());
    P->sched_ncls = (int)cth.size();
    P->h_cls_theta = cth;
    // the same entries as rows of 8 indexed by child position (holes = -1)
    std::vector<int16_t> rstart, rows;
    for (int k = 0; k < ntheta; k++) {
        if (by[k].empty()) continue;
        rstart.push_back((int16_t)(rows.size() / 8));
        std::vector<std::vector<int16_t>> perc(8);
        for (auto &e : by[k]) perc[e.first].push_back(e.second);
        size_t nr = 0;
        for (int c = 0; c < 8; c++) nr = std::max(nr, perc[c].size());
        for (size_t r = 0; r < nr; r++)
            for (int c = 0; c < 8; c++) rows.push_back(r < perc[c].size() ? perc[c][r] : (int16_t)-1);
    }
    rstart.push_back((int16_t)(rows.size() / 8));
    LHF_HIP(dev_malloc(&P->sched_row_start, sizeof(int16_t) * rstart.size()));
    LHF_HIP(dev_malloc(&P->sched_rows, sizeof(int16_t) * rows.size()));
    LHF_HIP(hipMemcpyAsync(P->sched_row_start, rstart.data(), sizeof(int16_t) * rstart.size(), hipMemcpyHostToDevice, st));
    LHF_HIP(hipMemcpyAsync(P->sched_rows, rows.data(), sizeof(int16_t) * rows.size(), hipMemcpyHostToDevice, st));
    LHF_HIP(dev_malloc(&P->sched_cls_start, sizeof(int16_t) * start.size()));
    LHF_HIP(dev_malloc(&P->sched_c, sizeof(int16_t) * ec.size()));
    LHF_HIP(dev_malloc(&P->sched_dir, sizeof(int16_t) * ed.size()));
    LHF_HIP(dev_malloc(&P->sched_cls_theta, sizeof(int16_t) * cth.size()));
    LHF_HIP(hipMemcpyAsync(P->sched_cls_start, start.data(), sizeof(int16_t) * start.size(), hipMemcpyHostToDevice, st));
    LHF_HIP(hipMemcpyAsync(P->sched_c, ec.data(), sizeof(int16_t) * ec.size(), hipMemcpyHostToDevice, st));
    LHF_HIP(hipMemcpyAsync(P->sched_dir, ed.data(), sizeof(int16_t) * ed.size(), hipMemcpyHostToDevice, st));
    LHF_HIP(hipMemcpyAsync(P->sched_cls_theta, cth.data(), sizeof(int16_t) * cth.size(), hipMemcpyHostToDevice, st));
    return LHF_OK;
}

template <typename T>
static lhf_status build_tables(lhf_plan *P, hipStream_t st)
{
    std::vector<int16_t> cls;
    std::vector<double> theta;
    theta_classes(cls, theta);
    P->n_theta = (int)theta.size();
    P->h_theta = theta;
    const int p = P->p;
    const size_t RS = rot_set_size(p);
    LHF_HIP(dev_malloc(&P->rot, sizeof(T) * RS * ROT_NKIND * theta.size()));
    LHF_HIP(dev_malloc(&P->zph, sizeof(T) * NDIR * 2 * p));
    LHF_HIP(dev_malloc(&P->coax, sizeof(T) * 28 * (2 * p + 2)));
    LHF_HIP(dev_malloc(&P->dir_theta, sizeof(int16_t) * NDIR));
    LHF_HIP(dev_malloc(&P->dtmp, sizeof(double) * theta.size()));
    LHF_HIP(hipMemcpyAsync(P->dir_theta, cls.data(), sizeof(int16_t) * NDIR, hipMemcpyHostToDevice, st));
    LHF_HIP(hipMemcpyAsync(P->dtmp, theta.data(), sizeof(double) * theta.size(), hipMemcpyHostToDevice, st));
    const int Dmax = 2 * p - 1;
    size_t shm = sizeof(double) * (3 * (size_t)Dmax * Dmax + 2 * p);
    hipLaunchKernelGGL(k_rot<T>, dim3((unsigned)theta.size(), (unsigned)p), dim3(256), shm, st, p, P->dtmp,
                       (T *)P->rot);
    hipLaunchKernelGGL(k_zph<T>, dim3((NDIR * p + 255) / 256), dim3(256), 0, st, p, (T *)P->zph);
    hipLaunchKernelGGL(k_coax<T>, dim3(1), dim3(32), 0, st, p, (T *)P->coax);
    LHF_HIP(hipGetLastError());
    // batched M2M and L2L: two lanes per part vector (p = 8-16) or four (FP64 p = 20-24)
    P->use_mmhalf = P->mm_kind == LHF_MM_HALF;
    if (P->use_mmhalf && !mmhalf_build(P, st)) {
        set_error("batched M2M/L2L set-up failed");
        return LHF_ERR_HIP;
    }
    P->use_mmquarter = P->mm_kind == LHF_MM_QUARTER;
    if (P->use_mmquarter && !mmquarter_build(P, st)) {
        set_error("quarter-vector M2M/L2L set-up failed");
        return LHF_ERR_HIP;
    }
    // batched M2L (decided with the tree): schedule, padded rotation blocks, dense box maps
    if (P->use_tile) {
        lhf_status s = build_schedule(P, cls, (int)theta.size(), st);
        if (s != LHF_OK) return s;
        const bool tile_ok = P->m2l_kind == LHF_M2L_TILE || P->m2l_kind == LHF_M2L_TILE1;
        if (tile_ok && !wpad_build(P, st)) {
            set_error("allocation of the padded rotation table failed");
            return LHF_ERR_HIP;
        }
        for (int l = 2; l <= P->depth; l++) {
            const size_t cells = (size_t)P->nsys << (3 * l);
            LHF_HIP(dev_malloc(&P->dmap[l], sizeof(int32_t) * cells));
            LHF_HIP(hipMemsetAsync(P->dmap[l], 0xff, sizeof(int32_t) * cells, st));
            dmap_build(P, l, st);
        }
        // two schedule rows per batch where the ownership tile allows it (FP32 p = 8, 10: 14% faster
        // M2L on the 2^20 cube than one row)
        P->tile2 = P->precision == LHF_FP32 && (p == 8 || p == 10) && P->m2l_kind == LHF_M2L_TILE;
        // the matrix-core kernel walks the same schedule; it is slower than the VALU kernels at
        // every order measured (FP32 p = 16 on the 4M ring: 524 ms against 121 ms for the
        // half-vector kernel), so it runs only on request
        P->use_mfma = P->m2l_kind == LHF_M2L_MFMA;
        if (P->use_mfma && !wmfma_build(P, st)) {
            set_error("matrix-core M2L set-up failed");
            return LHF_ERR_HIP;
        }
        P->use_half = P->m2l_kind == LHF_M2L_HALF;
        if (P->use_half && !whalf_build(P, st)) {
            set_error("half-vector M2L set-up failed");
            return LHF_ERR_HIP;
        }
        P->use_qmfma = P->m2l_kind == LHF_M2L_QMFMA;
        if (P->use_qmfma && !qmfma_build(P, st)) {
            set_error("matrix-core quarter-layout M2L set-up failed");
            return LHF_ERR_HIP;
        }
        P->use_quarter = P->m2l_kind == LHF_M2L_QUARTER;
        if (P->use_quarter && !wquarter_build(P, st)) {
            set_error("quarter-vector M2L set-up failed");
            return LHF_ERR_HIP;
        }
    }
    return LHF_OK;
}

static void free_profile(lhf_plan *P)
{
    if (P->prof_ev) {
        for (int k = 0; k < P->prof_cap * PROF_EV_PER_EXEC; k++) (void)hipEventDestroy(P->prof_ev[k]);
        delete[] P->prof_ev;
    }
    P->prof_ev = nullptr;
    P->prof_cap = P->prof_used = 0;
}

static void free_plan(lhf_plan *P)
{
    if (!P) return;
    // the blocks go back to the cache, where another plan may take them at once: nothing queued
    // on any stream may still use them
    (void)hipDeviceSynchronize();
    free_profile(P);
    void *bufs[] = {P->perm, P->xs, P->ws, P->vfar, P->xw, P->bkey, P->bstart, P->bcount, P->bparent, P->bchild0,
                    P->bnchild, P->vcount, P->vsrc, P->vdir, P->ulist, P->eleaf, P->M, P->Lc, P->rot,
                    P->zph, P->dir_theta, P->coax, P->dflag, P->dtmp, P->sys_geo, P->sys_a, P->sys_off,
                    P->blev, P->leaves, P->nl_start, P->nl_ent, P->qs, P->wx_start, P->wx_ent, P->l2pv};
    for (void *b : bufs)
        if (b) (void)dev_free(b);
    for (int l = 0; l <= MAXDEPTH; l++)
        if (P->dmap[l]) (void)dev_free(P->dmap[l]);
    void *sb[] = {P->sched_cls_start, P->sched_c, P->sched_dir, P->sched_cls_theta, P->wpad, P->sched_row_start,
                  P->sched_rows, P->wmfma, P->whalf, P->mh, P->dtab, P->wmm, P->wll, P->qsched};
    for (void *b : sb)
        if (b) (void)dev_free(b);
    delete P;
}

static double core_k(double r, double a)
{
    // K(r; a) of eq. vem1
    return erf(r / (a * sqrt(2.0))) - sqrt(2.0 / M_PI) * (r / a) * exp(-r * r / (2.0 * a * a));
}

template <typename T>
static lhf_status plan_create_t(lhf_plan *P, const void *x, hipStream_t st)
{
    const int64_t n = P->n;
    const int d = P->depth;
    const int ns = P->nsys;
    const bool adaptive = P->adaptive;
    const int tpb = 256;
    const unsigned nblk = (unsigned)((n + tpb - 1) / tpb);
    auto grid = [&](int64_t m) { return dim3((unsigned)((m + tpb - 1) / tpb)); };
    // per-level temporaries are sized by the number of cells or n, whichever is smaller
    auto level_cap = [&](int l) { return std::min<int64_t>(n, (int64_t)ns << (3 * l)); };
    // ---- temporaries (all freed by cleanup)
    uint64_t *key = nullptr, *skey = nullptr;
    int32_t *idx = nullptr, *flag = nullptr, *id = nullptr, *lcnt = nullptr, *wcnt = nullptr;
    int64_t *dnb = nullptr, *dcnt = nullptr, *dad = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    std::vector<uint64_t *> lkey(d + 1, nullptr);
    std::vector<int32_t *> lstart(d + 1, nullptr), kid(d + 1, nullptr);
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);  // no queued kernel may still use a temporary
        for (void *b : {(void *)key, (void *)skey, (void *)idx, (void *)flag, (void *)id, (void *)dnb, (void *)dcnt,
                        (void *)dad, (void *)lcnt, (void *)wcnt, tmp})
            if (b) (void)dev_free(b);
        for (int l = 0; l <= d; l++) {
            if (lkey[l]) (void)dev_free(lkey[l]);
            if (lstart[l]) (void)dev_free(lstart[l]);
            if (kid[l]) (void)dev_free(kid[l]);
        }
    };
#define CK(call)                                        \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) {                         \
            cleanup();                                  \
            return hip_fail(_e, #call);                 \
        }                                               \
    } while (0)
    // ---- keys and sort
    CK(dev_malloc(&key, sizeof(uint64_t) * n));
    CK(dev_malloc(&skey, sizeof(uint64_t) * n));
    CK(dev_malloc(&idx, sizeof(int32_t) * n));
    CK(dev_malloc(&P->perm, sizeof(int32_t) * n));
    CK(dev_malloc(&flag, sizeof(int32_t) * n));
    CK(dev_malloc(&id, sizeof(int32_t) * n));
    CK(dev_malloc(&dnb, sizeof(int64_t) * (MAXDEPTH + 1)));
    CK(dev_malloc(&dcnt, sizeof(int64_t) * 6));
    CK(dev_malloc(&P->dflag, sizeof(int32_t) * 4));
    CK(hipMemsetAsync(P->dflag, 0, sizeof(int32_t) * 4, st));
    CK(hipMemsetAsync(dcnt, 0, sizeof(int64_t) * 6, st));
    CK(dev_malloc(&P->sys_geo, sizeof(double) * 4 * ns));
    CK(dev_malloc(&P->sys_a, sizeof(double) * ns));
    CK(dev_malloc(&P->sys_off, sizeof(int64_t) * (ns + 1)));
    CK(hipMemcpyAsync(P->sys_geo, P->h_sys_geo.data(), sizeof(double) * 4 * ns, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(P->sys_a, P->h_sys_a.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(P->sys_off, P->h_sys_off.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_keys<T>, dim3(nblk), dim3(tpb), 0, st, n, (const T *)x, ns, P->sys_off, P->sys_geo, d, key,
                       idx, P->dflag);
    CK(hipGetLastError());
    // the system index occupies the key bits above the 3*depth Morton bits
    int sys_bits = 0;
    while (((int64_t)1 << sys_bits) < ns) sys_bits++;
    const int end_bit = 3 * d + sys_bits;
    size_t sort_bytes = 0, scan_bytes = 0;
    CK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key, skey, idx, P->perm, (int)n, 0, end_bit, st));
    CK(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, flag, id, (int)n, st));
    tmp_bytes = std::max(sort_bytes, scan_bytes);
    CK(dev_malloc(&tmp, tmp_bytes));
    CK(hipcub::DeviceRadixSort::SortPairs(tmp, sort_bytes, key, skey, idx, P->perm, (int)n, 0, end_bit, st));
    CK(dev_malloc(&P->xs, sizeof(T) * 3 * n));
    CK(dev_malloc(&P->ws, sizeof(T) * 3 * n));
    CK(dev_malloc(&P->qs, sizeof(T) * n));
    // far-field v, s (and grad v when the plan may be asked for it), sorted order, SoA
    CK(dev_malloc(&P->vfar, sizeof(T) * (P->out_grad ? 15 : 6) * n));
    CK(dev_malloc(&P->xw, sizeof(T) * 8 * n));
    CK(dev_malloc(&P->eleaf, sizeof(int32_t) * n));
    hipLaunchKernelGGL(k_gather_x<T>, dim3(nblk), dim3(tpb), 0, st, n, (const T *)x, P->perm, (T *)P->xs);
    // ---- every non-empty box of every level
    for (int l = d; l >= 0; l--) {
        const int64_t cap = level_cap(l);
        CK(dev_malloc(&lkey[l], sizeof(uint64_t) * cap));
        CK(dev_malloc(&lstart[l], sizeof(int32_t) * cap));
        const int sh = 3 * (d - l);
        hipLaunchKernelGGL(k_level_flags, dim3(nblk), dim3(tpb), 0, st, n, skey, sh, flag);
        CK(hipcub::DeviceScan::InclusiveSum(tmp, scan_bytes, flag, id, (int)n, st));
        hipLaunchKernelGGL(k_level_fill, dim3(nblk), dim3(tpb), 0, st, n, skey, sh, flag, id, lkey[l], lstart[l],
                           l == d ? P->eleaf : nullptr, dnb + l);
    }
    // ---- adaptive tree: keep flags, kept boxes and leaves per level
    if (adaptive) {
        CK(dev_malloc(&dad, sizeof(int64_t) * 2 * (MAXDEPTH + 1)));
        CK(hipMemsetAsync(dad, 0, sizeof(int64_t) * 2 * (MAXDEPTH + 1), st));
        for (int l = 0; l <= d; l++) {
            const int64_t cap = level_cap(l);
            CK(dev_malloc(&kid[l], sizeof(int32_t) * cap));
            hipLaunchKernelGGL(k_akeep, grid(cap), dim3(tpb), 0, st, cap, l, d, (int64_t)P->max_per_leaf, n, dnb,
                               lkey[l], lstart[l], l ? lkey[l - 1] : nullptr, l ? lstart[l - 1] : nullptr, flag,
                               dad + MAXDEPTH + 1);
            size_t need = 0;
            CK(hipcub::DeviceScan::InclusiveSum(nullptr, need, flag, kid[l], (int)cap, st));
            if (need > tmp_bytes) {
                cleanup();
                set_error("internal: scan workspace too small");
                return LHF_ERR_HIP;
            }
            CK(hipcub::DeviceScan::InclusiveSum(tmp, need, flag, kid[l], (int)cap, st));
            hipLaunchKernelGGL(k_last_i32, dim3(1), dim3(1), 0, st, cap, kid[l], dad + l);
        }
        CK(hipGetLastError());
    }
    // ---- host synchronisation: tree sizes and input flags
    int64_t hnb[MAXDEPTH + 1], had[2 * (MAXDEPTH + 1)];
    int32_t hflag[4];
    CK(hipMemcpyAsync(hnb, dnb, sizeof(int64_t) * (d + 1), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(hflag, P->dflag, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
    if (adaptive) CK(hipMemcpyAsync(had, dad, sizeof(int64_t) * 2 * (MAXDEPTH + 1), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (hflag[1]) {
        cleanup();
        set_error("non-finite element coordinate");
        return LHF_ERR_NONFINITE;
    }
    if (hflag[0]) {
        cleanup();
        set_error("element outside the domain cube");
        return LHF_ERR_DOMAIN;
    }
    int64_t kept[MAXDEPTH + 1];
    P->nleaf = 0;
    for (int l = 0; l <= d; l++) {
        kept[l] = adaptive ? had[l] : hnb[l];
        if (adaptive) P->nleaf += had[MAXDEPTH + 1 + l];
    }
    if (!adaptive) P->nleaf = hnb[d];
    int64_t tot = 0;
    LevelTab lt;
    memset(&lt, 0, sizeof(lt));
    P->max_level = 0;
    for (int l = 0; l <= d; l++) {
        P->lev[l].nb = kept[l];
        P->lev[l].off = tot;
        lt.off[l] = tot;
        lt.nb[l] = kept[l];
        tot += kept[l];
        if (kept[l] > 0) P->max_level = l;
    }
    lt.off[d + 1] = tot;
    P->nbox = tot;
    const int P2 = P->p * P->p;
    CK(dev_malloc(&P->bkey, sizeof(uint64_t) * tot));
    CK(dev_malloc(&P->bstart, sizeof(int32_t) * tot));
    CK(dev_malloc(&P->bcount, sizeof(int32_t) * tot));
    CK(dev_malloc(&P->bparent, sizeof(int32_t) * tot));
    CK(dev_malloc(&P->bchild0, sizeof(int32_t) * tot));
    CK(dev_malloc(&P->bnchild, sizeof(int32_t) * tot));
    CK(dev_malloc(&P->vcount, sizeof(int32_t) * tot));
    // batched M2L: used when a batched kernel exists for (precision, p) and the dense box maps
    // stay small (levels <= 8, at most 2^28 cells); then the V-lists are only counted
    P->use_tile = P->m2l_kind != LHF_M2L_GENERIC;
    if (!P->use_tile) {
        CK(dev_malloc(&P->vsrc, sizeof(int32_t) * tot * VMAX));
        CK(dev_malloc(&P->vdir, sizeof(int16_t) * tot * VMAX));
    }
    CK(dev_malloc(&P->M, sizeof(T) * tot * 2 * P2));
    CK(dev_malloc(&P->Lc, sizeof(T) * tot * 2 * P2));
    // L2P velocity coefficients, per leaf [3][p(p+1)/2] complex
    CK(dev_malloc(&P->l2pv, sizeof(T) * (size_t)std::max<int64_t>(P->nleaf, 1) * 3 * P->p * (P->p + 1)));
    // multipoles of levels 0 and 1 are never formed, yet kernels read box 0 as a stand-in
    // source for inactive lanes: every multipole starts as a defined zero
    CK(hipMemsetAsync(P->M, 0, sizeof(T) * tot * 2 * P2, st));
    CK(hipMemsetAsync(P->vcount, 0, sizeof(int32_t) * tot, st));
    for (int l = 0; l <= d; l++) {
        if (adaptive) {
            const int64_t cap = level_cap(l);
            hipLaunchKernelGGL(k_acompact, grid(cap), dim3(tpb), 0, st, cap, l, n, dnb, kid[l], lkey[l], lstart[l],
                               P->bkey + lt.off[l], P->bstart + lt.off[l], P->bcount + lt.off[l]);
        } else {
            CK(hipMemcpyAsync(P->bkey + lt.off[l], lkey[l], sizeof(uint64_t) * hnb[l], hipMemcpyDeviceToDevice, st));
            CK(hipMemcpyAsync(P->bstart + lt.off[l], lstart[l], sizeof(int32_t) * hnb[l], hipMemcpyDeviceToDevice,
                              st));
            hipLaunchKernelGGL(k_counts, grid(hnb[l]), dim3(tpb), 0, st, hnb[l], n, P->bstart + lt.off[l],
                               P->bcount + lt.off[l]);
        }
    }
    hipLaunchKernelGGL(k_links, grid(tot), dim3(tpb), 0, st, tot, d, lt, P->bkey, P->bparent, P->bchild0, P->bnchild);
    // V-lists: filled for the generic M2L; counted from the box maps after build_tables otherwise
    if (!P->use_tile)
        for (int l = 2; l <= d; l++)
            if (kept[l] > 0)
                hipLaunchKernelGGL(k_vlist, grid(kept[l]), dim3(tpb), 0, st, lt.off[l], kept[l], l, P->bkey,
                                   P->vcount, P->vsrc, P->vdir);
    if (!adaptive) {
        CK(dev_malloc(&P->ulist, sizeof(int32_t) * hnb[d] * 27));
        hipLaunchKernelGGL(k_ulist, grid(hnb[d]), dim3(tpb), 0, st, lt.off[d], hnb[d], d, P->bkey, P->bcount,
                           P->ulist, dcnt + 1);
        hipLaunchKernelGGL(k_add_i32, dim3(nblk), dim3(tpb), 0, st, n, P->eleaf, (int32_t)lt.off[d]);
    } else {
        // levels, the leaf list in element order, the leaf of every element
        const int64_t nl = P->nleaf;
        CK(dev_malloc(&P->blev, sizeof(int8_t) * tot));
        CK(dev_malloc(&P->leaves, sizeof(int32_t) * nl));
        CK(dev_malloc(&P->nl_start, sizeof(int32_t) * (nl + 1)));
        CK(dev_malloc(&lcnt, sizeof(int32_t) * (nl + 1)));
        int32_t *head = flag, *ishead = idx;
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk), dim3(tpb), 0, st, n, head, -1);
        hipLaunchKernelGGL(k_blev, grid(tot), dim3(tpb), 0, st, tot, d, lt, (int64_t)P->max_per_leaf, P->bstart,
                           P->bcount, P->blev, head);
        hipLaunchKernelGGL(k_is_head, dim3(nblk), dim3(tpb), 0, st, n, head, ishead);
        CK(hipcub::DeviceScan::InclusiveSum(tmp, scan_bytes, ishead, id, (int)n, st));
        hipLaunchKernelGGL(k_leaf_list, dim3(nblk), dim3(tpb), 0, st, n, head, id, P->leaves);
        hipLaunchKernelGGL(k_leaf_fill, dim3((unsigned)nl), dim3(64), 0, st, nl, P->leaves, P->bstart, P->bcount,
                           P->eleaf);
        // near-field source lists: count, scan, size on the host, fill
        // (with W/X by expansions, a second list per leaf: the W boxes and X sources)
        const int wxe = P->wx_exp ? 1 : 0;
        if (wxe) {
            CK(dev_malloc(&wcnt, sizeof(int32_t) * (nl + 1)));
            CK(dev_malloc(&P->wx_start, sizeof(int32_t) * (nl + 1)));
            hipLaunchKernelGGL(k_fill_i32, grid(nl + 1), dim3(tpb), 0, st, nl + 1, wcnt, 0);
        }
        hipLaunchKernelGGL(k_fill_i32, grid(nl + 1), dim3(tpb), 0, st, nl + 1, lcnt, 0);
        hipLaunchKernelGGL(k_adlist<0>, grid(nl), dim3(tpb), 0, st, nl, d, lt, P->leaves, P->blev, P->bkey,
                           P->bcount, P->bchild0, P->bnchild, lcnt, nullptr, dcnt, P->dflag, wxe, wcnt, nullptr);
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, lcnt, P->nl_start, (int)(nl + 1), st));
        if (need > tmp_bytes) {
            cleanup();
            set_error("internal: scan workspace too small");
            return LHF_ERR_HIP;
        }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, lcnt, P->nl_start, (int)(nl + 1), st));
        if (wxe) CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, wcnt, P->wx_start, (int)(nl + 1), st));
        int32_t nent = 0, nwx = 0;
        CK(hipMemcpyAsync(&nent, P->nl_start + nl, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        if (wxe) CK(hipMemcpyAsync(&nwx, P->wx_start + nl, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        CK(dev_malloc(&P->nl_ent, sizeof(int32_t) * std::max<int64_t>(nent, 1)));
        if (wxe) CK(dev_malloc(&P->wx_ent, sizeof(int32_t) * std::max<int64_t>(nwx, 1)));
        hipLaunchKernelGGL(k_adlist<1>, grid(nl), dim3(tpb), 0, st, nl, d, lt, P->leaves, P->blev, P->bkey,
                           P->bcount, P->bchild0, P->bnchild, P->nl_start, P->nl_ent, dcnt, P->dflag, wxe,
                           P->wx_start, P->wx_ent);
    }
    CK(hipGetLastError());
    lhf_status ts = build_tables<T>(P, st);
    if (ts != LHF_OK) {
        cleanup();
        return ts;
    }
    if (P->use_tile)
        for (int l = 2; l <= d; l++)
            if (kept[l] > 0)
                hipLaunchKernelGGL(k_vcount_map, grid(kept[l]), dim3(tpb), 0, st, lt.off[l], kept[l], l, P->bkey,
                                   P->dmap[l], P->vcount);
    hipLaunchKernelGGL(k_sum_i32, dim3(256), dim3(256), 0, st, tot, P->vcount, dcnt);
    CK(hipGetLastError());
    int64_t hc[6];
    CK(hipMemcpyAsync(hc, dcnt, sizeof(int64_t) * 6, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(hflag, P->dflag, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    cleanup();
    if (hflag[2]) {
        set_error("internal: adaptive near-list walk exceeded its stack");
        return LHF_ERR_HIP;
    }
    P->n_m2l = hc[0];
    P->n_p2p = hc[1];
    P->n_wx = hc[2];
    P->n_m2p = hc[4];
    P->n_p2l = hc[5];
#undef CK
    return LHF_OK;
}

// ---- order from tolerance ------------------------------------------------------------------
// Relative L2 errors of v and s against the split-kernel direct sum per truncation number p
// (index p, 1..24), measured with the FP64 oracle FMM on seeded inputs of two classes:
//   uniform:  16384 elements uniform in the unit cube, depth 4 (four per leaf), core radius
//             a = 0.5 N^(-1/3), 256 sample targets;
//   adaptive: the 4,194,304-element vortex ring with 10% uniform background, at most 64 elements
//             per leaf down to level 8, a = 0.5 N^(-1/3), 128 sample targets (even p; odd p take
//             the next even order's value).
// Each entry is the larger of the two errors.  FP32 arithmetic adds a rounding floor.
#include "lhf_calib.inc"
constexpr double FP32_FLOOR = 1e-6;  // FP32 rounding of the translations and sums (measured <= 7e-7)

static double calib_max(bool adaptive, int p, double *ev, double *es)
{
    const double *t = adaptive ? CALIB_ADAPTIVE : CALIB_UNIFORM;
    p = std::max(1, std::min(p, MAXP));
    if (ev) *ev = t[2 * p];
    if (es) *es = t[2 * p + 1];
    return std::max(t[2 * p], t[2 * p + 1]);
}

void calib_error(bool adaptive, int p, double *ev, double *es) { calib_max(adaptive, p, ev, es); }

// smallest p whose calibrated error is <= tol; false (and the largest p) if none is
bool choose_order(bool adaptive, int precision, double tol, int *p)
{
    const int pmax = precision == LHF_FP64 ? MAXP : 16;
    for (int q = 1; q <= pmax; q++) {
        double e = calib_max(adaptive, q, nullptr, nullptr);
        if (precision == LHF_FP32) e = std::max(e, FP32_FLOOR);
        if (e <= tol) {
            *p = q;
            return true;
        }
    }
    *p = pmax;
    return false;
}

// ---- kernel choice ---------------------------------------------------------------------------
static bool m2l_available(int k, int precision, int p)
{
    switch (k) {
    case LHF_M2L_HALF: return m2l_half_supported(precision, p);
    case LHF_M2L_QUARTER: return m2l_quarter_supported(precision, p);
    case LHF_M2L_QMFMA: return m2l_qmfma_supported(precision, p);
    case LHF_M2L_TILE:
    case LHF_M2L_TILE1: return m2l_tile_supported(precision, p);
    case LHF_M2L_MFMA: return m2l_mfma_supported(precision, p);
    case LHF_M2L_GENERIC: return true;
    default: return false;
    }
}

// the kernel accumulates each target in a fixed order (no atomics)
bool kernel_deterministic(int precision, int p, int k)
{
    switch (k) {
    case LHF_M2L_HALF: return m2l_half_owned(precision, p);
    case LHF_M2L_QUARTER: return false;  // LDS atomics
    case LHF_M2L_QMFMA: return false;    // LDS atomics
    case LHF_M2L_TILE:
    case LHF_M2L_TILE1: return m2l_tile_owned(precision, p);
    default: return true;  // matrix-core (one parent per wavefront, register sums), generic (per box)
    }
}

static const char *m2l_name(int k)
{
    static const char *nm[] = {"AUTO", "HALF", "TILE", "TILE1", "MFMA", "GENERIC", "QUARTER", "QMFMA"};
    return (k >= 0 && k <= 7) ? nm[k] : "?";
}

// Resolve the descriptor's kernel requests (host only, before any launch).  AUTO takes the
// fastest kernel measured for (precision, p): the quarter-vector kernel at FP64 p >= 16, the
// half-vector kernel where it is instantiated, else the one-lane tile, else the generic per-box
// kernel; with LHF_DETERMINISTIC only kernels
// without atomics qualify (then the matrix-core kernel, which is deterministic, precedes the
// generic one).  Batched kernels need the dense box maps: depth <= 8 and at most 2^28 cells.
lhf_status resolve_kernels(const lhf_desc *d, int p, bool dmap_ok, int *m2l, int *mm)
{
    const bool det = (d->flags & LHF_DETERMINISTIC) != 0;
    const int prec = d->precision;
    int k = d->m2l_kernel;
    if (k == LHF_M2L_AUTO) {
        k = LHF_M2L_GENERIC;
        if (dmap_ok) {
            // FP64 p >= 16: the quarter-vector kernel (two wavefronts per SIMD where the half-vector
            // kernel holds one, tiles of consecutive targets, pipelined table reads; M2L per execute
            // on the 4M ring: 119 against 245 ms at p = 16, 440 against 1091 ms at p = 23); at p <= 12
            // the half-vector kernel is faster (2^20 cube, p = 12: 48 against 71 ms)
            const bool quarter_first = prec == LHF_FP64 && p >= 16;
            const int order[] = {quarter_first ? LHF_M2L_QUARTER : LHF_M2L_HALF, LHF_M2L_HALF, LHF_M2L_TILE,
                                 LHF_M2L_MFMA};
            for (int c : order) {
                if (c == LHF_M2L_MFMA && !det) continue;
                if (m2l_available(c, prec, p) && (!det || kernel_deterministic(prec, p, c))) {
                    k = c;
                    break;
                }
            }
        }
    } else {
        if (!m2l_available(k, prec, p)) {
            set_error(std::string("m2l_kernel ") + m2l_name(k) + " has no instantiation for this precision and p");
            return LHF_ERR_UNSUPPORTED;
        }
        if (k != LHF_M2L_GENERIC && !dmap_ok) {
            set_error(std::string("m2l_kernel ") + m2l_name(k) + " needs depth <= 8 and n_systems * 8^depth <= 2^28");
            return LHF_ERR_UNSUPPORTED;
        }
        if (det && !kernel_deterministic(prec, p, k)) {
            set_error(std::string("m2l_kernel ") + m2l_name(k) +
                      " accumulates with atomics at this precision and p: not deterministic");
            return LHF_ERR_UNSUPPORTED;
        }
    }
    int mk = d->mm_kernel;
    if (mk == LHF_MM_AUTO)
        mk = mm_half_supported(prec, p)      ? LHF_MM_HALF
             : mm_quarter_supported(prec, p) ? LHF_MM_QUARTER
                                             : LHF_MM_GENERIC;
    else if (mk == LHF_MM_HALF && !mm_half_supported(prec, p)) {
        set_error("mm_kernel HALF has no instantiation for this precision and p");
        return LHF_ERR_UNSUPPORTED;
    } else if (mk == LHF_MM_QUARTER && !mm_quarter_supported(prec, p)) {
        set_error("mm_kernel QUARTER has no instantiation for this precision and p");
        return LHF_ERR_UNSUPPORTED;
    }
    *m2l = k;
    *mm = mk;
    return LHF_OK;
}

// Checked plan construction shared by every creation entry point: nsys systems,
// system s owning elements off[s] .. off[s+1]-1 of x, with cube (lo[3s..3s+2], len[s])
// and core radius a[s] (host arrays).
lhf_status plan_new(lhf_plan **out, const lhf_desc *d, int nsys, const int64_t *off, const void *x,
                    const double *lo, const double *len, const double *a, hipStream_t stream)
{
    *out = nullptr;
    if (!d) return arg_error("desc is NULL");
    if (nsys < 1) return arg_error("n_systems must be >= 1");
    if (!off || !lo || !len || !a) return arg_error("system arrays must be non-NULL");
    if (off[0] != 0) return arg_error("sys_offsets[0] must be 0");
    for (int s = 0; s < nsys; s++)
        if (off[s + 1] < off[s]) return arg_error("sys_offsets must be non-decreasing");
    const int64_t n = off[nsys];
    if (n < 1) return arg_error("n must be >= 1");
    if (n > (int64_t)0x7fffffff) return arg_error("n must fit in int32");
    if (!x) return arg_error("x is NULL");
    if (d->precision != LHF_FP64 && d->precision != LHF_FP32) return arg_error("unknown precision");
    const int pmax = d->precision == LHF_FP64 ? MAXP : 16;
    if (d->p < 0 || d->p > pmax) return arg_error("p out of range (FP64: 1..24, FP32: 1..16; 0: from tol)");
    if (d->flags & ~(LHF_SINGULAR | LHF_DETERMINISTIC | LHF_OUT_GRAD | LHF_WX_EXPANSIONS))
        return arg_error("unknown flag bits");
    if (d->reserved != 0) return arg_error("reserved descriptor field must be 0");
    if (d->translation == LHF_TRANS_DIRECT) {
        set_error("translation = LHF_TRANS_DIRECT (full O(p^4) matrices) is not built in this library");
        return LHF_ERR_UNSUPPORTED;
    }
    if (d->translation != LHF_TRANS_RCR) return arg_error("unknown translation scheme");
    if (d->m2l_kernel < LHF_M2L_AUTO || d->m2l_kernel > LHF_M2L_QMFMA) return arg_error("unknown m2l_kernel");
    if (d->mm_kernel < LHF_MM_AUTO || d->mm_kernel > LHF_MM_QUARTER) return arg_error("unknown mm_kernel");
    if (d->depth < 2 || d->depth > MAXDEPTH) return arg_error("depth out of range (2..10)");
    if (d->max_per_leaf < 0) return arg_error("max_per_leaf must be >= 0");
    if (!(d->tol > 0.0)) return arg_error("tol must be > 0");
    if ((int64_t)nsys > ((int64_t)1 << (63 - 3 * d->depth)) / 2) return arg_error("too many systems for this depth");
    for (int s = 0; s < nsys; s++) {
        if (!(len[s] > 0.0) || !isfinite(len[s])) return arg_error("cube sides must be finite and > 0");
        for (int k = 0; k < 3; k++)
            if (!isfinite(lo[3 * s + k])) return arg_error("cube origins must be finite");
        if (!(a[s] >= 0.0) || !isfinite(a[s])) return arg_error("core radius a must be finite and >= 0");
    }
    // order: as given, or the smallest calibrated order that reaches tol
    int p = d->p;
    bool tol_unmet = false;
    const bool adaptive_tree = d->max_per_leaf > 0;
    if (p == 0) tol_unmet = !choose_order(adaptive_tree, d->precision, d->tol, &p);
    int m2l_kind = 0, mm_kind = 0;
    {
        const bool dmap_ok = d->depth <= 8 && ((int64_t)nsys << (3 * d->depth)) <= ((int64_t)1 << 28);
        lhf_status ks = resolve_kernels(d, p, dmap_ok, &m2l_kind, &mm_kind);
        if (ks != LHF_OK) return ks;
    }
    lhf_plan *P = new lhf_plan();
    P->desc = *d;
    P->desc.p = p;
    P->n = n;
    P->p = p;
    P->m2l_kind = m2l_kind;
    P->mm_kind = mm_kind;
    P->deterministic = kernel_deterministic(d->precision, p, m2l_kind);
    P->p_from_tol = d->p == 0;
    P->out_grad = (d->flags & LHF_OUT_GRAD) != 0;
    calib_error(adaptive_tree, p, &P->calib_err_v, &P->calib_err_s);
    P->depth = d->depth;
    P->precision = d->precision;
    P->tsize = d->precision == LHF_FP64 ? 8 : 4;
    P->stream = stream;
    P->adaptive = d->max_per_leaf > 0;
    P->max_per_leaf = d->max_per_leaf;
    P->wx_exp = P->adaptive && (d->flags & LHF_WX_EXPANSIONS) != 0;
    P->nsys = nsys;
    P->h_sys_off.assign(off, off + nsys + 1);
    P->h_sys_geo.resize(4 * (size_t)nsys);
    P->h_sys_a.resize(nsys);
    for (int s = 0; s < nsys; s++) {
        for (int k = 0; k < 3; k++) P->h_sys_geo[4 * s + k] = lo[3 * s + k];
        P->h_sys_geo[4 * s + 3] = len[s];
        P->h_sys_a[s] = (d->flags & LHF_SINGULAR) ? 0.0 : a[s];
    }
    lhf_status st = d->precision == LHF_FP64 ? plan_create_t<double>(P, x, stream) : plan_create_t<float>(P, x, stream);
    if (st < 0) {
        free_plan(P);
        return st;
    }
    *out = P;
    // warn when, in some system, the far field's singular kernel differs from the core by more than tol
    for (int s = 0; s < nsys; s++) {
        const double as = P->h_sys_a[s];
        if (as > 0.0 && 1.0 - core_k(len[s] / (double)(1 << P->max_level), as) > d->tol) P->warnings |= 1;
    }
    if (tol_unmet) P->warnings |= 2;
    // both warnings are kept in the plan's statistics; the status names the one that bounds the
    // accuracy more directly (an order that cannot reach tol)
    return tol_unmet ? LHF_WARN_TOL_UNMET : (P->warnings & 1) ? LHF_WARN_CORE_SPLIT : LHF_OK;
}

void plan_free(lhf_plan *P) { free_plan(P); }

// Device memory of lhf_evaluate_noalloc: one copy of this array per device, held until the
// process ends.  Its name is a host-side stand-in in host code; kernels only ever receive the
// device address that hipGetSymbolAddress returns for the current device (noalloc_scratch).
constexpr size_t NOALLOC_BYTES = (size_t)256 << 20;
constexpr int64_t NOALLOC_MAX_N = (int64_t)1 << 17;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mu;
constexpr int MAX_DEVICES = 64;
void *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// device address of 'scratch' on the current device, looked up once per device
static lhf_status noalloc_scratch(void **out)
{
    int dev = 0;
    LHF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return arg_error("device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                     "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LHF_OK;
}

}  // namespace lhf

using namespace lhf;

extern "C" {

void lhf_desc_default(lhf_desc *d)
{
    if (!d) return;
    memset(d, 0, sizeof(*d));
    d->p = 12;
    d->tol = 1e-6;
    d->depth = 4;
    d->domain_len = 1.0;
    d->precision = LHF_FP64;
}

const char *lhf_last_error(void) { return g_err.c_str(); }

const char *lhf_version(void) { return "lhfmm 0.1 (gfx950)"; }

lhf_status lhf_plan_create(lhf_plan **out, const lhf_desc *d, int64_t n, const void *x, double a, void *stream)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (!d) return arg_error("desc is NULL");
    if (n < 1) return arg_error("n must be >= 1");
    if (!(d->domain_len > 0.0) || !isfinite(d->domain_len))
        return arg_error("domain_len must be > 0 (bounding-cube mode is not supported)");
    const int64_t off[2] = {0, n};
    return plan_new(out, d, 1, off, x, d->domain_lo, &d->domain_len, &a, (hipStream_t)stream);
}

lhf_status lhf_plan_create_multi(lhf_plan **out, const lhf_desc *d, int32_t n_systems, const int64_t *sys_offsets,
                                 const void *x, const double *sys_lo, const double *sys_len, const double *sys_a,
                                 void *stream)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    return plan_new(out, d, n_systems, sys_offsets, x, sys_lo, sys_len, sys_a, (hipStream_t)stream);
}

lhf_status lhf_execute_io(lhf_plan *plan, const lhf_io *io, void *stream)
{
    if (!plan) return arg_error("plan is NULL");
    if (!io) return arg_error("io is NULL");
    if (!io->omega || !io->v || !io->s) return arg_error("omega, v and s must be non-NULL");
    if (io->what < 1 || io->what > 3) return arg_error("what must be 1, 2 or 3");
    if (io->reserved != 0) return arg_error("reserved io field must be 0");
    if ((io->grad_v || io->beta) && !plan->out_grad) {
        set_error("grad_v or beta requested from a plan created without LHF_OUT_GRAD");
        return LHF_ERR_STATE;
    }
    plan->stream = (hipStream_t)stream;
    return execute_impl(plan, io, (hipStream_t)stream);
}

lhf_status lhf_execute_scalar(lhf_plan *plan, const void *q, void *phi, void *grad_phi, void *stream)
{
    if (!plan) return arg_error("plan is NULL");
    if (!q || !phi) return arg_error("q and phi must be non-NULL");
    if (plan->adaptive || plan->nsys != 1) {
        set_error("the scalar FMM runs on single-system uniform trees only");
        return LHF_ERR_UNSUPPORTED;
    }
    plan->stream = (hipStream_t)stream;
    return execute_scalar_impl(plan, q, phi, grad_phi, (hipStream_t)stream);
}

lhf_status lhf_execute_parts(lhf_plan *plan, const void *omega, void *v, void *s, void *grad_v, int32_t what,
                             void *stream)
{
    lhf_io io;
    memset(&io, 0, sizeof(io));
    io.omega = omega;
    io.v = v;
    io.s = s;
    io.grad_v = grad_v;
    io.what = what;
    return lhf_execute_io(plan, &io, stream);
}

lhf_status lhf_execute(lhf_plan *plan, const void *omega, void *v, void *s, void *grad_v, void *stream)
{
    return lhf_execute_parts(plan, omega, v, s, grad_v, 3, stream);
}

lhf_status lhf_evaluate(const lhf_desc *d, int64_t n, const void *x, const void *omega, double a, void *v, void *s,
                        void *stream)
{
    lhf_plan *P = nullptr;
    lhf_status st = lhf_plan_create(&P, d, n, x, a, stream);
    if (st < 0) return st;
    lhf_status e = lhf_execute(P, omega, v, s, nullptr, stream);
    lhf_status dd = lhf_plan_destroy(P);
    if (e < 0) return e;
    if (dd < 0) return dd;
    return st;
}

lhf_status lhf_evaluate_noalloc(const lhf_desc *d, int64_t n, const void *x, const void *omega, double a, void *v,
                                void *s, void *stream)
{
    if (!d) return arg_error("desc is NULL");
    if (!x || !omega || !v || !s) return arg_error("x, omega, v and s must be non-NULL");
    if (n < 1) return arg_error("n must be >= 1");
    if (n > NOALLOC_MAX_N) {
        set_error("lhf_evaluate_noalloc: n = " + std::to_string(n) + " exceeds its maximum of " +
                  std::to_string(NOALLOC_MAX_N) + " elements");
        return LHF_ERR_WORKSPACE;
    }
    void *base = nullptr;
    lhf_status st = noalloc_scratch(&base);
    if (st != LHF_OK) return st;
    Arena ar;
    ar.base = (char *)base;
    ar.cap = NOALLOC_BYTES;
    t_arena = &ar;
    lhf_plan *P = nullptr;
    st = lhf_plan_create(&P, d, n, x, a, stream);
    lhf_status e = LHF_OK, dd = LHF_OK;
    if (st >= 0) {
        e = lhf_execute(P, omega, v, s, nullptr, stream);
        dd = lhf_plan_destroy(P);  // synchronises; its blocks return to nothing (arena)
    }
    t_arena = nullptr;
    if (ar.need) {
        set_error("lhf_evaluate_noalloc: the plan needs more than the " + std::to_string(NOALLOC_BYTES >> 20) +
                  " MiB of its fixed device array (asked for " + std::to_string(ar.need) + " bytes)");
        return LHF_ERR_WORKSPACE;
    }
    if (st < 0) return st;
    if (e < 0) return e;
    if (dd < 0) return dd;
    return st;
}

lhf_status lhf_plan_stats(const lhf_plan *P, lhf_stats *out)
{
    if (!P || !out) return arg_error("plan and out must be non-NULL");
    memset(out, 0, sizeof(*out));
    out->n = P->n;
    out->depth = P->depth;
    out->p = P->p;
    for (int l = 0; l <= P->depth; l++) out->boxes[l] = P->lev[l].nb;
    out->n_m2l = P->n_m2l;
    // one M2M per box below level 2 (into its parent) and one L2L per box below level 2
    int64_t nm2m = 0;
    for (int l = 3; l <= P->depth; l++) nm2m += P->lev[l].nb;
    out->n_m2m = nm2m;
    out->n_l2l = nm2m;
    out->n_p2p_pairs = P->n_p2p;
    out->n_theta_classes = P->n_theta;
    out->max_level = P->max_level;
    out->n_leaves = P->nleaf;
    out->n_wx_pairs = P->n_wx;
    out->m2l_kernel = P->m2l_kind;
    out->mm_kernel = P->mm_kind;
    out->deterministic = P->deterministic ? 1 : 0;
    out->p_from_tol = P->p_from_tol ? 1 : 0;
    out->calib_err_v = P->calib_err_v;
    out->calib_err_s = P->calib_err_s;
    out->warnings = P->warnings;
    out->wx_expansions = P->wx_exp ? 1 : 0;
    out->n_m2p = P->n_m2p;
    out->n_p2l = P->n_p2l;
    return LHF_OK;
}

lhf_status lhf_profile_begin(lhf_plan *P, int32_t max_exec)
{
    if (!P) return arg_error("plan is NULL");
    if (max_exec < 1 || max_exec > 100000) return arg_error("max_exec must be in 1..100000");
    free_profile(P);
    const int ne = max_exec * PROF_EV_PER_EXEC;
    P->prof_ev = new hipEvent_t[ne];
    for (int k = 0; k < ne; k++) {
        hipError_t e = hipEventCreate(&P->prof_ev[k]);
        if (e != hipSuccess) {
            P->prof_cap = k / PROF_EV_PER_EXEC;
            for (int j = k; j < ne; j++) P->prof_ev[j] = nullptr;
            for (int j = 0; j < k; j++) (void)hipEventDestroy(P->prof_ev[j]);
            delete[] P->prof_ev;
            P->prof_ev = nullptr;
            P->prof_cap = 0;
            return hip_fail(e, "hipEventCreate");
        }
    }
    P->prof_cap = max_exec;
    P->prof_used = 0;
    return LHF_OK;
}

lhf_status lhf_profile_end(lhf_plan *P, double *phase_ms, int32_t *n_exec)
{
    if (!P || !phase_ms || !n_exec) return arg_error("plan, phase_ms and n_exec must be non-NULL");
    if (!P->prof_ev) {
        set_error("lhf_profile_begin was not called");
        return LHF_ERR_STATE;
    }
    for (int k = 0; k < LHF_NPHASE; k++) phase_ms[k] = 0.0;
    for (int e = 0; e < P->prof_used; e++) {
        hipEvent_t *ev = P->prof_ev + (size_t)e * PROF_EV_PER_EXEC;
        LHF_HIP(hipEventSynchronize(ev[6]));
        for (int k = 0; k < 6; k++) {
            float ms = 0.f;
            LHF_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            phase_ms[k] += ms;
        }
        for (int l = 2; l <= P->depth; l++) {
            float ms = 0.f;
            LHF_HIP(hipEventElapsedTime(&ms, ev[7 + 2 * l], ev[8 + 2 * l]));
            phase_ms[6] += ms;
        }
    }
    *n_exec = P->prof_used;
    free_profile(P);
    return LHF_OK;
}

constexpr int LHF_SHAPE_LEVELS = 9;  // lhf_shapes.m2l_tile: levels 0 .. 8 (the batched M2L kernels' range)
static_assert(sizeof(((lhf_shapes *)nullptr)->m2l_tile) / sizeof(int32_t) == LHF_SHAPE_LEVELS, "lhf_shapes");

static std::string shapes_key(const lhf_plan *P)
{
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    return arch + "/" + (P->precision == LHF_FP64 ? "fp64" : "fp32") + "/p" + std::to_string(P->p) + "/" +
           (P->adaptive ? "adaptive" : "uniform") + "/d" + std::to_string(P->depth) + "/n" + std::to_string(P->n);
}

// shapes cache: a JSON array with one object per line
//   {"key": "gfx950/fp64/p23/adaptive/d8/n4194304", "m2l_tile": [0, 0, 1, 1, 4, 6, 6, 6, 6], "p2p_tile": 128}
static bool read_shapes(const char *path, const std::string &key, lhf_shapes *out, std::vector<std::string> *lines)
{
    FILE *f = fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (fgets(line, sizeof(line), f)) {
        char k[256];
        lhf_shapes sh;
        int *t = sh.m2l_tile;
        if (sscanf(line, " {\"key\": \"%255[^\"]\", \"m2l_tile\": [%d, %d, %d, %d, %d, %d, %d, %d, %d], \"p2p_tile\": %d}", k,
                   &t[0], &t[1], &t[2], &t[3], &t[4], &t[5], &t[6], &t[7], &t[8], &sh.p2p_tile) != 11)
            continue;
        std::string ln(line);
        while (!ln.empty() && (ln.back() == '\n' || ln.back() == ',' || ln.back() == ' ')) ln.pop_back();
        lines->push_back(ln.substr(ln.find('{')));
        if (k == key) {
            *out = sh;
            found = true;
        }
    }
    fclose(f);
    return found;
}

static lhf_status check_shapes(const lhf_plan *P, const lhf_shapes *sh)
{
    const int maxns = P->use_quarter ? m2l_quarter_max_ns(P->p) : P->use_qmfma ? m2l_qmfma_max_ns(P->p) : 0;
    for (int l = 0; l < LHF_SHAPE_LEVELS; l++)
        if (sh->m2l_tile[l] < 0 || sh->m2l_tile[l] > std::max(maxns, 0) || (maxns == 0 && sh->m2l_tile[l] != 0))
            return arg_error("m2l_tile out of range for this plan's M2L kernel");
    if (sh->p2p_tile != 0 && sh->p2p_tile != 64 && sh->p2p_tile != 128 && sh->p2p_tile != 256)
        return arg_error("p2p_tile must be 0, 64, 128 or 256");
    return LHF_OK;
}

lhf_status lhf_plan_set_shapes(lhf_plan *P, const lhf_shapes *sh)
{
    if (!P || !sh) return arg_error("plan and shapes must be non-NULL");
    lhf_status s = check_shapes(P, sh);
    if (s != LHF_OK) return s;
    for (int l = 0; l < LHF_SHAPE_LEVELS; l++) P->m2l_ns[l] = sh->m2l_tile[l];
    P->p2p_ts = sh->p2p_tile;
    return LHF_OK;
}

lhf_status lhf_plan_get_shapes(const lhf_plan *P, lhf_shapes *sh)
{
    if (!P || !sh) return arg_error("plan and shapes must be non-NULL");
    for (int l = 0; l < LHF_SHAPE_LEVELS; l++) sh->m2l_tile[l] = P->m2l_ns[l];
    sh->p2p_tile = P->p2p_ts;
    return LHF_OK;
}

lhf_status lhf_plan_autotune(lhf_plan *P, const void *omega, const char *cache_path, lhf_shapes *out, void *stream)
{
    if (!P) return arg_error("plan is NULL");
    if (!omega) return arg_error("omega is NULL");
    const std::string key = shapes_key(P);
    std::vector<std::string> lines;
    lhf_shapes sh;
    memset(&sh, 0, sizeof(sh));
    if (cache_path && cache_path[0] && read_shapes(cache_path, key, &sh, &lines)) {
        lhf_status s = lhf_plan_set_shapes(P, &sh);
        if (s != LHF_OK) return s;
        if (out) *out = sh;
        return LHF_OK;
    }
    P->stream = (hipStream_t)stream;
    int ns[MAXDEPTH + 1], ts = 0;
    lhf_status rs = autotune_impl(P, omega, ns, &ts, (hipStream_t)stream);
    if (rs != LHF_OK) return rs;
    for (int l = 0; l < LHF_SHAPE_LEVELS; l++) sh.m2l_tile[l] = ns[l];
    sh.p2p_tile = ts;
    if (out) *out = sh;
    if (cache_path && cache_path[0]) {
        char buf[512];
        const int *t = sh.m2l_tile;
        snprintf(buf, sizeof(buf), "{\"key\": \"%s\", \"m2l_tile\": [%d, %d, %d, %d, %d, %d, %d, %d, %d], \"p2p_tile\": %d}",
                 key.c_str(), t[0], t[1], t[2], t[3], t[4], t[5], t[6], t[7], t[8], sh.p2p_tile);
        lines.push_back(buf);
        const std::string tmp = std::string(cache_path) + ".tmp";
        FILE *f = fopen(tmp.c_str(), "w");
        bool ok = f != nullptr;
        if (ok) {
            fprintf(f, "[\n");
            for (size_t i = 0; i < lines.size(); i++) fprintf(f, " %s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
            fprintf(f, "]\n");
            ok = fclose(f) == 0 && rename(tmp.c_str(), cache_path) == 0;
        }
        if (!ok) {
            set_error(std::string("could not write the shapes cache ") + cache_path);
            return LHF_ERR_ARG;
        }
    }
    return LHF_OK;
}

lhf_status lhf_release_cached_memory(void)
{
    lhf::MemCache &m = lhf::mem_cache();
    std::lock_guard<std::mutex> lk(m.mu);
    lhf::mem_trim_locked(m, -1, 0);
    return LHF_OK;
}

lhf_status lhf_plan_destroy(lhf_plan *P)
{
    if (!P) return LHF_OK;
    hipError_t e = hipDeviceSynchronize();  // executes may have been queued on any stream
    free_plan(P);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return LHF_OK;
}

}  // extern "C"

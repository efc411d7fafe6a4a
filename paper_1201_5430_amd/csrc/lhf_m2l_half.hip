// lhf_m2l_half.hip -- batched M2L with each translation's coefficient vector split over two
// lanes by the parity of m (p = 8, 10, 12, 16 in both precisions).
//
// The translation is the same as in the one-lane tile kernel: rotation about z and y,
// coaxial (S|R) shift, R-conversion (eq. rcr1), back-rotation (Sec. 4.4), for both
// potentials, summed into the local expansions of the tile's targets in LDS.  What differs
// is the lane layout.  Holding a whole part vector per lane (P(P+1)/2 values) fills the
// register file at these orders and leaves one wavefront per SIMD, which cannot hide the
// latency of its own LDS reads and dependent FMAs.  Here
//   lane = 8 t + 4 pot + 2 part + h      (t: translation of the batch, 8 per wavefront)
// and the lane with parity h holds the entries m = 2j + h (j = 0 .. n/2) of every order n:
//   * z-rotations act entry by entry (partner part by a DPP quad swap);
//   * the coaxial shift and the conversion act column by column (fixed m), so they stay in
//     the lane; the conversion's other-potential partner comes by ds_swizzle;
//   * the y-rotation of order n mixes all m: each lane forms the partial sums over its own
//     columns for its own output rows (o) and for its partner's rows (t), and a DPP pair swap
//     adds the partner's t to the lane's o.  The rotation blocks are stored per (kind, part,
//     parity) as [o rows | t rows] x own columns, zero where m or m' exceeds n.
// Slots of odd lanes whose m exceeds n (even n) stay zero and are never read back.
// The sources of a level are first copied into the same lane layout (k_mhalf), so a lane
// loads its entries as whole 16-byte vectors from one address; in shared mode the LDS
// accumulators of the targets use it too, so the accumulation needs no per-entry selects.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lhf_internal.h"
#include "lhf_m2l_common.h"

namespace lhf {
namespace hv {

// entries of order n held by one lane: m = 2j + h, j < S(n)
__host__ __device__ constexpr int S(int n) { return n / 2 + 1; }
__host__ __device__ constexpr int hoff(int n)
{
    int o = 0;
    for (int k = 0; k < n; k++) o += S(k);
    return o;
}
template <typename T>
__host__ __device__ constexpr int E() { return 16 / (int)sizeof(T); }
// rotation rows padded to whole 16-byte vectors
template <typename T>
__host__ __device__ constexpr int RL(int n) { return (S(n) + E<T>() - 1) / E<T>() * E<T>(); }
// offset of order n's block in one (kind, part, parity) table: sum_{k<n} 2 S(k) RL(k)
template <typename T>
__host__ __device__ constexpr int woff(int n)
{
    int o = 0;
    for (int k = 0; k < n; k++) o += 2 * S(k) * RL<T>(k);
    return o;
}

template <typename T, int P>
struct Shape {
    static constexpr int NH = hoff(P);      // entries per lane
    static constexpr int WH = woff<T>(P);   // one (kind, part, parity) rotation table
    // tables one 16-byte vector apart beyond their length: the four tables a wavefront reads
    // at once (part x parity) start in different LDS banks
    static constexpr int WHS = WH + E<T>();
    static constexpr int P2 = P * P;
    // one lane's entries padded to whole 16-byte vectors: the stride of the source layout
    static constexpr int NHP = (NH + E<T>() - 1) / E<T>() * E<T>();
};

// FP64 orders above 16: one class's rotation tables (8 x WHS entries, 105 KB at p = 20, 176 KB
// at p = 24) and the accumulators of a whole sibling group no longer fit the LDS together.  A
// tile then holds half a sibling group (four targets: children 4h .. 4h + 3 of one parent), and
// only the forward (S-basis) tables are staged: the backward R-basis block of a polar angle is a
// diagonal similarity of the transposed forward block,
//   Re: W_back = D W_fwd^T D^-1, D = diag(1, -1/2, 1/2, -1/2, ..)  (m = 0, 1, 2, ..),
//   Im: W_back = D W_fwd^T D^-1, D = diag((-1)^m)                  (m = 1, 2, ..),
// (the N_m rescalings of the two bases cancel, the (-1)^(m+m') of the S basis and the pairing of
// +-m into the real-packed blocks leave these factors), so the back-rotation runs on the staged
// forward tables read row by row
template <typename T, int P>
constexpr bool half_tiles()
{
    return sizeof(T) == 8 && P > 16;
}
// rotation tables staged in LDS per class
template <typename T, int P>
constexpr int staged_tables()
{
    return half_tiles<T, P>() ? 4 : 8;
}

// packed (phi, chi) expansion [pot][n^2 + (Re: m | Im: n + m)] -> lane layout
// [role = 4 pot + 2 part + h][RS] (RS >= hoff(P)): position of packed index k
template <int P, int RS>
__device__ inline int entry_lane(int k)
{
    const int pot = k / (P * P), q = k % (P * P);
    int n = (int)sqrtf((float)q);  // floor(sqrt(q)), corrected for rounding
    if ((n + 1) * (n + 1) <= q) n++;
    if (n * n > q) n--;
    const int i = q - n * n, part = i > n, m = part ? i - n : i;
    const int a = n >> 1, hn = (n & 1) ? (a + 1) * (a + 1) : a * (a + 1);  // hoff(n)
    return (4 * pot + 2 * part + (m & 1)) * RS + hn + (m >> 1);
}

template <typename T>
struct V16;
template <>
struct V16<float> {
    using type = float4;
};
template <>
struct V16<double> {
    using type = double2;
};

// sum_{i<N} W[i] x[i], W read as 16-byte vectors
template <typename T>
__device__ __attribute__((always_inline)) inline T dotw(const T *W, const T *x, const int N)
{
    using V = typename V16<T>::type;
    constexpr int e = E<T>();
    T a = 0;
#pragma unroll
    for (int q = 0; q < (N + e - 1) / e; q++) {
        const V w = ((const V *)W)[q];
        const T *wp = (const T *)&w;
#pragma unroll
        for (int k = 0; k < e; k++)
            if (q * e + k < N) a += wp[k] * x[q * e + k];
    }
    return a;
}

// acc[i] += a W[i], i < N, W read as 16-byte vectors
template <typename T>
__device__ __attribute__((always_inline)) inline void axpyw(const T *W, const T a, T *acc, const int N)
{
    using V = typename V16<T>::type;
    constexpr int e = E<T>();
#pragma unroll
    for (int q = 0; q < (N + e - 1) / e; q++) {
        const V w = ((const V *)W)[q];
        const T *wp = (const T *)&w;
#pragma unroll
        for (int k = 0; k < e; k++)
            if (q * e + k < N) acc[q * e + k] += a * wp[k];
    }
}

// accumulator type of the LDS local expansions.  Shared mode: FP64 for both paths (LDS FP64
// atomic adds are much cheaper than FP32 ones here, and the FP32 path gains a wider sum).
// Ownership mode: plain adds in the working precision.
template <typename T, bool OWN>
struct AccT {
    using type = double;
};
template <typename T>
struct AccT<T, true> {
    using type = T;
};
template <typename T, bool OWN>
using Acc = typename AccT<T, OWN>::type;

// LDS accumulator of a target: the lane layout [role = 4 pot + 2 part + h][rs], one target
// every ss entries.  A wavefront instruction accumulates one entry for 8 targets x 8 roles;
// rs >= hoff(P) and ss >= 8 rs are the smallest paddings that spread those 64 addresses most
// evenly over 32 (first) and 64 (then) four-byte LDS banks
struct AccStride {
    int rs, ss;
};
constexpr int bank_load(int rs, int ss, int words, int nb)
{
    int cnt[64] = {};
    for (int t = 0; t < 8; t++)
        for (int r = 0; r < 8; r++)
            for (int k = 0; k < words; k++) cnt[((t * ss + r * rs) * words + k) % nb]++;
    int mx = 0;
    for (int b = 0; b < nb; b++) mx = cnt[b] > mx ? cnt[b] : mx;
    return mx;
}
constexpr AccStride acc_stride(int nh, int words)
{
    AccStride best{nh, 8 * nh + 1};
    int bc = 1 << 30;
    for (int d = 0; d <= 4; d++)
        for (int e = 1; e <= 20; e++) {
            const int rs = nh + d, ss = 8 * rs + e;
            const int c = (bank_load(rs, ss, words, 32) * 128 + bank_load(rs, ss, words, 64)) * 256 + 8 * d + e;
            if (c < bc) {
                bc = c;
                best = AccStride{rs, ss};
            }
        }
    return best;
}
template <typename T, int P, bool OWN>
constexpr AccStride acc_stride()
{
    return acc_stride(hoff(P), (int)sizeof(Acc<T, OWN>) / 4);
}
// entries per target slot.  Ownership mode keeps the packed order ([pot][P^2 + 1], odd slot
// stride), which is 15-20% smaller: at FP32 p = 10 it lets four workgroups share a compute
// unit instead of three (M2L on the 2^20 cube 25.3 against 26.6 ms)
template <typename T, int P, bool OWN>
constexpr int acc_slot()
{
    return OWN ? 2 * (P * P + 1) + 1 : acc_stride<T, P, OWN>().ss;
}
// position inside a slot of packed index k (0 <= k < 2 P^2)
template <int P, bool OWN, int RS>
__device__ inline int acc_pos(int k)
{
    if constexpr (OWN) return k >= P * P ? k + 1 : k;
    else return entry_lane<P, RS>(k);
}

// LDS footprint of a tile of NPAR sibling groups
template <typename T, int P, bool OWN>
constexpr size_t tile_bytes(int npar)
{
    using Sh = Shape<T, P>;
    const int nslot = half_tiles<T, P>() ? 4 : 8 * npar;
    return sizeof(T) * (size_t)staged_tables<T, P>() * Sh::WHS +
           sizeof(Acc<T, OWN>) * (size_t)(nslot + 1) * acc_slot<T, P, OWN>() + sizeof(int) * 3 * nslot +
           sizeof(int16_t) * (64 + (OWN ? 0 : 1512));
}
// two workgroups per compute unit (160 KB of LDS)
constexpr size_t LDS_HALF = 81920;
// ownership mode (FP32 p <= 10): one parent per wavefront; shared mode: the largest of 4, 2, 1
// parents that leaves room for two workgroups per compute unit
template <typename T, int P>
constexpr bool tile_own()
{
    return sizeof(T) == 4 && P <= 10;
}
// wavefronts per SIMD the register allocation aims at: two, except FP64 p = 16, whose 72-double
// part vectors need the whole register file (its tile leaves room for one workgroup anyway)
template <typename T, int P>
constexpr int min_waves()
{
    return (sizeof(T) == 8 && P > 12) ? 1 : 2;
}
template <typename T, int P>
constexpr int tile_npar()
{
    return tile_own<T, P>() ? 4
           : half_tiles<T, P>() ? 1
           : tile_bytes<T, P, false>(4) <= LDS_HALF ? 4 : (tile_bytes<T, P, false>(2) <= LDS_HALF ? 2 : 1);
}
// the scalar translations always run in shared mode (LDS atomics); the largest parent count
// that leaves room for two workgroups per compute unit
template <typename T, int P>
constexpr int tile_npar_sc()
{
    return tile_bytes<T, P, false>(4) <= LDS_HALF ? 4 : (tile_bytes<T, P, false>(2) <= LDS_HALF ? 2 : 1);
}
// tiles of one level: NPAR sibling groups each, or half a sibling group each
template <typename T, int P, int NPAR>
constexpr int64_t n_tiles(int64_t npar)
{
    return half_tiles<T, P>() ? 2 * npar : (npar + NPAR - 1) / NPAR;
}

}  // namespace hv

// NPAR sibling groups per tile.  OWN = false: shared by the four wavefronts, which walk each
// class's entry list 32 translations at a time and accumulate with LDS atomics.  OWN = true
// (NPAR = 4): wavefront w owns sibling group w and walks the class's rows of 8 (one column
// per child position), so the 8 translations of a batch hit 8 distinct targets that no other
// lane touches: accumulation is a plain LDS read-add-write.
// Tiles without any child box leave at once; a wavefront skips batches with no active lane.
// SC (scalar harmonic FMM, p <= 16, shared mode): only the potential phi is translated, without
// conversion (chi is absent); the lanes of the other potential carry a second translation, so a
// wavefront runs 16 translations per batch, and the sources come in the four-role scalar lane
// layout.
template <typename T, int P, int NPAR, bool OWN, bool SC = false>
__global__ void __launch_bounds__(256, (hv::min_waves<T, P>())) k_m2l_half(int level, int64_t poff, int64_t npar,
                                                  const uint64_t *__restrict__ bkey,
                                                  const int32_t *__restrict__ bchild0,
                                                  const int32_t *__restrict__ bnchild,
                                                  const int32_t *__restrict__ dmap, const T *__restrict__ Mh,
                                                  int64_t soff, T *__restrict__ Lc, const T *__restrict__ wh,
                                                  int64_t wstride, M2LSched sch,
                                                  const int16_t *__restrict__ cls_theta,
                                                  const double *__restrict__ dtab)
{
    using Sh = hv::Shape<T, P>;
    using hv::hoff;
    using hv::S;
    constexpr int P2 = Sh::P2, NH = Sh::NH, NHP = Sh::NHP;
    constexpr int ARS = hv::acc_stride<T, P, OWN>().rs, SSTA = hv::acc_slot<T, P, OWN>();
    constexpr bool HT = hv::half_tiles<T, P>();       // half a sibling group per tile, forward tables only
    constexpr bool GW = HT;                           // vectors fill the register file (see the coax)
    constexpr int NSLOT = HT ? 4 : 8 * NPAR;
    constexpr int NENT = 1512;  // schedule entries of one sibling group
    extern __shared__ char smem[];
    using A = hv::Acc<T, OWN>;
    static_assert(!OWN || NPAR == 4, "ownership mode: one sibling group per wavefront");
    static_assert(!HT || (NPAR == 1 && !OWN), "half tiles: shared mode, one parent");
    static_assert(!SC || (!HT && !OWN), "scalar translations: orders up to 16, shared mode");
    constexpr int NROLE = SC ? 4 : 8;      // lane roles of one translation
    constexpr int NPOT = SC ? 1 : 2;       // potentials in the target slots
    T *Wl = (T *)smem;                                // [kind: fwd S, back R][part][parity][WHS]
    A *acc = (A *)(Wl + hv::staged_tables<T, P>() * Sh::WHS);  // [NSLOT + 1][SSTA] (last slot absorbs)
    int *slot_xyz = (int *)(acc + (NSLOT + 1) * SSTA);  // [NSLOT] packed target coordinates, -1: no box
    int *slot_box = slot_xyz + NSLOT;                 // [NSLOT] target box
    int *slot_sys = slot_box + NSLOT;                 // [NSLOT] system of the target
    int16_t *cst = (int16_t *)(slot_sys + NSLOT);     // [ncls + 1] class starts
    int16_t *ent = cst + 64;                          // [NENT] (dir << 3) | child position

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware tile order: consecutive tiles stay on one XCD (shared L2)
    const int64_t ntiles = hv::n_tiles<T, P, NPAR>(npar);
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int ncls = sch.ncls;
    const int hf = HT ? (int)(tile & 1) : 0;  // half tiles: children 4 hf .. 4 hf + 3

    int has_box = 0;
    if (tid < NSLOT) {
        const int i = HT ? 0 : tid >> 3, c = HT ? 4 * hf + tid : tid & 7;
        int box = -1, xyz = -1, sys = 0;
        const int64_t q = HT ? (tile >> 1) : (int64_t)NPAR * tile + i;
        if (q < npar) {
            const int64_t pb = poff + q;
            const int c0 = bchild0[pb], nc = bnchild[pb];
            for (int k = 0; k < nc; k++)
                if ((int)(bkey[c0 + k] & 7u) == c) box = c0 + k;
        }
        if (box >= 0) {
            const uint64_t key = bkey[box];
            uint32_t ix = 0, iy = 0, iz = 0;
            for (int b = 0; b < level; b++) {
                ix |= (uint32_t)((key >> (3 * b)) & 1u) << b;
                iy |= (uint32_t)((key >> (3 * b + 1)) & 1u) << b;
                iz |= (uint32_t)((key >> (3 * b + 2)) & 1u) << b;
            }
            xyz = (int)(ix | (iy << 10) | (iz << 20));
            sys = (int)(key >> (3 * level));
        }
        slot_box[tid] = box;
        slot_xyz[tid] = xyz;
        slot_sys[tid] = sys;
        has_box = box >= 0;
    }
    // a tile whose parents have no children (leaves of an adaptive tree) has nothing to do
    if (!__syncthreads_or(has_box)) return;
    if constexpr (HT) {
        // the class entries of this half, compacted per class: (dir << 3) | slot (child - 4 hf)
        if (tid < ncls) {
            int cnt = 0;
            for (int e = sch.cls_start[tid]; e < sch.cls_start[tid + 1]; e++) cnt += (sch.ent_c[e] >> 2) == hf;
            cst[tid + 1] = (int16_t)cnt;
        }
        __syncthreads();
        if (tid == 0) {
            cst[0] = 0;
            for (int k = 0; k < ncls; k++) cst[k + 1] = (int16_t)(cst[k] + cst[k + 1]);
        }
        __syncthreads();
        if (tid < ncls) {
            int o = cst[tid];
            for (int e = sch.cls_start[tid]; e < sch.cls_start[tid + 1]; e++)
                if ((sch.ent_c[e] >> 2) == hf) ent[o++] = (int16_t)((sch.ent_dir[e] << 3) | (sch.ent_c[e] & 3));
        }
    } else {
        if (!OWN)
            for (int i = tid; i < NENT; i += 256) ent[i] = (int16_t)((sch.ent_dir[i] << 3) | sch.ent_c[i]);
        for (int i = tid; i <= ncls; i += 256) cst[i] = OWN ? sch.row_start[i] : sch.cls_start[i];
    }
    __syncthreads();
    // local expansions of the targets into their slots (shared mode: the lane layout, whose
    // entries without an (n, m) start at zero and are never read back)
    for (int idx = tid; idx < NSLOT * SSTA; idx += 256) acc[idx] = (A)0;
    __syncthreads();
    for (int idx = tid; idx < NSLOT * NPOT * P2; idx += 256) {
        const int sl = idx / (NPOT * P2), r = idx % (NPOT * P2);
        const int box = slot_box[sl];
        if (box >= 0) acc[sl * SSTA + hv::acc_pos<P, OWN, ARS>(r)] = (A)Lc[(size_t)box * 2 * P2 + r];
    }

    const int side = 1 << level;
    const int t = lane >> 3, pot = SC ? 0 : (lane >> 2) & 1, part = (lane >> 1) & 1, h = lane & 1;
    const int t2 = SC ? (lane >> 2) & 1 : 0;  // scalar: second translation of the lane group

    struct Job {
        int slot, dir, src;
    };
    // translation tr of class k (8 per wavefront and batch): (slot, dir) from LDS, source by one load
    auto setup = [&](int k, int r0) -> Job {
        Job j{NSLOT, 0, -1};
        if (k >= ncls) return j;
        int dir, slot;
        if (OWN) {
            // row r0 of class k; column t = child position of the wavefront's sibling group
            dir = sch.rows[(size_t)(cst[k] + r0) * 8 + t];
            if (dir < 0) return j;
            slot = wave * 8 + t;
        } else {
            const int e0 = cst[k], cnt = cst[k + 1] - e0;
            const int tr = r0 + (SC ? wave * 16 + 2 * t + t2 : wave * 8 + t);
            if (tr >= NPAR * cnt) return j;
            const int code = ent[e0 + tr / NPAR];
            dir = code >> 3;
            slot = (tr % NPAR) * 8 + (code & 7);
        }
        const int xyz = slot_xyz[slot];
        if (xyz < 0) return j;
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        if (sx < 0 || sy < 0 || sz < 0 || sx >= side || sy >= side || sz >= side) return j;
        const int src = dmap[(((size_t)slot_sys[slot] * side + sz) * side + sy) * side + sx];
        if (src < 0) return j;
        j.slot = slot;
        j.dir = dir;
        j.src = src;
        return j;
    };
    auto advance = [&](int &k, int &r0) {
        r0 += (OWN ? 1 : 32) * (SC ? 2 : 1);
        if (k < ncls && r0 >= (OWN ? 1 : NPAR) * (cst[k + 1] - cst[k])) {
            k++;
            r0 = 0;
        }
    };
    // this lane's entries of the source (order n, m = 2j + h; zeros where m > n or (Im, m = 0)),
    // stored contiguously per lane role by k_mhalf: whole 16-byte vectors from one address
    auto load_part = [&](const Job &j, T *dst) {
        using V = typename hv::V16<T>::type;
        constexpr int e = hv::E<T>();
        const V *sp =
            (const V *)(Mh + ((size_t)(j.src >= 0 ? j.src - soff : 0) * NROLE + (lane & (NROLE - 1))) * NHP);
#pragma unroll
        for (int q = 0; q < NHP / e; q++) {
            const V x = sp[q];
            const T *xp = (const T *)&x;
#pragma unroll
            for (int k = 0; k < e; k++)
                if (q * e + k < NH) dst[q * e + k] = xp[k];
        }
    };

    int k = 0, r0 = 0;   // current batch
    int k1 = 0, r1 = 0;  // next batch
    advance(k1, r1);
    Job cur = setup(k, r0), nxt = setup(k1, r1);
    // the rotation tables of one class, staged in LDS with 16-byte loads.  Where registers
    // allow, a batch whose successor starts a new class loads the new tables into registers
    // first, so that they arrive during the batch and only the LDS write sits between the
    // two barriers of the class change
    constexpr int N16 = (int)(hv::staged_tables<T, P>() * Sh::WHS * sizeof(T) / 16);
    constexpr bool PREF = hv::min_waves<T, P>() > 1;
    constexpr int NPF = PREF ? (N16 + 255) / 256 : 1;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 pf[NPF];
    auto fetch = [&](int kc) __attribute__((always_inline)) {
        const u32x4 *src4 = (const u32x4 *)(wh + (size_t)cls_theta[kc] * wstride);
#pragma unroll
        for (int q = 0; q < NPF; q++) pf[q] = src4[q * 256 + tid < N16 ? q * 256 + tid : 0];
    };
    int staged = -1, fetched = -1;
    while (k < ncls) {
        if (k != staged) {
            __syncthreads();
            uint4 *dst4 = (uint4 *)Wl;
            if constexpr (PREF) {
                if (fetched != k) fetch(k);
#pragma unroll
                for (int q = 0; q < NPF; q++)
                    if (tid + 256 * q < N16) ((u32x4 *)dst4)[tid + 256 * q] = pf[q];
            } else {
                const uint4 *src4 = (const uint4 *)(wh + (size_t)cls_theta[k] * wstride);
#pragma unroll 4
                for (int i = tid; i < N16; i += 256) dst4[i] = src4[i];
            }
            __syncthreads();
            staged = k;
        }
        // ownership mode: the lane's role (parity, part, potential) is made opaque per batch, so
        // the compiler recomputes the per-lane constants derived from it instead of holding
        // them all in registers (FP32 p = 10: 143 -> 107 VGPRs, 30.4 -> 27.2 ms on the 2^20
        // cube); in shared mode that trade costs SGPR spills and time
        const int wo = (part * 2 + h) * Sh::WHS;
        int hh = h, pp = part, po = pot;
        if (OWN) asm volatile("" : "+v"(hh), "+v"(pp), "+v"(po));
        const T *Wf = Wl + wo;
        const T *Wb = Wl + (HT ? (pp * 2 + 1 - hh) * Sh::WHS : 4 * Sh::WHS + wo);  // HT: the partner's forward table

        const Job j = cur;
        const bool act = j.src >= 0;
        // look one batch further ahead: its source index now
        int k2 = k1, r2 = r1;
        advance(k2, r2);
        const Job nn = setup(k2, r2);
        if constexpr (PREF) {
            if (k1 != k && k1 < ncls) {  // the next batch starts a new class
                fetch(k1);
                fetched = k1;
            }
        }
        if (__ballot(act) != 0ull) {  // wavefront-uniform: skip batches with no active lane
        T v[NH];
        load_part(j, v);

        // |t|, 1/|t| and e^{i phi} of the direction, from the plan's table (FP64)
        const double2 d0 = ((const double2 *)dtab)[2 * j.dir], d1 = ((const double2 *)dtab)[2 * j.dir + 1];
        const T tau = (T)d0.x, itau = (T)d0.y;
        const double cph = d1.x, sph = d1.y;
        const double c2 = cph * cph - sph * sph, s2 = 2.0 * cph * sph;  // e^{2 i phi}
        // 1. rotate about z by +phi: Re' = re c - im s, Im' = im c + re s (m = 2j + h)
        {
            const T sgn = pp ? (T)1 : (T)-1;
            double cm = hh ? cph : 1.0, sm = hh ? sph : 0.0;
#pragma unroll
            for (int jj = 0; jj < (P + 1) / 2; jj++) {
                const T cz = (T)cm, sz = (T)sm * sgn;
#pragma unroll
                for (int n = 2 * jj; n < P; n++) {
                    const T x = v[hoff(n) + jj];
                    const T o = dpp_f<DPP_XOR2>(x);
                    v[hoff(n) + jj] = x * cz + o * sz;
                }
                const double a = cm * c2 - sm * s2, b = sm * c2 + cm * s2;
                cm = a;
                sm = b;
            }
        }
        // 2. and 5. rotation about y of every order: partial sums over the lane's columns for
        //    its own rows (o) and its partner's rows (t), then o + partner's t
        auto rotate_y = [&](const T *W) __attribute__((always_inline)) {
#pragma unroll
            for (int n = 0; n < P; n++) {
                const T *Wn = W + hv::woff<T>(n);
                constexpr int SM = P / 2 + 1;
                T o[SM], tt[SM];
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    o[jj] = hv::dotw<T>(Wn + jj * hv::RL<T>(n), &v[hoff(n)], S(n));
                    tt[jj] = hv::dotw<T>(Wn + (S(n) + jj) * hv::RL<T>(n), &v[hoff(n)], S(n));
                    // at one wavefront per SIMD (FP64 p = 16) finish each pair of rows before the
                    // next: 251 against 329 ms of M2L on the 4M ring; elsewhere the scheduler's
                    // own interleaving is faster
                    if constexpr (hv::min_waves<T, P>() == 1) asm volatile("" : "+v"(o[jj]), "+v"(tt[jj]));
                }
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) v[hoff(n) + jj] = o[jj] + dpp_f<DPP_XOR1>(tt[jj]);
            }
        };
        rotate_y(Wf);
        // 3+4. per column m = 2c + h: coaxial (S|R) shift out_n = tau^-(n+1) sum_n' (n+n')! tau^-n' in_n'
        //      (chi to order P), then the R-conversion (eq. rcr1, scaled)
        //        phi~ = phi + i tau m/n chi ,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
        {
            // tau^-k: a table at the orders whose registers allow it; running products where the
            // vectors fill the register file (global-table mode)
            constexpr int NPW = GW ? 1 : P + 2;
            T pw[NPW];
            pw[0] = (T)1;
#pragma unroll
            for (int q = 1; q < NPW; q++) pw[q] = pw[q - 1] * itau;
            T pc = (T)1;  // GW: tau^-(2c) of the current column
            const T itau2 = itau * itau;
            const T wphi = po ? (T)0 : (T)1, wchi = po ? (T)1 : (T)0;
            const T sconv = pp ? (T)1 : (T)-1;
            const T keep0 = hh ? (T)0 : (T)1;  // slot (n = 2c, c) holds m = 2c + h: empty on odd lanes
#pragma unroll
            for (int c = 0; c < (P + 1) / 2; c++) {
                const int n0 = 2 * c;
                const T mval = (T)(2 * c + hh);
                T out[P + 1];
                if constexpr (GW) {
                    // scale the column in place, then the Hankel sums
                    T q = pc;
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) {
                        v[hoff(n2) + c] *= q;
                        q *= itau;
                    }
                    T qo = pc * itau;
#pragma unroll
                    for (int n = n0; n <= (SC ? P - 1 : P); n++) {
                        T a = 0;
#pragma unroll
                        for (int n2 = n0; n2 < P; n2++) a += (T)dfact(n + n2) * v[hoff(n2) + c];
                        out[n] = a * qo;
                        qo *= itau;
                    }
                    pc *= itau2;
                } else {
                    T cl[P];
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) cl[n2] = v[hoff(n2) + c] * pw[n2];
#pragma unroll
                    for (int n = n0; n <= (SC ? P - 1 : P); n++) {
                        T a = 0;
#pragma unroll
                        for (int n2 = n0; n2 < P; n2++) a += (T)dfact(n + n2) * cl[n2];
                        out[n] = a * pw[n + 1];
                    }
                }
#pragma unroll
                for (int n = n0; n < P; n++) {
                    T val;
                    if constexpr (SC) {
                        val = out[n];  // a single potential: no conversion
                    } else {
                        const T other = swz_xor<6>(out[n]);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                        const T fphi = (n > 0) ? tau * mval * (T)(1.0 / (double)n) * sconv * wphi : (T)0;
                        const T fchi = -tau * (T)(1.0 / (double)(n + 1)) * wchi;
                        val = out[n] + fphi * other + fchi * out[n + 1];
                    }
                    if (n == n0) val *= keep0;
                    v[hoff(n) + c] = val;
                }
                // FP32 and FP64 p = 16: one column at a time (FP32 p = 16 on the 4M ring: 107 ms
                // with this fence, 109 ms without); FP64 p = 12 gains from interleaving columns
                // with the y-rotations' LDS reads (2^20 cube: 59.3 -> 50.4 ms without it)
                if constexpr (sizeof(T) == 4 || hv::min_waves<T, P>() == 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
        if constexpr (HT) {
            // 5. back-rotation with the forward tables: v <- D W_fwd^T D^-1 v.  The lane's inputs
            //    (m = 2j + h) scale by D^-1 and multiply rows j of its own table's o block (outputs of
            //    its parity) and of the partner table's t block (outputs of the other parity); the
            //    partner's partial sums arrive by the DPP pair swap, then D scales the outputs
            const T sg = hh ? (T)-1 : (T)1;  // (-1)^m on this lane
            const T fin = pp ? sg : (T)2 * sg, fout = pp ? sg : (T)0.5 * sg;
#pragma unroll
            for (int n = 0; n < P; n++) {
                const T *Won = Wf + hv::woff<T>(n);
                const T *Wpn = Wb + hv::woff<T>(n) + S(n) * hv::RL<T>(n);
                constexpr int SM = P / 2 + 1;
                T o[SM], tt[SM];
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    o[jj] = 0;
                    tt[jj] = 0;
                }
#pragma unroll
                for (int j = 0; j < S(n); j++) {
                    // m = 0 (j = 0 on even lanes, Re part) is not doubled by D^-1
                    const T xj = v[hoff(n) + j] * ((j == 0 && !hh && !pp) ? (T)1 : fin);
                    hv::axpyw<T>(Won + j * hv::RL<T>(n), xj, o, S(n));
                    hv::axpyw<T>(Wpn + j * hv::RL<T>(n), xj, tt, S(n));
                }
#pragma unroll
                for (int jj = 0; jj < S(n); jj++)
                    v[hoff(n) + jj] = (o[jj] + dpp_f<DPP_XOR1>(tt[jj])) * ((jj == 0 && !hh && !pp) ? (T)1 : fout);
            }
        } else {
            rotate_y(Wb);
        }
        // 6. back-rotation about z (-phi) and accumulation into the target slot (inactive lanes
        //    add into the spare slot; in ownership mode so do entries without an (n, m))
        {
            A *ap = acc + (size_t)(act ? j.slot : NSLOT) * SSTA + (OWN ? po * (P2 + 1) : (lane & (NROLE - 1)) * ARS);
            A *spare = acc + (size_t)NSLOT * SSTA + (OWN ? po * (P2 + 1) : 0);
            const T sgn = pp ? (T)-1 : (T)1;  // Re' = re c + im s, Im' = im c - re s
            double cm = hh ? cph : 1.0, sm = hh ? sph : 0.0;
#pragma unroll
            for (int jj = 0; jj < (P + 1) / 2; jj++) {
                const T cz = (T)cm, sz = (T)sm * sgn;
                {
                    const double a = cm * c2 - sm * s2, b = sm * c2 + cm * s2;
                    cm = a;
                    sm = b;
                }
                const int m = 2 * jj + hh;
#pragma unroll
                for (int n = 2 * jj; n < P; n++) {
                    const T x = v[hoff(n) + jj];
                    const T o = dpp_f<DPP_XOR2>(x);
                    const T val = x * cz + o * sz;
                    if constexpr (OWN) {
                        const bool ok = m <= n && !(pp && m == 0);
                        const int off = n * n + (pp ? n : 0) + m;  // < P^2 also where !ok
                        *((ok ? ap : spare) + off) += (A)val;
                    } else {
                        atomicAdd(ap + hoff(n) + jj, (A)val);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        }  // active batch

        cur = nxt;
        nxt = nn;
        k = k1;
        r0 = r1;
        k1 = k2;
        r1 = r2;
    }
    __syncthreads();
    for (int idx = tid; idx < NSLOT * NPOT * P2; idx += 256) {
        const int sl = idx / (NPOT * P2), r = idx % (NPOT * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + r] = (T)acc[sl * SSTA + hv::acc_pos<P, OWN, ARS>(r)];
    }
}

// the sources of one level in the lane layout of the half-vector M2L: box b of the level at
// Mh[(b * 8 + role) * NHP], role = 4 pot + 2 part + h (the lane's low three bits), entry
// hoff(n) + j = order n, m = 2j + h of that potential and part; zero where m > n, for (Im, m = 0)
// and in the padding
template <typename T, int P, int NR = 8>
__global__ void __launch_bounds__(256) k_mhalf(int64_t off, int64_t nb, const T *__restrict__ M, T *__restrict__ Mh)
{
    using Sh = hv::Shape<T, P>;
    constexpr int NHP = Sh::NHP, NH = Sh::NH, NE = NR * NHP, P2 = P * P;  // NR = 4: phi only (scalar)
    // packed index of every lane-layout entry of a box (-1: zero)
    __shared__ int16_t src[NE];
    for (int t = threadIdx.x; t < NE; t += blockDim.x) {
        const int r = t / NHP, e = t % NHP;
        const int pot = r >> 2, part = (r >> 1) & 1, h = r & 1;
        int k = -1;
        if (e < NH) {
            int n = 0;
            while (hv::hoff(n + 1) <= e) n++;
            const int m = 2 * (e - hv::hoff(n)) + h;
            if (m <= n && !(part && m == 0)) k = pot * P2 + n * n + (part ? n : 0) + m;
        }
        src[t] = (int16_t)k;
    }
    __syncthreads();
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const T *mb = M + (size_t)(off + b) * 2 * P2;
        T *hb = Mh + (size_t)b * NE;
        for (int t = threadIdx.x; t < NE; t += blockDim.x) {
            const int k = src[t];
            hb[t] = k >= 0 ? mb[k] : (T)0;
        }
    }
}

// per direction code d = (dz + 3) 49 + (dy + 3) 7 + dx + 3 of a translation t = (dx, dy, dz) (in
// box sides): |t|, 1/|t| and e^{i phi} = (dx + i dy)/sqrt(dx^2 + dy^2) (1 on the z axis), FP64
__global__ void k_dirtab(double *__restrict__ tab)
{
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= 343) return;
    const int dx = d % 7 - 3, dy = (d / 7) % 7 - 3, dz = d / 49 - 3;
    const double tau = sqrt((double)(dx * dx + dy * dy + dz * dz));
    const double rho = sqrt((double)(dx * dx + dy * dy));
    tab[4 * d + 0] = tau;
    tab[4 * d + 1] = tau > 0.0 ? 1.0 / tau : 0.0;
    tab[4 * d + 2] = rho > 0.0 ? (double)dx / rho : 1.0;
    tab[4 * d + 3] = rho > 0.0 ? (double)dy / rho : 0.0;
}

// Rotation tables of every polar-angle class in the half-vector layout:
// [kind: forward S, backward R][part: Re, Im][parity h][order n][o rows, t rows][RL(n)]
// (each table padded to WHS entries),
// row j of o is m' = 2j + h, row j of t is m' = 2j + 1 - h, column i is m = 2i + h; the Im
// block (m, m' >= 1) is embedded with zeros at m = 0 and m' = 0; zero where m or m' > n.
template <typename T, int P>
__global__ void k_whalf(const T *__restrict__ rot, T *__restrict__ wh, int64_t stride, int kind_f, int kind_b)
{
    using Sh = hv::Shape<T, P>;
    const int th = blockIdx.x;
    const int RS = rot_set_size(P);
    const T *Rf = rot + ((size_t)th * ROT_NKIND + kind_f) * RS;
    const T *Rb = rot + ((size_t)th * ROT_NKIND + kind_b) * RS;
    for (int idx = threadIdx.x; idx < stride; idx += blockDim.x) {
        T val = (T)0;
        const int tb = idx / Sh::WHS, e = idx % Sh::WHS;
        const int kind = tb >> 2, part = (tb >> 1) & 1, h = tb & 1;
        if (e >= Sh::WH) {
            wh[(size_t)th * stride + idx] = val;
            continue;
        }
        int n = 0;
        while (hv::woff<T>(n + 1) <= e) n++;
        const int r = e - hv::woff<T>(n), row = r / hv::RL<T>(n), i = r % hv::RL<T>(n);
        const int ot = row / hv::S(n), jr = row % hv::S(n);
        const int mp = 2 * jr + (ot ? 1 - h : h), m = 2 * i + h;
        if (i < hv::S(n) && mp <= n && m <= n) {
            const T *blk = (kind ? Rb : Rf) + rot_block_off(n);
            if (part == 0) val = blk[mp * (n + 1) + m];
            else if (mp > 0 && m > 0) val = blk[(n + 1) * (n + 1) + (mp - 1) * n + (m - 1)];
        }
        wh[(size_t)th * stride + idx] = val;
    }
}

// ---------------------------------------------------------------------------
// M2M and L2L in the same half-vector layout.  One wavefront per parent box; its 64 lanes are
//   lane = 8 c + 4 pot + 2 part + h      (c: octant of the child)
// so the eight child translations of the parent run side by side.  Their directions use two
// polar-angle classes (the z bit of the octant), staged once per workgroup.  Coaxial shift
// (S|S for M2M, R|R for L2L) and conversion (S for M2M, R for L2L, eq. rcr1 and its S form)
// act column by column inside the lane, as in the M2L kernel.  M2M sums the eight results over
// c (lane butterfly) into the parent's multipole; L2L writes each child's local expansion.
// KIND 0 = M2M (child -> parent), 2 = L2L (parent -> child); the coefficients are those of the
// generic per-box kernels: cf_k = (-tau_p)^k / k!, tau_p = sqrt(3)/4, conversion tau sqrt(3)/4
// (M2M) and sqrt(3)/2 (L2L).
// ---------------------------------------------------------------------------
namespace hv {
// class stride in LDS: eight tables plus 64 bytes, so the two classes' tables read together
// fall in different banks
template <typename T, int P>
constexpr int mm_cstride()
{
    return 8 * Shape<T, P>::WHS + 64 / (int)sizeof(T);
}
template <typename T, int P>
constexpr size_t mm_bytes()
{
    return sizeof(T) * 2 * (size_t)mm_cstride<T, P>();
}
__host__ __device__ constexpr double taup() { return 0.4330127018922193; }  // sqrt(3)/4
// (-tau_p)^k / k! as a compile-time constant
__host__ __device__ constexpr double mm_cf(int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; i++) c *= -taup() / (double)i;
    return c;
}
}  // namespace hv

// the value of lane ^ 32 (v_permlane32_swap of the value with itself: the two results sum to
// the lane's value plus its partner's)
__device__ inline float xor32_sum(float v)
{
    const unsigned u = __float_as_uint(v);
    const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline double xor32_sum(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)(u & 0xffffffffull), hi = (unsigned)(u >> 32);
    const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const double a = __longlong_as_double((long long)(((unsigned long long)rh[0] << 32) | rl[0]));
    const double b = __longlong_as_double((long long)(((unsigned long long)rh[1] << 32) | rl[1]));
    return a + b;
}

template <typename T, int P, int KIND>
__global__ void __launch_bounds__(256, (hv::min_waves<T, P>())) k_mm_half(int64_t poff, int64_t npar,
                                                                        const int32_t *__restrict__ bchild0,
                                                                        const int32_t *__restrict__ bnchild,
                                                                        const uint64_t *__restrict__ bkey,
                                                                        const T *__restrict__ src_exp,
                                                                        T *__restrict__ dst_exp,
                                                                        const T *__restrict__ wtab, int64_t wstride,
                                                                        const int16_t *__restrict__ dir_theta,
                                                                        const T *__restrict__ zph)
{
    static_assert(KIND == 0 || KIND == 2, "M2M or L2L");
    using Sh = hv::Shape<T, P>;
    using hv::hoff;
    using hv::S;
    constexpr int P2 = Sh::P2, NH = Sh::NH, CST = hv::mm_cstride<T, P>();
    constexpr int DIR0 = NDIR_M2L + (KIND == 0 ? 0 : 8);  // child->parent (M2M), parent->child (L2L)
    extern __shared__ char smem[];
    T *Wl = (T *)smem;  // [class: z bit 0, 1][kind: fwd, back][part][parity][WHS]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = 0; k < 2; k++) {
        const int cls = dir_theta[DIR0 + 4 * k];
        const uint4 *s4 = (const uint4 *)(wtab + (size_t)cls * wstride);
        uint4 *d4 = (uint4 *)(Wl + k * CST);
        constexpr int N16 = (int)(8 * Sh::WHS * sizeof(T) / 16);
        for (int i = tid; i < N16; i += 256) d4[i] = s4[i];
    }
    __syncthreads();

    const int c = lane >> 3, pot = (lane >> 2) & 1, part = (lane >> 1) & 1, h = lane & 1;
    const int dir = DIR0 + c;

    for (int64_t q = (int64_t)blockIdx.x * 4 + wave; q < npar; q += (int64_t)gridDim.x * 4) {
        // opaque per-parent offsets: keep the compiler from hoisting the loop-invariant rotation
        // entries and phases out of the parent loop (which would exhaust the register file)
        int wo = (c >> 2) * CST + (part * 2 + h) * Sh::WHS, zo = dir * 2 * P + h, hh = h, pp = part, po = pot;
        asm volatile("" : "+v"(wo), "+v"(zo), "+v"(hh), "+v"(pp), "+v"(po));
        const T *Wf = Wl + wo;
        const T *Wb = Wf + 4 * Sh::WHS;
        const T *zc = zph + zo, *zs = zc + P;  // cos, sin of m phi at m = 2j + h: zc[2j], zs[2j]
        const int64_t b = poff + q;
        const int nc = bnchild[b];
        if (nc == 0) continue;  // M2M: a leaf keeps its own multipole; L2L: nothing below
        const int c0 = bchild0[b];
        int cb = -1;
        for (int k = 0; k < nc; k++)
            if ((int)(bkey[c0 + k] & 7u) == c) cb = c0 + k;
        const bool act = cb >= 0;
        const T *sp = src_exp + (size_t)(KIND == 0 ? (act ? cb : 0) : b) * 2 * P2 + po * P2;
        T v[NH];
#pragma unroll
        for (int n = 0; n < P; n++)
#pragma unroll
            for (int jj = 0; jj < S(n); jj++) {
                const int m = 2 * jj + hh;
                const bool ok = act && m <= n && !(pp && m == 0);
                const T x = sp[ok ? n * n + pp * n + m : 0];
                v[hoff(n) + jj] = ok ? x : (T)0;
            }
        // 1. rotate about z by +phi: Re' = re c - im s, Im' = im c + re s
        {
            const T sgn = pp ? (T)1 : (T)-1;
#pragma unroll
            for (int jj = 0; jj < P / 2; jj++) {
                const T cj = zc[2 * jj], sj = zs[2 * jj] * sgn;
#pragma unroll
                for (int n = 2 * jj; n < P; n++) {
                    const T x = v[hoff(n) + jj];
                    const T o = dpp_f<DPP_XOR2>(x);
                    v[hoff(n) + jj] = x * cj + o * sj;
                }
            }
        }
        auto rotate_y = [&](const T *W) __attribute__((always_inline)) {
#pragma unroll
            for (int n = 0; n < P; n++) {
                const T *Wn = W + hv::woff<T>(n);
                constexpr int SM = P / 2 + 1;
                T o[SM], tt[SM];
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    o[jj] = hv::dotw<T>(Wn + jj * hv::RL<T>(n), &v[hoff(n)], S(n));
                    tt[jj] = hv::dotw<T>(Wn + (S(n) + jj) * hv::RL<T>(n), &v[hoff(n)], S(n));
                    asm volatile("" : "+v"(o[jj]), "+v"(tt[jj]));
                }
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) v[hoff(n) + jj] = o[jj] + dpp_f<DPP_XOR1>(tt[jj]);
            }
        };
        rotate_y(Wf);
        // 3+4. per column m = 2c' + h: coaxial shift, then the conversion
        {
            const T wphi = po ? (T)0 : (T)1, wchi = po ? (T)1 : (T)0;
            const T keep0 = hh ? (T)0 : (T)1;  // slot (n = 2c', c') holds m = 2c' + h: empty on odd lanes
#pragma unroll
            for (int cc = 0; cc < P / 2; cc++) {
                const int n0 = 2 * cc;
                const T mval = (T)(2 * cc + hh);
                T in[P];
#pragma unroll
                for (int n2 = n0; n2 < P; n2++) in[n2] = v[hoff(n2) + cc];
                T out[P];
                if (KIND == 0) {
                    // (S|S): out_n = sum_{n' = m}^{n} cf_{n-n'} (1/2 [phi] | 1 [chi]) 2^-n' in_n'
                    const T s0 = po ? (T)1 : (T)0.5;
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) in[n2] *= (T)(1.0 / (double)(1ull << n2));
#pragma unroll
                    for (int n = n0; n < P; n++) {
                        T a = 0;
#pragma unroll
                        for (int n2 = n0; n2 <= n; n2++) a += (T)hv::mm_cf(n - n2) * in[n2];
                        out[n] = a * s0;
                    }
                } else {
                    // (R|R): out_n = (1 [phi] | 1/2 [chi]) 2^-n sum_{n' = n}^{p-1} cf_{n'-n} in_n'
                    const T s0 = po ? (T)0.5 : (T)1;
#pragma unroll
                    for (int n = n0; n < P; n++) {
                        T a = 0;
#pragma unroll
                        for (int n2 = n; n2 < P; n2++) a += (T)hv::mm_cf(n2 - n) * in[n2];
                        out[n] = a * (s0 * (T)(1.0 / (double)(1ull << n)));
                    }
                }
#pragma unroll
                for (int n = n0; n < P; n++) {
                    const T other = swz_xor<6>(out[n]);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                    T val;
                    if (KIND == 0) {
                        // S-conversion: phi~ = phi - i tau m/(n+1) chi,  chi~_n = chi_n + tau/n chi_{n-1}
                        const T tau = (T)hv::taup();
                        const T fphi = tau * mval * (T)(1.0 / (double)(n + 1)) * (pp ? (T)-1 : (T)1) * wphi;
                        const T prev = (n > n0) ? out[n - 1] : (T)0;
                        const T fchi = (n > 0) ? tau * (T)(1.0 / (double)n) * wchi : (T)0;
                        val = out[n] + fphi * other + fchi * prev;
                    } else {
                        // R-conversion: phi~ = phi + i tau m/n chi,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
                        const T tau = (T)(2.0 * hv::taup());
                        const T fphi =
                            (n > 0) ? tau * mval * (T)(1.0 / (double)n) * (pp ? (T)1 : (T)-1) * wphi : (T)0;
                        const T next = (n + 1 < P) ? out[n + 1] : (T)0;
                        const T fchi = -tau * (T)(1.0 / (double)(n + 1)) * wchi;
                        val = out[n] + fphi * other + fchi * next;
                    }
                    if (n == n0) val *= keep0;
                    v[hoff(n) + cc] = val;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        rotate_y(Wb);
        // 6. rotate about z by -phi: Re' = re c + im s, Im' = im c - re s
        {
            const T sgn = pp ? (T)-1 : (T)1;
#pragma unroll
            for (int jj = 0; jj < P / 2; jj++) {
                const T cj = zc[2 * jj], sj = zs[2 * jj] * sgn;
#pragma unroll
                for (int n = 2 * jj; n < P; n++) {
                    const T x = v[hoff(n) + jj];
                    const T o = dpp_f<DPP_XOR2>(x);
                    v[hoff(n) + jj] = x * cj + o * sj;
                }
            }
        }
        if (KIND == 0) {
            // sum over the eight children: lane butterfly over the octant bits (lane ^ 8, 16, 32)
#pragma unroll
            for (int q2 = 0; q2 < NH; q2++) {
                T x = v[q2];
                x += swz_xor<8>(x);
                x += swz_xor<16>(x);
                v[q2] = xor32_sum(x);
            }
            if (c == 0) {
                T *dp = dst_exp + (size_t)b * 2 * P2 + po * P2;
#pragma unroll
                for (int n = 0; n < P; n++)
#pragma unroll
                    for (int jj = 0; jj < S(n); jj++) {
                        const int m = 2 * jj + hh;
                        if (m <= n && !(pp && m == 0)) dp[n * n + pp * n + m] = v[hoff(n) + jj];
                    }
            }
        } else if (act) {
            T *dp = dst_exp + (size_t)cb * 2 * P2 + po * P2;
#pragma unroll
            for (int n = 0; n < P; n++)
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    const int m = 2 * jj + hh;
                    if (m <= n && !(pp && m == 0)) dp[n * n + pp * n + m] = v[hoff(n) + jj];
                }
        }
    }
}

// zero local expansions (level 2 has no parent expansion to shift)
template <typename T>
__global__ void k_zero_exp(int64_t count, T *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (T)0;
}

namespace {

template <typename T, int P>
static bool whalf_build_t(lhf_plan *Pl, hipStream_t st)
{
    constexpr int NPAR = hv::tile_npar<T, P>();
    constexpr bool OWN = hv::tile_own<T, P>();
    constexpr size_t shm = hv::tile_bytes<T, P, OWN>(NPAR);
    static_assert(shm <= 163840, "tile exceeds the LDS");
    const int64_t stride = 8 * (int64_t)hv::Shape<T, P>::WHS;
    if (dev_malloc(&Pl->whalf, sizeof(T) * stride * Pl->n_theta) != hipSuccess) return false;
    k_whalf<T, P><<<dim3((unsigned)Pl->n_theta), dim3(256), 0, st>>>((const T *)Pl->rot, (T *)Pl->whalf, stride,
                                                                      ROT_S_FWD, ROT_R_BACK);
    if (dev_malloc(&Pl->dtab, sizeof(double) * 4 * 343) != hipSuccess) return false;
    k_dirtab<<<dim3(2), dim3(256), 0, st>>>(Pl->dtab);
    // sources in the kernel's lane layout, one level at a time: room for the largest level
    int64_t nbmax = 0;
    for (int l = 2; l <= Pl->depth; l++) nbmax = std::max(nbmax, Pl->lev[l].nb);
    if (nbmax > 0 && dev_malloc(&Pl->mh, sizeof(T) * 8 * hv::Shape<T, P>::NHP * nbmax) != hipSuccess) return false;
    if constexpr (!hv::half_tiles<T, P>()) {
        constexpr int NPS = hv::tile_npar_sc<T, P>();
        if (hipFuncSetAttribute((const void *)k_m2l_half<T, P, NPS, false, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)hv::tile_bytes<T, P, false>(NPS)) != hipSuccess)
            return false;
    }
    return hipFuncSetAttribute((const void *)k_m2l_half<T, P, NPAR, OWN>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) == hipSuccess;
}

template <typename T, int P, bool SC = false>
static void launch_half(const lhf_plan *Pl, int level, hipStream_t st)
{
    // scalar translations: shared mode (two schedule rows per batch would share their targets)
    constexpr bool OWN = SC ? false : hv::tile_own<T, P>();
    constexpr int NPAR = SC ? hv::tile_npar_sc<T, P>() : hv::tile_npar<T, P>();
    const int64_t poff = Pl->lev[level - 1].off, npar = Pl->lev[level - 1].nb;
    const int64_t soff = Pl->lev[level].off, nb = Pl->lev[level].nb;
    if (nb == 0 || npar == 0) return;
    const int64_t ntiles = hv::n_tiles<T, P, NPAR>(npar);
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls, Pl->sched_row_start, Pl->sched_rows};
    k_m2l_half<T, P, NPAR, OWN, SC><<<dim3((unsigned)(per * 8)), dim3(256),
                                                          hv::tile_bytes<T, P, OWN>(NPAR),
                                                     st>>>(
        level, poff, npar, Pl->bkey, Pl->bchild0, Pl->bnchild, Pl->dmap[level], (const T *)Pl->mh, soff,
        (T *)Pl->Lc, (const T *)Pl->whalf, 8 * (int64_t)hv::Shape<T, P>::WHS, sch, Pl->sched_cls_theta, Pl->dtab);
}

// the sources of level l in the half-vector kernel's lane layout
template <typename T, int P, int NR = 8>
static void stage_half(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t nb = Pl->lev[level].nb;
    if (nb == 0) return;
    k_mhalf<T, P, NR><<<dim3((unsigned)std::min<int64_t>(nb, 8192)), dim3(256), 0, st>>>(
        Pl->lev[level].off, nb, (const T *)Pl->M, (T *)Pl->mh);
}

// rotation tables of the M2M (S basis both ways) and L2L (R basis both ways) shifts
template <typename T, int P>
static bool mmhalf_build_t(lhf_plan *Pl, hipStream_t st)
{
    const int64_t stride = 8 * (int64_t)hv::Shape<T, P>::WHS;
    if (dev_malloc(&Pl->wmm, sizeof(T) * stride * Pl->n_theta) != hipSuccess) return false;
    if (dev_malloc(&Pl->wll, sizeof(T) * stride * Pl->n_theta) != hipSuccess) return false;
    k_whalf<T, P><<<dim3((unsigned)Pl->n_theta), dim3(256), 0, st>>>((const T *)Pl->rot, (T *)Pl->wmm, stride,
                                                                      ROT_S_FWD, ROT_S_BACK);
    k_whalf<T, P><<<dim3((unsigned)Pl->n_theta), dim3(256), 0, st>>>((const T *)Pl->rot, (T *)Pl->wll, stride,
                                                                      ROT_R_FWD, ROT_R_BACK);
    constexpr size_t shm = hv::mm_bytes<T, P>();
    static_assert(shm <= 163840, "rotation tables exceed the LDS");
    return hipFuncSetAttribute((const void *)k_mm_half<T, P, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm) == hipSuccess &&
           hipFuncSetAttribute((const void *)k_mm_half<T, P, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm) == hipSuccess;
}

// KIND 0: M2M into the parents of level l; KIND 2: L2L from level l - 1 into level l (l >= 3)
template <typename T, int P, int KIND>
static void launch_mm(const lhf_plan *Pl, int l, hipStream_t st)
{
    const int lp = KIND == 0 ? l : l - 1;
    const int64_t poff = Pl->lev[lp].off, npar = Pl->lev[lp].nb;
    if (npar == 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((npar + 3) / 4, 2048);
    const T *src = (const T *)(KIND == 0 ? Pl->M : Pl->Lc);
    T *dst = (T *)(KIND == 0 ? Pl->M : Pl->Lc);
    k_mm_half<T, P, KIND><<<dim3(grid), dim3(256), hv::mm_bytes<T, P>(), st>>>(
        poff, npar, Pl->bchild0, Pl->bnchild, Pl->bkey, src, dst, (const T *)(KIND == 0 ? Pl->wmm : Pl->wll),
        8 * (int64_t)hv::Shape<T, P>::WHS, Pl->dir_theta, (const T *)Pl->zph);
}

template <typename T>
static void zero_level(const lhf_plan *Pl, int l, hipStream_t st)
{
    const int64_t cnt = Pl->lev[l].nb * 2 * (int64_t)Pl->p * Pl->p;
    if (cnt == 0) return;
    k_zero_exp<T><<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st>>>(
        cnt, (T *)Pl->Lc + Pl->lev[l].off * 2 * (int64_t)Pl->p * Pl->p);
}

}  // namespace

bool mmhalf_build(lhf_plan *Pl, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: return mmhalf_build_t<double, 8>(Pl, st);
        case 10: return mmhalf_build_t<double, 10>(Pl, st);
        case 12: return mmhalf_build_t<double, 12>(Pl, st);
        case 16: return mmhalf_build_t<double, 16>(Pl, st);
        }
    } else {
        switch (Pl->p) {
        case 8: return mmhalf_build_t<float, 8>(Pl, st);
        case 10: return mmhalf_build_t<float, 10>(Pl, st);
        case 12: return mmhalf_build_t<float, 12>(Pl, st);
        case 16: return mmhalf_build_t<float, 16>(Pl, st);
        }
    }
    return false;
}

template <int KIND>
static void mm_dispatch(const lhf_plan *Pl, int l, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: launch_mm<double, 8, KIND>(Pl, l, st); break;
        case 10: launch_mm<double, 10, KIND>(Pl, l, st); break;
        case 12: launch_mm<double, 12, KIND>(Pl, l, st); break;
        case 16: launch_mm<double, 16, KIND>(Pl, l, st); break;
        }
    } else {
        switch (Pl->p) {
        case 8: launch_mm<float, 8, KIND>(Pl, l, st); break;
        case 10: launch_mm<float, 10, KIND>(Pl, l, st); break;
        case 12: launch_mm<float, 12, KIND>(Pl, l, st); break;
        case 16: launch_mm<float, 16, KIND>(Pl, l, st); break;
        }
    }
}

// M2M into the boxes of level l from their children
void m2m_half_launch(const lhf_plan *Pl, int l, hipStream_t st) { mm_dispatch<0>(Pl, l, st); }

// L2L into the boxes of level l from their parents; level 2 starts from zero
void l2l_half_launch(const lhf_plan *Pl, int l, hipStream_t st)
{
    if (l <= 2) {
        if (Pl->precision == LHF_FP64) zero_level<double>(Pl, l, st);
        else zero_level<float>(Pl, l, st);
        return;
    }
    mm_dispatch<2>(Pl, l, st);
}

// scalar harmonic FMM (phi only): the orders without half tiles
bool m2l_half_scalar_supported(int precision, int p)
{
    (void)precision;
    return p == 8 || p == 10 || p == 12 || p == 16;
}

void m2l_half_scalar_stage(const lhf_plan *Pl, int level, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: stage_half<double, 8, 4>(Pl, level, st); break;
        case 10: stage_half<double, 10, 4>(Pl, level, st); break;
        case 12: stage_half<double, 12, 4>(Pl, level, st); break;
        case 16: stage_half<double, 16, 4>(Pl, level, st); break;
        }
    } else {
        switch (Pl->p) {
        case 8: stage_half<float, 8, 4>(Pl, level, st); break;
        case 10: stage_half<float, 10, 4>(Pl, level, st); break;
        case 12: stage_half<float, 12, 4>(Pl, level, st); break;
        case 16: stage_half<float, 16, 4>(Pl, level, st); break;
        }
    }
}

void m2l_half_scalar_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: launch_half<double, 8, true>(Pl, level, st); break;
        case 10: launch_half<double, 10, true>(Pl, level, st); break;
        case 12: launch_half<double, 12, true>(Pl, level, st); break;
        case 16: launch_half<double, 16, true>(Pl, level, st); break;
        }
    } else {
        switch (Pl->p) {
        case 8: launch_half<float, 8, true>(Pl, level, st); break;
        case 10: launch_half<float, 10, true>(Pl, level, st); break;
        case 12: launch_half<float, 12, true>(Pl, level, st); break;
        case 16: launch_half<float, 16, true>(Pl, level, st); break;
        }
    }
}

bool m2l_half_supported(int precision, int p)
{
    if (precision == LHF_FP64) return p == 8 || p == 10 || p == 12 || p == 16 || p == 20 || p == 22 || p == 23 || p == 24;
    return p == 8 || p == 10 || p == 12 || p == 16;
}

// the batched M2M / L2L kernels stage both classes' tables in LDS: orders up to 16
bool mm_half_supported(int precision, int p)
{
    (void)precision;
    return p == 8 || p == 10 || p == 12 || p == 16;
}

// true if the half-vector kernel runs in ownership mode (no atomics) for this (precision, p)
bool m2l_half_owned(int precision, int p)
{
    if (!m2l_half_supported(precision, p)) return false;
    if (precision == LHF_FP64) {
        switch (p) {
        case 8: return hv::tile_own<double, 8>();
        case 10: return hv::tile_own<double, 10>();
        case 12: return hv::tile_own<double, 12>();
        case 16: return hv::tile_own<double, 16>();
        default: return hv::tile_own<double, 24>();
        }
    }
    switch (p) {
    case 8: return hv::tile_own<float, 8>();
    case 10: return hv::tile_own<float, 10>();
    case 12: return hv::tile_own<float, 12>();
    default: return hv::tile_own<float, 16>();
    }
}

bool whalf_build(lhf_plan *Pl, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: return whalf_build_t<double, 8>(Pl, st);
        case 10: return whalf_build_t<double, 10>(Pl, st);
        case 12: return whalf_build_t<double, 12>(Pl, st);
        case 16: return whalf_build_t<double, 16>(Pl, st);
        case 20: return whalf_build_t<double, 20>(Pl, st);
        case 22: return whalf_build_t<double, 22>(Pl, st);
        case 23: return whalf_build_t<double, 23>(Pl, st);
        case 24: return whalf_build_t<double, 24>(Pl, st);
        }
    } else {
        switch (Pl->p) {
        case 8: return whalf_build_t<float, 8>(Pl, st);
        case 10: return whalf_build_t<float, 10>(Pl, st);
        case 12: return whalf_build_t<float, 12>(Pl, st);
        case 16: return whalf_build_t<float, 16>(Pl, st);
        }
    }
    return false;
}

void m2l_half_stage(const lhf_plan *Pl, int level, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: stage_half<double, 8>(Pl, level, st); break;
        case 10: stage_half<double, 10>(Pl, level, st); break;
        case 12: stage_half<double, 12>(Pl, level, st); break;
        case 16: stage_half<double, 16>(Pl, level, st); break;
        case 20: stage_half<double, 20>(Pl, level, st); break;
        case 22: stage_half<double, 22>(Pl, level, st); break;
        case 23: stage_half<double, 23>(Pl, level, st); break;
        case 24: stage_half<double, 24>(Pl, level, st); break;
        }
    } else {
        switch (Pl->p) {
        case 8: stage_half<float, 8>(Pl, level, st); break;
        case 10: stage_half<float, 10>(Pl, level, st); break;
        case 12: stage_half<float, 12>(Pl, level, st); break;
        case 16: stage_half<float, 16>(Pl, level, st); break;
        }
    }
}

void m2l_half_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 8: launch_half<double, 8>(Pl, level, st); break;
        case 10: launch_half<double, 10>(Pl, level, st); break;
        case 12: launch_half<double, 12>(Pl, level, st); break;
        case 16: launch_half<double, 16>(Pl, level, st); break;
        case 20: launch_half<double, 20>(Pl, level, st); break;
        case 22: launch_half<double, 22>(Pl, level, st); break;
        case 23: launch_half<double, 23>(Pl, level, st); break;
        case 24: launch_half<double, 24>(Pl, level, st); break;
        }
    } else {
        switch (Pl->p) {
        case 8: launch_half<float, 8>(Pl, level, st); break;
        case 10: launch_half<float, 10>(Pl, level, st); break;
        case 12: launch_half<float, 12>(Pl, level, st); break;
        case 16: launch_half<float, 16>(Pl, level, st); break;
        }
    }
}

}  // namespace lhf

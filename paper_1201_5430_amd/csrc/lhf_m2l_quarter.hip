// lhf_m2l_quarter.hip -- batched FP64 M2L at high orders with each translation's coefficient
// vector split over four lanes by m mod 4.
//
// The translation is the RCR scheme of Sec. 4.4 (rotation about z and y, coaxial (S|R) shift
// with chi carried to order p, R-conversion of eq. rcr1, back-rotation) for both potentials,
// as in the half-vector kernel.  What differs is how much of a vector one lane holds.  At
// FP64 orders 16-24 half a part vector is 72-156 doubles: the register file then holds one
// wavefront per SIMD and, from p = 22 on, spills.  Here
//   lane = 16 t + 8 pot + 4 part + q      (t: translation of the batch, 4 per wavefront)
// and the lane with residue q holds the entries m = 4j + q (j = 0 .. n/4) of every order n
// (78 doubles at p = 23):
//   * z-rotations act entry by entry (the partner part, lane ^ 4, by two DPP moves);
//   * the coaxial shift and the conversion act column by column (fixed m) inside the lane;
//     the conversion's other-potential partner (lane ^ 12) by ds_swizzle;
//   * the y-rotation of order n mixes all m: each lane forms partial sums over its own columns
//     for the output rows of all four residues (groups k = 0..3, residue q ^ k), and a two-step
//     butterfly inside the quad (DPP lane ^ 1, then lane ^ 2) leaves each lane the full sums of
//     its own rows: out = (G0 + G1[^1]) + (G2 + G3[^1])[^2].
// Only the forward (S-basis) rotation tables are staged (one (part, residue) table per lane
// role); the back-rotation uses W_back = D W_fwd^T D^-1 (D = diag(1, -1/2, 1/2, ..) on the Re
// block, diag((-1)^m) on the Im block, as in the half-vector kernel), reading rows of the
// table of residue q ^ k for output group k.  A polar angle pi - theta runs on the staged table
// of theta with signs (see the kernel).  A tile is up to nslot() consecutive target boxes of the
// level and eight wavefronts share it: one workgroup per compute unit with two wavefronts per
// SIMD; the columns of consecutive classes continue round the wavefronts.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lhf_internal.h"
#include "lhf_m2l_common.h"

namespace lhf {
namespace qv {

// the value of lane ^ 4 by two DPP moves (VALU only, no LDS-pipe traffic): row_half_mirror
// (lane ^ 7 within eight lanes), then quad_perm [3,2,1,0] (lane ^ 3)
__device__ inline double xor4(double v)
{
    return dpp_f<DPP_XOR3>(dpp_f<0x141>(v));
}

// entries of order n held by one lane: m = 4j + q, j < S(n)
__host__ __device__ constexpr int S(int n) { return n / 4 + 1; }
__host__ __device__ constexpr int hoff(int n)
{
    int o = 0;
    for (int k = 0; k < n; k++) o += S(k);
    return o;
}
constexpr int E = 2;  // doubles per 16-byte vector
// table rows padded to whole 16-byte vectors
__host__ __device__ constexpr int RL(int n) { return (S(n) + E - 1) / E * E; }
// offset of order n's block in one (part, residue) table: [group k][row j'][RL(n) columns]
__host__ __device__ constexpr int woff(int n)
{
    int o = 0;
    for (int k = 0; k < n; k++) o += 4 * S(k) * RL(k);
    return o;
}

template <int P>
struct Shape {
    static constexpr int NQ = hoff(P);               // entries per lane
    static constexpr int WQ = woff(P);               // one (part, residue) table
    static constexpr int WQS = WQ + E;               // tables one 16-byte vector apart
    static constexpr int NQP = (NQ + E - 1) / E * E; // source layout stride per lane role
    static constexpr int P2 = P * P;
    static constexpr int ARS = NQ + 1;               // accumulator stride per lane role (odd)
    static constexpr int SSTA = 16 * ARS + 1;        // accumulator stride per target slot
};
constexpr int NTHREADS = 512;
constexpr int NV = 189;      // interaction offsets of one target box
constexpr int MAXCLS = 64;   // polar-angle classes (49 for the 316 offsets of the 7^3 stencil)
constexpr int LDS_MAX = 163840;

// Target slots of a tile: as many consecutive target boxes of the level as the LDS holds
// beside one class's rotation tables (6 at p = 23, 5 at p = 24), at most 16.
template <int P>
constexpr int nslot()
{
    using Sh = Shape<P>;
    const int fixed = (int)sizeof(double) * 8 * Sh::WQS + (int)sizeof(int16_t) * (2 * MAXCLS + 1) + 64;
    const int per = (int)sizeof(double) * Sh::SSTA + (int)sizeof(int16_t) * (NV + MAXCLS) + 4 * (int)sizeof(int);
    const int n = (LDS_MAX - fixed) / per;
    return n > 16 ? 16 : n;
}

template <int P>
constexpr size_t tile_bytes()
{
    using Sh = Shape<P>;
    constexpr int NS = nslot<P>();
    return sizeof(double) * (size_t)8 * Sh::WQS + sizeof(double) * (size_t)NS * Sh::SSTA + sizeof(int) * 4 * NS +
           sizeof(int16_t) * ((2 * MAXCLS + 1) + MAXCLS * NS + NV * NS);
}

// packed (phi, chi) expansion index k -> position in a target slot (lane layout)
template <int P>
__device__ inline int acc_pos(int k)
{
    using Sh = Shape<P>;
    const int pot = k / Sh::P2, qq = k % Sh::P2;
    int n = (int)sqrtf((float)qq);
    if ((n + 1) * (n + 1) <= qq) n++;
    if (n * n > qq) n--;
    const int i = qq - n * n, part = i > n, m = part ? i - n : i;
    return (8 * pot + 4 * part + (m & 3)) * Sh::ARS + hoff(n) + (m >> 2);
}

}  // namespace qv

template <int P>
__global__ void __launch_bounds__(qv::NTHREADS, 1) k_m2l_quarter(int level, int64_t soff, int64_t nb, int ns,
                                                                const uint64_t *__restrict__ bkey,
                                                                const int32_t *__restrict__ dmap,
                                                                const double *__restrict__ Mq,
                                                                double *__restrict__ Lc,
                                                                const double *__restrict__ wq, int64_t wstride,
                                                                M2LSched sch, const int16_t *__restrict__ qsched,
                                                                const double *__restrict__ dtab)
{
    using Sh = qv::Shape<P>;
    using qv::hoff;
    using qv::S;
    constexpr int P2 = Sh::P2, NQ = Sh::NQ, NQP = Sh::NQP, ARS = Sh::ARS, SSTA = Sh::SSTA, WQS = Sh::WQS;
    constexpr int NSLOT = qv::nslot<P>(), NT = qv::NTHREADS, MAXCLS = qv::MAXCLS;
    extern __shared__ char smem[];
    double *Wl = (double *)smem;                       // [part][residue][WQS] forward tables
    double *acc = Wl + 8 * WQS;                        // [NSLOT][SSTA]
    int *slot_xyz = (int *)(acc + NSLOT * SSTA);       // [NSLOT] packed target coordinates, -1: no box
    int *slot_box = slot_xyz + NSLOT;                  // [NSLOT] target box
    int *slot_sys = slot_box + NSLOT;                  // [NSLOT] system of the target
    int *slot_c = slot_sys + NSLOT;                    // [NSLOT] child position of the target
    int16_t *cst = (int16_t *)(slot_c + NSLOT);        // [ncls + 1] class starts in ent
    int16_t *kcnt = cst + (MAXCLS + 1);                // [ncls][NSLOT] entries per (class, slot)
    int16_t *ent = kcnt + MAXCLS * NSLOT;              // [<= NV * NSLOT] (dir << 4) | slot, by class
    int16_t *coff = ent + qv::NV * NSLOT;                // [ncls] wavefront of each class's first column

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware tile order: consecutive tiles stay on one XCD (shared L2)
    const int64_t ntiles = (nb + ns - 1) / ns;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int ncls = sch.ncls;
    const int side = 1 << level;

    // the tile's targets: ns consecutive boxes of the level (Morton order)
    if (tid < NSLOT) {
        int box = -1, xyz = -1, sys = 0, c = 0;
        const int64_t b = tile * ns + tid;
        if (tid < ns && b < nb) {
            box = (int)(soff + b);
            const uint64_t key = bkey[box];
            uint32_t ix = 0, iy = 0, iz = 0;
            for (int bb = 0; bb < level; bb++) {
                ix |= (uint32_t)((key >> (3 * bb)) & 1u) << bb;
                iy |= (uint32_t)((key >> (3 * bb + 1)) & 1u) << bb;
                iz |= (uint32_t)((key >> (3 * bb + 2)) & 1u) << bb;
            }
            xyz = (int)(ix | (iy << 10) | (iz << 20));
            sys = (int)(key >> (3 * level));
            c = (int)(key & 7u);
        }
        slot_box[tid] = box;
        slot_xyz[tid] = xyz;
        slot_sys[tid] = sys;
        slot_c[tid] = c;
    }
    __syncthreads();
    // source box of offset dir from the target in slot sl, -1 if it is outside the system's cube or empty
    auto source_of = [&](int dir, int sl) -> int {
        const int xyz = slot_xyz[sl];
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        const bool inb = xyz >= 0 && sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
        return inb ? dmap[(((size_t)slot_sys[sl] * side + sz) * side + sy) * side + sx] : -1;
    };
    // per (class, slot): the V-list offsets of the slot's child position in that class whose
    // source box exists; counted, scanned, then listed class by class
    for (int ks = tid; ks < ncls * NSLOT; ks += NT) {
        const int kk = ks / NSLOT, sl = ks % NSLOT, ko = qsched[kk];
        int cnt = 0;
        if (slot_box[sl] >= 0)
            for (int r = sch.row_start[ko]; r < sch.row_start[ko + 1]; r++) {
                const int dir = sch.rows[r * 8 + slot_c[sl]];
                if (dir >= 0 && source_of(dir, sl) >= 0) cnt++;
            }
        kcnt[ks] = (int16_t)cnt;
    }
    __syncthreads();
    if (tid == 0) {
        int o = 0;
        for (int kk = 0; kk < ncls; kk++) {
            cst[kk] = (int16_t)o;
            for (int sl = 0; sl < NSLOT; sl++) o += kcnt[kk * NSLOT + sl];
        }
        cst[ncls] = (int16_t)o;
        // the columns of consecutive classes continue round the eight wavefronts: classes on one staged
        // table (a polar angle and its mirror) run without a barrier between them, and their last,
        // partly filled rounds then land on different wavefronts
        int w8 = 0;
        for (int kk = 0; kk < ncls; kk++) {
            coff[kk] = (int16_t)w8;
            w8 = (w8 + ((cst[kk + 1] - cst[kk] + 3) >> 2)) & 7;
        }
    }
    __syncthreads();
    for (int ks = tid; ks < ncls * NSLOT; ks += NT) {
        const int kk = ks / NSLOT, sl = ks % NSLOT, ko = qsched[kk];
        int o = cst[kk];
        for (int s2 = 0; s2 < sl; s2++) o += kcnt[kk * NSLOT + s2];
        if (slot_box[sl] >= 0)
            for (int r = sch.row_start[ko]; r < sch.row_start[ko + 1]; r++) {
                const int dir = sch.rows[r * 8 + slot_c[sl]];
                if (dir >= 0 && source_of(dir, sl) >= 0) ent[o++] = (int16_t)((dir << 4) | sl);
            }
    }
    // the targets' local expansions into their slots (entries without an (n, m) stay zero)
    for (int idx = tid; idx < NSLOT * SSTA; idx += NT) acc[idx] = 0.0;
    __syncthreads();
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += NT) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) acc[sl * SSTA + qv::acc_pos<P>(r)] = Lc[(size_t)box * 2 * P2 + r];
    }

    const int t = lane >> 4, pot = (lane >> 3) & 1, part = (lane >> 2) & 1, q = lane & 3;

    struct Job {
        int slot, dir, src;
    };
    // translation of class k for this lane group: the class's entries, read as a 4 x Q matrix
    // (Q = ceil(count / 4)) column by column, so that the four translations of one wavefront
    // come from four places of the list (different targets where the class has several).
    // (slot, dir) from LDS, source by one load.  Branch-free (every load at a valid address, the
    // result chosen by selects): the batch body must run with all lanes active, since its DPP
    // exchanges read other lanes' registers and a register restored inside a divergent region
    // would hold a stale value in the lanes that region skipped
    auto setup = [&](int k, int r0) -> Job {
        const bool kin = k < ncls;
        const int kc = kin ? k : 0;
        const int e0 = cst[kc], cnt = kin ? cst[kc + 1] - e0 : 0;
        const int Q = (cnt + 3) >> 2;
        const int col = (r0 >> 2) + ((wave - coff[kc]) & 7), e = t * Q + col;
        const bool ok0 = col < Q && e < cnt;
        const int code = ent[ok0 ? e0 + e : 0];
        const int dir = ok0 ? code >> 4 : 0, slot = code & 15;
        const int xyz = slot_xyz[slot];
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        const bool inb = ok0 && xyz >= 0 && sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
        const size_t di = inb ? (((size_t)slot_sys[slot] * side + sz) * side + sy) * side + sx : 0;
        const int src = dmap[di];
        const bool ok = inb && src >= 0;
        return Job{ok ? slot : -1, ok ? dir : 0, ok ? src : -1};
    };
    // the first class at or after k with entries (ncls if none)
    auto nonempty = [&](int k) {
        while (k < ncls && cst[k + 1] == cst[k]) k++;
        return k;
    };
    auto advance = [&](int &k, int &r0) {
        r0 += 8 * 4;
        if (k < ncls && r0 >= 4 * ((cst[k + 1] - cst[k] + 3) >> 2)) {
            k = nonempty(k + 1);
            r0 = 0;
        }
    };
    // this lane's entries of the source, stored contiguously per lane role by k_mquarter
    auto load_part = [&](const Job &j, double *dst) {
        const double2 *sp = (const double2 *)(Mq + ((size_t)(j.src >= 0 ? j.src - soff : 0) * 16 + (lane & 15)) * NQP);
#pragma unroll
        for (int i = 0; i < NQP / 2; i++) {
            const double2 x = sp[i];
            dst[2 * i] = x.x;
            if (2 * i + 1 < NQ) dst[2 * i + 1] = x.y;
        }
    };

    int k = nonempty(0), r0 = 0;  // current batch
    int k1 = k, r1 = 0;           // next batch
    advance(k1, r1);
    Job cur = setup(k, r0), nxt = setup(k1, r1);
    constexpr int N16 = 8 * WQS * 8 / 16;
    int staged = -1;
    while (k < ncls) {
        const int tb = qsched[ncls + k];  // a mirrored class reuses the staged table
        if (tb != staged) {
            __syncthreads();
            const uint4 *src4 = (const uint4 *)(wq + (size_t)tb * wstride);
            uint4 *dst4 = (uint4 *)Wl;
#pragma unroll 4
            for (int i = tid; i < N16; i += NT) dst4[i] = src4[i];
            __syncthreads();
            staged = tb;
        }
        const bool mir = qsched[2 * ncls + k] != 0;
        const Job j = cur;
        const bool act = j.src >= 0;
        int k2 = k1, r2 = r1;
        advance(k2, r2);
        const Job nn = setup(k2, r2);
        if (__ballot(act) != 0ull) {  // wavefront-uniform: skip batches with no active lane
            double v[NQ];
            load_part(j, v);
            const double2 d0 = ((const double2 *)dtab)[2 * j.dir], d1 = ((const double2 *)dtab)[2 * j.dir + 1];
            const double tau = d0.x, itau = d0.y;
            const double cph = d1.x, sph = d1.y;
            // e^{i q phi} (by selects: no lane-dependent loop) and e^{4 i phi}
            const double c2 = cph * cph - sph * sph, s2 = 2.0 * cph * sph;
            const double c3 = c2 * cph - s2 * sph, s3 = s2 * cph + c2 * sph;
            const double c4 = c2 * c2 - s2 * s2, s4 = 2.0 * c2 * s2;
            const double cq = q == 0 ? 1.0 : q == 1 ? cph : q == 2 ? c2 : c3;
            const double sq = q == 0 ? 0.0 : q == 1 ? sph : q == 2 ? s2 : s3;
            // a mirrored class (theta' = pi - theta) runs on the staged table of theta: per order n the
            // S-basis rotation block is W(theta') = c_n D W(theta) D with D = diag((-1)^m) and c_n = (-1)^n
            // on the Re block, -(-1)^n on the Im block; D acts as the sign (-1)^q of this lane's entries
            const double sgq = (mir && (q & 1)) ? -1.0 : 1.0;
            const double g0 = mir ? sgq * (part ? -1.0 : 1.0) : 1.0, g1 = mir ? -g0 : g0;  // c_n (-1)^q, n even / odd
            const double itm = mir ? -itau : itau;
            // 1. rotate about z by +phi: Re' = re c - im s, Im' = im c + re s (m = 4j + q)
            {
                const double sgn = part ? 1.0 : -1.0;
                double cm = cq * sgq, sm = sq * sgq;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
                    const double sz = sm * sgn;
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double x = v[hoff(n) + jj];
                        const double o = qv::xor4(x);
                        v[hoff(n) + jj] = x * cm + o * sz;
                    }
                    const double a = cm * c4 - sm * s4, b = sm * c4 + cm * s4;
                    cm = a;
                    sm = b;
                }
            }
            // 2. rotation about y of every order with this lane's forward table: partial sums of the
            //    four output groups over the lane's columns, then the quad butterfly
            {
                const double *Wf = Wl + (part * 4 + q) * WQS;
#pragma unroll
                for (int n = 0; n < P; n++) {
                    const double *Wn = Wf + qv::woff(n);
                    constexpr int SM = (P - 1) / 4 + 1;
                    double g[4][SM];
                    // the table rows (output group kk, row jj) in pairs, each pair's LDS reads issued
                    // before the previous pair is computed (software pipelining: two pairs of rows in
                    // registers, so the LDS latency overlaps the dot products)
                    {
                        constexpr int GR = 2;  // rows per group
                        constexpr int RLMAX = qv::RL(P - 1) / 2;
                        const int R = 4 * S(n), H = qv::RL(n) / 2, NG = (R + GR - 1) / GR;
                        double2 buf[2][GR][RLMAX];
                        auto ld = [&](int gg, double2 (&b)[GR][RLMAX]) __attribute__((always_inline)) {
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++)
                                        if (h < H) b[rr][h] = ((const double2 *)(Wn + row * qv::RL(n)))[h];
                                }
                            }
                        };
                        ld(0, buf[0]);
#pragma unroll
                        for (int gg = 0; gg < (4 * S(P - 1) + GR - 1) / GR; gg++) {
                            if (gg >= NG) break;
                            if (gg + 1 < NG) ld(gg + 1, buf[(gg + 1) & 1]);
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
                                    const int kk = row / S(n), jj = row % S(n);
                                    double a = 0;
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++) {
                                        if (h >= H) break;
                                        a += buf[gg & 1][rr][h].x * v[hoff(n) + 2 * h];
                                        if (2 * h + 1 < S(n)) a += buf[gg & 1][rr][h].y * v[hoff(n) + 2 * h + 1];
                                    }
                                    g[kk][jj] = a;
                                }
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < S(n); jj++) {
                        const double a = g[0][jj] + dpp_f<DPP_XOR1>(g[1][jj]);
                        const double b = g[2][jj] + dpp_f<DPP_XOR1>(g[3][jj]);
                        v[hoff(n) + jj] = a + dpp_f<DPP_XOR2>(b);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // 3+4. per column m = 4c + q: coaxial (S|R) shift out_n = tau^-(n+1) sum_n' (n+n')! tau^-n' in_n'
            //      (chi to order P), then the R-conversion (eq. rcr1, scaled)
            //        phi~ = phi + i tau m/n chi ,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
            {
                const double wphi = pot ? 0.0 : 1.0, wchi = pot ? 1.0 : 0.0;
                const double sconv = part ? 1.0 : -1.0;
                const double itau4 = (itau * itau) * (itau * itau);
                double pc = 1.0;  // tau^-(4c)
#pragma unroll
                for (int c = 0; c < S(P - 1); c++) {
                    const int n0 = 4 * c;
                    const double mval = (double)(4 * c + q);
                    double out[P + 1];
                    {
                        double s = pc * g0;
#pragma unroll
                        for (int n2 = n0; n2 < P; n2++) {
                            v[hoff(n2) + c] *= s;
                            s *= itm;
                        }
                        double so = pc * itau;
#pragma unroll
                        for (int n = n0; n <= P; n++) {
                            double a = 0;
#pragma unroll
                            for (int n2 = n0; n2 < P; n2++) a += dfact(n + n2) * v[hoff(n2) + c];
                            out[n] = a * so;
                            so *= itau;
                        }
                    }
                    pc *= itau4;
#pragma unroll
                    for (int n = n0; n < P; n++) {
                        const double other = swz_xor<12>(out[n]);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                        const double fphi = (n > 0) ? tau * mval * (1.0 / (double)n) * sconv * wphi : 0.0;
                        const double fchi = -tau * (1.0 / (double)(n + 1)) * wchi;
                        double val = out[n] + fphi * other + fchi * out[n + 1];
                        v[hoff(n) + c] = (n - n0 < q) ? 0.0 : val;  // slot (n, c) holds m = 4c + q > n: empty
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // 5. back-rotation with the forward tables: v <- D W_fwd^T D^-1 v.  Output group k
            //    (residue q ^ k) takes rows j of the table of residue q ^ k, group k; the quad
            //    butterfly gathers the groups; D scales the outputs
            {
                const double sg = (q & 1) ? -1.0 : 1.0;  // (-1)^m on this lane
                const double fin = part ? sg : 2.0 * sg, fout = part ? sg : 0.5 * sg;
                const double fin0 = fin * g0, fin1 = fin * g1;  // with the mirrored class's input signs
                const double *Wp = Wl + part * 4 * WQS;
#pragma unroll
                for (int n = 0; n < P; n++) {
                    constexpr int SM = (P - 1) / 4 + 1;
                    double g[4][SM];
#pragma unroll
                    for (int kk = 0; kk < 4; kk++)
#pragma unroll
                        for (int jj = 0; jj < S(n); jj++) g[kk][jj] = 0.0;
                    // the rows one at a time (input slot jj outer, output group kk inner), each row's LDS
                    // reads issued before the previous row is accumulated (software pipelining)
                    {
                        constexpr int GR = 1;  // rows per group
                        constexpr int RLMAX = qv::RL(P - 1) / 2;
                        const int R = 4 * S(n), H = qv::RL(n) / 2, NG = (R + GR - 1) / GR;
                        double2 buf[2][GR][RLMAX];
                        auto ld = [&](int gg, double2 (&b)[GR][RLMAX]) __attribute__((always_inline)) {
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
                                    const int jj = row / 4, kk = row % 4;
                                    const double *wr = Wp + (q ^ kk) * WQS + qv::woff(n) + (kk * S(n) + jj) * qv::RL(n);
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++)
                                        if (h < H) b[rr][h] = ((const double2 *)wr)[h];
                                }
                            }
                        };
                        ld(0, buf[0]);
#pragma unroll
                        for (int gg = 0; gg < (4 * S(P - 1) + GR - 1) / GR; gg++) {
                            if (gg >= NG) break;
                            if (gg + 1 < NG) ld(gg + 1, buf[(gg + 1) & 1]);
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
                                    const int jj = row / 4, kk = row % 4;
                                    // m = 0 (q = 0, j = 0, Re part) is not doubled by D^-1
                                    const double xj = v[hoff(n) + jj] * ((jj == 0 && q == 0 && !part) ? ((n & 1) ? g1 : g0) : ((n & 1) ? fin1 : fin0));
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++) {
                                        if (h >= H) break;
                                        g[kk][2 * h] += xj * buf[gg & 1][rr][h].x;
                                        if (2 * h + 1 < S(n)) g[kk][2 * h + 1] += xj * buf[gg & 1][rr][h].y;
                                    }
                                }
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < S(n); jj++) {
                        const double a = g[0][jj] + dpp_f<DPP_XOR1>(g[1][jj]);
                        const double b = g[2][jj] + dpp_f<DPP_XOR1>(g[3][jj]);
                        v[hoff(n) + jj] = (a + dpp_f<DPP_XOR2>(b)) * ((jj == 0 && q == 0 && !part) ? 1.0 : fout);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // 6. back-rotation about z (-phi) and accumulation into the target slot
            {
                double *ap = acc + (size_t)(act ? j.slot : 0) * SSTA + (lane & 15) * ARS;
                const double sgn = part ? -1.0 : 1.0;  // Re' = re c + im s, Im' = im c - re s
                double cm = cq * sgq, sm = sq * sgq;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
                    const double sz = sm * sgn;
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double x = v[hoff(n) + jj];
                        const double o = qv::xor4(x);
                        const double val = x * cm + o * sz;
                        // no branch: a conditional add would let the compiler sink the whole
                        // translation into it and keep every partial sum live (inactive lanes add 0)
                        atomicAdd(ap + hoff(n) + jj, act ? val : 0.0);
                    }
                    const double a = cm * c4 - sm * s4, b = sm * c4 + cm * s4;
                    cm = a;
                    sm = b;
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
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += NT) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + r] = acc[sl * SSTA + qv::acc_pos<P>(r)];
    }
}

// ---------------------------------------------------------------------------
// The same M2L with the rotations about y on the matrix cores (v_mfma_f64_16x16x4f64), the
// coefficient vectors kept in registers in the instruction's operand layout.
//
// A wavefront holds eight translations of one polar-angle class, both potentials: the 16 MFMA
// columns j = 2 t + pot (t: translation, 0..7).  Lane l = 16 k + j holds, for its column, the
// entries m = 4 jj + k of every order n and of both parts (Re, Im) -- slot hoff(n) + jj, the
// residue layout of the quarter-vector kernel with both parts in one lane.  This is exactly how
// the instruction wants its operands: B[k][j] comes from lane j + 16 k, and D rows 4 r + k of
// column j land in lane j + 16 k, register r.  So the rotation of order n, part p is, per block b
// of 16 output rows,
//   D_b = sum_s A_{b,s} B_s,  A_{b,s}[i][kk] = W_p[16 b + i][4 s + kk],  B_s[kk][j] = slot (n, s),
// and D_b's register r is the lane's output slot 4 b + r: no lane exchange at all.  W_p is the
// class's forward S-basis block of order n (the Im block embedded in (n+1) x (n+1) with a zero row
// and column m = 0), staged in LDS; lane l reads A[l % 16][l / 16].  The back-rotation reads the
// same table transposed through the diagonal similarity W_back = D W_fwd^T D^-1 (scalings of the
// inputs and outputs).  z-rotations act on (Re, Im) inside the lane; the coaxial shift and the
// conversion act on the lane's column m as in the quarter-vector kernel, the other potential of
// the conversion coming from lane ^ 1 (one DPP move).  Four wavefronts per workgroup, one
// workgroup per compute unit: the 156-double vector per lane takes the register file of one
// wavefront per SIMD (VGPRs and AGPRs).
// ---------------------------------------------------------------------------
namespace qm {
constexpr int NTHREADS = 256;
constexpr int NV = 189;
constexpr int MAXCLS = 64;
__host__ __device__ constexpr int rsz(int P) { return P * (2 * P * P + 1) / 3; }  // one rotation set
template <int P>
constexpr int nslot()
{
    const int fixed = (int)sizeof(double) * rsz(P) + (int)sizeof(int16_t) * (MAXCLS + 1) + 64;
    const int per = (int)sizeof(double) * 2 * P * P + (int)sizeof(int16_t) * (NV + MAXCLS) + 4 * (int)sizeof(int);
    const int n = (qv::LDS_MAX - fixed) / per;
    return n > 16 ? 16 : n;
}
template <int P>
constexpr size_t tile_bytes()
{
    constexpr int NS = nslot<P>();
    return sizeof(double) * ((size_t)rsz(P) + (size_t)NS * 2 * P * P) + sizeof(int) * 4 * NS +
           sizeof(int16_t) * ((MAXCLS + 1) + MAXCLS * NS + NV * NS);
}
typedef double v4d __attribute__((ext_vector_type(4)));
}  // namespace qm

template <int P>
__global__ void __launch_bounds__(qm::NTHREADS, 1) k_m2l_qmfma(int level, int64_t soff, int64_t nb, int ns,
                                                               const uint64_t *__restrict__ bkey,
                                                               const int32_t *__restrict__ dmap,
                                                               const double *__restrict__ Mq,
                                                               double *__restrict__ Lc,
                                                               const double *__restrict__ rot, M2LSched sch,
                                                               const int16_t *__restrict__ cls_theta,
                                                               const double *__restrict__ dtab)
{
    using Sh = qv::Shape<P>;
    using qv::hoff;
    using qv::S;
    using qm::v4d;
    constexpr int P2 = Sh::P2, NQ = Sh::NQ, NQP = Sh::NQP, RS = qm::rsz(P);
    constexpr int NSLOT = qm::nslot<P>(), NT = qm::NTHREADS, MAXCLS = qm::MAXCLS;
    extern __shared__ char smem[];
    double *Wl = (double *)smem;                       // [RS] the class's forward S-basis blocks
    double *acc = Wl + RS;                             // [NSLOT][2 P^2] targets, packed (pot, n, part, m)
    int *slot_xyz = (int *)(acc + NSLOT * 2 * P2);     // [NSLOT] packed target coordinates, -1: no box
    int *slot_box = slot_xyz + NSLOT;
    int *slot_sys = slot_box + NSLOT;
    int *slot_c = slot_sys + NSLOT;
    int16_t *cst = (int16_t *)(slot_c + NSLOT);        // [ncls + 1] class starts in ent
    int16_t *kcnt = cst + (MAXCLS + 1);                // [ncls][NSLOT]
    int16_t *ent = kcnt + MAXCLS * NSLOT;              // [<= NV * NSLOT] (dir << 4) | slot, by class

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ntiles = (nb + ns - 1) / ns;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int ncls = sch.ncls;
    const int side = 1 << level;

    if (tid < NSLOT) {
        int box = -1, xyz = -1, sys = 0, c = 0;
        const int64_t b = tile * ns + tid;
        if (tid < ns && b < nb) {
            box = (int)(soff + b);
            const uint64_t key = bkey[box];
            uint32_t ix = 0, iy = 0, iz = 0;
            for (int bb = 0; bb < level; bb++) {
                ix |= (uint32_t)((key >> (3 * bb)) & 1u) << bb;
                iy |= (uint32_t)((key >> (3 * bb + 1)) & 1u) << bb;
                iz |= (uint32_t)((key >> (3 * bb + 2)) & 1u) << bb;
            }
            xyz = (int)(ix | (iy << 10) | (iz << 20));
            sys = (int)(key >> (3 * level));
            c = (int)(key & 7u);
        }
        slot_box[tid] = box;
        slot_xyz[tid] = xyz;
        slot_sys[tid] = sys;
        slot_c[tid] = c;
    }
    __syncthreads();
    auto source_of = [&](int dir, int sl) -> int {
        const int xyz = slot_xyz[sl];
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        const bool inb = xyz >= 0 && sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
        return inb ? dmap[(((size_t)slot_sys[sl] * side + sz) * side + sy) * side + sx] : -1;
    };
    for (int ks = tid; ks < ncls * NSLOT; ks += NT) {
        const int kk = ks / NSLOT, sl = ks % NSLOT;
        int cnt = 0;
        if (slot_box[sl] >= 0)
            for (int r = sch.row_start[kk]; r < sch.row_start[kk + 1]; r++) {
                const int dir = sch.rows[r * 8 + slot_c[sl]];
                if (dir >= 0 && source_of(dir, sl) >= 0) cnt++;
            }
        kcnt[ks] = (int16_t)cnt;
    }
    __syncthreads();
    if (tid == 0) {
        int o = 0;
        for (int kk = 0; kk < ncls; kk++) {
            cst[kk] = (int16_t)o;
            for (int sl = 0; sl < NSLOT; sl++) o += kcnt[kk * NSLOT + sl];
        }
        cst[ncls] = (int16_t)o;
    }
    __syncthreads();
    for (int ks = tid; ks < ncls * NSLOT; ks += NT) {
        const int kk = ks / NSLOT, sl = ks % NSLOT;
        int o = cst[kk];
        for (int s2 = 0; s2 < sl; s2++) o += kcnt[kk * NSLOT + s2];
        if (slot_box[sl] >= 0)
            for (int r = sch.row_start[kk]; r < sch.row_start[kk + 1]; r++) {
                const int dir = sch.rows[r * 8 + slot_c[sl]];
                if (dir >= 0 && source_of(dir, sl) >= 0) ent[o++] = (int16_t)((dir << 4) | sl);
            }
    }
    // the targets' local expansions into their slots (packed as in Lc)
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += NT) {
        const int sl = idx / (2 * P2);
        const int box = slot_box[sl];
        acc[idx] = box >= 0 ? Lc[(size_t)box * 2 * P2 + idx % (2 * P2)] : 0.0;
    }
    __syncthreads();

    const int k = lane >> 4, col = lane & 15, tt = col >> 1, pot = col & 1;

    struct Job {
        int slot, dir, src;
    };
    // translation (wave, tt) of class kk: the class's entries read as an 8 x Q matrix column by
    // column (Q = ceil(count / 8)); branch-free, every load at a valid address
    auto setup = [&](int kk, int r0) -> Job {
        const bool kin = kk < ncls;
        const int kc = kin ? kk : 0;
        const int e0 = cst[kc], cnt = kin ? cst[kc + 1] - e0 : 0;
        const int Q = (cnt + 7) >> 3;
        const int cc = (r0 >> 3) + wave, e = tt * Q + cc;
        const bool ok0 = cc < Q && e < cnt;
        const int code = ent[ok0 ? e0 + e : 0];
        const int dir = ok0 ? code >> 4 : 0, slot = code & 15;
        const int xyz = slot_xyz[slot < NSLOT ? slot : 0];
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        const bool inb = ok0 && xyz >= 0 && sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side;
        const size_t di = inb ? (((size_t)slot_sys[slot] * side + sz) * side + sy) * side + sx : 0;
        const int src = dmap[di];
        const bool ok = inb && src >= 0;
        return Job{ok ? slot : -1, ok ? dir : 0, ok ? src : -1};
    };
    auto nonempty = [&](int kk) {
        while (kk < ncls && cst[kk + 1] == cst[kk]) kk++;
        return kk;
    };
    auto advance = [&](int &kk, int &r0) {
        r0 += 8 * (NT / 64);
        if (kk < ncls && r0 >= 8 * ((cst[kk + 1] - cst[kk] + 7) >> 3)) {
            kk = nonempty(kk + 1);
            r0 = 0;
        }
    };

    // the y rotation of order n, part p (vv: that part's entries), on the matrix cores.  BACK: the
    // transposed table with the D scalings (inputs by D^-1, outputs by D)
    const double sg = (k & 1) ? -1.0 : 1.0;  // (-1)^m on this lane's entries
    auto rotate_part = [&](double (&vv)[NQ], const int p, const int n, const bool back, const int ai, const int ak)
                           __attribute__((always_inline)) {
        constexpr int NB = (P + 15) / 16;
        const int nbk = (n + 1 + 15) / 16, nst = (n + 1 + 3) / 4;
        v4d d[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) d[b] = v4d{0.0, 0.0, 0.0, 0.0};
        const double *blk = Wl + rot_block_off(n) + (p ? (n + 1) * (n + 1) : 0);
        const int ld = p ? n : n + 1;  // row length of the stored block
#pragma unroll
        for (int s = 0; s < (P + 3) / 4; s++) {
            if (s >= nst) break;
            // B: this lane's slot (n, s) (m = 4 s + k), scaled by D^-1 on the way back
            double bval = vv[hoff(n) + s];
            if (back) bval *= (p ? sg : ((s == 0 && k == 0) ? 1.0 : 2.0 * sg));
#pragma unroll
            for (int b = 0; b < NB; b++) {
                if (b >= nbk) break;
                // A[ai][ak]: forward W[16 b + ai][4 s + ak], back W[4 s + ak][16 b + ai]; outside the
                // block (or the Im block's row and column m = 0) zero, read at a valid address
                const int mo = 16 * b + ai, mi = 4 * s + ak;
                const int r = back ? mi : mo, c = back ? mo : mi;
                const bool ok = r <= n && c <= n && (p == 0 || (r >= 1 && c >= 1));
                const int at = ok ? (p ? (r - 1) * ld + (c - 1) : r * ld + c) : 0;
                const double araw = blk[at];
                const double a = ok ? araw : 0.0;
                d[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bval, d[b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int jj = 0; jj < S(n); jj++) {
            double o = d[jj / 4][jj % 4];
            if (back) o *= (p ? sg : ((jj == 0 && k == 0) ? 1.0 : 0.5 * sg));
            vv[hoff(n) + jj] = o;
        }
    };
    auto rotate_y = [&](double (&vre)[NQ], double (&vim)[NQ], const bool back) __attribute__((always_inline)) {
#pragma unroll
        for (int n = 0; n < P; n++) {
            // the lane's A entry, opaque per order: the compiler would otherwise precompute the LDS
            // offsets of every MFMA of the translation once, outside the batch loop, and keep them
            int ai = lane & 15, ak = lane >> 4;
            asm volatile("" : "+v"(ai), "+v"(ak));
            rotate_part(vre, 0, n, back, ai, ak);
            rotate_part(vim, 1, n, back, ai, ak);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    int kc = nonempty(0), r0 = 0;
    int k1 = kc, r1 = 0;
    advance(k1, r1);
    Job cur = setup(kc, r0), nxt = setup(k1, r1);
    int staged = -1;
    while (kc < ncls) {
        if (kc != staged) {
            __syncthreads();
            const double *srcw = rot + ((size_t)cls_theta[kc] * ROT_NKIND + ROT_S_FWD) * RS;
#pragma unroll 8
            for (int i = tid; i < RS; i += NT) Wl[i] = srcw[i];
            __syncthreads();
            staged = kc;
        }
        const Job j = cur;
        const bool act = j.src >= 0;
        int k2 = k1, r2 = r1;
        advance(k2, r2);
        const Job nn = setup(k2, r2);
        if (__ballot(act) != 0ull) {
            double vre[NQ], vim[NQ];
            // the source's entries of this lane's potential, both parts (quarter layout of k_mquarter)
            {
                const double2 *spr =
                    (const double2 *)(Mq + ((size_t)(act ? j.src - soff : 0) * 16 + 8 * pot + 0 + k) * NQP);
                const double2 *spi =
                    (const double2 *)(Mq + ((size_t)(act ? j.src - soff : 0) * 16 + 8 * pot + 4 + k) * NQP);
#pragma unroll
                for (int i = 0; i < NQP / 2; i++) {
                    const double2 x = spr[i], y = spi[i];
                    vre[2 * i] = act ? x.x : 0.0;
                    vim[2 * i] = act ? y.x : 0.0;
                    if (2 * i + 1 < NQ) {
                        vre[2 * i + 1] = act ? x.y : 0.0;
                        vim[2 * i + 1] = act ? y.y : 0.0;
                    }
                }
            }
            const double2 d0 = ((const double2 *)dtab)[2 * j.dir], d1 = ((const double2 *)dtab)[2 * j.dir + 1];
            const double tau = d0.x, itau = d0.y;
            const double cph = d1.x, sph = d1.y;
            const double c2 = cph * cph - sph * sph, s2 = 2.0 * cph * sph;
            const double c3 = c2 * cph - s2 * sph, s3 = s2 * cph + c2 * sph;
            const double c4 = c2 * c2 - s2 * s2, s4 = 2.0 * c2 * s2;
            const double cq = k == 0 ? 1.0 : k == 1 ? cph : k == 2 ? c2 : c3;
            const double sq = k == 0 ? 0.0 : k == 1 ? sph : k == 2 ? s2 : s3;
            // 1. rotate about z by +phi: Re' = re c - im s, Im' = im c + re s (m = 4 jj + k)
            {
                double cm = cq, sm = sq;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double re = vre[hoff(n) + jj], im = vim[hoff(n) + jj];
                        vre[hoff(n) + jj] = re * cm - im * sm;
                        vim[hoff(n) + jj] = im * cm + re * sm;
                    }
                    const double a = cm * c4 - sm * s4, b = sm * c4 + cm * s4;
                    cm = a;
                    sm = b;
                }
            }
            // 2. rotation about y (S basis)
            rotate_y(vre, vim, false);
            // 3+4. per column m = 4c + k and part: coaxial (S|R) shift with chi to order P, then the
            //      R-conversion (eq. rcr1, scaled): phi~ = phi + i tau m/n chi, chi~_n = chi_n - tau/(n+1) chi_{n+1}
            {
                const double wphi = pot ? 0.0 : 1.0, wchi = pot ? 1.0 : 0.0;
                const double itau4 = (itau * itau) * (itau * itau);
                double pc = 1.0;  // tau^-(4c)
                auto coax = [&](double (&vv)[NQ], double (&out)[P + 1], const int c) __attribute__((always_inline)) {
                    const int n0 = 4 * c;
                    // the column through an opaque copy: otherwise the compiler starts the sums of every
                    // column while the rotation produces their entries and runs out of registers
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) asm volatile("" : "+v"(vv[hoff(n2) + c]));
                    double sc = pc;
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) {
                        vv[hoff(n2) + c] *= sc;
                        sc *= itau;
                    }
                    double so = pc * itau;
#pragma unroll
                    for (int n = n0; n <= P; n++) {
                        double a = 0;
#pragma unroll
                        for (int n2 = n0; n2 < P; n2++) a += dfact(n + n2) * vv[hoff(n2) + c];
                        out[n] = a * so;
                        so *= itau;
                    }
                };
                auto convert = [&](double (&vv)[NQ], const double (&out)[P + 1], const double (&oth)[P + 1],
                                   const double sconv, const int c) __attribute__((always_inline)) {
                    const int n0 = 4 * c;
                    const double mval = (double)(4 * c + k);
#pragma unroll
                    for (int n = n0; n < P; n++) {
                        // phi-Re <-> chi-Im, phi-Im <-> chi-Re: the other part of the other potential
                        const double other = dpp_f<DPP_XOR1>(oth[n]);
                        const double fphi = (n > 0) ? tau * mval * (1.0 / (double)n) * sconv * wphi : 0.0;
                        const double fchi = -tau * (1.0 / (double)(n + 1)) * wchi;
                        const double val = out[n] + fphi * other + fchi * out[n + 1];
                        vv[hoff(n) + c] = (n - n0 < k) ? 0.0 : val;
                    }
                };
#pragma unroll
                for (int c = 0; c < S(P - 1); c++) {
                    double outr[P + 1], outi[P + 1];
                    coax(vre, outr, c);
                    coax(vim, outi, c);
                    pc *= itau4;
                    convert(vre, outr, outi, -1.0, c);
                    convert(vim, outi, outr, 1.0, c);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // 5. back-rotation about y (R basis, through the transposed forward table)
            rotate_y(vre, vim, true);
            // 6. back-rotation about z (-phi) and accumulation into the target slot
            {
                double *ap = acc + (size_t)(act ? j.slot : 0) * 2 * P2 + pot * P2;
                double cm = cq, sm = sq;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
                    const int m = 4 * jj + k;
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double re = vre[hoff(n) + jj], im = vim[hoff(n) + jj];
                        const double vr = re * cm + im * sm, vi = im * cm - re * sm;
                        const bool okr = act && m <= n, oki = act && m <= n && m > 0;
                        // no branch around the adds (inactive lanes add 0 at a valid address)
                        atomicAdd(ap + n * n + (okr ? m : 0), okr ? vr : 0.0);
                        atomicAdd(ap + n * n + n + (oki ? m : 0), oki ? vi : 0.0);
                    }
                    const double a = cm * c4 - sm * s4, b = sm * c4 + cm * s4;
                    cm = a;
                    sm = b;
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        cur = nxt;
        nxt = nn;
        kc = k1;
        r0 = r1;
        k1 = k2;
        r1 = r2;
    }
    __syncthreads();
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += NT) {
        const int sl = idx / (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + idx % (2 * P2)] = acc[idx];
    }
}

// the sources of one level in the quarter layout: box b of the level at Mq[(b * 16 + role) * NQP],
// role = 8 pot + 4 part + q (the lane's low four bits), entry hoff(n) + j = order n, m = 4j + q of
// that potential and part; zero where m > n, for (Im, m = 0) and in the padding
template <int P>
__global__ void __launch_bounds__(256) k_mquarter(int64_t off, int64_t nb, const double *__restrict__ M,
                                                  double *__restrict__ Mq)
{
    using Sh = qv::Shape<P>;
    constexpr int NQP = Sh::NQP, NQ = Sh::NQ, NE = 16 * NQP, P2 = P * P;
    __shared__ int16_t src[NE];
    for (int t = threadIdx.x; t < NE; t += blockDim.x) {
        const int r = t / NQP, e = t % NQP;
        const int pot = r >> 3, part = (r >> 2) & 1, q = r & 3;
        int k = -1;
        if (e < NQ) {
            int n = 0;
            while (qv::hoff(n + 1) <= e) n++;
            const int m = 4 * (e - qv::hoff(n)) + q;
            if (m <= n && !(part && m == 0)) k = pot * P2 + n * n + (part ? n : 0) + m;
        }
        src[t] = (int16_t)k;
    }
    __syncthreads();
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const double *mb = M + (size_t)(off + b) * 2 * P2;
        double *hb = Mq + (size_t)b * NE;
        for (int t = threadIdx.x; t < NE; t += blockDim.x) {
            const int k = src[t];
            hb[t] = k >= 0 ? mb[k] : 0.0;
        }
    }
}

// Forward (S-basis) rotation tables of every polar-angle class in the quarter layout:
// [part: Re, Im][residue q][order n][group k][row j'][RL(n)] (each table padded to WQS entries);
// row j' of group k is m' = 4j' + (q ^ k), column i is m = 4i + q; the Im block (m, m' >= 1) is
// embedded with zeros at m = 0 and m' = 0; zero where m or m' > n.
template <int P>
__global__ void k_wquarter(const double *__restrict__ rot, double *__restrict__ wq, int64_t stride)
{
    using Sh = qv::Shape<P>;
    const int th = blockIdx.x;
    const double *Rf = rot + ((size_t)th * ROT_NKIND + ROT_S_FWD) * rot_set_size(P);
    for (int idx = threadIdx.x; idx < stride; idx += blockDim.x) {
        double val = 0.0;
        const int tb = idx / Sh::WQS, e = idx % Sh::WQS;
        const int part = tb >> 2, q = tb & 3;
        if (e < Sh::WQ) {
            int n = 0;
            while (qv::woff(n + 1) <= e) n++;
            const int r = e - qv::woff(n), row = r / qv::RL(n), i = r % qv::RL(n);
            const int kk = row / qv::S(n), jr = row % qv::S(n);
            const int mp = 4 * jr + (q ^ kk), m = 4 * i + q;
            if (i < qv::S(n) && mp <= n && m <= n) {
                const double *blk = Rf + rot_block_off(n);
                if (part == 0) val = blk[mp * (n + 1) + m];
                else if (mp > 0 && m > 0) val = blk[(n + 1) * (n + 1) + (mp - 1) * n + (m - 1)];
            }
        }
        wq[(size_t)th * stride + idx] = val;
    }
}

__global__ void k_dirtab_q(double *__restrict__ tab)
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

// ---------------------------------------------------------------------------
// M2M and L2L at the high orders in the same lane layout.  One wavefront per parent box; its
// children's shifts four at a time (one per 16 lanes: t = lane >> 4), the same RCR steps as the
// M2L above: rotation about z (phases of the child direction), rotation about y (forward table
// of the direction's polar class), coaxial (S|S) (M2M) or (R|R) (L2L) shift along z by the
// parent-child distance with the S- or R-conversion (eq. rcr1) per column m = 4c + q, rotation
// back about y (the class's back table, read as rows like the forward one) and about z.
// M2M sums the four shifts by lane exchanges (lane ^ 16, ^ 32) and the wavefront writes the
// parent's multipole (first group of children) or adds to it (second group); L2L writes each
// child's local expansion.  The rotation tables (a class's forward and back tables, 186 KB at
// p = 23) are read from global memory: only two polar classes occur, so they stay in the caches.
// ---------------------------------------------------------------------------
namespace qv {
__host__ __device__ constexpr double taup() { return 0.4330127018922193; }  // sqrt(3)/4
// (-tau_p)^k / k! as a compile-time constant
__host__ __device__ constexpr double mm_cf(int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; i++) c *= -taup() / (double)i;
    return c;
}
// the sum of a lane's value over lanes l, l ^ 32 (permlane32 swap of the value with itself)
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
}  // namespace qv

template <int P, int KIND>
__global__ void __launch_bounds__(256, 1) k_mm_quarter(int64_t poff, int64_t npar, const int32_t *__restrict__ bchild0,
                                                       const int32_t *__restrict__ bnchild,
                                                       const int32_t *__restrict__ bparent,
                                                       const uint64_t *__restrict__ bkey,
                                                    const double *__restrict__ src_exp, double *__restrict__ dst_exp,
                                                    const double *__restrict__ wq, int64_t wstride,
                                                    const int16_t *__restrict__ dir_theta,
                                                    const double *__restrict__ zph)
{
    static_assert(KIND == 0 || KIND == 2, "M2M or L2L");
    using Sh = qv::Shape<P>;
    using qv::hoff;
    using qv::S;
    constexpr int P2 = Sh::P2, NQ = Sh::NQ, WQS = Sh::WQS;
    constexpr int DIR0 = NDIR_M2L + (KIND == 0 ? 0 : 8);  // child->parent (M2M), parent->child (L2L)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = lane >> 4, pot0 = (lane >> 3) & 1, part0 = (lane >> 2) & 1, q0 = lane & 3;
    // coefficient tables in LDS, read through an opaque pointer (as compile-time constants the
    // compiler would keep all of them in registers across the loop): (-tau_p)^k / k!, 1 / n
    __shared__ double ktab[2 * 32];
    if (threadIdx.x < 32) {
        ktab[threadIdx.x] = threadIdx.x < P ? qv::mm_cf(threadIdx.x) : 0.0;
        ktab[32 + threadIdx.x] = threadIdx.x ? 1.0 / (double)threadIdx.x : 0.0;
    }
    __syncthreads();

    // M2M: one wavefront per parent (poff, npar: the parents' level), its children four at a time;
    // L2L: four consecutive children per wavefront (poff, npar: the children's level)
    for (int64_t pq = (int64_t)blockIdx.x * 4 + wave; KIND == 0 ? pq < npar : 4 * pq < npar;
         pq += (int64_t)gridDim.x * 4) {
        const int64_t b0 = KIND == 0 ? poff + pq : 0;
        const int nc = KIND == 0 ? bnchild[b0] : (npar - 4 * pq < 4 ? (int)(npar - 4 * pq) : 4);
        if (nc == 0) continue;  // M2M: a leaf keeps its own multipole
        const int c0 = KIND == 0 ? bchild0[b0] : (int)(poff + 4 * pq);
        for (int bt = 0; bt < nc; bt += 4) {
            // the lane's role, opaque per batch: keeps the compiler from hoisting the per-lane gather
            // and scatter offsets of all entries out of the loop (which would exhaust the registers)
            int part = part0, q = q0, pot = pot0;
            asm volatile("" : "+v"(part), "+v"(q), "+v"(pot));
            const bool act = bt + t < nc;
            const int cb = c0 + (act ? bt + t : 0);
            const int64_t b = KIND == 0 ? b0 : (int64_t)bparent[cb];  // the parent
            const int oct = (int)(bkey[cb] & 7u);
            const int dir = DIR0 + oct;
            const double *Wt = wq + (size_t)dir_theta[dir] * 2 * wstride + (part * 4 + q) * WQS;  // forward
            const double *zc = zph + (size_t)dir * 2 * P, *zs = zc + P;  // cos, sin of m phi
            // the source's entries m = 4j + q of this lane's potential and part
            const double *sp = src_exp + (size_t)(KIND == 0 ? cb : b) * 2 * P2 + pot * P2;
            double v[NQ];
            // all loads first (clamped to the row: every address inside the box), then the masks
#pragma unroll
            for (int n = 0; n < P; n++)
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    const int m = 4 * jj + q;
                    v[hoff(n) + jj] = sp[n * n + part * n + (m <= n ? m : n)];
                }
#pragma unroll
            for (int n = 0; n < P; n++)
#pragma unroll
                for (int jj = 0; jj < S(n); jj++) {
                    const int m = 4 * jj + q;
                    const bool ok = act && m <= n && !(part && m == 0);
                    v[hoff(n) + jj] = ok ? v[hoff(n) + jj] : 0.0;
                }
            // 1. rotate about z by +phi: Re' = re c - im s, Im' = im c + re s
            {
                const double sgn = part ? 1.0 : -1.0;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
                    const int m = 4 * jj + q < P ? 4 * jj + q : 0;
                    const double cm = zc[m], sz = zs[m] * sgn;
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double x = v[hoff(n) + jj];
                        const double o = qv::xor4(x);
                        v[hoff(n) + jj] = x * cm + o * sz;
                    }
                }
            }
            // 2. and 5.: rotation about y of every order with table W: partial sums of the four
            //    output groups over the lane's columns, then the quad butterfly
            auto rotate_y = [&](const double *W) __attribute__((always_inline)) {
#pragma unroll
                for (int n = 0; n < P; n++) {
                    // one opaque base address per order: the rows' loads take immediate offsets from it
                    // (precomputed addresses of every row would fill the register file)
                    const double *Wn = W + qv::woff(n);
                    asm volatile("" : "+v"(Wn));
                    constexpr int SM = (P - 1) / 4 + 1;
                    double g[4][SM];
                    // the table rows in pairs, the next pair's loads issued before this pair's dot
                    // products (software pipelining, as in the M2L above)
                    {
                        constexpr int GR = 2;
                        constexpr int RLMAX = qv::RL(P - 1) / 2;
                        const int R = 4 * S(n), H = qv::RL(n) / 2, NG = (R + GR - 1) / GR;
                        double2 buf[2][GR][RLMAX];
                        auto ld = [&](int gg, double2 (&b)[GR][RLMAX]) __attribute__((always_inline)) {
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++)
                                        if (h < H) b[rr][h] = ((const double2 *)(Wn + row * qv::RL(n)))[h];
                                }
                            }
                        };
                        ld(0, buf[0]);
#pragma unroll
                        for (int gg = 0; gg < (4 * S(P - 1) + GR - 1) / GR; gg++) {
                            if (gg >= NG) break;
                            if (gg + 1 < NG) ld(gg + 1, buf[(gg + 1) & 1]);
#pragma unroll
                            for (int rr = 0; rr < GR; rr++) {
                                const int row = gg * GR + rr;
                                if (row < R) {
                                    const int kk = row / S(n), jj = row % S(n);
                                    double a = 0;
#pragma unroll
                                    for (int h = 0; h < RLMAX; h++) {
                                        if (h >= H) break;
                                        a += buf[gg & 1][rr][h].x * v[hoff(n) + 2 * h];
                                        if (2 * h + 1 < S(n)) a += buf[gg & 1][rr][h].y * v[hoff(n) + 2 * h + 1];
                                    }
                                    g[kk][jj] = a;
                                }
                            }
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
#pragma unroll
                    for (int jj = 0; jj < S(n); jj++) {
                        const double a = g[0][jj] + dpp_f<DPP_XOR1>(g[1][jj]);
                        const double bb = g[2][jj] + dpp_f<DPP_XOR1>(g[3][jj]);
                        v[hoff(n) + jj] = a + dpp_f<DPP_XOR2>(bb);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            rotate_y(Wt);
            // 3+4. per column m = 4c + q: coaxial shift, then the conversion
            {
                const double *kt = ktab;
                asm volatile("" : "+v"(kt));
                const double *cf = kt, *rn = kt + 32;
                const double wphi = pot ? 0.0 : 1.0, wchi = pot ? 1.0 : 0.0;
#pragma unroll
                for (int c = 0; c < S(P - 1); c++) {
                    const int n0 = 4 * c;
                    const double mval = (double)(4 * c + q);
                    // the column's entries are read in place (they are overwritten only after out[]),
                    // through an opaque copy: otherwise the compiler starts the sums of every column
                    // while the rotation produces their entries and runs out of registers
#pragma unroll
                    for (int n2 = n0; n2 < P; n2++) asm volatile("" : "+v"(v[hoff(n2) + c]));
                    double out[P];
                    if (KIND == 0) {
                        // (S|S): out_n = sum_{n' = m}^{n} cf_{n-n'} (1/2 [phi] | 1 [chi]) 2^-n' in_n'
                        const int e0 = pot ? 0 : -1;
#pragma unroll
                        for (int n2 = n0; n2 < P; n2++) v[hoff(n2) + c] = ldexp(v[hoff(n2) + c], e0 - n2);
#pragma unroll
                        for (int n = n0; n < P; n++) {
                            double a = 0;
#pragma unroll
                            for (int n2 = n0; n2 <= n; n2++) a += cf[n - n2] * v[hoff(n2) + c];
                            out[n] = a;
                        }
                    } else {
                        // (R|R): out_n = (1 [phi] | 1/2 [chi]) 2^-n sum_{n' = n}^{p-1} cf_{n'-n} in_n'
                        const int e0 = pot ? -1 : 0;
#pragma unroll
                        for (int n = n0; n < P; n++) {
                            double a = 0;
#pragma unroll
                            for (int n2 = n; n2 < P; n2++) a += cf[n2 - n] * v[hoff(n2) + c];
                            out[n] = ldexp(a, e0 - n);
                        }
                    }
#pragma unroll
                    for (int n = n0; n < P; n++) {
                        const double other = swz_xor<12>(out[n]);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                        double val;
                        if (KIND == 0) {
                            // S-conversion: phi~ = phi - i tau m/(n+1) chi,  chi~_n = chi_n + tau/n chi_{n-1}
                            const double tau = qv::taup();
                            const double fphi = tau * mval * rn[n + 1] * (part ? -1.0 : 1.0) * wphi;
                            const double prev = (n > n0) ? out[n - 1] : 0.0;
                            const double fchi = tau * rn[n] * wchi;  // rn[0] = 0
                            val = out[n] + fphi * other + fchi * prev;
                        } else {
                            // R-conversion: phi~ = phi + i tau m/n chi,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
                            const double tau = 2.0 * qv::taup();
                            const double fphi = tau * mval * rn[n] * (part ? 1.0 : -1.0) * wphi;  // rn[0] = 0
                            const double next = (n + 1 < P) ? out[n + 1] : 0.0;
                            const double fchi = -tau * rn[n + 1] * wchi;
                            val = out[n] + fphi * other + fchi * next;
                        }
                        v[hoff(n) + c] = (n - n0 < q) ? 0.0 : val;  // slot (n, c) holds m = 4c + q > n: empty
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            rotate_y(Wt + wstride);  // the back table of the class
            // the lane's role again, opaque: the offsets and phases of the gather and of step 1 are
            // recomputed rather than kept live through the translation
            asm volatile("" : "+v"(part), "+v"(q), "+v"(pot));
            zc = zph + (size_t)dir * 2 * P;
            asm volatile("" : "+v"(zc));
            zs = zc + P;
            // 6. rotate about z by -phi: Re' = re c + im s, Im' = im c - re s
            {
                const double sgn = part ? -1.0 : 1.0;
#pragma unroll
                for (int jj = 0; jj < S(P - 1); jj++) {
                    const int m = 4 * jj + q < P ? 4 * jj + q : 0;
                    const double cm = zc[m], sz = zs[m] * sgn;
#pragma unroll
                    for (int n = 4 * jj; n < P; n++) {
                        const double x = v[hoff(n) + jj];
                        const double o = qv::xor4(x);
                        v[hoff(n) + jj] = x * cm + o * sz;
                    }
                }
            }
            if (KIND == 0) {
                // sum over the four children of this group (lane ^ 16, ^ 32); the first group writes
                // the parent's multipole, the second adds to it
#pragma unroll
                for (int i = 0; i < NQ; i++) {
                    double x = v[i];
                    x += swz_xor<16>(x);
                    v[i] = qv::xor32_sum(x);
                }
                if (t == 0) {
                    double *dp = dst_exp + (size_t)b * 2 * P2 + pot * P2;
#pragma unroll
                    for (int n = 0; n < P; n++)
#pragma unroll
                        for (int jj = 0; jj < S(n); jj++) {
                            const int m = 4 * jj + q;
                            if (m <= n && !(part && m == 0)) {
                                const int k = n * n + part * n + m;
                                dp[k] = bt ? dp[k] + v[hoff(n) + jj] : v[hoff(n) + jj];
                            }
                        }
                }
            } else if (act) {
                double *dp = dst_exp + (size_t)cb * 2 * P2 + pot * P2;
#pragma unroll
                for (int n = 0; n < P; n++)
#pragma unroll
                    for (int jj = 0; jj < S(n); jj++) {
                        const int m = 4 * jj + q;
                        if (m <= n && !(part && m == 0)) dp[n * n + part * n + m] = v[hoff(n) + jj];
                    }
            }
        }
    }
}

// Forward and back rotation tables of every polar-angle class for M2M (S basis both ways) or L2L
// (R basis both ways) in the quarter layout of k_wquarter: [class][fwd, back][part][residue][WQS]
template <int P>
__global__ void k_wquarter_mm(const double *__restrict__ rot, double *__restrict__ wq, int64_t stride, int kfwd,
                              int kback)
{
    using Sh = qv::Shape<P>;
    const int th = blockIdx.x, fb = blockIdx.y;
    const double *Rf = rot + ((size_t)th * ROT_NKIND + (fb ? kback : kfwd)) * rot_set_size(P);
    double *dst = wq + ((size_t)th * 2 + fb) * stride;
    for (int idx = threadIdx.x; idx < stride; idx += blockDim.x) {
        double val = 0.0;
        const int tb = idx / Sh::WQS, e = idx % Sh::WQS;
        const int part = tb >> 2, q = tb & 3;
        if (e < Sh::WQ) {
            int n = 0;
            while (qv::woff(n + 1) <= e) n++;
            const int r = e - qv::woff(n), row = r / qv::RL(n), i = r % qv::RL(n);
            const int kk = row / qv::S(n), jr = row % qv::S(n);
            const int mp = 4 * jr + (q ^ kk), m = 4 * i + q;
            if (i < qv::S(n) && mp <= n && m <= n) {
                const double *blk = Rf + rot_block_off(n);
                if (part == 0) val = blk[mp * (n + 1) + m];
                else if (mp > 0 && m > 0) val = blk[(n + 1) * (n + 1) + (mp - 1) * n + (m - 1)];
            }
        }
        dst[idx] = val;
    }
}

namespace {

template <int P>
static bool wquarter_build_t(lhf_plan *Pl, hipStream_t st)
{
    constexpr size_t shm = qv::tile_bytes<P>();
    static_assert(shm <= (size_t)qv::LDS_MAX, "tile exceeds the LDS");
    static_assert(qv::nslot<P>() >= 1, "no target slot fits beside the tables");
    if (Pl->sched_ncls > qv::MAXCLS) return false;
    const int64_t stride = 8 * (int64_t)qv::Shape<P>::WQS;
    if (dev_malloc(&Pl->whalf, sizeof(double) * stride * Pl->n_theta) != hipSuccess) return false;
    k_wquarter<P><<<dim3((unsigned)Pl->n_theta), dim3(256), 0, st>>>((const double *)Pl->rot, (double *)Pl->whalf,
                                                                     stride);
    // class order of the kernel: each polar angle theta > pi/2 right after its mirror pi - theta, whose
    // table it reuses (one staging for both); [order | staged table | mirrored]
    {
        const int nc = Pl->sched_ncls;
        std::vector<int16_t> &qs = Pl->h_qsched;
        qs.assign(3 * (size_t)nc, 0);
        std::vector<char> used(nc, 0);
        auto th = [&](int c) { return Pl->h_theta[Pl->h_cls_theta[c]]; };
        const double pi = 3.14159265358979323846;
        int o = 0;
        for (int a = 0; a < nc; a++) {
            if (used[a]) continue;
            int b = -1;
            for (int c = 0; c < nc && b < 0; c++)
                if (c != a && !used[c] && std::fabs(th(a) + th(c) - pi) < 1e-9) b = c;
            int can = a, mir = b;
            if (b >= 0 && th(a) > 0.5 * pi) std::swap(can, mir);
            used[a] = 1;
            if (b >= 0) used[b] = 1;
            qs[o] = (int16_t)can;
            qs[nc + o] = Pl->h_cls_theta[can];
            qs[2 * nc + o] = 0;
            o++;
            if (b >= 0) {
                qs[o] = (int16_t)mir;
                qs[nc + o] = Pl->h_cls_theta[can];
                qs[2 * nc + o] = 1;
                o++;
            }
        }
        if (dev_malloc(&Pl->qsched, sizeof(int16_t) * qs.size()) != hipSuccess) return false;
        if (hipMemcpyAsync(Pl->qsched, qs.data(), sizeof(int16_t) * qs.size(), hipMemcpyHostToDevice, st) != hipSuccess)
            return false;
    }
    if (dev_malloc(&Pl->dtab, sizeof(double) * 4 * 343) != hipSuccess) return false;
    k_dirtab_q<<<dim3(2), dim3(256), 0, st>>>(Pl->dtab);
    int64_t nbmax = 0;
    for (int l = 2; l <= Pl->depth; l++) nbmax = std::max(nbmax, Pl->lev[l].nb);
    if (nbmax > 0 && dev_malloc(&Pl->mh, sizeof(double) * 16 * qv::Shape<P>::NQP * nbmax) != hipSuccess) return false;
    return hipFuncSetAttribute((const void *)k_m2l_quarter<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm) == hipSuccess;
}

template <int P>
static void stage_quarter(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t nb = Pl->lev[level].nb;
    if (nb == 0) return;
    k_mquarter<P><<<dim3((unsigned)std::min<int64_t>(nb, 8192)), dim3(256), 0, st>>>(
        Pl->lev[level].off, nb, (const double *)Pl->M, (double *)Pl->mh);
}

template <int P>
static bool qmfma_build_t(lhf_plan *Pl, hipStream_t st)
{
    constexpr size_t shm = qm::tile_bytes<P>();
    static_assert(shm <= (size_t)qv::LDS_MAX, "tile exceeds the LDS");
    static_assert(qm::nslot<P>() >= 1, "no target slot fits beside the table");
    if (Pl->sched_ncls > qm::MAXCLS) return false;
    if (dev_malloc(&Pl->dtab, sizeof(double) * 4 * 343) != hipSuccess) return false;
    k_dirtab_q<<<dim3(2), dim3(256), 0, st>>>(Pl->dtab);
    int64_t nbmax = 0;
    for (int l = 2; l <= Pl->depth; l++) nbmax = std::max(nbmax, Pl->lev[l].nb);
    if (nbmax > 0 && dev_malloc(&Pl->mh, sizeof(double) * 16 * qv::Shape<P>::NQP * nbmax) != hipSuccess) return false;
    return hipFuncSetAttribute((const void *)k_m2l_qmfma<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm) == hipSuccess;
}

template <int P>
static void launch_qmfma(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t soff = Pl->lev[level].off, nb = Pl->lev[level].nb;
    if (nb == 0) return;
    const int ns = Pl->m2l_ns[level] > 0
                       ? std::min(Pl->m2l_ns[level], qm::nslot<P>())
                       : (int)std::max<int64_t>(1, std::min<int64_t>(qm::nslot<P>(), (nb + 1023) / 1024));
    const int64_t ntiles = (nb + ns - 1) / ns;
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls, Pl->sched_row_start, Pl->sched_rows};
    k_m2l_qmfma<P><<<dim3((unsigned)(per * 8)), dim3(qm::NTHREADS), qm::tile_bytes<P>(), st>>>(
        level, soff, nb, ns, Pl->bkey, Pl->dmap[level], (const double *)Pl->mh, (double *)Pl->Lc,
        (const double *)Pl->rot, sch, Pl->sched_cls_theta, Pl->dtab);
}

template <int P>
static void launch_quarter(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t soff = Pl->lev[level].off, nb = Pl->lev[level].nb;
    if (nb == 0) return;
    // the plan's tuned choice, else as many slots as fit but no fewer than ~1024 tiles where the
    // level has the boxes
    const int ns = Pl->m2l_ns[level] > 0
                       ? std::min(Pl->m2l_ns[level], qv::nslot<P>())
                       : (int)std::max<int64_t>(1, std::min<int64_t>(qv::nslot<P>(), (nb + 1023) / 1024));
    const int64_t ntiles = (nb + ns - 1) / ns;
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls, Pl->sched_row_start, Pl->sched_rows};
    k_m2l_quarter<P><<<dim3((unsigned)(per * 8)), dim3(qv::NTHREADS), qv::tile_bytes<P>(), st>>>(
        level, soff, nb, ns, Pl->bkey, Pl->dmap[level], (const double *)Pl->mh, (double *)Pl->Lc,
        (const double *)Pl->whalf, 8 * (int64_t)qv::Shape<P>::WQS, sch, Pl->qsched, Pl->dtab);
}


template <int P>
static bool mmquarter_build_t(lhf_plan *Pl, hipStream_t st)
{
    const int64_t stride = 8 * (int64_t)qv::Shape<P>::WQS;
    if (dev_malloc(&Pl->wmm, sizeof(double) * 2 * stride * Pl->n_theta) != hipSuccess) return false;
    if (dev_malloc(&Pl->wll, sizeof(double) * 2 * stride * Pl->n_theta) != hipSuccess) return false;
    k_wquarter_mm<P><<<dim3((unsigned)Pl->n_theta, 2), dim3(256), 0, st>>>((const double *)Pl->rot, (double *)Pl->wmm,
                                                                           stride, ROT_S_FWD, ROT_S_BACK);
    k_wquarter_mm<P><<<dim3((unsigned)Pl->n_theta, 2), dim3(256), 0, st>>>((const double *)Pl->rot, (double *)Pl->wll,
                                                                           stride, ROT_R_FWD, ROT_R_BACK);
    return hipGetLastError() == hipSuccess;
}

// KIND 0: M2M into the parents of level l; KIND 2: L2L from level l - 1 into level l (l >= 3)
template <int P, int KIND>
static void launch_mm_quarter(const lhf_plan *Pl, int l, hipStream_t st)
{
    // M2M: the parents of level l; L2L: the children of level l
    const int64_t off = Pl->lev[l].off, nb = Pl->lev[l].nb;
    if (nb == 0) return;
    const int64_t nwave = KIND == 0 ? nb : (nb + 3) / 4;
    const unsigned grid = (unsigned)std::min<int64_t>((nwave + 3) / 4, 16384);
    const double *src = (const double *)(KIND == 0 ? Pl->M : Pl->Lc);
    double *dst = (double *)(KIND == 0 ? Pl->M : Pl->Lc);
    k_mm_quarter<P, KIND><<<dim3(grid), dim3(256), 0, st>>>(
        off, nb, Pl->bchild0, Pl->bnchild, Pl->bparent, Pl->bkey, src, dst,
        (const double *)(KIND == 0 ? Pl->wmm : Pl->wll),
        8 * (int64_t)qv::Shape<P>::WQS, Pl->dir_theta, (const double *)Pl->zph);
}

__global__ void k_zero_exp_q(int64_t count, double *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = 0.0;
}

template <int KIND>
static void mm_quarter_dispatch(const lhf_plan *Pl, int l, hipStream_t st)
{
    switch (Pl->p) {
    case 20: launch_mm_quarter<20, KIND>(Pl, l, st); break;
    case 22: launch_mm_quarter<22, KIND>(Pl, l, st); break;
    case 23: launch_mm_quarter<23, KIND>(Pl, l, st); break;
    case 24: launch_mm_quarter<24, KIND>(Pl, l, st); break;
    }
}

}  // namespace

// targets per tile the quarter-vector M2L can take at order p (0: no such kernel)
int m2l_quarter_max_ns(int p)
{
    switch (p) {
    case 8: return qv::nslot<8>();
    case 10: return qv::nslot<10>();
    case 12: return qv::nslot<12>();
    case 16: return qv::nslot<16>();
    case 20: return qv::nslot<20>();
    case 22: return qv::nslot<22>();
    case 23: return qv::nslot<23>();
    case 24: return qv::nslot<24>();
    }
    return 0;
}

bool m2l_quarter_supported(int precision, int p)
{
    return precision == LHF_FP64 && (p == 8 || p == 10 || p == 12 || p == 16 || p == 20 || p == 22 || p == 23 || p == 24);
}

bool wquarter_build(lhf_plan *Pl, hipStream_t st)
{
    switch (Pl->p) {
    case 8: return wquarter_build_t<8>(Pl, st);
    case 10: return wquarter_build_t<10>(Pl, st);
    case 12: return wquarter_build_t<12>(Pl, st);
    case 16: return wquarter_build_t<16>(Pl, st);
    case 20: return wquarter_build_t<20>(Pl, st);
    case 22: return wquarter_build_t<22>(Pl, st);
    case 23: return wquarter_build_t<23>(Pl, st);
    case 24: return wquarter_build_t<24>(Pl, st);
    }
    return false;
}

void m2l_quarter_stage(const lhf_plan *Pl, int level, hipStream_t st)
{
    switch (Pl->p) {
    case 8: stage_quarter<8>(Pl, level, st); break;
    case 10: stage_quarter<10>(Pl, level, st); break;
    case 12: stage_quarter<12>(Pl, level, st); break;
    case 16: stage_quarter<16>(Pl, level, st); break;
    case 20: stage_quarter<20>(Pl, level, st); break;
    case 22: stage_quarter<22>(Pl, level, st); break;
    case 23: stage_quarter<23>(Pl, level, st); break;
    case 24: stage_quarter<24>(Pl, level, st); break;
    }
}

void m2l_quarter_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    switch (Pl->p) {
    case 8: launch_quarter<8>(Pl, level, st); break;
    case 10: launch_quarter<10>(Pl, level, st); break;
    case 12: launch_quarter<12>(Pl, level, st); break;
    case 16: launch_quarter<16>(Pl, level, st); break;
    case 20: launch_quarter<20>(Pl, level, st); break;
    case 22: launch_quarter<22>(Pl, level, st); break;
    case 23: launch_quarter<23>(Pl, level, st); break;
    case 24: launch_quarter<24>(Pl, level, st); break;
    }
}

// the matrix-core M2L in the quarter residue layout (FP64 p = 20, 22, 23, 24)
bool m2l_qmfma_supported(int precision, int p)
{
    return precision == LHF_FP64 && (p == 20 || p == 22 || p == 23 || p == 24);
}

int m2l_qmfma_max_ns(int p)
{
    switch (p) {
    case 20: return qm::nslot<20>();
    case 22: return qm::nslot<22>();
    case 23: return qm::nslot<23>();
    case 24: return qm::nslot<24>();
    }
    return 0;
}

bool qmfma_build(lhf_plan *Pl, hipStream_t st)
{
    switch (Pl->p) {
    case 20: return qmfma_build_t<20>(Pl, st);
    case 22: return qmfma_build_t<22>(Pl, st);
    case 23: return qmfma_build_t<23>(Pl, st);
    case 24: return qmfma_build_t<24>(Pl, st);
    }
    return false;
}

void m2l_qmfma_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    switch (Pl->p) {
    case 20: launch_qmfma<20>(Pl, level, st); break;
    case 22: launch_qmfma<22>(Pl, level, st); break;
    case 23: launch_qmfma<23>(Pl, level, st); break;
    case 24: launch_qmfma<24>(Pl, level, st); break;
    }
}

bool mm_quarter_supported(int precision, int p)
{
    return precision == LHF_FP64 && (p == 20 || p == 22 || p == 23 || p == 24);
}

bool mmquarter_build(lhf_plan *Pl, hipStream_t st)
{
    switch (Pl->p) {
    case 20: return mmquarter_build_t<20>(Pl, st);
    case 22: return mmquarter_build_t<22>(Pl, st);
    case 23: return mmquarter_build_t<23>(Pl, st);
    case 24: return mmquarter_build_t<24>(Pl, st);
    }
    return false;
}

// M2M into the boxes of level l from their children
void m2m_quarter_launch(const lhf_plan *Pl, int l, hipStream_t st) { mm_quarter_dispatch<0>(Pl, l, st); }

// L2L into the boxes of level l from their parents; level 2 starts from zero
void l2l_quarter_launch(const lhf_plan *Pl, int l, hipStream_t st)
{
    if (l <= 2) {
        const int64_t cnt = Pl->lev[l].nb * 2 * (int64_t)Pl->p * Pl->p;
        if (cnt > 0)
            k_zero_exp_q<<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st>>>(
                cnt, (double *)Pl->Lc + Pl->lev[l].off * 2 * (int64_t)Pl->p * Pl->p);
        return;
    }
    mm_quarter_dispatch<2>(Pl, l, st);
}

}  // namespace lhf

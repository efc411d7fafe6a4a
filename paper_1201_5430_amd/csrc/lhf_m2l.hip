// lhf_m2l.hip -- batched multipole-to-local translation (the dominant stage).
//
// Each M2L translation is rotation -> coaxial (S|R) shift -> R-conversion
// (eq. rcr1) -> back-rotation (Sec. 4.4), applied to the two potentials.
// Work is organised so that translations sharing a rotation matrix run side
// by side:
//   * a workgroup owns a tile of two sibling groups (the <= 16 children of two
//     consecutive parent boxes) and accumulates their local expansions in LDS;
//   * the tile's translations (8 child positions x 189 offsets per sibling
//     group) are walked in polar-angle classes (49 classes); the forward (S
//     basis) and backward (R basis) rotation blocks of the class are staged in
//     LDS once and read as broadcasts;
//   * one lane = one (translation, potential, Re|Im part); the whole part
//     vector of P(P+1)/2 (+ one extra order for chi) values lives in
//     registers, so rotations and the coaxial shift are register FMAs;
//   * the coaxial shift along z by tau = |t|/h is
//       out_n = tau^-(n+1) sum_{n'} (n+n')! (tau^-n' in_n'),
//     i.e. one constant Hankel matrix of factorials between per-lane scalings;
//   * the conversion couples phi-Re with chi-Im and phi-Im with chi-Re: the
//     four lanes of a translation form a quad, so a quad swap supplies them;
//   * the back z-rotation needs the Re and Im parts: a pair swap supplies
//     them, then each lane adds its part into the LDS accumulator.
// The Im part is processed in the Re shape with a zero m = 0 slot, so every
// lane runs the same instruction stream.
#include <hip/hip_runtime.h>

#include "lhf_internal.h"
#include "lhf_m2l_common.h"

namespace lhf {

// rotation rows are padded to a multiple of E = 16 bytes so they load as 16-byte vectors
template <typename T>
__host__ __device__ constexpr int vecE() { return 16 / (int)sizeof(T); }
template <typename T>
__host__ __device__ constexpr int rowlen(int n) { return ((n + 1 + vecE<T>() - 1) / vecE<T>()) * vecE<T>(); }
template <typename T>
__host__ __device__ constexpr int wrow_off(int n)  // offset of order n's block: sum_{k<n} (k+1) rowlen(k)
{
    int o = 0;
    for (int k = 0; k < n; k++) o += (k + 1) * rowlen<T>(k);
    return o;
}

template <typename T, int P>
struct M2LShape {
    static constexpr int NV = P * (P + 1) / 2;      // (n, m <= n), n < P
    static constexpr int WB = wrow_off<T>(P);       // one padded rotation set (all orders)
};

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
};
template <>
struct Vec16<double> {
    using type = double2;
};

// one output row: sum_m W[m] in[m], W read as 16-byte vectors
template <typename T, bool WIDE>
__device__ __attribute__((always_inline)) inline T rowdot(const T *W, const T *in, const int N1)
{
    T a = 0;
    if (WIDE) {
        using V = typename Vec16<T>::type;
        constexpr int E = vecE<T>();
        const V *Wv = (const V *)W;
#pragma unroll
        for (int q = 0; q < (N1 + E - 1) / E; q++) {
            const V w = Wv[q];
            const T *wp = (const T *)&w;
#pragma unroll
            for (int e = 0; e < E; e++)
                if (q * E + e < N1) a += wp[e] * in[q * E + e];
        }
    } else {
        // element reads: every lane of a part reads the same address (LDS broadcast)
#pragma unroll
        for (int m = 0; m < N1; m++) a += W[m] * in[m];
    }
    return a;
}

// OWN = true: each wavefront owns two of the tile's eight sibling groups and walks the
// row table, so the 16 translations of a batch always have distinct targets that no
// other wavefront touches: accumulation is a plain LDS read-add-write.  OWN = false:
// the four wavefronts share the tile's targets and accumulate with LDS atomics.
// NREAL <= NPAR parents of the tile are real: in ownership mode the LDS may hold fewer than
// the eight sibling groups the wavefront layout addresses, and the missing ones stay empty.
template <typename T, int P, int NPAR, bool OWN, int NREAL>
__global__ void __launch_bounds__(256) k_m2l_tile(int level, int64_t poff, int64_t npar, int64_t loff, int64_t nbl,
                                                  const uint64_t *__restrict__ bkey, const int32_t *__restrict__ bchild0,
                                                  const int32_t *__restrict__ bnchild, const int32_t *__restrict__ dmap,
                                                  const T *__restrict__ M, T *__restrict__ Lc,
                                                  const T *__restrict__ wpad, int64_t wstride,
                                                  M2LSched sch, const int16_t *__restrict__ cls_theta)
{
    using S = M2LShape<T, P>;
    constexpr int P2 = P * P;
    // rotation rows per pinned group: two where registers allow, one for the largest vectors
    constexpr int RG = (sizeof(T) * P >= 64) ? 1 : 2;
    // 16-byte rotation-row reads for FP64; element reads (broadcast) for FP32
    constexpr bool WIDE = sizeof(T) == 8;
    // the next batch's source vector is loaded during the current batch where registers allow
    constexpr bool PREFETCH = (int)sizeof(T) * S::NV <= 256;
    constexpr int NSLOT = 8 * NPAR;              // addressable target slots
    constexpr int NACC = 8 * NREAL;              // slots with an accumulator (the rest never have a box)
    constexpr int SST = 2 * P2 + 1;              // odd slot stride: slots fall in different LDS banks
    constexpr int NENT = 1512;                   // schedule entries of one sibling group
    extern __shared__ char smem[];
    T *Wl = (T *)smem;                           // [2 kinds: fwd S, back R][2 parts][WB], 16-byte aligned
    T *acc = Wl + 4 * S::WB;                     // [NACC + 1][SST] (last slot absorbs inactive lanes)
    int *slot_xyz = (int *)(acc + (NACC + 1) * SST);  // [NSLOT] packed target coordinates, -1: no box
    int *slot_box = slot_xyz + NSLOT;            // [NSLOT] target box
    int *slot_sys = slot_box + NSLOT;            // [NSLOT] system of the target (offset into dmap)
    int16_t *cst = (int16_t *)(slot_sys + NSLOT);       // [ncls + 1] class starts (entries or rows)
    int16_t *ent = cst + 64;                     // [NENT] (dir << 3) | child position (shared mode)

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware tile order: consecutive tiles stay on one XCD (shared L2)
    const int64_t ntiles = (npar + NREAL - 1) / NREAL;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int ncls = sch.ncls;

    // slots: parent i (0..NPAR-1) x child position c (0..7)
    if (tid < NSLOT) {
        const int i = tid >> 3, c = tid & 7;
        int box = -1, xyz = -1;
        const int64_t q = (int64_t)NREAL * tile + i;
        if (i < NREAL && q < npar) {
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
            slot_sys[tid] = (int)(key >> (3 * level));
        } else {
            slot_sys[tid] = 0;
        }
        slot_box[tid] = box;
        slot_xyz[tid] = xyz;
    }
    if (!OWN)
        for (int i = tid; i < NENT; i += 256) ent[i] = (int16_t)((sch.ent_dir[i] << 3) | sch.ent_c[i]);
    for (int i = tid; i <= ncls; i += 256) cst[i] = OWN ? sch.row_start[i] : sch.cls_start[i];
    __syncthreads();
    for (int idx = tid; idx < NACC * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        acc[sl * SST + r] = box >= 0 ? Lc[(size_t)box * 2 * P2 + r] : (T)0;
    }

    const int side = 1 << level;
    const int t = lane >> 2, pot = (lane >> 1) & 1, part = lane & 1;

    // per-lane description of one batch position: (slot, dir) from LDS, source box by one global load
    struct Job {
        int slot, dir, src;
    };
    auto setup = [&](int k, int r0) -> Job {
        Job j{NACC, 0, -1};
        if (k >= ncls) return j;
        int slot, dir;
        if (OWN) {
            // r0 = row of the class; column = child position; wavefront w owns parents 2w, 2w+1
            const int col = t >> 1;
            dir = sch.rows[(size_t)(cst[k] + r0) * 8 + col];
            if (dir < 0) return j;
            slot = (2 * wave + (t & 1)) * 8 + col;
        } else {
            const int e0 = cst[k], cnt = cst[k + 1] - e0;
            const int tr = r0 + wave * 16 + t;
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
        if (OWN) {
            r0 += 1;
            if (k < ncls && r0 >= cst[k + 1] - cst[k]) {
                k++;
                r0 = 0;
            }
        } else {
            r0 += 64;
            if (k < ncls && r0 >= NPAR * (cst[k + 1] - cst[k])) {
                k++;
                r0 = 0;
            }
        }
    };
    auto load_part = [&](const Job &j, T *dst) {
        const T *sp = M + (size_t)(j.src >= 0 ? j.src : 0) * 2 * P2 + pot * P2;
#pragma unroll
        for (int n = 0; n < P; n++)
#pragma unroll
            for (int m = 0; m <= n; m++)
                dst[tri(n) + m] = (m == 0) ? (part ? (T)0 : sp[pk_re(n, 0)]) : sp[part ? pk_im(n, m) : pk_re(n, m)];
    };

    int k = 0, r0 = 0;           // current batch
    int k1 = 0, r1 = 0;          // next batch
    advance(k1, r1);
    Job cur = setup(k, r0), nxt = setup(k1, r1);
    T nv[PREFETCH ? S::NV : 1];
    if (PREFETCH) load_part(cur, nv);
    int staged = -1;
    while (k < ncls) {
        if (k != staged) {
            // stage the class's rotation blocks (precomputed in the LDS layout) with 16-byte loads
            __syncthreads();
            const uint4 *src4 = (const uint4 *)(wpad + (size_t)cls_theta[k] * wstride);
            uint4 *dst4 = (uint4 *)Wl;
            constexpr int N16 = (int)(4 * S::WB * sizeof(T) / 16);
#pragma unroll 8
            for (int i = tid; i < N16; i += 256) dst4[i] = src4[i];
            __syncthreads();
            staged = k;
        }
        // opaque per-batch offsets keep the compiler from hoisting every matrix entry
        // of the class out of the batch loop (which would exhaust the register file)
        int wfo = part * S::WB, wbo = 2 * S::WB + part * S::WB;
        asm volatile("" : "+v"(wfo), "+v"(wbo));
        const T *Wf = Wl + wfo;
        const T *Wb = Wl + wbo;

        const Job j = cur;
        const bool act = j.src >= 0;
        T v[S::NV];
        if (PREFETCH) {
#pragma unroll
            for (int q = 0; q < S::NV; q++) v[q] = nv[q];
        } else {
            load_part(j, v);
        }
        // look one batch further ahead: its source index now, its data right after
        int k2 = k1, r2 = r1;
        advance(k2, r2);
        const Job nn = setup(k2, r2);
        if (PREFETCH) load_part(nxt, nv);

        const int dir = j.dir;
        const int dx = dir % 7 - 3, dy = (dir / 7) % 7 - 3, dz = dir / 49 - 3;
        const T tau = (T)sqrt((double)(dx * dx + dy * dy + dz * dz));
        // e^{i phi} of the direction (phi = atan2(dy, dx); 0 on the z axis), FP64
        double cph = 1.0, sph = 0.0;
        {
            const double rho = sqrt((double)(dx * dx + dy * dy));
            if (rho > 0.0) {
                cph = (double)dx / rho;
                sph = (double)dy / rho;
            }
        }
        const T sgn_in = part ? (T)1 : (T)-1;   // z-rotation by +phi: Re' = re c - im s, Im' = im c + re s
        // 1. rotate about z by +phi using the partner lane's other part
        {
            double cm = 1.0, sm = 0.0;
#pragma unroll
            for (int m = 0; m < P; m++) {
                const T cz = (T)cm, sz = (T)sm * sgn_in;
#pragma unroll
                for (int n = m; n < P; n++) {
                    const T mine = v[tri(n) + m];
                    const T oth = dpp_f<DPP_XOR1>(mine);
                    if (m > 0) v[tri(n) + m] = mine * cz + oth * sz;
                }
                const double c2 = cm * cph - sm * sph, s2 = sm * cph + cm * sph;
                cm = c2;
                sm = s2;
            }
        }
        // 2. rotation about y (forward, S basis), two output rows per pinned group
#pragma unroll
        for (int n = 0; n < P; n++) {
            T in[P];
#pragma unroll
            for (int m = 0; m <= n; m++) in[m] = v[tri(n) + m];
            const T *W = Wf + wrow_off<T>(n);
#pragma unroll
            for (int mp = 0; mp <= n; mp += RG) {
                T a0 = rowdot<T, WIDE>(W + mp * rowlen<T>(n), in, n + 1);
                if (RG == 2 && mp + 1 <= n) {
                    T a1 = rowdot<T, WIDE>(W + (mp + 1) * rowlen<T>(n), in, n + 1);
                    asm volatile("" : "+v"(a0), "+v"(a1));
                    v[tri(n) + mp] = a0;
                    v[tri(n) + mp + 1] = a1;
                } else {
                    asm volatile("" : "+v"(a0));
                    v[tri(n) + mp] = a0;
                }
            }
        }
        // 3+4. per column m: coaxial (S|R) shift out_n = tau^-(n+1) sum_n' (n+n')! tau^-n' in_n'
        //      (chi to order P), then the R-conversion (eq. rcr1, scaled)
        //        phi~ = phi + i tau m/n chi ,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
        {
            const T itau = (T)1 / tau;
            T pw[P + 2];
            pw[0] = (T)1;
#pragma unroll
            for (int k = 1; k <= P + 1; k++) pw[k] = pw[k - 1] * itau;
            // lane roles as 0/1 weights (branch-free): phi lanes take the chi of the other part
            const T wphi = pot ? (T)0 : (T)1, wchi = pot ? (T)1 : (T)0;
            const T sconv = part ? (T)1 : (T)-1;
#pragma unroll
            for (int m = 0; m < P; m++) {
                T col[P];
#pragma unroll
                for (int n2 = m; n2 < P; n2++) col[n2] = v[tri(n2) + m] * pw[n2];
                T out[P + 1];
#pragma unroll
                for (int n = m; n <= P; n++) {
                    T a = 0;
#pragma unroll
                    for (int n2 = m; n2 < P; n2++) a += (T)dfact(n + n2) * col[n2];
                    out[n] = a * pw[n + 1];
                }
#pragma unroll
                for (int n = m; n < P; n++) {
                    const T other = dpp_f<DPP_XOR3>(out[n]);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                    const T fphi = (n > 0) ? tau * (T)((double)m / (double)n) * sconv * wphi : (T)0;
                    const T fchi = -tau * (T)(1.0 / (double)(n + 1)) * wchi;
                    v[tri(n) + m] = out[n] + fphi * other + fchi * out[n + 1];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // 5. back-rotation about y (R basis)
#pragma unroll
        for (int n = 0; n < P; n++) {
            T in[P];
#pragma unroll
            for (int m = 0; m <= n; m++) in[m] = v[tri(n) + m];
            const T *W = Wb + wrow_off<T>(n);
#pragma unroll
            for (int mp = 0; mp <= n; mp += RG) {
                T a0 = rowdot<T, WIDE>(W + mp * rowlen<T>(n), in, n + 1);
                if (RG == 2 && mp + 1 <= n) {
                    T a1 = rowdot<T, WIDE>(W + (mp + 1) * rowlen<T>(n), in, n + 1);
                    asm volatile("" : "+v"(a0), "+v"(a1));
                    v[tri(n) + mp] = a0;
                    v[tri(n) + mp + 1] = a1;
                } else {
                    asm volatile("" : "+v"(a0));
                    v[tri(n) + mp] = a0;
                }
            }
        }
        // 6. back-rotation about z (-phi) and accumulation into the target slot (branch-free;
        //    inactive lanes add into the spare slot)
        {
            T *ap = acc + (size_t)(act ? j.slot : NACC) * SST + pot * P2;
            T *spare = acc + (size_t)NACC * SST + pot * P2;
            const T sgn_out = part ? (T)-1 : (T)1;  // Re' = re c + im s, Im' = im c - re s
            double cm = 1.0, sm = 0.0;
#pragma unroll
            for (int m = 0; m < P; m++) {
                const T cz = (T)cm, sz = (T)sm * sgn_out;
                {
                    const double c2 = cm * cph - sm * sph, s2 = sm * cph + cm * sph;
                    cm = c2;
                    sm = s2;
                }
#pragma unroll
                for (int n = m; n < P; n++) {
                    const T mine = v[tri(n) + m];
                    const T oth = dpp_f<DPP_XOR1>(mine);
                    const int off = (m == 0) ? pk_re(n, 0) : (part ? pk_im(n, m) : pk_re(n, m));
                    const T val = (m == 0) ? mine : mine * cz + oth * sz;
                    if (OWN) {
                        // m = 0 has no imaginary part: the Im lane must not touch the Re entry
                        T *dst = (m == 0 && part) ? spare + off : ap + off;
                        *dst += val;
                    } else {
                        atomicAdd(&ap[off], val);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }

        cur = nxt;
        nxt = nn;
        k = k1;
        r0 = r1;
        k1 = k2;
        r1 = r2;
    }
    __syncthreads();
    for (int idx = tid; idx < NACC * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + r] = acc[sl * SST + r];
    }
}

// Ownership mode with two schedule rows per batch.  Each lane carries the translations of
// rows r and r+1 of its (parent, child position): both have the same target, so every
// rotation row read from LDS serves two translations and one accumulation adds both.  (The
// rotation-row broadcasts, not the arithmetic, bound the one-row kernel.)
template <typename T, int P>
__global__ void __launch_bounds__(256) k_m2l_tile2(int level, int64_t poff, int64_t npar,
                                                   const uint64_t *__restrict__ bkey,
                                                   const int32_t *__restrict__ bchild0,
                                                   const int32_t *__restrict__ bnchild, const int32_t *__restrict__ dmap,
                                                   const T *__restrict__ M, T *__restrict__ Lc,
                                                   const T *__restrict__ wpad, int64_t wstride, M2LSched sch,
                                                   const int16_t *__restrict__ cls_theta)
{
    using S = M2LShape<T, P>;
    constexpr int P2 = P * P;
    constexpr bool WIDE = sizeof(T) == 8;
    constexpr int NSLOT = 64;
    constexpr int SST = 2 * P2 + 1;
    extern __shared__ char smem[];
    T *Wl = (T *)smem;                           // [2 kinds][2 parts][WB]
    T *acc = Wl + 4 * S::WB;                     // [NSLOT + 1][SST] (last slot: Im lanes of m = 0)
    int *slot_xyz = (int *)(acc + (NSLOT + 1) * SST);
    int *slot_box = slot_xyz + NSLOT;
    int *slot_sys = slot_box + NSLOT;
    int16_t *cst = (int16_t *)(slot_sys + NSLOT);  // [ncls + 1] row starts

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ntiles = (npar + 7) / 8;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int ncls = sch.ncls;
    if (tid < NSLOT) {
        const int i = tid >> 3, c = tid & 7;
        int box = -1, xyz = -1, sys = 0;
        const int64_t q = (int64_t)8 * tile + i;
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
    }
    for (int i = tid; i <= ncls; i += 256) cst[i] = sch.row_start[i];
    __syncthreads();
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        acc[sl * SST + r] = box >= 0 ? Lc[(size_t)box * 2 * P2 + r] : (T)0;
    }

    const int side = 1 << level;
    const int t = lane >> 2, pot = (lane >> 1) & 1, part = lane & 1;
    const int col = t >> 1;
    const int slot = (2 * wave + (t & 1)) * 8 + col;  // this lane's target, the same for every row
    // source box of this lane's translation in row r of class k (-1: none)
    auto source = [&](int k, int r, int &dir) -> int {
        dir = 0;
        if (k >= ncls || r >= cst[k + 1] - cst[k]) return -1;
        dir = sch.rows[(size_t)(cst[k] + r) * 8 + col];
        const int xyz = slot_xyz[slot];
        if (dir < 0 || xyz < 0) return -1;
        const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                  sz = (xyz >> 20) - (dir / 49 - 3);
        if (sx < 0 || sy < 0 || sz < 0 || sx >= side || sy >= side || sz >= side) return -1;
        return dmap[(((size_t)slot_sys[slot] * side + sz) * side + sy) * side + sx];
    };
    // a missing source gives zeros by selection, never by scaling what box 0 holds (the two
    // translations of a lane share one accumulation, so a NaN there would reach the target)
    auto load_part = [&](int src, T *dst) {
        const T *sp = M + (size_t)(src >= 0 ? src : 0) * 2 * P2 + pot * P2;
        const bool on = src >= 0;
#pragma unroll
        for (int n = 0; n < P; n++)
#pragma unroll
            for (int m = 0; m <= n; m++) {
                const T x = (m == 0) ? (part ? (T)0 : sp[pk_re(n, 0)]) : sp[part ? pk_im(n, m) : pk_re(n, m)];
                dst[tri(n) + m] = on ? x : (T)0;
            }
    };
    // two dot products sharing one read of the rotation row
    auto rowdot2 = [&](const T *W, const T *a, const T *b, const int N1, T &ra, T &rb) {
        T x = 0, y = 0;
        if (WIDE) {
            using Vt = typename Vec16<T>::type;
            constexpr int E = vecE<T>();
            const Vt *Wv = (const Vt *)W;
#pragma unroll
            for (int q = 0; q < (P + E - 1) / E; q++) {
                if (q * E >= N1) break;
                const Vt w = Wv[q];
                const T *wp = (const T *)&w;
#pragma unroll
                for (int e = 0; e < E; e++)
                    if (q * E + e < N1) {
                        x += wp[e] * a[q * E + e];
                        y += wp[e] * b[q * E + e];
                    }
            }
        } else {
#pragma unroll
            for (int m = 0; m < P; m++)
                if (m < N1) {
                    const T w = W[m];
                    x += w * a[m];
                    y += w * b[m];
                }
        }
        ra = x;
        rb = y;
    };
    auto rotate_y = [&](const T *Wbase, T *v0, T *v1) {
#pragma unroll
        for (int n = 0; n < P; n++) {
            T in0[P], in1[P];
#pragma unroll
            for (int m = 0; m <= n; m++) {
                in0[m] = v0[tri(n) + m];
                in1[m] = v1[tri(n) + m];
            }
            const T *W = Wbase + wrow_off<T>(n);
#pragma unroll
            for (int mp = 0; mp <= n; mp++) {
                T a0, a1;
                rowdot2(W + mp * rowlen<T>(n), in0, in1, n + 1, a0, a1);
                asm volatile("" : "+v"(a0), "+v"(a1));
                v0[tri(n) + mp] = a0;
                v1[tri(n) + mp] = a1;
            }
        }
    };
    auto angles = [&](int dir, double &cph, double &sph, T &tau) {
        const int dx = dir % 7 - 3, dy = (dir / 7) % 7 - 3, dz = dir / 49 - 3;
        tau = (T)sqrt((double)(dx * dx + dy * dy + dz * dz));
        cph = 1.0;
        sph = 0.0;
        const double rho = sqrt((double)(dx * dx + dy * dy));
        if (rho > 0.0) {
            cph = (double)dx / rho;
            sph = (double)dy / rho;
        }
    };
    // rotation about z by +phi (sgn = -1 on Re lanes, +1 on Im lanes) using the pair partner
    auto rotate_z = [&](T *v, double cph, double sph, T sgn) {
        double cm = 1.0, sm = 0.0;
#pragma unroll
        for (int m = 0; m < P; m++) {
            const T cz = (T)cm, sz = (T)sm * sgn;
#pragma unroll
            for (int n = m; n < P; n++) {
                const T mine = v[tri(n) + m];
                const T oth = dpp_f<DPP_XOR1>(mine);
                if (m > 0) v[tri(n) + m] = mine * cz + oth * sz;
            }
            const double c2 = cm * cph - sm * sph, s2 = sm * cph + cm * sph;
            cm = c2;
            sm = s2;
        }
    };
    // coaxial (S|R) shift by tau and the R-conversion (eq. rcr1, scaled bar form)
    auto coax = [&](T *v, T tau) {
        const T itau = (T)1 / tau;
        T pw[P + 2];
        pw[0] = (T)1;
#pragma unroll
        for (int k = 1; k <= P + 1; k++) pw[k] = pw[k - 1] * itau;
        const T wphi = pot ? (T)0 : (T)1, wchi = pot ? (T)1 : (T)0;
        const T sconv = part ? (T)1 : (T)-1;
#pragma unroll
        for (int m = 0; m < P; m++) {
            T cl[P];
#pragma unroll
            for (int n2 = m; n2 < P; n2++) cl[n2] = v[tri(n2) + m] * pw[n2];
            T out[P + 1];
#pragma unroll
            for (int n = m; n <= P; n++) {
                T a = 0;
#pragma unroll
                for (int n2 = m; n2 < P; n2++) a += (T)dfact(n + n2) * cl[n2];
                out[n] = a * pw[n + 1];
            }
#pragma unroll
            for (int n = m; n < P; n++) {
                const T other = dpp_f<DPP_XOR3>(out[n]);
                const T fphi = (n > 0) ? tau * (T)((double)m / (double)n) * sconv * wphi : (T)0;
                const T fchi = -tau * (T)(1.0 / (double)(n + 1)) * wchi;
                v[tri(n) + m] = out[n] + fphi * other + fchi * out[n + 1];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    int k = 0, r0 = 0, staged = -1;
    int d0, d1;
    int s0 = source(0, 0, d0), s1 = source(0, 1, d1);
    while (k < ncls) {
        if (k != staged) {
            __syncthreads();
            const uint4 *src4 = (const uint4 *)(wpad + (size_t)cls_theta[k] * wstride);
            uint4 *dst4 = (uint4 *)Wl;
            constexpr int N16 = (int)(4 * S::WB * sizeof(T) / 16);
#pragma unroll 8
            for (int i = tid; i < N16; i += 256) dst4[i] = src4[i];
            __syncthreads();
            staged = k;
        }
        int wfo = part * S::WB, wbo = 2 * S::WB + part * S::WB;
        asm volatile("" : "+v"(wfo), "+v"(wbo));
        const T *Wf = Wl + wfo;
        const T *Wb = Wl + wbo;
        const int dir0 = d0, dir1 = d1, src0 = s0, src1 = s1;
        // the next batch: its sources are looked up now
        int k1 = k, r1 = r0 + 2;
        if (r1 >= cst[k + 1] - cst[k]) {
            k1 = k + 1;
            r1 = 0;
        }
        s0 = source(k1, r1, d0);
        s1 = source(k1, r1 + 1, d1);

        T v0[S::NV], v1[S::NV];
        load_part(src0, v0);
        load_part(src1, v1);
        double c0, sn0, c1, sn1;
        T tau0, tau1;
        angles(dir0, c0, sn0, tau0);
        angles(dir1, c1, sn1, tau1);
        if (src0 < 0) tau0 = (T)1;
        if (src1 < 0) tau1 = (T)1;
        const T sgn_in = part ? (T)1 : (T)-1;
        rotate_z(v0, c0, sn0, sgn_in);
        rotate_z(v1, c1, sn1, sgn_in);
        rotate_y(Wf, v0, v1);
        coax(v0, tau0);
        coax(v1, tau1);
        rotate_y(Wb, v0, v1);
        // back about z (-phi) for each, then one accumulation of the sum
        {
            T *ap = acc + (size_t)slot * SST + pot * P2;
            T *spare = acc + (size_t)NSLOT * SST + pot * P2;
            const T sgn_out = part ? (T)-1 : (T)1;
            double cm0 = 1.0, sm0 = 0.0, cm1 = 1.0, sm1 = 0.0;
#pragma unroll
            for (int m = 0; m < P; m++) {
                const T cz0 = (T)cm0, sz0 = (T)sm0 * sgn_out, cz1 = (T)cm1, sz1 = (T)sm1 * sgn_out;
                {
                    const double a = cm0 * c0 - sm0 * sn0, b = sm0 * c0 + cm0 * sn0;
                    cm0 = a;
                    sm0 = b;
                    const double a1 = cm1 * c1 - sm1 * sn1, b1 = sm1 * c1 + cm1 * sn1;
                    cm1 = a1;
                    sm1 = b1;
                }
#pragma unroll
                for (int n = m; n < P; n++) {
                    const T x0 = v0[tri(n) + m], x1 = v1[tri(n) + m];
                    const T o0 = dpp_f<DPP_XOR1>(x0), o1 = dpp_f<DPP_XOR1>(x1);
                    const int off = (m == 0) ? pk_re(n, 0) : (part ? pk_im(n, m) : pk_re(n, m));
                    const T val = (m == 0) ? x0 + x1 : x0 * cz0 + o0 * sz0 + x1 * cz1 + o1 * sz1;
                    T *dst = (m == 0 && part) ? spare + off : ap + off;
                    *dst += val;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        k = k1;
        r0 = r1;
    }
    __syncthreads();
    for (int idx = tid; idx < NSLOT * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + r] = acc[sl * SST + r];
    }
}

// dense box map of one level: dmap[(z*side + y)*side + x] = global box index or -1
__global__ void k_dmap(int level, int64_t off, int64_t nb, const uint64_t *__restrict__ bkey, int32_t *__restrict__ dmap)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const uint64_t key = bkey[off + b];
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int q = 0; q < level; q++) {
        ix |= (uint32_t)((key >> (3 * q)) & 1u) << q;
        iy |= (uint32_t)((key >> (3 * q + 1)) & 1u) << q;
        iz |= (uint32_t)((key >> (3 * q + 2)) & 1u) << q;
    }
    const size_t side = (size_t)1 << level;
    const size_t sys = key >> (3 * level);
    dmap[((sys * side + iz) * side + iy) * side + ix] = (int32_t)(off + b);
}

// per-class stride (elements) of the padded rotation blocks, a multiple of 16 bytes
template <typename T, int P>
static int64_t wpad_stride()
{
    return 4 * (int64_t)M2LShape<T, P>::WB;  // a multiple of 16 bytes (padded rows)
}

// Padded rotation blocks of every polar-angle class in the tiled kernel's LDS layout:
// [kind: forward S, backward R][part: Re, Im][order n][(n+1) x (n+1)], the Im block of
// order n (n x n) embedded with a zero m = 0 row and column.
template <typename T, int P>
__global__ void k_wpad(int ntheta, const T *__restrict__ rot, T *__restrict__ wpad, int64_t stride)
{
    using S = M2LShape<T, P>;
    const int th = blockIdx.x;
    const int RS = rot_set_size(P);
    const T *Rf = rot + ((size_t)th * ROT_NKIND + ROT_S_FWD) * RS;
    const T *Rb = rot + ((size_t)th * ROT_NKIND + ROT_R_BACK) * RS;
    for (int idx = threadIdx.x; idx < stride; idx += blockDim.x) {
        T val = (T)0;
        if (idx < 4 * S::WB) {
            const int kind = idx / (2 * S::WB), rem = idx % (2 * S::WB);
            const int pt = rem / S::WB, j = rem % S::WB;
            int n = 0;
            while (wrow_off<T>(n + 1) <= j) n++;
            const int jj = j - wrow_off<T>(n), mp = jj / rowlen<T>(n), m = jj % rowlen<T>(n);
            const T *blk = (kind ? Rb : Rf) + rot_block_off(n);
            if (m <= n) {
                if (pt == 0) val = blk[mp * (n + 1) + m];
                else if (mp > 0 && m > 0) val = blk[(n + 1) * (n + 1) + (mp - 1) * n + (m - 1)];
            }
        }
        wpad[(size_t)th * stride + idx] = val;
    }
}

template <typename T, int P>
static size_t wpad_build_t(lhf_plan *Pl, hipStream_t st)
{
    const int64_t stride = wpad_stride<T, P>();
    if (dev_malloc(&Pl->wpad, sizeof(T) * stride * Pl->n_theta) != hipSuccess) return 0;
    k_wpad<T, P><<<dim3((unsigned)Pl->n_theta), dim3(256), 0, st>>>(Pl->n_theta, (const T *)Pl->rot, (T *)Pl->wpad,
                                                                     stride);
    return (size_t)stride;
}

// LDS footprint of a tile addressing NPAR sibling groups of which NREAL hold accumulators
// (OWN: no entry list in LDS)
template <typename T, int P>
constexpr size_t tile_bytes(int npar, bool own, int nreal)
{
    return sizeof(T) * ((size_t)(8 * nreal + 1) * (2 * P * P + 1) + 4 * M2LShape<T, P>::WB) +
           sizeof(int) * 3 * 8 * npar + sizeof(int16_t) * (64 + (own ? 0 : 1512));
}
// LDS of one workgroup on gfx950 (160 KB per compute unit, all of it addressable by one group)
constexpr size_t LDS_MAX = 163840;
// Budget used to choose the tile: 64 KB.  Ownership mode with fewer real sibling groups in
// up to 160 KB (FP64 p = 12: 7 of 8) measured no faster than the shared mode (112 vs 108 ms
// per execute on the 2^20 cube), so the choice stays within 64 KB and leaves room for two
// workgroups per compute unit.
constexpr size_t LDS_TILE = 65536;
// ownership mode (no atomics): the eight sibling groups the wavefronts own, if they fit;
// otherwise shared mode with 4 or 2 sibling groups
template <typename T, int P>
constexpr int tile_nreal_own()
{
    return tile_bytes<T, P>(8, true, 8) <= LDS_TILE ? 8 : 0;
}
template <typename T, int P>
constexpr bool tile_own()
{
    return tile_nreal_own<T, P>() > 0;
}
template <typename T, int P>
constexpr int tile_npar()
{
    return tile_own<T, P>() ? 8 : (tile_bytes<T, P>(4, false, 4) <= LDS_TILE ? 4 : 2);
}
template <typename T, int P>
constexpr int tile_nreal()
{
    return tile_own<T, P>() ? tile_nreal_own<T, P>() : tile_npar<T, P>();
}

template <typename T, int P>
static size_t m2l_tile_shmem()
{
    return tile_bytes<T, P>(tile_npar<T, P>(), tile_own<T, P>(), tile_nreal<T, P>());
}

// allow the tile's dynamic LDS beyond the default 64 KB
template <typename T, int P>
static bool tile_attr_t()
{
    constexpr int NPAR = tile_npar<T, P>();
    constexpr bool OWN = tile_own<T, P>();
    constexpr int NREAL = tile_nreal<T, P>();
    static_assert(tile_bytes<T, P>(NPAR, OWN, NREAL) <= LDS_MAX, "tile exceeds the LDS");
    return hipFuncSetAttribute((const void *)k_m2l_tile<T, P, NPAR, OWN, NREAL>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)m2l_tile_shmem<T, P>()) == hipSuccess;
}

template <typename T, int P>
static void launch_tile(const lhf_plan *Pl, int level, hipStream_t st)
{
    constexpr int NPAR = tile_npar<T, P>();
    constexpr bool OWN = tile_own<T, P>();
    constexpr int NREAL = tile_nreal<T, P>();
    const int64_t poff = Pl->lev[level - 1].off, npar = Pl->lev[level - 1].nb;
    const int64_t ntiles = (npar + NREAL - 1) / NREAL;
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls, Pl->sched_row_start, Pl->sched_rows};
    const size_t shm = m2l_tile_shmem<T, P>();
    k_m2l_tile<T, P, NPAR, OWN, NREAL><<<dim3((unsigned)(per * 8)), dim3(256), shm, st>>>(
        level, poff, npar, Pl->lev[level].off, Pl->lev[level].nb, Pl->bkey, Pl->bchild0, Pl->bnchild,
        Pl->dmap[level], (const T *)Pl->M, (T *)Pl->Lc, (const T *)Pl->wpad, wpad_stride<T, P>(), sch,
        Pl->sched_cls_theta);
}

// two rows per batch (ownership-mode orders only)
template <typename T, int P>
static void launch_tile2(const lhf_plan *Pl, int level, hipStream_t st)
{
    static_assert(tile_own<T, P>(), "two-row tiles need the ownership mode");
    const int64_t poff = Pl->lev[level - 1].off, npar = Pl->lev[level - 1].nb;
    const int64_t ntiles = (npar + 7) / 8;
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls, Pl->sched_row_start, Pl->sched_rows};
    const size_t shm = m2l_tile_shmem<T, P>();
    k_m2l_tile2<T, P><<<dim3((unsigned)(per * 8)), dim3(256), shm, st>>>(
        level, poff, npar, Pl->bkey, Pl->bchild0, Pl->bnchild, Pl->dmap[level], (const T *)Pl->M, (T *)Pl->Lc,
        (const T *)Pl->wpad, wpad_stride<T, P>(), sch, Pl->sched_cls_theta);
}

// true if the tiled kernel handles this (precision, p)
bool m2l_tile_supported(int precision, int p)
{
    // LDS per workgroup must stay within 64 KB: FP64 p = 16 would need 113 KB
    if (precision == LHF_FP64) return p == 4 || p == 6 || p == 8 || p == 10 || p == 12;
    return p == 4 || p == 6 || p == 8 || p == 10 || p == 12 || p == 16;
}

// true if the tiled kernel runs in ownership mode (no atomics: a fixed summation order) for
// this (precision, p)
bool m2l_tile_owned(int precision, int p)
{
    if (precision == LHF_FP64) {
        switch (p) {
        case 4: return tile_own<double, 4>();
        case 6: return tile_own<double, 6>();
        case 8: return tile_own<double, 8>();
        case 10: return tile_own<double, 10>();
        case 12: return tile_own<double, 12>();
        default: return false;
        }
    }
    switch (p) {
    case 4: return tile_own<float, 4>();
    case 6: return tile_own<float, 6>();
    case 8: return tile_own<float, 8>();
    case 10: return tile_own<float, 10>();
    case 12: return tile_own<float, 12>();
    case 16: return tile_own<float, 16>();
    default: return false;
    }
}

void m2l_tile_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int p = Pl->p;
    if (Pl->precision == LHF_FP64) {
        switch (p) {
        case 4: launch_tile<double, 4>(Pl, level, st); break;
        case 6: launch_tile<double, 6>(Pl, level, st); break;
        case 8: launch_tile<double, 8>(Pl, level, st); break;
        case 10: launch_tile<double, 10>(Pl, level, st); break;
        case 12: launch_tile<double, 12>(Pl, level, st); break;
        }
    } else {
        switch (p) {
        case 4: launch_tile<float, 4>(Pl, level, st); break;
        case 6: launch_tile<float, 6>(Pl, level, st); break;
        case 8:
            if (Pl->tile2) launch_tile2<float, 8>(Pl, level, st);
            else launch_tile<float, 8>(Pl, level, st);
            break;
        case 10:
            if (Pl->tile2) launch_tile2<float, 10>(Pl, level, st);
            else launch_tile<float, 10>(Pl, level, st);
            break;
        case 12: launch_tile<float, 12>(Pl, level, st); break;
        case 16: launch_tile<float, 16>(Pl, level, st); break;
        }
    }
}

bool wpad_build(lhf_plan *Pl, hipStream_t st)
{
    size_t r = 0;
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 4: r = wpad_build_t<double, 4>(Pl, st) && tile_attr_t<double, 4>(); break;
        case 6: r = wpad_build_t<double, 6>(Pl, st) && tile_attr_t<double, 6>(); break;
        case 8: r = wpad_build_t<double, 8>(Pl, st) && tile_attr_t<double, 8>(); break;
        case 10: r = wpad_build_t<double, 10>(Pl, st) && tile_attr_t<double, 10>(); break;
        case 12: r = wpad_build_t<double, 12>(Pl, st) && tile_attr_t<double, 12>(); break;
        }
    } else {
        switch (Pl->p) {
        case 4: r = wpad_build_t<float, 4>(Pl, st) && tile_attr_t<float, 4>(); break;
        case 6: r = wpad_build_t<float, 6>(Pl, st) && tile_attr_t<float, 6>(); break;
        case 8: r = wpad_build_t<float, 8>(Pl, st) && tile_attr_t<float, 8>(); break;
        case 10: r = wpad_build_t<float, 10>(Pl, st) && tile_attr_t<float, 10>(); break;
        case 12: r = wpad_build_t<float, 12>(Pl, st) && tile_attr_t<float, 12>(); break;
        case 16: r = wpad_build_t<float, 16>(Pl, st) && tile_attr_t<float, 16>(); break;
        }
    }
    return r != 0;
}

void dmap_build(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t nb = Pl->lev[level].nb;
    if (nb == 0) return;  // an adaptive tree may leave deep levels empty
    hipLaunchKernelGGL(k_dmap, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, level, Pl->lev[level].off, nb,
                       Pl->bkey, Pl->dmap[level]);
}

}  // namespace lhf

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

namespace lhf {

template <int P>
struct M2LShape {
    static constexpr int NV = P * (P + 1) / 2;        // (n, m <= n), n < P
    static constexpr int NVX = NV + P + 1;            // + order P (chi extra row), m <= P
    static constexpr int WB = P * (P + 1) * (2 * P + 1) / 6;  // sum_{n<P} (n+1)^2
};

__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }
__host__ __device__ constexpr int woff(int n) { return n * (n + 1) * (2 * n + 1) / 6; }

template <typename T>
__device__ inline T shfl_xor_t(T v, int mask)
{
    return __shfl_xor(v, mask, 64);
}

// factorials as constants
__device__ constexpr double dfact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= (double)i;
    return f;
}

struct M2LSched {
    // static schedule of one sibling group, sorted by polar-angle class
    const int16_t *cls_start;  // [ncls+1]
    const int16_t *ent_c;      // [1512] child position of the target
    const int16_t *ent_dir;    // [1512] direction code of t = c_T - c_S
    int ncls;
};

template <typename T, int P>
__global__ void __launch_bounds__(256) k_m2l_tile(int level, int64_t poff, int64_t npar, int64_t loff, int64_t nbl,
                                                  const uint64_t *__restrict__ bkey, const int32_t *__restrict__ bchild0,
                                                  const int32_t *__restrict__ bnchild, const int32_t *__restrict__ dmap,
                                                  const T *__restrict__ M, T *__restrict__ Lc,
                                                  const T *__restrict__ rot, const T *__restrict__ zph,
                                                  M2LSched sch, const int16_t *__restrict__ cls_theta)
{
    using S = M2LShape<P>;
    constexpr int P2 = P * P;
    extern __shared__ char smem[];
    T *acc = (T *)smem;                       // [16][2][P2]
    T *Wl = acc + 16 * 2 * P2;                // [2 kinds: fwd S, back R][2 parts][WB]
    int *slot_box = (int *)(Wl + 4 * S::WB);  // [16] target box per slot (-1: none)

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // XCD-aware tile order: consecutive tiles stay on one XCD (shared L2)
    const int64_t ntiles = (npar + 1) / 2;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;

    // slots: parent i (0,1) x child position c (0..7)
    if (tid < 16) {
        const int i = tid >> 3, c = tid & 7;
        int box = -1;
        const int64_t q = 2 * tile + i;
        if (q < npar) {
            const int64_t pb = poff + q;
            const int c0 = bchild0[pb], nc = bnchild[pb];
            for (int k = 0; k < nc; k++)
                if ((int)(bkey[c0 + k] & 7u) == c) box = c0 + k;
        }
        slot_box[tid] = box;
    }
    __syncthreads();
    for (int idx = tid; idx < 16 * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        acc[idx] = box >= 0 ? Lc[(size_t)box * 2 * P2 + r] : (T)0;
    }

    const int RS = rot_set_size(P);
    const int side = 1 << level;
    const int t = lane >> 2, pot = (lane >> 1) & 1, part = lane & 1;

    for (int k = 0; k < sch.ncls; k++) {
        const int e0 = sch.cls_start[k], cnt = sch.cls_start[k + 1] - e0;
        __syncthreads();  // previous class finished with Wl
        {
            // stage the class's rotation blocks; Im blocks padded to (n+1)^2 with a zero m=0 row/col
            const int th = cls_theta[k];
            const T *Rf = rot + ((size_t)th * ROT_NKIND + ROT_S_FWD) * RS;
            const T *Rb = rot + ((size_t)th * ROT_NKIND + ROT_R_BACK) * RS;
            for (int idx = tid; idx < 4 * S::WB; idx += 256) {
                const int kind = idx / (2 * S::WB), rem = idx % (2 * S::WB);
                const int pt = rem / S::WB, j = rem % S::WB;
                int n = 0;
                while (woff(n + 1) <= j) n++;
                const int jj = j - woff(n), mp = jj / (n + 1), m = jj % (n + 1);
                const T *R = kind ? Rb : Rf;
                const T *blk = R + rot_block_off(n);
                T val;
                if (pt == 0) val = blk[mp * (n + 1) + m];
                else val = (mp == 0 || m == 0) ? (T)0 : blk[(n + 1) * (n + 1) + (mp - 1) * n + (m - 1)];
                Wl[idx] = val;
            }
        }
        __syncthreads();
        const int ntr = 2 * cnt;
        for (int r0 = 0; r0 < ntr; r0 += 64) {
            // opaque per-batch offsets keep the compiler from hoisting every matrix entry
            // of the class out of the batch loop (which would exhaust the register file)
            int wfo = part * S::WB, wbo = 2 * S::WB + part * S::WB;
            asm volatile("" : "+v"(wfo), "+v"(wbo));
            const T *Wf = Wl + wfo;
            const T *Wb = Wl + wbo;
            const int tr = r0 + wave * 16 + t;
            bool act = tr < ntr;
            int slot = 0, src = -1, dir = 0;
            if (act) {
                const int par = tr / cnt, e = e0 + tr % cnt;
                const int c = sch.ent_c[e];
                dir = sch.ent_dir[e];
                slot = par * 8 + c;
                const int tb = slot_box[slot];
                if (tb < 0) {
                    act = false;
                } else {
                    const uint64_t key = bkey[tb];
                    uint32_t ix = 0, iy = 0, iz = 0;
                    for (int b = 0; b < level; b++) {
                        ix |= (uint32_t)((key >> (3 * b)) & 1u) << b;
                        iy |= (uint32_t)((key >> (3 * b + 1)) & 1u) << b;
                        iz |= (uint32_t)((key >> (3 * b + 2)) & 1u) << b;
                    }
                    const int sx = (int)ix - (dir % 7 - 3), sy = (int)iy - ((dir / 7) % 7 - 3),
                              sz = (int)iz - (dir / 49 - 3);
                    if (sx < 0 || sy < 0 || sz < 0 || sx >= side || sy >= side || sz >= side) {
                        act = false;
                    } else {
                        src = dmap[((size_t)sz * side + sy) * side + sx];
                        if (src < 0) act = false;
                    }
                }
            }
            const int dx = dir % 7 - 3, dy = (dir / 7) % 7 - 3, dz = dir / 49 - 3;
            const T tau = (T)sqrt((double)(dx * dx + dy * dy + dz * dz));
            const T *zp = zph + (size_t)dir * 2 * P;
            T v[S::NV];
            // 1. load the source part and rotate about z by +phi
            {
                const T *sp = M + (size_t)(act ? src : 0) * 2 * P2 + pot * P2;
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const T cz = zp[m], sz = zp[P + m];
#pragma unroll
                    for (int n = m; n < P; n++) {
                        T re = sp[pk_re(n, m)];
                        T im = (m > 0) ? sp[pk_im(n, m)] : (T)0;
                        T val;
                        if (m == 0) val = part ? (T)0 : re;
                        else val = part ? (re * sz + im * cz) : (re * cz - im * sz);
                        v[tri(n) + m] = val;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // 2. rotation about y (forward, S basis), one output row at a time
#pragma unroll
            for (int n = 0; n < P; n++) {
                T in[P];
#pragma unroll
                for (int m = 0; m <= n; m++) in[m] = v[tri(n) + m];
                const T *W = Wf + woff(n);
#pragma unroll
                for (int mp = 0; mp <= n; mp++) {
                    T a = 0;
#pragma unroll
                    for (int m = 0; m <= n; m++) a += W[mp * (n + 1) + m] * in[m];
                    asm volatile("" : "+v"(a));  // finish this row here: bounds the live matrix entries
                    v[tri(n) + mp] = a;
                }
            }
            // 3+4. per column m: coaxial (S|R) shift out_n = tau^-(n+1) sum_n' (n+n')! tau^-n' in_n'
            //      (chi to order P), then the R-conversion (eq. rcr1, scaled)
            //        phi~ = phi + i tau m/n chi ,  chi~_n = chi_n - tau/(n+1) chi_{n+1}
            {
                const T itau = (T)1 / tau;
#pragma unroll
                for (int m = 0; m < P; m++) {
                    T col[P];
                    T pwn = (T)1;
#pragma unroll
                    for (int k = 0; k < m; k++) pwn *= itau;
#pragma unroll
                    for (int n2 = m; n2 < P; n2++) {
                        col[n2] = v[tri(n2) + m] * pwn;
                        pwn *= itau;
                    }
                    T out[P + 1];
                    T pwo = itau;
#pragma unroll
                    for (int k = 0; k < m; k++) pwo *= itau;
#pragma unroll
                    for (int n = m; n <= P; n++) {
                        T a = 0;
#pragma unroll
                        for (int n2 = m; n2 < P; n2++) a += (T)dfact(n + n2) * col[n2];
                        out[n] = a * pwo;
                        pwo *= itau;
                    }
#pragma unroll
                    for (int n = m; n < P; n++) {
                        const T other = shfl_xor_t(out[n], 3);  // phi-Re <-> chi-Im, phi-Im <-> chi-Re
                        T r;
                        if (pot == 0) {
                            const T f = (n > 0) ? tau * (T)((double)m / (double)n) : (T)0;
                            r = out[n] + (part ? f * other : -f * other);
                        } else {
                            r = out[n] - tau * (T)(1.0 / (double)(n + 1)) * out[n + 1];
                        }
                        v[tri(n) + m] = r;
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
                const T *W = Wb + woff(n);
#pragma unroll
                for (int mp = 0; mp <= n; mp++) {
                    T a = 0;
#pragma unroll
                    for (int m = 0; m <= n; m++) a += W[mp * (n + 1) + m] * in[m];
                    asm volatile("" : "+v"(a));  // finish this row here: bounds the live matrix entries
                    v[tri(n) + mp] = a;
                }
            }
            // 6. back-rotation about z (-phi) and accumulation into the target slot
            {
                T *ap = acc + (size_t)slot * 2 * P2 + pot * P2;
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const T cz = zp[m], sz = zp[P + m];
#pragma unroll
                    for (int n = m; n < P; n++) {
                        const T mine = v[tri(n) + m];
                        const T oth = shfl_xor_t(mine, 1);
                        if (act) {
                            if (m == 0) {
                                if (!part) atomicAdd(&ap[pk_re(n, 0)], mine);
                            } else {
                                const T re = part ? oth : mine, im = part ? mine : oth;
                                if (!part) atomicAdd(&ap[pk_re(n, m)], re * cz + im * sz);
                                else atomicAdd(&ap[pk_im(n, m)], -re * sz + im * cz);
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < 16 * 2 * P2; idx += 256) {
        const int sl = idx / (2 * P2), r = idx % (2 * P2);
        const int box = slot_box[sl];
        if (box >= 0) Lc[(size_t)box * 2 * P2 + r] = acc[idx];
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
    dmap[((size_t)iz * side + iy) * side + ix] = (int32_t)(off + b);
}

template <typename T, int P>
static size_t m2l_tile_shmem()
{
    using S = M2LShape<P>;
    return sizeof(T) * (16 * 2 * P * P + 4 * S::WB) + sizeof(int) * 16;
}

template <typename T, int P>
static void launch_tile(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t poff = Pl->lev[level - 1].off, npar = Pl->lev[level - 1].nb;
    const int64_t ntiles = (npar + 1) / 2;
    const int64_t per = (ntiles + 7) / 8;
    M2LSched sch{Pl->sched_cls_start, Pl->sched_c, Pl->sched_dir, Pl->sched_ncls};
    const size_t shm = m2l_tile_shmem<T, P>();
    k_m2l_tile<T, P><<<dim3((unsigned)(per * 8)), dim3(256), shm, st>>>(
        level, poff, npar, Pl->lev[level].off, Pl->lev[level].nb, Pl->bkey, Pl->bchild0, Pl->bnchild,
        Pl->dmap[level], (const T *)Pl->M, (T *)Pl->Lc, (const T *)Pl->rot, (const T *)Pl->zph, sch,
        Pl->sched_cls_theta);
}

// true if the tiled kernel handles this (precision, p)
bool m2l_tile_supported(int precision, int p)
{
    // LDS per workgroup must stay within 64 KB: FP64 p = 16 would need 113 KB
    if (precision == LHF_FP64) return p == 4 || p == 6 || p == 8 || p == 10 || p == 12;
    return p == 4 || p == 6 || p == 8 || p == 10 || p == 12 || p == 16;
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
        case 8: launch_tile<float, 8>(Pl, level, st); break;
        case 10: launch_tile<float, 10>(Pl, level, st); break;
        case 12: launch_tile<float, 12>(Pl, level, st); break;
        case 16: launch_tile<float, 16>(Pl, level, st); break;
        }
    }
}

void dmap_build(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t nb = Pl->lev[level].nb;
    hipLaunchKernelGGL(k_dmap, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, level, Pl->lev[level].off, nb,
                       Pl->bkey, Pl->dmap[level]);
}

}  // namespace lhf

// lhf_m2l_mfma.hip -- batched multipole-to-local translation on the matrix cores.
//
// The same translation as the VALU tile kernel (rotation about z, rotation about y
// in the S basis, coaxial (S|R) shift with the R-conversion of eq. rcr1, rotation
// back about y in the R basis and about z; Sec. 4.4), organised as dense small-matrix
// products over a batch of translations so that the three matrix stages run as
// 16x16x4 MFMA chains:
//   * a batch = the 8 translations of one row of the class schedule for one parent
//     box (one per child position, so 8 distinct targets), both potentials:
//     16 columns (translation t, potential) of one MFMA;
//   * per wavefront, the batch's coefficients live in LDS as X[part][(n,m)][16]
//     (part = Re or Im of the scaled bar coefficients, (n,m) in triangular order);
//     every stage reads its B operand from there and writes its D result back;
//   * y rotations: per order n, Y_n = W_n X_n with the class's rotation block as the
//     A operand (the forward and back blocks of the class are staged in LDS once per
//     class and shared by the workgroup's four wavefronts);
//   * coaxial shift, per column m: out_n = tau^-(n+1) sum_n' (n+n')! tau^-n' in_n' --
//     the constant factorial (Hankel) matrix is the A operand, the per-translation
//     tau powers scale the B operand on the way in and D on the way out;
//   * the R-conversion couples phi with chi of the other part (the partner column,
//     8 columns away) and chi_n with chi_{n+1} (the next output row): the coaxial
//     outputs of one column m go through a small per-wavefront LDS buffer, from which
//     each lane reads the partner values it needs;
//   * z rotations are element-wise and fused into the gather of the sources and the
//     accumulation into the targets.
// A workgroup owns 4 parent boxes, one per wavefront.  Every batch of a wavefront hits the
// same 8 targets (the children of its parent), so the local expansions accumulate in
// registers: lane (g, column) owns the packed entries g, g+4, .. of its column's target
// and potential, from the L2L value loaded at the start to the store at the end.  The
// job (source box) of the next batch is looked up while the current one computes.
#include <hip/hip_runtime.h>

#include "lhf_internal.h"

namespace lhf {

namespace mf {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// 16x16x4 products: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// four D entries of column l % 16: rows 4 (l/16) + r for FP32 (blocked), rows 4 r + l/16 for
// FP64 (interleaved) -- measured lane layouts of the two instructions.
template <typename T>
struct Acc4;
template <>
struct Acc4<float> {
    using type = v4f;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ type mma(float a, float b, type c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Acc4<double> {
    using type = v4d;
    static __device__ __forceinline__ int row(int g, int r) { return 4 * r + g; }
    static __device__ __forceinline__ type mma(double a, double b, type c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }
__host__ __device__ constexpr int nch(int k) { return (k + 3) / 4; }

// A-operand slots of one rotation kind: Re blocks (K = n+1) then Im blocks (K = n)
template <int P>
__host__ __device__ constexpr int rot_slots()
{
    int s = 0;
    for (int n = 0; n < P; n++) s += nch(n + 1) + nch(n);
    return s;
}
template <int P>
__host__ __device__ constexpr int slot_off(int part, int n)
{
    int s = 0;
    if (part == 1)
        for (int k = 0; k < P; k++) s += nch(k + 1);
    for (int k = 0; k < n; k++) s += part ? nch(k) : nch(k + 1);
    return s;
}

}  // namespace mf

namespace mf {

// LDS layout of a workgroup (T elements first, then 32-bit words)
template <typename T, int P>
struct Lds {
    static constexpr int NV = tri(P), NVI = tri(P - 1), NX = NV + NVI;  // NX = P^2
    static constexpr int RS = P * (2 * P * P + 1) / 3;
    static constexpr int XW = (NX + 1) * 16;      // X rows + one dummy row (masked writes)
    static constexpr int ZW = 2 * 32 * 16;        // coaxial outputs of one column m, both parts
    static constexpr int CS = 8 * 2 * P, PW = 8 * (P + 2);
    // per wavefront
    static constexpr int WAVE_T = XW + ZW + CS + PW + 8;
    // shared
    static constexpr int SHARED_T = 2 * RS + (2 * P + 2) + (P + 2);
    static constexpr int NA = P * P / 4;
    static constexpr size_t bytes()
    {
        return sizeof(T) * (size_t)(4 * WAVE_T + SHARED_T) + sizeof(int) * (3 * 32 + 4 * 16 + NA * 64) +
               sizeof(int16_t) * 64;
    }
};

}  // namespace mf

// LDS-staged formulation: per wavefront the batch's coefficients live in LDS as
// X[row][16 columns] (Re rows (n, m <= n), then Im rows (n, 1 <= m <= n)); each stage reads
// its B operand from there and writes its D result back.
template <typename T, int P>
__global__ void __launch_bounds__(256) k_m2l_mfma(int level, int64_t poff, int64_t npar, const uint64_t *__restrict__ bkey,
                                                  const int32_t *__restrict__ bchild0, const int32_t *__restrict__ bnchild,
                                                  const int32_t *__restrict__ dmap, const T *__restrict__ M,
                                                  T *__restrict__ Lc, const T *__restrict__ rot,
                                                  const int16_t *__restrict__ row_start, const int16_t *__restrict__ rows,
                                                  int ncls, const int16_t *__restrict__ cls_theta)
{
    using namespace mf;
    using L = Lds<T, P>;
    using V4 = typename Acc4<T>::type;
    constexpr int P2 = P * P;
    constexpr int NV = L::NV;
    constexpr int RS = L::RS;
    constexpr int NA = L::NA;
    static_assert(P2 % 4 == 0, "even truncation numbers only");
    extern __shared__ char smem_raw[];
    T *wall = (T *)smem_raw;                       // [4][WAVE_T]
    T *Wl = wall + 4 * L::WAVE_T;                  // [2][RS] forward (S basis), back (R basis)
    T *fct = Wl + 2 * RS;                          // [2P+2] k!
    T *rcp = fct + 2 * P + 2;                      // [P+2] 1/k
    int *slot_xyz = (int *)(rcp + P + 2);          // [32]
    int *slot_box = slot_xyz + 32;
    int *slot_sys = slot_box + 32;
    int *jall = slot_sys + 32;                     // [4][16]: src[8], slot[8]
    int *etab = jall + 64;                         // [NA][64] per-lane entry table
    int16_t *cst = (int16_t *)(etab + NA * 64);    // [ncls + 1] <= 64

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ntiles = (npar + 3) / 4;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;

    // target slots: parent i (0..3, = wavefront) x child position c (0..7)
    if (tid < 32) {
        const int i = tid >> 3, c = tid & 7;
        int box = -1, xyz = -1, sys = 0;
        const int64_t q = 4 * tile + i;
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
    for (int i = tid; i <= ncls; i += 256) cst[i] = row_start[i];
    if (tid < 2 * P + 2) {
        double f = 1.0;
        for (int k = 2; k <= tid; k++) f *= (double)k;
        fct[tid] = (T)f;
    }
    if (tid < P + 2) rcp[tid] = tid ? (T)(1.0 / (double)tid) : (T)0;
    // entry table of lane (g, column): packed entry u = g + 4 i ->
    //   bits 0..8 X row of the entry, 9..17 X row of the other part of the same (n, m)
    //   (the entry's own row when m = 0), 18..26 packed offset of that other part, 27..31 m
    for (int idx = tid; idx < NA * 64; idx += 256) {
        const int i = idx / 64, g = (idx % 64) >> 4;
        const int u = g + 4 * i;
        int n = 0;
        while ((n + 1) * (n + 1) <= u) n++;
        const int r = u - n * n, part = r > n, m = part ? r - n : r;
        const int xrow = part ? NV + tri(n - 1) + m - 1 : tri(n) + m;
        int prow = xrow, pu = u;
        if (m > 0) {
            prow = part ? tri(n) + m : NV + tri(n - 1) + m - 1;
            pu = part ? n * n + m : n * n + n + m;
        }
        etab[idx] = xrow | (prow << 9) | (pu << 18) | (m << 27);
    }
    __syncthreads();

    T *wbase = wall + (size_t)wave * L::WAVE_T;
    T *X = wbase;                                  // rows: Re (n, m <= n), Im (n, 1 <= m <= n), dummy
    T *Z = X + L::XW;                              // [2][32][16]
    T *cs = Z + L::ZW;                             // [8][P][2] cos, sin of m phi
    T *pw = cs + L::CS;                            // [8][P+2] tau^-k
    T *jtau = pw + L::PW;                          // [8]
    int *jsrc = jall + wave * 16, *jslot = jsrc + 8;
    const int side = 1 << level;
    const int sbase = wave * 8;

    // this lane's accumulators: packed entries g + 4 i of (target col & 7, potential col >> 3)
    T accr[NA];
    {
        const int col = lane & 15, g = lane >> 4;
        const int box = slot_box[sbase + (col & 7)];
        const T *lp = Lc + (size_t)(box >= 0 ? box : 0) * 2 * P2 + (col >> 3) * P2;
#pragma unroll
        for (int i = 0; i < NA; i++) accr[i] = box >= 0 ? lp[g + 4 * i] : (T)0;
    }

    // job of one row for lanes 0..7 (child position c = lane): direction code and source box
    auto job = [&](int R, int &dir, int &src) {
        dir = -1;
        src = -1;
        if (lane < 8 && R < cst[ncls]) {
            const int slot = sbase + lane;
            dir = rows[(size_t)R * 8 + lane];
            const int xyz = slot_xyz[slot];
            if (dir >= 0 && xyz >= 0) {
                const int sx = (xyz & 1023) - (dir % 7 - 3), sy = ((xyz >> 10) & 1023) - ((dir / 7) % 7 - 3),
                          sz = (xyz >> 20) - (dir / 49 - 3);
                if (sx >= 0 && sy >= 0 && sz >= 0 && sx < side && sy < side && sz < side)
                    src = dmap[(((size_t)slot_sys[slot] * side + sz) * side + sy) * side + sx];
            }
        }
    };
    // only the compiler is held back here: LDS operations of one wavefront execute in order
    auto wsync = [&]() {
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
    };

    const int NR = cst[ncls];
    int cur_dir, cur_src;
    job(0, cur_dir, cur_src);
    int k = -1;
    for (int R = 0; R < NR; R++) {
        // a new class: stage its forward and back rotation blocks (all wavefronts take part)
        if (k < 0 || R >= cst[k + 1]) {
            while (R >= cst[k + 1]) k++;
            __syncthreads();
            const T *rf = rot + (size_t)cls_theta[k] * ROT_NKIND * RS;
            for (int i = tid; i < RS; i += 256) {
                Wl[i] = rf[ROT_S_FWD * RS + i];
                Wl[RS + i] = rf[ROT_R_BACK * RS + i];
            }
            __syncthreads();
        }
        // this batch's jobs, and the next batch's lookup issued now
        const int dir = cur_dir, srcj = cur_src;
        job(R + 1, cur_dir, cur_src);
        const int active = srcj >= 0;
        if (lane < 8) {
            jsrc[lane] = srcj;
            jslot[lane] = sbase + lane;
            if (active) {
                const int dx = dir % 7 - 3, dy = (dir / 7) % 7 - 3, dz = dir / 49 - 3;
                const double tau = sqrt((double)(dx * dx + dy * dy + dz * dz));
                const double rho = sqrt((double)(dx * dx + dy * dy));
                const double cph = rho > 0.0 ? (double)dx / rho : 1.0, sph = rho > 0.0 ? (double)dy / rho : 0.0;
                double cm = 1.0, sm = 0.0;
                for (int m = 0; m < P; m++) {
                    cs[(lane * P + m) * 2] = (T)cm;
                    cs[(lane * P + m) * 2 + 1] = (T)sm;
                    const double c2 = cm * cph - sm * sph, s2 = sm * cph + cm * sph;
                    cm = c2;
                    sm = s2;
                }
                const double it = 1.0 / tau;
                double pk = 1.0;
                for (int kk = 0; kk < P + 2; kk++) {
                    pw[lane * (P + 2) + kk] = (T)pk;
                    pk *= it;
                }
                jtau[lane] = (T)tau;
            }
        }
        const unsigned long long anyact = __ballot(active);
        wsync();
        if (anyact == 0ull) continue;  // wave-uniform: every child of this row is a hole

        // lane roles, laundered per batch: every per-lane index and address below is
        // recomputed here instead of being hoisted out of the loop (register file)
        int lid = lane;
        asm volatile("" : "+v"(lid));
        const int col = lid & 15, g = lid >> 4, t = col & 7, pot = col >> 3;
        const int ai = lid & 15, akq = lid >> 4;   // A-operand coordinates (row, k)
        const int src = jsrc[t];
        const bool act = src >= 0;
        const T tau = jtau[t];
        const T *cst_t = cs + t * 2 * P;
        const T *pw_t = pw + t * (P + 2);
        // ---- gather the sources, rotated about z by +phi, into X (lane: packed entries g + 4i)
        {
            const T *sp = M + (size_t)(act ? src : 0) * 2 * P2 + pot * P2;
#pragma unroll
            for (int i = 0; i < NA; i++) {
                const int e = etab[i * 64 + lid];
                const int xrow = e & 511, pu = (e >> 18) & 511, m = (e >> 27) & 31;
                const int u = g + 4 * i;
                const T own = sp[u], oth = sp[pu];
                const T c = cst_t[2 * m], s = cst_t[2 * m + 1];
                // Re: re c - im s;  Im: im c + re s
                const T sg = xrow >= NV ? (T)1 : (T)-1;
                X[xrow * 16 + col] = act ? own * c + sg * oth * s : (T)0;
            }
        }
        wsync();
        // A operand of a rotation block: lane (i, kq) holds W[row][col] of order n, chunk c
        auto wa = [&](int kind, int part, int n, int c) -> T {
            const int mp = ai + part, m = 4 * c + akq + part;
            const bool ok = mp <= n && m <= n;
            const int off = part ? (n + 1) * (n + 1) + (mp - 1) * n + (m - 1) : mp * (n + 1) + m;
            const T w = Wl[kind * RS + rot_block_off(n) + (ok ? off : 0)];
            return ok ? w : (T)0;
        };
        auto rotate = [&](int kind) {
#pragma unroll
            for (int part = 0; part < 2; part++) {
#pragma unroll
                for (int n = 0; n < P; n++) {
                    const int K = part ? n : n + 1;
                    if (K == 0) continue;
                    const int base = part ? NV + tri(n - 1) : tri(n);
                    V4 d = {0, 0, 0, 0};
#pragma unroll
                    for (int c = 0; c < nch(K); c++) {
                        const int kk = 4 * c + g;
                        const T b = X[(base + (kk < K ? kk : 0)) * 16 + col];
                        d = Acc4<T>::mma(wa(kind, part, n, c), kk < K ? b : (T)0, d);
                    }
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) {
                        const int i = Acc4<T>::row(g, rr);
                        X[(i < K ? base + i : L::NX) * 16 + col] = d[rr];
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        };
        // ---- rotation about y, forward (S basis): Y_n = W_n X_n per part and order
        rotate(0);
        wsync();
        // ---- coaxial shift, per column m: raw outputs tau^-(n+1) sum_n' (n+n')! tau^-n' in_n'
        //      (rows n = m..P) into Z, then the R-conversion (eq. rcr1, scaled bar form)
        //        phi~_n = phi_n + i tau m/n chi_n ,   chi~_n = chi_n - tau/(n+1) chi_{n+1}
        //      back into X
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int K = P - m, nrow = P + 1 - m;
#pragma unroll
            for (int part = 0; part < 2; part++) {
                if (part == 1 && m == 0) continue;
#pragma unroll
                for (int rb = 0; rb < 2; rb++) {
                    if (16 * rb >= nrow) continue;
                    V4 d = {0, 0, 0, 0};
#pragma unroll
                    for (int c = 0; c < nch(K); c++) {
                        const int np = m + 4 * c + g;  // input order n'
                        const bool okb = np < P;
                        const int npc = okb ? np : m;
                        const int row = part ? NV + tri(npc - 1) + m - 1 : tri(npc) + m;
                        const T b = X[row * 16 + col] * pw_t[npc];
                        const bool oka = (16 * rb + ai < nrow) && (4 * c + akq < K);
                        const T a = fct[oka ? 2 * m + 16 * rb + ai + 4 * c + akq : 0];
                        d = Acc4<T>::mma(oka ? a : (T)0, okb ? b : (T)0, d);
                    }
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) {
                        const int j = 16 * rb + Acc4<T>::row(g, rr);  // output row n = m + j
                        const int n1 = m + j + 1 <= P + 1 ? m + j + 1 : 0;
                        Z[(part * 32 + j) * 16 + col] = d[rr] * pw_t[n1];
                    }
                }
            }
            wsync();
            // conversion: lane (g, column) takes rows j = g, g + 4, .. (n = m + j < P)
#pragma unroll
            for (int j0 = 0; j0 < P - m; j0 += 4) {
                const int j = j0 + g;
                const bool okr = j < P - m;
                const int jj = okr ? j : 0;
                const int n = m + jj;
                const T zre = Z[jj * 16 + col];
                const T zim = m > 0 ? Z[(32 + jj) * 16 + col] : (T)0;
                // phi lanes: chi of the same translation (column + 8), other part
                const T pre = Z[jj * 16 + (col ^ 8)];
                const T pim = m > 0 ? Z[(32 + jj) * 16 + (col ^ 8)] : (T)0;
                // chi lanes: chi_{n+1}
                const T nre = Z[(jj + 1) * 16 + col];
                const T nim = m > 0 ? Z[(32 + jj + 1) * 16 + col] : (T)0;
                const T fphi = tau * (T)m * rcp[n > 0 ? n : 0];
                const T fchi = tau * rcp[n + 1];
                const T yre = pot ? zre - fchi * nre : zre - fphi * pim;
                const T yim = pot ? zim - fchi * nim : zim + fphi * pre;
                X[(okr ? tri(n) + m : L::NX) * 16 + col] = yre;
                if (m > 0) X[(okr ? NV + tri(n - 1) + m - 1 : L::NX) * 16 + col] = yim;
            }
            wsync();
        }
        // ---- rotation about y, back (R basis)
        rotate(1);
        wsync();
        // ---- rotation back about z (-phi) and accumulation into the lane's registers
        if (act) {
#pragma unroll
            for (int i = 0; i < NA; i++) {
                const int e = etab[i * 64 + lid];
                const int xrow = e & 511, prow = (e >> 9) & 511, m = (e >> 27) & 31;
                const T own = X[xrow * 16 + col], oth = X[prow * 16 + col];
                const T c = cst_t[2 * m], s = cst_t[2 * m + 1];
                // Re: re c + im s;  Im: im c - re s
                const T sg = xrow >= NV ? (T)-1 : (T)1;
                accr[i] += own * c + sg * oth * s;
            }
        }
        wsync();
    }
    {
        const int col = lane & 15, g = lane >> 4;
        const int box = slot_box[sbase + (col & 7)];
        if (box >= 0) {
            T *lp = Lc + (size_t)box * 2 * P2 + (col >> 3) * P2;
#pragma unroll
            for (int i = 0; i < NA; i++) lp[g + 4 * i] = accr[i];
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

template <typename T, int P>
static bool mfma_setup_t()
{
    constexpr size_t shm = mf::Lds<T, P>::bytes();
    return hipFuncSetAttribute((const void *)k_m2l_mfma<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) ==
           hipSuccess;
}

template <typename T, int P>
static void launch_mfma(const lhf_plan *Pl, int level, hipStream_t st)
{
    const int64_t npar = Pl->lev[level - 1].nb;
    const int64_t ntiles = (npar + 3) / 4;
    const int64_t per = (ntiles + 7) / 8;
    constexpr size_t shm = mf::Lds<T, P>::bytes();
    k_m2l_mfma<T, P><<<dim3((unsigned)(per * 8)), dim3(256), shm, st>>>(
        level, Pl->lev[level - 1].off, npar, Pl->bkey, Pl->bchild0, Pl->bnchild, Pl->dmap[level], (const T *)Pl->M,
        (T *)Pl->Lc, (const T *)Pl->rot, Pl->sched_row_start, Pl->sched_rows, Pl->sched_ncls, Pl->sched_cls_theta);
}

}  // namespace

static_assert(mf::Lds<double, 12>::bytes() <= 163840, "FP64 p = 12 buffers exceed the LDS");
static_assert(mf::Lds<float, 16>::bytes() <= 163840, "FP32 p = 16 buffers exceed the LDS");

// matrix-core M2L instantiations: FP64 p in {4, 6, 8, 10, 12}, FP32 p in {4, 6, 8, 10, 12, 16}
bool m2l_mfma_supported(int precision, int p)
{
    if (precision == LHF_FP64) return p == 4 || p == 6 || p == 8 || p == 10 || p == 12;
    return p == 4 || p == 6 || p == 8 || p == 10 || p == 12 || p == 16;
}

bool wmfma_build(lhf_plan *Pl, hipStream_t)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 4: return mfma_setup_t<double, 4>();
        case 6: return mfma_setup_t<double, 6>();
        case 8: return mfma_setup_t<double, 8>();
        case 10: return mfma_setup_t<double, 10>();
        case 12: return mfma_setup_t<double, 12>();
        }
    } else {
        switch (Pl->p) {
        case 4: return mfma_setup_t<float, 4>();
        case 6: return mfma_setup_t<float, 6>();
        case 8: return mfma_setup_t<float, 8>();
        case 10: return mfma_setup_t<float, 10>();
        case 12: return mfma_setup_t<float, 12>();
        case 16: return mfma_setup_t<float, 16>();
        }
    }
    return false;
}

void m2l_mfma_launch(const lhf_plan *Pl, int level, hipStream_t st)
{
    if (Pl->precision == LHF_FP64) {
        switch (Pl->p) {
        case 4: launch_mfma<double, 4>(Pl, level, st); break;
        case 6: launch_mfma<double, 6>(Pl, level, st); break;
        case 8: launch_mfma<double, 8>(Pl, level, st); break;
        case 10: launch_mfma<double, 10>(Pl, level, st); break;
        case 12: launch_mfma<double, 12>(Pl, level, st); break;
        }
    } else {
        switch (Pl->p) {
        case 4: launch_mfma<float, 4>(Pl, level, st); break;
        case 6: launch_mfma<float, 6>(Pl, level, st); break;
        case 8: launch_mfma<float, 8>(Pl, level, st); break;
        case 10: launch_mfma<float, 10>(Pl, level, st); break;
        case 12: launch_mfma<float, 12>(Pl, level, st); break;
        case 16: launch_mfma<float, 16>(Pl, level, st); break;
        }
    }
}

}  // namespace lhf

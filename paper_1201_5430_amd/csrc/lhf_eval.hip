// lhf_eval.hip -- the evaluation kernels of liblhfmm (one FMM pass).
//
//   P2M    multipole (phi, chi) of each leaf, Method 2 (eq. eve4)
//   M2M    child -> parent, rotation / coaxial (S|S) / S-conversion (eq. rcr1) / back-rotation
//   M2L    V-list source -> target, rotation / coaxial (S|R) / R-conversion / back-rotation;
//          chi-hat is carried to order p before the conversion, then truncated
//   L2L    parent -> child, rotation / coaxial (R|R) / R-conversion / back-rotation
//   L2P    v (eq. evf3) and grad v (eq. dt3 with t = e_l, eq. evf6) at each element, s = (grad v) omega
//   P2P    near field over adjacent leaves with the Gaussian core (eqs. 2, vem1)
//
// All expansions are in the scaled bar form documented in lhf_internal.h.
// Work decomposition: one 64-lane wavefront per box (P2M, M2M, M2L, L2L,
// L2P) and one lane per element (P2P).  A wavefront keeps the target box's
// accumulator in registers (lane owns packed rows lane, lane+64, ...), and the
// per-translation intermediate vectors in LDS.
#include <hip/hip_runtime.h>

#include <cstring>
#include <functional>

#include <algorithm>
#include <math.h>

#include "lhf_internal.h"

namespace lhf {

void m2l_tile_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_mfma_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_half_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_half_stage(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_quarter_launch(const lhf_plan *Pl, int level, hipStream_t st);
bool m2l_half_scalar_supported(int precision, int p);
void m2l_half_scalar_stage(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_half_scalar_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2l_quarter_stage(const lhf_plan *Pl, int level, hipStream_t st);
int m2l_quarter_max_ns(int p);
int m2l_qmfma_max_ns(int p);
void m2l_qmfma_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2m_half_launch(const lhf_plan *Pl, int level, hipStream_t st);
void l2l_half_launch(const lhf_plan *Pl, int level, hipStream_t st);
void m2m_quarter_launch(const lhf_plan *Pl, int level, hipStream_t st);
void l2l_quarter_launch(const lhf_plan *Pl, int level, hipStream_t st);

constexpr int WAVE = 64;
constexpr int NRMAX = (2 * MAXP * MAXP + WAVE - 1) / WAVE;  // accumulator rows per lane
constexpr int NPMAX = (MAXP * (MAXP + 1) / 2 + WAVE - 1) / WAVE;  // (n, m >= 0) pairs per lane

__device__ inline void decode_row(int q, int &n, int &m, int &part)
{
    int nn = (int)sqrtf((float)q);
    while (nn * nn > q) --nn;
    while ((nn + 1) * (nn + 1) <= q) ++nn;
    int j = q - nn * nn;
    n = nn;
    if (j <= nn) {
        part = 0;
        m = j;
    } else {
        part = 1;
        m = j - nn;
    }
}

// centre and side of a box; the key carries the system index above its 3*level Morton bits,
// and sys_geo[4s..4s+3] = (lo0, lo1, lo2, L) is that system's cube
__device__ inline void box_centre(uint64_t key, int level, const double *__restrict__ sys_geo, double &c0,
                                  double &c1, double &c2, double &h)
{
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < level; b++) {
        ix |= (uint32_t)((key >> (3 * b)) & 1u) << b;
        iy |= (uint32_t)((key >> (3 * b + 1)) & 1u) << b;
        iz |= (uint32_t)((key >> (3 * b + 2)) & 1u) << b;
    }
    const double *g = sys_geo + 4 * (key >> (3 * level));
    h = g[3] / (double)(1u << level);
    c0 = g[0] + ((double)ix + 0.5) * h;
    c1 = g[1] + ((double)iy + 0.5) * h;
    c2 = g[2] + ((double)iz + 0.5) * h;
}

// ---------------------------------------------------------------------------
// P2M: one workgroup per leaf, one thread per (n, m >= 0) pair (64 * ceil(p(p+1)/2 / 64) threads).
// For each element, the threads (element, m) build the column m of Rt_n^m(xhat)
// (R_n^m = (-1)^n i^m Rt_n^m) by the recurrence
//   Rt_m^m = -(x+iy)/(2m) Rt_{m-1}^{m-1},  Rt_{m+1}^m = z Rt_m^m,
//   Rt_n^m = ((2n-1) z Rt_{n-1}^m - r^2 Rt_{n-2}^m) / ((n-m)(n+m)),
// (the divisions by tables of reciprocals), then every thread adds the eq. eve4 contributions of
// its (n, m) pair (both potentials, Re and Im).  The columns are stored as triangles (n, m <= n).
// ---------------------------------------------------------------------------
// SC: scalar harmonic FMM -- phi = sum q g_n^m (the expansion of eq. rsbf5 of each source), chi = 0.
// SEG: vortex filaments -- each element is a segment (centre x, vector sl) expanded as nq
// Gauss-Legendre points x + sl xi_j / 2 of strength omega w_j / 2 (eqs. vf5, vf6); quad holds
// (xi_j, w_j).
constexpr int P2M_MAXT = 512;  // threads per workgroup at most (p(p+1)/2 = 300 at p = 24)

__host__ __device__ inline int tri_idx(int n, int m) { return n * (n + 1) / 2 + m; }

// workgroup size, elements per chunk and LDS bytes of k_p2m at order p for elements of tsize bytes
inline void p2m_config(int p, size_t tsize, int &nthr, int &ch, size_t &shm)
{
    const int TRI = p * (p + 1) / 2;
    nthr = std::min(P2M_MAXT, (TRI + WAVE - 1) / WAVE * WAVE);
    const size_t fixed = tsize * (size_t)(TRI + p + 1);
    const size_t per = tsize * (size_t)(2 * TRI + 4);
    ch = (int)std::max<size_t>(1, std::min<size_t>(16, (40960 - fixed) / per));
    shm = fixed + per * (size_t)ch;
}

template <typename T, bool SC = false, bool SEG = false>
__global__ void __launch_bounds__(P2M_MAXT) k_p2m(int p, int depth, int64_t leaf_off, const int32_t *__restrict__ leaves,
                                                  const int8_t *__restrict__ blev, const uint64_t *__restrict__ bkey,
                                                  const int32_t *__restrict__ bstart, const int32_t *__restrict__ bcount,
                                                  const T *__restrict__ xs, const T *__restrict__ ws,
                                                  const T *__restrict__ qs, int64_t n,
                                                  const double *__restrict__ sys_geo, T *__restrict__ M, int ch,
                                                  const T *__restrict__ sl = nullptr, int nq = 1,
                                                  const double *__restrict__ quad = nullptr)
{
    // the leaf's elements in chunks of ch: first the threads form the regular solid harmonics of
    // the chunk's (element, m) columns, then every thread adds the chunk's contributions to its
    // coefficient pair (two barriers per chunk)
    extern __shared__ char smem[];
    const int TRI = p * (p + 1) / 2, P2 = p * p;
    T *rinv = (T *)smem;                 // [TRI] 1 / ((n - m)(n + m)) at (n, m), n >= m + 2
    T *kinv = rinv + TRI;                // [p + 1] -1 / (2k)
    T *Rre = kinv + p + 1;               // [ch][TRI]  (element, n, m <= n)
    T *Rim = Rre + (size_t)ch * TRI;
    T *wsh = Rim + (size_t)ch * TRI;     // [ch][4] strengths: omega, q (0 without monopoles)
    const int tid = threadIdx.x, nthr = blockDim.x;
    // uniform tree: leaves leaf_off + blockIdx.x at level depth; adaptive: leaves[blockIdx.x] at blev[]
    const int64_t b = leaves ? (int64_t)leaves[blockIdx.x] : leaf_off + blockIdx.x;
    const int level = blev ? (int)blev[b] : depth;
    if (level < 2) return;  // no far field above level 2
    double c0, c1, c2, hd;
    box_centre(bkey[b], level, sys_geo, c0, c1, c2, hd);
    const T ih = (T)(1.0 / hd);
    for (int t = tid; t < TRI; t += nthr) {
        int nn = 0;
        while (tri_idx(nn + 1, 0) <= t) nn++;
        const int m = t - tri_idx(nn, 0);
        rinv[t] = nn >= m + 2 ? (T)(1.0 / (double)((nn - m) * (nn + m))) : (T)0;
    }
    for (int k = tid; k <= p; k += nthr) kinv[k] = k ? (T)(-0.5 / (double)k) : (T)0;
    // this thread's (n, m) pair
    const bool own = tid < TRI;
    int nn = 0;
    while (own && tri_idx(nn + 1, 0) <= tid) nn++;
    const int m = own ? tid - tri_idx(nn, 0) : 0;
    T acc[4] = {0, 0, 0, 0};  // Re a, Im a, Re b, Im b
    const int s0 = bstart[b], cnt = bcount[b] * (SEG ? nq : 1);  // SEG: (element, quadrature point)
    for (int e0 = 0; e0 < cnt; e0 += ch) {
        const int ne = min(ch, cnt - e0);
        __syncthreads();  // the previous chunk's tables are no longer read (first pass: the reciprocals are written)
        for (int q = tid; q < ne * p; q += nthr) {
            const int e = q / p, mc = q - e * p;
            const int i = SEG ? s0 + (e0 + e) / nq : s0 + e0 + e;
            T px = xs[i], py = xs[n + i], pz = xs[2 * n + i], wf = (T)1;
            if constexpr (SEG) {
                const int jq = (e0 + e) % nq;
                const T hx = (T)(0.5 * quad[2 * jq]);
                px += hx * sl[i];
                py += hx * sl[n + i];
                pz += hx * sl[2 * n + i];
                wf = (T)(0.5 * quad[2 * jq + 1]);
            }
            const T x = (px - (T)c0) * ih, y = (py - (T)c1) * ih, z = (pz - (T)c2) * ih;
            const T r2 = x * x + y * y + z * z;
            T *Re = Rre + (size_t)e * TRI, *Im = Rim + (size_t)e * TRI;
            // Rt_m^m = (-(x+iy)/2)^m / m!, then up in n
            T are = 1, aim = 0;
            for (int k = 1; k <= mc; k++) {
                const T f = kinv[k];
                const T nre = f * (are * x - aim * y), nim = f * (are * y + aim * x);
                are = nre;
                aim = nim;
            }
            Re[tri_idx(mc, mc)] = are;
            Im[tri_idx(mc, mc)] = aim;
            if (mc + 1 < p) {
                T p2re = are, p2im = aim, p1re = z * are, p1im = z * aim;
                Re[tri_idx(mc + 1, mc)] = p1re;
                Im[tri_idx(mc + 1, mc)] = p1im;
                for (int k = mc + 2; k < p; k++) {
                    const T inv = rinv[tri_idx(k, mc)], zc = (T)(2 * k - 1) * z;
                    const T cre = (zc * p1re - r2 * p2re) * inv;
                    const T cim = (zc * p1im - r2 * p2im) * inv;
                    Re[tri_idx(k, mc)] = cre;
                    Im[tri_idx(k, mc)] = cim;
                    p2re = p1re;
                    p2im = p1im;
                    p1re = cre;
                    p1im = cim;
                }
            }
            if (mc == 0) {
                wsh[4 * e] = SC ? (T)0 : wf * ws[i];
                wsh[4 * e + 1] = SC ? (T)0 : wf * ws[n + i];
                wsh[4 * e + 2] = SC ? (T)0 : wf * ws[2 * n + i];
                wsh[4 * e + 3] = qs ? wf * qs[i] : (T)0;
            }
        }
        __syncthreads();
        if (!own) continue;
        // the three conj(Rt) values of order n (phi) and of order n - 1 (chi) serve all four
        // outputs (Re and Im of a and b)
        const T sgn = (m & 1) ? (T)-1 : (T)1;
        for (int e = 0; e < ne; e++) {
            const T *Re = Rre + (size_t)e * TRI, *Im = Rim + (size_t)e * TRI;
            const T wx = wsh[4 * e], wy = wsh[4 * e + 1], wz = wsh[4 * e + 2], qe = wsh[4 * e + 3];
            // conj(Rt_n^k), with the convention conj(Rt_n^{-1}) = -Rt_n^1 that makes the m >= 1
            // formulas valid at m = 0 as well
            auto C = [&](int n2, int kk, T &re, T &im) {
                if (n2 < 0 || kk > n2) {
                    re = 0;
                    im = 0;
                } else if (kk == -1) {
                    if (n2 >= 1) {
                        re = -Re[tri_idx(n2, 1)];
                        im = -Im[tri_idx(n2, 1)];
                    } else {
                        re = 0;
                        im = 0;
                    }
                } else {
                    re = Re[tri_idx(n2, kk)];
                    im = -Im[tri_idx(n2, kk)];
                }
            };
            const T wmre = wx, wmim = -wy;  // wx - i wy
            const T wpre = wx, wpim = wy;   // wx + i wy
            if constexpr (SC) {
                T c3re, c3im;
                C(nn, m, c3re, c3im);
                acc[0] += qe * sgn * c3re;
                acc[1] += qe * sgn * c3im;
                continue;
            }
            {
                // a = -i (-1)^m / (n+1) [ (wx-iwy)(n-m+1)/2 C(m-1) + (wx+iwy)(n+m+1)/2 C(m+1) + wz m C(m) ]
                T c1re, c1im, c2re, c2im, c3re, c3im;
                C(nn, m - 1, c1re, c1im);
                C(nn, m + 1, c2re, c2im);
                C(nn, m, c3re, c3im);
                T f1 = (T)(nn - m + 1) * (T)0.5, f2 = (T)(nn + m + 1) * (T)0.5, f3 = wz * (T)m;
                T sre = f1 * (wmre * c1re - wmim * c1im) + f2 * (wpre * c2re - wpim * c2im) + f3 * c3re;
                T sim = f1 * (wmre * c1im + wmim * c1re) + f2 * (wpre * c2im + wpim * c2re) + f3 * c3im;
                T sc = sgn / (T)(nn + 1);
                // -i (sre + i sim) = sim - i sre; monopole q (eq. 7): phi gains -q g_n^m = -q (-1)^m C(m)
                acc[0] += sc * sim - qe * sgn * c3re;
                acc[1] += -sc * sre - qe * sgn * c3im;
            }
            if (nn >= 1) {
                // b = (-1)^m / n [ -1/2 (wx-iwy) C'(m-1) + 1/2 (wx+iwy) C'(m+1) + wz C'(m) ]
                T c1re, c1im, c2re, c2im, c3re, c3im;
                C(nn - 1, m - 1, c1re, c1im);
                C(nn - 1, m + 1, c2re, c2im);
                C(nn - 1, m, c3re, c3im);
                T sre = (T)-0.5 * (wmre * c1re - wmim * c1im) + (T)0.5 * (wpre * c2re - wpim * c2im) + wz * c3re;
                T sim = (T)-0.5 * (wmre * c1im + wmim * c1re) + (T)0.5 * (wpre * c2im + wpim * c2re) + wz * c3im;
                T sc = sgn / (T)nn;
                acc[2] += sc * sre;
                acc[3] += sc * sim;
            }
        }
    }
    if (!own) return;
    T *out = M + (size_t)b * 2 * P2;
    out[pk_re(nn, m)] = acc[0] * ih;
    out[P2 + pk_re(nn, m)] = acc[2] * ih;
    if (m > 0) {
        out[pk_im(nn, m)] = acc[1] * ih;
        out[P2 + pk_im(nn, m)] = acc[3] * ih;
    }
}

// ---------------------------------------------------------------------------
// Rotation / coaxial / conversion / back-rotation of one expansion by one
// wavefront.  KIND: 0 = M2M, 1 = M2L, 2 = L2L.
//   src    : 2 p^2 input reals (global memory)
//   X, Y   : LDS, 2 p^2 each;  Z : LDS, 2 (p+1)^2
//   Wf, Wb : forward / backward rotation sets of the direction's polar-angle class
//   zc, zs : cos(m phi), sin(m phi) of the direction, m < p
//   cf     : coaxial coefficients (M2L: k!/tau^(k+1), k <= 2p;  M2M/L2L: (-tau_p)^k/k!)
//   tau    : |t| / h used by the conversion (M2L: |t|/h, M2M: |t|/h_parent, L2L: |t|/h_child)
// The result is added into the lane's accumulator rows.
// ---------------------------------------------------------------------------
template <typename T, int KIND>
__device__ __attribute__((always_inline)) void rcr(int p, const T *__restrict__ src, T *X, T *Y, T *Z, const T *__restrict__ Wf,
                    const T *__restrict__ Wb, const T *__restrict__ zc, const T *__restrict__ zs,
                    const T *cf, T tau, T *acc)
{
    const int lane = threadIdx.x;
    const int P2 = p * p, R2 = 2 * P2;
    const int ZS = (p + 1) * (p + 1);
    // 1. load and rotate about z by +phi: c^m <- e^{i m phi} c^m
    for (int r = lane; r < R2; r += WAVE) {
        const int pot = r >= P2;
        int n, m, part;
        decode_row(r - pot * P2, n, m, part);
        const T *s = src + pot * P2;
        if (m == 0) {
            X[r] = s[pk_re(n, 0)];
        } else {
            T re = s[pk_re(n, m)], im = s[pk_im(n, m)];
            T c = zc[m], sn = zs[m];
            X[r] = part ? (re * sn + im * c) : (re * c - im * sn);
        }
    }
    __syncthreads();
    // 2. rotation about y (real, Re and Im blocks)
    for (int r = lane; r < R2; r += WAVE) {
        const int pot = r >= P2;
        int n, m, part;
        decode_row(r - pot * P2, n, m, part);
        const T *W = Wf + rot_block_off(n);
        const T *x = X + pot * P2 + n * n;
        T a = 0;
        if (!part) {
            const T *row = W + m * (n + 1);
            for (int k = 0; k <= n; k++) a += row[k] * x[k];
        } else {
            const T *row = W + (n + 1) * (n + 1) + (m - 1) * n;
            for (int k = 0; k < n; k++) a += row[k] * x[n + 1 + k];
        }
        Y[r] = a;
    }
    __syncthreads();
    // 3. coaxial translation along z (per m, per part)
    for (int r = lane; r < 2 * ZS; r += WAVE) {
        const int pot = r >= ZS;
        int n, m, part;
        decode_row(r - pot * ZS, n, m, part);
        T a = 0;
        if (KIND == 1) {
            // (S|R): out_n = sum_{n'=m}^{p-1} (n+n')!/tau^(n+n'+1) in_n'; chi to order p
            if (m < p && (n < p || pot == 1)) {
                const T *y = Y + pot * P2;
                for (int n2 = m; n2 < p; n2++) a += cf[n + n2] * y[n2 * n2 + m + (part ? n2 : 0)];
            }
        } else if (KIND == 0) {
            // (S|S): out_n = sum_{n'=m}^{n} (-tau_p)^(n-n')/(n-n')! 2^-(n'+1) [phi] / 2^-n' [chi] in_n'
            if (n < p) {
                const T *y = Y + pot * P2;
                T sc = pot ? (T)1 : (T)0.5;
                for (int k = 0; k < m; k++) sc *= (T)0.5;
                for (int n2 = m; n2 <= n; n2++) {
                    a += cf[n - n2] * sc * y[n2 * n2 + m + (part ? n2 : 0)];
                    sc *= (T)0.5;
                }
            }
        } else {
            // (R|R): out_n = 2^-n [phi] / 2^-(n+1) [chi] * sum_{n'=n}^{p-1} (-tau_p)^(n'-n)/(n'-n)! in_n'
            if (n < p) {
                const T *y = Y + pot * P2;
                for (int n2 = n; n2 < p; n2++) a += cf[n2 - n] * y[n2 * n2 + m + (part ? n2 : 0)];
                T sc = pot ? (T)0.5 : (T)1;
                for (int k = 0; k < n; k++) sc *= (T)0.5;
                a *= sc;
            }
        }
        Z[r] = a;
    }
    __syncthreads();
    // 4. conversion in the rotated frame (eq. rcr1, scaled)
    for (int r = lane; r < R2; r += WAVE) {
        const int pot = r >= P2;
        int n, m, part;
        decode_row(r - pot * P2, n, m, part);
        const T *Zp = Z, *Zc = Z + ZS;
        T out;
        if (KIND == 0) {
            // S-conversion: a~ = a - i tau m/(n+1) b ;  b~_n = b_n + tau/n b_{n-1}
            if (pot == 0) {
                T f = tau * (T)m / (T)(n + 1);
                if (!part) out = Zp[pk_re(n, m)] + (m ? f * Zc[pk_im(n, m)] : (T)0);
                else out = Zp[pk_im(n, m)] - f * Zc[pk_re(n, m)];
            } else {
                out = Zc[n * n + m + (part ? n : 0)];
                if (n >= 1 && m <= n - 1) out += tau / (T)n * Zc[(n - 1) * (n - 1) + m + (part ? n - 1 : 0)];
            }
        } else {
            // R-conversion: c~ = c + i tau m/n d ;  d~_n = d_n - tau/(n+1) d_{n+1}
            if (pot == 0) {
                T f = n > 0 ? tau * (T)m / (T)n : (T)0;
                if (!part) out = Zp[pk_re(n, m)] - (m ? f * Zc[pk_im(n, m)] : (T)0);
                else out = Zp[pk_im(n, m)] + f * Zc[pk_re(n, m)];
            } else {
                out = Zc[n * n + m + (part ? n : 0)];
                const int n1 = n + 1;
                if (KIND == 1 || n1 < p) out -= tau / (T)(n + 1) * Zc[n1 * n1 + m + (part ? n1 : 0)];
            }
        }
        X[r] = out;
    }
    __syncthreads();
    // 5. back-rotation about y
    for (int r = lane; r < R2; r += WAVE) {
        const int pot = r >= P2;
        int n, m, part;
        decode_row(r - pot * P2, n, m, part);
        const T *W = Wb + rot_block_off(n);
        const T *x = X + pot * P2 + n * n;
        T a = 0;
        if (!part) {
            const T *row = W + m * (n + 1);
            for (int k = 0; k <= n; k++) a += row[k] * x[k];
        } else {
            const T *row = W + (n + 1) * (n + 1) + (m - 1) * n;
            for (int k = 0; k < n; k++) a += row[k] * x[n + 1 + k];
        }
        Y[r] = a;
    }
    __syncthreads();
    // 6. rotate about z by -phi and accumulate
#pragma unroll
    for (int k = 0; k < NRMAX; k++) {
        const int r = lane + WAVE * k;
        if (r >= R2) break;
        const int pot = r >= P2;
        int n, m, part;
        decode_row(r - pot * P2, n, m, part);
        const T *y = Y + pot * P2;
        if (m == 0) {
            acc[k] += y[pk_re(n, 0)];
        } else {
            T re = y[pk_re(n, m)], im = y[pk_im(n, m)];
            T c = zc[m], sn = zs[m];
            acc[k] += part ? (-re * sn + im * c) : (re * c + im * sn);
        }
    }
    __syncthreads();
}

struct EvalArgs {
    int p, depth;
    int64_t n;
    double lo0, lo1, lo2, L;
};

// M2M for one level: wavefront per parent box
template <typename T>
__global__ void __launch_bounds__(WAVE) k_m2m(int p, int64_t off, const int32_t *__restrict__ bchild0,
                                              const int32_t *__restrict__ bnchild, const uint64_t *__restrict__ bkey,
                                              T *__restrict__ M, const T *__restrict__ rot, const T *__restrict__ zph,
                                              const int16_t *__restrict__ dir_theta)
{
    extern __shared__ char smem[];
    const int P2 = p * p, ZS = (p + 1) * (p + 1);
    T *X = (T *)smem, *Y = X + 2 * P2, *Z = Y + 2 * P2, *cf = Z + 2 * ZS;
    const int lane = threadIdx.x;
    const int64_t b = off + blockIdx.x;
    if (bnchild[b] == 0) return;  // a leaf keeps the multipole of its own elements
    if (lane < p) {
        // (-tau_p)^k / k!, tau_p = sqrt(3)/4
        double t = 1.0, tp = -0.4330127018922193;
        for (int k = 1; k <= lane; k++) t *= tp / (double)k;
        cf[lane] = (T)t;
    }
    __syncthreads();
    T acc[NRMAX];
#pragma unroll
    for (int k = 0; k < NRMAX; k++) acc[k] = 0;
    const int rs = rot_set_size(p);
    const int c0 = bchild0[b], nc = bnchild[b];
    for (int c = 0; c < nc; c++) {
        const int cb = c0 + c;
        const int oct = (int)(bkey[cb] & 7u);
        const int dir = NDIR_M2L + oct;  // t = parent - child
        const T *R = rot + (size_t)dir_theta[dir] * ROT_NKIND * rs;
        const T *zp = zph + (size_t)dir * 2 * p;
        rcr<T, 0>(p, M + (size_t)cb * 2 * P2, X, Y, Z, R + ROT_S_FWD * rs, R + ROT_S_BACK * rs, zp, zp + p, cf,
                  (T)0.4330127018922193, acc);
    }
    T *out = M + (size_t)b * 2 * P2;
#pragma unroll
    for (int k = 0; k < NRMAX; k++) {
        const int r = lane + WAVE * k;
        if (r >= 2 * P2) break;
        out[r] = acc[k];
    }
}

// Downward pass for one level: L2L from the parent (levels > 2) + M2L over the V-list
template <typename T>
__global__ void __launch_bounds__(WAVE) k_down(int p, int level, int do_m2l, int64_t off, const int32_t *__restrict__ bparent,
                                               const uint64_t *__restrict__ bkey, const int32_t *__restrict__ vcount,
                                               const int32_t *__restrict__ vsrc, const int16_t *__restrict__ vdir,
                                               const T *__restrict__ M, T *__restrict__ Lc, const T *__restrict__ rot,
                                               const T *__restrict__ zph, const int16_t *__restrict__ dir_theta,
                                               const T *__restrict__ coax)
{
    extern __shared__ char smem[];
    const int P2 = p * p, ZS = (p + 1) * (p + 1);
    T *X = (T *)smem, *Y = X + 2 * P2, *Z = Y + 2 * P2, *cf = Z + 2 * ZS;
    const int lane = threadIdx.x;
    const int64_t b = off + blockIdx.x;
    const int rs = rot_set_size(p);
    T acc[NRMAX];
#pragma unroll
    for (int k = 0; k < NRMAX; k++) acc[k] = 0;
    if (level > 2) {
        if (lane < p) {
            double t = 1.0, tp = -0.4330127018922193;
            for (int k = 1; k <= lane; k++) t *= tp / (double)k;
            cf[lane] = (T)t;
        }
        __syncthreads();
        const int oct = (int)(bkey[b] & 7u);
        const int dir = NDIR_M2L + 8 + oct;  // t = child - parent
        const T *R = rot + (size_t)dir_theta[dir] * ROT_NKIND * rs;
        const T *zp = zph + (size_t)dir * 2 * p;
        rcr<T, 2>(p, Lc + (size_t)bparent[b] * 2 * P2, X, Y, Z, R + ROT_R_FWD * rs, R + ROT_R_BACK * rs, zp,
                  zp + p, cf, (T)0.8660254037844386, acc);
    }
    const int nv = do_m2l ? vcount[b] : 0;
    for (int j = 0; j < nv; j++) {
        const int src = vsrc[(size_t)b * VMAX + j];
        const int dir = vdir[(size_t)b * VMAX + j];
        const int dx = dir % 7 - 3, dy = (dir / 7) % 7 - 3, dz = dir / 49 - 3;
        const int d2 = dx * dx + dy * dy + dz * dz;
        const T *R = rot + (size_t)dir_theta[dir] * ROT_NKIND * rs;
        const T *zp = zph + (size_t)dir * 2 * p;
        rcr<T, 1>(p, M + (size_t)src * 2 * P2, X, Y, Z, R + ROT_S_FWD * rs, R + ROT_R_BACK * rs, zp, zp + p,
                  coax + (size_t)d2 * (2 * p + 2), (T)sqrt((double)d2), acc);
    }
    T *out = Lc + (size_t)b * 2 * P2;
#pragma unroll
    for (int k = 0; k < NRMAX; k++) {
        const int r = lane + WAVE * k;
        if (r >= 2 * P2) break;
        out[r] = acc[k];
    }
}

// Compensated running sum (Knuth's TwoSum, branch-free): the rounding error of each
// addition is carried in c.  The near field adds one source box's partial sum at a
// time, so the accumulation error no longer grows with the number of source boxes.
template <typename T>
struct CompSum {
    T s = 0, c = 0;
    __device__ __forceinline__ void add(T x)
    {
        const T t = s + x;
        const T bp = t - s;
        c += (s - (t - bp)) + (x - bp);
        s = t;
    }
    __device__ __forceinline__ T value() const { return s + c; }
};

// L2P accumulator: compensated in FP32 (the p(p+1)/2 terms of a local expansion partly cancel;
// a compensated sum keeps the FP32 far field at the rounding of its terms), plain in FP64
template <typename T>
struct L2PAcc {
    T s = 0;
    __device__ __forceinline__ void add(T x) { s += x; }
    __device__ __forceinline__ T value() const { return s; }
};
template <>
struct L2PAcc<float> : CompSum<float> {
};

// ---------------------------------------------------------------------------
// L2P: one wavefront per leaf.  The velocity coefficients (eq. evf3, bar form)
//   Vx = 1/2 [-P_{n+1}^{m-1} + P_{n+1}^{m+1} - i(n-m) X_n^{m+1} - i(n+m) X_n^{m-1}]
//   Vy = 1/2 [ i P_{n+1}^{m-1} + i P_{n+1}^{m+1} + (n-m) X_n^{m+1} - (n+m) X_n^{m-1}]
//   Vz = -P_{n+1}^m - i m X_n^m
// (P = phi, X = chi of the leaf's local expansion, c^{-1} := -conj(c^1)) are
// formed in LDS; the derivatives u_lk = D_{e_l} v_k (eq. dt3) are applied on
// the fly:  u_x = 1/2(-V^{m-1} + V^{m+1}),  u_y = i/2 (V^{m-1} + V^{m+1}),
// u_z = -V^m (all at order n+1).  Each lane evaluates one element:
//   F(xhat) = sum_n (-1)^n [F_n^0 Rt_n^0 + 2 Re sum_{m>0} F_n^m Rt_n^m].
// ---------------------------------------------------------------------------
// Four leaves per 64-lane workgroup, 16 lanes each (leaves hold a few elements at the depths
// that minimise the total work, so one wavefront per leaf would leave most lanes idle).  The
// velocity coefficients go to a per-leaf block of global memory (Vg, [3][TRI] complex, column-major
// in (n, m): the column sweep of the evaluation then reads consecutive addresses) rather than to
// LDS: at high orders the LDS copies of four leaves (53 KB at p = 23 in FP64) left 3 wavefronts
// per compute unit.  The recurrence divides by a table of reciprocals built in LDS.
constexpr int L2P_LPB = 4;   // leaves per workgroup
constexpr int L2P_LANES = WAVE / L2P_LPB;

// column-major offset of (n, m), m <= n < p: columns m = 0 .. p-1 of lengths p - m
__host__ __device__ inline int cm_idx(int p, int n, int m) { return m * p - m * (m - 1) / 2 + (n - m); }

template <typename T>
struct Cplx {
    T re, im;
};

template <typename T>
__global__ void __launch_bounds__(WAVE) k_l2p(int p, int depth, int64_t nleaf, int64_t leaf_off,
                                              const int32_t *__restrict__ leaves, const int8_t *__restrict__ blev,
                                              const uint64_t *__restrict__ bkey, const int32_t *__restrict__ bstart,
                                              const int32_t *__restrict__ bcount, const T *__restrict__ xs,
                                              const T *__restrict__ ws, int64_t n, const double *__restrict__ sys_geo,
                                              const T *__restrict__ Lc, T *__restrict__ vfar, int grad,
                                              Cplx<T> *__restrict__ Vg)
{
    extern __shared__ char smem[];
    const int P2 = p * p;
    const int TRI = p * (p + 1) / 2;  // (n, m >= 0) pairs, n < p
    T *rinv = (T *)smem;              // [TRI] 1 / ((n - m)(n + m)) at cm_idx(n, m), n >= m + 2
    T *kinv = rinv + TRI;             // [p + 1] -1 / (2k)
    for (int m = 0; m < p; m++)
        for (int nn = m + threadIdx.x; nn < p; nn += WAVE)
            rinv[cm_idx(p, nn, m)] = nn >= m + 2 ? (T)(1.0 / (double)((nn - m) * (nn + m))) : (T)0;
    for (int k = threadIdx.x; k <= p; k += WAVE) kinv[k] = k ? (T)(-0.5 / (double)k) : (T)0;
    const int g = threadIdx.x / L2P_LANES, lane = threadIdx.x % L2P_LANES;
    const int64_t li = (int64_t)blockIdx.x * L2P_LPB + g;
    const bool has = li < nleaf;
    const int64_t b = has ? (leaves ? (int64_t)leaves[li] : leaf_off + li) : 0;
    const int level = has ? (blev ? (int)blev[b] : depth) : 0;
    const bool far = has && level >= 2;  // a leaf above level 2 has no local expansion: far field zero
    Cplx<T> *V = Vg + (size_t)(has ? li : 0) * 3 * TRI;  // this leaf's [3][TRI]
    const T *cd = Lc + (size_t)b * 2 * P2;
    auto get = [&](int pot, int nn, int m, T &re, T &im) {
        if (nn < 0 || nn >= p) {
            re = 0;
            im = 0;
            return;
        }
        const T *c = cd + pot * P2;
        if (m == -1) {
            if (nn >= 1) {
                re = -c[pk_re(nn, 1)];
                im = c[pk_im(nn, 1)];
            } else {
                re = 0;
                im = 0;
            }
        } else if (m > nn) {
            re = 0;
            im = 0;
        } else {
            re = c[pk_re(nn, m)];
            im = m ? c[pk_im(nn, m)] : (T)0;
        }
    };
    if (far)
        for (int t = lane; t < TRI; t += L2P_LANES) {
            int nn = 0;
            while ((nn + 1) * (nn + 2) / 2 <= t) nn++;
            const int m = t - nn * (nn + 1) / 2;
            T pm1r, pm1i, pp1r, pp1i, p0r, p0i, xm1r, xm1i, xp1r, xp1i, x0r, x0i;
            get(0, nn + 1, m - 1, pm1r, pm1i);
            get(0, nn + 1, m + 1, pp1r, pp1i);
            get(0, nn + 1, m, p0r, p0i);
            get(1, nn, m - 1, xm1r, xm1i);
            get(1, nn, m + 1, xp1r, xp1i);
            get(1, nn, m, x0r, x0i);
            const T a = (T)(nn - m), c = (T)(nn + m);
            const int ci = cm_idx(p, nn, m);
            // Vx = 1/2[-Pm1 + Pp1 - i a Xp1 - i c Xm1]
            V[ci] = Cplx<T>{(T)0.5 * (-pm1r + pp1r + a * xp1i + c * xm1i), (T)0.5 * (-pm1i + pp1i - a * xp1r - c * xm1r)};
            // Vy = 1/2[i Pm1 + i Pp1 + a Xp1 - c Xm1]
            V[TRI + ci] =
                Cplx<T>{(T)0.5 * (-pm1i - pp1i + a * xp1r - c * xm1r), (T)0.5 * (pm1r + pp1r + a * xp1i - c * xm1i)};
            // Vz = -P0 - i m X0
            V[2 * TRI + ci] = Cplx<T>{-p0r + (T)m * x0i, -p0i - (T)m * x0r};
        }
    __syncthreads();  // the leaf's coefficients (global memory, written by this workgroup) and the tables
    if (!has) return;
    const int s0 = bstart[b], cnt = bcount[b];
    if (!far) {
        const int nk = grad ? 15 : 6;
        for (int e = lane; e < cnt; e += L2P_LANES)
            for (int k = 0; k < nk; k++) vfar[(size_t)k * n + s0 + e] = (T)0;
        return;
    }
    double c0, c1, c2, hd;
    box_centre(bkey[b], level, sys_geo, c0, c1, c2, hd);
    const T ih = (T)(1.0 / hd);
    // V_k at (nn, m) for m = -1 .. nn + 1 (V^{-1} = -conj(V^1), zero beyond the triangle)
    auto vget = [&](int k, int nn, int m, T &re, T &im) {
        if (nn >= p || nn < 0 || m > nn) {
            re = 0;
            im = 0;
            return;
        }
        if (m == -1) {
            if (nn >= 1) {
                const Cplx<T> c = V[k * TRI + cm_idx(p, nn, 1)];
                re = -c.re;
                im = c.im;
            } else {
                re = 0;
                im = 0;
            }
            return;
        }
        const Cplx<T> c = V[k * TRI + cm_idx(p, nn, m)];
        re = c.re;
        im = c.im;
    };
    for (int e0 = 0; e0 < cnt; e0 += L2P_LANES) {
        const int e = e0 + lane;
        const bool act = e < cnt;
        const int i = s0 + (act ? e : 0);
        const T x = (xs[i] - (T)c0) * ih, y = (xs[n + i] - (T)c1) * ih, z = (xs[2 * n + i] - (T)c2) * ih;
        const T r2 = x * x + y * y + z * z;
        L2PAcc<T> v[3], gr[9];
        // walk the columns m; Rt_m^m by recurrence, then up in n
        T mre = 1, mim = 0;
        for (int m = 0; m < p; m++) {
            if (m > 0) {
                const T f = kinv[m];
                T nre = f * (mre * x - mim * y), nim = f * (mre * y + mim * x);
                mre = nre;
                mim = nim;
            }
            T p1re = mre, p1im = mim, p2re = 0, p2im = 0;
            const T wgt = m ? (T)2 : (T)1;
            for (int nn = m; nn < p; nn++) {
                T rre, rim;
                if (nn == m) {
                    rre = mre;
                    rim = mim;
                } else if (nn == m + 1) {
                    rre = z * p1re;
                    rim = z * p1im;
                } else {
                    const T inv = rinv[cm_idx(p, nn, m)];
                    rre = ((T)(2 * nn - 1) * z * p1re - r2 * p2re) * inv;
                    rim = ((T)(2 * nn - 1) * z * p1im - r2 * p2im) * inv;
                }
                if (nn > m) {
                    p2re = p1re;
                    p2im = p1im;
                    p1re = rre;
                    p1im = rim;
                }
                const T sw = ((nn & 1) ? -wgt : wgt);
                // velocity
                for (int k = 0; k < 3; k++) {
                    T fr, fi;
                    vget(k, nn, m, fr, fi);
                    v[k].add(sw * (fr * rre - fi * rim));
                    // gradient: u_x, u_y, u_z of v_k at (nn, m) from V_k at nn+1
                    T ar, ai, br, bi, cr, ci;
                    vget(k, nn + 1, m - 1, ar, ai);
                    vget(k, nn + 1, m + 1, br, bi);
                    vget(k, nn + 1, m, cr, ci);
                    T uxr = (T)0.5 * (br - ar), uxi = (T)0.5 * (bi - ai);
                    T uyr = (T)-0.5 * (ai + bi), uyi = (T)0.5 * (ar + br);
                    T uzr = -cr, uzi = -ci;
                    gr[3 * k + 0].add(sw * (uxr * rre - uxi * rim));
                    gr[3 * k + 1].add(sw * (uyr * rre - uyi * rim));
                    gr[3 * k + 2].add(sw * (uzr * rre - uzi * rim));
                }
            }
        }
        if (act) {
            const T wx = ws[i], wy = ws[n + i], wz = ws[2 * n + i];
            const T ih2 = ih * ih;
            T g[9];
            for (int k = 0; k < 9; k++) g[k] = gr[k].value();
            for (int k = 0; k < 3; k++) {
                vfar[k * n + i] = v[k].value() * ih;
                vfar[(3 + k) * n + i] = (g[3 * k] * wx + g[3 * k + 1] * wy + g[3 * k + 2] * wz) * ih2;
            }
            // grad v (row k = component, column l = derivative), rows 6..14 of the far-field array
            if (grad)
                for (int k = 0; k < 9; k++) vfar[(6 + k) * n + i] = g[k] * ih2;
        }
    }
}

// ---------------------------------------------------------------------------
// W/X interactions by expansions (adaptive tree, LHF_WX_EXPANSIONS).
//
// Scaled S basis: St_n^m(x) = (n-m)! P_n^m(cos theta) e^{i m phi} / r^(n+1) (Condon-Shortley
// P_n^m), St_n^{-m} = (-1)^m conj(St_n^m); S_n^m = (-i)^m St_n^m.  Column m by
//   St_0^0 = 1/r,  St_m^m = -(2m-1)(x+iy)/r^2 St_{m-1}^{m-1},  St_{m+1}^m = (2m+1) z/r^2 St_m^m,
//   St_n^m = ((2n-1) z St_{n-1}^m - (n+m-1)(n-m-1) St_{n-2}^m) / r^2.
// In these functions the paper's derivative relations (eq. mr4) and the rotational operator in
// the S basis (eq. drt5) read
//   d_x St_n^m = (St_{n+1}^{m+1} - St_{n+1}^{m-1})/2,  d_y St_n^m = (St_{n+1}^{m+1} + St_{n+1}^{m-1})/(2i),
//   d_z St_n^m = -St_{n+1}^m,
//   D_{r x t} St_n^m = -i/2 [(t_x + i t_y)(n+m) St_n^{m-1} + (t_x - i t_y)(n-m) St_n^{m+1}] - i t_z m St_n^m,
// and in the local basis Rt (R_n^m = (-1)^n i^m Rt_n^m; eqs. dt2 and drt4)
//   D_t Rt_n^m = (t_x - i t_y)/2 Rt_{n-1}^{m+1} - (t_x + i t_y)/2 Rt_{n-1}^{m-1} + t_z Rt_{n-1}^m,
//   D_{r x t} Rt_n^m = -i/2 [(t_x + i t_y)(n-m+1) Rt_n^{m-1} + (t_x - i t_y)(n+m+1) Rt_n^{m+1}] - i t_z m Rt_n^m.
// ---------------------------------------------------------------------------

// P2L: one wavefront per leaf b (level >= 2) with X sources.  In the leaf's scaled frame
// (xhat = (x - c)/h) the potential of a unit source is 1/|yhat - xhat| = sum Rt_n^m(yhat) U_n^m,
// U_n^m = conj(St_n^m(xhat)).  Its field grad U x omega - q grad U is the Lamb-Helmholtz pair
//   Phi_n = -[D_{r x omega} U]_n / n - q U_n,   Chi_n = [D_omega U]_n / (n+1)
// (Phi from r . v, Chi from curl v: both sides are harmonic and homogeneous order by order),
// so the leaf's stored local coefficients gain c_n^m += (-1)^n Phi_n^m / h and
// d_n^m += (-1)^n Chi_n^m / h (the bar form: c = i^m phi h^n, d = i^m chi h^(n+1)).
// Elements in chunks of ch: the lanes first form the St columns of the chunk in LDS, then every
// lane adds the chunk's contributions to its (n, m) pairs (both potentials, Re and Im).  Runs after the downward pass
// and before L2P; only the leaf's own wavefront writes its local expansion.
template <typename T>
__global__ void __launch_bounds__(WAVE) k_p2l(int p, const int32_t *__restrict__ leaves,
                                              const int8_t *__restrict__ blev, const uint64_t *__restrict__ bkey,
                                              const int32_t *__restrict__ bstart, const int32_t *__restrict__ bcount,
                                              const int32_t *__restrict__ wx_start, const int32_t *__restrict__ wx_ent,
                                              const T *__restrict__ xs, const T *__restrict__ ws,
                                              const T *__restrict__ qs, int64_t n, const double *__restrict__ sys_geo,
                                              T *__restrict__ Lc, int ch)
{
    extern __shared__ char smem[];
    const int P1 = p + 1, SS = P1 * P1, P2 = p * p, TRI = p * (p + 1) / 2;
    T *Sre = (T *)smem;               // [ch][n <= p][m <= n]
    T *Sim = Sre + (size_t)ch * SS;
    T *wsh = Sim + (size_t)ch * SS;   // [ch][4]: omega, q
    const int lane = threadIdx.x;
    const int64_t li = blockIdx.x;
    const int b = leaves[li];
    const int level = blev[b];
    const int ea = wx_start[li], eb = wx_start[li + 1];
    int anyx = 0;
    for (int e = ea + lane; e < eb; e += WAVE) anyx |= wx_ent[e] & 1;
    if (level < 2 || !__syncthreads_or(anyx)) return;
    double c0, c1, c2, hd;
    box_centre(bkey[b], level, sys_geo, c0, c1, c2, hd);
    const T ih = (T)(1.0 / hd);
    T acc[4 * NPMAX];  // per (n, m) pair of the lane: Re c, Im c, Re d, Im d
#pragma unroll
    for (int k = 0; k < 4 * NPMAX; k++) acc[k] = 0;
    for (int e = ea; e < eb; e++) {
        const int code = wx_ent[e];
        if (!(code & 1)) continue;
        const int q = code >> 1, s0 = bstart[q], cnt = bcount[q];
        for (int e0 = 0; e0 < cnt; e0 += ch) {
            const int ne = min(ch, cnt - e0);
            __syncthreads();  // the previous chunk's columns are no longer read
            for (int t = lane; t < ne * P1; t += WAVE) {
                const int el = t / P1, m = t - el * P1;
                const int i = s0 + e0 + el;
                const T x = (xs[i] - (T)c0) * ih, y = (xs[n + i] - (T)c1) * ih, z = (xs[2 * n + i] - (T)c2) * ih;
                const T ir2 = (T)1 / (x * x + y * y + z * z);
                T are = sqrt(ir2), aim = 0;  // St_0^0 = 1/r, then up the diagonal to St_m^m
                for (int k = 1; k <= m; k++) {
                    const T f = -(T)(2 * k - 1) * ir2;
                    const T nre = f * (are * x - aim * y), nim = f * (are * y + aim * x);
                    are = nre;
                    aim = nim;
                }
                T *Re = Sre + (size_t)el * SS, *Im = Sim + (size_t)el * SS;
                Re[m * P1 + m] = are;
                Im[m * P1 + m] = aim;
                T p2re = 0, p2im = 0, p1re = are, p1im = aim;
                for (int nn = m + 1; nn <= p; nn++) {
                    const T a1 = (T)(2 * nn - 1) * z * ir2, a2 = (T)((nn + m - 1) * (nn - m - 1)) * ir2;
                    const T cre = a1 * p1re - a2 * p2re, cim = a1 * p1im - a2 * p2im;
                    Re[nn * P1 + m] = cre;
                    Im[nn * P1 + m] = cim;
                    p2re = p1re;
                    p2im = p1im;
                    p1re = cre;
                    p1im = cim;
                }
                if (m == 0) {
                    wsh[4 * el] = ws[i];
                    wsh[4 * el + 1] = ws[n + i];
                    wsh[4 * el + 2] = ws[2 * n + i];
                    wsh[4 * el + 3] = qs ? qs[i] : (T)0;
                }
            }
            __syncthreads();
            // lane per (n, m >= 0) pair: the U values of orders n and n + 1 serve all four outputs
#pragma unroll
            for (int k = 0; k < NPMAX; k++) {
                const int t = lane + WAVE * k;
                if (t >= TRI) break;
                int nn = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
                while (nn * (nn + 1) / 2 > t) --nn;
                while ((nn + 1) * (nn + 2) / 2 <= t) ++nn;
                const int m = t - nn * (nn + 1) / 2;
                const T sgn = (nn & 1) ? (T)-1 : (T)1;
                for (int el = 0; el < ne; el++) {
                    const T *Re = Sre + (size_t)el * SS, *Im = Sim + (size_t)el * SS;
                    const T wx = wsh[4 * el], wy = wsh[4 * el + 1], wz = wsh[4 * el + 2], qe = wsh[4 * el + 3];
                    // U_n2^kk = conj(St_n2^kk); U_n2^{-1} = -conj(U_n2^1) = -St_n2^1
                    auto U = [&](int n2, int kk, T &re, T &im) {
                        if (n2 < 0 || n2 > p || kk > n2) {
                            re = 0;
                            im = 0;
                        } else if (kk == -1) {
                            re = n2 >= 1 ? -Re[n2 * P1 + 1] : (T)0;
                            im = n2 >= 1 ? -Im[n2 * P1 + 1] : (T)0;
                        } else {
                            re = Re[n2 * P1 + kk];
                            im = -Im[n2 * P1 + kk];
                        }
                    };
                    {
                        // Phi = -D/n - q U, D = -(i/2)[(wx+iwy)(n-m) U^{m+1} + (wx-iwy)(n+m) U^{m-1}] - i wz m U^m
                        T upr, upi, umr, umi, u0r, u0i;
                        U(nn, m + 1, upr, upi);
                        U(nn, m - 1, umr, umi);
                        U(nn, m, u0r, u0i);
                        const T fa = (T)(nn - m), fb = (T)(nn + m);
                        const T xr = fa * (wx * upr - wy * upi) + fb * (wx * umr + wy * umi);
                        const T xi = fa * (wx * upi + wy * upr) + fb * (wx * umi - wy * umr);
                        const T dre = (T)0.5 * xi + wz * (T)m * u0i;
                        const T dim = (T)-0.5 * xr - wz * (T)m * u0r;
                        const T inv = nn > 0 ? (T)1 / (T)nn : (T)0;
                        acc[4 * k + 0] += sgn * (-dre * inv - qe * u0r);
                        acc[4 * k + 1] += sgn * (-dim * inv - qe * u0i);
                    }
                    {
                        // Chi = [1/2 (wx-iwy) U_{n+1}^{m-1} - 1/2 (wx+iwy) U_{n+1}^{m+1} + wz U_{n+1}^m] / (n+1)
                        T umr, umi, upr, upi, u0r, u0i;
                        U(nn + 1, m - 1, umr, umi);
                        U(nn + 1, m + 1, upr, upi);
                        U(nn + 1, m, u0r, u0i);
                        const T inv = (T)1 / (T)(nn + 1);
                        acc[4 * k + 2] +=
                            sgn * ((T)0.5 * (wx * umr + wy * umi) - (T)0.5 * (wx * upr - wy * upi) + wz * u0r) * inv;
                        acc[4 * k + 3] +=
                            sgn * ((T)0.5 * (wx * umi - wy * umr) - (T)0.5 * (wx * upi + wy * upr) + wz * u0i) * inv;
                    }
                }
            }
        }
    }
    T *out = Lc + (size_t)b * 2 * P2;
#pragma unroll
    for (int k = 0; k < NPMAX; k++) {
        const int t = lane + WAVE * k;
        if (t >= TRI) break;
        int nn = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (nn * (nn + 1) / 2 > t) --nn;
        while ((nn + 1) * (nn + 2) / 2 <= t) ++nn;
        const int m = t - nn * (nn + 1) / 2;
        out[pk_re(nn, m)] += acc[4 * k] * ih;
        out[P2 + pk_re(nn, m)] += acc[4 * k + 2] * ih;
        if (m > 0) {
            out[pk_im(nn, m)] += acc[4 * k + 1] * ih;
            out[P2 + pk_im(nn, m)] += acc[4 * k + 3] * ih;
        }
    }
}

// M2P: one wavefront per leaf with W boxes, a lane per target element.  For each W box q
// (centre c, side h) the velocity coefficients of its multipole in the St basis,
//   V_x = (A_{N-1}^{M-1} - A_{N-1}^{M+1})/2 - i/2 [(N+M+1) B_N^{M+1} + (N-M+1) B_N^{M-1}]
//   V_y = -i/2 (A_{N-1}^{M-1} + A_{N-1}^{M+1}) + 1/2 [(N+M+1) B_N^{M+1} - (N-M+1) B_N^{M-1}]
//   V_z = -A_{N-1}^M - i M B_N^M,     A = (-1)^m a, B = (-1)^m b  (a, b: the stored bar form)
// (v = grad phi + grad chi x r, eq. evf3's S-basis counterpart), are formed in LDS for N <= p;
// each lane evaluates v = sum V_N^M St_N^M(yhat)/h and grad v from the derivative relations
// at N + 1 (/h^2), yhat = (y - c)/h, and adds them (and s = grad v . omega) to the far field
// that L2P wrote.
template <typename T>
__global__ void __launch_bounds__(WAVE) k_m2p(int p, const int32_t *__restrict__ leaves,
                                              const int8_t *__restrict__ blev, const uint64_t *__restrict__ bkey,
                                              const int32_t *__restrict__ bstart, const int32_t *__restrict__ bcount,
                                              const int32_t *__restrict__ wx_start, const int32_t *__restrict__ wx_ent,
                                              const T *__restrict__ xs, const T *__restrict__ ws, int64_t n,
                                              const double *__restrict__ sys_geo, const T *__restrict__ M,
                                              T *__restrict__ vfar, int grad)
{
    extern __shared__ char smem[];
    const int P2 = p * p, TRI = (p + 1) * (p + 2) / 2;  // (N, M >= 0), N <= p
    T *Vre = (T *)smem, *Vim = Vre + 3 * TRI;           // [3][TRI]
    const int lane = threadIdx.x;
    const int64_t li = blockIdx.x;
    const int b = leaves[li];
    const int ea = wx_start[li], eb = wx_start[li + 1];
    int anyw = 0;
    for (int e = ea + lane; e < eb; e += WAVE) anyw |= !(wx_ent[e] & 1);
    if (!__syncthreads_or(anyw)) return;
    const int s0 = bstart[b], cnt = bcount[b];
    auto vget = [&](int k, int nn, int m, T &re, T &im) {
        if (nn < 0 || nn > p || m > nn) {
            re = 0;
            im = 0;
        } else if (m == -1) {  // V^{-1} = -conj(V^1)
            const int t = nn * (nn + 1) / 2 + 1;
            re = nn >= 1 ? -Vre[k * TRI + t] : (T)0;
            im = nn >= 1 ? Vim[k * TRI + t] : (T)0;
        } else {
            const int t = nn * (nn + 1) / 2 + m;
            re = Vre[k * TRI + t];
            im = Vim[k * TRI + t];
        }
    };
    for (int tb = 0; tb < cnt; tb += WAVE) {
        const int e = tb + lane;
        const bool act = e < cnt;
        const int i = s0 + (act ? e : 0);
        const T yx = xs[i], yy = xs[n + i], yz = xs[2 * n + i];
        L2PAcc<T> v[3], g[9];
        for (int en = ea; en < eb; en++) {
            const int code = wx_ent[en];
            if (code & 1) continue;
            const int q = code >> 1, lq = blev[q];
            const T *ab = M + (size_t)q * 2 * P2;
            __syncthreads();  // the previous box's coefficients are no longer read
            for (int t = lane; t < TRI; t += WAVE) {
                int nn = 0;
                while ((nn + 1) * (nn + 2) / 2 <= t) nn++;
                const int m = t - nn * (nn + 1) / 2;
                // A_n^k (pot 0) or B_n^k (pot 1) = (-1)^k (stored a or b); k = -1: -conj(X^1)
                auto X = [&](int pot, int n2, int kk, T &re, T &im) {
                    if (n2 < 0 || n2 >= p || kk > n2 || (kk == -1 && n2 < 1)) {
                        re = 0;
                        im = 0;
                        return;
                    }
                    const T *c = ab + pot * P2;
                    const int ka = kk < 0 ? 1 : kk;
                    T r = c[pk_re(n2, ka)], s = ka ? c[pk_im(n2, ka)] : (T)0;
                    if (ka & 1) {
                        r = -r;
                        s = -s;
                    }
                    if (kk < 0) {
                        re = -r;
                        im = s;
                    } else {
                        re = r;
                        im = s;
                    }
                };
                T amr, ami, apr, api, a0r, a0i, bmr, bmi, bpr, bpi, b0r, b0i;
                X(0, nn - 1, m - 1, amr, ami);
                X(0, nn - 1, m + 1, apr, api);
                X(0, nn - 1, m, a0r, a0i);
                X(1, nn, m - 1, bmr, bmi);
                X(1, nn, m + 1, bpr, bpi);
                X(1, nn, m, b0r, b0i);
                const T fp = (T)(nn + m + 1), fm = (T)(nn - m + 1);
                // V_x = (A- - A+)/2 - i/2 (fp B+ + fm B-)
                Vre[t] = (T)0.5 * (amr - apr) + (T)0.5 * (fp * bpi + fm * bmi);
                Vim[t] = (T)0.5 * (ami - api) - (T)0.5 * (fp * bpr + fm * bmr);
                // V_y = -i/2 (A- + A+) + 1/2 (fp B+ - fm B-)
                Vre[TRI + t] = (T)0.5 * (ami + api) + (T)0.5 * (fp * bpr - fm * bmr);
                Vim[TRI + t] = (T)-0.5 * (amr + apr) + (T)0.5 * (fp * bpi - fm * bmi);
                // V_z = -A0 - i m B0
                Vre[2 * TRI + t] = -a0r + (T)m * b0i;
                Vim[2 * TRI + t] = -a0i - (T)m * b0r;
            }
            __syncthreads();
            double c0, c1, c2, hd;
            box_centre(bkey[q], lq, sys_geo, c0, c1, c2, hd);
            const T ihq = (T)(1.0 / hd);
            const T x = (yx - (T)c0) * ihq, y = (yy - (T)c1) * ihq, z = (yz - (T)c2) * ihq;
            const T ir2 = (T)1 / (x * x + y * y + z * z);
            L2PAcc<T> vl[3], gl[9];
            T mre = sqrt(ir2), mim = 0;  // St_m^m
            for (int m = 0; m <= p + 1; m++) {
                if (m > 0) {
                    const T f = -(T)(2 * m - 1) * ir2;
                    const T nre = f * (mre * x - mim * y), nim = f * (mre * y + mim * x);
                    mre = nre;
                    mim = nim;
                }
                const T wgt = m ? (T)2 : (T)1;
                T p1re = mre, p1im = mim, p2re = 0, p2im = 0;
                for (int nn = m; nn <= p + 1; nn++) {
                    T sre, sim;
                    if (nn == m) {
                        sre = mre;
                        sim = mim;
                    } else {
                        const T a1 = (T)(2 * nn - 1) * z * ir2, a2 = (T)((nn + m - 1) * (nn - m - 1)) * ir2;
                        sre = a1 * p1re - a2 * p2re;
                        sim = a1 * p1im - a2 * p2im;
                        p2re = p1re;
                        p2im = p1im;
                        p1re = sre;
                        p1im = sim;
                    }
                    for (int k = 0; k < 3; k++) {
                        T fr, fi;
                        if (nn <= p) {
                            vget(k, nn, m, fr, fi);
                            vl[k].add(wgt * (fr * sre - fi * sim));
                        }
                        // d_x, d_y, d_z of V_k at (nn, m) from its coefficients at nn - 1
                        T ar, ai, br, bi, cr, ci;
                        vget(k, nn - 1, m - 1, ar, ai);
                        vget(k, nn - 1, m + 1, br, bi);
                        vget(k, nn - 1, m, cr, ci);
                        const T gxr = (T)0.5 * (ar - br), gxi = (T)0.5 * (ai - bi);
                        const T gyr = (T)0.5 * (ai + bi), gyi = (T)-0.5 * (ar + br);
                        gl[3 * k + 0].add(wgt * (gxr * sre - gxi * sim));
                        gl[3 * k + 1].add(wgt * (gyr * sre - gyi * sim));
                        gl[3 * k + 2].add(wgt * (-cr * sre + ci * sim));
                    }
                }
            }
            const T ihq2 = ihq * ihq;
            for (int k = 0; k < 3; k++) v[k].add(vl[k].value() * ihq);
            for (int k = 0; k < 9; k++) g[k].add(gl[k].value() * ihq2);
        }
        if (act) {
            const T wx = ws[i], wy = ws[n + i], wz = ws[2 * n + i];
            T gg[9];
            for (int k = 0; k < 9; k++) gg[k] = g[k].value();
            for (int k = 0; k < 3; k++) {
                vfar[k * n + i] += v[k].value();
                vfar[(3 + k) * n + i] += gg[3 * k] * wx + gg[3 * k + 1] * wy + gg[3 * k + 2] * wz;
            }
            if (grad)
                for (int k = 0; k < 9; k++) vfar[(6 + k) * n + i] += gg[k];
        }
    }
}

// ---------------------------------------------------------------------------
// P2P near field + combination + un-permutation: one lane per sorted element.
// f = K/r^3, g = f'/r with the Gaussian core of eq. vem1; for u = r^2/(2a^2)
// below 0.02 the Taylor series
//   f = sqrt(2/pi)/a^3 sum_k (-u)^k/(k!(2k+3)),  g = sqrt(2/pi)/a^5 sum_{k>=1} (-1)^k u^(k-1)/((k-1)!(2k+3))
// replaces the closed form (which cancels there).
//   v += f (w_i x r),  s += f (w_i x w_j) + g (w_j . r)(w_i x r)
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void kernel_fg(T r2, T a, int smooth, T &f, T &g)
{
    // 1/a and its powers are loop-invariant (hoisted out of the pair loops): the pair costs
    // multiplications by them, not divisions; 1/r from one reciprocal square root
    if (!smooth) {
        const T ir = rsqrt(r2);
        const T ir2 = ir * ir;
        f = ir2 * ir;
        g = (T)-3 * f * ir2;
        return;
    }
    const T c = (T)0.79788456080286535588;  // sqrt(2/pi)
    const T ia = (T)1 / a;
    const T ia2 = ia * ia;
    const T u = (T)0.5 * r2 * ia2;
    // far enough out the core is 1 to working precision: 1 - K = erfc(sqrt u) + sqrt(2/pi)(r/a)e^-u
    // and the relative change of g is sqrt(2/pi) e^-u (r/a)^3 / 3; both stay below 4e-9 for
    // u >= 24 (FP32) and below 3e-18 for u >= 46 (FP64)
    if (u >= (sizeof(T) == 4 ? (T)24 : (T)46)) {
        const T ir = rsqrt(r2);
        const T ir2 = ir * ir;
        f = ir2 * ir;
        g = (T)-3 * f * ir2;
        return;
    }
    const T ia3 = ia2 * ia;
    if (u < (T)0.02) {
        // the series of K / r^3 and of its derivative term in u (coefficients folded at compile time)
        T fs = 0, gs = 0, term = 1, t2 = -1;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            fs += term * (T)(1.0 / (2 * k + 3));
            term *= -u * (T)(1.0 / (k + 1));
        }
#pragma unroll
        for (int k = 1; k < 13; k++) {
            gs += t2 * (T)(1.0 / (2 * k + 3));
            t2 *= -u * (T)(1.0 / k);
        }
        f = c * ia3 * fs;
        g = c * ia3 * ia2 * gs;
    } else {
        const T ir = rsqrt(r2);
        const T r = r2 * ir;
        const T ex = exp(-u);
        const T ria = r * ia;
        const T K = erf(ria * (T)0.70710678118654752440) - c * ria * ex;
        const T ir2 = ir * ir;
        f = K * ir2 * ir;
        g = c * ex * ia3 * ir2 - (T)3 * f * ir2;
    }
}

// one packed element record: position, strength and (slot 6) monopole strength
template <typename T>
struct Rec {
    T x, y, z, wx, wy, wz, q;
};
template <bool Q>
__device__ __forceinline__ Rec<float> load_rec(const float *__restrict__ xw, int k)
{
    const float4 a = *(const float4 *)(xw + 8 * (size_t)k);
    if constexpr (Q) {
        const float4 b = *(const float4 *)(xw + 8 * (size_t)k + 4);
        return {a.x, a.y, a.z, a.w, b.x, b.y, b.z};
    } else {
        const float2 b = *(const float2 *)(xw + 8 * (size_t)k + 4);
        return {a.x, a.y, a.z, a.w, b.x, b.y, 0.f};
    }
}
template <bool Q>
__device__ __forceinline__ Rec<double> load_rec(const double *__restrict__ xw, int k)
{
    const double2 a = *(const double2 *)(xw + 8 * (size_t)k);
    const double2 b = *(const double2 *)(xw + 8 * (size_t)k + 2);
    const double2 c = *(const double2 *)(xw + 8 * (size_t)k + 4);
    const double qv = Q ? xw[8 * (size_t)k + 6] : 0.0;
    return {a.x, a.y, b.x, b.y, c.x, c.y, qv};
}

// contribution of sorted source k to the target (xj, wj); r = x_j - x_k.  With Q the source's
// monopole strength adds q f r to v and q (f w_j + g r (w_j . r)) to s (eq. 7, same kernel)
template <typename T, bool Q>
__device__ __forceinline__ void p2p_pair(const Rec<T> &q, T xj, T yj, T zj, T wjx, T wjy, T wjz, T a, int smooth,
                                         T &v0, T &v1, T &v2, T &s0, T &s1, T &s2)
{
    const T rx = xj - q.x, ry = yj - q.y, rz = zj - q.z;
    const T r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == (T)0 && !smooth) return;  // coincident distinct points, singular kernel: no contribution
    T f, g;
    kernel_fg<T>(r2, a, smooth, f, g);
    const T wix = q.wx, wiy = q.wy, wiz = q.wz;
    const T cx = wiy * rz - wiz * ry, cy = wiz * rx - wix * rz, cz = wix * ry - wiy * rx;
    const T dd = g * (wjx * rx + wjy * ry + wjz * rz);
    v0 += f * cx;
    v1 += f * cy;
    v2 += f * cz;
    s0 += f * (wiy * wjz - wiz * wjy) + dd * cx;
    s1 += f * (wiz * wjx - wix * wjz) + dd * cy;
    s2 += f * (wix * wjy - wiy * wjx) + dd * cz;
    if constexpr (Q) {
        const T qf = q.q * f, qd = q.q * dd;
        v0 += qf * rx;
        v1 += qf * ry;
        v2 += qf * rz;
        s0 += qf * wjx + qd * rx;
        s1 += qf * wjy + qd * ry;
        s2 += qf * wjz + qd * rz;
    }
}

// the same pair with the velocity gradient: d_l (f (w_i x r))_k = g r_l (w_i x r)_k + f eps_{k a l} w_i,a
template <typename T, bool Q>
__device__ __forceinline__ void p2p_pair_grad(const Rec<T> &q, T xj, T yj, T zj, T wjx, T wjy, T wjz, T a,
                                              int smooth, T *acc)
{
    const T rx = xj - q.x, ry = yj - q.y, rz = zj - q.z;
    const T r2 = rx * rx + ry * ry + rz * rz;
    if (r2 == (T)0 && !smooth) return;
    T f, g;
    kernel_fg<T>(r2, a, smooth, f, g);
    const T wix = q.wx, wiy = q.wy, wiz = q.wz;
    const T cx = wiy * rz - wiz * ry, cy = wiz * rx - wix * rz, cz = wix * ry - wiy * rx;
    const T dd = g * (wjx * rx + wjy * ry + wjz * rz);
    acc[0] += f * cx;
    acc[1] += f * cy;
    acc[2] += f * cz;
    acc[3] += f * (wiy * wjz - wiz * wjy) + dd * cx;
    acc[4] += f * (wiz * wjx - wix * wjz) + dd * cy;
    acc[5] += f * (wix * wjy - wiy * wjx) + dd * cz;
    const T gx = g * rx, gy = g * ry, gz = g * rz;
    acc[6] += gx * cx;
    acc[7] += gy * cx - f * wiz;
    acc[8] += gz * cx + f * wiy;
    acc[9] += gx * cy + f * wiz;
    acc[10] += gy * cy;
    acc[11] += gz * cy - f * wix;
    acc[12] += gx * cz - f * wiy;
    acc[13] += gy * cz + f * wix;
    acc[14] += gz * cz;
    if constexpr (Q) {
        // q (f r, f w_j + g r (w_j . r), f delta_kl + g r_k r_l)
        const T qf = q.q * f, qd = q.q * dd, qgx = q.q * gx, qgy = q.q * gy, qgz = q.q * gz;
        acc[0] += qf * rx;
        acc[1] += qf * ry;
        acc[2] += qf * rz;
        acc[3] += qf * wjx + qd * rx;
        acc[4] += qf * wjy + qd * ry;
        acc[5] += qf * wjz + qd * rz;
        acc[6] += qgx * rx + qf;
        acc[7] += qgy * rx;
        acc[8] += qgz * rx;
        acc[9] += qgx * ry;
        acc[10] += qgy * ry + qf;
        acc[11] += qgz * ry;
        acc[12] += qgx * rz;
        acc[13] += qgy * rz;
        acc[14] += qgz * rz + qf;
    }
}

// far field + near field -> outputs in input order
template <typename T, bool GRAD>
__device__ __forceinline__ void p2p_store(int64_t i, int64_t n, const int32_t *__restrict__ perm,
                                          const CompSum<T> *acc, T *__restrict__ vout, T *__restrict__ sout,
                                          T *__restrict__ gout, T *__restrict__ bout)
{
    const int64_t o = perm[i];
    vout[3 * o] = acc[0].value();
    vout[3 * o + 1] = acc[1].value();
    vout[3 * o + 2] = acc[2].value();
    sout[3 * o] = acc[3].value();
    sout[3 * o + 1] = acc[4].value();
    sout[3 * o + 2] = acc[5].value();
    if constexpr (GRAD) {
        T b = 0;
        for (int k = 0; k < 9; k++) {
            const T gk = acc[6 + k].value();
            if (gout) gout[9 * o + k] = gk;
            b += gk * gk;
        }
        if (bout) bout[o] = b;  // beta = grad v : grad v
    }
}

// near-field sum of one target over the elements st .. st+ct-1 (self excluded), added box by
// box into compensated accumulators: v, s and, with GRAD, grad v
template <typename T, bool GRAD, bool Q>
__device__ __forceinline__ void p2p_box(int i, int st, int ct, const T *__restrict__ xw, T xj, T yj, T zj, T wjx,
                                        T wjy, T wjz, T a, int sm, CompSum<T> *acc)
{
    if constexpr (GRAD) {
        T b[15];
        for (int k = 0; k < 15; k++) b[k] = 0;
        for (int e = 0; e < ct; e++) {
            const int k = st + e;
            if (k == i) continue;
            p2p_pair_grad<T, Q>(load_rec<Q>(xw, k), xj, yj, zj, wjx, wjy, wjz, a, sm, b);
        }
        for (int k = 0; k < 15; k++) acc[k].add(b[k]);
    } else {
        T v0 = 0, v1 = 0, v2 = 0, s0 = 0, s1 = 0, s2 = 0;
        for (int e = 0; e < ct; e++) {
            const int k = st + e;
            if (k == i) continue;
            p2p_pair<T, Q>(load_rec<Q>(xw, k), xj, yj, zj, wjx, wjy, wjz, a, sm, v0, v1, v2, s0, s1, s2);
        }
        acc[0].add(v0);
        acc[1].add(v1);
        acc[2].add(v2);
        acc[3].add(s0);
        acc[4].add(s1);
        acc[5].add(s2);
    }
}

// uniform tree: one lane per sorted element over the 27 adjacent leaves (sources read from L1/L2:
// the 64 targets of a wavefront are a few leaves of one neighbourhood), then combination with the
// far field and un-permutation.  At the few elements per leaf of the uniform workloads this is
// faster than staging each leaf's sources through LDS (2^20 cube FP64: 2.0 against 2.95 ms).
template <typename T, bool GRAD, bool Q>
__global__ void __launch_bounds__(256) k_p2p(int64_t n, int depth, int64_t leaf_off, const int32_t *__restrict__ eleaf,
                                             const int32_t *__restrict__ ulist, const uint64_t *__restrict__ bkey,
                                             const int32_t *__restrict__ bstart, const int32_t *__restrict__ bcount,
                                             const T *__restrict__ xs, const T *__restrict__ ws,
                                             const T *__restrict__ xw, const double *__restrict__ sys_a, int what,
                                             const T *__restrict__ vfar,
                                             const int32_t *__restrict__ perm, T *__restrict__ vout,
                                             T *__restrict__ sout, T *__restrict__ gout, T *__restrict__ bout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // core radius of the element's system (0: singular kernel)
    const T a = (T)sys_a[bkey[eleaf[i]] >> (3 * depth)];
    const int smooth = a > (T)0;
    constexpr int NA = GRAD ? 15 : 6;
    CompSum<T> acc[NA];
    const T xj = xs[i], yj = xs[n + i], zj = xs[2 * n + i];
    const T wjx = ws[i], wjy = ws[n + i], wjz = ws[2 * n + i];
    if (what & 1)
        for (int k = 0; k < NA; k++) acc[k].add(vfar[(size_t)k * n + i]);
    if (what & 2) {
        const int lf = eleaf[i];
        const int32_t *U = ulist + (size_t)(lf - leaf_off) * 27;
        for (int q = 0; q < 27; q++) {
            const int nb = U[q];
            if (nb < 0) continue;
            p2p_box<T, GRAD, Q>((int)i, bstart[nb], bcount[nb], xw, xj, yj, zj, wjx, wjy, wjz, a, smooth, acc);
        }
    }
    p2p_store<T, GRAD>(i, n, perm, acc, vout, sout, gout, bout);
}

// adaptive tree: near field of one target leaf per 64-lane workgroup, then combination with the
// far field and un-permutation.  The leaf's source list (U-list leaves with the smoothed kernel,
// then W/X boxes with the singular one) is staged through LDS in tiles of P2P_TS element records,
// walked by the whole wavefront in list order.  Each
// target takes G = 64 / c lanes (c: targets in the chunk, at most 64), lane k of a target sums the
// tile's records k, k + G, ..; the G partial sums of a target are added in lane order at the end,
// so the result is deterministic.  Smoothed and singular sources never share a tile (uniform
// branch in the kernel).  Per tile the lane's partial sums enter compensated accumulators.
constexpr int P2P_TS = 128;

template <typename T, bool GRAD, bool Q, int TS = P2P_TS>
__global__ void __launch_bounds__(64) k_p2p_tile(int64_t n, const int32_t *__restrict__ leaves,
                                                 const int8_t *__restrict__ blev, const int32_t *__restrict__ nl_start,
                                                 const int32_t *__restrict__ nl_ent, const uint64_t *__restrict__ bkey, const int32_t *__restrict__ bstart,
                                                 const int32_t *__restrict__ bcount, const T *__restrict__ xw,
                                                 const double *__restrict__ sys_a, int what,
                                                 const T *__restrict__ vfar, const int32_t *__restrict__ perm,
                                                 T *__restrict__ vout, T *__restrict__ sout, T *__restrict__ gout,
                                                 T *__restrict__ bout)
{
    constexpr int NA = GRAD ? 15 : 6;
    __shared__ T tr[7][TS];          // x y z wx wy wz q of the staged sources
    __shared__ int tix[TS];          // their sorted indices (self exclusion)
    __shared__ T red[64 * NA];       // partial sums of the lanes
    const int lane = threadIdx.x;
    const int64_t lp = blockIdx.x;
    const int b = leaves[lp];
    const int lev = blev[b];
    const T a = (T)sys_a[bkey[b] >> (3 * lev)];
    const int smooth = a > (T)0;
    const int s0 = bstart[b], cnt = bcount[b];
    const int ea = nl_start[lp], eb = nl_start[lp + 1];
    for (int tb = 0; tb < cnt; tb += 64) {
        const int c = min(64, cnt - tb);
        const int G = 64 / c;
        const int t = lane / G, k = lane - t * G;
        const bool tact = t < c;
        const int i = s0 + tb + (tact ? t : 0);
        const Rec<T> me = load_rec<false>(xw, i);
        CompSum<T> acc[NA];
        if (what & 2) {
            for (int pass = 0; pass < 2; pass++) {
                const int sm = smooth && pass == 0;
                int e = ea, o = 0;
                while (true) {
                    // fill a tile: the wavefront walks the list together
                    int fill = 0;
                    while (fill < TS && e < eb) {
                        const int code = nl_ent[e];
                        const int src = code >> 1;
                        if ((code & 1) != pass) {
                            e++;
                            continue;
                        }
                        const int st = bstart[src], ct = bcount[src];
                        const int m = min(ct - o, TS - fill);
                        for (int u = lane; u < m; u += 64) {
                            const Rec<T> r = load_rec<Q>(xw, st + o + u);
                            tr[0][fill + u] = r.x;
                            tr[1][fill + u] = r.y;
                            tr[2][fill + u] = r.z;
                            tr[3][fill + u] = r.wx;
                            tr[4][fill + u] = r.wy;
                            tr[5][fill + u] = r.wz;
                            if (Q) tr[6][fill + u] = r.q;
                            tix[fill + u] = st + o + u;
                        }
                        fill += m;
                        o += m;
                        if (o == ct) {
                            e++;
                            o = 0;
                        }
                    }
                    if (fill == 0) break;
                    __syncthreads();
                    if (tact) {
                        T part[NA];
#pragma unroll
                        for (int q = 0; q < NA; q++) part[q] = 0;
                        for (int j = k; j < fill; j += G) {
                            if (tix[j] == i) continue;
                            const Rec<T> r{tr[0][j], tr[1][j], tr[2][j], tr[3][j], tr[4][j], tr[5][j],
                                           Q ? tr[6][j] : (T)0};
                            if constexpr (GRAD) p2p_pair_grad<T, Q>(r, me.x, me.y, me.z, me.wx, me.wy, me.wz, a, sm, part);
                            else
                                p2p_pair<T, Q>(r, me.x, me.y, me.z, me.wx, me.wy, me.wz, a, sm, part[0], part[1],
                                               part[2], part[3], part[4], part[5]);
                        }
#pragma unroll
                        for (int q = 0; q < NA; q++) acc[q].add(part[q]);
                    }
                    __syncthreads();  // the tile is overwritten next
                }
            }
        }
        // the G lanes of a target, added in lane order, then the far field
#pragma unroll
        for (int q = 0; q < NA; q++) red[lane * NA + q] = acc[q].value();
        __syncthreads();
        if (lane < c) {
            const int64_t ii = s0 + tb + lane;
            CompSum<T> tot[NA];
            if (what & 1)
                for (int q = 0; q < NA; q++) tot[q].add(vfar[(size_t)q * n + ii]);
            for (int kk = 0; kk < G; kk++)
                for (int q = 0; q < NA; q++) tot[q].add(red[(lane * G + kk) * NA + q]);
            p2p_store<T, GRAD>(ii, n, perm, tot, vout, sout, gout, bout);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Scalar harmonic FMM (the single-potential comparison workload): Phi = sum q / r and grad Phi.
// ---------------------------------------------------------------------------
// L2P of Phi and grad Phi: Phi(y) = sum (-1)^n c_n^m Rt_n^m(yhat) (bar form, no scale factor),
// grad Phi = (1/h) sum (-1)^n V Rt with the velocity coefficients of eq. evf3 at chi = 0.
// Four leaves per 64-lane workgroup as in k_l2p; rows 0 (Phi) and 1..3 (grad Phi) of vfar.
template <typename T>
__global__ void __launch_bounds__(WAVE) k_l2p_scalar(int p, int depth, int64_t nleaf, int64_t leaf_off,
                                                     const uint64_t *__restrict__ bkey,
                                                     const int32_t *__restrict__ bstart,
                                                     const int32_t *__restrict__ bcount, const T *__restrict__ xs,
                                                     int64_t n, const double *__restrict__ sys_geo,
                                                     const T *__restrict__ Lc, T *__restrict__ vfar)
{
    extern __shared__ char smem[];
    const int P2 = p * p;
    const int TRI = p * (p + 1) / 2;
    const int g = threadIdx.x / L2P_LANES, lane = threadIdx.x % L2P_LANES;
    T *Cre = (T *)smem + (size_t)g * 8 * TRI, *Cim = Cre + 4 * TRI;  // [4][TRI]: Phi, V_x, V_y, V_z
    const int64_t li = (int64_t)blockIdx.x * L2P_LPB + g;
    const bool has = li < nleaf;
    const int64_t b = has ? leaf_off + li : 0;
    const T *cd = Lc + (size_t)b * 2 * P2;
    auto get = [&](int nn, int m, T &re, T &im) {
        if (nn < 0 || nn >= p || m > nn || (m == -1 && nn < 1)) {
            re = 0;
            im = 0;
        } else if (m == -1) {
            re = -cd[pk_re(nn, 1)];
            im = cd[pk_im(nn, 1)];
        } else {
            re = cd[pk_re(nn, m)];
            im = m ? cd[pk_im(nn, m)] : (T)0;
        }
    };
    if (has)
        for (int t = lane; t < TRI; t += L2P_LANES) {
            int nn = 0;
            while ((nn + 1) * (nn + 2) / 2 <= t) nn++;
            const int m = t - nn * (nn + 1) / 2;
            T c0r, c0i, pm1r, pm1i, pp1r, pp1i, p0r, p0i;
            get(nn, m, c0r, c0i);
            get(nn + 1, m - 1, pm1r, pm1i);
            get(nn + 1, m + 1, pp1r, pp1i);
            get(nn + 1, m, p0r, p0i);
            Cre[t] = c0r;
            Cim[t] = c0i;
            Cre[TRI + t] = (T)0.5 * (-pm1r + pp1r);  // V_x = 1/2 (-P^{m-1} + P^{m+1})
            Cim[TRI + t] = (T)0.5 * (-pm1i + pp1i);
            Cre[2 * TRI + t] = (T)0.5 * (-pm1i - pp1i);  // V_y = i/2 (P^{m-1} + P^{m+1})
            Cim[2 * TRI + t] = (T)0.5 * (pm1r + pp1r);
            Cre[3 * TRI + t] = -p0r;  // V_z = -P^m
            Cim[3 * TRI + t] = -p0i;
        }
    __syncthreads();
    if (!has) return;
    const int s0 = bstart[b], cnt = bcount[b];
    double c0, c1, c2, hd;
    box_centre(bkey[b], depth, sys_geo, c0, c1, c2, hd);
    const T ih = (T)(1.0 / hd);
    for (int e0 = 0; e0 < cnt; e0 += L2P_LANES) {
        const int e = e0 + lane;
        if (e >= cnt) break;
        const int i = s0 + e;
        const T x = (xs[i] - (T)c0) * ih, y = (xs[n + i] - (T)c1) * ih, z = (xs[2 * n + i] - (T)c2) * ih;
        const T r2 = x * x + y * y + z * z;
        L2PAcc<T> f[4];
        T mre = 1, mim = 0;
        for (int m = 0; m < p; m++) {
            if (m > 0) {
                const T fm = (T)(-0.5) / (T)m;
                const T nre = fm * (mre * x - mim * y), nim = fm * (mre * y + mim * x);
                mre = nre;
                mim = nim;
            }
            T p1re = mre, p1im = mim, p2re = 0, p2im = 0;
            const T wgt = m ? (T)2 : (T)1;
            for (int nn = m; nn < p; nn++) {
                T rre, rim;
                if (nn == m) {
                    rre = mre;
                    rim = mim;
                } else if (nn == m + 1) {
                    rre = z * p1re;
                    rim = z * p1im;
                } else {
                    const T inv = (T)1 / (T)((nn - m) * (nn + m));
                    rre = ((T)(2 * nn - 1) * z * p1re - r2 * p2re) * inv;
                    rim = ((T)(2 * nn - 1) * z * p1im - r2 * p2im) * inv;
                }
                if (nn > m) {
                    p2re = p1re;
                    p2im = p1im;
                    p1re = rre;
                    p1im = rim;
                }
                const T sw = (nn & 1) ? -wgt : wgt;
                const int t = nn * (nn + 1) / 2 + m;
                for (int k = 0; k < 4; k++) f[k].add(sw * (Cre[k * TRI + t] * rre - Cim[k * TRI + t] * rim));
            }
        }
        vfar[i] = f[0].value();
        for (int k = 1; k < 4; k++) vfar[(size_t)k * n + i] = f[k].value() * ih;
    }
}

// near field of the scalar FMM on the uniform tree, lane per target over the 27 adjacent leaves
// (singular kernel), combined with the far field and written in input order
template <typename T>
__global__ void __launch_bounds__(256) k_p2p_scalar(int64_t n, int64_t leaf_off, const int32_t *__restrict__ eleaf,
                                                    const int32_t *__restrict__ ulist,
                                                    const int32_t *__restrict__ bstart,
                                                    const int32_t *__restrict__ bcount, const T *__restrict__ xw,
                                                    const T *__restrict__ vfar, const int32_t *__restrict__ perm,
                                                    T *__restrict__ phi, T *__restrict__ gphi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T xj = xw[8 * i], yj = xw[8 * i + 1], zj = xw[8 * i + 2];
    CompSum<T> acc[4];
    for (int k = 0; k < 4; k++) acc[k].add(vfar[(size_t)k * n + i]);
    const int32_t *U = ulist + (size_t)(eleaf[i] - leaf_off) * 27;
    for (int u = 0; u < 27; u++) {
        const int nb = U[u];
        if (nb < 0) continue;
        T f = 0, g0 = 0, g1 = 0, g2 = 0;
        const int st = bstart[nb], ct = bcount[nb];
        for (int k = st; k < st + ct; k++) {
            if (k == i) continue;
            const Rec<T> r = load_rec<true>(xw, k);
            const T rx = xj - r.x, ry = yj - r.y, rz = zj - r.z;
            const T r2 = rx * rx + ry * ry + rz * rz;
            if (r2 == (T)0) continue;
            const T ir = (T)1 / sqrt(r2), qir = r.q * ir, qir3 = qir * ir * ir;
            f += qir;
            g0 -= qir3 * rx;
            g1 -= qir3 * ry;
            g2 -= qir3 * rz;
        }
        acc[0].add(f);
        acc[1].add(g0);
        acc[2].add(g1);
        acc[3].add(g2);
    }
    const int64_t o = perm[i];
    phi[o] = acc[0].value();
    if (gphi)
        for (int k = 0; k < 3; k++) gphi[3 * o + k] = acc[1 + k].value();
}

// gather the source strengths into the sorted order and the near-field records (no vortex part)
template <typename T>
__global__ void k_gather_q(int64_t n, const T *__restrict__ q, const int32_t *__restrict__ perm,
                           const T *__restrict__ xs, T *__restrict__ qs, T *__restrict__ xw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T qo = q[perm[i]];
    qs[i] = qo;
    T *r = xw + 8 * i;
    r[0] = xs[i];
    r[1] = xs[n + i];
    r[2] = xs[2 * n + i];
    r[3] = r[4] = r[5] = (T)0;
    r[6] = qo;
    r[7] = (T)0;
}

// ---------------------------------------------------------------------------
// Vortex filaments: near field at the vertices.  Lane per sorted point; a vertex point sums the
// segments whose centres lie in the 27 adjacent leaves with eq. dis2 (no 1/(4 pi)):
//   v += G (r1 x r2) / (r1 r2 + r1 . r2) (1/r1 + 1/r2),  r1 = y - x1, r2 = y - x2,
// skipping the segments it is a vertex of (and any point on a segment's line); then far + near
// into the vertex's output row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_p2p_filament(int64_t n, int64_t leaf_off, const int32_t *__restrict__ eleaf,
                                                      const int32_t *__restrict__ ulist,
                                                      const int32_t *__restrict__ bstart,
                                                      const int32_t *__restrict__ bcount, const T *__restrict__ xs,
                                                      const int32_t *__restrict__ sseg,
                                                      const int32_t *__restrict__ svid, const T *__restrict__ gam,
                                                      const T *__restrict__ X, const T *__restrict__ vfar,
                                                      T *__restrict__ vout)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int vid = svid[i];
    if (vid < 0) return;  // a segment centre: not a receiver
    const T yx = X[3 * vid], yy = X[3 * vid + 1], yz = X[3 * vid + 2];
    CompSum<T> acc[3];
    for (int k = 0; k < 3; k++) acc[k].add(vfar[(size_t)k * n + i]);
    const int32_t *U = ulist + (size_t)(eleaf[i] - leaf_off) * 27;
    for (int u = 0; u < 27; u++) {
        const int nb = U[u];
        if (nb < 0) continue;
        T v0 = 0, v1 = 0, v2 = 0;
        const int st = bstart[nb], ct = bcount[nb];
        for (int k = st; k < st + ct; k++) {
            const int a = sseg[2 * k], b = sseg[2 * k + 1];
            if (a < 0 || a == vid || b == vid) continue;
            const T r1x = yx - X[3 * a], r1y = yy - X[3 * a + 1], r1z = yz - X[3 * a + 2];
            const T r2x = yx - X[3 * b], r2y = yy - X[3 * b + 1], r2z = yz - X[3 * b + 2];
            const T cx = r1y * r2z - r1z * r2y, cy = r1z * r2x - r1x * r2z, cz = r1x * r2y - r1y * r2x;
            const T ra = sqrt(r1x * r1x + r1y * r1y + r1z * r1z), rb = sqrt(r2x * r2x + r2y * r2y + r2z * r2z);
            const T den = ra * rb + r1x * r2x + r1y * r2y + r1z * r2z;
            if (ra == (T)0 || rb == (T)0 || den == (T)0 || cx * cx + cy * cy + cz * cz == (T)0) continue;
            const T f = gam[k] * ((T)1 / ra + (T)1 / rb) / den;
            v0 += f * cx;
            v1 += f * cy;
            v2 += f * cz;
        }
        acc[0].add(v0);
        acc[1].add(v1);
        acc[2].add(v2);
    }
    for (int k = 0; k < 3; k++) vout[3 * (size_t)vid + k] = acc[k].value();
}

// gather omega into the sorted SoA layout
template <typename T>
__global__ void k_gather_w(int64_t n, const T *__restrict__ w, const T *__restrict__ q,
                           const int32_t *__restrict__ perm, const T *__restrict__ xs, T *__restrict__ ws,
                           T *__restrict__ qs, T *__restrict__ xw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    const T wx = w[3 * o], wy = w[3 * o + 1], wz = w[3 * o + 2];
    ws[i] = wx;
    ws[n + i] = wy;
    ws[2 * n + i] = wz;
    // the near field reads an element as one record (two 16-byte loads in FP32, three in FP64)
    T *r = xw + 8 * i;
    r[0] = xs[i];
    r[1] = xs[n + i];
    r[2] = xs[2 * n + i];
    r[3] = wx;
    r[4] = wy;
    r[5] = wz;
    const T qo = q ? q[o] : (T)0;
    r[6] = qo;
    r[7] = (T)0;
    if (q) qs[i] = qo;
}

template <typename T, bool GRAD, bool Q>
static void p2p_launch(lhf_plan *P, int what, T *v, T *s, T *g, T *b, unsigned nblk, int tpb, hipStream_t st)
{
    const int64_t n = P->n;
    const int d = P->depth;
    if (P->adaptive) {
        if (P->nleaf == 0) return;
        // the source tile: the plan's tuned choice on the v, s path, else the built-in one
        const int ts = (!GRAD && !Q && P->p2p_ts > 0) ? P->p2p_ts : P2P_TS;
#define LHF_P2P_TILE(TSV)                                                                                       \
    hipLaunchKernelGGL((k_p2p_tile<T, GRAD, Q, TSV>), dim3((unsigned)P->nleaf), dim3(64), 0, st, n, P->leaves,     \
                       P->blev, P->nl_start, P->nl_ent, P->bkey, P->bstart, P->bcount, (const T *)P->xw,           \
                       P->sys_a, what, (const T *)P->vfar, P->perm, v, s, g, b)
        if constexpr (!GRAD && !Q) {
            if (ts == 64) LHF_P2P_TILE(64);
            else if (ts == 256) LHF_P2P_TILE(256);
            else LHF_P2P_TILE(P2P_TS);
        } else {
            LHF_P2P_TILE(P2P_TS);
        }
#undef LHF_P2P_TILE
    } else {
        hipLaunchKernelGGL((k_p2p<T, GRAD, Q>), dim3(nblk), dim3(tpb), 0, st, n, d, P->lev[d].off, P->eleaf,
                           P->ulist, P->bkey, P->bstart, P->bcount, (const T *)P->xs, (const T *)P->ws,
                           (const T *)P->xw, P->sys_a, what, (const T *)P->vfar, P->perm, v, s, g, b);
    }
}

// M2M into levels depth-1 .. 2, then per level L2L and M2L (events ev[3] after the upward pass and
// ev[7 + 2l], ev[8 + 2l] around the M2L of level l).  scalar: the expansions carry phi only (chi is
// zero and stays zero through every translation); where the half-vector kernel has a scalar
// instantiation it translates phi alone, the other kernels run on (phi, 0).
template <typename T>
static void translations(lhf_plan *P, hipStream_t st, bool scalar, const std::function<void(int)> &mark)
{
    const int p = P->p, d = P->depth;
    const int P2 = p * p, ZS = (p + 1) * (p + 1);
    T *M = (T *)P->M, *Lc = (T *)P->Lc;
    const T *rot = (const T *)P->rot, *zph = (const T *)P->zph, *coax = (const T *)P->coax;
    const bool sc_half = scalar && P->use_half && !P->use_mfma && m2l_half_scalar_supported(P->precision, p);
        size_t sh_rcr = sizeof(T) * (4 * P2 + 2 * ZS + 2 * p + 2);
    for (int l = d - 1; l >= 2; l--) {
        if (P->lev[l].nb == 0) continue;
        if (P->use_mmhalf) m2m_half_launch(P, l, st);
        else if (P->use_mmquarter) m2m_quarter_launch(P, l, st);
        else
            hipLaunchKernelGGL(k_m2m<T>, dim3((unsigned)P->lev[l].nb), dim3(WAVE), sh_rcr, st, p, P->lev[l].off,
                               P->bchild0, P->bnchild, P->bkey, M, rot, zph, P->dir_theta);
    }
    mark(3);
    for (int l = 2; l <= d; l++) {
        if (P->lev[l].nb == 0) {
            mark(7 + 2 * l);
            mark(8 + 2 * l);
            continue;
        }
        if (P->use_tile) {
            // L2L from the parents (zeros at level 2), then the batched M2L adds into it
            if (P->use_mmhalf) l2l_half_launch(P, l, st);
            else if (P->use_mmquarter) l2l_quarter_launch(P, l, st);
            else
                hipLaunchKernelGGL(k_down<T>, dim3((unsigned)P->lev[l].nb), dim3(WAVE), sh_rcr, st, p, l, 0,
                                   P->lev[l].off, P->bparent, P->bkey, P->vcount, P->vsrc, P->vdir, (const T *)M,
                                   Lc, rot, zph, P->dir_theta, coax);
            // the half-vector kernel reads its sources from a copy in its lane layout
            // (timed with L2L, outside the M2L phase)
            if (sc_half) m2l_half_scalar_stage(P, l, st);
            else if (!P->use_mfma && P->use_half) m2l_half_stage(P, l, st);
            if (P->use_quarter || P->use_qmfma) m2l_quarter_stage(P, l, st);
            mark(7 + 2 * l);
            if (P->use_mfma) m2l_mfma_launch(P, l, st);
            else if (sc_half) m2l_half_scalar_launch(P, l, st);
            else if (P->use_half) m2l_half_launch(P, l, st);
            else if (P->use_quarter) m2l_quarter_launch(P, l, st);
            else if (P->use_qmfma) m2l_qmfma_launch(P, l, st);
            else m2l_tile_launch(P, l, st);
            mark(8 + 2 * l);
        } else {
            mark(7 + 2 * l);
            hipLaunchKernelGGL(k_down<T>, dim3((unsigned)P->lev[l].nb), dim3(WAVE), sh_rcr, st, p, l, 1,
                               P->lev[l].off, P->bparent, P->bkey, P->vcount, P->vsrc, P->vdir, (const T *)M, Lc,
                               rot, zph, P->dir_theta, coax);
            mark(8 + 2 * l);
        }
    }
}

template <typename T>
static lhf_status execute_t(lhf_plan *P, const lhf_io *io, hipStream_t st)
{
    const void *omega = io->omega;
    const T *qin = (const T *)io->q;
    void *v = io->v, *s = io->s, *grad_v = io->grad_v, *beta = io->beta;
    const int what = io->what;
    const int p = P->p, d = P->depth;
    const int64_t n = P->n;
    const int P2 = p * p, ZS = (p + 1) * (p + 1);
    T *xs = (T *)P->xs, *ws = (T *)P->ws, *M = (T *)P->M, *Lc = (T *)P->Lc, *vfar = (T *)P->vfar;
    const T *rot = (const T *)P->rot, *zph = (const T *)P->zph, *coax = (const T *)P->coax;
    const int tpb = 256;
    const unsigned nblk = (unsigned)((n + tpb - 1) / tpb);
    hipEvent_t *ev = nullptr;
    if (P->prof_ev && P->prof_used < P->prof_cap) ev = P->prof_ev + (size_t)(P->prof_used++) * PROF_EV_PER_EXEC;
    // ev[0..6]: phase boundaries; ev[7 + 2l], ev[8 + 2l]: around the M2L launch of level l
    const std::function<void(int)> mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    hipLaunchKernelGGL(k_gather_w<T>, dim3(nblk), dim3(tpb), 0, st, n, (const T *)omega, qin, P->perm,
                       (const T *)xs, ws, (T *)P->qs, (T *)P->xw);
    mark(1);
    // uniform tree: the leaves are the boxes of level d; adaptive: the explicit leaf list
    const int64_t loff = P->lev[d].off, nleaf = P->adaptive ? P->nleaf : P->lev[d].nb;
    if (what & 1) {
        int nthr, ch;
        size_t sh_p2m;
        p2m_config(p, sizeof(T), nthr, ch, sh_p2m);
        hipLaunchKernelGGL(k_p2m<T>, dim3((unsigned)nleaf), dim3(nthr), sh_p2m, st, p, d, loff, P->leaves, P->blev,
                           P->bkey, P->bstart, P->bcount, (const T *)xs, (const T *)ws, qin ? (const T *)P->qs : nullptr,
                           n, P->sys_geo, M, ch);
        mark(2);
        translations<T>(P, st, false, mark);
        mark(4);
        // W/X by expansions: X sources into the leaves' local expansions before L2P, W boxes'
        // multipoles evaluated at the leaves' elements after it
        if (P->wx_exp) {
            const int SS = (p + 1) * (p + 1);
            const int chl = std::max(1, std::min(8, (int)(49152 / (sizeof(T) * (2 * SS + 4)))));
            hipLaunchKernelGGL(k_p2l<T>, dim3((unsigned)nleaf), dim3(WAVE), sizeof(T) * (size_t)chl * (2 * SS + 4), st,
                               p, P->leaves, P->blev, P->bkey, P->bstart, P->bcount, P->wx_start, P->wx_ent,
                               (const T *)xs, (const T *)ws, qin ? (const T *)P->qs : nullptr, n, P->sys_geo, Lc,
                               chl);
        }
        const int TRI = p * (p + 1) / 2;
        hipLaunchKernelGGL(k_l2p<T>, dim3((unsigned)((nleaf + L2P_LPB - 1) / L2P_LPB)), dim3(WAVE),
                           sizeof(T) * (size_t)(TRI + p + 1), st, p, d, nleaf, loff, P->leaves, P->blev, P->bkey,
                           P->bstart, P->bcount, (const T *)xs, (const T *)ws, n, P->sys_geo, (const T *)Lc, vfar,
                           (grad_v || beta) ? 1 : 0, (Cplx<T> *)P->l2pv);
        if (P->wx_exp) {
            const int TRI1 = (p + 1) * (p + 2) / 2;
            hipLaunchKernelGGL(k_m2p<T>, dim3((unsigned)nleaf), dim3(WAVE), sizeof(T) * 6 * (size_t)TRI1, st, p,
                               P->leaves, P->blev, P->bkey, P->bstart, P->bcount, P->wx_start, P->wx_ent,
                               (const T *)xs, (const T *)ws, n, P->sys_geo, (const T *)M, vfar,
                               (grad_v || beta) ? 1 : 0);
        }
    } else {
        mark(2);
        mark(3);
        for (int l = 2; l <= d; l++) {
            mark(7 + 2 * l);
            mark(8 + 2 * l);
        }
        mark(4);
    }
    mark(5);
    const bool gr = grad_v || beta;
    T *vo = (T *)v, *so = (T *)s, *go = (T *)grad_v, *bo = (T *)beta;
    if (gr && qin) p2p_launch<T, true, true>(P, what, vo, so, go, bo, nblk, tpb, st);
    else if (gr) p2p_launch<T, true, false>(P, what, vo, so, go, bo, nblk, tpb, st);
    else if (qin) p2p_launch<T, false, true>(P, what, vo, so, nullptr, nullptr, nblk, tpb, st);
    else p2p_launch<T, false, false>(P, what, vo, so, nullptr, nullptr, nblk, tpb, st);
    mark(6);
    LHF_HIP(hipGetLastError());
    return LHF_OK;
}

// scalar harmonic FMM on the plan's uniform tree: Phi and grad Phi of the sources q (singular
// kernel); gphi may be null
template <typename T>
static lhf_status execute_scalar_t(lhf_plan *P, const T *q, T *phi, T *gphi, hipStream_t st)
{
    const int p = P->p, d = P->depth;
    const int64_t n = P->n;
    const int P2 = p * p;
    T *xs = (T *)P->xs, *M = (T *)P->M, *vfar = (T *)P->vfar;
    const int tpb = 256;
    const unsigned nblk = (unsigned)((n + tpb - 1) / tpb);
    hipEvent_t *ev = nullptr;
    if (P->prof_ev && P->prof_used < P->prof_cap) ev = P->prof_ev + (size_t)(P->prof_used++) * PROF_EV_PER_EXEC;
    const std::function<void(int)> mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    hipLaunchKernelGGL(k_gather_q<T>, dim3(nblk), dim3(tpb), 0, st, n, q, P->perm, (const T *)xs, (T *)P->qs,
                       (T *)P->xw);
    mark(1);
    const int64_t loff = P->lev[d].off, nleaf = P->lev[d].nb;
    int nthr, ch;
    size_t sh_p2m;
    p2m_config(p, sizeof(T), nthr, ch, sh_p2m);
    hipLaunchKernelGGL((k_p2m<T, true>), dim3((unsigned)nleaf), dim3(nthr), sh_p2m, st,
                       p, d, loff, nullptr, nullptr, P->bkey, P->bstart, P->bcount, (const T *)xs, (const T *)P->ws,
                       (const T *)P->qs, n, P->sys_geo, M, ch);
    mark(2);
    translations<T>(P, st, true, mark);
    mark(4);
    const int TRI = p * (p + 1) / 2;
    hipLaunchKernelGGL(k_l2p_scalar<T>, dim3((unsigned)((nleaf + L2P_LPB - 1) / L2P_LPB)), dim3(WAVE),
                       sizeof(T) * L2P_LPB * 8 * TRI, st, p, d, nleaf, loff, P->bkey, P->bstart, P->bcount,
                       (const T *)xs, n, P->sys_geo, (const T *)P->Lc, vfar);
    mark(5);
    hipLaunchKernelGGL(k_p2p_scalar<T>, dim3(nblk), dim3(tpb), 0, st, n, loff, P->eleaf, P->ulist, P->bstart,
                       P->bcount, (const T *)P->xw, (const T *)vfar, P->perm, phi, gphi);
    mark(6);
    LHF_HIP(hipGetLastError());
    return LHF_OK;
}

lhf_status execute_scalar_impl(lhf_plan *P, const void *q, void *phi, void *gphi, hipStream_t st)
{
    if (P->precision == LHF_FP64)
        return execute_scalar_t<double>(P, (const double *)q, (double *)phi, (double *)gphi, st);
    return execute_scalar_t<float>(P, (const float *)q, (float *)phi, (float *)gphi, st);
}

// vortex filaments: far field of the segments (quadrature P2M) and the analytic near field at the
// vertices; omega [n][3] input order (G l at segment centres, 0 at vertices), sgam [n] the sorted
// circulations, sl / sseg / svid the sorted segment vectors, endpoints and vertex indices
template <typename T>
static lhf_status execute_filament_t(lhf_plan *P, const T *omega, const T *sgam, const T *sl, const int32_t *sseg,
                                     const int32_t *svid, const T *X, int nq, const double *quad, T *vout,
                                     hipStream_t st)
{
    const int p = P->p, d = P->depth;
    const int64_t n = P->n;
    const int P2 = p * p;
    T *xs = (T *)P->xs, *ws = (T *)P->ws, *M = (T *)P->M, *vfar = (T *)P->vfar;
    const int tpb = 256;
    const unsigned nblk = (unsigned)((n + tpb - 1) / tpb);
    hipEvent_t *ev = nullptr;
    if (P->prof_ev && P->prof_used < P->prof_cap) ev = P->prof_ev + (size_t)(P->prof_used++) * PROF_EV_PER_EXEC;
    const std::function<void(int)> mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    hipLaunchKernelGGL(k_gather_w<T>, dim3(nblk), dim3(tpb), 0, st, n, omega, (const T *)nullptr, P->perm,
                       (const T *)xs, ws, (T *)P->qs, (T *)P->xw);
    mark(1);
    const int64_t loff = P->lev[d].off, nleaf = P->lev[d].nb;
    int nthr, ch;
    size_t sh_p2m;
    p2m_config(p, sizeof(T), nthr, ch, sh_p2m);
    hipLaunchKernelGGL((k_p2m<T, false, true>), dim3((unsigned)nleaf), dim3(nthr), sh_p2m, st, p, d, loff, nullptr, nullptr, P->bkey, P->bstart,
                       P->bcount, (const T *)xs, (const T *)ws, (const T *)nullptr, n, P->sys_geo, M, ch, sl, nq,
                       quad);
    mark(2);
    translations<T>(P, st, false, mark);
    mark(4);
    const int TRI = p * (p + 1) / 2;
    hipLaunchKernelGGL(k_l2p<T>, dim3((unsigned)((nleaf + L2P_LPB - 1) / L2P_LPB)), dim3(WAVE),
                       sizeof(T) * (size_t)(TRI + p + 1), st, p, d, nleaf, loff, nullptr, nullptr, P->bkey, P->bstart,
                       P->bcount, (const T *)xs, (const T *)ws, n, P->sys_geo, (const T *)P->Lc, vfar, 0,
                       (Cplx<T> *)P->l2pv);
    mark(5);
    hipLaunchKernelGGL(k_p2p_filament<T>, dim3(nblk), dim3(tpb), 0, st, n, loff, P->eleaf, P->ulist, P->bstart,
                       P->bcount, (const T *)xs, sseg, svid, sgam, X, (const T *)vfar, vout);
    mark(6);
    LHF_HIP(hipGetLastError());
    return LHF_OK;
}

lhf_status execute_filament_impl(lhf_plan *P, const void *omega, const void *sgam, const void *sl,
                                 const int32_t *sseg, const int32_t *svid, const void *X, int nq,
                                 const double *quad, void *v, hipStream_t st)
{
    if (P->precision == LHF_FP64)
        return execute_filament_t<double>(P, (const double *)omega, (const double *)sgam, (const double *)sl, sseg,
                                          svid, (const double *)X, nq, quad, (double *)v, st);
    return execute_filament_t<float>(P, (const float *)omega, (const float *)sgam, (const float *)sl, sseg, svid,
                                     (const float *)X, nq, quad, (float *)v, st);
}

lhf_status execute_impl(lhf_plan *P, const lhf_io *io, hipStream_t st)
{
    if (P->precision == LHF_FP64) return execute_t<double>(P, io, st);
    return execute_t<float>(P, io, st);
}

// Run-time kernel shapes measured on the plan's own tree: after one whole evaluation (every
// level's multipoles in place), each level's quarter-vector M2L is launched once per candidate
// number of targets per tile, and the adaptive near field once per candidate source tile; the
// fastest of each is kept in the plan.  The timed launches leave the local expansions and the
// outputs of scratch buffers inconsistent: the next execute recomputes all of them.
template <typename T>
static lhf_status autotune_t(lhf_plan *P, const T *omega, int *ns, int *ts, hipStream_t st)
{
    const int64_t n = P->n;
    T *v = nullptr, *s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lhf_status rs = LHF_OK;
    auto fail = [&](hipError_t e, const char *what) {
        if (rs == LHF_OK) rs = hip_fail(e, what);
    };
    hipError_t e = dev_malloc(&v, sizeof(T) * 3 * (size_t)n);
    if (e == hipSuccess) e = dev_malloc(&s, sizeof(T) * 3 * (size_t)n);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) fail(e, "autotune buffers");
    if (rs == LHF_OK) {
        lhf_io io;
        memset(&io, 0, sizeof(io));
        io.omega = omega;
        io.v = v;
        io.s = s;
        io.what = 3;
        rs = execute_t<T>(P, &io, st);
    }
    auto timed = [&](const std::function<void()> &launch) -> float {
        float ms = -1.0f;
        if (rs != LHF_OK) return ms;
        hipError_t r = hipEventRecord(e0, st);
        launch();
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (r != hipSuccess) fail(r, "autotune timing");
        return ms;
    };
    for (int l = 0; l <= MAXDEPTH; l++) ns[l] = 0;
    const int maxns = P->use_quarter ? m2l_quarter_max_ns(P->p) : P->use_qmfma ? m2l_qmfma_max_ns(P->p) : 0;
    for (int l = 2; l <= P->depth && maxns > 0 && rs == LHF_OK; l++) {
        if (P->lev[l].nb == 0) continue;
        m2l_quarter_stage(P, l, st);
        int best = 0;
        float tbest = 0;
        for (int c : {1, 2, 3, 4, 6, 8, 10, 12, 16}) {
            if (c > maxns) break;
            P->m2l_ns[l] = c;
            const float t = timed([&] {
                if (P->use_qmfma) m2l_qmfma_launch(P, l, st);
                else m2l_quarter_launch(P, l, st);
            });
            if (t >= 0 && (best == 0 || t < tbest)) {
                best = c;
                tbest = t;
            }
        }
        P->m2l_ns[l] = ns[l] = best;
    }
    *ts = 0;
    if (P->adaptive && P->nleaf > 0 && rs == LHF_OK) {
        int best = 0;
        float tbest = 0;
        for (int c : {64, 128, 256}) {
            P->p2p_ts = c;
            const float t = timed([&] { p2p_launch<T, false, false>(P, 2, v, s, nullptr, nullptr, 0, 0, st); });
            if (t >= 0 && (best == 0 || t < tbest)) {
                best = c;
                tbest = t;
            }
        }
        P->p2p_ts = *ts = best;
    }
    if (rs == LHF_OK) {
        hipError_t r = hipGetLastError();
        if (r == hipSuccess) r = hipStreamSynchronize(st);
        if (r != hipSuccess) fail(r, "autotune launches");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (v) (void)dev_free(v);
    if (s) (void)dev_free(s);
    return rs;
}

lhf_status autotune_impl(lhf_plan *P, const void *omega, int *ns, int *ts, hipStream_t st)
{
    if (P->precision == LHF_FP64) return autotune_t<double>(P, (const double *)omega, ns, ts, st);
    return autotune_t<float>(P, (const float *)omega, ns, ts, st);
}

}  // namespace lhf

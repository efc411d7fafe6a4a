// lhf_filament.hip -- vortex filaments (Sec. 5.3, App. B): closed or open polygonal filaments of
// straight segments with constant circulation, the velocity evaluated at the vertices.
//
// The plan's octree is built over the segment centres (the sources) and the vertices (the
// receivers), one point each.  A segment enters the far field through the multipole of its
// Gauss-Legendre points (eqs. vf5, vf6) with nq = floor((p - 1)/2) + 1 points (eq. vf7), the
// near field through the closed form of eq. dis2; both without the factor 1/(4 pi), as the
// particle path (v = sum omega x r / r^3), so that a short segment acts as the point vortex of
// strength G l at its centre.  The translations, L2P and the tree are the particle path's.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "lhf_internal.h"

struct lhf_filament {
    lhf_plan *plan = nullptr;
    int64_t nv = 0, ns = 0, n = 0;
    int precision = LHF_FP64;
    void *X = nullptr;        // vertices [nv][3] (copy)
    int32_t *seg = nullptr;   // segments [ns][2] vertex indices (copy)
    void *pts = nullptr;      // plan points [n][3]: segment centres, then vertices
    void *omega = nullptr;    // [n][3] per execute: G l at the centres, 0 at the vertices
    void *sl = nullptr;       // segment vectors in the plan's sorted order [3][n] (0 at vertices)
    void *sgam = nullptr;     // circulations in sorted order [n] (0 at vertices)
    int32_t *sseg = nullptr;  // endpoints in sorted order [n][2] (-1 at vertices)
    int32_t *svid = nullptr;  // vertex index of a sorted point (-1 at segment centres)
    double *quad = nullptr;   // [nq][2]: Gauss-Legendre abscissa, weight
    int nq = 1;
};

namespace lhf {
namespace {

// Gauss-Legendre rule on [-1, 1]: the roots of P_nq by Newton's iteration from the asymptotic
// guesses cos(pi (k - 1/4) / (nq + 1/2)), weights 2 / ((1 - x^2) P_nq'(x)^2)
void gauss_legendre(int nq, double *xi, double *w)
{
    for (int k = 1; k <= nq; k++) {
        double x = std::cos(M_PI * (k - 0.25) / (nq + 0.5));
        double dpn = 1.0;
        for (int it = 0; it < 60; it++) {
            // P_nq(x) and P_{nq-1}(x) by the three-term recurrence
            double pm = 0.0, pn = 1.0;
            for (int j = 1; j <= nq; j++) {
                const double pp = ((2 * j - 1) * x * pn - (j - 1) * pm) / j;
                pm = pn;
                pn = pp;
            }
            dpn = nq * (pm - x * pn) / (1.0 - x * x);
            const double step = pn / dpn;
            x -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(x) + 1e-300) break;
        }
        double pm = 0.0, pn = 1.0;
        for (int j = 1; j <= nq; j++) {
            const double pp = ((2 * j - 1) * x * pn - (j - 1) * pm) / j;
            pm = pn;
            pn = pp;
        }
        dpn = nq * (pm - x * pn) / (1.0 - x * x);
        xi[k - 1] = x;
        w[k - 1] = 2.0 / ((1.0 - x * x) * dpn * dpn);
    }
}

template <typename T>
__global__ void k_fil_points(int64_t ns, int64_t nv, const T *__restrict__ X, const int32_t *__restrict__ seg,
                             T *__restrict__ pts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns + nv) return;
    for (int d = 0; d < 3; d++)
        pts[3 * i + d] = i < ns ? (T)0.5 * (X[3 * seg[2 * i] + d] + X[3 * seg[2 * i + 1] + d]) : X[3 * (i - ns) + d];
}

// sorted-order segment data from the plan's permutation (sorted position -> input point)
template <typename T>
__global__ void k_fil_sorted(int64_t n, int64_t ns, const int32_t *__restrict__ perm, const T *__restrict__ X,
                             const int32_t *__restrict__ seg, T *__restrict__ sl, int32_t *__restrict__ sseg,
                             int32_t *__restrict__ svid)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm[i];
    if (o < ns) {
        const int a = seg[2 * o], b = seg[2 * o + 1];
        for (int d = 0; d < 3; d++) sl[(size_t)d * n + i] = X[3 * b + d] - X[3 * a + d];
        sseg[2 * i] = a;
        sseg[2 * i + 1] = b;
        svid[i] = -1;
    } else {
        for (int d = 0; d < 3; d++) sl[(size_t)d * n + i] = (T)0;
        sseg[2 * i] = sseg[2 * i + 1] = -1;
        svid[i] = (int32_t)(o - ns);
    }
}

// per execute: omega = G l at the centres (input order), the sorted circulations
template <typename T>
__global__ void k_fil_omega(int64_t n, int64_t ns, const int32_t *__restrict__ perm, const T *__restrict__ X,
                            const int32_t *__restrict__ seg, const T *__restrict__ G, T *__restrict__ omega,
                            T *__restrict__ sgam)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i < ns) {
        const int a = seg[2 * i], b = seg[2 * i + 1];
        for (int d = 0; d < 3; d++) omega[3 * i + d] = G[i] * (X[3 * b + d] - X[3 * a + d]);
    } else {
        for (int d = 0; d < 3; d++) omega[3 * i + d] = (T)0;
    }
    const int64_t o = perm[i];
    sgam[i] = o < ns ? G[o] : (T)0;
}

void fil_free(lhf_filament *F)
{
    if (!F) return;
    (void)hipDeviceSynchronize();
    if (F->plan) lhf_plan_destroy(F->plan);
    for (void *b : {F->X, (void *)F->seg, F->pts, F->omega, F->sl, F->sgam, (void *)F->sseg, (void *)F->svid,
                    (void *)F->quad})
        if (b) (void)dev_free(b);
    delete F;
}

template <typename T>
lhf_status fil_create_t(lhf_filament *F, const lhf_desc *d, const void *X, const int32_t *seg, hipStream_t st)
{
    const int64_t n = F->n, nv = F->nv, ns = F->ns;
    const unsigned nb = (unsigned)((n + 255) / 256);
    LHF_HIP(dev_malloc(&F->X, sizeof(T) * 3 * nv));
    LHF_HIP(dev_malloc(&F->seg, sizeof(int32_t) * 2 * ns));
    LHF_HIP(dev_malloc(&F->pts, sizeof(T) * 3 * n));
    LHF_HIP(dev_malloc(&F->omega, sizeof(T) * 3 * n));
    LHF_HIP(dev_malloc(&F->sl, sizeof(T) * 3 * n));
    LHF_HIP(dev_malloc(&F->sgam, sizeof(T) * n));
    LHF_HIP(dev_malloc(&F->sseg, sizeof(int32_t) * 2 * n));
    LHF_HIP(dev_malloc(&F->svid, sizeof(int32_t) * n));
    LHF_HIP(hipMemcpyAsync(F->X, X, sizeof(T) * 3 * nv, hipMemcpyDeviceToDevice, st));
    LHF_HIP(hipMemcpyAsync(F->seg, seg, sizeof(int32_t) * 2 * ns, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fil_points<T>, dim3(nb), dim3(256), 0, st, ns, nv, (const T *)F->X, F->seg, (T *)F->pts);
    LHF_HIP(hipGetLastError());
    lhf_status s = lhf_plan_create(&F->plan, d, n, F->pts, 0.0, st);
    if (s < 0) return s;
    hipLaunchKernelGGL(k_fil_sorted<T>, dim3(nb), dim3(256), 0, st, n, ns, F->plan->perm, (const T *)F->X, F->seg,
                       (T *)F->sl, F->sseg, F->svid);
    LHF_HIP(hipGetLastError());
    // quadrature of eq. vf7
    F->nq = (F->plan->p - 1) / 2 + 1;
    std::vector<double> xi(F->nq), w(F->nq), q(2 * F->nq);
    gauss_legendre(F->nq, xi.data(), w.data());
    for (int k = 0; k < F->nq; k++) {
        q[2 * k] = xi[k];
        q[2 * k + 1] = w[k];
    }
    LHF_HIP(dev_malloc(&F->quad, sizeof(double) * 2 * F->nq));
    LHF_HIP(hipMemcpyAsync(F->quad, q.data(), sizeof(double) * 2 * F->nq, hipMemcpyHostToDevice, st));
    LHF_HIP(hipStreamSynchronize(st));
    return s;
}

}  // namespace
}  // namespace lhf

using namespace lhf;

lhf_status lhf_filament_create(lhf_filament **out, const lhf_desc *d, int64_t nv, const void *X, int64_t ns,
                               const int32_t *seg, void *stream)
{
    if (!out) return arg_error("out is NULL");
    *out = nullptr;
    if (!d || !X || !seg) return arg_error("d, X and seg must be non-NULL");
    if (nv < 2 || ns < 1) return arg_error("need nv >= 2 vertices and ns >= 1 segments");
    if (nv + ns > ((int64_t)1 << 30)) return arg_error("nv + ns exceeds 2^30");
    if (d->max_per_leaf != 0) {
        set_error("vortex filaments run on uniform trees only (max_per_leaf = 0)");
        return LHF_ERR_UNSUPPORTED;
    }
    if (d->precision != LHF_FP64 && d->precision != LHF_FP32) return arg_error("unknown precision");
    hipStream_t st = (hipStream_t)stream;
    // segment indices are checked on the host before any kernel reads vertices through them
    std::vector<int32_t> hs(2 * (size_t)ns);
    hipError_t e = hipMemcpy(hs.data(), seg, sizeof(int32_t) * 2 * ns, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(seg)");
    for (int64_t i = 0; i < 2 * ns; i++)
        if (hs[i] < 0 || hs[i] >= nv) return arg_error("segment vertex index out of range");
    for (int64_t i = 0; i < ns; i++)
        if (hs[2 * i] == hs[2 * i + 1]) return arg_error("segment with coincident end indices");
    lhf_filament *F = new lhf_filament();
    F->nv = nv;
    F->ns = ns;
    F->n = nv + ns;
    F->precision = d->precision;
    lhf_status s = d->precision == LHF_FP64 ? fil_create_t<double>(F, d, X, seg, st) : fil_create_t<float>(F, d, X, seg, st);
    if (s < 0) {
        fil_free(F);
        return s;
    }
    *out = F;
    return s;
}

lhf_status lhf_filament_execute(lhf_filament *F, const void *G, void *v, void *stream)
{
    if (!F) return arg_error("filament is NULL");
    if (!G || !v) return arg_error("G and v must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    const unsigned nb = (unsigned)((F->n + 255) / 256);
    if (F->precision == LHF_FP64)
        hipLaunchKernelGGL(k_fil_omega<double>, dim3(nb), dim3(256), 0, st, F->n, F->ns, F->plan->perm,
                           (const double *)F->X, F->seg, (const double *)G, (double *)F->omega, (double *)F->sgam);
    else
        hipLaunchKernelGGL(k_fil_omega<float>, dim3(nb), dim3(256), 0, st, F->n, F->ns, F->plan->perm,
                           (const float *)F->X, F->seg, (const float *)G, (float *)F->omega, (float *)F->sgam);
    LHF_HIP(hipGetLastError());
    F->plan->stream = st;
    return execute_filament_impl(F->plan, F->omega, F->sgam, F->sl, F->sseg, F->svid, F->X, F->nq, F->quad, v, st);
}

lhf_plan *lhf_filament_plan(lhf_filament *F) { return F ? F->plan : nullptr; }

lhf_status lhf_filament_destroy(lhf_filament *F)
{
    fil_free(F);
    return LHF_OK;
}

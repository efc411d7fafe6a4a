// lhf_internal.h -- internal definitions of liblhfmm (HIP, gfx950).
//
// Coefficient representation used by every device kernel ("scaled bar form"):
// for a box of side h and a real harmonic function with coefficients c_n^m of
// the paper's basis (eq. rsbf2), only m >= 0 is stored (c_n^{-m} =
// (-1)^m conj(c_n^m) for real functions) and the stored value is i^m c_n^m,
// scaled per order so that values stay O(1) for every level and fit FP32:
//   multipole (S basis):  a = i^m phi_n^m / h^(n+1),   b = i^m chi_n^m / h^n
//   local     (R basis):  c = i^m phi_n^m * h^n,        d = i^m chi_n^m * h^(n+1)
// With the i^m factor, rotations about the y axis have REAL matrices and act on
// the real parts and the imaginary parts separately.  Packed layout of one
// potential: the block of order n starts at n*n and holds
//   [Re m=0, Re m=1, .., Re m=n, Im m=1, .., Im m=n]   (2n+1 reals),
// p^2 reals per potential, two potentials (phi, chi) per box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lhfmm.h"

namespace lhf {

constexpr int QBITS = 21;
constexpr int MAXP = 24;
constexpr int MAXDEPTH = 10;
constexpr int NDIR_M2L = 343;    // codes (dx+3) + 7 (dy+3) + 49 (dz+3), dx..dz in [-3,3]
constexpr int NDIR = NDIR_M2L + 16;  // + 8 child->parent and 8 parent->child directions
constexpr int VMAX = 189;        // interaction-list bound per box (6^3 - 3^3)
constexpr int PROF_EV_PER_EXEC = 7 + 2 * (MAXDEPTH + 1);  // phase marks + a pair per level

// packed index of (n, m) real part / imaginary part (m >= 1)
__host__ __device__ inline int pk_re(int n, int m) { return n * n + m; }
__host__ __device__ inline int pk_im(int n, int m) { return n * n + n + m; }

// size of one rotation-matrix set (all orders n < p, Re and Im blocks)
__host__ __device__ inline int rot_set_size(int p) { return p * (2 * p * p + 1) / 3; }
// offset of order n's blocks inside a set
__host__ __device__ inline int rot_block_off(int n) { return n * (2 * n * n + 1) / 3; }

// rotation kinds stored per polar-angle class
enum RotKind { ROT_S_FWD = 0, ROT_R_FWD = 1, ROT_S_BACK = 2, ROT_R_BACK = 3, ROT_NKIND = 4 };

struct TreeLevel {
    int64_t nb = 0;         // non-empty boxes at this level
    int64_t off = 0;        // global box index of the first box of the level
};

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace lhf

// The plan (opaque to callers).
struct lhf_plan {
    lhf_desc desc;
    int64_t n = 0;
    int p = 0, depth = 0;
    int precision = 0;      // LHF_FP64 / LHF_FP32
    size_t tsize = 8;       // bytes per real
    hipStream_t stream = nullptr;

    // independent systems sharing the plan: system s owns input elements
    // sys_off[s] .. sys_off[s+1]-1, has its own cube and core radius, and its
    // index is prefixed to every Morton key (so no list crosses systems)
    int nsys = 1;
    std::vector<int64_t> h_sys_off;   // [nsys + 1]
    std::vector<double> h_sys_geo;    // [nsys][4]: lo0, lo1, lo2, L
    std::vector<double> h_sys_a;      // [nsys]: core radius (0: singular)
    double *sys_geo = nullptr;        // device copies
    double *sys_a = nullptr;
    int64_t *sys_off = nullptr;

    lhf::TreeLevel lev[lhf::MAXDEPTH + 1];
    int64_t nbox = 0;       // all levels
    int64_t n_m2l = 0, n_p2p = 0;
    int n_theta = 0;

    // device buffers
    int32_t *perm = nullptr;     // sorted position -> input index
    void *xs = nullptr;          // sorted coordinates, SoA [3][n], T
    void *ws = nullptr;          // sorted strengths, SoA [3][n], T (filled by execute)
    void *qs = nullptr;          // sorted monopole strengths [n], T (filled by an execute given q)
    void *vfar = nullptr;        // far-field v, s (+ grad v) in sorted order, SoA [6 or 15][n], T
    void *xw = nullptr;          // sorted elements packed for the near field: [n][8] T = x y z wx wy wz - -
    uint64_t *bkey = nullptr;    // [nbox] Morton key of every box (level-local)
    int32_t *bstart = nullptr;   // [nbox] first sorted element
    int32_t *bcount = nullptr;   // [nbox] number of elements
    int32_t *bparent = nullptr;  // [nbox] global index of the parent (-1 at level 0)
    int32_t *bchild0 = nullptr;  // [nbox] global index of the first child (-1 if leaf)
    int32_t *bnchild = nullptr;  // [nbox] number of children
    int32_t *vcount = nullptr;   // [nbox] V-list length
    int32_t *vsrc = nullptr;     // [nbox][189] V-list source boxes (global index)
    int16_t *vdir = nullptr;     // [nbox][189] direction code of t = c_target - c_source
    int32_t *ulist = nullptr;    // [nleaf][27] adjacent leaves (global index, -1 = none); uniform tree
    int32_t *eleaf = nullptr;    // [n] leaf of each sorted element: global box index (uniform tree)
                                 //     or position in 'leaves' (adaptive tree)

    // adaptive tree (boxes split while they hold more than max_per_leaf elements, down to
    // level 'depth'): leaves on several levels, per-leaf near-field source lists
    bool adaptive = false;
    int max_per_leaf = 0;
    int max_level = 0;           // deepest level holding a box
    int64_t nleaf = 0;
    int64_t n_wx = 0;            // element pairs summed directly for W/X interactions
    int8_t *blev = nullptr;      // [nbox] level of every box
    int32_t *leaves = nullptr;   // [nleaf] leaf boxes in element (Morton) order
    int32_t *nl_start = nullptr; // [nleaf + 1] source-list offsets per leaf
    int32_t *nl_ent = nullptr;   // source entries (box << 1) | singular
    // W/X by expansions (LHF_WX_EXPANSIONS): per-leaf lists of W boxes (M2P) and X sources (P2L)
    bool wx_exp = false;
    int32_t *wx_start = nullptr; // [nleaf + 1] offsets
    int32_t *wx_ent = nullptr;   // entries (box << 1) | is_x
    int64_t n_m2p = 0, n_p2l = 0;
    void *M = nullptr;           // multipoles [nbox][2][p^2], T
    void *Lc = nullptr;          // locals     [nbox][2][p^2], T
    void *l2pv = nullptr;        // L2P velocity coefficients [nleaf][3][p(p+1)/2] complex, T
    void *rot = nullptr;         // rotation sets [n_theta][4][rot_set_size(p)], T
    void *zph = nullptr;         // z phases [NDIR][2][p] (cos m phi, sin m phi), T
    int16_t *dir_theta = nullptr;   // [NDIR] polar-angle class of every direction
    void *coax = nullptr;        // M2L coaxial Hankel vectors [28][2p+2], T, indexed by |d|^2
    int32_t *dflag = nullptr;    // device status flags
    double *dtmp = nullptr;

    // batched M2L: dense box map per level (levels <= 8) and the static
    // translation schedule of one sibling group sorted by polar-angle class
    int32_t *dmap[lhf::MAXDEPTH + 1] = {nullptr};
    int16_t *sched_cls_start = nullptr;  // [ncls + 1]
    int16_t *sched_c = nullptr;          // [1512] child position of the target
    int16_t *sched_dir = nullptr;        // [1512] direction code
    int16_t *sched_cls_theta = nullptr;  // [ncls] rotation-table class
    int16_t *sched_row_start = nullptr;  // [ncls + 1] first row of each class in sched_rows
    int16_t *sched_rows = nullptr;       // [nrows][8] direction codes by child position (-1: hole)
    int sched_ncls = 0;
    bool use_tile = false;
    void *wpad = nullptr;                // padded per-class rotation blocks (tiled M2L layout)
    bool use_mfma = false;               // matrix-core M2L (same schedule and box maps)
    bool use_half = false;               // VALU M2L with each vector split over two lanes (large p)
    bool use_quarter = false;            // VALU M2L with each vector split over four lanes (FP64, high p)
    bool use_qmfma = false;              // matrix-core M2L in the same residue layout (FP64, high p)
    void *whalf = nullptr;               // its rotation tables
    int16_t *qsched = nullptr;           // quarter-vector M2L: [3][ncls] class order, staged table, mirrored
    std::vector<double> h_theta;         // host copies: polar angle of every rotation-table class
    std::vector<int16_t> h_cls_theta;    //   and the table class of every schedule class
    std::vector<int16_t> h_qsched;       //   and of qsched (kept until the plan is destroyed)
    void *mh = nullptr;                  // its sources, one level at a time, in its lane layout
    double *dtab = nullptr;              // its per-direction |t|, 1/|t|, e^{i phi} ([343][4])
    bool use_mmhalf = false;             // batched M2M and L2L in the same layout
    bool use_mmquarter = false;          // batched M2M and L2L, four lanes per part vector (FP64 p = 20-24)
    int m2l_ns[lhf::MAXDEPTH + 1] = {};  // targets per tile of the quarter-vector M2L per level (0: built-in)
    int p2p_ts = 0;                      // sources per LDS tile of the adaptive near field (0: built-in)
    void *wmm = nullptr, *wll = nullptr; // their rotation tables (S basis, R basis)
    bool tile2 = false;                  // VALU tile with two schedule rows per batch (FP32 p = 8, 10)
    void *wmfma = nullptr;               // per-class rotation blocks in MFMA A-operand lane order

    // kernel choice (resolved from the descriptor) and order selection
    int m2l_kind = LHF_M2L_GENERIC;      // LHF_M2L_HALF / TILE / TILE1 / MFMA / GENERIC
    int mm_kind = LHF_MM_GENERIC;        // LHF_MM_HALF / GENERIC
    bool deterministic = true;           // every kernel accumulates in a fixed order
    bool p_from_tol = false;             // p chosen from tol by the calibration table
    double calib_err_v = 0, calib_err_s = 0;
    bool out_grad = false;               // vfar holds grad v too ([15][n] instead of [6][n])
    int warnings = 0;                    // 1: core split above tol, 2: tol not reachable

    // phase profiling: events[k][0..LHF_NPHASE] for the k-th profiled execute
    hipEvent_t *prof_ev = nullptr;
    int prof_cap = 0, prof_used = 0;
};

namespace lhf {
void set_error(const std::string &msg);
lhf_status hip_fail(hipError_t e, const char *what);
lhf_status arg_error(const std::string &msg);
// checked construction of a plan over nsys systems (host offsets, cubes and core radii)
lhf_status plan_new(lhf_plan **out, const lhf_desc *d, int nsys, const int64_t *off, const void *x,
                    const double *lo, const double *len, const double *a, hipStream_t stream);
void plan_free(lhf_plan *P);

// Device memory of plans and their temporaries.  Freed blocks are kept per (device, rounded
// size) and handed to the next request of that size (a plan rebuilt every step allocates the
// same sizes); LHF_NO_MEMCACHE=1 calls hipMalloc/hipFree directly.  A block may be freed only
// once no queued work uses it (plan destruction synchronizes the device first).
hipError_t dev_malloc_raw(void **p, size_t bytes);
hipError_t dev_free(void *p);
template <typename T>
inline hipError_t dev_malloc(T **p, size_t bytes)
{
    return dev_malloc_raw((void **)p, bytes);
}
lhf_status execute_impl(lhf_plan *P, const lhf_io *io, hipStream_t st);
lhf_status execute_scalar_impl(lhf_plan *P, const void *q, void *phi, void *gphi, hipStream_t st);
lhf_status execute_filament_impl(lhf_plan *P, const void *omega, const void *sgam, const void *sl,
                                 const int32_t *sseg, const int32_t *svid, const void *X, int nq,
                                 const double *quad, void *v, hipStream_t st);
// order from tolerance and kernel choice (host only)
bool choose_order(bool adaptive, int precision, double tol, int *p);
void calib_error(bool adaptive, int p, double *ev, double *es);
bool kernel_deterministic(int precision, int p, int m2l_kind);
lhf_status resolve_kernels(const lhf_desc *d, int p, bool dmap_ok, int *m2l, int *mm);
}  // namespace lhf

#define LHF_HIP(call)                                                  \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return lhf::hip_fail(_e, #call);         \
    } while (0)

// lhf_m2l_common.h -- device helpers shared by the VALU M2L kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lhf {

__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }

// factorials as compile-time constants
__device__ constexpr double dfact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= (double)i;
    return f;
}

// lane permutations within groups of four by DPP (VALU, no LDS traffic)
template <int CTRL>
__device__ inline float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_f(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_XOR3 = 0x1B;  // quad_perm [3,2,1,0]

// lane exchange within groups of 32 by ds_swizzle in bit-mask mode (and 0x1F, or 0, xor X)
template <int X>
__device__ inline float swz_xor(float v)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (X << 10)));
}
template <int X>
__device__ inline double swz_xor(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), 0x1F | (X << 10));
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x1F | (X << 10));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct M2LSched {
    // static schedule of one sibling group, sorted by polar-angle class
    const int16_t *cls_start;  // [ncls+1]
    const int16_t *ent_c;      // [1512] child position of the target
    const int16_t *ent_dir;    // [1512] direction code of t = c_T - c_S
    int ncls;
    // the same entries as rows of 8 (column = child position, -1 = hole)
    const int16_t *row_start;  // [ncls+1] first row of each class
    const int16_t *rows;       // [nrows][8] direction codes
};

}  // namespace lhf

// Lattice stencil of the kernel translation units.  Each of them is built
// once per lattice, with MDLBM_Q = 19 (D3Q19) or 15 (D3Q15, the lattice of
// the paper's Sec. 2.2), and defines its launchers in namespace mdlbm::q19 or
// mdlbm::q15; the API picks one set by lbm_config.lattice.  Both numberings
// put the rest velocity first, then the axis velocities, and give the
// opposite of an odd direction i as i + 1.
#pragma once

#ifndef MDLBM_Q
#define MDLBM_Q 19
#endif

#if MDLBM_Q == 19
#define MDLBM_QNS q19
#elif MDLBM_Q == 15
#define MDLBM_QNS q15
#else
#error "MDLBM_Q must be 19 or 15"
#endif

namespace mdlbm {

constexpr int kQ = MDLBM_Q;

#if MDLBM_Q == 19
// D3Q19: 0 rest; 1-6 axes; 7-18 face diagonals.
__host__ __device__ constexpr int cx(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i)
{
    return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i)
{
    return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr double wgt(int i)
{
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr float wgtf(int i)
{
    return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
#else
// D3Q15: 0 rest; 1-6 axes; 7-14 cube diagonals (1,1,1), (-1,-1,-1),
// (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1), (1,-1,-1).
__host__ __device__ constexpr int cx(int i)
{
    return (i == 1 || i == 7 || i == 9 || i == 11 || i == 14) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 13) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i)
{
    return (i == 3 || i == 7 || i == 9 || i == 12 || i == 13) ? 1
         : (i == 4 || i == 8 || i == 10 || i == 11 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i)
{
    return (i == 5 || i == 7 || i == 10 || i == 11 || i == 13) ? 1
         : (i == 6 || i == 8 || i == 9 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr double wgt(int i)
{
    return i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0);
}
__host__ __device__ constexpr float wgtf(int i)
{
    return i == 0 ? 2.0f / 9.0f : (i <= 6 ? 1.0f / 9.0f : 1.0f / 72.0f);
}
#endif
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Largest |e_i| of the lattice, rounded up in FP32: sqrt 2 (D3Q19), sqrt 3 (D3Q15).
constexpr float kMaxSpeedUp = (MDLBM_Q == 19) ? 1.4143f : 1.7321f;

}  // namespace mdlbm

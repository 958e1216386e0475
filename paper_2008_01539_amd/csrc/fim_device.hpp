// Device helpers: deterministic wave and block reductions, and the
// XCD-aware workgroup-to-tile map.
#pragma once

#include "fim_internal.hpp"

namespace fimk {

// One DPP move of a double (both halves with the same control); lanes
// that the row mask leaves out, or whose source is out of range, read 0.
template <int CTRL, int ROWS = 0xf>
__device__ inline double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, true),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, true));
}

// Sum over the wave, returned in every lane; fixed order (deterministic).
// Cross-lane steps are DPP register moves (no LDS round trips): swaps of
// neighbours and pairs inside each quad, mirrors inside each half-row and
// row (every lane then holds its 16-lane row sum), then rows 0+1 and 2+3
// (row broadcast of lane 15) and all four (row broadcast of lane 31) into
// row 3; lane 63 holds the total.
__device__ inline double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);         // row_half_mirror
    v += dpp_f64<0x140>(v);         // row_mirror
    v += dpp_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                            __builtin_amdgcn_readlane(__double2loint(v), 63));
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

__device__ inline int wave_max_i(int v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Sum of K values over the block (blockDim.x a multiple of 64, <= 1024);
// fixed butterfly + fixed wave order: deterministic for a given shape.
template <int K>
__device__ inline void block_sum(double (&v)[K]) {
    __shared__ double sh[K][1024 / WAVE];
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const int nw = blockDim.x / WAVE;
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) sh[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        double r = 0.0;
        for (int q = 0; q < nw; q++) r += sh[k][q];
        v[k] = r;
    }
}

template <int K>
__device__ inline void block_max(double (&v)[K]) {
    __shared__ double sh[K][1024 / WAVE];
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const int nw = blockDim.x / WAVE;
#pragma unroll
    for (int k = 0; k < K; k++) v[k] = wave_max(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < K; k++) sh[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        double r = sh[k][0];
        for (int q = 1; q < nw; q++) r = fmax(r, sh[k][q]);
        v[k] = r;
    }
}

__device__ inline int block_sum_i(int v) {
    __shared__ int sh[1024 / WAVE];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    int r = 0;
    for (int q = 0; q < (int)(blockDim.x / WAVE); q++) r += sh[q];
    return r;
}

__host__ __device__ inline int nblocks(long n, int nt = NT) { return (int)((n + nt - 1) / nt); }

// The dispatcher hands workgroups to the XCDs round robin (workgroup g to
// XCD g mod 8), and each XCD has its own L2.  For a segment of nbk
// workgroups starting at g0, xcd_tile maps workgroup g to a tile index in
// [0, nbk) such that the workgroups of one XCD take consecutive tiles:
// each XCD then works on one contiguous range of rows, and the neighbour
// rows its gathers touch mostly sit in its own L2.  A bijection for any
// g0 and nbk; tile t covers the same rows whichever workgroup runs it.
constexpr int N_XCD = 8;
__host__ __device__ inline int xcd_tile(int g0, int nbk, int g) {
    const int off = g0 % N_XCD;          // XCD slot of the first workgroup
    const int q = g - g0 + off;          // position from an aligned start
    const int x = q % N_XCD, end = off + nbk;
    int t = 0;
    for (int y = 0; y < x; y++) {
        const int f = y >= off ? y : y + N_XCD;   // first position on XCD y
        if (f < end) t += (end - f + N_XCD - 1) / N_XCD;
    }
    const int f = x >= off ? x : x + N_XCD;
    return t + (q - f) / N_XCD;
}

} // namespace fimk

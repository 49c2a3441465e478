// Shared device/host helpers of the iPEPS library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/ipeps.h"

namespace ipeps {

// A HIP call that fails throws; the C ABI layer turns it into IPEPS_EDEVICE.
struct hip_error : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct status_error : std::runtime_error {
    int code;
    status_error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            throw ::ipeps::hip_error(std::string(#expr) + ": " + hipGetErrorString(e_) +   \
                                     " at " __FILE__ ":" + std::to_string(__LINE__));       \
    } while (0)

#define IPEPS_REQUIRE(cond, code, msg)                       \
    do {                                                     \
        if (!(cond)) throw ::ipeps::status_error(code, msg); \
    } while (0)

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Several jobs of one layout in one launch: the jobs' device buffers were
// allocated in the same order and sizes, so every buffer of job j sits
// delta[j] bytes from the same buffer of the lead job.  A kernel of `batch`
// matrices per job then runs per_job * njobs blocks (or block rows): block b
// works on matrix b % per_job of job b / per_job.  delta == NULL: one job,
// the plain batch.
struct JobMap {
    const long* delta = nullptr;
    int per_job = 1;
    int njobs = 1;
};
template <typename T>
__device__ inline T* jptr(T* p, const JobMap& jm, int b) {
    return jm.delta && p ? (T*)((char*)p + jm.delta[b / jm.per_job]) : p;
}
__device__ inline int jlocal(const JobMap& jm, int b) { return jm.delta ? b % jm.per_job : b; }

// ------------------------------------------------------------- complex FP64
struct cplx {
    double re, im;
};
__host__ __device__ inline cplx cmake(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
    return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx cconj(cplx a) { return cplx{a.re, -a.im}; }
// conj(a) * b
__host__ __device__ inline cplx cdotc(cplx a, cplx b) {
    return cplx{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
__host__ __device__ inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------- wave reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over each aligned group of 16 lanes with DPP moves (quad swaps, half-row
// and row mirrors); every lane of the group gets the same bits.
__device__ inline double dpp_move(double v, int ctrl_sel) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (ctrl_sel) {
        case 0:
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, true);
            break;
        case 1:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, true);
            break;
        case 2:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, true);  // row_half_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, true);
            break;
        default:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, true);  // row_mirror
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, true);
            break;
    }
    return __hiloint2double(hi, lo);
}
__device__ inline double group16_sum(double v) {
    v += dpp_move(v, 0);
    v += dpp_move(v, 1);
    v += dpp_move(v, 2);
    v += dpp_move(v, 3);
    return v;
}

// Block-wide sum of one double per thread; `red` must hold blockDim.x/64
// doubles of LDS.  All threads receive the result.
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}
__device__ inline double block_max(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    __syncthreads();
    return s;
}

// Stateless counter-based uniform in [0,1) (SplitMix64 finaliser).
// 1/x and 1/sqrt(x) for finite x > 0 (FP64): the hardware estimates refined by
// two Newton steps (each squares the relative error), accurate to rounding.
__device__ inline double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ inline double fast_rsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

__device__ inline double hash_uniform(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (counter + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace ipeps

// wave.h -- device helpers shared by the engines: the counter-based random
// numbers and the wave-level reductions and scans.
//
// Philox4x32-10 is the generator of Salmon, Moraes, Dror & Shaw, "Parallel
// random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32 x 32 -> 64
// bit products, the key bumped by two Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flipmc {
namespace {

constexpr double kTwoPi = 6.283185307179586;

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t a0 = 0xD2511F53u * c0, a1 = __umulhi(0xD2511F53u, c0);
        const uint32_t b0 = 0xCD9E8D57u * c2, b1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = b1 ^ c1 ^ k0;
        const uint32_t n2 = a1 ^ c3 ^ k1;
        c0 = n0;
        c1 = b0;
        c2 = n2;
        c3 = a0;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ double unit_open(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

__device__ __forceinline__ double unit_53(uint32_t lo, uint32_t hi)
{
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    return (double)((v >> 11) + 1) * 0x1p-53;
}

template <typename Real>
struct alignas(16) R4 {
    Real x, y, z, w;
};

// ---------------------------------------------------------------- wave ops --

__device__ __forceinline__ uint32_t rl_u(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ float rl_f(float v, int l) { return __int_as_float((int)rl_u(__float_as_uint(v), l)); }
__device__ __forceinline__ double rl_d(double v, int l)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = rl_u((uint32_t)b, l), hi = rl_u((uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)((hi << 32) | lo));
}
__device__ __forceinline__ float rl_r(float v, int l) { return rl_f(v, l); }
__device__ __forceinline__ double rl_r(double v, int l) { return rl_d(v, l); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v)
{
#pragma unroll
    for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Wave-wide sum with DPP row shifts and row broadcasts (a fixed addition
// order, so the result does not depend on timing); every lane gets it.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, kRowMask, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, kRowMask, 0xf, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_move<0x111, 0xf>(v);  // row_shr:1
    v += dpp_move<0x112, 0xf>(v);  // row_shr:2
    v += dpp_move<0x114, 0xf>(v);  // row_shr:4
    v += dpp_move<0x118, 0xf>(v);  // row_shr:8  -> lane 15 of a row holds the row sum
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 -> lane 31 holds rows 0 + 1
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 -> lane 63 holds all rows
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __longlong_as_double((long long)((hi << 32) | lo));
}

// The accepted dE of a sweep from the per-cell sums (each in its cell's trial
// order): lane l adds cells l, l + 64, ... in turn, then the DPP sum.  Every
// engine reduces the same way, so E_acc does not depend on how the cells were
// spread over waves and workgroups.  Call with a whole wave.
__device__ __forceinline__ double sweep_energy(const double* ecell, uint32_t ncell)
{
    double a = 0.0;
    for (uint32_t c = (uint32_t)__lane_id(); c < ncell; c += 64u) a += ecell[c];
    return wave_sum_dpp(a);
}

// Exclusive prefix sum over the wave; *total gets the wave total.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total)
{
    const int lane = __lane_id();
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    *total = __shfl(inc, 63);
    return inc - v;
}

__device__ __forceinline__ uint32_t rank_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place exclusive scan of a[0..n) by a whole workgroup of kT threads.
template <int kT>
__device__ void block_excl_scan_t(uint32_t* a, uint32_t n, uint32_t* scratch)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (n + kT - 1) / kT;
    const uint32_t beg = min(n, tid * per), end = min(n, beg + per);
    uint32_t s = 0;
    for (uint32_t i = beg; i < end; ++i) s += a[i];
    uint32_t tot;
    const uint32_t ex = wave_excl_scan(s, &tot);
    if (lane == 0) scratch[wave] = tot;
    __syncthreads();
    uint32_t run = ex;
    for (int w = 0; w < wave; ++w) run += scratch[w];
    for (uint32_t i = beg; i < end; ++i) {
        const uint32_t t = a[i];
        a[i] = run;
        run += t;
    }
    __syncthreads();
}

}  // namespace
}  // namespace flipmc

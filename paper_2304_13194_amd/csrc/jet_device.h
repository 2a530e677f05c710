// Device helpers: SplitMix64, wave64 reductions/scans, LDS ordering.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream64(uint64_t seed, uint64_t i)
{
    return mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

// Order this wave's LDS traffic across lanes. The LDS executes a wave's DS
// instructions in issue order, so it is enough to keep the compiler from
// moving LDS operations across this point and to let earlier LDS operations
// retire (lgkmcnt(0)); outstanding global loads are not waited for.
__device__ __forceinline__ void lds_fence_wave()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt(63) expcnt(7) lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("" ::: "memory");
}

template <int G>
__device__ __forceinline__ uint64_t gmax_u64(uint64_t x)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        uint64_t y = __shfl_xor(x, o, G);
        x = x > y ? x : y;
    }
    return x;
}
template <int G, typename T>
__device__ __forceinline__ T gsum(T x)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
    return x;
}

// Inclusive scan over the 64 lanes of a converged wave.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x)
{
    const int l = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (l >= d) x += y;
    }
    return x;
}

// Append `value` for every active lane with `pred` to list[0..] using one
// atomic per wave on *counter. Positions among the wave's lanes follow lane
// order; order across waves is arbitrary (list order never affects results).
__device__ __forceinline__ void wave_append(bool pred, int32_t *counter, int32_t *list, int32_t value)
{
    uint64_t m = __ballot(pred);
    if (m == 0) return;
    const int l = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (l == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, 64);
    if (pred) list[base + __popcll(m & ((1ull << l) - 1ull))] = value;
}

// Block-wide append: like wave_append with one atomic per block. Every
// thread of the block (blockDim.x == NT) must call; s_cnt holds NT/64 + 1
// ints.
template <int NT>
__device__ __forceinline__ void block_append(bool pred, int32_t *counter, int32_t *list, int32_t value, int32_t *s_cnt)
{
    const uint64_t m = __ballot(pred);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) s_cnt[w] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < NT / 64; i++) {
            const int c = s_cnt[i];
            s_cnt[i] = t;
            t += c;
        }
        s_cnt[NT / 64] = t ? atomicAdd(counter, t) : 0;
    }
    __syncthreads();
    if (pred) list[s_cnt[NT / 64] + s_cnt[w] + __popcll(m & ((1ull << l) - 1ull))] = value;
    __syncthreads();
}

// Block-wide (blockDim.x == NT) reductions / exclusive scan. `scratch` must
// hold NT/64 elements; every thread of the block must call.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T x, T *scratch)
{
    x = gsum<64>(x);
    if (__lane_id() == 0) scratch[threadIdx.x >> 6] = x;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) t += scratch[i];
    __syncthreads();
    return t;
}
template <int NT>
__device__ __forceinline__ uint64_t block_max_u64(uint64_t x, uint64_t *scratch)
{
    x = gmax_u64<64>(x);
    if (__lane_id() == 0) scratch[threadIdx.x >> 6] = x;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) t = scratch[i] > t ? scratch[i] : t;
    __syncthreads();
    return t;
}
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *scratch, T &total)
{
    T inc = wave_incl_scan(x);
    if (__lane_id() == 63) scratch[threadIdx.x >> 6] = inc;
    __syncthreads();
    T off = 0, tot = 0;
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NT / 64; i++) {
        T s = scratch[i];
        if (i < wv) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

// slot() of the loss buckets for an int32 loss: 0 (< 0), 1 (= 0), 2 + floor(log2 x).
__device__ __forceinline__ int loss_slot(int x)
{
    if (x < 0) return 0;
    if (x == 0) return 1;
    return 33 - __clz(x);  // 2 + (31 - clz)
}

}  // namespace jet

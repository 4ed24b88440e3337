// Device helpers shared by the hard-disk (mpmc_kernels.hip) and hard-sphere
// (sphere_kernels.hip) kernels: the counter-based random numbers, per-lane
// register arrays indexed only at compile time, the XCD-aware workgroup
// order, a wave reduction, the votes of a lane group and the pair distance of
// the overlap test.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace mpmc {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round two 32x32
// products of words 0 and 2 with the round multipliers, XOR with words 1, 3
// and the round key; the key advances by the Weyl constants.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int i)
{
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// The chain's squared pair distance (the overlap test of Alg. 2 is
// r^2 < 1): dx*dx rounded, each further square added by one fused
// multiply-add, as the CPU oracle evaluates it.
__device__ __forceinline__ float pair_r2(float dx, float dy) { return __builtin_fmaf(dy, dy, dx * dx); }
__device__ __forceinline__ float pair_r2(float dx, float dy, float dz)
{
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Uniform integer in [0, k): high word of the 64-bit product v * k.
__device__ __forceinline__ uint32_t bounded(uint32_t v, uint32_t k) { return __umulhi(v, k); }

// Small per-lane register arrays.  Every element access below uses a
// compile-time index (C++17 fold expressions over an index sequence), so the
// arrays live in VGPRs from the first optimisation pass on; run-time slots
// are handled by select networks, never by indexing.
template <typename T, int N, int... I>
__device__ __forceinline__ T rsel_(const T (&a)[N], int i, std::integer_sequence<int, I...>)
{
    T r = a[0];
    ((r = (I == i) ? a[I] : r), ...);
    return r;
}
template <typename T, int N>
__device__ __forceinline__ T rsel(const T (&a)[N], int i)
{
    return rsel_(a, i, std::make_integer_sequence<int, N>{});
}

// Rotate the first n entries left by one: a[0..n) <- a[1], ..., a[n-1], a[0].
template <typename T, int N, int... I>
__device__ __forceinline__ void rrot_(T (&a)[N], int n, std::integer_sequence<int, I...>)
{
    const T first = a[0];
    ((a[I] = (I + 1 < n) ? a[(I + 1 < N) ? I + 1 : I] : ((I == n - 1) ? first : a[I])), ...);
}
template <typename T, int N>
__device__ __forceinline__ void rrot(T (&a)[N], int n)
{
    rrot_(a, n, std::make_integer_sequence<int, N>{});
}

// a[q] <- a[perm nibble q] for every q: apply a permutation packed as 4-bit
// source indices.
template <typename T, int N, int... I>
__device__ __forceinline__ void rperm_(T (&a)[N], uint32_t P, std::integer_sequence<int, I...>)
{
    const T old[N] = {a[I]...};
    ((a[I] = rsel(old, (int)((P >> (4 * I)) & 0xFu))), ...);
}
template <typename T, int N>
__device__ __forceinline__ void rperm(T (&a)[N], uint32_t P)
{
    rperm_(a, P, std::make_integer_sequence<int, N>{});
}

// As rrot and rperm over the first M entries only, for n <= M: the entries
// at or past M are the ones the full forms leave unchanged.
template <int M, typename T, int N, int... I>
__device__ __forceinline__ void rrot_m_(T (&a)[N], int n, std::integer_sequence<int, I...>)
{
    const T first = a[0];
    ((a[I] = (I + 1 < n) ? a[(I + 1 < M) ? I + 1 : I] : ((I == n - 1) ? first : a[I])), ...);
}
template <int M, typename T, int N>
__device__ __forceinline__ void rrot_m(T (&a)[N], int n)
{
    static_assert(M <= N, "prefix longer than the array");
    rrot_m_<M>(a, n, std::make_integer_sequence<int, M>{});
}
template <int M, typename T, int N, int... I>
__device__ __forceinline__ void rperm_m_(T (&a)[N], uint32_t P, std::integer_sequence<int, I...>)
{
    const T old[M] = {a[I]...};
    ((a[I] = rsel(old, (int)((P >> (4 * I)) & 0xFu))), ...);
}
template <int M, typename T, int N>
__device__ __forceinline__ void rperm_m(T (&a)[N], uint32_t P)
{
    static_assert(M <= N, "prefix longer than the array");
    rperm_m_<M>(a, P, std::make_integer_sequence<int, M>{});
}

// Swap nibbles i and j of a packed permutation.
__device__ __forceinline__ uint32_t nib_swap(uint32_t P, int i, int j)
{
    const uint32_t vi = (P >> (4 * i)) & 0xFu, vj = (P >> (4 * j)) & 0xFu;
    P &= ~((0xFu << (4 * i)) | (0xFu << (4 * j)));
    return P | (vj << (4 * i)) | (vi << (4 * j));
}

// Workgroup id -> logical tile, so that consecutive tiles (neighbouring
// cells) run on the same XCD: workgroups are dispatched round-robin over the
// eight XCDs, each with its own L2.  The grid is launched as 8 * per groups;
// tiles >= the logical count do no work.
__device__ __forceinline__ int xcd_tile(int per)
{
    return (int)(blockIdx.x % 8u) * per + (int)(blockIdx.x / 8u);
}

__device__ __forceinline__ unsigned wave_sum_u32(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exchange with the neighbouring lane of a group of two or four (DPP quad
// permutations [1,0,3,2] and [2,3,0,1]; groups are quad-aligned).
__device__ __forceinline__ uint32_t lane_xor1(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_xor2(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
}
template <int LPC>
__device__ __forceinline__ bool group_all(bool v)
{
    uint32_t x = v ? 1u : 0u;
    if (LPC >= 2) x &= lane_xor1(x);
    if (LPC >= 4) x &= lane_xor2(x);
    return x != 0u;
}
template <int LPC>
__device__ __forceinline__ bool group_any(bool v)
{
    uint32_t x = v ? 1u : 0u;
    if (LPC >= 2) x |= lane_xor1(x);
    if (LPC >= 4) x |= lane_xor2(x);
    return x != 0u;
}

}  // namespace mpmc

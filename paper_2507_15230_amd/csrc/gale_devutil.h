// gale_devutil.h -- device helpers shared by the relation kernels: a
// workgroup exclusive scan, register sorting networks and per-wave sorts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gale {
// ---------------------------------------------------------------------------
// lane exchanges within a wave by DPP (data-parallel primitives: the VALU
// reads another lane's register directly) where a pattern exists, else by
// the LDS crossbar (__shfl_xor).  DPP controls of the GFX9 family:
// quad_perm(a, b, c, d) = a | b << 2 | c << 4 | d << 6, row_shl:n = 0x100 + n,
// row_shr:n = 0x110 + n, row_ror:n = 0x120 + n (rows of 16 lanes),
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.  Every lane of the wave must
// be active.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int dpp_xor1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_xor2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_xor8(int v) { return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_xor4(int v) {
    // lanes with bit 2 set take lane - 4 (row_shr:4), the others lane + 4 (row_shl:4)
    const int dn = __builtin_amdgcn_mov_dpp(v, 0x114, 0xF, 0xF, false);
    const int up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xF, 0xF, false);
    return (threadIdx.x & 4) ? dn : up;
}
// the value of lane ^ j (j a power of two below 64)
__device__ __forceinline__ int lane_xor(int v, int j) {
    switch (j) {
        case 1: return dpp_xor1(v);
        case 2: return dpp_xor2(v);
        case 4: return dpp_xor4(v);
        case 8: return dpp_xor8(v);
        default: return __shfl_xor(v, j, 64);
    }
}

// Inclusive sum over the lanes up to this one: shifts within rows of 16 lanes,
// then each row's total broadcast to the rows above it.
__device__ __forceinline__ int wave_incl_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1 and 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2 and 3
    return x;
}

// ---------------------------------------------------------------------------
// workgroup exclusive scan (wave64 DPP sums + one LDS word per wave)
// ---------------------------------------------------------------------------
// Two buffers of wave totals, used alternately (par flips on every call), so
// that the next call may start writing while threads still read this one's.
template <int B>
__device__ __forceinline__ int block_excl_scan(int v, int &total, int &par) {
    constexpr int NW = B / 64;
    __shared__ int s_wave[2][NW + 1];
    int *sw = s_wave[par];
    par ^= 1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int x = wave_incl_sum(v);
    if (lane == 63) sw[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const int t = lane < NW ? sw[lane] : 0;
        int y = t;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            const int z = __shfl_up(y, d, 64);
            if (lane >= d) y += z;
        }
        if (lane < NW) sw[lane] = y - t;
        if (lane == NW - 1) sw[NW] = y;
    }
    __syncthreads();
    total = sw[NW];
    return x - v + sw[wid];
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_sum(int x) {
    #pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ int wave_excl_scan(int v, int &total) {
    const int x = wave_incl_sum(v);
    total = __shfl(x, 63, 64);
    return x - v;
}

__device__ __forceinline__ bool has_vertex(int4 t, int u) {
    return t.x == u || t.y == u || t.z == u || t.w == u;
}

__device__ __forceinline__ void cswap_u(uint32_t &x, uint32_t &y) {
    const uint32_t lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
}

// Sort N registers ascending (bitonic network, N a power of two).
template <int N>
__device__ __forceinline__ void sort_regs(uint32_t (&v)[N]) {
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    if ((i & k) == 0)
                        cswap_u(v[i], v[l]);
                    else
                        cswap_u(v[l], v[i]);
                }
            }
        }
    }
}

// One wave sorts a list of n keys (n wave-uniform, every lane active) and
// writes it ascending to dst[0, n); key(i) gives the i-th key (< 2^31, all
// distinct).  Up to 64 K keys: a bitonic network over elements e = K lane + k
// (partners within a lane's registers for strides below K, across lanes by
// lane_xor above).
template <int K, class F>
__device__ __forceinline__ void wave_bitonic(int n, const F &key, int32_t *dst) {
    // lane l holds keys K l .. K l + K - 1: partners fewer than K apart are
    // in the lane's own registers, the others K j' apart in lane l ^ j'
    const int lane = threadIdx.x & 63;
    uint32_t v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = K * lane + k;
        v[k] = e < n ? (uint32_t)key(e) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int s = 2; s <= 64 * K; s <<= 1) {
#pragma unroll
        for (int j = s >> 1; j > 0; j >>= 1) {
            if (j < K) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int l = k ^ j;
                    if (l > k) {
                        // the pair (K lane + k, K lane + l) ascends where bit s of its index is clear
                        if (((K * lane + k) & s) == 0)
                            cswap_u(v[k], v[l]);
                        else
                            cswap_u(v[l], v[k]);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int e = K * lane + k;
                    const uint32_t w = (uint32_t)lane_xor((int)v[k], j / K);
                    // the lower element of an ascending pair keeps the minimum
                    const bool keep_min = ((e & j) == 0) == ((e & s) == 0);
                    v[k] = keep_min ? min(v[k], w) : max(v[k], w);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = K * lane + k;
        if (e < n) dst[e] = (int32_t)v[k];
    }
}

// Longer lists: each key goes to its rank (the number of smaller keys),
// 256 keys per sweep over the list.
template <class F>
__device__ __forceinline__ void wave_rank_sort(int n, const F &key, int32_t *dst) {
    constexpr int K = 4;
    const int lane = threadIdx.x & 63;
    for (int i0 = 0; i0 < n; i0 += 64 * K) {
        uint32_t x[K];
        int rk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = i0 + lane + 64 * k;
            x[k] = i < n ? (uint32_t)key(i) : 0xFFFFFFFFu;
            rk[k] = 0;
        }
        for (int j = 0; j < n; ++j) {
            const uint32_t y = (uint32_t)key(j);
#pragma unroll
            for (int k = 0; k < K; ++k) rk[k] += y < x[k];
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (i0 + lane + 64 * k < n) dst[rk[k]] = (int32_t)x[k];
    }
}

template <class F>
__device__ __forceinline__ void wave_sort(int n, const F &key, int32_t *dst) {
    if (n <= 64)
        wave_bitonic<1>(n, key, dst);
    else if (n <= 128)
        wave_bitonic<2>(n, key, dst);
    else if (n <= 256)
        wave_bitonic<4>(n, key, dst);
    else
        wave_rank_sort(n, key, dst);
}

}  // namespace gale

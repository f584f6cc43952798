// Velocity sets and population storage codecs for the gfx950 kernels.
//
// D3Q19 follows Table I of the paper (rest weight 1/3, six axis velocities
// 1/18, twelve face diagonals 1/36); D2Q9 is its 2D analogue (4/9, 1/9,
// 1/36).  Both list the rest velocity first and then opposite pairs next to
// each other, so opp(i) = i + 1 for odd i and i - 1 for even i > 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iblb {

template <int DIM>
struct Lattice;

template <>
struct Lattice<2> {
    static constexpr int Q = 9;
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0},
                                    {0, 1, 0},  {0, -1, 0},  {1, 1, 0},
                                    {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}};
    static constexpr float w[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,
                                   1.f / 9.f,  1.f / 9.f,  1.f / 36.f,
                                   1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

template <>
struct Lattice<3> {
    static constexpr int Q = 19;
    static constexpr int c[19][3] = {
        {0, 0, 0},  {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
        {0, 0, 1},  {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
        {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1},  {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
    static constexpr float w[19] = {
        1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
        1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
        1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
        1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Storage of a population deviation f_i - w_i.  Loads widen to fp32;
// stores round to nearest even.
enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Buffer descriptors for the lattice kernel's population traffic: a
// buffer_load/buffer_store takes a 32-bit byte offset per lane and keeps the
// 64-bit base in scalar registers, so no lane forms a 64-bit address.
// kBufNT: the cache-policy bit of a non-temporal access (nt); kBufSC1: the
// sc1 scope bit.
constexpr int kBufNT = 2;
constexpr int kBufSC1 = 16;
constexpr int kBufWord3 = 0x00020000;  // descriptor word 3: raw (untyped) 32-bit data
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufWord3);
}

template <int S>
struct Codec;

template <>
struct Codec<ST_F32> {
    using T = float;
    static __device__ __forceinline__ float load(const T* p, int i) { return p[i]; }
    static __device__ __forceinline__ float load_nt(const T* p, int i) { return __builtin_nontemporal_load(p + i); }
    static __device__ __forceinline__ void store(T* p, int i, float v) { p[i] = v; }
    static __device__ __forceinline__ void store_nt(T* p, int i, float v) {
        __builtin_nontemporal_store(v, p + i);
    }
    template <int AUX>
    static __device__ __forceinline__ float load_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX));
    }
    template <int AUX>
    static __device__ __forceinline__ void store_buf(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, AUX);
    }
    static __host__ __device__ __forceinline__ T from_double(double v) { return (float)v; }
    static __host__ __device__ __forceinline__ double to_double(T v) { return (double)v; }
};

template <>
struct Codec<ST_F16> {
    using T = _Float16;
    static __device__ __forceinline__ float load(const T* p, int i) { return (float)p[i]; }
    static __device__ __forceinline__ float load_nt(const T* p, int i) {
        return (float)__builtin_nontemporal_load(p + i);
    }
    static __device__ __forceinline__ void store(T* p, int i, float v) { p[i] = (_Float16)v; }
    static __device__ __forceinline__ void store_nt(T* p, int i, float v) {
        __builtin_nontemporal_store((_Float16)v, p + i);
    }
    template <int AUX>
    static __device__ __forceinline__ float load_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, AUX));
    }
    template <int AUX>
    static __device__ __forceinline__ void store_buf(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)v), r, (int)off, 0,
                                              AUX);
    }
    // exchange values are narrowed through fp32 (nearest even at each step)
    static __device__ __forceinline__ T from_double(double v) { return (_Float16)(float)v; }
    static __device__ __forceinline__ double to_double(T v) { return (double)(float)v; }
};

__host__ __device__ __forceinline__ uint16_t f32_to_bf16_rne(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

template <>
struct Codec<ST_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float load(const T* p, int i) { return bf16_to_f32(p[i]); }
    static __device__ __forceinline__ float load_nt(const T* p, int i) {
        return bf16_to_f32(__builtin_nontemporal_load(p + i));
    }
    static __device__ __forceinline__ void store(T* p, int i, float v) { p[i] = f32_to_bf16_rne(v); }
    static __device__ __forceinline__ void store_nt(T* p, int i, float v) {
        __builtin_nontemporal_store(f32_to_bf16_rne(v), p + i);
    }
    template <int AUX>
    static __device__ __forceinline__ float load_buf(__amdgpu_buffer_rsrc_t r, unsigned off) {
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, AUX));
    }
    template <int AUX>
    static __device__ __forceinline__ void store_buf(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_rne(v), r, (int)off, 0, AUX);
    }
    // exchange values are narrowed through fp32 (nearest even at each step)
    static __device__ __forceinline__ T from_double(double v) { return f32_to_bf16_rne((float)v); }
    static __device__ __forceinline__ double to_double(T v) { return (double)bf16_to_f32(v); }
};

template <int S>
constexpr int storage_bytes() { return S == ST_F32 ? 4 : 2; }

// Cache policy of the lattice kernel's non-temporal population stores: fp32
// stores also set sc1 (3D step 233.4 -> 232.0 us, 8192x4096 D2Q9 lattice
// alone 424 -> 410 us on the MI355X); 16-bit stores keep nt alone (with sc1
// the D2Q9 fp16 kernel took 236 against 230 us).
template <int S>
constexpr int nt_store_policy() { return S == ST_F32 ? (kBufNT | kBufSC1) : kBufNT; }

}  // namespace iblb

// Device-side helpers shared by the gfx950 kernels (not part of the ABI).
//
// Grid traversal: every streaming kernel runs ht.nblocks workgroups of kBlock
// threads.  Workgroup b owns a contiguous chunk of the frequency grid in the
// storage order of Sec. 3.1.2; chunks are dealt so that each of the 8 XCDs
// (which receive workgroups round robin) sweeps one contiguous eighth of the
// grid, keeping a stencil's neighbours in that XCD's L2.
//
// Reductions never use device-scope fences (on gfx950 each one writes back
// and invalidates the XCD's L2).  A kernel stores one partial per workgroup
// with a plain store; the next kernel on the stream (kernel boundaries make
// the stores visible) reduces all partials in its prologue, in the same fixed
// order in every workgroup, so every workgroup sees bit-identical totals.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "qp_internal.h"

namespace qp {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

// ---- structured-buffer gathers ----
// A buffer resource (four scalar registers) names `count` records of `stride`
// bytes at `base`.  A load at record index j reads base + j * stride, with the
// product formed by the address unit (so one 32-bit index register serves
// every resource, whatever the record size), and an index at or beyond
// `count` returns zero without a memory access.
typedef int rsrc_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
__device__ f32x2_t struct_load_f32x2(rsrc_t r, int index, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v2f32");
__device__ f64x2_t struct_load_f64x2(rsrc_t r, int index, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v2f64");

// gfx9 resource word 3: 32-bit data format, no swizzle, no thread-id offset.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, int stride, unsigned count)
{
    const unsigned long long a = (unsigned long long)base;
    rsrc_t r;
    r.x = __builtin_amdgcn_readfirstlane((int)(unsigned)a);
    r.y = __builtin_amdgcn_readfirstlane(
        (int)(((unsigned)(a >> 32) & 0xffffu) | ((unsigned)stride << 16)));
    r.z = __builtin_amdgcn_readfirstlane((int)count);
    r.w = kRsrcWord3;
    return r;
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ f32x4_t struct_load_f32x4(rsrc_t r, int index, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v4f32");

// Element i of right-hand side k in a family of K vectors of D entries:
// FP64 families are vector-major (vector k starts at k D); float families
// (the FP32-IR inner solve) interleave the right-hand sides (entry i of all
// K together), so one gather of K * 8 bytes serves them all.
template <typename T>
__device__ __forceinline__ size_t vec_at(int k, int K, size_t D, size_t i)
{
    return (sizeof(T) == 4) ? i * (size_t)K + k : (size_t)k * D + i;
}

template <typename T> __device__ __forceinline__ cplx_t<T> gather(rsrc_t r, int index);
template <> __device__ __forceinline__ float2 gather<float>(rsrc_t r, int index)
{
    const f32x2_t v = struct_load_f32x2(r, index, 0, 0, 0);
    return make_float2(v.x, v.y);
}
template <> __device__ __forceinline__ double2 gather<double>(rsrc_t r, int index)
{
    const f64x2_t v = struct_load_f64x2(r, index, 0, 0, 0);
    return make_double2(v.x, v.y);
}

// Chunk of workgroup b of nb (a grouped launch gives each problem its own
// range of workgroups; b and nb are then the problem's).
__device__ __forceinline__ void chunk_of_block_at(const Table *__restrict__ tab, int b, int nb,
                                                  int &begin, int &end)
{
    const int logical = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    begin = logical * tab->chunk;
    end = min(begin + tab->chunk, tab->D);
}

__device__ __forceinline__ void chunk_of_block(const Table *__restrict__ tab, int &begin, int &end)
{
    chunk_of_block_at(tab, (int)blockIdx.x, (int)gridDim.x, begin, end);
}

// floor(x / N) for 0 <= x < 2^31 by multiply-shift (magic from the host).
__device__ __forceinline__ int div_n(const Table *__restrict__ tab, int x)
{
    return (int)(((uint64_t)(uint32_t)x * tab->magic) >> tab->shift);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// Workgroup sum (or min) of NV values; the result is returned in every thread.
template <int NV, bool MIN = false>
__device__ __forceinline__ void block_reduce(double (&v)[NV])
{
    __shared__ double red[NV][kWaves];
    const int lane = threadIdx.x % kWave;
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = MIN ? wave_min(v[k]) : wave_sum(v[k]);
        if (lane == 0) red[k][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = red[k][0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t = MIN ? fmin(t, red[k][w]) : t + red[k][w];
        v[k] = t;
    }
    __syncthreads();
}

// Store workgroup b's totals: part[k * kMaxBlocks + b].
template <int NV, bool MIN = false>
__device__ __forceinline__ void store_partials_at(double (&v)[NV], double *__restrict__ part, int b)
{
    block_reduce<NV, MIN>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[k * kMaxBlocks + b] = v[k];
    }
}

template <int NV, bool MIN = false>
__device__ __forceinline__ void store_partials(double (&v)[NV], double *__restrict__ part)
{
    store_partials_at<NV, MIN>(v, part, (int)blockIdx.x);
}

// Partial sums a thread takes of each value: b = threadIdx.x + t kBlock.
constexpr int kPartPer = kMaxBlocks / kBlock;
static_assert(kMaxBlocks % kBlock == 0, "partials are dealt evenly over a workgroup");

// Issues the loads of this thread's partials of NV values at once (every
// slot below kMaxBlocks exists; slots at or beyond the count are not used),
// so that they cost one round trip to memory rather than one each.
template <int NV>
__device__ __forceinline__ void fetch_partials(const double *__restrict__ part,
                                               double (&p)[NV][kPartPer])
{
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int t = 0; t < kPartPer; ++t) p[k][t] = part[k * kMaxBlocks + threadIdx.x + t * kBlock];
}

// Sum (or min) of the first nb partials fetched above; same order in every
// workgroup, result in every thread.
template <int NV, bool MIN = false>
__device__ __forceinline__ void sum_partials(const double (&p)[NV][kPartPer], int nb, double (&v)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = MIN ? INFINITY : 0.0;
#pragma unroll
        for (int t = 0; t < kPartPer; ++t)
            if ((int)threadIdx.x + t * kBlock < nb) s = MIN ? fmin(s, p[k][t]) : s + p[k][t];
        v[k] = s;
    }
    block_reduce<NV, MIN>(v);
}

// Sum (or min) of the nb partials a previous kernel stored.
template <int NV, bool MIN = false>
__device__ __forceinline__ void load_totals(const double *__restrict__ part, int nb, double (&v)[NV])
{
    double p[NV][kPartPer];
    fetch_partials<NV>(part, p);
    sum_partials<NV, MIN>(p, nb, v);
}

__device__ __forceinline__ bool finite(double x) { return x == x && fabs(x) != INFINITY; }

// Keeps a uniform value's load at this point of the program (an empty asm
// statement that reads it from a scalar register).  A kernel's state flags,
// scalars and table fields were written by earlier launches, so each load
// is a round trip to memory; loaded together before the first branch they
// cost one, where the compiler would otherwise sink each below the branch
// that first needs it and chain them one after the other.
__device__ __forceinline__ void pin(int v) { asm volatile("" : : "s"(v)); }
__device__ __forceinline__ void pin(float v) { asm volatile("" : : "s"(v)); }
__device__ __forceinline__ void pin(double v) { asm volatile("" : : "s"(v)); }

}  // namespace qp

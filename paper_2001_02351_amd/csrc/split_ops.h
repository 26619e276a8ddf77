// The split-BF16 operands of the contraction (Eq. chi, reduced-precision
// form): the layout shared by the kernels that write them (the split
// preparation from FP64 M, and the FP32 pair kernels directly) and the
// contraction that reads them.
//
//   A: FP32 complex, 1 KB blocks [KP/8][NGP/16][4][16][2]: for a group of 8
//      pairs and 16 rows, pair quarter q holds rows 0..15 x pairs 2q, 2q+1
//   B: 2 NT BF16 planes [2 NT][KP/8][NGP][8] (the NT re terms, then the NT
//      im terms), 8 consecutive pairs of one row in 16 bytes
// with KP = pairs padded to 32 and NGP = ng padded to 128; every padding slot
// holds zero.  Each FP32 value x is written as x_0 + x_1 (+ x_2) with
// x_s = bf16 of what the earlier terms leave (each remainder exact in FP32).
#pragma once

#include <hip/hip_runtime.h>

#include "rp_internal.h"

namespace rp {

template <int NT> __device__ __forceinline__ void split(float x, __bf16 (&t)[NT])
{
    float r = x;
#pragma unroll
    for (int s = 0; s < NT; s++) {
        t[s] = (__bf16)r;
        if (s + 1 < NT) r = r - (float)t[s];
    }
}

// element of A holding pair P (index within the call's pairs) at row g
__device__ __forceinline__ long ops_a_index(const SplitOps &o, long P, int g)
{
    return ((P >> 3) * (long)(o.NGP >> 4) + (g >> 4)) * 128 + ((P & 7) >> 1) * 32 + (g & 15) * 2 + (P & 1);
}

// BF16 element of plane s holding pair P at row g
__device__ __forceinline__ long ops_b_index(const SplitOps &o, int s, long P, int g)
{
    return ((long)s * o.npg * o.NGP + (P >> 3) * (long)o.NGP + g) * 8 + (P & 7);
}

// pair P, row g: the FP32 value (re, im) into A and its split terms into B
__device__ __forceinline__ void ops_store(const SplitOps &o, long P, int g, float re, float im)
{
    ((float2 *)o.A)[ops_a_index(o, P, g)] = make_float2(re, im);
    unsigned short *B = (unsigned short *)o.B;
    float r = re, i = im;
    for (int s = 0; s < o.nterm; s++) {
        const __bf16 tr = (__bf16)r, ti = (__bf16)i;
        B[ops_b_index(o, s, P, g)] = __builtin_bit_cast(unsigned short, tr);
        B[ops_b_index(o, o.nterm + s, P, g)] = __builtin_bit_cast(unsigned short, ti);
        r = r - (float)tr;
        i = i - (float)ti;
    }
}

// pairs P (even) and P + 1 of one group, row g: one 16-byte store into A and
// one 4-byte store per plane, the same values as two ops_store calls
__device__ __forceinline__ void ops_store2(const SplitOps &o, long P, int g, float2 v0, float2 v1)
{
    *(float4 *)((float2 *)o.A + ops_a_index(o, P, g)) = make_float4(v0.x, v0.y, v1.x, v1.y);
    unsigned short *B = (unsigned short *)o.B;
    float r0 = v0.x, r1 = v1.x, i0 = v0.y, i1 = v1.y;
    for (int s = 0; s < o.nterm; s++) {
        const __bf16 a0 = (__bf16)r0, a1 = (__bf16)r1, b0 = (__bf16)i0, b1 = (__bf16)i1;
        const unsigned wr = (unsigned)__builtin_bit_cast(unsigned short, a0) |
                            ((unsigned)__builtin_bit_cast(unsigned short, a1) << 16);
        const unsigned wi = (unsigned)__builtin_bit_cast(unsigned short, b0) |
                            ((unsigned)__builtin_bit_cast(unsigned short, b1) << 16);
        *(unsigned *)(B + ops_b_index(o, s, P, g)) = wr;
        *(unsigned *)(B + ops_b_index(o, o.nterm + s, P, g)) = wi;
        r0 = r0 - (float)a0;
        r1 = r1 - (float)a1;
        i0 = i0 - (float)b0;
        i1 = i1 - (float)b1;
    }
}

}  // namespace rp

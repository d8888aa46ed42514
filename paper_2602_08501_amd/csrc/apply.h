// Device helpers shared by the kernels: reading caller int8 LLRs, and (batch
// decoder and server) applying an accepted move w_p to a stage-2 column (Eq. (4): the centre moves to
// c xor w_p; the stored -z changes sign on supp(w_p)).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpwsd {

// Caller int8 LLRs are read in [-127, 127]: in each byte of x a value of
// -128 (0x80) becomes -127 (0x81), the others are unchanged.  The symmetric
// range keeps every negation of z exact in int8.
__device__ inline uint32_t read_q4(uint32_t x)
{
    const uint32_t t = x ^ 0x80808080u;                         // 0x80 bytes become 0
    const uint32_t nz = ((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t;  // bit 7: byte of t nonzero
    return x + ((~nz & 0x80808080u) >> 7);
}
__device__ inline int read_q1(int8_t v) { return v < -127 ? -127 : (int)v; }

// Bytes 0 / 1 from the low 4 bits of nib: byte b is bit b (the four shifted
// copies of the nibble in the 24-bit product do not overlap).
__device__ inline uint32_t bit_bytes(uint32_t nib) { return __umul24(nib & 15u, 0x00204081u) & 0x01010101u; }

// Sum of the int8 lanes of x whose bit is set in the low 4 bits of nib.
__device__ inline int masked_sum4(uint32_t x, uint32_t nib, int acc)
{
    return __builtin_amdgcn_sdot4((int)x, (int)bit_bytes(nib), acc, false);
}

// Negate the int8 lanes of x whose bit is set in the low 4 bits of nib
// (two's complement per byte, no carry between bytes).
__device__ inline uint32_t neg_bytes(uint32_t x, uint32_t nib)
{
    const uint32_t one = bit_bytes(nib);  // bit b -> byte b
    const uint32_t t = x ^ (one * 0xFFu);
    return ((t & 0x7F7F7F7Fu) + one) ^ (t & 0x80808080u);
}

// Flip the N centre bits cw[N/8] and the signs of zneg[N] (int8) on the
// support of the packed move row mv[N/8]; 16 positions per step, the -z
// column read and written in independent 16-byte pieces (zneg 16-byte aligned).
__device__ inline void apply_move_i8(const uint8_t* __restrict__ mv, uint8_t* __restrict__ cw,
                                     int8_t* __restrict__ zneg, int N)
{
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    const uint16_t* m16 = reinterpret_cast<const uint16_t*>(mv);
    uint16_t* c16 = reinterpret_cast<uint16_t*>(cw);
    v4i_t* zp = reinterpret_cast<v4i_t*>(zneg);
    for (int g = 0; g < N / 16; g += 4) {  // 64 positions at a time
        uint32_t bits[4];
        v4i_t zv[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            bits[h] = g + h < N / 16 ? m16[g + h] : 0u;
            if (g + h < N / 16) zv[h] = zp[g + h];
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            if (g + h >= N / 16) continue;
            c16[g + h] = (uint16_t)(c16[g + h] ^ bits[h]);
#pragma unroll
            for (int d = 0; d < 4; ++d) zv[h][d] = (int)neg_bytes((uint32_t)zv[h][d], bits[h] >> (4 * d));
            zp[g + h] = zv[h];
        }
    }
}

// Flip the signs of zneg[N] (int8, 16-byte aligned) on the positions whose
// bit is set in the packed move row held in registers, mb[N/32].
template <int NW>
__device__ inline void flip_z_i8(const uint32_t (&mb)[NW], int8_t* __restrict__ zneg)
{
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    v4i_t* zp = reinterpret_cast<v4i_t*>(zneg);
    v4i_t zv[2 * NW];
#pragma unroll
    for (int g = 0; g < 2 * NW; ++g) zv[g] = zp[g];
#pragma unroll
    for (int g = 0; g < 2 * NW; ++g) {
        const uint32_t bits = mb[g >> 1] >> (16 * (g & 1));
#pragma unroll
        for (int d = 0; d < 4; ++d) zv[g][d] = (int)neg_bytes((uint32_t)zv[g][d], bits >> (4 * d));
        zp[g] = zv[g];
    }
}

}  // namespace mpwsd

// Layout of a paired-half move table (mpwsd_group_moves), shared by the host
// builder and the device search.
//
// Positions x of RM(r, m), N = 2^m, are split by the int8 search into four
// lane groups of N/4 consecutive positions: x = lg (N/4) + t.  A "normal"
// u (1 <= u < N) with a nonzero low part u_lo = u mod N/4 cuts the positions
// into the halves {x : u.x = 0} and {x : u.x = 1}; each lane group holds N/8
// positions of each half, so a half can be gathered without moving data
// between lanes.  A move whose support lies in the half u.x = 0 (a flat whose
// direction space is orthogonal to u) is stored as a row of N/2 bits over
// that half, and the SAME row scores its translate by e_i, i the lowest set
// bit of u_lo, against the other half: x -> x ^ e_i maps one half onto the
// other and keeps the order of positions, hence the canonical order of moves.
//
// Order of the N/2 positions of half h within a row, k = lg (N/8) + e
// (lane group lg, element e < N/8):
//     x = lg (N/4) + ins(e, i, b ^ h),   b = par(u_lo & ins(e, i, 0)) ^ par(u_hi & lg)
// where ins(e, i, v) inserts bit v at position i of e, u_hi = u / (N/4) and
// par is the parity of the set bits.
//
// Blob (host or device bytes, 256-byte aligned sections):
//     [0, 256)        header: magic, version, m, N, P, chunks, KW = N/2, extras
//     u[chunks]       int32 normal of each chunk of 128 rows
//     rows            [chunks][128][KW] int8, ready for the matrix cores:
//                     -128 where the row's move has position k, else 0;
//                     16-byte segment s of row r is stored at segment
//                     s ^ swz(r), swz(r) = (r / (256 / KW)) mod (KW / 16), so
//                     that the search reads a 16-row tile from LDS without
//                     bank conflicts after copying chunks verbatim
//     canon           [chunks][2][128] int32: index in the original table of
//                     the move a row scores against half 0 / half 1
//                     (P for padding rows, which are all zero)
//     sel             [N/4][SELW] int32, per normal u: v_perm_b32 selectors
//                     that gather the halves from a lane group's N/4 bytes of
//                     z and scatter them back (see below)
//     xrows           [extras][N/8] the moves whose direction space has no
//                     normal below N/4 (4096 of the 10668 moves of RM(2,7)),
//                     bit-packed as in the plain table, ascending index; the
//                     search scores them with the plain N-long rows
//     xcanon          [extras] int32 their indices in the original table
// Within a chunk the rows are sorted by canonical index, for both halves.
// Normals are below N/4 (u_hi = 0), so every lane group splits alike.
//
// Selectors of normal u (i = lowest set bit, S = max(i - 2, 0), W = N/32
// output dwords per half, a lane group's bytes as LDW = N/16 dwords d):
//     sel[0]              S
//     sel[1 + h W + k]    output dword k of half h = perm(z[lo + 2^S], z[lo],
//                         sel), lo = ins(k, S, 0)
//     sel[1 + 2 W + d]    z[d] = perm(half1[k], half0[k], sel) for the k with
//                         d in {lo, lo + 2^S}
// where perm(a, b, s) picks byte j from byte (s >> 8j) & 7 of a:b (b low).
#pragma once

#include <cstddef>
#include <cstdint>

namespace mpwsd {

constexpr uint32_t kGroupMagic = 0x4757504Du;  // "MPWG"
constexpr int kGroupVersion = 4;
constexpr int kGroupRows = 128;                // rows per chunk

struct GroupLayout {
    int N, KW, SELW;
    int64_t chunks, extras;
    size_t u_off, rows_off, canon_off, sel_off, xrows_off, xcanon_off, bytes;
};

inline size_t group_align(size_t x) { return (x + 255) & ~size_t(255); }

inline GroupLayout group_layout(int m, int64_t chunks, int64_t extras)
{
    GroupLayout g{};
    g.N = 1 << m;
    g.KW = g.N / 2;
    g.chunks = chunks;
    g.extras = extras;
    g.u_off = 256;
    g.rows_off = g.u_off + group_align(sizeof(int32_t) * (size_t)chunks);
    g.canon_off = g.rows_off + (size_t)chunks * kGroupRows * (size_t)g.KW;
    g.SELW = g.N / 4;  // 1 + 2 (N/32) + N/16 = N/8 + 1 entries, padded
    g.sel_off = g.canon_off + (size_t)chunks * 2 * kGroupRows * sizeof(int32_t);
    g.xrows_off = g.sel_off + group_align((size_t)(g.N / 4) * g.SELW * sizeof(int32_t));
    g.xcanon_off = g.xrows_off + group_align((size_t)extras * (size_t)(g.N / 8));
    g.bytes = g.xcanon_off + group_align((size_t)extras * sizeof(int32_t));
    return g;
}

// Bounds on the chunks of a table of P moves, `extras` of them kept apart:
// (P - extras)/2 rows, one partly filled chunk per normal at most.
inline int64_t group_min_chunks(int64_t P, int64_t extras) { return ((P - extras) / 2 + kGroupRows - 1) / kGroupRows; }
inline int64_t group_max_chunks(int m, int64_t P) { return (P / 2 + kGroupRows - 1) / kGroupRows + (1 << m); }

// segment swizzle of row r (see the layout above)
inline int group_swizzle(int KW, int r) { return (r / (256 / KW)) % (KW / 16); }

struct GroupHeader {
    uint32_t magic;
    int32_t version, m, N;
    int64_t P, chunks;
    int32_t KW, reserved;
    int64_t extras;
};

}  // namespace mpwsd

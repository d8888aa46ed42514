/*
 * Reference oracle for multipoint code-weight sphere decoding (MP-WSD).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, scalar CPU
 * implementation of what the decoder computes.  It is used by the test suite,
 * by the smoke check and by the CPU-baseline leg of the benchmark, and by
 * nothing else.  It shares no code, header, table or constant generator with
 * the HIP library: everything below is written from the paper's definitions
 * (Jo, Choi, Kim, Lee, "Multipoint Code-Weight Sphere Decoding: Parallel
 * Near-ML Decoding for Short-Blocklength Codes").
 *
 * Arithmetic modes.  Every real-valued quantity is held in a double, and
 * `rnd(mode, x)` is applied after every addition:
 *   ORC_INT  integer inputs (quantized LLRs); every value stays an integer far
 *            below 2^53, so double arithmetic is exact integer arithmetic;
 *   ORC_F32  each result is rounded to binary32, which reproduces IEEE single
 *            precision exactly for + and - (double has more than 2*24+2 bits);
 *   ORC_F64  plain double.
 * min, |.| and sign changes are exact in every mode.
 *
 * Bit vectors are one byte per bit (0/1) throughout, for readability.
 *
 * Parity status: every exported function is pinned by a CPU test against
 * closed forms, brute force, or invariants the paper states; the binary32
 * mode of every function that has one is pinned against a separate numpy
 * float32 evaluation of the same definitions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

enum { ORC_INT = 0, ORC_F32 = 1, ORC_F64 = 2 };

/* Move tables are support lists supp[P][stride] (ascending positions); a
 * move of weight below the stride ends with this marker.                    */
#define ORC_SUPP_END 0xFFFF

static double rnd(int mode, double x) { return mode == ORC_F32 ? (double)(float)x : x; }

static int popcount_int(unsigned v) { int c = 0; while (v) { c += v & 1u; v >>= 1; } return c; }

/* ------------------------------------------------------------------------- */
/* Reed-Muller code RM(r, m) in the polar (Kronecker) form.  Sec. II-B:
 * c = m G.  Rows of F^{(x)m}, F = [[1,0],[1,1]], natural index order:
 * entry (i, j) is 1 iff every bit set in j is also set in i.  Row i is the
 * evaluation of a monomial of degree m - popcount(i); RM(r, m) keeps the rows
 * with popcount(i) >= m - r.                                                 */

static int64_t binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t v = 1;
    for (int i = 1; i <= k; ++i) v = v * (n - k + i) / i;
    return v;
}

int orc_rm_dims(int r, int m, int* N, int* K)
{
    if (m < 1 || m > 10 || r < 0 || r > m) return -1;
    int k = 0;
    for (int d = 0; d <= r; ++d) k += (int)binom(m, d);
    *N = 1 << m;
    *K = k;
    return 0;
}

/* Information positions A, ascending.  Returns K. */
int orc_rm_info_set(int r, int m, int32_t* A)
{
    int n = 1 << m, k = 0;
    for (int i = 0; i < n; ++i)
        if (popcount_int((unsigned)i) >= m - r) A[k++] = i;
    return k;
}

/* c = u G with G = F^{(x)m}, straight from the definition of G: O(N^2). */
void orc_encode_def(int m, const uint8_t* u, uint8_t* c)
{
    int n = 1 << m;
    for (int j = 0; j < n; ++j) {
        int acc = 0;
        for (int i = 0; i < n; ++i)
            if ((j & ~i) == 0) acc ^= u[i];
        c[j] = (uint8_t)acc;
    }
}

/* The same map by the Kronecker factorisation, one factor F per index bit:
 * for every pair (a, a + 2^s) with bit s of a clear, x[a] ^= x[a + 2^s]. */
void orc_encode(int m, const uint8_t* u, uint8_t* c)
{
    int n = 1 << m;
    memcpy(c, u, (size_t)n);
    for (int s = 0; s < m; ++s) {
        int h = 1 << s;
        for (int a = 0; a < n; ++a)
            if ((a & h) == 0) c[a] ^= c[a + h];
    }
}

/* ------------------------------------------------------------------------- */
/* Code-weight sphere S_1(0) without the zero word, Sec. II-C, Eq. (2)-(3).
 * The minimum-weight codewords of RM(r, m) are the incidence vectors of the
 * (m-r)-dimensional affine subspaces (flats) of the point set F_2^m, where
 * coordinate j is the point whose bits are the bits of j.
 *
 * Enumeration here: every k-dimensional linear subspace V (k = m - r) is
 * given by the unique reduced-echelon basis (pivot = highest set bit, each
 * basis vector zero at the other pivots); each flat is a coset a + V, taken
 * once by requiring a to be the smallest point of its coset.  The moves are
 * then put in canonical order: ascending by the sorted support tuple,
 * compared lexicographically.                                                */

typedef struct { int m, k, w; int64_t count, cap; uint16_t* supp; } flat_sink;

static void emit_cosets(flat_sink* fs, const int* basis)
{
    int n = 1 << fs->m, k = fs->k, w = 1 << k;
    int pts[1 << 10];
    int span[1 << 10];
    for (int s = 0; s < w; ++s) {
        int v = 0;
        for (int b = 0; b < k; ++b) if (s & (1 << b)) v ^= basis[b];
        span[s] = v;
    }
    for (int a = 0; a < n; ++a) {
        int is_min = 1;
        for (int s = 0; s < w; ++s) { pts[s] = a ^ span[s]; if (pts[s] < a) is_min = 0; }
        if (!is_min) continue;
        if (fs->supp && fs->count < fs->cap) {
            /* sort the w points ascending (insertion sort) */
            for (int i = 1; i < w; ++i) {
                int x = pts[i], j = i - 1;
                while (j >= 0 && pts[j] > x) { pts[j + 1] = pts[j]; --j; }
                pts[j + 1] = x;
            }
            for (int i = 0; i < w; ++i) fs->supp[fs->count * w + i] = (uint16_t)pts[i];
        }
        fs->count++;
    }
}

/* Recursively choose the pivots (strictly decreasing) and then the free
 * bits of each basis vector. */
static void enum_free(flat_sink* fs, int* basis, const int* piv, int row)
{
    if (row == fs->k) { emit_cosets(fs, basis); return; }
    int p = piv[row];
    /* free positions of this row: bits below the pivot that are not pivots */
    int freepos[16], nf = 0;
    for (int b = 0; b < p; ++b) {
        int isp = 0;
        for (int t = 0; t < fs->k; ++t) if (piv[t] == b) isp = 1;
        if (!isp) freepos[nf++] = b;
    }
    for (int mask = 0; mask < (1 << nf); ++mask) {
        int v = 1 << p;
        for (int t = 0; t < nf; ++t) if (mask & (1 << t)) v |= 1 << freepos[t];
        basis[row] = v;
        enum_free(fs, basis, piv, row + 1);
    }
}

static void enum_pivots(flat_sink* fs, int* piv, int row, int below)
{
    if (row == fs->k) { int basis[16]; enum_free(fs, basis, piv, 0); return; }
    for (int p = below - 1; p >= fs->k - row - 1; --p) {
        piv[row] = p;
        enum_pivots(fs, piv, row + 1, p);
    }
}

static int g_cmp_w;
static int cmp_supp(const void* a, const void* b)
{
    const uint16_t* x = (const uint16_t*)a;
    const uint16_t* y = (const uint16_t*)b;
    for (int i = 0; i < g_cmp_w; ++i)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/* Fills supp[P][w] (sorted support of each move, canonical order) when supp
 * is non-NULL and cap >= P.  Returns P, or -1 on bad arguments / short cap. */
int64_t orc_moves(int r, int m, uint16_t* supp, int64_t cap, int* w_out)
{
    if (m < 1 || m > 10 || r < 0 || r >= m) return -1;
    flat_sink fs = { m, m - r, 1 << (m - r), 0, cap, supp };
    int piv[16];
    enum_pivots(&fs, piv, 0, m);
    *w_out = fs.w;
    if (supp) {
        if (fs.count > cap) return -1;
        g_cmp_w = fs.w;
        qsort(supp, (size_t)fs.count, sizeof(uint16_t) * (size_t)fs.w, cmp_supp);
    }
    return fs.count;
}

/* Bit-packed rows: bit j of a row is byte j/8, bit j%8 (least significant
 * bit first).  rows[P][N/8].  Support rows may end early with 0xFFFF.      */
void orc_pack_supports(int m, int64_t P, int w, const uint16_t* supp, uint8_t* rows)
{
    int nb = (1 << m) / 8;
    memset(rows, 0, (size_t)(P * nb));
    for (int64_t p = 0; p < P; ++p)
        for (int i = 0; i < w && supp[p * w + i] != ORC_SUPP_END; ++i) {
            int j = supp[p * w + i];
            rows[p * nb + j / 8] |= (uint8_t)(1u << (j % 8));
        }
}

/* ------------------------------------------------------------------------- */
/* Spheres of larger radius, Eq. (1)-(2): S_rho(0) is the union of the shells
 * C_{d_l}(0), l = 0..rho, where d_0 = 0 < d_1 < d_2 < ... are the distinct
 * weights that occur in the code.  The oracle finds them by visiting every
 * codeword: the 2^K messages in Gray-code order, each step adding one row of
 * G = F^{(x)m} (the row of the information position whose message bit
 * changes), and the weight recounted in full.  K <= 30.                     */

typedef void (*cw_visit)(const uint8_t* c, int n, int w, void* ctx);

static int visit_codewords(int r, int m, cw_visit visit, void* ctx)
{
    int n, K;
    if (orc_rm_dims(r, m, &n, &K) != 0 || K > 30) return -1;
    int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    orc_rm_info_set(r, m, A);
    uint8_t* c = (uint8_t*)calloc((size_t)n, 1);
    visit(c, n, 0, ctx);
    for (int64_t g = 1; g < ((int64_t)1 << K); ++g) {
        /* Gray codes of g-1 and g differ in the lowest set bit of g */
        int b = 0;
        while (!((g >> b) & 1)) ++b;
        int row = A[b];
        for (int j = 0; j < n; ++j)
            if ((j & ~row) == 0) c[j] ^= 1;
        int w = 0;
        for (int j = 0; j < n; ++j) w += c[j];
        visit(c, n, w, ctx);
    }
    free(A);
    free(c);
    return 0;
}

static void count_weight(const uint8_t* c, int n, int w, void* ctx)
{
    (void)c; (void)n;
    ((int64_t*)ctx)[w]++;
}

/* A[0..N]: the number of codewords of each weight.  Returns 0, or -1. */
int orc_weight_distribution(int r, int m, int64_t* A)
{
    if (m < 1 || m > 10 || r < 0 || r > m) return -1;
    memset(A, 0, sizeof(int64_t) * (size_t)((1 << m) + 1));
    return visit_codewords(r, m, count_weight, A);
}

typedef struct { int wlo, whi, stride; int64_t count, cap; uint16_t* supp; } sphere_sink;

static void collect_word(const uint8_t* c, int n, int w, void* ctx)
{
    sphere_sink* s = (sphere_sink*)ctx;
    if (w < s->wlo || w > s->whi) return;
    if (s->supp && s->count < s->cap) {
        uint16_t* row = s->supp + s->count * s->stride;
        int k = 0;
        for (int j = 0; j < n; ++j) if (c[j]) row[k++] = (uint16_t)j;
        while (k < s->stride) row[k++] = ORC_SUPP_END;
    }
    s->count++;
}

static int cmp_weight_supp(const void* a, const void* b)
{
    const uint16_t* x = (const uint16_t*)a;
    const uint16_t* y = (const uint16_t*)b;
    int wx = 0, wy = 0;
    while (wx < g_cmp_w && x[wx] != ORC_SUPP_END) ++wx;
    while (wy < g_cmp_w && y[wy] != ORC_SUPP_END) ++wy;
    if (wx != wy) return wx < wy ? -1 : 1;
    return cmp_supp(a, b);
}

/* The nonzero codewords of S_rho(0) (weights d_1 .. d_rho): supp[P][stride]
 * receives the ascending support of each, padded with ORC_SUPP_END, sorted by
 * weight and then by the support tuple compared lexicographically (for
 * rho = 1 the order of orc_moves).  *stride = d_rho.  Fills supp when it is
 * non-NULL and cap >= P.  Returns P, or -1 on bad arguments, short cap, or
 * when the code has fewer than rho nonzero weights.                          */
int64_t orc_sphere(int r, int m, int rho, uint16_t* supp, int64_t cap, int* stride)
{
    int n = 1 << m;
    if (rho < 1) return -1;
    int64_t* A = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (orc_weight_distribution(r, m, A) != 0) { free(A); return -1; }
    int got = 0, wlo = -1, whi = -1;
    for (int w = 1; w <= n && got < rho; ++w)
        if (A[w]) { if (wlo < 0) wlo = w; whi = w; ++got; }
    int64_t P = 0;
    for (int w = wlo; w <= whi && got == rho; ++w) P += A[w];
    free(A);
    if (got < rho) return -1;
    *stride = whi;
    if (!supp) return P;
    if (cap < P) return -1;
    sphere_sink s = { wlo, whi, whi, 0, cap, supp };
    visit_codewords(r, m, collect_word, &s);
    g_cmp_w = whi;
    qsort(supp, (size_t)s.count, sizeof(uint16_t) * (size_t)whi, cmp_weight_supp);
    return s.count;
}

/* ------------------------------------------------------------------------- */
/* CRC precoding, Sec. II-B: v = payload || crc, K' = K + K_crc.  The
 * remainder of p(x) x^L divided by g(x), with the first payload bit the
 * highest-degree coefficient, written most significant bit first.  Computed
 * as a plain shift register (init 0, no reflection, no final xor).
 * poly holds g(x) including its x^L term, e.g. 0x43 for x^6 + x + 1.       */
void orc_crc(const uint8_t* bits, int n, int L, uint32_t poly, uint8_t* crc)
{
    uint32_t reg = 0, top = 1u << (L - 1), mask = (1u << L) - 1;
    for (int i = 0; i < n; ++i) {
        uint32_t fb = ((reg & top) ? 1u : 0u) ^ bits[i];
        reg = (reg << 1) & mask;
        if (fb) reg ^= poly & mask;
    }
    for (int i = 0; i < L; ++i) crc[i] = (uint8_t)((reg >> (L - 1 - i)) & 1u);
}

/* 1 iff the remainder of v(x) (n bits, first bit highest degree) is zero. */
int orc_crc_ok(const uint8_t* v, int n, int L, uint32_t poly)
{
    if (L == 0) return 1;
    uint32_t reg = 0, top = 1u << (L - 1), mask = (1u << L) - 1;
    for (int i = 0; i < n; ++i) {
        uint32_t fb = ((reg & top) ? 1u : 0u) ^ v[i];
        reg = (reg << 1) & mask;
        if (fb) reg ^= poly & mask;
    }
    /* reg now holds v(x) * x^L mod g; since gcd(x, g) = 1 this is zero
       iff v(x) mod g is zero. */
    return reg == 0;
}

/* ------------------------------------------------------------------------- */
/* LLR quantizer: q = clamp(round-half-even(fl32(y * s)), -127, 127). */
void orc_quantize(const float* y, int64_t n, float s, int8_t* q)
{
    for (int64_t i = 0; i < n; ++i) {
        float t = y[i] * s;
        float r = nearbyintf(t);
        if (r > 127.0f) r = 127.0f;
        if (r < -127.0f) r = -127.0f;
        q[i] = (int8_t)r;
    }
}

/* ------------------------------------------------------------------------- */
/* Stage 1: successive-cancellation list decoding, Sec. III-A, in the LLR
 * form with the min-sum check-node rule.  The decoder follows the recursive
 * structure of c = u F^{(x)m}: writing c = (c', c'') in halves,
 *     c' = enc(u_first) xor enc(u_second),   c'' = enc(u_second),
 * so the first half of u sees f(l', l'') and, once it is decided and
 * re-encoded into v, the second half sees g(l', l'', v).
 *     f(a, b)    = sgn(a) sgn(b) min(|a|, |b|),   sgn(0) = +1
 *     g(a, b, v) = b + (1 - 2v) a
 * A positive LLR favours bit 0 (x = 1 - 2c).  Every leaf LLR is recomputed
 * from the channel values from scratch (slow and obviously right).          */

static double f_op(double a, double b)
{
    double sa = a < 0 ? -1.0 : 1.0, sb = b < 0 ? -1.0 : 1.0;
    double ma = fabs(a), mb = fabs(b);
    return sa * sb * (ma < mb ? ma : mb);
}

static double g_op(int mode, double a, double b, int v) { return rnd(mode, b + (v ? -a : a)); }

/* LLRs of node (lev, b): the 2^lev values feeding leaves [b 2^lev, (b+1) 2^lev). */
static void node_llr(int mode, const double* ch, int m, const uint8_t* u, int lev, int b, double* out)
{
    int n = 1 << lev;
    if (lev == m) { memcpy(out, ch, sizeof(double) * (size_t)n); return; }
    double* par = (double*)malloc(sizeof(double) * (size_t)(2 * n));
    node_llr(mode, ch, m, u, lev + 1, b >> 1, par);
    if ((b & 1) == 0) {
        for (int k = 0; k < n; ++k) out[k] = f_op(par[k], par[k + n]);
    } else {
        uint8_t* v = (uint8_t*)malloc((size_t)n);
        orc_encode(lev, u + (size_t)(b - 1) * n, v);
        for (int k = 0; k < n; ++k) out[k] = g_op(mode, par[k], par[k + n], v[k]);
        free(v);
    }
    free(par);
}

/* Min-sum SCL with list size L.
 *   llr[N]: channel LLRs (q in ORC_INT mode, y in the float modes).
 *   frozen[N]: 1 for frozen positions (u = 0).
 * Path metric: PM += |l| whenever the chosen bit disagrees with the hard
 * decision of l (HD(l) = 1 iff l < 0); frozen positions take u = 0.
 * At an information bit every path spawns u = 0 and u = 1; the 2n children
 * are ranked by (PM, parent slot, u) ascending and the first min(L, 2n)
 * survive, taking slots in that order.  The output lists the surviving
 * paths by (PM, slot) ascending: out_u[L][N], out_c[L][N], out_pm[L].
 * Returns the number of paths (min(L, 2^K)).                                */
int orc_scl(int m, int L, int mode, const double* llr, const uint8_t* frozen,
            uint8_t* out_u, uint8_t* out_c, double* out_pm)
{
    int n = 1 << m;
    uint8_t* u = (uint8_t*)calloc((size_t)L * n, 1);
    uint8_t* u2 = (uint8_t*)calloc((size_t)L * n, 1);
    double* pm = (double*)calloc((size_t)L, sizeof(double));
    double* pm2 = (double*)calloc((size_t)L, sizeof(double));
    double* lam = (double*)calloc((size_t)L, sizeof(double));
    double* cpm = (double*)malloc(sizeof(double) * 2 * (size_t)L);
    int* cord = (int*)malloc(sizeof(int) * 2 * (size_t)L);
    int np = 1;
    for (int i = 0; i < n; ++i) {
        for (int l = 0; l < np; ++l) node_llr(mode, llr, m, u + (size_t)l * n, 0, i, &lam[l]);
        if (frozen[i]) {
            for (int l = 0; l < np; ++l) {
                u[(size_t)l * n + i] = 0;
                if (lam[l] < 0) pm[l] = rnd(mode, pm[l] + fabs(lam[l]));
            }
            continue;
        }
        /* candidates in (parent slot, u) order */
        int nc = 2 * np;
        for (int l = 0; l < np; ++l)
            for (int b = 0; b < 2; ++b) {
                int hd = lam[l] < 0 ? 1 : 0;
                cpm[2 * l + b] = (b == hd) ? pm[l] : rnd(mode, pm[l] + fabs(lam[l]));
                cord[2 * l + b] = 2 * l + b;
            }
        /* stable insertion sort of the candidates by PM */
        for (int a = 1; a < nc; ++a) {
            int x = cord[a], j = a - 1;
            while (j >= 0 && cpm[cord[j]] > cpm[x]) { cord[j + 1] = cord[j]; --j; }
            cord[j + 1] = x;
        }
        int keep = nc < L ? nc : L;
        for (int s = 0; s < keep; ++s) {
            int cand = cord[s], par = cand / 2, b = cand % 2;
            memcpy(u2 + (size_t)s * n, u + (size_t)par * n, (size_t)n);
            u2[(size_t)s * n + i] = (uint8_t)b;
            pm2[s] = cpm[cand];
        }
        memcpy(u, u2, (size_t)keep * n);
        memcpy(pm, pm2, sizeof(double) * (size_t)keep);
        np = keep;
    }
    /* final order: (PM, slot) ascending */
    int* ord = (int*)malloc(sizeof(int) * (size_t)np);
    for (int l = 0; l < np; ++l) ord[l] = l;
    for (int a = 1; a < np; ++a) {
        int x = ord[a], j = a - 1;
        while (j >= 0 && pm[ord[j]] > pm[x]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = x;
    }
    for (int s = 0; s < np; ++s) {
        memcpy(out_u + (size_t)s * n, u + (size_t)ord[s] * n, (size_t)n);
        orc_encode(m, out_u + (size_t)s * n, out_c + (size_t)s * n);
        out_pm[s] = pm[ord[s]];
    }
    free(ord); free(u); free(u2); free(pm); free(pm2); free(lam); free(cpm); free(cord);
    return np;
}

/* ------------------------------------------------------------------------- */
/* Ordered-statistics decoding of order k (the OSD stage 1 of Sec. III-A and
 * Sec. IV-A, after Fossorier and Lin).  For one received word:
 *   1. rank the positions by reliability |llr_j|, largest first, ties to the
 *      smaller position;
 *   2. walk the positions in that order and keep each one whose column of G
 *      is independent of the columns already kept, until K are kept: the most
 *      reliable basis b_0 .. b_{K-1} (MRB, in reliability order).  Gaussian
 *      elimination on the rows of G along the way leaves rows g_0 .. g_{K-1}
 *      with g_i(b_t) = [i == t]: the codeword that takes the values v on the
 *      MRB is sum_i v_i g_i;
 *   3. the candidates are, for every set e of at most k MRB indices, the
 *      codeword with v_i = HD(llr_{b_i}) xor [i in e] (HD(l) = 1 iff l < 0).
 *      They are numbered by |e| and then by the sorted index tuple of e in
 *      lexicographic order;
 *   4. the list is the L candidates of smallest metric (orc_metric), ties to
 *      the smaller candidate number, in that order.
 * anchors[L][N], metric[L] out; mrb[K] out (may be NULL).  Returns the
 * number of list entries, min(L, number of candidates), or -1.              */
double orc_metric(int mode, int n, const double* y, const uint8_t* c);

typedef struct { double met; int64_t num; uint8_t* c; } osd_cand;

static int cmp_osd(const void* a, const void* b)
{
    const osd_cand* x = (const osd_cand*)a;
    const osd_cand* y = (const osd_cand*)b;
    if (x->met != y->met) return x->met < y->met ? -1 : 1;
    return x->num < y->num ? -1 : (x->num > y->num ? 1 : 0);
}

int orc_osd(int r, int m, int order, int L, int mode, const double* llr,
            uint8_t* anchors, double* metric, int32_t* mrb_out)
{
    int n, K;
    if (orc_rm_dims(r, m, &n, &K) != 0 || order < 0 || order > K || L < 1) return -1;
    /* generator rows: row i of F^{(x)m} for the information positions */
    int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    orc_rm_info_set(r, m, A);
    uint8_t* G = (uint8_t*)malloc((size_t)K * n);
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < n; ++j) G[(size_t)i * n + j] = (uint8_t)((j & ~A[i]) == 0);
    /* 1. reliability order (selection by repeated scan: plain and slow) */
    int* ord = (int*)malloc(sizeof(int) * (size_t)n);
    uint8_t* used = (uint8_t*)calloc((size_t)n, 1);
    for (int s = 0; s < n; ++s) {
        int best = -1;
        for (int j = 0; j < n; ++j) {
            if (used[j]) continue;
            if (best < 0 || fabs(llr[j]) > fabs(llr[best])) best = j;
        }
        used[best] = 1;
        ord[s] = best;
    }
    /* 2. MRB by Gaussian elimination along the order */
    int* mrb = (int*)malloc(sizeof(int) * (size_t)K);
    int piv = 0;
    for (int s = 0; s < n && piv < K; ++s) {
        int j = ord[s], row = -1;
        for (int i = piv; i < K; ++i) if (G[(size_t)i * n + j]) { row = i; break; }
        if (row < 0) continue;  /* column j depends on the kept ones */
        if (row != piv)
            for (int t = 0; t < n; ++t) {
                uint8_t x = G[(size_t)row * n + t];
                G[(size_t)row * n + t] = G[(size_t)piv * n + t];
                G[(size_t)piv * n + t] = x;
            }
        for (int i = 0; i < K; ++i)
            if (i != piv && G[(size_t)i * n + j])
                for (int t = 0; t < n; ++t) G[(size_t)i * n + t] ^= G[(size_t)piv * n + t];
        mrb[piv++] = j;
    }
    if (mrb_out) for (int i = 0; i < K; ++i) mrb_out[i] = mrb[i];
    /* 3. candidates, in their numbering */
    int64_t C = 0;
    for (int s = 0; s <= order; ++s) C += binom(K, s);
    osd_cand* cand = (osd_cand*)malloc(sizeof(osd_cand) * (size_t)C);
    uint8_t* store = (uint8_t*)malloc((size_t)C * n);
    uint8_t* v = (uint8_t*)malloc((size_t)K);
    int e[64];
    int64_t num = 0;
    for (int s = 0; s <= order; ++s) {
        for (int t = 0; t < s; ++t) e[t] = t;  /* first tuple of size s */
        for (;;) {
            for (int i = 0; i < K; ++i) v[i] = (uint8_t)(llr[mrb[i]] < 0);
            for (int t = 0; t < s; ++t) v[e[t]] ^= 1;
            uint8_t* c = store + (size_t)num * n;
            memset(c, 0, (size_t)n);
            for (int i = 0; i < K; ++i)
                if (v[i]) for (int t = 0; t < n; ++t) c[t] ^= G[(size_t)i * n + t];
            cand[num].met = orc_metric(mode, n, llr, c);
            cand[num].num = num;
            cand[num].c = c;
            ++num;
            /* next tuple of size s in lexicographic order */
            int t = s - 1;
            while (t >= 0 && e[t] == K - s + t) --t;
            if (t < 0) break;
            ++e[t];
            for (int u = t + 1; u < s; ++u) e[u] = e[u - 1] + 1;
        }
    }
    /* 4. the L best */
    qsort(cand, (size_t)C, sizeof(osd_cand), cmp_osd);
    int nl = (int)(C < L ? C : L);
    for (int k = 0; k < nl; ++k) {
        memcpy(anchors + (size_t)k * n, cand[k].c, (size_t)n);
        metric[k] = cand[k].met;
    }
    free(A); free(G); free(ord); free(used); free(mrb); free(cand); free(store); free(v);
    return nl;
}

/* ------------------------------------------------------------------------- */
/* Metrics.  ED(c) = ||y - x(c)||^2 with x = 1 - 2c (Sec. II-B), summed in
 * index order.  In ORC_INT mode the decoder uses the exact integer metric
 * M(c) = sum_{j : c_j = 1} q_j, which differs from the squared distance to q
 * by a constant and a positive factor: ||q - x(c)||^2 = const + 4 M(c).     */
double orc_metric(int mode, int n, const double* y, const uint8_t* c)
{
    double e = 0.0;
    if (mode == ORC_INT) {
        for (int j = 0; j < n; ++j) if (c[j]) e += y[j];
        return e;
    }
    for (int j = 0; j < n; ++j) {
        double x = c[j] ? -1.0 : 1.0;
        double d = rnd(mode, y[j] - x);
        e = rnd(mode, e + rnd(mode, d * d));
    }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Stage 2, Sec. III-B, Eq. (4), Alg. 1, with the correlation gain of Eq. (5).
 * For the path centred at c, moving to c xor w changes the squared distance
 * by 4 * sum_{j in supp(w)} z_j with z_j = y_j (1 - 2 c_j) = y_j x_j(c),
 * i.e. by -2 G(w).  Each iteration scores every move w_p of the table (the
 * nonzero words of S_rho(0), any radius; supp rows of stride w) by
 *     S_p = sum_{j in supp(w_p)} z_j        (ascending j, rnd after each add)
 * and takes p* = the smallest p attaining the minimum.  The move is accepted
 * iff S_p* < 0 (strict improvement, Sec. III-B); otherwise the path stops
 * and every later log entry is -1.
 *
 * One path: c[N] is updated in place, log[T] receives p* or -1.            */
void orc_stage2_path(int mode, int n, int64_t P, int w, const uint16_t* supp,
                     const double* y, uint8_t* c, int T, int32_t* log)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    int active = 1;
    for (int t = 0; t < T; ++t) {
        if (!active) { log[t] = -1; continue; }
        for (int j = 0; j < n; ++j) z[j] = c[j] ? -y[j] : y[j];
        int64_t best = -1;
        double bs = 0.0;
        for (int64_t p = 0; p < P; ++p) {
            double s = 0.0;
            for (int i = 0; i < w && supp[p * w + i] != ORC_SUPP_END; ++i) s = rnd(mode, s + z[supp[p * w + i]]);
            if (best < 0 || s < bs) { best = p; bs = s; }
        }
        if (best >= 0 && bs < 0) {
            for (int i = 0; i < w && supp[best * w + i] != ORC_SUPP_END; ++i) c[supp[best * w + i]] ^= 1;
            log[t] = (int32_t)best;
        } else {
            log[t] = -1;
            active = 0;
        }
    }
    free(z);
}

/* All paths of one frame, then the final choice (Alg. 1 return step): the
 * path with the smallest metric, ties to the smallest path index (the list
 * is in ascending path-metric order, Sec. IV-A).
 *   anchors[L][N] in, paths_out[L][N] out (final centres), logs[L][T],
 *   metric[L]; returns k*. */
int orc_stage2_frame(int mode, int n, int64_t P, int w, const uint16_t* supp,
                     const double* y, int L, const uint8_t* anchors, int T,
                     uint8_t* paths_out, int32_t* logs, double* metric)
{
    int kbest = 0;
    for (int k = 0; k < L; ++k) {
        uint8_t* c = paths_out + (size_t)k * n;
        memcpy(c, anchors + (size_t)k * n, (size_t)n);
        orc_stage2_path(mode, n, P, w, supp, y, c, T, logs + (size_t)k * T);
        metric[k] = orc_metric(mode, n, y, c);
        if (metric[k] < metric[kbest]) kbest = k;
    }
    return kbest;
}

/* ------------------------------------------------------------------------- */
/* The filtered form of the search (Sec. III-B, Eq. (4)-(5), and the filter
 * size rule of Sec. IV-A), in double precision.  Every path is improved on
 * its own, from its anchor, for at most J rounds.  In a round, with c the
 * path's current centre:
 *   - each move w gets its correlation gain G(w) = sum over supp(w) of
 *     -2 y_j x_j(c) (Eq. (5));
 *   - the mfilt moves of largest gain are kept (equal gains: smaller index
 *     first);
 *   - for each kept move the squared distance ||y - x(c xor w)||^2 is
 *     evaluated directly, and the smallest one (equal distances: smaller
 *     index) is taken;
 *   - if it is strictly below ||y - x(c)||^2 the centre moves there and the
 *     round logs the move; otherwise the path ends and logs -1 from here on.
 * A stopped path would meet the same centre again, so rounds in which no
 * path moves change nothing and need no separate stopping rule.  The
 * estimate is the path whose final centre is closest to y, the first such
 * path on equal distances.  This form exists to check that the filter does
 * not change the outcome of the full-argmin form used everywhere else.   */
typedef struct { double g; int64_t p; } gain_item;
static int cmp_gain(const void* a, const void* b)
{
    const gain_item* x = (const gain_item*)a;
    const gain_item* y = (const gain_item*)b;
    if (x->g != y->g) return x->g > y->g ? -1 : 1;
    return x->p < y->p ? -1 : (x->p > y->p ? 1 : 0);
}

static double sq_dist(int n, const double* y, const uint8_t* c)
{
    double e = 0.0;
    for (int j = 0; j < n; ++j) { double d = y[j] - (c[j] ? -1.0 : 1.0); e += d * d; }
    return e;
}

int orc_stage2_alg1(int n, int64_t P, int w, const uint16_t* supp, const double* y,
                    int L, const uint8_t* anchors, int J, int64_t mfilt,
                    uint8_t* paths_out, int32_t* logs)
{
    uint8_t* trial = (uint8_t*)malloc((size_t)n);
    gain_item* gi = (gain_item*)malloc(sizeof(gain_item) * (size_t)P);
    int64_t keep = mfilt < P ? mfilt : P;
    memcpy(paths_out, anchors, (size_t)L * n);
    for (int i = 0; i < L * J; ++i) logs[i] = -1;
    for (int k = 0; k < L; ++k) {
        uint8_t* c = paths_out + (size_t)k * n;
        for (int round = 0; round < J; ++round) {
            for (int64_t p = 0; p < P; ++p) {
                double g = 0.0;
                for (int i = 0; i < w && supp[p * w + i] != ORC_SUPP_END; ++i) {
                    int j = supp[p * w + i];
                    g += -2.0 * y[j] * (c[j] ? -1.0 : 1.0);
                }
                gi[p].g = g;
                gi[p].p = p;
            }
            qsort(gi, (size_t)P, sizeof(gain_item), cmp_gain);
            int64_t best = -1;
            double best_d = 0.0;
            for (int64_t t = 0; t < keep; ++t) {
                int64_t p = gi[t].p;
                memcpy(trial, c, (size_t)n);
                for (int i = 0; i < w && supp[p * w + i] != ORC_SUPP_END; ++i) trial[supp[p * w + i]] ^= 1;
                double d = sq_dist(n, y, trial);
                if (best < 0 || d < best_d || (d == best_d && p < best)) { best = p; best_d = d; }
            }
            if (best < 0 || !(best_d < sq_dist(n, y, c))) break;
            for (int i = 0; i < w && supp[best * w + i] != ORC_SUPP_END; ++i) c[supp[best * w + i]] ^= 1;
            logs[k * J + round] = (int32_t)best;
        }
    }
    int kb = 0;
    double bd = sq_dist(n, y, paths_out);
    for (int k = 1; k < L; ++k) {
        double d = sq_dist(n, y, paths_out + (size_t)k * n);
        if (d < bd) { bd = d; kb = k; }
    }
    free(trial); free(gi);
    return kb;
}

/* ------------------------------------------------------------------------- */
/* Maximum-likelihood decoding by exhaustive search over all 2^K codewords
 * (the MLD benchmark of Sec. IV-A); small K only.  Returns the smallest
 * metric; best_c receives the first codeword (in enumeration order of the
 * information bits) attaining it.                                           */
double orc_ml(int r, int m, int mode, const double* y, uint8_t* best_c)
{
    int n = 1 << m, N, K;
    orc_rm_dims(r, m, &N, &K);
    int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    orc_rm_info_set(r, m, A);
    uint8_t* u = (uint8_t*)malloc((size_t)n);
    uint8_t* c = (uint8_t*)malloc((size_t)n);
    double best = 0.0;
    for (int64_t msg = 0; msg < ((int64_t)1 << K); ++msg) {
        memset(u, 0, (size_t)n);
        for (int t = 0; t < K; ++t) u[A[t]] = (uint8_t)((msg >> t) & 1);
        orc_encode(m, u, c);
        double e = orc_metric(mode, n, y, c);
        if (msg == 0 || e < best) { best = e; memcpy(best_c, c, (size_t)n); }
    }
    free(A); free(u); free(c);
    return best;
}

/* ------------------------------------------------------------------------- */
/* The two-stage decoder of Sec. III for a batch of frames.  Stage 1 is SCL
 * with list size L on RM(r, m) (frozen = positions outside the information
 * set A); information bit t of v goes to u_{A[t]} (A ascending).  If the CRC
 * over v of the best list entry passes, that entry is the decision
 * (Sec. III-A); otherwise the L list entries are the anchors of stage 2.
 *
 *   llr[F][N]      channel values (q or y, as doubles)
 *   out_c[F][N]    decision
 *   out_anchor[F][L][N], crc_ok[F], out_k[F] (chosen path, 0 if stage 1
 *   ended the frame), out_metric[F], out_logs[F][L][T] (-1 when unused).
 * Frames [f0, f1) only, so callers can split the batch across threads.     */
void orc_decode_batch(int r, int m, int crc_len, uint32_t crc_poly, int L, int T, int mode,
                      int64_t P, int w, const uint16_t* supp,
                      const double* llr, int64_t f0, int64_t f1,
                      uint8_t* out_c, uint8_t* out_anchor, uint8_t* crc_ok,
                      int32_t* out_k, double* out_metric, int32_t* out_logs)
{
    int n = 1 << m, N, K;
    orc_rm_dims(r, m, &N, &K);
    int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    orc_rm_info_set(r, m, A);
    uint8_t* frozen = (uint8_t*)malloc((size_t)n);
    memset(frozen, 1, (size_t)n);
    for (int t = 0; t < K; ++t) frozen[A[t]] = 0;
    uint8_t* lu = (uint8_t*)calloc((size_t)L * n, 1);
    uint8_t* lc = (uint8_t*)calloc((size_t)L * n, 1);
    uint8_t* paths = (uint8_t*)calloc((size_t)L * n, 1);
    double* pm = (double*)calloc((size_t)L, sizeof(double));
    double* met = (double*)calloc((size_t)L, sizeof(double));
    uint8_t* v = (uint8_t*)malloc((size_t)K);
    for (int64_t f = f0; f < f1; ++f) {
        const double* y = llr + (size_t)f * n;
        int np = orc_scl(m, L, mode, y, frozen, lu, lc, pm);
        for (int s = np; s < L; ++s) memcpy(lc + (size_t)s * n, lc, (size_t)n);
        memcpy(out_anchor + (size_t)f * L * n, lc, (size_t)L * n);
        for (int t = 0; t < K; ++t) v[t] = lu[A[t]];
        int ok = crc_len > 0 ? orc_crc_ok(v, K, crc_len, crc_poly) : 0;
        crc_ok[f] = (uint8_t)ok;
        int32_t* lg = out_logs + (size_t)f * L * T;
        for (int i = 0; i < L * T; ++i) lg[i] = -1;
        if (ok) {
            memcpy(out_c + (size_t)f * n, lc, (size_t)n);
            out_k[f] = 0;
            out_metric[f] = orc_metric(mode, n, y, lc);
            continue;
        }
        int kb = orc_stage2_frame(mode, n, P, w, supp, y, L, lc, T, paths, lg, met);
        memcpy(out_c + (size_t)f * n, paths + (size_t)kb * n, (size_t)n);
        out_k[f] = kb;
        out_metric[f] = met[kb];
    }
    free(A); free(frozen); free(lu); free(lc); free(paths); free(pm); free(met); free(v);
}

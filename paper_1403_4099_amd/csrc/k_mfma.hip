// BF16x2 pair-sum on MFMA: v_pj = C_jj + 2 sum_{i<j} [s_pi = s_pj] (hi_ji + lo_ji),
// the sum over i read off a one-hot contraction (c_s is the diagonal of
// Y^T C Y, Eq. 6). Two kernels, chosen per shape by the tuner (Variant::packed):
//
// Column kernel (one column per stock). One wave owns 16 stocks
// j = jt0 .. jt0+15 and walks the rows i < j in chunks of 32 with
// v_mfma_f32_16x16x32_bf16:
//   A[m][k] = 2^125 C[jt0 + m][i0 + k]       (hi, then lo: two MFMAs)
//   B[k][n] = 2^-125 [s_{i0+k} = s_{jt0+n}] [i0 + k < jt0 + n]
//   D[m][n] += sum_k A[m][k] B[k][n];  D[n][n] = partial sum for stock jt0+n
// Lane l supplies row m = l%16 of A and column n = l%16 of B over the same
// eight k = 8(l/16)..+7, so its A row and B column are both stock jt0 + l%16.
// In a chunk the 16 lanes of a row group need the same 8 row codes per
// individual; each lane reads B/4 different dwords (two row codes each) and
// the xor takes its row operand from the lane that holds it (DPP row
// broadcast), so a chunk costs one B*64-byte LDS read per wave. The i < j mask
// is applied to B in the chunk that reaches the diagonal.
//
// Packed kernel (compacted columns). The columns are not one per stock but
// one per distinct label that the wave's 16 stocks carry in an individual and
// that at least one other stock of that individual shares (n_s >= 2; a
// singleton's sum is 0), packed over the workgroup's individuals into as few
// groups of 16 columns as they need: a chunk issues ceil(sum_b K_b / 16) MFMA
// pairs (groups run in pairs) instead of one pair per individual. Stock m of
// individual b reads its sum from D[m][column of (b, its label)]; the label
// sets come from a bit mask per individual of the labels with n_s >= 2
// (k_nsmask), and individuals past P or evaluated by the cluster-pair kernel
// get no columns. A lane of a column group reads the 8 row codes of its own
// column's individual (16 bytes, row codes staged per individual), the i < j
// mask is applied to A (once per chunk: A's row m is stock jt0 + m), and the
// FP32 sums are flushed through a wave-private LDS buffer. Fewer MFMAs, but
// per-lane row-code reads, a per-block column set-up and the flushes cost
// LDS and scalar work the column kernel does not have.
//
// Label codes (both kernels). A workgroup serves one block of 64 stocks,
// which carry at most 64 distinct labels per individual. Each such label gets
// a code (the block position of one stock that has it, 0..63); a row whose
// label is not among them gets the code kCodeNone. Codes are stored shifted
// into bits 8..15 of a 16-bit word, so for a row word r and a column word c
// the saturating difference 0x0100 - (r ^ c) is 0x0100 (the bf16 number
// 2^-125) when the labels are equal and 0 otherwise: two packed 16-bit ALU ops
// build two B elements. The 2^-125 is undone by keeping A as the split parts
// times 2^125 (a workspace copy made once per call); every product is then
// exactly the split part, as with a one-hot of 1.0.
//
// A is loaded once per (wave, chunk), one chunk ahead, by direct
// memory-to-LDS loads into a two-slot ring per wave (no registers hold it in
// flight; the column kernel addresses them through buffer descriptors, the
// packed kernel through global addresses), and reused by every individual or
// column group. FP32
// accumulation is flushed into FP64 at every 512-row boundary (no FP32 partial
// sum spans more than 512 rows). Both kernels give the same sums bit for bit:
// a stock's column holds the same one-hot values in either, and its FP32
// partial sums see the same products in the same chunks.
#include "pga_internal.hpp"

#include <type_traits>
#include <utility>

namespace pga {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr int kCodeShift = 8;
constexpr uint16_t kOneHot = 0x0100;        // bf16 2^-125
constexpr uint8_t kCodeNone = 0xFF;         // row label not present in the column block
constexpr uint32_t kCodeFree = 0xFE;        // column of a group left unused: matches no row

__device__ __forceinline__ uint32_t onehot2(uint32_t rows2, uint32_t col2) {
    const u16x2 x = __builtin_bit_cast(u16x2, rows2 ^ col2);
    const u16x2 one = {kOneHot, kOneHot};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(one, x));
}

// Row codes in the xor of lane t of a row group come from lane T of that
// group (DPP row broadcast; T a compile-time constant).
template <int T>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + T, 0xF, 0xF, false);
}

template <int... I, typename F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F &&f) {
    (f(std::integral_constant<int, I>{}), ...);
}

// Position of individual b's dword within a staged row pair: lane t of a row
// group reads positions (B/4)(t/4) .. +B/4-1, i.e. individuals t/4, t/4 + 4, ...
template <int B>
__host__ __device__ constexpr int mfma_pos(int b) {
    return (B / 4) * (b & 3) + (b >> 2);
}

// LDS of one workgroup (dynamic): row codes, kMfmaRowCodes 16-bit words (the
// code shifted into bits 8..15), as dwords [row pair][mfma_pos(b)] holding the
// rows 2q (low half) and 2q + 1 of individual b; then the label -> code
// tables [B][cstride] (bytes, cstride >= N); then each wave's ring of
// kMfmaASlots A slots, 2 KB each (the 16 x 32 hi tile, then the lo tile, in
// lane order), filled by direct buffer-to-LDS loads one chunk ahead.
struct MfmaLdsCols {
    uint32_t *rows;
    uint8_t *code;
    unsigned char *aring;
    int cstride;
};

// One column block jb (64 stocks, 16 per wave) for the B individuals of batch pb.
// On entry every code table entry below N holds kCodeNone; the entries it sets
// stay set (the launching kernel clears the tables before the next block).
template <int B>
__device__ __forceinline__ void mfma_block_cols(const InstDesc &d, int jb, int pb, int parity, const MfmaLdsCols &s) {
    constexpr int RC = kMfmaRowCodes / B;                     // rows staged per pass
    const int N = d.N, P = d.P, ld = d.ld_h;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform, kept scalar
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int q = 16 * wave + n;                              // position of this lane's stock in the block
    const int jt0 = jb * kMfmaCols + 16 * wave;
    const int j = jt0 + n;
    const int pbase = pb * B;
    const int32_t *__restrict__ labels = d.pop[parity];
    const uint16_t *__restrict__ hs = d.hs;
    const uint16_t *__restrict__ ls = d.ls;
    auto code = [&](int b, int l) -> uint8_t & { return s.code[(size_t)b * s.cstride + l]; };

    // Column labels; lanes with g == 0 register them in the code table. Stock,
    // individual and label are clamped into range as in the staging below: a
    // column past N or an individual past P is not stored, and a clamped
    // duplicate only writes a consistent code (the position of some stock with
    // that label) into its own individual's table.
    const uint32_t lmax = (uint32_t)(N - 1);
    const int jc = min(j, N - 1);
    uint32_t lj[B];
#pragma unroll
    for (int b = 0; b < B; ++b)
        lj[b] = min((uint32_t)gld(labels + (size_t)min(pbase + b, P - 1) * N + jc), lmax);
    if (g == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) code(b, (int)lj[b]) = (uint8_t)q;
    }
    __syncthreads();
    uint32_t col2[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const uint32_t c = code(b, (int)lj[b]);
        col2[b] = (c << kCodeShift) | (c << (16 + kCodeShift));
    }

    floatx4 acc[B];
    double acc64[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc64[b] = 0.0;
    }
    const int dreg = n & 3;                                   // lane holds D[n][n] in register n & 3 ...
    const bool diag_lane = (n >> 2) == g;                     // ... when its 4-row group contains row n

    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const float v = dreg == 0 ? acc[b][0] : dreg == 1 ? acc[b][1] : dreg == 2 ? acc[b][2] : acc[b][3];
            acc64[b] += (double)v;
            acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // Only waves with jt0 < N load A, and then j < ld for every lane (ld is a
    // multiple of 32 and jt0 a multiple of 16), so the loads need no guard. The
    // scaled copies are tile-major (a_tile_offset): the wave's 16 x 32 A block is
    // 1 KB of consecutive bytes in lane order.
    // Chunk i0's A goes to ring slot ((i0 - c0) / 32) % kMfmaASlots of this wave:
    // a direct buffer-to-LDS load puts lane l's 16 bytes at slot + 16 l, exactly
    // where the same lane reads them back. The loads address the scaled copies
    // through buffer descriptors: the lane's byte offset (16 l) stays in one
    // register and the chunk's offset is a scalar, so moving to the next chunk
    // costs no vector instruction.
    const size_t a_row = (size_t)(jt0 >> 4) * (size_t)(ld >> 5);
    unsigned char *const my_ring = s.aring + (size_t)wave * kMfmaASlots * 2048;
    auto slot_of = [&](int i0, int c0) { return my_ring + (size_t)(((i0 - c0) >> 5) % kMfmaASlots) * 2048; };
    const int a_bytes = 2 * ld * ld;                          // each scaled copy: ld x ld bf16
    const __amdgpu_buffer_rsrc_t hs_r = __builtin_amdgcn_make_buffer_rsrc((void *)hs, (short)0, a_bytes, kBufWord3);
    const __amdgpu_buffer_rsrc_t ls_r = __builtin_amdgcn_make_buffer_rsrc((void *)ls, (short)0, a_bytes, kBufWord3);
    const uint32_t lane_off = 16u * (uint32_t)lane;
    auto load_a = [&](int i0, int c0) {
        const uint32_t tile_off = (uint32_t)((a_row + (size_t)(i0 >> 5)) * 1024);   // uniform
        unsigned char *sl = slot_of(i0, c0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(hs_r, (__attribute__((address_space(3))) void *)sl, 16, lane_off,
                                                 tile_off, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ls_r, (__attribute__((address_space(3))) void *)(sl + 1024), 16,
                                                 lane_off, tile_off, 0, 0);
    };
    auto read_a = [&](int i0, int c0, uint4 &ah, uint4 &al) {
        const unsigned char *sl = slot_of(i0, c0);
        ah = *(const uint4 *)(sl + 16 * lane);
        al = *(const uint4 *)(sl + 1024 + 16 * lane);
    };
    // Lane t of row group g reads, into R[k], rows i0 + 8g + 2(t%4), +1 of individual 4k + t/4.
    auto read_r = [&](int i0, int c0, uint32_t (&R)[B / 4]) {
        const uint32_t *rp = s.rows + (size_t)(((i0 - c0) >> 1) + 4 * g + (n & 3)) * B + (B / 4) * (n >> 2);
        if constexpr (B == 4) {
            R[0] = *rp;
        } else if constexpr (B == 8) {
            const uint2 q2 = *(const uint2 *)rp;
            R[0] = q2.x;
            R[1] = q2.y;
        } else {
            const uint4 q4 = *(const uint4 *)rp;
            R[0] = q4.x;
            R[1] = q4.y;
            R[2] = q4.z;
            R[3] = q4.w;
        }
    };
    auto chunk = [&](auto masked_tag, int i0, int c0, uint4 ah, uint4 al, const uint32_t (&R)[B / 4]) {
        constexpr bool masked = decltype(masked_tag)::value;
        const int ik = i0 + 8 * g;                            // first of this lane's 8 rows
        uint32_t m[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        if constexpr (masked) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                m[r] = ((ik + 2 * r < j) ? 0xFFFFu : 0u) | ((ik + 2 * r + 1 < j) ? 0xFFFF0000u : 0u);
        }
        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah);
        const bf16x8 Al = __builtin_bit_cast(bf16x8, al);
        // B columns of individuals b and b + 1: dword e of b (rows ik + 2e, +1) is in
        // R[b/4] of lane 4(b%4) + e. All 8 broadcast xors are issued before the 8
        // saturating subtracts, so no subtract waits on the xor just before it.
        auto bcols = [&](auto bc, bf16x8 &B0, bf16x8 &B1) {
            constexpr int b = decltype(bc)::value;
            constexpr int t0 = 4 * (b & 3), t1 = 4 * ((b + 1) & 3);
            const uint32_t r0 = R[b >> 2], r1 = R[(b + 1) >> 2];
            const uint32_t x0 = row_bcast<t0 + 0>(r0) ^ col2[b], x1 = row_bcast<t0 + 1>(r0) ^ col2[b];
            const uint32_t x2 = row_bcast<t0 + 2>(r0) ^ col2[b], x3 = row_bcast<t0 + 3>(r0) ^ col2[b];
            const uint32_t y0 = row_bcast<t1 + 0>(r1) ^ col2[b + 1], y1 = row_bcast<t1 + 1>(r1) ^ col2[b + 1];
            const uint32_t y2 = row_bcast<t1 + 2>(r1) ^ col2[b + 1], y3 = row_bcast<t1 + 3>(r1) ^ col2[b + 1];
            uint4 v{onehot2(x0, 0u), onehot2(x1, 0u), onehot2(x2, 0u), onehot2(x3, 0u)};
            uint4 u{onehot2(y0, 0u), onehot2(y1, 0u), onehot2(y2, 0u), onehot2(y3, 0u)};
            if constexpr (masked) {
                v.x &= m[0]; v.y &= m[1]; v.z &= m[2]; v.w &= m[3];
                u.x &= m[0]; u.y &= m[1]; u.z &= m[2]; u.w &= m[3];
            }
            B0 = __builtin_bit_cast(bf16x8, v);
            B1 = __builtin_bit_cast(bf16x8, u);
        };
        static_for(std::make_integer_sequence<int, B / 2>{}, [&](auto hb) {
            constexpr int b = 2 * decltype(hb)::value;
            bf16x8 B0, B1;
            bcols(std::integral_constant<int, b>{}, B0, B1);
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B0, acc[b], 0, 0, 0);
            acc[b + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B1, acc[b + 1], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B0, acc[b], 0, 0, 0);
            acc[b + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B1, acc[b + 1], 0, 0, 0);
        });
        if (((i0 + 32) % kMfmaFlushRows) == 0) flush();
    };
    // Chunks [i0, end) of one kind. A chunk first reads its A and row codes from
    // LDS (its A was loaded during the previous chunk), then starts the load of
    // the next chunk's A into the other slot, then computes.
    auto run = [&](auto masked_tag, int &i0, int end, int cend, int c0) {
        for (; i0 < end; i0 += 32) {
            uint4 ah, al;
            read_a(i0, c0, ah, al);
            uint32_t R[B / 4];
            read_r(i0, c0, R);
            if (i0 + 32 < cend) load_a(i0 + 32, c0);
            chunk(masked_tag, i0, c0, ah, al, R);
        }
    };

    const int wg_iend = min(jb * kMfmaCols + kMfmaCols, N);   // rows any wave of the group needs
    const int my_iend = jt0 < N ? min(jt0 + 16, N) : 0;       // rows this wave needs (i < j <= jt0+15)
    const int i_diag = (jt0 / 32) * 32;                       // first chunk that may hold i >= j

    for (int c0 = 0; c0 < wg_iend; c0 += RC) {
        const int rows = min(RC, wg_iend - c0);
        const int rows32 = (rows + 31) & ~31;                 // chunks read whole 32-row groups
        // Thread t stages row pairs t + 256k of every individual: all 2 * PK * B
        // labels are loaded before the first table lookup, so the pass costs one
        // memory latency; each row pair is written as B consecutive dwords.
        // Nothing here needs a validity test, only in-bounds addresses: rows past
        // the pass (only past N, in its last 32-row chunk) meet zero-padded A;
        // individuals past P are not stored; a label outside [0, N) makes the
        // finish kernel give its individual -inf whatever its sums. So row and
        // individual indices are clamped into range, and labels to N - 1.
        constexpr int PK = RC / 512;
        const uint32_t rlast = (uint32_t)(rows - 1), lmax = (uint32_t)(N - 1);
        uint32_t lab[PK][2][B];
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const uint32_t r = 2u * (uint32_t)(threadIdx.x + 256 * k);
            const uint32_t r0 = min(r, rlast), r1 = min(r + 1u, rlast);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int32_t *lp = labels + (size_t)min(pbase + b, P - 1) * N + c0;   // uniform
                lab[k][0][b] = (uint32_t)gld(lp + r0);
                lab[k][1][b] = (uint32_t)gld(lp + r1);
            }
        }
#pragma unroll
        for (int k = 0; k < PK; ++k)                          // all table reads, then all writes
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < B; ++b) lab[k][h][b] = code(b, (int)min(lab[k][h][b], lmax));
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int q = threadIdx.x + 256 * k;
            if (2 * q < rows32) {
                uint32_t w[B];
#pragma unroll
                for (int b = 0; b < B; ++b)                       // code of row 2q in bits 8..15, of 2q+1 in 24..31
                    w[mfma_pos<B>(b)] = __builtin_amdgcn_perm(lab[k][1][b], lab[k][0][b], 0x040C000Cu);
#pragma unroll
                for (int v = 0; v < B / 4; ++v)
                    *(uint4 *)(s.rows + (size_t)q * B + 4 * v) = uint4{w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]};
            }
        }
        __syncthreads();
        const int cend = min(c0 + RC, my_iend);
        if (c0 < cend) {
            load_a(c0, c0);
            int i0 = c0;
            const int uend = min(cend, max(c0, i_diag));        // chunks entirely below the diagonal
            run(std::false_type{}, i0, uend, cend, c0);
            run(std::true_type{}, i0, cend, cend, c0);
        }
        __syncthreads();
    }
    flush();
    if (diag_lane && j < N) {
        const double cjj = gld(d.C + (size_t)j * N + j);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            if (p < P) gst(d.wsum + (size_t)p * N + j, fma(2.0, acc64[b], cjj));
        }
    }
}

// ---- LUT kernel: the one-hot read from LDS -----------------------------------------
// Per pass of lut_rows(B) rows, each staged (row, individual) toggles a bit
// pattern in a 16-bit row mask word: word [chunk][b][code][row group] encodes
// in bits 4..11 which of the 8 rows of that row group of that 32-row chunk
// carry the label whose block code is `code` in individual b, as the xor of
// the patterns lut_pat(e) of those rows e. The patterns are linearly
// independent, so the word identifies the row set, and shifted by 4 it is the
// byte offset of the set's entry in the one-hot table at LDS offset 0 (16
// bytes: the bf16 octet whose element e is 2^-125 for the rows e of the set
// and 0 otherwise). The patterns' low nibbles differ, so the empty set and
// the 8 single rows, the common words, fall in different LDS bank groups.
// The B operand of lane (row group g, column n) for individual b is then one
// 16-bit LDS read (its column code's word for row group g) and one 16-byte
// LDS read, with no vector ALU work: LDS reads proceed beside the MFMAs,
// while vector ALU work and MFMAs of a SIMD take turns. The i < j mask of the
// diagonal chunk is applied to A (row m of A is stock jt0 + m, the stock whose
// column meets it on the diagonal).
// The row masks are double-buffered: while the waves compute pass p from one
// buffer, each thread stages pass p + 1 into the other (its labels were
// loaded during pass p - 1), so a pass costs one barrier and no exposed
// global-memory latency. Patterns are toggled with LDS atomic xors; before
// staging a pass into a buffer, a thread toggles off the patterns it set
// there two passes earlier (xors of different threads commute).
// lut_pat(e): low nibbles 1, 2, 4, 8, 3, 5, 6, 9; high nibble 0 for e < 4, 1 << (e - 4) above.
__host__ __device__ constexpr uint32_t lut_pat(uint32_t e) {
    return ((0x96538421u >> (4 * e)) & 0xFu) | (e >= 4 ? (1u << (e - 4)) << 4 : 0u);
}
static_assert(lut_pat(0) == 0x01 && lut_pat(3) == 0x08 && lut_pat(4) == 0x13 && lut_pat(5) == 0x25 &&
                  lut_pat(6) == 0x46 && lut_pat(7) == 0x89,
              "row patterns");

__device__ __forceinline__ void lut_table_init(unsigned char *lds) {
    const uint32_t x = threadIdx.x;                           // 256 threads: row set x, one entry each
    uint32_t v = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) v ^= (x >> e & 1u) ? lut_pat(e) : 0u;
    uint4 o;
    o.x = ((x & 1u) ? 0x0100u : 0u) | ((x & 2u) ? 0x01000000u : 0u);
    o.y = ((x & 4u) ? 0x0100u : 0u) | ((x & 8u) ? 0x01000000u : 0u);
    o.z = ((x & 16u) ? 0x0100u : 0u) | ((x & 32u) ? 0x01000000u : 0u);
    o.w = ((x & 64u) ? 0x0100u : 0u) | ((x & 128u) ? 0x01000000u : 0u);
    *(uint4 *)(lds + 16 * v) = o;
    uint4 *mask = (uint4 *)(lds + kLutMaskOff);               // every row mask word starts clear
    for (uint32_t w = threadIdx.x; w < 2 * kLutMaskBytes / 16; w += 256) mask[w] = uint4{0u, 0u, 0u, 0u};
}

// One column block jb (64 stocks, 16 per wave) for the B individuals of batch pb.
// On entry every code table entry below N holds kCodeNone and every row mask
// word is 0; both are restored on exit.
template <int B>
__device__ __forceinline__ void mfma_block_lut(const InstDesc &d, int jb, int pb, int parity, unsigned char *lds,
                                               int cstride) {
    constexpr int RC = lut_rows(B);                           // rows per pass
    constexpr int NCH = RC / 32;                              // chunks per pass
    constexpr int SL = RC * B / 256;                          // (row, individual) slots per thread and pass
    constexpr uint32_t kChunkBytes = (uint32_t)B * 512;       // row mask words of one chunk
    static_assert(RC * B == 1024 && SL == 4 && NCH % 2 == 0 && NCH * kChunkBytes == kLutMaskBytes,
                  "LUT pass layout");
    const int N = d.N, P = d.P, ld = d.ld_h;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform, kept scalar
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int q = 16 * wave + n;                              // position of this lane's stock in the block
    const int jt0 = jb * kMfmaCols + 16 * wave;
    const int j = jt0 + n;
    const int pbase = pb * B;
    const int32_t *__restrict__ labels = d.pop[parity];
    const uint16_t *__restrict__ hs = d.hs;
    const uint16_t *__restrict__ ls = d.ls;
    uint8_t *const code_tab = lds + kLutCodeOff;
    auto code = [&](int b, int l) -> uint8_t & { return code_tab[(size_t)b * cstride + l]; };

    // Column labels, registered as in the column kernel (and read again at
    // the end to restore the table, rather than held in registers).
    const uint32_t lmax = (uint32_t)(N - 1);
    const int jc = min(j, N - 1);
    auto col_label = [&](int b) { return min((uint32_t)gld(labels + (size_t)min(pbase + b, P - 1) * N + jc), lmax); };
    uint32_t madr[B];
#pragma unroll
    for (int b = 0; b < B; ++b) madr[b] = col_label(b);
    if (g == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) code(b, (int)madr[b]) = (uint8_t)q;
    }
    __syncthreads();
    // LDS address of this lane's row mask word in chunk 0 of the buffer of the
    // current pass, per individual; `flip` moves it to the other buffer.
#pragma unroll
    for (int b = 0; b < B; ++b)
        madr[b] = (uint32_t)kLutMaskOff + (uint32_t)(b * 64 + code(b, (int)madr[b])) * 8u + 2u * (uint32_t)g;
    int flip = (int)kLutMaskBytes;

    floatx4 acc[B];
    double acc64[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc64[b] = 0.0;
    }
    const int dreg = n & 3;
    const bool diag_lane = (n >> 2) == g;
    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const float v = dreg == 0 ? acc[b][0] : dreg == 1 ? acc[b][1] : dreg == 2 ? acc[b][2] : acc[b][3];
            acc64[b] += (double)v;
            acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // A goes to registers one chunk ahead (two sets, by chunk parity). The
    // scaled copies are tile-major: a wave's 16 x 32 block of a part is 1 KB in
    // lane order. Only waves with jt0 < N load, and then every address is
    // inside the ld x ld copy.
    const size_t a_row = (size_t)(jt0 >> 4) * (size_t)(ld >> 5);
    auto load_a = [&](int i0, uint4 &h, uint4 &l) {
        const size_t off = (a_row + (size_t)(i0 >> 5)) * 512 + (size_t)lane * 8;
        h = gld_u4(hs + off);
        l = gld_u4(ls + off);
    };
    uint4 a0h, a0l, a1h, a1l;
    a1h = a1l = uint4{0u, 0u, 0u, 0u};

    // Staging slots of this thread: slot u is row r_u = (t + 256 u) % RC of
    // individual b_u = (t + 256 u) / RC of a pass. Per slot, fixed for the block:
    // srow (r_u), slab (label offset of row 0 of individual b_u), scod (LDS
    // address of b_u's code table), smsk (address of the slot's row mask word
    // for code 0 in the first buffer). scur / snxt: the word whose pattern the
    // slot toggled in the current pass's buffer / in the other buffer
    // (0xFFFFFFFF: none).
    const int wg_iend = min(jb * kMfmaCols + kMfmaCols, N);   // rows any wave of the group needs
    const int my_iend = jt0 < N ? min(jt0 + 16, N) : 0;       // rows this wave needs (i < j <= jt0+15)
    int srow[SL];
    uint32_t slab[SL], scod[SL], smsk[SL], scur[SL], snxt[SL], lab[SL];
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        const int s = threadIdx.x + 256 * u;
        const int b = s / RC, r = s % RC, rg = (r & 31) >> 3;
        srow[u] = r;
        slab[u] = (uint32_t)min(pbase + b, P - 1) * (uint32_t)N;
        scod[u] = (uint32_t)kLutCodeOff + (uint32_t)(b * cstride);
        smsk[u] = (uint32_t)kLutMaskOff + (uint32_t)(r >> 5) * kChunkBytes + (uint32_t)b * 512u + 4u * (uint32_t)(rg >> 1);
        scur[u] = snxt[u] = 0xFFFFFFFFu;
    }
    auto slot_pat = [&](int u) {
        const int r = srow[u], rg = (r & 31) >> 3;
        return (lut_pat((uint32_t)(r & 7)) << 4) << (16 * (rg & 1));
    };
    auto toggle = [&](uint32_t addr, int u) {
        if (addr != 0xFFFFFFFFu)
            __hip_atomic_fetch_xor((uint32_t *)(lds + addr), slot_pat(u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto load_labels = [&](int c0) {                          // rows past N are clamped (and set nothing)
#pragma unroll
        for (int u = 0; u < SL; ++u) lab[u] = (uint32_t)gld(labels + slab[u] + min(c0 + srow[u], N - 1));
    };
    // Toggle off the patterns recorded in sa, then toggle on those of the pass
    // at c0 (labels in lab) in the buffer at byte offset buf from the first,
    // recording them in sa.
    auto stage = [&](int c0, uint32_t buf, uint32_t (&sa)[SL]) {
        uint32_t cd[SL];
#pragma unroll
        for (int u = 0; u < SL; ++u) cd[u] = lds[scod[u] + min(lab[u], lmax)];
#pragma unroll
        for (int u = 0; u < SL; ++u) toggle(sa[u], u);
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            sa[u] = c0 + srow[u] < wg_iend && cd[u] != kCodeNone ? smsk[u] + buf + cd[u] * 8u : 0xFFFFFFFFu;
            toggle(sa[u], u);
        }
    };

    load_labels(0);
    stage(0, 0u, scur);
    if (RC < wg_iend) load_labels(RC);
    __syncthreads();
    // Per chunk: read the B operands (their row mask words were read during the
    // previous chunk), read the next chunk's words, load the next chunk's A
    // (two register sets by chunk parity; a pass is an even number of chunks,
    // so the parity carries over), then the MFMAs.
    if (my_iend > 0) load_a(0, a0h, a0l);
    uint32_t buf = 0;                                         // byte offset of the current pass's buffer
    for (int c0 = 0; c0 < wg_iend; c0 += RC) {
        const int cend = min(c0 + RC, my_iend);
        if (c0 < cend) {
            uint32_t idx[B];
#pragma unroll
            for (int b = 0; b < B; ++b) idx[b] = *(const uint16_t *)(lds + madr[b]);
            static_for(std::make_integer_sequence<int, NCH>{}, [&](auto chc) {
                constexpr int ch = decltype(chc)::value;
                const int i0 = c0 + 32 * ch;
                if (i0 < cend) {
                    uint4 &ch_h = (ch & 1) ? a1h : a0h, &ch_l = (ch & 1) ? a1l : a0l;
                    uint4 &nx_h = (ch & 1) ? a0h : a1h, &nx_l = (ch & 1) ? a0l : a1l;
                    // The table sits at the start of the dynamic LDS, which is LDS
                    // address 0 (the kernel has no static LDS; the launcher checks
                    // this), so a row mask word is the entry's LDS address as is.
                    pga_u32x4 bo[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) bo[b] = *(const __attribute__((address_space(3))) pga_u32x4 *)(size_t)idx[b];
                    if constexpr (ch + 1 < NCH) {
                        if (i0 + 32 < cend) {
#pragma unroll
                            for (int b = 0; b < B; ++b) idx[b] = *(const uint16_t *)(lds + madr[b] + (ch + 1) * kChunkBytes);
                        }
                    }
                    if (i0 + 32 < my_iend) load_a(i0 + 32, nx_h, nx_l);
                    if (i0 + 32 > jt0) {                          // the chunk reaches the diagonal: keep i < j
                        const int ik = i0 + 8 * g;
                        uint32_t m[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            m[r] = ((ik + 2 * r < j) ? 0xFFFFu : 0u) | ((ik + 2 * r + 1 < j) ? 0xFFFF0000u : 0u);
                        ch_h.x &= m[0]; ch_h.y &= m[1]; ch_h.z &= m[2]; ch_h.w &= m[3];
                        ch_l.x &= m[0]; ch_l.y &= m[1]; ch_l.z &= m[2]; ch_l.w &= m[3];
                    }
                    const bf16x8 Ah = __builtin_bit_cast(bf16x8, ch_h);
                    const bf16x8 Al = __builtin_bit_cast(bf16x8, ch_l);
                    // All hi products, then all lo: consecutive MFMAs are independent.
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, __builtin_bit_cast(bf16x8, bo[b]), acc[b], 0, 0, 0);
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, __builtin_bit_cast(bf16x8, bo[b]), acc[b], 0, 0, 0);
                    if (((i0 + 32) % kMfmaFlushRows) == 0) flush();
                }
            });
        }
        // Stage the next pass into the other buffer, start the label loads of
        // the pass after, then let every wave move on.
        const int cn = c0 + RC;
        if (cn < wg_iend) {
            stage(cn, buf ^ (uint32_t)kLutMaskBytes, snxt);
            if (cn + RC < wg_iend) load_labels(cn + RC);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SL; ++u) {
            const uint32_t t = scur[u];
            scur[u] = snxt[u];
            snxt[u] = t;
        }
#pragma unroll
        for (int b = 0; b < B; ++b) madr[b] += (uint32_t)flip;
        flip = -flip;
        buf ^= (uint32_t)kLutMaskBytes;
    }
    // Toggle off the patterns of the last two passes (every wave is past the last barrier).
#pragma unroll
    for (int u = 0; u < SL; ++u) {
        toggle(scur[u], u);
        toggle(snxt[u], u);
    }
    flush();
    if (diag_lane && j < N) {
        const double cjj = gld(d.C + (size_t)j * N + j);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            if (p < P) gst(d.wsum + (size_t)p * N + j, fma(2.0, acc64[b], cjj));
        }
    }
    if (g == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) code(b, (int)col_label(b)) = kCodeNone;
    }
}

// ---- labels with n_s >= 2 ------------------------------------------------------
// Bit l of word l / 32 of row p of d.ns2 is set when label l is held by at
// least two stocks of individual p (one workgroup per individual: an LDS
// histogram, then one ballot per 64 labels). Individuals evaluated by the
// cluster-pair kernel are skipped (their rows are not read). Labels outside
// [0, N) are not counted; such an individual gets -inf in the finish.
__global__ __launch_bounds__(256) void k_nsmask(Tables t, int parity) {
    extern __shared__ int ns_cnt[];
    const int gi = blockIdx.x;
    if (gi >= t.inds[t.n_inst]) return;
    const int k = find_inst(t.inds, t.n_inst, gi);
    const InstDesc &d = t.desc[k];
    if (!d.ns2 || inst_stopped(d)) return;                    // uniform
    const int p = gi - t.inds[k];
    if (d.route && gld(d.route + p) == 0) return;
    const int N = d.N;
    const int32_t *lab = d.pop[parity] + (size_t)p * N;
    for (int s = threadIdx.x; s < N; s += 256) ns_cnt[s] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += 256) {
        const int l = gld(lab + j);
        if ((unsigned)l < (unsigned)N) atomicAdd(&ns_cnt[l], 1);
    }
    __syncthreads();
    const int ldm = (N + 31) >> 5;
    uint32_t *out = d.ns2 + (size_t)p * ldm;
    for (int l0 = 64 * (threadIdx.x >> 6); l0 < N; l0 += 256) {
        const int l = l0 + (threadIdx.x & 63);
        const unsigned long long m = __ballot(l < N && ns_cnt[l] >= 2);
        if ((threadIdx.x & 63) == 0) {
            gst(out + (l0 >> 5), (uint32_t)m);
            if ((l0 >> 5) + 1 < ldm) gst(out + (l0 >> 5) + 1, (uint32_t)(m >> 32));
        }
    }
}

hipError_t launch_nsmask(Tables t, int total_inds, int max_n, int parity, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nsmask, dim3(total_inds), dim3(256), sizeof(int) * (size_t)max_n, s, t, parity);
    return hipGetLastError();
}

// LDS of one workgroup (dynamic): row codes [B][RS] (16-bit words, the code
// shifted into bits 8..15; RS = RC + 8), the label -> code tables [B][cstride]
// (bytes, cstride >= N), each wave's ring of kMfmaASlots A slots (2 KB each:
// the 16 x 32 hi tile, then the lo tile, in lane order) filled by direct
// global-to-LDS loads one chunk ahead, and 1 KB per wave for the column table
// and the flushes.
struct MfmaLdsPacked {
    uint16_t *rows;
    uint8_t *code;
    unsigned char *aring;
    uint32_t *scratch;
    int cstride;
};

__device__ __forceinline__ uint32_t shfl_xor32(uint32_t v, int m) {
    return (uint32_t)__shfl_xor((int)v, m, 64);
}

// One column block jb (64 stocks, 16 per wave) for the B individuals of batch pb.
// On entry every code table entry below N holds kCodeNone; the entries it sets
// stay set (the launching kernel clears the tables before the next block).
template <int B>
__device__ __forceinline__ void mfma_block_packed(const InstDesc &d, int jb, int pb, int parity, const MfmaLdsPacked &s) {
    constexpr int RC = mfma_rows(B);                          // rows staged per pass
    constexpr int RS = mfma_row_stride(B);
    constexpr int BU = B / 4;                                 // individuals a lane keeps: g, g + 4, ...
    const int N = d.N, P = d.P, ld = d.ld_h;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform, kept scalar
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int q = 16 * wave + n;                              // position of this lane's stock in the block
    const int jt0 = jb * kMfmaCols + 16 * wave;
    const int j = jt0 + n;
    const int pbase = pb * B;
    const int32_t *__restrict__ labels = d.pop[parity];
    const uint16_t *__restrict__ hs = d.hs;
    const uint16_t *__restrict__ ls = d.ls;
    auto code = [&](int b, int l) -> uint8_t & { return s.code[(size_t)b * s.cstride + l]; };

    // Individuals of the batch evaluated here (uniform): inside P and not taken
    // by the cluster-pair kernel.
    bool live[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int p = pbase + b;
        live[b] = p < P && !(d.route && gld(d.route + p) == 0);
    }
    // Column labels; lanes with g == 0 register them in the code table. Stock,
    // individual and label are clamped into range as in the staging below: a
    // column past N or an individual that is not live gets no column, and a
    // clamped duplicate only writes a consistent code (the position of some
    // stock with that label) into its own individual's table.
    const uint32_t lmax = (uint32_t)(N - 1);
    const int jc = min(j, N - 1);
    uint32_t lj[B];
#pragma unroll
    for (int b = 0; b < B; ++b)
        lj[b] = min((uint32_t)gld(labels + (size_t)min(pbase + b, P - 1) * N + jc), lmax);
    const int ldm = (N + 31) >> 5;
    uint32_t nsw[B];
#pragma unroll
    for (int b = 0; b < B; ++b) nsw[b] = gld(d.ns2 + (size_t)min(pbase + b, P - 1) * ldm + (lj[b] >> 5));
    if (g == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) code(b, (int)lj[b]) = (uint8_t)q;
    }
    __syncthreads();

    // Columns of this wave: per individual, the set of codes of the labels that
    // its 16 stocks here carry with n_s >= 2 (a 64-bit set, OR over the 16
    // lanes of a row group; the four row groups hold the same stocks), numbered
    // individual by individual in ascending code order. slot: this lane's
    // column per individual (-1 for none); nq column groups of 16 in all.
    uint32_t cc[B];
    int slot[B];
    int S = 0;
#pragma unroll
    for (int b = 0; b < B; ++b) {
        cc[b] = code(b, (int)lj[b]);
        const bool ns = live[b] && j < N && ((nsw[b] >> (lj[b] & 31)) & 1u);
        uint32_t lo = (ns && cc[b] < 32) ? (1u << cc[b]) : 0u;
        uint32_t hi = (ns && cc[b] >= 32) ? (1u << (cc[b] - 32)) : 0u;
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) {
            lo |= shfl_xor32(lo, m);
            hi |= shfl_xor32(hi, m);
        }
        const uint64_t M = ((uint64_t)hi << 32) | lo;
        slot[b] = ns ? S + __popcll(M & ((1ull << cc[b]) - 1ull)) : -1;
        S += __popcll(M);
    }
    const int nq = __builtin_amdgcn_readfirstlane((S + 15) >> 4);
    const int nq2 = (nq + 1) & ~1;                            // groups run in pairs
    // Column table in this wave's scratch: entry c = (individual << 8) | code,
    // kCodeFree where unused; lane n of group t takes entry 16 t + n.
    uint32_t *tbl = s.scratch + 256 * wave;
    for (int e = lane; e < 16 * B; e += 64) tbl[e] = kCodeFree;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b)
        if (slot[b] >= 0) tbl[slot[b]] = ((uint32_t)b << 8) | cc[b];
    __syncthreads();
    uint32_t col2[B], rofs[B];
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const uint32_t e = tbl[16 * t + n];
        const uint32_t c = e & 0xFFu;
        col2[t] = (c << kCodeShift) | (c << (16 + kCodeShift));
        rofs[t] = (e >> 8) * (uint32_t)RS + 8u * (uint32_t)g;   // this lane's 8 rows of that individual
    }
    // the slots of the individuals this lane keeps (b = g + 4 u)
    int myslot[BU];
    bool mylive[BU];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
        const int b0 = 4 * u;
        myslot[u] = g == 0 ? slot[b0] : g == 1 ? slot[b0 + 1] : g == 2 ? slot[b0 + 2] : slot[b0 + 3];
        mylive[u] = g == 0 ? live[b0] : g == 1 ? live[b0 + 1] : g == 2 ? live[b0 + 2] : live[b0 + 3];
    }
    __syncthreads();                                          // the table is read before any flush reuses it

    floatx4 acc[B];
    double acc64[BU];
#pragma unroll
    for (int t = 0; t < B; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < BU; ++u) acc64[u] = 0.0;

    // Flush: each group's D (this lane: rows 4g .. 4g + 3 of column n) goes to the
    // wave's scratch column-major, and each lane adds D[n][its column] of every
    // individual it keeps whose column lies in that group. LDS operations of one
    // wave complete in order, so a group's reads precede the next group's writes.
    float *fb = (float *)(s.scratch + 256 * wave);
    auto flush = [&]() {
        static_for(std::make_integer_sequence<int, B>{}, [&](auto tc) {
            constexpr int t = decltype(tc)::value;
            if (t < nq2) {
                *(floatx4 *)(fb + 16 * n + 4 * g) = acc[t];
#pragma unroll
                for (int u = 0; u < BU; ++u) {
                    const int c = myslot[u] - 16 * t;
                    if (c >= 0 && c < 16) acc64[u] += (double)fb[16 * c + n];
                }
                acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
        });
    };
    // Only waves with jt0 < N load A, and then j < ld for every lane (ld is a
    // multiple of 32 and jt0 a multiple of 16), so the loads need no guard. The
    // scaled copies are tile-major (a_tile_offset): the wave's 16 x 32 A block is
    // 1 KB of consecutive bytes in lane order.
    // Chunk i0's A goes to ring slot ((i0 - c0) / 32) % kMfmaASlots of this wave:
    // a direct global-to-LDS load puts lane l's 16 bytes at slot + 16 l, exactly
    // where the same lane reads them back.
    const size_t a_row = (size_t)(jt0 >> 4) * (size_t)(ld >> 5);
    unsigned char *const my_ring = s.aring + (size_t)wave * kMfmaASlots * 2048;
    auto slot_of = [&](int i0, int c0) { return my_ring + (size_t)(((i0 - c0) >> 5) % kMfmaASlots) * 2048; };
    auto load_a = [&](int i0, int c0) {
        const size_t off = (a_row + (size_t)(i0 >> 5)) * 512 + (size_t)lane * 8;
        unsigned char *sl = slot_of(i0, c0);
        __builtin_amdgcn_global_load_lds((const void *)(hs + off), (__attribute__((address_space(3))) void *)sl, 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void *)(ls + off), (__attribute__((address_space(3))) void *)(sl + 1024), 16,
                                         0, 0);
    };
    auto read_a = [&](int i0, int c0, uint4 &ah, uint4 &al) {
        const unsigned char *sl = slot_of(i0, c0);
        ah = *(const uint4 *)(sl + 16 * lane);
        al = *(const uint4 *)(sl + 1024 + 16 * lane);
    };
    // B column of group t: the 8 row codes of this lane's rows of the column's
    // individual against the column's code.
    auto bcol = [&](const uint16_t *rb, int t) -> bf16x8 {
        const uint4 r = *(const uint4 *)(rb + rofs[t]);
        uint4 v;
        v.x = onehot2(r.x, col2[t]);
        v.y = onehot2(r.y, col2[t]);
        v.z = onehot2(r.z, col2[t]);
        v.w = onehot2(r.w, col2[t]);
        return __builtin_bit_cast(bf16x8, v);
    };
    auto chunk = [&](auto masked_tag, int i0, int c0, uint4 ah, uint4 al) {
        constexpr bool masked = decltype(masked_tag)::value;
        if constexpr (masked) {                               // A row n is stock j: keep rows i < j
            const int ik = i0 + 8 * g;                        // first of this lane's 8 rows
            uint32_t m[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                m[r] = ((ik + 2 * r < j) ? 0xFFFFu : 0u) | ((ik + 2 * r + 1 < j) ? 0xFFFF0000u : 0u);
            ah.x &= m[0]; ah.y &= m[1]; ah.z &= m[2]; ah.w &= m[3];
            al.x &= m[0]; al.y &= m[1]; al.z &= m[2]; al.w &= m[3];
        }
        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah);
        const bf16x8 Al = __builtin_bit_cast(bf16x8, al);
        const uint16_t *rb = s.rows + (i0 - c0);
        // groups in pairs (the hi and lo MFMAs of one group depend on each other;
        // the other group's fill the gap); an odd last group is paired with
        // free columns, whose sums are 0
        static_for(std::make_integer_sequence<int, B / 2>{}, [&](auto hc) {
            constexpr int t = 2 * decltype(hc)::value;
            if (t < nq) {                                     // uniform
                const bf16x8 B0 = bcol(rb, t);
                const bf16x8 B1 = bcol(rb, t + 1);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B0, acc[t], 0, 0, 0);
                acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B1, acc[t + 1], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B0, acc[t], 0, 0, 0);
                acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B1, acc[t + 1], 0, 0, 0);
            }
        });
        if (((i0 + 32) % kMfmaFlushRows) == 0) flush();
    };
    // Chunks [i0, end) of one kind. A chunk first reads its A from LDS (loaded
    // during the previous chunk), then starts the load of the next chunk's A
    // into the other slot, then computes.
    auto run = [&](auto masked_tag, int &i0, int end, int cend, int c0) {
        for (; i0 < end; i0 += 32) {
            uint4 ah, al;
            read_a(i0, c0, ah, al);
            if (i0 + 32 < cend) load_a(i0 + 32, c0);
            chunk(masked_tag, i0, c0, ah, al);
        }
    };

    const int wg_iend = min(jb * kMfmaCols + kMfmaCols, N);   // rows any wave of the group needs
    const int my_iend = (jt0 < N && nq > 0) ? min(jt0 + 16, N) : 0;   // rows this wave needs (i < j <= jt0+15)
    const int i_diag = (jt0 / 32) * 32;                       // first chunk that may hold i >= j

    for (int c0 = 0; c0 < wg_iend; c0 += RC) {
        const int rows = min(RC, wg_iend - c0);
        const int rows32 = (rows + 31) & ~31;                 // chunks read whole 32-row groups
        // Thread t stages row pairs t + 256k of every individual: all 2 * PK * B
        // labels are loaded before the first table lookup, so the pass costs one
        // memory latency; each row pair of an individual is one dword.
        // Nothing here needs a validity test, only in-bounds addresses: rows past
        // the pass (only past N, in its last 32-row chunk) meet zero-padded A;
        // individuals that are not live have no column; a label outside [0, N)
        // makes the finish kernel give its individual -inf whatever its sums. So
        // row and individual indices are clamped into range, and labels to N - 1.
        constexpr int PK = RC / 512;
        const uint32_t rlast = (uint32_t)(rows - 1);
        uint32_t lab[PK][2][B];
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const uint32_t r = 2u * (uint32_t)(threadIdx.x + 256 * k);
            const uint32_t r0 = min(r, rlast), r1 = min(r + 1u, rlast);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int32_t *lp = labels + (size_t)min(pbase + b, P - 1) * N + c0;   // uniform
                lab[k][0][b] = (uint32_t)gld(lp + r0);
                lab[k][1][b] = (uint32_t)gld(lp + r1);
            }
        }
#pragma unroll
        for (int k = 0; k < PK; ++k)                          // all table reads, then all writes
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int b = 0; b < B; ++b) lab[k][h][b] = code(b, (int)min(lab[k][h][b], lmax));
#pragma unroll
        for (int k = 0; k < PK; ++k) {
            const int qd = threadIdx.x + 256 * k;
            if (2 * qd < rows32) {
#pragma unroll
                for (int b = 0; b < B; ++b)                   // code of row 2qd in bits 8..15, of 2qd+1 in 24..31
                    *(uint32_t *)(s.rows + (size_t)b * RS + 2 * qd) =
                        (lab[k][0][b] << kCodeShift) | (lab[k][1][b] << (16 + kCodeShift));
            }
        }
        __syncthreads();
        const int cend = min(c0 + RC, my_iend);
        if (c0 < cend) {
            load_a(c0, c0);
            int i0 = c0;
            const int uend = min(cend, max(c0, i_diag));        // chunks entirely below the diagonal
            run(std::false_type{}, i0, uend, cend, c0);
            run(std::true_type{}, i0, cend, cend, c0);
        }
        __syncthreads();
    }
    flush();
    if (j < N) {
        const double cjj = gld(d.C + (size_t)j * N + j);
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            const int p = pbase + g + 4 * u;
            if (mylive[u]) gst(d.wsum + (size_t)p * N + j, fma(2.0, acc64[u], cjj));
        }
    }
}

// The triangle is folded: column blocks n_jb-1-jp and jp share a workgroup, so every
// workgroup processes the same number of row chunks.
template <int B, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    KIND == kKindLut ? (B == 8 ? 2 : 3) : (B == 16 ? 2 : 4)))) void k_pairsum_mfma(Tables t, int parity,
                                                                                     int order, int cstride) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int total = t.tiles[t.n_inst];                  // the grid may exceed it (capacity-sized graph)
    if ((int)blockIdx.x >= total) return;
    const int tile = order ? xcd_tile(blockIdx.x, total) : blockIdx.x;
    const int k = find_inst(t.tiles, t.n_inst, tile);
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;                              // uniform over the workgroup
    const int local = tile - t.tiles[k];
    const int n_jb = (d.N + kMfmaCols - 1) / kMfmaCols;
    const int n_pairs = (n_jb + 1) / 2;
    const TilePos tp = tile_pos(local, n_pairs, (d.P + B - 1) / B, order);
    const int jp = tp.jp, pb = tp.pb;
    if (d.route) {                                            // uniform: skip batches the cluster-pair
        int any = 0;                                          // kernel evaluated entirely
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (pb * B + b < d.P) any |= gld(d.route + pb * B + b);
        if (!any) return;
    }
    // Label -> code tables: every entry set to kCodeNone (B tables of cstride bytes,
    // one contiguous, 16-byte aligned region; cstride >= N is a multiple of 16). The
    // column and packed blocks leave their entries set, and the tables are cleared
    // again between the two blocks of a folded pair (a block's last reads of them
    // precede the barrier that closes its row loop); the LUT block restores its own
    // entries.
    uint8_t *code = lds + mfma_lds_code_off(B, KIND);
    auto clear_codes = [&]() {
        const int n16 = B * cstride / 16;
        for (int i = threadIdx.x; i < n16; i += 256)
            *(uint4 *)(code + 16 * (size_t)i) = uint4{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    };
    clear_codes();
    if constexpr (KIND == kKindLut) lut_table_init(lds);
    __syncthreads();
    if constexpr (KIND == kKindPacked) {
        const MfmaLdsPacked s{(uint16_t *)lds, code, lds + mfma_lds_ring_off(B, cstride, KIND),
                              (uint32_t *)(lds + mfma_lds_scratch_off(B, cstride, KIND)), cstride};
        mfma_block_packed<B>(d, n_jb - 1 - jp, pb, parity, s);
        if (jp != n_jb - 1 - jp) {
            clear_codes();
            __syncthreads();
            mfma_block_packed<B>(d, jp, pb, parity, s);
        }
    } else if constexpr (KIND == kKindLut) {
        mfma_block_lut<B>(d, n_jb - 1 - jp, pb, parity, lds, cstride);
        if (jp != n_jb - 1 - jp) {
            __syncthreads();
            mfma_block_lut<B>(d, jp, pb, parity, lds, cstride);
        }
    } else {
        const MfmaLdsCols s{(uint32_t *)lds, code, lds + mfma_lds_ring_off(B, cstride, KIND), cstride};
        mfma_block_cols<B>(d, n_jb - 1 - jp, pb, parity, s);
        if (jp != n_jb - 1 - jp) {
            clear_codes();
            __syncthreads();
            mfma_block_cols<B>(d, jp, pb, parity, s);
        }
    }
}

// The LUT kernel addresses its table by absolute LDS address, which requires
// the dynamic LDS to start at address 0: no static LDS in the kernel.
template <int B, int KIND>
bool mfma_static_lds_ok() {
    if constexpr (KIND != kKindLut) {
        return true;
    } else {
        static const bool ok = [] {
            hipFuncAttributes a{};
            return hipFuncGetAttributes(&a, reinterpret_cast<const void *>(&k_pairsum_mfma<B, KIND>)) == hipSuccess &&
                   a.sharedSizeBytes == 0;
        }();
        return ok;
    }
}

template <int KIND>
hipError_t launch_mfma_b(Tables t, int total_tiles, int parity, int ipg, int order, int cstride, size_t lds,
                         hipStream_t s) {
    if (ipg == 8) {
        if (!mfma_static_lds_ok<8, KIND>()) return hipErrorInvalidKernelFile;
        hipLaunchKernelGGL((k_pairsum_mfma<8, KIND>), dim3(total_tiles), dim3(256), lds, s, t, parity, order, cstride);
    } else if (ipg == 4) {
        if (!mfma_static_lds_ok<4, KIND>()) return hipErrorInvalidKernelFile;
        hipLaunchKernelGGL((k_pairsum_mfma<4, KIND>), dim3(total_tiles), dim3(256), lds, s, t, parity, order, cstride);
    } else if (ipg == 16 && KIND != kKindLut) {               // the LUT kernel has no 16-individual form
        if constexpr (KIND != kKindLut)
            hipLaunchKernelGGL((k_pairsum_mfma<16, KIND>), dim3(total_tiles), dim3(256), lds, s, t, parity, order,
                               cstride);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pairsum_mfma(Tables t, int total_tiles, int parity, const Variant &v, int max_n,
                               hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    if (!variant_ok(v, max_n)) return hipErrorInvalidValue;
    const int cstride = (int)mfma_code_stride(max_n);
    const size_t lds = mfma_lds_bytes(v.ipg, max_n, v.kind);
    if (v.kind == kKindPacked) return launch_mfma_b<kKindPacked>(t, total_tiles, parity, v.ipg, v.order, cstride, lds, s);
    if (v.kind == kKindLut) return launch_mfma_b<kKindLut>(t, total_tiles, parity, v.ipg, v.order, cstride, lds, s);
    return launch_mfma_b<kKindCols>(t, total_tiles, parity, v.ipg, v.order, cstride, lds, s);
}

// ---- scaled split parts ----------------------------------------------------------
// hs = hi * 2^125, ls = lo * 2^125 over the ld x ld split of every instance
// (blockIdx.y), stored tile-major: the 16 x 32 block of rows 16 tj.. and columns
// 32 ti.. is 512 consecutive elements at (tj * ld / 32 + ti) * 512, element
// (16 tj + n, 32 ti + 8 g + e) at (16 g + n) * 8 + e, i.e. in the order the
// lanes (16 g + n) of the pair-sum wave read them. The scaling is exact:
// |hi|, |lo| <= 1, so the result is a normal bf16 with the same significand
// (NaN and infinities stay so).
__device__ __forceinline__ uint32_t scale2(uint32_t w) {
    const float a = __uint_as_float(w << 16) * 0x1p125f;
    const float b = __uint_as_float(w & 0xFFFF0000u) * 0x1p125f;
    return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xFFFF0000u);
}

__global__ __launch_bounds__(256) void k_scale_split(Tables t) {
    const InstDesc &d = t.desc[blockIdx.y];
    if (d.P == 0) return;                                     // a padding slot of a capacity-sized launch
    const size_t n8 = (size_t)d.ld_h * d.ld_h / 8;            // ld is a multiple of 32
    const size_t ld = (size_t)d.ld_h;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < n8; v += (size_t)gridDim.x * 256) {
        const size_t row = 8 * v / ld, col = 8 * v % ld;   // 8 consecutive columns of one row
        const size_t dst = ((row >> 4) * (ld >> 5) + (col >> 5)) * 512 + ((((col & 31) >> 3) << 4) + (row & 15)) * 8;
        const uint4 h = gld_u4(d.hi + 8 * v);
        const uint4 l = gld_u4(d.lo + 8 * v);
        const pga_u32x4 hs = {scale2(h.x), scale2(h.y), scale2(h.z), scale2(h.w)};
        const pga_u32x4 ls = {scale2(l.x), scale2(l.y), scale2(l.z), scale2(l.w)};
        *(PGA_GLOBAL pga_u32x4 *)(d.hs + dst) = hs;
        *(PGA_GLOBAL pga_u32x4 *)(d.ls + dst) = ls;
    }
}

hipError_t launch_scale_split(Tables t, int max_ld, hipStream_t s) {
    if (t.n_inst <= 0 || max_ld <= 0) return hipSuccess;
    const size_t n8 = (size_t)max_ld * max_ld / 8;
    const int gx = (int)std::min<size_t>((n8 + 255) / 256, 1024);
    hipLaunchKernelGGL(k_scale_split, dim3(gx, t.n_inst), dim3(256), 0, s, t);
    return hipGetLastError();
}

}  // namespace pga

// Internal declarations shared by the libpga translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pga.h"

namespace pga {

// Device-side descriptor of one GA instance (or of one pga_fitness call).
// Written into the workspace before the kernels run; every kernel finds its
// instance through it, so the same kernels serve one instance or a ragged
// batch, and a captured HIP graph stays valid when pointers change.
struct InstDesc {
    int32_t N, P, E, ld_h;
    const double *C;
    const uint16_t *hi, *lo;    // BF16 split parts (ld_h x ld_h)
    uint16_t *hs, *ls;          // split parts times 2^125, tile-major (workspace; BF16x2 form only)
    int32_t *pop[2];            // ping-pong population buffers
    double *fitness;            // P
    double *stats;              // (G + 1) x 4 or null
    double *wsum;               // P x N: v_pj = C_jj + 2 sum_{i<j} [s_pi = s_pj] C_ij
    int32_t *elite;             // PGA_E_MAX
    int32_t *n_s_out;           // P x N or null
    double *c_s_out;            // P x N or null
    uint32_t p_cross, p_mut;
    uint64_t seed;
    uint32_t inst_id, gen0;
    pga_term_state *term;       // termination state or null
    int32_t stall_gens;         // 0: no termination test
    int32_t ind0;               // first global individual index
    double tol;
    int32_t selection;          // PGA_SELECT_*
    int32_t pad_;
    int32_t *sus_rank;          // P: 1-based rank (SUS only; workspace)
    uint64_t *sus_cum;          // P: inclusive prefix of the SUS weights (workspace)
    int32_t *route;             // P: 1 = evaluated by pair-sum + finish, 0 = by the cluster-pair
                                // kernel (workspace); null: every individual takes the pair-sum
    double *diag;               // N + 1: C_jj, contiguous, then 1 if every C_jj is 1 (workspace; with route)
    uint32_t *ns2;              // P x ceil(N / 32): bit l set when label l has n_s >= 2 (workspace; BF16x2 form)
};

// Prefix tables: for n instances, arrays of n + 1 exclusive prefix sums.
struct Tables {
    const InstDesc *desc;
    const int32_t *tiles;       // prefix of pair-sum tiles (of the kernel variant in use)
    const int32_t *inds;        // prefix of individuals
    int32_t *sq;                // route list counters (see list_count)
    int32_t *sq_list;           // route list entries (see list_entry)
    int32_t n_inst;
};

// Workgroups of one launch are handed to the eight XCDs in turn (workgroup i
// to XCD i mod 8), each XCD with its own L2.
constexpr int kXcds = 8;

// Route lists. With the cluster-pair route on, an evaluation of the population
// of parity q sorts its individuals into two lists: those the cluster-pair
// kernel evaluates (kListSparse) and those the pair-sum and finish evaluate
// (kListDense), so that each of those launches has a workgroup per listed
// individual only. A list is cut into kListSlices slices with a counter each,
// so that its appends do not all meet on one address; an entry is the pair
// (index in the instance, instance). The route kernel of parity q fills the
// lists of q and empties those of 1 - q, which the evaluation before it used.
constexpr int kListSlices = 1024;
constexpr int kListSparse = 0, kListDense = 1;
constexpr int kListCounters = 4 * kListSlices;     // [parity][list][slice]
// Slices in use for a route launch of n_wg four-individual workgroups (one per
// workgroup up to kListSlices, so the list launches of a small population are
// no larger than a workgroup per individual), and entries per slice.
__host__ __device__ constexpr int list_slices(int n_wg) {
    return n_wg < 1 ? 1 : (n_wg < kListSlices ? n_wg : kListSlices);
}
__host__ __device__ constexpr int list_slice_cap(int n_wg) {
    return 4 * ((n_wg + list_slices(n_wg) - 1) / list_slices(n_wg));
}
// int32 words of both lists' entries
__host__ __device__ constexpr size_t list_words(int n_wg) {
    return (size_t)2 * 2 * kListSlices * (size_t)list_slice_cap(n_wg);
}

// ---- geometry of the pair-sum kernels --------------------------------------
constexpr int kFp64Waves = 4;                      // waves per workgroup, one column (stock) per lane
constexpr int kFp64Cols = 64;                      // columns per workgroup
constexpr int kMfmaWaves = 4;                      // waves per workgroup, 16 columns each
constexpr int kMfmaCols = 16 * kMfmaWaves;         // columns per workgroup
constexpr int kMfmaRowCodes = 8192;                // row codes staged in LDS per workgroup (column kernel)
constexpr int kMfmaFlushRows = 512;                // FP32 accumulators are flushed to FP64 every 512 rows
constexpr int kMaxLdsBytes = 65536;                // LDS a workgroup may allocate
// Fourth word of a raw buffer descriptor (no swizzle, no stride, 32-bit data
// format): byte addressing from the base, loads past num_records return zero.
constexpr int kBufWord3 = 0x00020000;

inline int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }
// Pair-sum tiles fold the triangle: column blocks jb and n_jb - 1 - jb share a workgroup.
inline int32_t fold_pairs(int32_t N, int32_t cols) { return (ceil_div(N, cols) + 1) / 2; }
inline int32_t split_ld(int32_t N) { return (int32_t)(((int64_t)N + 31) / 32 * 32); }

// A pair-sum kernel variant (what the autotuner chooses between):
//   ipg    individuals per group: per wave in the FP64 kernel (the workgroup
//          holds 4 x ipg), per workgroup in the MFMA kernel;
//   order  tile order: 0 workgroup b runs tile b, column pairs fastest;
//          1 tiles renumbered so each XCD gets a contiguous range, column
//          pairs fastest (an XCD sees few individual batches, all columns);
//          2 as 1 with individual batches fastest (an XCD sees few column
//          pairs, so their C rows stay in its L2);
//   kind   MFMA form only: how the B operand (the one-hot) is made and how
//          many columns there are:
//          kKindCols   one column per stock, one-hot built in registers from
//                      row codes (a DPP broadcast, an xor and a saturating
//                      subtract per two elements);
//          kKindPacked compacted columns (one per label with n_s >= 2, packed
//                      over the workgroup's individuals), one-hot built in
//                      registers from each lane's own row codes;
//          kKindLut    one column per stock, one-hot read from LDS: an 8-bit
//                      row mask per (individual, label code, row group) indexes
//                      a 256-entry table of bf16 one-hot octets.
// Every variant performs the same arithmetic in the same order per
// individual, so all of them give bitwise identical results.
constexpr int32_t kKindCols = 0, kKindPacked = 1, kKindLut = 2;
struct Variant {
    int32_t form, ipg, order, kind;
};
int n_variants(int form);
Variant variant_at(int form, int idx);
inline int32_t pair_tiles(int32_t N, int32_t P, const Variant &v) {
    const int per = v.form == PGA_FORM_FP64 ? kFp64Waves * v.ipg : v.ipg;
    return fold_pairs(N, 64) * ceil_div(P, per);
}
inline size_t mfma_code_stride(int max_n) { return ((size_t)max_n + 15) / 16 * 16; }
constexpr int kMfmaASlots = 2;                     // A ring slots per wave (2 KB each) in the MFMA kernel
// Rows of row codes staged per pass and individual by the packed kernel (a
// multiple of 512), and the per-individual stride of its staged codes in 16-bit
// words (16 bytes of padding).
__host__ __device__ constexpr int mfma_rows(int ipg) { return 4096 / ipg > 512 ? 4096 / ipg : 512; }
__host__ __device__ constexpr int mfma_row_stride(int ipg) { return mfma_rows(ipg) + 8; }
// LDS of the MFMA kernels.
// Column and packed kernels: row codes (the column kernel: kMfmaRowCodes words
// for all individuals; the packed kernel: [ipg][stride]), label -> code tables,
// A rings, and for the packed kernel 1 KB per wave of scratch.
// LUT kernel, at fixed offsets: the one-hot table (256 x 16 bytes), two
// buffers of row masks (16 KB each: [chunk][ipg][64 codes][4 row groups]
// 16-bit words of lut_rows(ipg) rows, one pass), then the label -> code tables.
__host__ __device__ constexpr size_t mfma_align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kLutTableBytes = 256 * 16;
constexpr size_t kLutMaskOff = kLutTableBytes;
constexpr size_t kLutMaskBytes = 16384;             // one buffer
constexpr size_t kLutCodeOff = kLutMaskOff + 2 * kLutMaskBytes;
__host__ __device__ constexpr int lut_rows(int ipg) { return (int)(kLutMaskBytes / 512) * 32 / ipg; }
__host__ __device__ constexpr size_t mfma_lds_code_off(int ipg, int kind) {
    return kind == kKindLut      ? kLutCodeOff
           : kind == kKindPacked ? mfma_align256(sizeof(uint16_t) * (size_t)ipg * mfma_row_stride(ipg))
                                 : sizeof(uint16_t) * (size_t)kMfmaRowCodes;
}
__host__ __device__ constexpr size_t mfma_lds_ring_off(int ipg, int cstride, int kind) {
    return mfma_lds_code_off(ipg, kind) + mfma_align256((size_t)ipg * cstride);
}
__host__ __device__ constexpr size_t mfma_lds_scratch_off(int ipg, int cstride, int kind) {
    return mfma_lds_ring_off(ipg, cstride, kind) + (size_t)kMfmaWaves * kMfmaASlots * 2048;
}
inline size_t mfma_lds_bytes(int ipg, int max_n, int kind) {
    const int cstride = (int)mfma_code_stride(max_n);
    if (kind == kKindLut) return kLutCodeOff + (size_t)ipg * cstride;
    return mfma_lds_scratch_off(ipg, cstride, kind) + (kind == kKindPacked ? (size_t)kMfmaWaves * 1024 : 0);
}
static_assert(mfma_lds_code_off(4, kKindPacked) % 256 == 0 && mfma_lds_code_off(8, kKindPacked) % 256 == 0 &&
                  mfma_lds_code_off(16, kKindPacked) % 256 == 0 && mfma_lds_code_off(8, kKindCols) % 256 == 0 &&
                  kLutMaskOff % 256 == 0 && kLutCodeOff % 256 == 0,
              "MFMA LDS regions are 256-byte aligned");
static_assert(lut_rows(4) % 32 == 0 && lut_rows(8) % 32 == 0 && lut_rows(16) % 32 == 0 &&
                  lut_rows(8) * 8 / 32 * 512 == (int)kLutMaskBytes,
              "a LUT pass is whole 32-row chunks and its row masks fill the mask region");
inline bool variant_ok(const Variant &v, int max_n) {
    return v.form != PGA_FORM_BF16X2 ||
           (mfma_lds_bytes(v.ipg, max_n, v.kind) <= (size_t)kMaxLdsBytes && (v.kind != kKindLut || v.ipg <= 8));
}

struct TilePos {
    int jp, pb;
};
// (column pair, individual batch) of tile `local` of an instance.
__device__ __forceinline__ TilePos tile_pos(int local, int n_pairs, int n_pb, int order) {
    if (order == 2) return TilePos{local / n_pb, local % n_pb};
    return TilePos{local % n_pairs, local / n_pairs};
}

// Workgroup b of T runs tile xcd_tile(b, T): the hardware deals workgroups to
// the 8 XCDs round-robin (b mod 8), so XCD x receives the contiguous tiles
// [start_x, start_x + count_x) and shares their labels in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int T) {
    const int q = T >> 3, r = T & 7, x = b & 7, i = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) ---------------------
enum : uint32_t { kTagInit = 0, kTagSel = 1, kTagXov = 2, kTagMut = 3, kTagSus = 4, kTagShuf = 5 };

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(uint32_t blk, uint32_t who, uint32_t gen, uint32_t tag,
                                   uint32_t inst, uint64_t seed) {
    return philox4x32_10(blk, who, gen, tag | (inst << 4), (uint32_t)seed, (uint32_t)(seed >> 32));
}

// floor(w * m / 2^32)
__device__ __forceinline__ uint32_t scale_u32(uint32_t w, uint32_t m) { return __umulhi(w, m); }

// ---- explicit global-memory access ------------------------------------------
// Pointers read from a descriptor are generic; the compiler then emits flat
// loads, which count on the same wait counter as LDS operations, so a wait for
// an LDS result would also wait for every in-flight prefetch. These helpers
// access global memory through address-space-1 pointers (global loads/stores).
#define PGA_GLOBAL __attribute__((address_space(1)))
typedef uint32_t pga_u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gld(const T *p) { return *(const PGA_GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ void gst(T *p, T v) { *(PGA_GLOBAL T *)p = v; }
__device__ __forceinline__ uint4 gld_u4(const void *p) {
    const pga_u32x4 v = *(const PGA_GLOBAL pga_u32x4 *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Instance lookup: largest k with prefix[k] <= t (prefix is exclusive, n + 1 entries).
__device__ __forceinline__ int find_inst(const int32_t *prefix, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// A stopped instance (termination test fired) is skipped by every kernel.
__device__ __forceinline__ bool inst_stopped(const InstDesc &d) {
    return d.term != nullptr && gld(&d.term->stopped) != 0;
}

// Total order used for ranking, elites and tournaments: higher fitness first,
// then lower index. -inf compares equal to -inf, so ties among invalid
// individuals also go to the lower index.
__device__ __forceinline__ bool ranks_before(double fa, int a, double fb, int b) {
    return fa > fb || (fa == fb && a < b);
}

// Cluster-pair route limit of an instance of N stocks: frac N (N - 1) / 2 pairs,
// and every pair when N <= 64 (a 64-stock block is the pair-sum's smallest unit
// of work per individual, and its finish a workgroup per individual, while the
// cluster-pair evaluation is bounded by the N (N - 1) / 2 <= 2016 pairs).
constexpr int kRouteAllPairsMaxN = 64;
__host__ __device__ __forceinline__ double route_limit(int N, double frac) {
    const double all = 0.5 * (double)N * (double)(N - 1);
    return N <= kRouteAllPairsMaxN ? all : floor(frac * all);
}

__device__ __forceinline__ int32_t *list_count(const Tables &t, int parity, int list, int slice) {
    return t.sq + (2 * parity + list) * kListSlices + slice;
}
__device__ __forceinline__ int32_t *list_entry(const Tables &t, int list, int slice, int cap, int at) {
    return t.sq_list + 2 * (((size_t)list * kListSlices + slice) * cap + at);
}
// Individual p of instance k (global index g) joins list L of `parity` in the
// slice of its four-individual group, g / 4 mod slices, with its route flag
// (one thread). A slice then holds at most the list_slice_cap individuals of
// its groups, whichever kernel classified them.
__device__ __forceinline__ void route_append(const Tables &t, const InstDesc &d, int k, int p, int g, int parity,
                                             int L, int slices, int cap) {
    gst(d.route + p, L == kListSparse ? 0 : 1);
    const int slice = (g >> 2) % slices;
    int32_t *e = list_entry(t, L, slice, cap, atomicAdd(list_count(t, parity, L, slice), 1));
    gst(e, p);
    gst(e + 1, k);
}

// ---- launchers (defined in the kernel translation units) ---------------------
hipError_t launch_row_stats(const double *R, int N, int T, int64_t ld, double *mu, double *ss,
                            int32_t *status, hipStream_t s);
hipError_t launch_corr(const double *R, int N, int T, int64_t ld, const double *mu, const double *ss,
                       double *C, double *part, hipStream_t s);
size_t gram_ws_doubles(int N);      // partial Gram tiles of the FP64 MFMA Gram (correlation, EWMA)
hipError_t launch_split(const double *C, int N, uint16_t *hi, uint16_t *lo, hipStream_t s);
hipError_t launch_ewma(const double *R, int N, int T, int64_t ld, double lam, int reset, int market, double *S,
                       double *C, double *X, double *part, int32_t *status, hipStream_t s);

hipError_t launch_write_desc(const InstDesc &d, int32_t tiles, InstDesc *dst, int32_t *prefix2, hipStream_t s);
hipError_t launch_pairsum_fp64(Tables t, int total_tiles, int parity, const Variant &v, hipStream_t s);
hipError_t launch_pairsum_mfma(Tables t, int total_tiles, int parity, const Variant &v, int max_n,
                               hipStream_t s);
hipError_t launch_scale_split(Tables t, int max_ld, hipStream_t s);
hipError_t launch_nsmask(Tables t, int total_inds, int max_n, int parity, hipStream_t s);
// listed: evaluate the dense route list of this parity (cluster-pair route on), else every individual.
hipError_t launch_finish(Tables t, int total_inds, int max_n, int parity, int listed, int32_t *status, hipStream_t s);
hipError_t launch_diag(Tables t, int max_n, hipStream_t s);
// listed: route lists (kManyInds individuals or more), filled by the route kernel unless the breed
// launch before already did (lists_ready); else a workgroup per individual.
hipError_t launch_sparse(Tables t, int total_inds, int max_n, int parity, double frac, int listed, int lists_ready,
                         int32_t *status, hipStream_t s);

hipError_t launch_init(Tables t, int total_inds, hipStream_t s);
hipError_t launch_rank(Tables t, int gen_off, int final, hipStream_t s);
// by_wave: one wave per slot instead of one workgroup per slot.
// classify (wave form, route lists in use, largest N <= 64): each slot's writer
// appends the new individual to the next evaluation's sparse list, so that
// evaluation needs no route kernel.
hipError_t launch_breed(Tables t, int total_inds, int parity, int gen_off, int fold, int by_wave, int max_n,
                        int classify, hipStream_t s);
// Launches of at least kManyInds individuals (more than the chip holds at a
// workgroup each) take the per-individual kernels' throughput forms: the
// route lists and one wave per breed slot. Smaller ones (a serving batch, one
// instance of a few thousand) are latency-bound: there a route launch is a
// step more on every generation, and a workgroup per slot finishes sooner.
constexpr int kManyInds = 8192;
// Largest N bred with one wave per slot: above it a workgroup per slot keeps more
// genes of one child in flight.
constexpr int kBreedWaveMaxN = 1024;
hipError_t launch_sus(Tables t, int max_p, hipStream_t s);
hipError_t launch_copy_back(Tables t, int total_inds, int G, hipStream_t s);
// Records a hipError_t for pga_last_hip_error() on this thread.
void note_hip_error(int e);

// pga_fitness with a choice of whether launches may be event-timed (the
// allocation-free entry point passes false).
int fitness_call(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N, const int32_t *labels,
                 int32_t P, int32_t form, double *fitness, int32_t *n_s, double *c_s, int32_t *status, void *ws,
                 size_t ws_bytes, hipStream_t s, bool timing_allowed);

hipError_t launch_best(const double *fitness, const int32_t *labels, int P, int N, int32_t *out,
                       double *out_f, hipStream_t s);

}  // namespace pga

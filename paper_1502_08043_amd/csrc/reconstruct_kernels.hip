// Reconstruction of <ij|kl> from the per-node tables (Eq. 14):
//   <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q tau_q(o_x) tau_q(o_y) tau_q(o_z),
// o_d = (m_d, m'_d) = ((n_k - n_i)_d, (n_l - n_j)_d).
//
// Layout.  tau is symmetric under (m, m') -> (m', m) and (m, m') -> (-m, -m'),
// so the table is stored folded: E orbit representatives per node (about a
// quarter of nd^2).  A rectangular box stacks its three direction tables
// (E = 3 E1 rows, direction d at rows d E1 ..), and the decode offsets each
// direction's entry into its own table; the passes see one taller slab.
// In HBM the folded table is [E][Qp]: the Qp (Q padded to a multiple of 32,
// zero) node values of one entry are contiguous.  Each entry
// carries W_q^(1/3) (the mesh weights are positive), so a node term is the
// plain product of three entries.
//
// Schedule: node passes.  The node range is cut into P passes of c nodes,
// small enough for the [E][c] slab to sit in LDS.  Pass p is one launch of a
// persistent grid; every workgroup stages slab p once and then streams every
// quadruple through it.  The quadruples are first decoded into their three
// folded-entry indices (4 bytes when E <= 1024, else 8, kept in a scratch
// array); each pass adds its c node terms to an FP64 partial sum kept in the
// output array, and the last pass applies 1/(sqrt(pi) L).  Table refills
// from L2 are thus paid once per workgroup and pass, and the per-quadruple
// traffic is a plain HBM stream.
//
// Lanes.  G lanes share one quadruple and each lane owns W 16-byte words
// (2W nodes) of every row, c = 2 G W: word s + G k of chunk k.  Each row
// read of a quadruple is W aligned runs of G words.  LDS serves a 16-lane phase of a 128-bit read in one
// sweep of its 64 banks (256 bytes) when the phase's addresses fall in
// distinct banks, so the layouts differ in how often a phase clashes:
//   G = 16: a phase is one run of 256 bytes, always conflict-free;
//   G = 8, W = 2: rows are 256 bytes; odd groups read their chunks in the
//           opposite order, so the two runs of a phase are opposite halves;
//   G = 8, W = 1: rows are 128 bytes, a phase holds two rows that clash when
//           both sit in the same half, i.e. when their entry indices have
//           equal parity;
//   G = 4, W = 2: rows are 128 bytes read as two 64-byte quarters, odd groups
//           second chunk first; groups 0 and 2 (1 and 3) of a phase clash when
//           their entry indices have equal parity;
//   G = 4, W = 1: four random 64-byte quarters per phase;
//   G = 2, W = 4: rows are 128 bytes read as four 32-byte runs, group g
//           taking chunk k ^ (g mod 4) at step k; groups g and g + 4 of a
//           phase clash when their entry indices have equal parity;
//   G = 1, W = 8: one lane per quadruple, word k ^ (g mod 8) at step k;
//           lanes g and g + 24 (g + 8 and g + 16) of a 32-lane half-wave
//           clash on equal row parity (pair_lane below).
// The decode stores each quadruple's entries in ascending parity.  With
// several lanes per quadruple, the groups that may clash hold quadruples of
// different stream position (bit log2(8 / G) of e), and the stream word of
// one of them is stored in descending order instead, which puts opposite
// halves together where it can.  The one-lane passes pair their lanes
// themselves (pair_lane): a wave's quadruples are dealt so that the lanes
// that can clash hold complementary parity counts.
// Each lane accumulates one partial sum per quadruple of its group (R); a
// butterfly of DPP exchanges inside the 16-lane row halves the set at each
// step, so that after log2(G) steps lane s holds the full sum of one
// quadruple, which it writes.
//
// First pass.  All layouts with c = 16 read the same [E][16] slab, and a
// quadruple's packed word depends on its stream position only, so the first
// pass of such a table runs in the one-lane layout (G = 1, W = 8) and
// decodes the stream itself, the basis and fold map sitting in LDS beside
// the slab; the later passes use the table's layout, for whose lane groups
// the decode orders the entries.  Other tables decode in k_decode first.
//
// Fused schedule.  When the table's layout is the one-lane one and the
// basis and fold map fit in LDS beside its slab, one launch does all the
// passes (k_rec_fused): a workgroup decodes a chunk of 8 quadruples per
// lane (6 when the slab takes 8 words per lane) into registers, keeps their
// partial sums there, and for each node range restages the slab from L2
// (the whole folded table, 0.56 MB at 9171 planewaves and Q = 96, stays
// resident there) and adds its terms.  The stream is then read once and the
// results written once (24 bytes per quadruple instead of 28 + 20 per later
// pass), no decoded stream is stored, the next range's slab is loaded into
// registers while the current one is read, and the next chunk's quadruples
// while the last range is (with several ranges, decoded beside its reads).
// Larger chunks spill registers.  A last range with fewer real nodes reads
// only its first 1, 2 or 4 words.  With several
// ranges the chunk's quadruples are paired wave-wide (pair_wave) rather than
// slot by slot: a lane's position sets the order of its word reads and of
// each triple product, so the two schedules agree to that rounding, and
// bit for bit with one range.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "ffloat.h"
#include "pwc_internal.h"

// Fixed scratch of pwc_reconstruct_noalloc: the decoded-quadruple stream of
// one call, for callers that cannot allocate.  Every device that runs the
// library holds its own copy until the process ends.  In host code this name
// is a host-side stand-in, not a device address: host code uses only the
// address hipGetSymbolAddress returns for the current device
// (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[pwc::kNoAllocScratchBytes];

namespace pwc {
namespace {

constexpr int kThreads = 1024;   // one workgroup per CU when the slab is large
constexpr int kDepth = 4;        // stream iterations in flight per lane (3-4 measure alike)
// Quadruples per group and iteration: 4, fewer when each lane reads more
// words per row (the loads of an iteration must fit in registers).
template <int G>
constexpr int rows_per_group() { return G == 1 ? 1 : G == 2 ? 2 : 4; }
constexpr int log2i(int v) { return v <= 1 ? 0 : 1 + log2i(v / 2); }

struct PassArgs {
    const int4 *quads;
    int64_t n;
    int64_t n_pad;     // n rounded up to kStreamPad: the decoded stream's length
    int ord_g;         // lanes per quadruple of the passes the decode orders entries for
    int E1, ndir;      // entries per direction; 3 direction tables for a box, else 1
    const int32_t *basis;
    int N;
    const int32_t *fold;
    int K, nd;
    const void *tab;   // [E][Qp] double or float2: W_q^(1/3) tau_q
    int E, Qp, q0;     // this pass: nodes [q0, q0 + c) of every row
    int Q;             // nodes of the mesh (the rest of a padded row is zero)
    void *scratch;     // [n] packed folded entries
    double pref;
    double *out;
    int *err;
};

// The folded entries carry W_q^(1/3) (the mesh weights are positive), so a
// node term is the plain product of the three entries.
// FP64 arithmetic: one node term is (x * y) * z added with an FMA.
struct F64 {
    using V = double2;   // two adjacent nodes
    struct Acc { double v; };
    __device__ static void zero(Acc &a) { a.v = 0.0; }
    __device__ static void add2(Acc &a, V x, V y, V z) {
        a.v = fma(x.x * y.x, z.x, a.v);
        a.v = fma(x.y * y.y, z.y, a.v);
    }
    __device__ static double value(const Acc &a) { return a.v; }
};

// Split-FP32 arithmetic: table entries are (hi, lo) float pairs; node terms
// are float-float products, summed with TwoSum compensation.
struct FF {
    using V = float4;    // (hi0, lo0, hi1, lo1)
    struct Acc { float h, l; };
    __device__ static void zero(Acc &a) { a.h = a.l = 0.0f; }
    __device__ static void add2(Acc &a, V x, V y, V z) {
        ff_acc(a.h, a.l, ff_mul(ff_mul(ff{x.x, x.y}, ff{y.x, y.y}), ff{z.x, z.y}));
        ff_acc(a.h, a.l, ff_mul(ff_mul(ff{x.z, x.w}, ff{y.z, y.w}), ff{z.z, z.w}));
    }
    __device__ static double value(const Acc &a) { return ff_to_double(a.h, a.l); }
};

// Single-FP32 arithmetic: table entries W_q^(1/3) tau_q rounded once to FP32,
// four nodes per 16-byte word.  The four node products of a word are formed
// and summed pairwise in FP32 and the word's sum is added in FP64: per term
// 3 roundings of the entries, 2 of the product and 2 of the word sum.
struct F32 {
    using V = float4;    // four adjacent nodes
    struct Acc { double v; };
    __device__ static void zero(Acc &a) { a.v = 0.0; }
    // A word's four node terms summed pairwise in FP32: each pair as one
    // rounded triple product added into the other by a fused multiply-add
    // (at most 4 roundings of 2^-24 per term on top of the entries', as
    // with four products and two additions, in 9 operations instead of 11).
    __device__ static void add2(Acc &a, V x, V y, V z) {
        const float s01 = fmaf(x.x * y.x, z.x, (x.y * y.y) * z.y);
        const float s23 = fmaf(x.z * y.z, z.z, (x.w * y.w) * z.w);
        a.v += static_cast<double>(s01 + s23);
    }
    __device__ static double value(const Acc &a) { return a.v; }
};
template <typename A> constexpr int npw() { return 2; }
template <> constexpr int npw<F32>() { return 4; }

// Packed folded entries of one quadruple.  Pk32: three 10-bit fields and
// a flag in bit 30 (E <= 1024); Pk64: 16-bit fields, the flag in bit 31 of
// y.  The flag marks a quadruple with an out-of-range index; its fields are
// zero, so it still addresses row 0.
struct Pk32 {
    using T = uint32_t;
    static constexpr int kMaxE = 1024;
    __device__ static T pack(int a, int b, int c) {
        return static_cast<uint32_t>(a) | (static_cast<uint32_t>(b) << 10) |
               (static_cast<uint32_t>(c) << 20);
    }
    __device__ static T flagged() { return 1u << 30; }
    __device__ static uint32_t flag(T v) { return v >> 30; }
    __device__ static void unpack(T v, int &a, int &b, int &c) {
        a = v & 1023u;
        b = (v >> 10) & 1023u;
        c = (v >> 20) & 1023u;
    }
    // number of odd entries; the first and last entries swapped (flag kept);
    // the word sent to lane `lane` of the wave
    __device__ static int odd(T v) { return __popc(v & 0x100401u); }
    __device__ static T flip(T v) { return (v & 0xC00FFC00u) | ((v & 1023u) << 20) | ((v >> 20) & 1023u); }
    __device__ static T send(T v, int lane) { return __builtin_amdgcn_ds_permute(lane << 2, v); }
};
struct Pk64 {
    using T = uint2;
    __device__ static T pack(int a, int b, int c) {
        return make_uint2(static_cast<uint32_t>(a) | (static_cast<uint32_t>(b) << 16),
                          static_cast<uint32_t>(c));
    }
    __device__ static T flagged() { return make_uint2(0u, 1u << 31); }
    __device__ static uint32_t flag(T v) { return v.y >> 31; }
    __device__ static void unpack(T v, int &a, int &b, int &c) {
        a = v.x & 0xffffu;
        b = v.x >> 16;
        c = v.y & 0xffffu;
    }
    __device__ static int odd(T v) { return __popc(v.x & 0x10001u) + (v.y & 1u); }
    __device__ static T flip(T v) {
        return make_uint2((v.x & 0xffff0000u) | (v.y & 0xffffu), (v.y & 0xffff0000u) | (v.x & 0xffffu));
    }
    __device__ static T send(T v, int lane) {
        return make_uint2(__builtin_amdgcn_ds_permute(lane << 2, v.x), __builtin_amdgcn_ds_permute(lane << 2, v.y));
    }
};

// Lane exchanges inside a 16-lane DPP row.  quad_perm 0xB1 = (1,0,3,2),
// 0x4E = (2,3,0,1); row half mirror (0x141) pairs lane i with 7 - i, row
// mirror (0x140) with 15 - i.
template <int CTRL>
__device__ __forceinline__ double dpp_take(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// Per-iteration loads of one lane, issued one grid-stride iteration ahead
// of their use: the packed entries of the group's R quadruples and, after
// the first pass, the partial sum of the quadruple this lane writes.
template <typename PK, int R>
struct Stream {
    typename PK::T pk[R];
    double prev;
    int4 q;   // the quadruple this lane decodes (first pass with inline decode)
};

// Butterfly step: lanes on the `up` side keep b and send a, the others keep
// a and send b; the partner (DPP pattern CTRL) is on the opposite side.
template <int CTRL>
__device__ __forceinline__ double bfly(double a, double b, bool up) {
    return (up ? b : a) + dpp_take<CTRL>(up ? a : b);
}

// Reduce the R per-lane partial sums of a G-lane group (R <= G, both powers
// of two, groups aligned within 16-lane DPP rows).  The first log2 R steps
// are butterfly exchanges that halve the set, the rest plain sums, with
// partners at distance G/2, G/4, ... (row mirror 15 - s, half mirror 7 - s,
// then s ^ 2 and s ^ 1).  On return lane s holds the full sum of quadruple
// own_row(s) = (s >> (log2 G - log2 R)) mod R; lanes with zero low bits
// write it.
template <int G, int R>
__device__ __forceinline__ int own_row(int s) {
    return (s >> (log2i(G) - log2i(R))) & (R - 1);
}
template <int G, int R>
__device__ __forceinline__ bool row_writer(int s) {
    return (s & ((G / R) - 1)) == 0;
}
template <int CTRL>
__device__ __forceinline__ void reduce_step(double *v, int m, int s, int bit) {
    // m values in, m / 2 out when m > 1 (butterfly), else a plain sum
    if (m == 1) {
        v[0] += dpp_take<CTRL>(v[0]);
        return;
    }
    const bool up = (s >> bit) & 1;
#pragma unroll
    for (int i = 0; i < m / 2; ++i) v[i] = bfly<CTRL>(v[i], v[i + m / 2], up);
}
template <int G, int R>
__device__ __forceinline__ double group_reduce(double *v, int s) {
    static_assert(R <= G, "at most one quadruple per lane");
    int m = R;
    if (G >= 16) { reduce_step<0x140>(v, m, s, 3); m = m > 1 ? m / 2 : 1; }
    if (G >= 8) { reduce_step<0x141>(v, m, s, 2); m = m > 1 ? m / 2 : 1; }
    if (G >= 4) { reduce_step<0x4E>(v, m, s, 1); m = m > 1 ? m / 2 : 1; }
    if (G >= 2) { reduce_step<0xB1>(v, m, s, 0); }
    return v[0];
}

// Decode every quadruple into its packed folded entries, in the parity
// order its stream position asks for (above); an out-of-range index writes
// the flagged word and raises the error word.  Used when the basis and fold
// map do not fit in LDS beside the first pass's slab (the first pass
// decodes inline otherwise).  Positions n .. n_pad - 1 (the
// stream padded to whole pass tiles) get row 0, so the node passes read the
// stream without bounds checks.  A streaming kernel with many waves per CU.
// Each quadruple needs 7 dependent random gathers (4 basis vectors, 3 fold
// entries); when the basis and the fold map fit, they are staged in LDS
// first, where random gathers are far cheaper than divergent L1/L2 accesses.
constexpr int kDecodeThreads = 256, kDecodeBatch = 4;
constexpr int kStreamPad = 1024;   // every pass tile divides it

// Entries with odd parity last (ascending) or first (descending).  The two
// groups of a phase that may clash differ in bit log2(8 / G) of the stream
// position (G = 8: bit 0; 4: bit 1; 2: bit 2; 1: bit 3).
__device__ __forceinline__ bool descending_at(int64_t e, int G) {
    const int b = G >= 8 ? 0 : G == 4 ? 1 : G == 2 ? 2 : 3;
    return (e >> b) & 1;
}

__device__ __forceinline__ void order_by_parity(int &a, int &b, int &c) {
    auto cx = [](int &u, int &v) {
        if ((u & 1) > (v & 1)) {
            const int t = u;
            u = v;
            v = t;
        }
    };
    cx(a, b);
    cx(b, c);
    cx(a, b);
}

// Packed entries of quadruple v in ascending parity; basis and fold map
// from LDS copies or from global memory.
template <typename PK>
__device__ __forceinline__ typename PK::T decode_one(const PassArgs &a, const int32_t *basis,
                                                     const int16_t *lfold, const int32_t *gfold,
                                                     int4 v) {
    const unsigned N = static_cast<unsigned>(a.N);
    if (static_cast<unsigned>(v.x) >= N || static_cast<unsigned>(v.y) >= N ||
        static_cast<unsigned>(v.z) >= N || static_cast<unsigned>(v.w) >= N) {
        raise_error(a.err);
        return PK::flagged();
    }
    const int K = a.K, nd = a.nd;
    const uint32_t ni = basis[v.x], nj = basis[v.y], nk = basis[v.z], nl = basis[v.w];
    // A planewave's three components are the low three bytes of its packed
    // word (signed).  With the sign bits flipped each byte is the component
    // plus 128, so one addition and one subtraction form (n_k - n_i + K) in
    // all three bytes at once: every byte stays within [0, 2K] (|n| <= 24,
    // K = 2 nmax), so no carry or borrow crosses into the next.
    constexpr uint32_t kSign = 0x808080u;
    const uint32_t kk = static_cast<uint32_t>(K) * 0x010101u;
    const uint32_t ki = ((nk ^ kSign) + kk) - (ni ^ kSign), lj = ((nl ^ kSign) + kk) - (nj ^ kSign);
    // (difference + K) lies in [0, 2K] and nd = 2K + 1 is small: 24-bit products
    const int ix = __umul24(ki & 255u, nd) + (lj & 255u);
    const int iy = __umul24((ki >> 8) & 255u, nd) + ((lj >> 8) & 255u);
    const int iz = __umul24(ki >> 16, nd) + (lj >> 16);
    int fx = lfold ? lfold[ix] : gfold[ix];
    int fy = lfold ? lfold[iy] : gfold[iy];
    int fz = lfold ? lfold[iz] : gfold[iz];
    if (a.ndir == 3) {       // a box: each direction reads its own table's rows
        fy += a.E1;
        fz += 2 * a.E1;
    }
    order_by_parity(fx, fy, fz);   // the node term is a product: any order serves
    return PK::pack(fx, fy, fz);
}

// The word the stream holds for quadruple e: ascending parity for the
// one-lane passes (which pair their lanes themselves), else ascending or
// descending by stream position for the lane groups of the passes.
template <typename PK>
__device__ __forceinline__ typename PK::T stream_word(typename PK::T v, int64_t e, int ord_g) {
    return ord_g > 1 && descending_at(e, ord_g) ? PK::flip(v) : v;
}

template <typename PK, bool LDS_MAPS>
__global__ __launch_bounds__(kDecodeThreads) void k_decode(PassArgs a, int64_t n_pad) {
    extern __shared__ uint4 lds_dyn[];
    int32_t *lbasis = reinterpret_cast<int32_t *>(lds_dyn);
    int16_t *lfold = reinterpret_cast<int16_t *>(lbasis + a.N);
    const int nd2 = a.nd * a.nd;
    if (LDS_MAPS) {
        for (int i = threadIdx.x; i < a.N; i += kDecodeThreads) lbasis[i] = a.basis[i];
        for (int i = threadIdx.x; i < nd2; i += kDecodeThreads) lfold[i] = static_cast<int16_t>(a.fold[i]);
        __syncthreads();
    }
    typename PK::T *out = static_cast<typename PK::T *>(a.scratch);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kDecodeThreads * kDecodeBatch;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * kDecodeThreads * kDecodeBatch;
         base < n_pad; base += stride) {
        int4 q[kDecodeBatch];
#pragma unroll
        for (int b = 0; b < kDecodeBatch; ++b) {
            const int64_t e = base + b * kDecodeThreads + threadIdx.x;
            if (e < a.n) q[b] = a.quads[e];
        }
#pragma unroll
        for (int b = 0; b < kDecodeBatch; ++b) {
            const int64_t e = base + b * kDecodeThreads + threadIdx.x;
            if (e >= n_pad) continue;
            out[e] = e < a.n ? stream_word<PK>(decode_one<PK>(a, LDS_MAPS ? lbasis : a.basis,
                                                              LDS_MAPS ? lfold : nullptr, a.fold, q[b]),
                                               e, a.ord_g)
                             : PK::pack(0, 0, 0);
        }
    }
}

// Broadcast, inside a group, the packed word decoded by the group's lane r
// (lane r of each 4-lane quad, or of each lane pair when G = 2).
__device__ __forceinline__ uint32_t bcast_u32(uint32_t v, int ctrl_r) {
    switch (ctrl_r) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xf, 0xf, false);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xf, 0xf, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0xAA, 0xf, 0xf, false);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0xFF, 0xf, 0xf, false);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0xA0, 0xf, 0xf, false);   // pairs: lane 0
    default: return __builtin_amdgcn_mov_dpp(v, 0xF5, 0xf, 0xf, false);  // pairs: lane 1
    }
}
// R = 1: nothing to share; R = 2: from lane r of each lane pair; R = 4: from
// lane r of each 4-lane quad.
template <int R>
__device__ __forceinline__ uint32_t bcast_row(uint32_t v, int r) {
    return R == 1 ? v : bcast_u32(v, R == 2 ? 4 + r : r);
}
template <int R>
__device__ __forceinline__ uint2 bcast_row(uint2 v, int r) {
    return make_uint2(bcast_row<R>(v.x, r), bcast_row<R>(v.y, r));
}

// Lane pairing of the one-lane layout (G = 1).  On gfx950 a 128-bit LDS
// read serves the lanes of a 32-lane half-wave in two cycles of two 8-lane
// groups; with rows of 128 bytes (half the 64 banks) and lane g reading
// word k ^ (g mod 8) at step k, the read is conflict-free when lanes g and
// g + 24, and g + 8 and g + 16, of each half-wave hold rows of opposite
// parity (measured: random rows so paired take no conflict cycles; rows
// paired at g and g + 8, or not at all, take one per cycle).  A quadruple
// with c odd entries read in ascending parity and one with 3 - c odd
// entries read in descending parity meet opposite parities at all three
// reads, so the wave's 64 quadruples are dealt to lanes: pairs 0 .. m03 - 1
// take classes 0 (low lane) and 3 (high lane), the next m12 pairs classes 1
// and 2, and the quadruples left over fill the last pairs in order.  Pair
// p sits in half-wave p / 16 at lanes i and i + 24 (p mod 16 = i < 8) or
// i + 8 and i + 16 (p mod 16 = 8 + i); the high lanes are those with bit 4
// set.  Returns the lane that evaluates this lane's quadruple (a
// permutation of the wave; every lane must take part).
__device__ __forceinline__ int pair_lane(int cls) {
    // Two ballots carry every lane's class: its low bit in lo, its high bit in hi.
    const uint64_t lo = __builtin_amdgcn_ballot_w64(cls & 1), hi = __builtin_amdgcn_ballot_w64(cls & 2);
    const int n3 = __popcll(lo & hi), n1 = __popcll(lo & ~hi), n2 = __popcll(~lo & hi);
    const int n0 = 64 - n1 - n2 - n3;
    const int m03 = min(n0, n3), m12 = min(n1, n2), l03 = n0 + n3 - 2 * m03;
    const bool outer = cls == 0 || cls == 3;
    // The lanes of this lane's class: both bits equal to its own.
    const uint32_t m1 = 0u - static_cast<uint32_t>(cls & 1), m2 = 0u - static_cast<uint32_t>((cls >> 1) & 1);
    const uint32_t same_lo = ~((static_cast<uint32_t>(lo) ^ m1) | (static_cast<uint32_t>(hi) ^ m2));
    const uint32_t same_hi = ~((static_cast<uint32_t>(lo >> 32) ^ m1) | (static_cast<uint32_t>(hi >> 32) ^ m2));
    const int r = __builtin_amdgcn_mbcnt_hi(same_hi, __builtin_amdgcn_mbcnt_lo(same_lo, 0));
    const int m = outer ? m03 : m12;
    int pair, side;
    if (r < m) {                      // a matched pair: classes 0 and 1 low, 2 and 3 high
        pair = (outer ? 0 : m03) + r;
        side = cls >= 2;
    } else {                          // left over: in order, two per pair
        const int k = (outer ? 0 : l03) + r - m;
        pair = m03 + m12 + (k >> 1);
        side = k & 1;
    }
    const int i = pair & 7, second = (pair >> 3) & 1;
    return ((pair >> 4) << 5) | i | (side ? (second ? 16 : 24) : (second ? 8 : 0));
}

// Wave-wide pairing of a fused chunk: the wave's 64 NT quadruples (slot t of
// every lane, t < NT) dealt at once, in pair_lane's order (matched pairs of
// classes 0 and 3, then of 1 and 2, then the ones left over), pair P going
// to slot P / 32 at the lanes pair_lane gives pair P mod 32.  Dealt per slot,
// a wave's 64 quadruples leave about 9 without a complement, which put a
// conflict cycle on most reads of every slot; dealt over 64 NT, the count
// left over grows as the square root, and all of them sit in the last
// slots.  pk[t]: this lane's quadruple of slot t; returns in dest[t] the
// position (slot 64 + lane) that evaluates it.  The class ballots are taken
// again in the second sweep rather than kept (registers).
template <typename PK, int NT>
__device__ __forceinline__ void pair_wave(const typename PK::T (&pk)[NT], int (&dest)[NT]) {
    int n1 = 0, n2 = 0, n3 = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = PK::odd(pk[t]);
        const uint64_t lo = __builtin_amdgcn_ballot_w64(c & 1), hi = __builtin_amdgcn_ballot_w64(c & 2);
        n3 += __popcll(lo & hi);
        n1 += __popcll(lo & ~hi);
        n2 += __popcll(~lo & hi);
    }
    const int n0 = 64 * NT - n1 - n2 - n3;
    const int m03 = min(n0, n3), m12 = min(n1, n2), l03 = n0 + n3 - 2 * m03;
    int b0 = 0, b1 = 0, b2 = 0, b3 = 0;   // quadruples of each class in the earlier slots
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = PK::odd(pk[t]);
        const uint64_t lo = __builtin_amdgcn_ballot_w64(c & 1), hi = __builtin_amdgcn_ballot_w64(c & 2);
        const bool outer = c == 0 || c == 3;
        const uint32_t m1 = 0u - static_cast<uint32_t>(c & 1), m2 = 0u - static_cast<uint32_t>((c >> 1) & 1);
        const uint32_t same_lo = ~((static_cast<uint32_t>(lo) ^ m1) | (static_cast<uint32_t>(hi) ^ m2));
        const uint32_t same_hi = ~((static_cast<uint32_t>(lo >> 32) ^ m1) | (static_cast<uint32_t>(hi >> 32) ^ m2));
        const int before = c == 0 ? b0 : c == 1 ? b1 : c == 2 ? b2 : b3;
        const int r = before + __builtin_amdgcn_mbcnt_hi(same_hi, __builtin_amdgcn_mbcnt_lo(same_lo, 0));
        const int m = outer ? m03 : m12;
        int pair, side;
        if (r < m) {
            pair = (outer ? 0 : m03) + r;
            side = c >= 2;
        } else {
            const int k = (outer ? 0 : l03) + r - m;
            pair = m03 + m12 + (k >> 1);
            side = k & 1;
        }
        const int p = pair & 31, i = p & 7, second = (p >> 3) & 1;
        dest[t] = (pair >> 5) * 64 + (((p >> 4) << 5) | i | (side ? (second ? 16 : 24) : (second ? 8 : 0)));
        const int c3 = __popcll(lo & hi), c1 = __popcll(lo & ~hi), c2 = __popcll(~lo & hi);
        b0 += 64 - c1 - c2 - c3;
        b1 += c1;
        b2 += c2;
        b3 += c3;
    }
}

// One node pass.  LDS: the slab [E][G W] of 16-byte words (nodes q0 ..
// q0 + c - 1 of every folded entry).  Lane s of group g reads, for each of
// its R quadruples e = base + r NG + g, its W words of the three rows.
// DECODE (first pass only): the basis and fold map follow the slab in LDS,
// lane s of a group decodes quadruple s mod R itself, writes its packed word
// to the scratch stream for the later passes, and the group shares the R
// words by DPP broadcast.  Used with one lane per quadruple (G = 1, W = 8),
// where nothing is decoded twice or shared.
template <typename A, int G, int W, typename PK, bool FIRST, bool LAST, bool DECODE>
__global__ __launch_bounds__(kThreads) void k_rec_pass(PassArgs a) {
    static_assert(!DECODE || FIRST, "only the first pass decodes");
    using V = typename A::V;
    using T = typename PK::T;
    // A static slab: its LDS address is known when instructions are
    // selected, so row addresses need no base add.  One workgroup per CU
    // either way (1024 lanes of up to 128 registers).
    __shared__ uint4 lds_raw[kLdsMax / 16];
    constexpr int NG = kThreads / G, R = rows_per_group<G>(), TILE = NG * R;
    constexpr int ROWB = G * W * 16;                    // bytes per slab row
    // Groups of one phase whose runs would share banks read their W chunks in
    // different orders: group g takes chunk k ^ (g mod W) at step k.
    constexpr bool ROT = (W > 1 && G < 16);
    static_assert(kStreamPad % TILE == 0, "the padded stream covers every tile");
    const int s = threadIdx.x % G, g = threadIdx.x / G;
    const int rot = ROT ? (g & (W - 1)) : 0;
    const int own = own_row<G, R>(s);                   // quadruple this lane writes
    const bool writer = row_writer<G, R>(s);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * TILE;
    int64_t base = static_cast<int64_t>(blockIdx.x) * TILE;
    const T *sc = static_cast<const T *>(a.scratch) + g;
    const int rdec = s % R;                             // quadruple this lane decodes
    const int words = a.E * G * W;
    int32_t *lbasis = reinterpret_cast<int32_t *>(lds_raw + words);
    int16_t *lfold = reinterpret_cast<int16_t *>(lbasis + a.N);

    auto load = [&](Stream<PK, R> &st, int64_t b) {
        if (DECODE) {
            const int64_t e = b + rdec * NG + g;
            if (e < a.n) st.q = a.quads[e];
        } else {
            const T *p = sc + b;
#pragma unroll
            for (int r = 0; r < R; ++r) st.pk[r] = p[r * NG];
        }
        const int64_t e = b + own * NG + g;
        if (!FIRST && writer && e < a.n) st.prev = a.out[e];
    };
    // D stream buffers in turn: the loads for iteration i + D - 1 are issued
    // before iteration i computes.
    constexpr int D = DECODE ? 2 : kDepth;
    Stream<PK, R> st[D]{};
#pragma unroll
    for (int i = 0; i < D - 1; ++i)                     // overlaps the slab staging
        if (base + i * stride < a.n) load(st[i], base + i * stride);
    {
        V *dst = reinterpret_cast<V *>(lds_raw);
        const V *src = static_cast<const V *>(a.tab) + a.q0 / npw<A>();
        const int row = a.Qp / npw<A>();
        for (int i = threadIdx.x; i < words; i += kThreads) {
            const int e = i / (G * W), j = i % (G * W);
            dst[i] = src[static_cast<size_t>(e) * row + j];
        }
        if (DECODE) {
            for (int i = threadIdx.x; i < a.N; i += kThreads) lbasis[i] = a.basis[i];
            for (int i = threadIdx.x; i < a.nd * a.nd; i += kThreads)
                lfold[i] = static_cast<int16_t>(a.fold[i]);
        }
    }
    const char *lb = reinterpret_cast<const char *>(lds_raw);
    const uint32_t lane_b = static_cast<uint32_t>((s + G * rot) * 16);
    __syncthreads();

    auto body = [&](const Stream<PK, R> &st, int64_t b) {
        T pk[R];
        if (DECODE) {
            const int64_t e = b + rdec * NG + g;
            const T mine = e < a.n ? decode_one<PK>(a, lbasis, lfold, nullptr, st.q)
                                   : PK::pack(0, 0, 0);   // padding up to the tile end
            if (!LAST && s < R) const_cast<T *>(sc)[b + rdec * NG] = stream_word<PK>(mine, e, a.ord_g);
#pragma unroll
            for (int r = 0; r < R; ++r) pk[r] = bcast_row<R>(mine, r);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) pk[r] = st.pk[r];
        }
        // One lane per quadruple: evaluate the quadruple pair_lane deals
        // this lane, the high lane of each pair in descending parity.
        constexpr bool PAIR = G == 1;
        int dest = 0;
        T ev[R];
#pragma unroll
        for (int r = 0; r < R; ++r) ev[r] = pk[r];
        if (PAIR) {
            dest = pair_lane(PK::odd(pk[0]));
            ev[0] = PK::send(pk[0], dest);
            if (threadIdx.x & 16) ev[0] = PK::flip(ev[0]);   // high lane of its pair
        }
        V x[R][W], y[R][W], z[R][W];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int f0, f1, f2;
            PK::unpack(ev[r], f0, f1, f2);
            const uint32_t a0 = f0 * ROWB + lane_b, a1 = f1 * ROWB + lane_b, a2 = f2 * ROWB + lane_b;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                // chunk k ^ rot: row base + 16 (s + G (k ^ rot)) = a ^ (16 G k)
                const uint32_t o = k * G * 16;
                x[r][k] = *reinterpret_cast<const V *>(lb + (ROT ? (a0 ^ o) : a0 + o));
                y[r][k] = *reinterpret_cast<const V *>(lb + (ROT ? (a1 ^ o) : a1 + o));
                z[r][k] = *reinterpret_cast<const V *>(lb + (ROT ? (a2 ^ o) : a2 + o));
            }
        }
        double v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            typename A::Acc acc;
            A::zero(acc);
#pragma unroll
            for (int k = 0; k < W; ++k) A::add2(acc, x[r][k], y[r][k], z[r][k]);
            v[r] = A::value(acc);
        }
        double sum = group_reduce<G, R>(v, s);
        if (PAIR)   // back to the lane that holds the quadruple's stream slot
            sum = __hiloint2double(__builtin_amdgcn_ds_bpermute(dest << 2, __double2hiint(sum)),
                                   __builtin_amdgcn_ds_bpermute(dest << 2, __double2loint(sum)));
        const int64_t e = b + own * NG + g;
        if (writer && e < a.n) {
            double prev;
            if (FIRST) {   // the first pass marks a bad quadruple; later passes carry the NaN
                uint32_t bad = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) bad |= PK::flag(pk[r]) << r;
                prev = ((bad >> own) & 1) ? NAN : 0.0;
            } else {
                prev = st.prev;
            }
            a.out[e] = LAST ? (prev + sum) * a.pref : prev + sum;
        }
    };

    // A decoding pass covers the whole padded stream, so the later passes
    // (larger tiles) find every packed word they read written.
    const int64_t end = DECODE ? a.n_pad : a.n;
    while (base < end) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t ahead = base + (D - 1) * stride;
            if (ahead < end) load(st[(i + D - 1) % D], ahead);
            body(st[i], base);
            base += stride;
            if (base >= end) break;
        }
    }
}

// Fused one-lane node sums (see the header): NT quadruples per lane and
// chunk, SPT 16-byte slab words staged per lane.  Every node range of the
// padded rows (P ranges of 8 words per row) is added to the chunk's partial
// sums in range order, each range's terms in node order, exactly as the
// one-lane passes do; the pairing of a chunk's quadruples is formed once.

// Word 3 of a raw buffer resource on gfx9 parts (untyped access; the
// other fields are the base, a zero stride and the size in bytes), and the
// cache policy of a streaming (non-temporal) access.
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int kCachePolicyNT = 2;

// Quadruples per lane and chunk (NT): as many as fit in registers beside the
// staged slab words, 8 beside 6 words, 6 beside 8 (10 beside 6 spill); the
// host's fused_chunk_quads gives the same count.
constexpr int fused_chunk(int spt) { return spt <= 6 ? 8 : 6; }

// An empty register constraint: the compiler must assume the value is read
// and changed here, so what feeds it is computed before this point and what
// it feeds is formed after it (not hoisted out of the enclosing loop).
__device__ __forceinline__ void opaque(uint32_t &v) { __asm__ volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(double &v) { __asm__ volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(uint2 &v) {
    __asm__ volatile("" : "+v"(v.x));
    __asm__ volatile("" : "+v"(v.y));
}

// Slab words of node range p: word j of row e is 16-byte word p W + j of
// the padded row (row words); lane i stages words i + 1024 k.  The loads go
// through a buffer resource over the table (rsrc), which returns zero past
// its end: with no branch around a load, a wait for an earlier load counts
// exactly the loads issued after it, so the wait for the next chunk's
// quadruples does not also wait for these words.
template <int SPT>
__device__ __forceinline__ void fetch_slab(uint4 (&pre)[SPT], __amdgpu_buffer_rsrc_t rsrc, int row, int p) {
    uint32_t i0 = threadIdx.x;
    opaque(i0);   // the addresses are formed here, not kept in registers between fetches
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int i = static_cast<int>(i0) + k * kThreads;
        const int word = (i >> 3) * row + p * 8 + (i & 7);
        pre[k] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, word * 16, 0, 0));
    }
}

// One quadruple's terms of the staged node range, steps k0 .. k0 + N - 1
// of its three rows, added to s in step order.
template <typename A, int N>
__device__ __forceinline__ void fused_half(typename A::Acc &s, const char *lb, uint32_t a0, uint32_t a1, uint32_t a2,
                                           int k0) {
    using V = typename A::V;
    V x[N], y[N], z[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const uint32_t o = (k0 + k) * 16;
        x[k] = *reinterpret_cast<const V *>(lb + (a0 ^ o));
        y[k] = *reinterpret_cast<const V *>(lb + (a1 ^ o));
        z[k] = *reinterpret_cast<const V *>(lb + (a2 ^ o));
    }
#pragma unroll
    for (int k = 0; k < N; ++k) A::add2(s, x[k], y[k], z[k]);
}

// MULTI: more than one node range (the slab is restaged for every range of
// every chunk); else the one range is staged once.  WL: words of real nodes
// in the last range, rounded up to 1, 2, 4 or 8.
template <typename A, typename PK, int SPT, int NT, int WL, bool MULTI>
__global__ __launch_bounds__(kThreads) void k_rec_fused(PassArgs a, int P) {
    using T = typename PK::T;
    typedef int v4i __attribute__((ext_vector_type(4)));
    __shared__ uint4 lds_raw[kLdsMax / 16];
    constexpr int ROWB = 8 * 16;
    const int words = a.E * 8;
    // Several ranges: the slab area doubles as the exchange area of the
    // wave-wide pairing (8 bytes per quadruple, each wave its own part),
    // used between a chunk's last range and the next chunk's first stage.
    constexpr int XWORDS = kThreads * NT * 8 / 16;
    // This lane's 4-byte (x = 4) or 8-byte (x = 8) entry of slot 0 in the
    // wave's part, formed where it is used (not held through the loop).
    auto xslot0 = [&](int x) __attribute__((always_inline)) {
        uint32_t i = threadIdx.x;
        opaque(i);
        return reinterpret_cast<char *>(lds_raw) + (i >> 6) * (64 * NT * 8) + (i & 63) * x;
    };
    int32_t *lbasis = reinterpret_cast<int32_t *>(lds_raw + (MULTI ? max(words, XWORDS) : words));
    int16_t *lfold = reinterpret_cast<int16_t *>(lbasis + a.N);
    for (int i = threadIdx.x; i < a.N; i += kThreads) lbasis[i] = a.basis[i];
    for (int i = threadIdx.x; i < a.nd * a.nd; i += kThreads) lfold[i] = static_cast<int16_t>(a.fold[i]);
    const int row = a.Qp / npw<A>();
    // The whole folded table (E rows of row words): words past the slab read zero.
    const __amdgpu_buffer_rsrc_t slab_rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(a.tab), 0, a.E * row * 16, kBufferRsrcWord3);
    const char *lb = reinterpret_cast<const char *>(lds_raw);
    const int64_t chunk = static_cast<int64_t>(kThreads) * NT;
    const int64_t step = static_cast<int64_t>(gridDim.x) * chunk;

    // A chunk's quadruples are streamed once, loaded while the previous
    // chunk's last range is summed, through a buffer resource over the
    // chunk's part of the stream (past its end the loads return zero, and
    // the decode skips those lanes).
    auto chunk_len = [&](int64_t b) __attribute__((always_inline)) {   // quadruples of the chunk at b
        return static_cast<int>(max<int64_t>(0, min(a.n - b, chunk)));
    };
    v4i qn[NT];
    auto load_quads = [&](int64_t b) __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int4 *>(a.quads + min(b, a.n)), 0, chunk_len(b) * static_cast<int>(sizeof(int4)), kBufferRsrcWord3);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            qn[t] = __builtin_amdgcn_raw_buffer_load_b128(r, (t * kThreads + static_cast<int>(threadIdx.x)) * 16, 0,
                                                          kCachePolicyNT);
    };
    // A chunk's results go out through a buffer resource that covers the
    // chunk's part of the stream: stores past its end are dropped by the
    // hardware, with no branch around them (see fetch_slab).
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    auto store_results = [&](int64_t b, const double (&v)[NT]) __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            a.out + b, 0, chunk_len(b) * static_cast<int>(sizeof(double)), kBufferRsrcWord3);
#pragma unroll
        for (int t = 0; t < NT; ++t)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v[t]), r,
                                                  (t * kThreads + static_cast<int>(threadIdx.x)) * 8, 0, kCachePolicyNT);
    };
    uint4 pre[SPT];
    // The staged range into LDS, once every wave is done with the last.
    auto stage = [&]() __attribute__((always_inline)) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int i = threadIdx.x + k * kThreads;
            if (i < words) lds_raw[i] = pre[k];
        }
        __syncthreads();
    };
    load_quads(static_cast<int64_t>(blockIdx.x) * chunk);   // in the order of the loop's back edge
    fetch_slab<SPT>(pre, slab_rsrc, row, 0);
    if (!MULTI) stage();   // also orders the maps before the first decode
    else __syncthreads();  // the maps, before the first decode

    T ev[NT];
    double acc[NT];
    // One full range: each quadruple's terms in step order, its twelve reads
    // of a half in a block of their own (more in flight would spill).
    auto full_range = [&](auto after) __attribute__((always_inline)) {
        const uint32_t lane_r = static_cast<uint32_t>((threadIdx.x & 7) * 16);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            int f0, f1, f2;
            opaque(ev[t]);   // row addresses are formed per range, not kept for all eight
            PK::unpack(ev[t], f0, f1, f2);
            const uint32_t a0 = f0 * ROWB + lane_r, a1 = f1 * ROWB + lane_r, a2 = f2 * ROWB + lane_r;
            typename A::Acc s;
            A::zero(s);
            fused_half<A, 4>(s, lb, a0, a1, a2, 0);
            __builtin_amdgcn_sched_barrier(0);
            fused_half<A, 4>(s, lb, a0, a1, a2, 4);
            acc[t] = acc[t] + A::value(s);
            opaque(acc[t]);   // summed here, not where it is stored
            __builtin_amdgcn_sched_barrier(0);
            after(t);
        }
    };
    auto none = [](int) __attribute__((always_inline)) {};
    // The last range.  A short one (fewer than 8 words of real nodes) reads
    // its first WL words only, word k ^ (lane mod WL) at step k: the order in
    // which the full range meets those words, the others holding zero-weight
    // padding, so the sum is the full range's.
    auto last_range = [&](auto after) __attribute__((always_inline)) {
        if constexpr (WL == 8) {
            full_range(after);
        } else {
            const uint32_t lane_r = static_cast<uint32_t>((threadIdx.x & (WL - 1)) * 16);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                int f0, f1, f2;
                opaque(ev[t]);
                PK::unpack(ev[t], f0, f1, f2);
                typename A::Acc s;
                A::zero(s);
                fused_half<A, WL < 4 ? WL : 4>(s, lb, f0 * ROWB + lane_r, f1 * ROWB + lane_r, f2 * ROWB + lane_r, 0);
                acc[t] = acc[t] + A::value(s);
                opaque(acc[t]);
                __builtin_amdgcn_sched_barrier(0);
                after(t);
            }
        }
    };
    // Several ranges: the next chunk's quadruples are decoded during the
    // last range, quadruple t after the range's quadruple t + kDecodeLag
    // (their loads, issued just before the range, have landed by then), so
    // that the VALU work of the decode runs beside the range's LDS reads
    // instead of after the chunk, when every wave would run it at once.
    constexpr int kDecodeLag = 3;
    T pkn[NT];
    auto decode_one_next = [&](int t, int len) __attribute__((always_inline)) {
        const int4 q = make_int4(qn[t].x, qn[t].y, qn[t].z, qn[t].w);
        const bool real = t * kThreads + static_cast<int>(threadIdx.x) < len;
        pkn[t] = real ? decode_one<PK>(a, lbasis, lfold, nullptr, q) : PK::pack(0, 0, 0);
    };
    if constexpr (MULTI) {
        const int len0 = chunk_len(static_cast<int64_t>(blockIdx.x) * chunk);
#pragma unroll
        for (int t = 0; t < NT; ++t) decode_one_next(t, len0);
    }

    for (int64_t base = static_cast<int64_t>(blockIdx.x) * chunk; base < a.n; base += step) {
        // Decode and pair.  Several ranges: position dest[t] (slot 64 +
        // lane) of the wave evaluates this lane's quadruple t, and the packed
        // words go there through the exchange area; one range: lane dest[t]
        // of slot t does, and the word goes by one permute.
        int dest[NT];
        if constexpr (MULTI) {
            pair_wave<PK, NT>(pkn, dest);
            T *xw = reinterpret_cast<T *>(xslot0(4)) - (threadIdx.x & 63);   // the wave's part
#pragma unroll
            for (int t = 0; t < NT; ++t) xw[dest[t]] = pkn[t];
            // The wave's own part: its LDS operations complete in order.
            const T *xmine = reinterpret_cast<const T *>(xslot0(4));
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                ev[t] = xmine[t * 64];
                if (threadIdx.x & 16) ev[t] = PK::flip(ev[t]);   // high lane of its pair
                acc[t] = PK::flag(ev[t]) ? NAN : 0.0;   // a bad quadruple is NaN
            }
        } else {
            const int len = chunk_len(base);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int4 q = make_int4(qn[t].x, qn[t].y, qn[t].z, qn[t].w);
                const bool real = t * kThreads + static_cast<int>(threadIdx.x) < len;
                const T pk = real ? decode_one<PK>(a, lbasis, lfold, nullptr, q) : PK::pack(0, 0, 0);
                dest[t] = pair_lane(PK::odd(pk));
                ev[t] = PK::send(pk, dest[t]);
                if (threadIdx.x & 16) ev[t] = PK::flip(ev[t]);   // high lane of its pair
                acc[t] = PK::flag(ev[t]) ? NAN : 0.0;   // a bad quadruple is NaN
            }
        }
        if constexpr (MULTI) {
            for (int p = 0; p + 1 < P; ++p) {
                stage();
                fetch_slab<SPT>(pre, slab_rsrc, row, p + 1);   // the next range
                full_range(none);
            }
            stage();
            load_quads(base + step);
            const int len_next = chunk_len(base + step);
            last_range([&](int t) __attribute__((always_inline)) {
                if (t >= kDecodeLag) decode_one_next(t - kDecodeLag, len_next);
            });
#pragma unroll
            for (int t = NT - kDecodeLag; t < NT; ++t) decode_one_next(t, len_next);
        } else {
            load_quads(base + step);
            last_range(none);
        }
        double res[NT];
        if constexpr (MULTI) {
            // Every wave is done with the slab; the sums go back to their
            // quadruples' lanes through the exchange area.
            __syncthreads();
            double *xmine = reinterpret_cast<double *>(xslot0(8));
#pragma unroll
            for (int t = 0; t < NT; ++t) xmine[t * 64] = acc[t];
            const double *xd = reinterpret_cast<const double *>(xslot0(8)) - (threadIdx.x & 63);
#pragma unroll
            for (int t = 0; t < NT; ++t) res[t] = xd[dest[t]] * a.pref;
            // Read before the next chunk writes its packed words there (of
            // another type: the compiler must not move those stores up).
            __asm__ volatile("" ::: "memory");
            fetch_slab<SPT>(pre, slab_rsrc, row, 0);   // the next chunk's first range
        } else {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                res[t] = __hiloint2double(__builtin_amdgcn_ds_bpermute(dest[t] << 2, __double2hiint(acc[t])),
                                          __builtin_amdgcn_ds_bpermute(dest[t] << 2, __double2loint(acc[t]))) *
                         a.pref;
        }
        store_results(base, res);
    }
}

template <typename A, typename PK>
hipError_t launch_fused(const PassArgs &a, const Table &t, int P, hipStream_t s) {
    const int words = a.E * 8;
    if (words > 8 * kThreads) return hipErrorInvalidValue;
    const bool six = words <= 6 * kThreads;   // staged words per lane: 6, else 8
    const int64_t chunk = static_cast<int64_t>(kThreads) * (six ? fused_chunk(6) : fused_chunk(8));
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>((a.n + chunk - 1) / chunk, t.n_cu));
    // Words of the last range that hold real nodes, rounded up to 1, 2, 4 or 8.
    const int c = 8 * npw<A>();
    const int real = (a.Q - (P - 1) * c + npw<A>() - 1) / npw<A>();
    if (P < 1 || real < 1 || real > 8) return hipErrorInvalidValue;
    const int wlast = real <= 1 ? 1 : real <= 2 ? 2 : real <= 4 ? 4 : 8;
    using K = void (*)(PassArgs, int);
    constexpr int N6 = fused_chunk(6), N8 = fused_chunk(8);
    // [staged words per lane 6 or 8][one range or several][last range's words]
    static const K kern_of[2][2][4] = {
        {{k_rec_fused<A, PK, 6, N6, 1, false>, k_rec_fused<A, PK, 6, N6, 2, false>,
          k_rec_fused<A, PK, 6, N6, 4, false>, k_rec_fused<A, PK, 6, N6, 8, false>},
         {k_rec_fused<A, PK, 6, N6, 1, true>, k_rec_fused<A, PK, 6, N6, 2, true>,
          k_rec_fused<A, PK, 6, N6, 4, true>, k_rec_fused<A, PK, 6, N6, 8, true>}},
        {{k_rec_fused<A, PK, 8, N8, 1, false>, k_rec_fused<A, PK, 8, N8, 2, false>,
          k_rec_fused<A, PK, 8, N8, 4, false>, k_rec_fused<A, PK, 8, N8, 8, false>},
         {k_rec_fused<A, PK, 8, N8, 1, true>, k_rec_fused<A, PK, 8, N8, 2, true>,
          k_rec_fused<A, PK, 8, N8, 4, true>, k_rec_fused<A, PK, 8, N8, 8, true>}}};
    const int w = wlast == 1 ? 0 : wlast == 2 ? 1 : wlast == 4 ? 2 : 3;
    const K kern = kern_of[six ? 0 : 1][P > 1 ? 1 : 0][w];
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, a, P);
    return hipGetLastError();
}
using PassKernel = void (*)(PassArgs);

template <typename A, int G, int W, typename PK>
PassKernel pass_kernel(int p, int P, bool decode) {
    if (p == 0) {
        if (decode)   // one-lane first pass with the decode inline (c = 16 only)
            return P == 1 ? k_rec_pass<A, 1, 8, PK, true, true, true> : k_rec_pass<A, 1, 8, PK, true, false, true>;
        return P == 1 ? k_rec_pass<A, G, W, PK, true, true, false> : k_rec_pass<A, G, W, PK, true, false, false>;
    }
    return p == P - 1 ? k_rec_pass<A, G, W, PK, false, true, false> : k_rec_pass<A, G, W, PK, false, false, false>;
}

// stage_ev (optional): events recorded before the decode and after every
// launch of the first slab, for per-stage timing.
template <typename A, int G, int W, typename PK>
hipError_t run_passes(const PassArgs &a0, const Table &t, const FoldLayout &fl, hipStream_t s,
                      hipEvent_t *stage_ev) {
    const int P = fl.nchunk;
    const size_t lds = static_cast<size_t>(fl.E) * G * W * 16;   // slab bytes used
    if (lds > static_cast<size_t>(kLdsMax)) return hipErrorInvalidValue;
    hipError_t err0 = hipSuccess;
    constexpr int64_t tile_d = kThreads;   // the one-lane decoding pass
    constexpr int64_t tile = static_cast<int64_t>(kThreads / G) * rows_per_group<G>();
    // LDS copy of the basis (int32) and the fold map (int16) for the decode:
    // inside the first pass when they fit beside its slab, else in k_decode.
    const size_t maps_bytes = fold_maps_bytes(t.N, t.nd);
    const bool inline_decode = G * W == 8 && lds + maps_bytes <= static_cast<size_t>(kLdsMax);
    const size_t dmaps = (maps_bytes + 15) / 16 * 16;
    const bool maps_fit = dmaps <= static_cast<size_t>(kLdsMax);
    if (!inline_decode && maps_fit) {
        const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_decode<PK, true>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(dmaps));
        if (err != hipSuccess) return err;
    }
    // One launch for every pass, unless per-launch timing is asked for.
    // (fused_layout needs E <= 1024, so only the 4-byte packed entries occur)
    if constexpr (std::is_same<PK, Pk32>::value)
        if (!stage_ev && fused_layout(fl, maps_bytes)) return launch_fused<A, PK>(a0, t, P, s);
    if (!a0.scratch) return hipErrorInvalidValue;   // the separate launches need the decoded stream
    const int per_cu = 1;   // the static slab takes the CU's LDS
    // Slabs bound the scratch array: at most kRecSlab quadruples per slab.
    for (int64_t off = 0; off < a0.n; off += kRecSlab) {
        PassArgs a = a0;
        a.n = std::min<int64_t>(kRecSlab, a0.n - off);
        a.quads = a0.quads + off;
        a.out = a0.out + off;
        a.n_pad = (a.n + kStreamPad - 1) / kStreamPad * kStreamPad;
        hipEvent_t *ev = (off == 0) ? stage_ev : nullptr;
        if (ev && (err0 = hipEventRecord(ev[0], s)) != hipSuccess) return err0;
        hipError_t err;
        if (!inline_decode) {
            const int64_t n_pad = a.n_pad;
            const int64_t dblocks = (n_pad + kDecodeThreads * kDecodeBatch - 1) / (kDecodeThreads * kDecodeBatch);
            if (maps_fit) {
                const int dper = std::max(1, std::min(8, static_cast<int>(kLdsMax / dmaps)));
                const unsigned dgrid = static_cast<unsigned>(std::min<int64_t>(dblocks, int64_t(t.n_cu) * dper));
                hipLaunchKernelGGL((k_decode<PK, true>), dim3(dgrid), dim3(kDecodeThreads), dmaps, s, a, n_pad);
            } else {
                const unsigned dgrid = static_cast<unsigned>(std::min<int64_t>(dblocks, int64_t(t.n_cu) * 16));
                hipLaunchKernelGGL((k_decode<PK, false>), dim3(dgrid), dim3(kDecodeThreads), 0, s, a, n_pad);
            }
            err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
        if (ev && (err = hipEventRecord(ev[1], s)) != hipSuccess) return err;
        for (int p = 0; p < P; ++p) {
            a.q0 = p * npw<A>() * G * W;
            const bool dec = p == 0 && inline_decode;
            const int64_t tl = dec ? tile_d : tile, cover = dec ? a.n_pad : a.n;
            const unsigned grid = static_cast<unsigned>(std::min<int64_t>((cover + tl - 1) / tl, int64_t(t.n_cu) * per_cu));
            const PassKernel kern = pass_kernel<A, G, W, PK>(p, P, inline_decode);
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, a);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
            if (ev && (err = hipEventRecord(ev[2 + p], s)) != hipSuccess) return err;
        }
    }
    return hipSuccess;
}

template <typename A, int G, int W>
hipError_t run_pack(const PassArgs &a, const Table &t, const FoldLayout &fl, hipStream_t s,
                    hipEvent_t *ev) {
    return fl.E <= Pk32::kMaxE ? run_passes<A, G, W, Pk32>(a, t, fl, s, ev)
                               : run_passes<A, G, W, Pk64>(a, t, fl, s, ev);
}

template <typename A>
hipError_t run_layout(const PassArgs &a, const Table &t, const FoldLayout &fl, hipStream_t s,
                      hipEvent_t *ev) {
    const int G = fl.G, W = fl.W;
    if (G == 16 && W == 1) return run_pack<A, 16, 1>(a, t, fl, s, ev);
    if (G == 8 && W == 2) return run_pack<A, 8, 2>(a, t, fl, s, ev);
    if (G == 8 && W == 1) return run_pack<A, 8, 1>(a, t, fl, s, ev);
    if (G == 4 && W == 2) return run_pack<A, 4, 2>(a, t, fl, s, ev);
    if (G == 2 && W == 4) return run_pack<A, 2, 4>(a, t, fl, s, ev);
    if (G == 1 && W == 8) return run_pack<A, 1, 8>(a, t, fl, s, ev);
    if (G == 4 && W == 1) return run_pack<A, 4, 1>(a, t, fl, s, ev);
    return hipErrorInvalidValue;
}

}  // namespace

int packed_entry_bytes(int E) { return E <= Pk32::kMaxE ? 4 : 8; }

namespace {
// Device address of `scratch` on each device, looked up once per device with
// that device current (each device holds the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void **p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!q) return hipErrorInvalidSymbol;
        g_noalloc_ptr[dev] = q;
    }
    *p = g_noalloc_ptr[dev];
    return hipSuccess;
}

namespace {
const FoldLayout &layout_of(const Table &t, pwc_precision p) {
    return p == PWC_MIXED ? t.flm : p == PWC_FP32 ? t.fls : t.fl;
}

// The decoded stream of the separate launches: one slab, padded.
size_t passes_scratch_bytes(const Table &t, int64_t n) {
    const int64_t slab = std::min<int64_t>(n, kRecSlab);
    return static_cast<size_t>(packed_entry_bytes(t.fl.E)) *
           static_cast<size_t>((slab + kStreamPad - 1) / kStreamPad * kStreamPad);
}
}  // namespace

size_t reconstruct_scratch_bytes(const Table &t, int64_t n, pwc_precision p) {
    if (fused_layout(layout_of(t, p), fold_maps_bytes(t.N, t.nd))) return 0;
    return passes_scratch_bytes(t, n);
}

hipError_t launch_reconstruct(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                              pwc_precision p, hipStream_t s, hipEvent_t *stage_ev, int *d_err,
                              void *d_scratch) {
    if (n <= 0) return hipSuccess;
    PassArgs a{};
    a.quads = reinterpret_cast<const int4 *>(d_quads);
    a.n = n;
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.fold = t.d_fold;
    a.K = t.K;
    a.nd = t.nd;
    a.E = t.fl.E;
    a.E1 = t.E1;
    a.ndir = t.ndir;
    a.Qp = t.fl.Qp;
    a.Q = t.Q;
    a.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    a.ord_g = layout_of(t, p).G;
    a.out = d_out;
    a.err = d_err ? d_err : t.d_err;
    // The decoded stream: the caller's fixed scratch (it holds the whole
    // padded stream, checked by the caller), else a stream-ordered
    // allocation of one slab, freed behind the passes.
    hipError_t err = hipSuccess;
    // Per-launch timing always takes the separate launches, which keep the
    // decoded stream even where the fused schedule would not.
    const bool fused = !stage_ev && fused_layout(layout_of(t, p), fold_maps_bytes(t.N, t.nd));
    if (d_scratch || fused) {
        a.scratch = d_scratch;   // the fused schedule keeps no decoded stream
    } else {
        err = hipMallocAsync(&a.scratch, passes_scratch_bytes(t, n), s);
        if (err != hipSuccess) return err;
    }
    if (p == PWC_MIXED) {
        a.tab = t.d_tauHL;
        err = run_layout<FF>(a, t, t.flm, s, stage_ev);
    } else if (p == PWC_FP32) {
        a.tab = t.d_tau32;
        err = run_layout<F32>(a, t, t.fls, s, stage_ev);
    } else {
        a.tab = t.d_tauF;
        err = run_layout<F64>(a, t, t.fl, s, stage_ev);
    }
    if (!d_scratch && !fused) {
        const hipError_t e2 = hipFreeAsync(a.scratch, s);
        if (err == hipSuccess) err = e2;
    }
    return err;
}

}  // namespace pwc

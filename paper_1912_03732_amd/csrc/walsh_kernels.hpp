// walsh_kernels.hpp -- gfx950 kernels for the fused S-box Walsh transform.
//
// One column of the Walsh matrix (Eq. 1) per nonzero output mask b is the
// length-2^n fast Walsh-Hadamard transform (Algorithm 1) of the polarity
// truth table of x -> parity(b & S[x]) (Eq. 2).  The per-mask maximum of
// |W| is folded into the last butterfly stage (Algorithm 3) and the minimum
// over masks (Algorithm 6) into a device atomic, so the 2^(n+m) matrix is
// only written when a spectrum layout is requested.
//
// How the work maps onto CDNA4 (wave64, 256-thread workgroups):
//
//  * Bit-sliced component tables.  F[i][w] holds bit i of S[32w .. 32w+31]
//    as one 32-bit word, so the 32 polarity bits of mask b over a word are
//    G_b[w] = XOR_{i in b} F[i][w].  A thread group walks its masks in
//    Gray-code order, so moving to the next mask costs one XOR per word.
//
//  * Five butterfly stages for the price of a popcount.  For the 32 inputs
//    x' of one word, the 32-point transform of (-1)^g at output a' equals
//    32 - 2 * popcount(G ^ L(a')), where L(a') is the truth table of
//    x' -> parity(a' & x').  The kernel carries c'(a') = popcount - 16, so
//    that every later value is exactly -W/2 (no correction at a = 0).
//
//  * Packed 16-bit arithmetic.  c' lies in [-16, 16] and each later stage
//    at most doubles it, so after all n <= 16 stages |value| <= 2^15.  Two
//    values share one VGPR (v_pk_add_u16 / v_pk_sub_u16), wrapping mod 2^16.
//    Only +-32768 collide under the wrap (n = 16), and they have the same
//    magnitude, so max |value| is still exact when tracked as
//    max(max_i16, -min_i16) in 32 bits.  Modes that store values do the
//    last stage in 32-bit instead.
//
//  * Register / LDS split.  x = (x_hi : Q bits, x_lo : P bits).  Phase 1:
//    a thread owns one x_hi and all 2^P x_lo values (2^(P-1) packed VGPRs)
//    and runs the popcount stages plus the P - 5 remaining low stages in
//    registers.  One LDS transpose then gives each thread all x_hi values
//    for some low outputs and phase 2 runs the Q high stages in registers.
//    When Q == P the last high bit lives on lane bit 5 and is brought into
//    registers with v_permlane32_swap.  n <= 8 needs no exchange at all:
//    one lane owns one mask.
//
//  * Persistent workgroups pull items from a device counter; an item is a
//    run of consecutive Gray-code indices for each thread group of the
//    workgroup.  Batched launches use the same kernels with a job table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbw {

// Work-item and group indices straight from the compiler's builtins.  The
// library is built without IEEE mode, and the device library's functions
// behind threadIdx / blockIdx / blockDim / gridDim (built in IEEE mode) could
// then not be inlined: every kernel called them, which cost registers and
// made uniform indices look like per-lane values.
__device__ __forceinline__ unsigned tid_x() { return __builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ unsigned bid_x() { return __builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ unsigned bid_y() { return __builtin_amdgcn_workgroup_id_y(); }
__device__ __forceinline__ unsigned bdim_x() { return __builtin_amdgcn_workgroup_size_x(); }
__device__ __forceinline__ unsigned gdim_x() { return __builtin_amdgcn_grid_size_x() / __builtin_amdgcn_workgroup_size_x(); }

// Product of two values that fit in 24 bits (v_mul_i32_i24): the operands
// are sign-extended from bit 23, which the backend turns into the 24-bit
// multiply, where the device library's __mul24 would be a call here.
__device__ __forceinline__ int32_t mul24s(int32_t a, int32_t b) { return ((a << 8) >> 8) * ((b << 8) >> 8); }

constexpr int kWG = 256;  // threads per workgroup (4 waves)

// kSlab16: b-major rows of -W/2 as int16 into a slab (the a-major path transposes them)
enum Mode : int { kMax = 0, kStoreB = 1, kStoreA = 2, kBlock = 3, kHist = 4, kHistBig = 5, kSlab16 = 6 };

// |W| histogram: kHist counts the bins |W|/2 < kHistBins - 1 in LDS per
// workgroup and only the number of larger values in the last LDS bin (no
// data-dependent branch per value); if that number is not zero, the
// kHistBig pass recomputes the transforms and adds the large values to the
// global histogram one by one.
constexpr int kHistBins = 2048;

// One S-box evaluation as the kernels see it.
struct JobDesc {
  const void* S;         // table, s_elem_bytes per entry
  const uint32_t* F;     // bit-sliced component words, [m][nwords]
  int32_t* maxabs;       // 2^m entries or null
  int32_t* nl;           // 1 entry
  int32_t* spec;         // spectrum (layout per kernel mode) or null
  long long item_begin;  // first queue item of this job (batched launches)
  int n, m;
  int nwords;            // words per slice (2^(n-5), at least 1)
  int s_elem_bytes;
  int wscale;            // stored value = wscale * (-W/2): -2 for W, -1 for the LAT (W/2)
  int flags;             // kWordsFp4: F holds the sparse words of the n = 12 fp4 engine
};

// JobDesc::flags
constexpr int kWordsFp4 = 1;
constexpr int kSpecAMajor = 2;  // spec is a-major (else b-major): where the batched start values go
constexpr int kPrepInline = 4;  // a one-workgroup launch (n <= 8) prepares its box itself

struct KParams {
  const JobDesc* jobs;   // device job table, or null to use job0
  JobDesc job0;
  int njobs;
  int chunk;             // Gray indices per thread group per item
  int* queue;            // work counter, zero before the launch
  long long total_items;
  // n > 16, first pass: 2^16-point transforms of the 2^(n-16) blocks of x
  int32_t* blockout;     // [kcount][2^n] int32
  long long kbase;       // first Gray index of this batch of masks
  long long kcount;      // masks in this batch (0: all 2^m masks, block mode: required)
  int nblk_log;          // n - 16
  int hist_cut;          // large-value pass: adds the values with |W|/2 >= hist_cut
  long long row0;        // b-major store mode: row b goes to spec + (b - row0) * 2^n
  long long rows;        // ... and only rows [0, rows) exist there (0: all 2^m)
  unsigned long long* hist;  // histogram modes: [2^(n-1) + 1] counts of |W|/2
  unsigned long long* hist_over;  // values past the LDS bins seen by the counting pass
  const int* gate;       // if set, the launch does nothing unless *gate == gate_run
  int gate_run;
};

// The host passes these structs by value as kernel arguments; both
// compilation passes (host and gfx950) must see the same layout.
static_assert(sizeof(JobDesc) == 72 && alignof(JobDesc) == 8, "JobDesc layout");
static_assert(sizeof(KParams) == 184 && __builtin_offsetof(KParams, gate_run) == 176, "KParams layout");

// A gated launch returns at once unless an earlier launch of the same call
// left *gate == gate_run (a choice between two routes taken on the device).
__device__ __forceinline__ bool gated_off(const KParams& kp) { return kp.gate && *kp.gate != kp.gate_run; }

// Defined with the preparation kernels below.
__device__ __forceinline__ void init_job(const JobDesc& jd, bool first, int* queue, int nqueue, int layout,
                                         bool spec_row = true);
template <int EB>
__device__ void bitslice_wave(const void* S, int m, uint32_t* F, int nwords, long long x0);

// The next work item of this workgroup from the queue counter, in the order
// workgroups ask (workgroup-uniform, kept scalar).  The barriers also keep
// the previous item's LDS use apart from this one's.  (A fixed assignment,
// workgroup g taking items g, g + G, ..., with no atomic, was measured
// slower for every single-box workload, e.g. 16 x 16 fused 0.589 ->
// 0.626 ms: workgroups that start late or run slower are not evened out.)
__device__ __forceinline__ long long next_item(const KParams& kp, long long* s_item) {
  if (tid_x() == 0) *s_item = (long long)atomicAdd(kp.queue, 1);
  __syncthreads();
  const long long item = __builtin_amdgcn_readfirstlane((int)*s_item);
  __syncthreads();
  return item;
}

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) int32_t gint32;  // global memory
typedef __attribute__((address_space(1))) int16_t gint16;
typedef int16_t s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}

// Truth table of x' -> parity(a & x') over the 32 positions of a word.
__host__ __device__ constexpr uint32_t walsh_mask(int a) {
  return ((a & 1) ? 0xAAAAAAAAu : 0u) ^ ((a & 2) ? 0xCCCCCCCCu : 0u) ^ ((a & 4) ? 0xF0F0F0F0u : 0u) ^
         ((a & 8) ? 0xFF00FF00u : 0u) ^ ((a & 16) ? 0xFFFF0000u : 0u);
}

__host__ __device__ constexpr long long gray(long long k) { return k ^ (k >> 1); }

// Running max / min of packed int16 outputs.
struct Tracker {
  s16x2 hi, lo;
  __device__ __forceinline__ void reset() {
    hi = s16x2{-32768, -32768};
    lo = s16x2{32767, 32767};
  }
  __device__ __forceinline__ void add(uint32_t v) {
    const s16x2 s = __builtin_bit_cast(s16x2, v);
    hi = __builtin_elementwise_max(hi, s);
    lo = __builtin_elementwise_min(lo, s);
  }
  // max |value| in 32-bit; -(-32768) = 32768 is representable here.
  __device__ __forceinline__ int result() const {
    const int a = max((int)hi.x, (int)hi.y);
    const int b = -min((int)lo.x, (int)lo.y);
    return max(a, b);
  }
};

// 2^(P-1) packed registers; butterfly on register index bit `bit`.
template <int NR>
__device__ __forceinline__ void stage_regs(uint32_t (&R)[NR], int bit) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r & bit) continue;
    const uint32_t u = R[r], v = R[r | bit];
    R[r] = pk_add(u, v);
    R[r | bit] = pk_sub(u, v);
  }
}

// Lanes 0-31 keep A and receive B's lanes 0-31 ... : v_permlane32_swap exchanges
// the upper 32 lanes of the first operand with the lower 32 lanes of the second.
__device__ __forceinline__ void swap_halves(uint32_t& a, uint32_t& b) {
  auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}

// An opaque copy: keeps the compiler from hoisting the per-thread output
// addresses of the store modes out of the mask loop (hundreds of them,
// which would otherwise be precomputed and spilled).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

__device__ __forceinline__ int unpack_lo(uint32_t v) { return (int)(int16_t)(v & 0xFFFFu); }
__device__ __forceinline__ int unpack_hi(uint32_t v) { return (int)v >> 16; }

// Output index of low register u, half h (phase-1 packing: register bits 0-3
// are a0..a3, the half is a4, register bits 4.. are a5..).
__device__ __forceinline__ uint32_t aidx(int u, int h) {
  return (uint32_t)((u & 15) | (h << 4) | ((u >> 4) << 5));
}

template <int NW>
__device__ __forceinline__ void load_words(uint32_t (&G)[NW], const uint32_t* p, bool x0r) {
  if constexpr (NW >= 4) {
#pragma unroll
    for (int i = 0; i < NW; i += 4) {
      const uint4 v = *reinterpret_cast<const uint4*>(p + i);
      if (x0r) {
        G[i] ^= v.x; G[i + 1] ^= v.y; G[i + 2] ^= v.z; G[i + 3] ^= v.w;
      } else {
        G[i] = v.x; G[i + 1] = v.y; G[i + 2] = v.z; G[i + 3] = v.w;
      }
    }
  } else if constexpr (NW == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    if (x0r) { G[0] ^= v.x; G[1] ^= v.y; } else { G[0] = v.x; G[1] = v.y; }
  } else {
    if (x0r) G[0] ^= p[0]; else G[0] = p[0];
  }
}

// The words of the first mask of a walk, gray(k): the XOR of the slices of
// its set bits.  Slices are loaded four at a time, the loads of a group in
// flight together (one after another, each load waited for before the next
// was issued, this start cost a few microseconds per work item).
template <int NW>
__device__ __forceinline__ void gray_start(uint32_t (&G)[NW], const uint32_t* F, long long nwords, long long wb,
                                           long long gk, int m) {
#pragma unroll
  for (int w = 0; w < NW; ++w) G[w] = 0;
  for (int i0 = 0; i0 < m; i0 += 4) {
    uint32_t T[4][NW];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = i0 + t;
      if (i < m && ((gk >> i) & 1)) {
        load_words<NW>(T[t], F + (long long)i * nwords + wb, false);
      } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) T[t][w] = 0;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int w = 0; w < NW; ++w) G[w] ^= T[t][w];
  }
}

// ---------------------------------------------------------------------------
// Maximum (or minimum) over groups of W consecutive lanes, W a power of two:
// DPP moves inside each row of 16 lanes (quad swaps, half-row and row
// mirrors) leave the group's result in all its lanes; 32 lanes add one
// cross-row shuffle, a whole wave combines its four rows through readlane
// (uniform result).  Replaces chains of dependent LDS permutes.
// ---------------------------------------------------------------------------
template <bool IS_MAX>
__device__ __forceinline__ int pick(int a, int b) { return IS_MAX ? max(a, b) : min(a, b); }

template <int W, bool IS_MAX = true>
__device__ __forceinline__ int group_reduce(int v) {
  if constexpr (W >= 2) v = pick<IS_MAX>(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));   // quad 1,0,3,2
  if constexpr (W >= 4) v = pick<IS_MAX>(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));   // quad 2,3,0,1
  if constexpr (W >= 8) v = pick<IS_MAX>(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));  // half-row mirror
  if constexpr (W >= 16) v = pick<IS_MAX>(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false)); // row mirror
  if constexpr (W == 32) v = pick<IS_MAX>(v, __shfl_xor(v, 16, 64));
  if constexpr (W == 64)
    v = pick<IS_MAX>(pick<IS_MAX>(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
                     pick<IS_MAX>(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
  return v;
}
__device__ __forceinline__ int wave_max(int v) { return group_reduce<64, true>(v); }
__device__ __forceinline__ int wave_min(int v) { return group_reduce<64, false>(v); }

// NL = the minimum over a box's masks of 2^(n-1) - max|W|/2, taken with
// atomicMin.  The memory system serialises device-scope atomics on one
// address (about 10 ns apart: a 12 x 12 call took 20.6 / 33 / 59 us with
// 1,024 / 2,048 / 4,096 of them), so the kernels issue few: a launch over
// one box keeps each lane's candidate over all its items and adds one
// value per workgroup when it ends; a batched launch, whose consecutive
// items belong to different boxes, adds one value per wave and item.
// (12 x 12 fused 20.6 -> 12.3 us, 12 x 20 0.408 -> 0.375 ms, the 4096-box
// batch 0.86 -> 0.82 ms.)  Kernels whose workgroup works on one mask at a
// time (n = 16) keep one add per item, which is one atomic already.  Lanes
// without a candidate hold 0x7fffffff.
__device__ __forceinline__ void nl_add_wave(int32_t* nl, int v) {
  v = wave_min(v);
  if ((tid_x() & 63) == 0 && v != 0x7fffffff) atomicMin(nl, v);
}
__device__ __forceinline__ void nl_add_workgroup(int32_t* nl, int v) {
  __shared__ int s_min;
  v = wave_min(v);
  if (tid_x() == 0) s_min = 0x7fffffff;
  __syncthreads();
  if ((tid_x() & 63) == 0 && v != 0x7fffffff) atomicMin(&s_min, v);
  __syncthreads();
  if (tid_x() == 0 && s_min != 0x7fffffff) atomicMin(nl, s_min);
}

// ---------------------------------------------------------------------------
// Main fused kernel, n <= 16 (MODE kBlock: one 2^16 block of a larger n).
// ---------------------------------------------------------------------------
constexpr int kLdsStride = kWG + 1;  // padded LDS row (odd number of words)

// Workgroups per CU the register budget is tuned for: the 16-bit-input
// kernel with the two-round exchange fits two (<= 256 VGPRs per lane).
template <int N, int P_, int MODE>
constexpr int min_blocks() {
  return (N == 16 && P_ == 8 && (MODE == kMax || MODE == kStoreB || MODE == kSlab16 || MODE == kHist)) ? 2 : 1;  // kHistBig: 1
}

template <int N, int P_, int MODE>
__global__ __launch_bounds__(kWG, (min_blocks<N, P_, MODE>())) void k_walsh(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int P = (N <= 8) ? N : P_;
  constexpr int Q = N - P;
  static_assert(Q >= 0 && Q <= P, "bad split");
  static_assert(N <= 8 || (P >= 6 && P <= 8), "bad split");
  constexpr int NW = (N >= 5) ? (1 << (P - 5)) : 1;   // words per thread
  constexpr int NR = (N >= 5) ? NW * 16 : 1;          // packed registers
  constexpr int GPW = kWG >> Q;                       // thread groups per workgroup
  constexpr bool STORE = MODE != kMax;
  constexpr int SWZ_SHIFT = (Q >= 1 && Q <= P - 1) ? (P - 1 - Q) : 0;
  constexpr int U2 = (Q >= 1 && Q <= P - 1) ? (1 << (P - 1 - Q)) : 1;

  constexpr bool TWO_ROUND =
      ((MODE == kMax || MODE == kStoreB || MODE == kSlab16 || MODE == kHist || MODE == kHistBig) && Q == P && P == 8);
  constexpr int LDS_WORDS = (Q == 0) ? 1 : (Q <= P - 1) ? NR * kWG : (TWO_ROUND ? 64 : NR) * kLdsStride;
  __shared__ uint32_t lds[LDS_WORDS];
  __shared__ int red[kWG / 64];
  __shared__ long long s_item;
  __shared__ uint32_t hl[MODE == kHist ? kHistBins : 1];

  const int tid = tid_x();
  // histogram mode: counts since the last flush of hl (workgroup-uniform)
  long long hcount = 0;
  auto hist_flush = [&]() {
    for (int k = tid; k < kHistBins; k += kWG) {
      const uint32_t c = hl[k];
      if (c) {
        atomicAdd(k == kHistBins - 1 ? kp.hist_over : kp.hist + k, (unsigned long long)c);
        hl[k] = 0;
      }
    }
  };
  if constexpr (MODE == kHist)
    for (int k = tid; k < kHistBins; k += kWG) hl[k] = 0;  // ordered by the loop's first barrier
  if constexpr (MODE == kHistBig)
    if (*kp.hist_over == 0) return;  // no large value: nothing to add
  // A launch that is one workgroup over a whole small box (6 <= n <= 8, at
  // most 256 masks, one item) bit-slices the table (a wave per 64 entries,
  // a ballot per output bit) and sets the call's start values itself, so the
  // call is this one launch; it zeroes its queue counter too, from which
  // thread 0 then takes the item.  The barrier makes the words visible to
  // the workgroup.
  if constexpr (N >= 6 && N <= 8 && (MODE == kMax || MODE == kStoreB || MODE == kStoreA)) {
    if (kp.job0.flags & kPrepInline) {
      const JobDesc& j0 = kp.job0;
      if (tid == 0) *kp.queue = 0;
      init_job(j0, false, nullptr, 0, MODE == kStoreA ? 2 : 1);
      const long long x0 = tid & ~63;
      if (x0 < (1 << N)) {
        uint32_t* F = const_cast<uint32_t*>(j0.F);
        if (j0.s_elem_bytes == 1) bitslice_wave<1>(j0.S, j0.m, F, j0.nwords, x0);
        else if (j0.s_elem_bytes == 2) bitslice_wave<2>(j0.S, j0.m, F, j0.nwords, x0);
        else bitslice_wave<4>(j0.S, j0.m, F, j0.nwords, x0);
      }
      __syncthreads();
    }
  }
  // thread group in this workgroup (wave-uniform when a group spans whole waves)
  const int g = (Q >= 6) ? __builtin_amdgcn_readfirstlane(tid >> Q) : (tid >> Q);
  const int tg = tid & ((1 << Q) - 1);    // thread within the group
  const int lane = tid & 63;
  const int C = kp.chunk;

  // NL candidate of this lane: per item in a batch, over all its items for one box
  int runmin = 0x7fffffff;
  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;

    // ---- decode the item
    JobDesc jd;
    long long li;
    int xblk = 0;
    if constexpr (MODE == kBlock) {
      jd = kp.job0;
      xblk = (int)(item & ((1LL << kp.nblk_log) - 1));
      li = item >> kp.nblk_log;
    } else if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = kp.kbase + (li * GPW + g) * (long long)C;
    const long long kend = (kp.kcount > 0) ? (kp.kbase + kp.kcount) : (1LL << jd.m);
    const long long wb = (MODE == kBlock ? ((long long)xblk << 11) : 0) + (long long)tg * NW;
    const int n = jd.n;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      const bool inrange = k < kend;
      // ---- component words of mask gray(k) (Gray-code walk); the slice for
      // the next mask is fetched one mask ahead to hide its L2 latency
      if (step == 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] = 0;
        if (inrange) gray_start<NW>(G, jd.F, jd.nwords, wb, gray(k), jd.m);
      } else if (inrange) {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] ^= Fn[w];
      }
      if (step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      const uint32_t b = (uint32_t)gray(k);
      // a b-major slab holds rows [row0, row0 + rows) only
      const bool inslab = (MODE != kStoreB && MODE != kSlab16) || kp.rows == 0 ||
                          (unsigned long long)((long long)b - kp.row0) < (unsigned long long)kp.rows;
      const bool valid = inrange && k != 0 && inslab;
      const long long slot = k - kp.kbase;  // kBlock only

      int mx = 0;
      // Store modes: every emit happens under `valid` (one branch per mask,
      // not per store), through a global-address-space row pointer.
      gint32* gdst = nullptr;
      if constexpr (MODE == kStoreB) gdst = (gint32*)(jd.spec + ((size_t)(b - kp.row0) << N));
      if constexpr (MODE == kStoreA) gdst = (gint32*)(jd.spec + b);
      gint16* hdst = nullptr;  // kSlab16: int16 rows
      if constexpr (MODE == kSlab16)
        hdst = (gint16*)(reinterpret_cast<int16_t*>(jd.spec) + ((size_t)(b - kp.row0) << N));
      if constexpr (MODE == kBlock)
        gdst = (gint32*)(kp.blockout + ((size_t)slot << (16 + kp.nblk_log)) + ((size_t)xblk << 16));
      auto emit = [&](uint32_t a, int v) {  // v = -W(a,b)/2 (or the block value)
        mx = max(mx, v < 0 ? -v : v);
        if constexpr (MODE == kHist) atomicAdd(&hl[min(v < 0 ? -v : v, kHistBins - 1)], 1u);
        if constexpr (MODE == kHistBig) {
          const int av = v < 0 ? -v : v;
          if (av >= kp.hist_cut) atomicAdd(kp.hist + av, 1ull);
        }
        // a < 2^16 here, so a 32-bit byte offset from a scalar row base suffices
        if constexpr (MODE == kStoreB)
          *(gint32*)((__attribute__((address_space(1))) char*)gdst + (uint32_t)(a << 2)) = jd.wscale * v;
        if constexpr (MODE == kStoreA) gdst[(size_t)a << jd.m] = jd.wscale * v;
        // |v| <= 2^15; v = 2^15 (an affine component at n = 16) wraps to -2^15
        if constexpr (MODE == kSlab16)
          *(gint16*)((__attribute__((address_space(1))) char*)hdst + (uint32_t)(a << 1)) = (int16_t)v;
        if constexpr (MODE == kBlock)
          *(gint32*)((__attribute__((address_space(1))) char*)gdst + (uint32_t)(a << 2)) = v;
      };

      if constexpr (N < 5) {
        // ---- fewer than 32 inputs: the whole transform is popcounts
        constexpr uint32_t low = (N == 0) ? 1u : ((1u << (1 << N)) - 1u);
        if (!STORE || valid) {
#pragma unroll
          for (int a = 0; a < (1 << N); ++a) {
            const int c = __builtin_popcount((G[0] ^ walsh_mask(a)) & low) - (1 << (N - 1));
            emit((uint32_t)a, c);
          }
        }
      } else {
        // ---- phase 1: popcount stages (x0..x4) + register stages (x5..x_{P-1})
        uint32_t R[NR];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
#pragma unroll
          for (int a = 0; a < 16; ++a) {
            const int c0 = __builtin_popcount(G[w] ^ walsh_mask(a)) - 16;
            const int c1 = __builtin_popcount(G[w] ^ walsh_mask(a | 16)) - 16;
            R[w * 16 + a] = __builtin_amdgcn_perm((uint32_t)c1, (uint32_t)c0, 0x05040100u);
          }
        }
        constexpr int LAST1 = P - 2;  // highest register bit of phase 1
        if constexpr (Q == 0) {
          if constexpr (P == 5) {
            if constexpr (STORE) {
              if (valid) {
#pragma unroll
              for (int r = 0; r < NR; ++r) {
                emit(aidx(r, 0), unpack_lo(R[r]));
                emit(aidx(r, 1), unpack_hi(R[r]));
              }
            }
            } else {
              Tracker t; t.reset();
#pragma unroll
              for (int r = 0; r < NR; ++r) t.add(R[r]);
              mx = t.result();
            }
          } else {
#pragma unroll
            for (int d = 4; d < LAST1; ++d) stage_regs<NR>(R, 1 << d);
            constexpr int fb = 1 << LAST1;
            if constexpr (STORE) {
              if (valid) {
#pragma unroll
              for (int r = 0; r < NR; ++r) {
                if (r & fb) continue;
                const uint32_t u = R[r], v = R[r | fb];
                emit(aidx(r, 0), unpack_lo(u) + unpack_lo(v));
                emit(aidx(r, 1), unpack_hi(u) + unpack_hi(v));
                emit(aidx(r | fb, 0), unpack_lo(u) - unpack_lo(v));
                emit(aidx(r | fb, 1), unpack_hi(u) - unpack_hi(v));
              }
            }
            } else {
              Tracker t; t.reset();
#pragma unroll
              for (int r = 0; r < NR; ++r) {
                if (r & fb) continue;
                t.add(pk_add(R[r], R[r | fb]));
                t.add(pk_sub(R[r], R[r | fb]));
              }
              mx = t.result();
            }
          }
        } else {
#pragma unroll
          for (int d = 4; d <= LAST1; ++d) stage_regs<NR>(R, 1 << d);
          if constexpr (Q <= P - 1) {
            // ---- LDS transpose: row u (low output pair), column = thread,
            // columns XOR-swizzled by the reader's group-thread index
#pragma unroll
            for (int u = 0; u < NR; ++u) lds[u * kWG + (tid ^ ((u >> SWZ_SHIFT) & 31))] = R[u];
            __syncthreads();
            // thread (g, v): pairs u = v*U2 + j, all 2^Q high inputs
#pragma unroll
            for (int j = 0; j < U2; ++j) {
              const int u = tg * U2 + j;
              const int sw = tg & 31;
#pragma unroll
              for (int y = 0; y < (1 << Q); ++y)
                R[j * (1 << Q) + y] = lds[u * kWG + (((g << Q) + y) ^ sw)];
            }
#pragma unroll
            for (int d = 0; d < Q - 1; ++d) stage_regs<NR>(R, 1 << d);
            constexpr int fb = 1 << (Q - 1);
            if constexpr (STORE) {
              if (valid) {
#pragma unroll
              for (int r = 0; r < NR; ++r) {
                if (r & fb) continue;
                const int j = r >> Q, y = r & ((1 << Q) - 1);
                const int u = opaque(tg) * U2 + j;
                const uint32_t uu = R[r], vv = R[r | fb];
                emit(aidx(u, 0) | ((uint32_t)y << P), unpack_lo(uu) + unpack_lo(vv));
                emit(aidx(u, 1) | ((uint32_t)y << P), unpack_hi(uu) + unpack_hi(vv));
                emit(aidx(u, 0) | ((uint32_t)(y | fb) << P), unpack_lo(uu) - unpack_lo(vv));
                emit(aidx(u, 1) | ((uint32_t)(y | fb) << P), unpack_hi(uu) - unpack_hi(vv));
              }
            }
            } else {
              Tracker t; t.reset();
#pragma unroll
              for (int r = 0; r < NR; ++r) {
                if (r & fb) continue;
                t.add(pk_add(R[r], R[r | fb]));
                t.add(pk_sub(R[r], R[r | fb]));
              }
              mx = t.result();
            }
          } else {
            // Q == P: thread (u, h) with h on lane bit 5
            const int u = (tg & 31) | ((tg >> 6) << 5);
            const int h = (tg >> 5) & 1;
            constexpr int HALF = 1 << (Q - 1);
            constexpr int H2 = 1 << (Q - 2);
            if constexpr (TWO_ROUND) {
              // Two half-size rounds (64 KiB of LDS, two workgroups per CU).
              // Round r moves the elements (u, x_hi) with u[6] ^ x_hi[6] == r.
              // A writer (x_hi = tid) frees register half r ^ tid[6] and the
              // reader fills that same half with its i[6] == r ^ u[6] inputs,
              // so physical register j holds logical input j ^ (flip << 6).
              // The butterfly on bit 6 undoes the relabelling up to the sign
              // of one half, which the maximum does not see.
              const int wb6 = (tid >> 6) & 1;  // wave-uniform
              const int ru = u >> 6;           // wave-uniform
#pragma unroll
              for (int r = 0; r < 2; ++r) {
                if ((r ^ wb6) == 0) {
#pragma unroll
                  for (int j = 0; j < 64; ++j) lds[j * kLdsStride + tid] = R[j];
                } else {
#pragma unroll
                  for (int j = 0; j < 64; ++j) lds[j * kLdsStride + tid] = R[64 + j];
                }
                __syncthreads();
                const int src = (u & 63) * kLdsStride + h * HALF + ((r ^ ru) << 6);
                if ((r ^ wb6) == 0) {
#pragma unroll
                  for (int i = 0; i < 64; ++i) R[i] = lds[src + i];
                } else {
#pragma unroll
                  for (int i = 0; i < 64; ++i) R[64 + i] = lds[src + i];
                }
                if (r == 0) __syncthreads();
              }
            } else {
              // one round, rows padded to an odd stride: conflict-free both ways
#pragma unroll
              for (int u2 = 0; u2 < NR; ++u2) lds[u2 * kLdsStride + tid] = R[u2];
              __syncthreads();
              const int src = u * kLdsStride + (g << Q) + h * HALF;
#pragma unroll
              for (int i = 0; i < HALF; ++i) R[i] = lds[src + i];
            }
#pragma unroll
            for (int d = 0; d < Q - 1; ++d) stage_regs<NR>(R, 1 << d);
#pragma unroll
            for (int i = 0; i < H2; ++i) swap_halves(R[i], R[i + H2]);
            if constexpr (STORE) {
              if (valid) {
              // With the two-round exchange a wave whose physical register
              // halves are swapped (flip = tid[6] ^ u[6]) ends with the
              // lanes of h = 1 holding the negated outputs.
              int sgn = 1;
              if constexpr (TWO_ROUND) sgn = ((((tid >> 6) ^ (u >> 6)) & 1) && h) ? -1 : 1;
              const uint32_t abase = (uint32_t)opaque((int)(aidx(u, 0) | ((uint32_t)(h * H2) << P)));
#pragma unroll
              for (int i = 0; i < H2; ++i) {
                const uint32_t uu = R[i], vv = R[i + H2];
                const uint32_t a0 = abase + ((uint32_t)i << P);
                constexpr uint32_t top = 1u << (N - 1);
                emit(a0, sgn * (unpack_lo(uu) + unpack_lo(vv)));
                emit(a0 + 16, sgn * (unpack_hi(uu) + unpack_hi(vv)));
                emit(a0 + top, sgn * (unpack_lo(uu) - unpack_lo(vv)));
                emit(a0 + top + 16, sgn * (unpack_hi(uu) - unpack_hi(vv)));
              }
            }
            } else {
              Tracker t; t.reset();
#pragma unroll
              for (int i = 0; i < H2; ++i) {
                t.add(pk_add(R[i], R[i + H2]));
                t.add(pk_sub(R[i], R[i + H2]));
              }
              mx = t.result();
            }
          }
        }
      }

      // ---- per-mask maximum over the thread group
      if constexpr (Q >= 1) {
        constexpr int W = (Q < 6) ? (1 << Q) : 64;
        mx = group_reduce<W>(mx);
      }
      if constexpr (Q >= 7) {
        if (lane == 0) red[tid >> 6] = mx;
      }
      if constexpr (Q >= 1) __syncthreads();  // LDS rows are rewritten by the next mask
      if constexpr (Q >= 7) {
        constexpr int WPG = 1 << (Q - 6);  // waves per group
        int gm = 0;
#pragma unroll
        for (int w = 0; w < WPG; ++w) gm = max(gm, red[g * WPG + w]);
        mx = gm;
      }
      if constexpr (MODE != kBlock && MODE != kHistBig) {
        if (tg == 0 && valid) {
          if (jd.maxabs) jd.maxabs[b] = 2 * mx;
          runmin = min(runmin, (1 << (n - 1)) - mx);
        }
      }
    }
    if constexpr (MODE != kBlock && MODE != kHistBig) {
      if (GPW == 1) {  // one thread group a workgroup: one add an item (deferring it measured slower at n = 16)
        if (tg == 0 && runmin != 0x7fffffff) atomicMin(jd.nl, runmin);
        runmin = 0x7fffffff;
      } else if (kp.jobs != nullptr) {
        nl_add_wave(jd.nl, runmin);
        runmin = 0x7fffffff;
      }
    }
    if constexpr (MODE == kHist) {
      // keep every LDS count below 2^32
      hcount += ((long long)GPW * C) << N;
      if (hcount > (1LL << 31)) {
        __syncthreads();
        hist_flush();
        hcount = 0;
      }
    }
  }
  if constexpr (MODE != kBlock && MODE != kHistBig && GPW > 1)
    if (kp.jobs == nullptr) nl_add_workgroup(kp.job0.nl, runmin);
  if constexpr (MODE == kHist) {
    __syncthreads();
    hist_flush();
  }
}

// ---------------------------------------------------------------------------
// n = 16, max mode, matrix-core variant.
//
// Bits of x: x0..x4 inside a word (popcount stages, as above); x5..x7 index
// a thread's 8 words; x8..x15 = t, the thread in the workgroup (lane bits
// x8..x13, wave bits x14, x15).
//   1. Popcount stages, written straight as fp16 bit patterns:
//      bcnt(G ^ L(a'), 0x6600 - 16) is the pattern of 1536 + c' (the fp16
//      binade [1024, 2048) has unit spacing); two of them are packed over x5.
//      The offset 1536 is left in: it is uniform over every input of the
//      next transform, and a Hadamard column other than the first sums to
//      zero, so it only adds 32 * 1536 to output column 0 of that transform,
//      which the MFMA's accumulator input takes off again.
//   2. Exchange through LDS so that wave w receives the a' with a' >> 3 = w
//      from all four waves: lane l keeps t mod 64 and the register for
//      (a', v = (x6, x7), s) holds the x5 pair of thread t = l + 64 s.  In R
//      rounds (a' bits 1, 2 ... select the round), each small enough that
//      several workgroups share a CU.
//   3. Pass 1, for each (a', v): the 8 fp16 over (x5, s) are the A operand
//      (16 x 32, rows = t mod 16, K slots = (x5, x14, x15, x12, x13)) of
//      v_mfma_f32_16x16x32_f16 against the two 16-column halves of H_32,
//      with the offset correction as the accumulator input.  |value| <= 512.
//   4. The results are cast to fp16 (exact) and one packed-fp16 butterfly
//      stage runs over x7 (|value| <= 1024, exact).
//   5. Pass 2: in the result layout a lane holds rows 4 (lane / 16) + i of a
//      16 x 16 tile, column lane mod 16, so the four results of the tiles for
//      x6 = 0 and x6 = 1 form a new A operand whose K slots are
//      (x8, x9, x6, x10, x11); the same H_32 halves transform them.
//   6. |value| <= 2^15 at the end, exact in fp32; the maximum is taken with
//      abs modifiers.
// Every bit of x is transformed exactly once (5 + 5 + 1 + 5); which output
// index lands where does not matter for the maximum.
// ---------------------------------------------------------------------------
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pkf16_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, a) + __builtin_bit_cast(f16x2, b));
}
__device__ __forceinline__ uint32_t pkf16_sub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, a) - __builtin_bit_cast(f16x2, b));
}
__device__ __forceinline__ _Float16 hsign(int bits) { return (__builtin_popcount(bits) & 1) ? (_Float16)-1.0f : (_Float16)1.0f; }
__device__ __forceinline__ uint32_t pk_cvt_f16(float lo, float hi) {
  f16x2 r;
  r[0] = (_Float16)lo;
  r[1] = (_Float16)hi;
  return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ f16x8 as_f16x8(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3) {
  const f16x2 p0 = __builtin_bit_cast(f16x2, r0), p1 = __builtin_bit_cast(f16x2, r1);
  const f16x2 p2 = __builtin_bit_cast(f16x2, r2), p3 = __builtin_bit_cast(f16x2, r3);
  f16x8 v;
  v[0] = p0[0]; v[1] = p0[1]; v[2] = p1[0]; v[3] = p1[1];
  v[4] = p2[0]; v[5] = p2[1]; v[6] = p3[0]; v[7] = p3[1];
  return v;
}

template <int ROUNDS>
__global__ __launch_bounds__(kWG, ROUNDS) void k_walsh_mfma16(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int NW = 8;
  constexpr int TPR = 8 / ROUNDS;              // a' & 7 values per round
  constexpr int LDSW = 4 * TPR * 4 * 4 * 64;   // dest wave x (a' & 7) x v x source wave x lane
  static_assert(ROUNDS == 2 || ROUNDS == 4, "rounds");
  __shared__ uint32_t lds[LDSW];
  __shared__ int red[64 * 4];  // per mask of a run of 64: the 4 wave maxima
  __shared__ long long s_item;

  const int tid = tid_x();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int C = kp.chunk;

  // B operands: slot (g = lane / 16, j) is the 5-bit index kappa = j + 8 g;
  // column n = lane % 16 (+ 16 for the second half).
  f16x8 hb0, hb1;
  {
    const int g = lane >> 4, n = lane & 15;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kappa = j + 8 * g;
      hb0[j] = hsign(kappa & n);
      hb1[j] = hsign(kappa & (n + 16));
    }
  }
  // accumulator input of pass 1, first half: takes 32 * 1536 off column 0
  const float fix = (lane & 15) == 0 ? -49152.0f : 0.0f;
  const f32x4 cfix = {fix, fix, fix, fix};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};

  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;
    JobDesc jd;
    long long li;
    if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {  // batched: find the job owning this item
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = li * (long long)C;
    const long long kend = 1LL << jd.m;
    const long long wb = (long long)tid * NW;
    const int n = jd.n;
    int runmin = 0x7fffffff;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      const bool inrange = k < kend;
      if (step == 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] = 0;
        if (inrange) gray_start<NW>(G, jd.F, jd.nwords, wb, gray(k), jd.m);
      } else if (inrange) {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] ^= Fn[w];
      }
      if (step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {

        // ---- 1. popcount stages of the a' = dw * 8 + r * TPR + tt, to LDS
#pragma unroll
        for (int dw = 0; dw < 4; ++dw)
#pragma unroll
          for (int tt = 0; tt < TPR; ++tt) {
            const uint32_t L = walsh_mask(dw * 8 + r * TPR + tt);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const uint32_t c0 = __builtin_popcount(G[2 * v] ^ L) + (0x6600 - 16);
              const uint32_t c1 = __builtin_popcount(G[2 * v + 1] ^ L) + (0x6600 - 16);
              lds[(((dw * TPR + tt) * 4 + v) * 4 + wave) * 64 + lane] = __builtin_amdgcn_perm(c1, c0, 0x05040100u);
            }
          }
        __syncthreads();
        uint32_t R[TPR][4][4];
#pragma unroll
        for (int tt = 0; tt < TPR; ++tt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int s = 0; s < 4; ++s) R[tt][v][s] = lds[(((wave * TPR + tt) * 4 + v) * 4 + s) * 64 + lane];
        __syncthreads();
#pragma unroll
        for (int tt = 0; tt < TPR; ++tt) {
          // ---- 3. pass 1 per v, results to fp16: P[v][half][2]
          uint32_t P[4][2][2];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const f16x8 av = as_f16x8(R[tt][v][0], R[tt][v][1], R[tt][v][2], R[tt][v][3]);
            const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, cfix, 0, 0, 0);
            const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
            P[v][0][0] = pk_cvt_f16(d0[0], d0[1]);
            P[v][0][1] = pk_cvt_f16(d0[2], d0[3]);
            P[v][1][0] = pk_cvt_f16(d1[0], d1[1]);
            P[v][1][1] = pk_cvt_f16(d1[2], d1[3]);
          }
          // ---- 4. stage over x7 (v = x6 + 2 x7)
#pragma unroll
          for (int x6 = 0; x6 < 2; ++x6)
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
              for (int i = 0; i < 2; ++i) {
                const uint32_t p = P[x6][h][i], q = P[x6 + 2][h][i];
                P[x6][h][i] = pkf16_add(p, q);
                P[x6 + 2][h][i] = pkf16_sub(p, q);
              }
          // ---- 5. pass 2 per (a7, half), 6. the maximum
#pragma unroll
          for (int a7 = 0; a7 < 2; ++a7)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const f16x8 av = as_f16x8(P[2 * a7][h][0], P[2 * a7][h][1], P[2 * a7 + 1][h][0], P[2 * a7 + 1][h][1]);
              const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, zero, 0, 0, 0);
              const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
              // v_max3 with abs modifiers; the compiler inserts the wait
              // states an MFMA result needs before a VALU reads it
              m0 = fmaxf(fmaxf(m0, fabsf(e0[0])), fabsf(e1[0]));
              m1 = fmaxf(fmaxf(m1, fabsf(e0[1])), fabsf(e1[1]));
              m0 = fmaxf(fmaxf(m0, fabsf(e0[2])), fabsf(e1[2]));
              m1 = fmaxf(fmaxf(m1, fabsf(e0[3])), fabsf(e1[3]));
            }
        }
      }
      const int mx = wave_max((int)fmaxf(m0, m1));
      if (lane == 0) red[(step & 63) * 4 + wave] = mx;
      if ((step & 63) == 63 || step == C - 1) {
        // every 64 masks and at the item's end: wave 0 finishes the masks
        // kfirst + s0 .. kfirst + step, one per lane
        __syncthreads();
        if (wave == 0) {
          const long long s0 = step & ~63LL;
          const long long kk = kfirst + s0 + lane;
          int v = 0x7fffffff;
          if (s0 + lane <= step && kk < kend && kk != 0) {
            const int* pr = red + lane * 4;
            const int pm = max(max(pr[0], pr[1]), max(pr[2], pr[3]));
            if (jd.maxabs) jd.maxabs[(uint32_t)gray(kk)] = 2 * pm;
            v = (1 << (n - 1)) - pm;
          }
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
          runmin = min(runmin, v);
        }
        // no second barrier: red is next written after the next round's
        // first barrier, which wave 0 reaches only after these reads
      }
    }
    // a workgroup works on one mask at a time: already one add an item
    if (tid == 0 && runmin != 0x7fffffff) atomicMin(jd.nl, runmin);
  }
}

// ---------------------------------------------------------------------------
// n = 16, max mode, three matrix-core passes and no popcount stages: the
// first on fp4 (e2m1) operands taken straight from the bit-sliced words,
// the other two on fp16.
//
// Bits of x as in k_walsh_mfma16: x0..x4 inside a word, x5..x7 index a
// thread's 8 words, x8..x13 the lane, x14, x15 the wave.  A component value
// is carried as its bit: (-1)^bit = 1 - 2 bit, so with T the transform of
// the bits, W = 2^16 [a = 0] - 2 T, and the kernel tracks
// V = T - 2^15 [a = 0] = -W / 2.
//   1. Pass 1, v_mfma_scale_f32_16x16x128_f8f6f4 on e2m1: a word ANDed with
//      0x11111111 << t keeps bit t of every nibble (t = x0 + 2 x1, the
//      nibble = x2..x4), whose e2m1 value is 0.5, 1 or 2 for t = 0, 1, 2
//      (bit 3 is the sign, so t = 3 is first shifted down to 2); the
//      operand's power-of-two scale (2^1, 2^0, 2^-1) makes every kept bit
//      1.0.  K slots (x2, x3, x4 | x5, x6 | x12, x13), rows x8..x11, eight
//      16-column blocks of H_128.  Column 0 of block 0 gets -64 as the
//      accumulator input: the 2^9 tiles that reach output 0 remove 2^15.
//      |value| <= 64.
//   2. Pass 2, v_mfma_f32_16x16x32_f16: for a column block and a pair of
//      tile rows (x8, x9) the 8 pass-1 results over (t, x7) form the
//      operand's registers (t) and halves (x7); the lane's K slots are tile
//      rows x10, x11.  |value| <= 2048 (exact in fp16).
//   3. Exchange through LDS: a lane's upper two bits (pass-1 output bits
//      2, 3) trade places with the wave (x14, x15).
//   4. Pass 3, v_mfma_f32_16x16x32_f16 with K slots (pass-2 row bit 0 |
//      x8, x9 | x14, x15) against H_16 (x) I_2: the first slot is passed
//      through, the other four bits are transformed.  |value| <= 2^15.
//   5. The maximum of |V| with abs modifiers.
// Every bit of x is transformed once (7 + 5 + 4).  Rounds: the eight
// column blocks of pass 1 one or two at a time (CPR), each carried through
// passes 2 and 3, so one exchange holds an eighth or a quarter of a mask
// (double-buffered).
// ---------------------------------------------------------------------------
typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t fp4_sign_word(int kbase, int a) {
  // e2m1 +1 (0x2) or -1 (0xA) for the 8 nibbles k = kbase + nib against output a
  uint32_t w = 0;
#pragma unroll
  for (int nib = 0; nib < 8; ++nib) w |= ((__builtin_popcount((kbase + nib) & a) & 1) ? 0xAu : 0x2u) << (4 * nib);
  return w;
}

// CPR: pass-1 column blocks per round (2: four rounds of 8 KiB per wave and
// two workgroups per CU; 1: eight rounds of 4 KiB and fewer registers, so
// more workgroups fit).
template <int CPR>
constexpr int mx_slot_words() { return 16 * CPR + 4; }  // a lane's registers + 16 bytes of padding
template <int CPR>
constexpr int mx_min_waves() { return CPR == 2 ? 2 : 3; }

// HIST: also count every coefficient of the masks b != 0 into the LDS bins
// min(|W|/2, kMxHistBins - 1) (the last bin only counts the larger values,
// which the large-value pass then adds one by one); 6 KiB, so two
// workgroups still share a CU.
constexpr int kMxHistBins = 1536;

template <int CPR, bool HIST = false>
__global__ __launch_bounds__(kWG, (mx_min_waves<CPR>())) void k_walsh_mx16(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int NW = 8;
  constexpr int ROUNDS = 8 / CPR;
  constexpr int SLOT = mx_slot_words<CPR>();
  constexpr int BUF = kWG * SLOT;  // one exchange buffer
  static_assert(CPR == 1 || CPR == 2, "column blocks per round");
  __shared__ __attribute__((aligned(16))) uint32_t lds[2 * BUF];
  __shared__ int red[64 * 4];  // per mask of a run of 64: the 4 wave maxima
  __shared__ long long s_item;
  __shared__ uint32_t hl[HIST ? kMxHistBins : 1];
  if constexpr (HIST)
    for (int k = tid_x(); k < kMxHistBins; k += kWG) hl[k] = 0;  // ordered by the loop's first barrier
  long long hcount = 0;  // counts since the last flush of hl (workgroup-uniform)
  auto hist_flush = [&]() {
    for (int k = tid_x(); k < kMxHistBins; k += kWG) {
      const uint32_t c = hl[k];
      if (c) {
        atomicAdd(k == kMxHistBins - 1 ? kp.hist_over : kp.hist + k, (unsigned long long)c);
        hl[k] = 0;
      }
    }
  };

  const int tid = tid_x();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int C = kp.chunk;
  const int col = lane & 15, g = lane >> 4;

  // Pass-1 B operand of block cb, register p: nibble nib is slot
  // k = nib + 8 p + 32 g against output 16 cb + col.  The sign splits into a
  // part of (nib, p, col, cb & 1) and parity(g & (cb >> 1)), which flips
  // every nibble's sign bit.
  uint32_t B1b[2][4];
#pragma unroll
  for (int c0 = 0; c0 < 2; ++c0)
#pragma unroll
    for (int p = 0; p < 4; ++p) B1b[c0][p] = fp4_sign_word(8 * p, 16 * c0 + col);
  uint32_t gflip[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) gflip[c] = (__builtin_popcount(g & c) & 1) ? 0x88888888u : 0u;
  // Pass-2 B operands: the two 16-column halves of H_32, slot kappa = j + 8 g.
  f16x8 hb0, hb1;
  // Pass-3 B operands: slot j = h + 2 p3 (h passed through) + 8 g; MFMA hf keeps h = hf.
  f16x8 hc0, hc1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kappa = j + 8 * g;
    hb0[j] = hsign(kappa & col);
    hb1[j] = hsign(kappa & (col + 16));
    const int k4 = (j >> 1) | (g << 2);  // the four transformed bits (x8, x9, x14, x15)
    hc0[j] = (j & 1) ? (_Float16)0.0f : hsign(k4 & col);
    hc1[j] = (j & 1) ? hsign(k4 & col) : (_Float16)0.0f;
  }
  const float fix = col == 0 ? -64.0f : 0.0f;
  const f32x4 cfix = {fix, fix, fix, fix};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // exchange slots: written as (lane >> 4, wave, lane & 15), read with the
  // wave and the lane's upper bits swapped
  const int wslot = ((g * 4 + wave) * 16 + col) * SLOT;
  const int rslot = ((wave * 4 + g) * 16 + col) * SLOT;

  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;
    JobDesc jd;
    long long li;
    if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {  // batched: find the job owning this item
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = li * (long long)C;
    const long long kend = 1LL << jd.m;
    const long long wb = (long long)tid * NW;
    const int n = jd.n;
    int runmin = 0x7fffffff;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      const bool inrange = k < kend;
      const bool count = HIST && inrange && k != 0;  // the histogram covers b != 0 (wave-uniform)
      if (step == 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] = 0;
        if (inrange) {  // one load at a time: a work item here walks hundreds of masks, and
          // the batched start (gray_start) measured 0.8 % slower for this kernel
          const long long gk = gray(k);
          for (int i = 0; i < jd.m; ++i)
            if ((gk >> i) & 1) load_words<NW>(G, jd.F + (long long)i * jd.nwords + wb, true);
        }
      } else if (inrange) {
        if constexpr (CPR == 2) {
#pragma unroll
          for (int w = 0; w < NW; ++w) G[w] ^= Fn[w];
        } else {  // no prefetch register set: the slice is read when it is needed
          load_words<NW>(G, jd.F + (long long)__builtin_ctzll((unsigned long long)k) * jd.nwords + wb, true);
        }
      }
      if (CPR == 2 && step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      // pass-1 operands: A[t][x7] register p = bit t of every nibble of word 4 x7 + p
      i32x8 A[4][2];
#pragma unroll
      for (int x7 = 0; x7 < 2; ++x7)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const uint32_t w = G[4 * x7 + p];
          A[0][x7][p] = (int)(w & 0x11111111u);
          A[1][x7][p] = (int)(w & 0x22222222u);
          A[2][x7][p] = (int)(w & 0x44444444u);
          A[3][x7][p] = (int)((w >> 1) & 0x44444444u);
          A[0][x7][p + 4] = 0;
          A[1][x7][p + 4] = 0;
          A[2][x7][p + 4] = 0;
          A[3][x7][p + 4] = 0;
        }
      float m0 = 0.0f, m1 = 0.0f;
      // eight rounds stay a loop: unrolled, the rounds' live ranges overlap
#pragma unroll (CPR == 2 ? ROUNDS : 1)
      for (int r = 0; r < ROUNDS; ++r) {
        uint32_t* buf = lds + (r & 1) * BUF;
        // ---- pass 1 for the round's column blocks, cast, pass 2
        uint32_t X[CPR][2][2][4];  // [block][hf2][s][x8 x9]: pass-2 results as fp16 pairs (pass-3 operands)
#pragma unroll
        for (int cl = 0; cl < CPR; ++cl) {
          const int cb = CPR * r + cl;
          const uint32_t fl = gflip[cb >> 1];
          const i32x8 b = {(int)(B1b[cb & 1][0] ^ fl), (int)(B1b[cb & 1][1] ^ fl), (int)(B1b[cb & 1][2] ^ fl),
                           (int)(B1b[cb & 1][3] ^ fl), 0, 0, 0, 0};
          f32x4 D[4][2];
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int x7 = 0; x7 < 2; ++x7)
              D[t][x7] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                  A[t][x7], b, cb == 0 ? cfix : zero, 4, 4, 0, t == 0 ? 128 : (t == 1 ? 127 : 126), 0, 127);
#pragma unroll
          for (int i = 0; i < 4; ++i) {  // tile row pair (x8, x9)
            const f16x8 av = as_f16x8(pk_cvt_f16(D[0][0][i], D[0][1][i]), pk_cvt_f16(D[1][0][i], D[1][1][i]),
                                      pk_cvt_f16(D[2][0][i], D[2][1][i]), pk_cvt_f16(D[3][0][i], D[3][1][i]));
            const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, zero, 0, 0, 0);
            const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
            X[cl][0][0][i] = pk_cvt_f16(e0[0], e0[1]);
            X[cl][0][1][i] = pk_cvt_f16(e0[2], e0[3]);
            X[cl][1][0][i] = pk_cvt_f16(e1[0], e1[1]);
            X[cl][1][1][i] = pk_cvt_f16(e1[2], e1[3]);
          }
        }
        // ---- exchange (double-buffered: one barrier per round)
#pragma unroll
        for (int q = 0; q < 4 * CPR; ++q) {
          const int cl = q >> 2, hf = (q >> 1) & 1, s = q & 1;
          *reinterpret_cast<uint4*>(buf + wslot + 4 * q) =
              uint4{X[cl][hf][s][0], X[cl][hf][s][1], X[cl][hf][s][2], X[cl][hf][s][3]};
        }
        __syncthreads();
        uint32_t Y[4 * CPR][4];
#pragma unroll
        for (int q = 0; q < 4 * CPR; ++q) {
          const uint4 v = *reinterpret_cast<const uint4*>(buf + rslot + 4 * q);
          Y[q][0] = v.x; Y[q][1] = v.y; Y[q][2] = v.z; Y[q][3] = v.w;
        }
        // ---- pass 3 and the maximum
#pragma unroll
        for (int q = 0; q < 4 * CPR; ++q) {
          const f16x8 av = as_f16x8(Y[q][0], Y[q][1], Y[q][2], Y[q][3]);
          const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hc0, zero, 0, 0, 0);
          const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hc1, zero, 0, 0, 0);
          m0 = fmaxf(fmaxf(m0, fabsf(d0[0])), fabsf(d1[0]));
          m1 = fmaxf(fmaxf(m1, fabsf(d0[1])), fabsf(d1[1]));
          m0 = fmaxf(fmaxf(m0, fabsf(d0[2])), fabsf(d1[2]));
          m1 = fmaxf(fmaxf(m1, fabsf(d0[3])), fabsf(d1[3]));
          if constexpr (HIST) {
            if (count) {  // |V| = |W|/2 <= 2^15, an exact integer
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                atomicAdd(&hl[min((int)fabsf(d0[i]), kMxHistBins - 1)], 1u);
                atomicAdd(&hl[min((int)fabsf(d1[i]), kMxHistBins - 1)], 1u);
              }
            }
          }
        }
      }
      const int mx = wave_max((int)fmaxf(m0, m1));
      if (lane == 0) red[(step & 63) * 4 + wave] = mx;
      if ((step & 63) == 63 || step == C - 1) {
        __syncthreads();
        if (wave == 0) {
          const long long s0 = step & ~63LL;
          const long long kk = kfirst + s0 + lane;
          int v = 0x7fffffff;
          if (s0 + lane <= step && kk < kend && kk != 0) {
            const int* pr = red + lane * 4;
            const int pm = max(max(pr[0], pr[1]), max(pr[2], pr[3]));
            if (jd.maxabs) jd.maxabs[(uint32_t)gray(kk)] = 2 * pm;
            v = (1 << (n - 1)) - pm;
          }
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
          runmin = min(runmin, v);
        }
      }
    }
    // a workgroup works on one mask at a time: already one add an item
    if (tid == 0 && runmin != 0x7fffffff) atomicMin(jd.nl, runmin);
    if constexpr (HIST) {
      // keep every LDS count below 2^32
      hcount += (long long)C << 16;
      if (hcount > (1LL << 31)) {
        __syncthreads();
        hist_flush();
        hcount = 0;
      }
    }
  }
  if constexpr (HIST) {
    __syncthreads();
    hist_flush();
  }
}

// ---------------------------------------------------------------------------
// n = 12, max mode, matrix-core variant: one wave per mask, four masks per
// workgroup, no workgroup barrier inside a mask.
//
// Lane l holds words 2l, 2l + 1 of the mask (x5 = which word, x6..x11 = l).
//   1. Popcount stages as fp16 bit patterns (1536 + c', as in the n = 16
//      kernel), the x5 pair packed into one register.
//   2. A wave-private LDS transpose: lane (x8, x9, a'3, a'4, x10, x11)
//      receives register (x6, x7, a'0, a'1, a'2).  Rows of 68 words (one
//      per receiving register) keep both sides free of bank conflicts: a
//      write lands on bank 4 x6x7 + (receiving lane) mod 64, and the four
//      registers of an MFMA operand are read as pairs straight into place.
//   3. Pass 1, for each (a'0, a'1, a'2): the registers over (x6, x7) with
//      their x5 halves are the A operand of v_mfma_f32_16x16x32_f16 with rows
//      (x8, x9, a'3, a'4) = lane bits 0..3 and K slots (x5, x6, x7, x10, x11),
//      against the two halves of H_32; the accumulator input removes the
//      offset from column 0.  |value| <= 512, cast to fp16 exactly.
//   4. Pass 2: the four results of a lane are rows 4 (lane / 16) + i, i.e. K
//      slots (x8, x9, a'3, a'4) of v_mfma_f32_16x16x16_f16 against
//      H_4 (x8, x9) (x) I_4 (a'3, a'4), which transforms x8, x9 and passes the
//      rest through.  |value| <= 2048, exact.
// Every bit of x is transformed once (5 + 5 + 2).
// ---------------------------------------------------------------------------
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kWG, 4) void k_walsh_mfma12(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int NW = 2;
  constexpr int GPW = kWG / 64;               // masks (waves) per workgroup
  __shared__ uint32_t lds[GPW * 32 * 68];     // 8.5 KiB per wave: 32 rows of 68 words
  __shared__ long long s_item;

  const int tid = tid_x();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int C = kp.chunk;
  uint32_t* wl = lds + wave * (32 * 68);

  f16x8 hb0, hb1;
  f16x4 hc;
  {
    const int g = lane >> 4, n = lane & 15;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kappa = j + 8 * g;
      hb0[j] = hsign(kappa & n);
      hb1[j] = hsign(kappa & (n + 16));
    }
    // H_4 on K bits 0..1 and output bits 0..1, identity on bits 2..3
#pragma unroll
    for (int j = 0; j < 4; ++j) hc[j] = (g == (n >> 2)) ? hsign(j & n & 3) : (_Float16)0.0f;
  }
  const float fix = (lane & 15) == 0 ? -49152.0f : 0.0f;
  const f32x4 cfix = {fix, fix, fix, fix};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  // exchange addresses: source a' -> (register, lane) of the receiver
  const int xs = lane & 3;                                  // x6, x7
  const int dl0 = ((lane >> 2) & 3) | (((lane >> 4) & 3) << 4);  // x8, x9, x10, x11

  // NL candidate of this lane: per item in a batch, over all its items for one box
  int runmin = 0x7fffffff;
  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;
    JobDesc jd;
    long long li;
    if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = (li * GPW + wave) * (long long)C;
    const long long kend = 1LL << jd.m;
    const long long wb = (long long)lane * NW;
    const int n = jd.n;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      if (k >= kend) break;  // wave-uniform
      if (step == 0) {
        gray_start<NW>(G, jd.F, jd.nwords, wb, gray(k), jd.m);
      } else {
        G[0] ^= Fn[0];
        G[1] ^= Fn[1];
      }
      if (step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      // ---- 1-2. popcounts into the wave's LDS tile
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int a = 0; a < 32; ++a) {
        const uint32_t c0 = __builtin_popcount(G[0] ^ walsh_mask(a)) + (0x6600 - 16);
        const uint32_t c1 = __builtin_popcount(G[1] ^ walsh_mask(a)) + (0x6600 - 16);
        const int dreg = xs + 4 * (a & 7);
        const int dlane = dl0 | ((a >> 3) << 2);
        wl[dreg * 68 + dlane] = __builtin_amdgcn_perm(c1, c0, 0x05040100u);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      uint32_t R[32];
#pragma unroll
      for (int d = 0; d < 32; ++d) R[d] = wl[d * 68 + lane];
      // ---- 3-4. the two passes and the maximum: all first-pass products
      // first, so the casts of one wait on products issued long before
      float m0 = 0.0f, m1 = 0.0f;
      f32x4 d0[8], d1[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const f16x8 av = as_f16x8(R[4 * t], R[4 * t + 1], R[4 * t + 2], R[4 * t + 3]);
        d0[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, cfix, 0, 0, 0);
        d1[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        f16x4 a0, a1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a0[i] = (_Float16)d0[t][i];
          a1[i] = (_Float16)d1[t][i];
        }
        const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x16f16(a0, hc, zero, 0, 0, 0);
        const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, hc, zero, 0, 0, 0);
        m0 = fmaxf(fmaxf(m0, fabsf(e0[0])), fabsf(e1[0]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[1])), fabsf(e1[1]));
        m0 = fmaxf(fmaxf(m0, fabsf(e0[2])), fabsf(e1[2]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[3])), fabsf(e1[3]));
      }
      const int mx = wave_max((int)fmaxf(m0, m1));
      if (lane == 0 && k != 0) {
        if (jd.maxabs) jd.maxabs[(uint32_t)gray(k)] = 2 * mx;
        runmin = min(runmin, (1 << (n - 1)) - mx);
      }
    }
    if (kp.jobs != nullptr) {
      nl_add_wave(jd.nl, runmin);
      runmin = 0x7fffffff;
    }
  }
  if (kp.jobs == nullptr) nl_add_workgroup(kp.job0.nl, runmin);
}

// ---------------------------------------------------------------------------
// n = 12, max mode, two matrix-core passes (fp4, then fp16): one wave per
// mask, four masks per workgroup, no LDS and no barrier inside a mask.
//
// The table is bit-sliced into sparse words (bitslice_words_fp4): word w
// holds x = 16 w + j at bit 4 (j >> 1) + 1 + (j & 1), so x0 picks bit 1 or
// 2 of a nibble and x1..x3 the nibble; lane l holds words 4 l .. 4 l + 3
// (x4, x5 the register, x6..x11 the lane).  As in k_walsh_mx16 the bits
// themselves are transformed and V = T - 2^11 [a = 0] = -W / 2 is tracked.
//   1. Pass 1, v_mfma_scale_f32_16x16x128_f8f6f4 on e2m1: for x0 = 0, 1 the
//      operand is the four words ANDed with 0x22222222 or 0x44444444 (e2m1
//      1.0 or 2.0, operand scale 2^0 or 2^-1).  K slots (x1, x2, x3 | x4, x5 |
//      x10, x11), rows x6..x9, eight 16-column blocks of H_128; -64 at
//      column 0 of block 0 removes 2^11 over the 2^5 tiles reaching output 0.
//      |value| <= 64.
//   2. Pass 2, v_mfma_f32_16x16x32_f16: per column block the two results over
//      x0 become the operand's halves, the tile rows x6, x7 its registers and
//      the lane's tile rows x8, x9 its K slots.  |value| <= 2048.
//   3. The maximum of |V| with abs modifiers.
// Every bit of x is transformed once (7 + 5).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG, 3) void k_walsh_mx12(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int NW = 4;
  constexpr int GPW = kWG / 64;  // masks (waves) per workgroup
  __shared__ long long s_item;

  const int tid = tid_x();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int C = kp.chunk;
  const int col = lane & 15, g = lane >> 4;

  uint32_t B1b[2][4];
#pragma unroll
  for (int c0 = 0; c0 < 2; ++c0)
#pragma unroll
    for (int p = 0; p < 4; ++p) B1b[c0][p] = fp4_sign_word(8 * p, 16 * c0 + col);
  uint32_t gflip[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) gflip[c] = (__builtin_popcount(g & c) & 1) ? 0x88888888u : 0u;
  f16x8 hb0, hb1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kappa = j + 8 * g;
    hb0[j] = hsign(kappa & col);
    hb1[j] = hsign(kappa & (col + 16));
  }
  const float fix = col == 0 ? -64.0f : 0.0f;
  const f32x4 cfix = {fix, fix, fix, fix};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};

  // NL candidate of this lane: per item in a batch, over all its items for one box
  int runmin = 0x7fffffff;
  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;
    JobDesc jd;
    long long li;
    if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = (li * GPW + wave) * (long long)C;
    const long long kend = 1LL << jd.m;
    const long long wb = (long long)lane * NW;
    const int n = jd.n;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      if (k >= kend) break;  // wave-uniform
      if (step == 0) {
        gray_start<NW>(G, jd.F, jd.nwords, wb, gray(k), jd.m);
      } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] ^= Fn[w];
      }
      if (step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      const i32x8 a0 = {(int)(G[0] & 0x22222222u), (int)(G[1] & 0x22222222u), (int)(G[2] & 0x22222222u),
                        (int)(G[3] & 0x22222222u), 0, 0, 0, 0};
      const i32x8 a1 = {(int)(G[0] & 0x44444444u), (int)(G[1] & 0x44444444u), (int)(G[2] & 0x44444444u),
                        (int)(G[3] & 0x44444444u), 0, 0, 0, 0};
      // all 16 first-pass products first, then the casts and second-pass
      // products: each cast waits on a product issued long before, and the
      // wave keeps the matrix cores busy on its own (three waves a SIMD:
      // faster than five waves interleaving the passes, and than two or
      // four of this form; the host caps the residency at three)
      float m0 = 0.0f, m1 = 0.0f;
      f32x4 d0[8], d1[8];
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const uint32_t fl = gflip[cb >> 1];
        const i32x8 b = {(int)(B1b[cb & 1][0] ^ fl), (int)(B1b[cb & 1][1] ^ fl), (int)(B1b[cb & 1][2] ^ fl),
                         (int)(B1b[cb & 1][3] ^ fl), 0, 0, 0, 0};
        d0[cb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a0, b, cb == 0 ? cfix : zero, 4, 4, 0, 127, 0, 127);
        d1[cb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a1, b, cb == 0 ? cfix : zero, 4, 4, 0, 126, 0, 127);
      }
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const f16x8 av = as_f16x8(pk_cvt_f16(d0[cb][0], d1[cb][0]), pk_cvt_f16(d0[cb][1], d1[cb][1]),
                                  pk_cvt_f16(d0[cb][2], d1[cb][2]), pk_cvt_f16(d0[cb][3], d1[cb][3]));
        const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, zero, 0, 0, 0);
        const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
        m0 = fmaxf(fmaxf(m0, fabsf(e0[0])), fabsf(e1[0]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[1])), fabsf(e1[1]));
        m0 = fmaxf(fmaxf(m0, fabsf(e0[2])), fabsf(e1[2]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[3])), fabsf(e1[3]));
      }
      const int mx = wave_max((int)fmaxf(m0, m1));
      if (lane == 0 && k != 0) {
        if (jd.maxabs) jd.maxabs[(uint32_t)gray(k)] = 2 * mx;
        runmin = min(runmin, (1 << (n - 1)) - mx);
      }
    }
    if (kp.jobs != nullptr) {
      nl_add_wave(jd.nl, runmin);
      runmin = 0x7fffffff;
    }
  }
  if (kp.jobs == nullptr) nl_add_workgroup(kp.job0.nl, runmin);
}

// ---------------------------------------------------------------------------
// n = 12, max mode, the same two passes with the first on int8 operands
// (v_mfma_i32_16x16x64_i8, int32 accumulation), over the same sparse words.
// An operand byte must hold the bit itself (0 or 1), so each of the four
// bits of a byte that hold x values (bits 1, 2, 5, 6: x0, x1) gives its own
// operand, (G >> (1 + x0 + 4 x1)) & 0x01010101, whose K slots are (x2, x3 |
// x4, x5 | x10, x11): the byte, the register and the lane group.  x1 is transformed by accumulating
// its two products, the second against B with the sign of column bit 0
// flipped; x0 stays for pass 2 as in k_walsh_mx12, so the pass-1 outputs
// (same columns, |value| <= 64) and pass 2 are unchanged.  Per mask that is
// 32 int8 products of K = 64 where k_walsh_mx12 issues 16 fp4 products of
// K = 128 at the same 16 cycles each, and four times the operand
// extraction; kept as an alternative engine for the comparison.
// ---------------------------------------------------------------------------
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t i8_sign_word(int kbase, int a) {
  // int8 +1 (0x01) or -1 (0xFF) for the 4 bytes k = kbase + byte against output a
  uint32_t w = 0;
#pragma unroll
  for (int byte = 0; byte < 4; ++byte) w |= ((__builtin_popcount((kbase + byte) & a) & 1) ? 0xFFu : 0x01u) << (8 * byte);
  return w;
}

__global__ __launch_bounds__(kWG, 3) void k_walsh_i8x12(const KParams kp) {
  if (gated_off(kp)) return;
  constexpr int NW = 4;
  constexpr int GPW = kWG / 64;  // masks (waves) per workgroup
  constexpr uint32_t kFlip = 0xFEFEFEFEu;  // +1 <-> -1 in every byte
  __shared__ long long s_item;

  const int tid = tid_x();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int C = kp.chunk;
  const int col = lane & 15, g = lane >> 4;

  // B for x1 = 0: the K slots (byte, register) against pass-1 output bits
  // 1..4 (col >> 1, column-block bit 0); the lane group against column-block
  // bits 1, 2 is a whole-word flip, and x1 = 1 flips by column bit 0.
  uint32_t Bb[2][4];
#pragma unroll
  for (int c0 = 0; c0 < 2; ++c0)
#pragma unroll
    for (int r = 0; r < 4; ++r) Bb[c0][r] = i8_sign_word(4 * r, (16 * c0 + col) >> 1);
  uint32_t gflip[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) gflip[c] = (__builtin_popcount(g & c) & 1) ? kFlip : 0u;
  const uint32_t x1flip = (col & 1) ? kFlip : 0u;
  f16x8 hb0, hb1;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kappa = j + 8 * g;
    hb0[j] = hsign(kappa & col);
    hb1[j] = hsign(kappa & (col + 16));
  }
  const int ifix = col == 0 ? -64 : 0;
  const i32x4 cfix = {ifix, ifix, ifix, ifix};
  const i32x4 izero = {0, 0, 0, 0};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};

  // NL candidate of this lane: per item in a batch, over all its items for one box
  int runmin = 0x7fffffff;
  for (;;) {
    const long long item = next_item(kp, &s_item);
    if (item >= kp.total_items) break;
    JobDesc jd;
    long long li;
    if (kp.jobs == nullptr) {
      jd = kp.job0;
      li = item;
    } else {
      int lo = 0, hi = kp.njobs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
      }
      jd = kp.jobs[lo];
      li = item - jd.item_begin;
    }
    const long long kfirst = (li * GPW + wave) * (long long)C;
    const long long kend = 1LL << jd.m;
    const long long wb = (long long)lane * NW;
    const int n = jd.n;
    uint32_t G[NW], Fn[NW];

    for (int step = 0; step < C; ++step) {
      const long long k = kfirst + step;
      if (k >= kend) break;  // wave-uniform
      if (step == 0) {
        gray_start<NW>(G, jd.F, jd.nwords, wb, gray(k), jd.m);
      } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) G[w] ^= Fn[w];
      }
      if (step + 1 < C && k + 1 < kend) {
        const int i = __builtin_ctzll((unsigned long long)(k + 1));
        load_words<NW>(Fn, jd.F + (long long)i * jd.nwords + wb, false);
      }
      // the x1 flip, opaque per mask: the x1 = 1 operands are rebuilt per
      // mask rather than all 32 of them kept live across the loop
      uint32_t xf = x1flip;
      asm volatile("" : "+v"(xf));
      // A[x0][x1]: the bit at nibble position 1 + x0 of nibble x1 of every byte
      i32x4 A[2][2];
#pragma unroll
      for (int x0 = 0; x0 < 2; ++x0)
#pragma unroll
        for (int x1 = 0; x1 < 2; ++x1)
#pragma unroll
          for (int r = 0; r < NW; ++r) A[x0][x1][r] = (int)((G[r] >> (1 + x0 + 4 * x1)) & 0x01010101u);
      // all first-pass products first, then the casts and second-pass products
      float m0 = 0.0f, m1 = 0.0f;
      i32x4 d0[8], d1[8];
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const uint32_t fl = gflip[cb >> 1];
        i32x4 b0, b1;
#pragma unroll
        for (int r = 0; r < NW; ++r) {
          b0[r] = (int)(Bb[cb & 1][r] ^ fl);
          b1[r] = (int)(Bb[cb & 1][r] ^ fl ^ xf);
        }
        const i32x4 c = cb == 0 ? cfix : izero;
        d0[cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
            A[0][1], b1, __builtin_amdgcn_mfma_i32_16x16x64_i8(A[0][0], b0, c, 0, 0, 0), 0, 0, 0);
        d1[cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
            A[1][1], b1, __builtin_amdgcn_mfma_i32_16x16x64_i8(A[1][0], b0, c, 0, 0, 0), 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const f16x8 av = as_f16x8(pk_cvt_f16((float)d0[cb][0], (float)d1[cb][0]),
                                  pk_cvt_f16((float)d0[cb][1], (float)d1[cb][1]),
                                  pk_cvt_f16((float)d0[cb][2], (float)d1[cb][2]),
                                  pk_cvt_f16((float)d0[cb][3], (float)d1[cb][3]));
        const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb0, zero, 0, 0, 0);
        const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, hb1, zero, 0, 0, 0);
        m0 = fmaxf(fmaxf(m0, fabsf(e0[0])), fabsf(e1[0]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[1])), fabsf(e1[1]));
        m0 = fmaxf(fmaxf(m0, fabsf(e0[2])), fabsf(e1[2]));
        m1 = fmaxf(fmaxf(m1, fabsf(e0[3])), fabsf(e1[3]));
      }
      const int mx = wave_max((int)fmaxf(m0, m1));
      if (lane == 0 && k != 0) {
        if (jd.maxabs) jd.maxabs[(uint32_t)gray(k)] = 2 * mx;
        runmin = min(runmin, (1 << (n - 1)) - mx);
      }
    }
    if (kp.jobs != nullptr) {
      nl_add_wave(jd.nl, runmin);
      runmin = 0x7fffffff;
    }
  }
  if (kp.jobs == nullptr) nl_add_workgroup(kp.job0.nl, runmin);
}

// ---------------------------------------------------------------------------
// n = 16 + L, 1 <= L <= 4, max mode: recompute instead of materialising.
//
// Write x = (x_hi : L bits, x_lo : 16 bits).  For a fixed high output index
// a_hi the coefficients W(a_hi, a_lo) form one 2^16-point transform over
// x_lo whose inputs already sum over x_hi.  The table is bit-sliced so that
// a word holds the 2^L high inputs and 2^B (B = 5 - L) low inputs of one
// group of x_lo; the popcount stages then cover x_hi and the B low bits at
// once, and for a fixed a_hi each word yields 2^B outputs.  A task
// (mask b, a_hi) is thus a 2^16-point job of the same shape as the n = 16
// kernel: 3 + L register stages, the two-round LDS exchange, and 8 stages
// with the lane swap.  Values reach 2^(7+L) before the exchange (int16) and
// up to 2^(15+L) at the end, so the last L + 1 stages run in int32, a chunk
// of registers at a time.  A workgroup walks its masks in Gray-code order,
// keeping the mask's words G_b in a private global buffer (L2-resident,
// 2^(n-3) bytes) that each task streams back in.
// ---------------------------------------------------------------------------
struct BigParams {
  const uint32_t* FT;   // [m][2^(n-5)] words in the x_hi-inner layout
  uint32_t* gbuf;       // [grid][2^(n-5)] per-workgroup words of the current mask
  int32_t* maxabs;
  int32_t* nl;
  int* queue;
  long long total_items;
  int m;
  int chunk;
};

template <int L>
__global__ __launch_bounds__(kWG, 2) void k_walsh_big(const BigParams bp) {
  constexpr int N = 16 + L;
  constexpr int B = 5 - L;                 // low bits of x_lo inside a word
  constexpr int KB = 8 - B;                // word-group bits per thread
  constexpr int NWT = 1 << KB;             // words per thread
  constexpr int NR = 128;                  // packed registers
  constexpr int OPW = 1 << B;              // outputs per word for one a_hi
  constexpr int K16 = 7 - L;               // phase-2 stages still in int16
  constexpr int NK = 1 << (7 - K16);       // packed registers per int32 chunk
  static_assert(L >= 1 && L <= 4, "n = 17..20");
  constexpr long long NWORDS = 1LL << (N - 5);

  __shared__ uint32_t lds[64 * kLdsStride];
  __shared__ int red[kWG / 64];
  __shared__ long long s_item;

  const int tid = tid_x();
  const int lane = tid & 63;
  uint32_t* gb = bp.gbuf + (long long)bid_x() * NWORDS;
  const long long wbase = (long long)tid * NWT;  // this thread's words
  const long long kend = 1LL << bp.m;

  for (;;) {
    if (tid == 0) s_item = (long long)atomicAdd(bp.queue, 1);
    __syncthreads();
    const long long item = s_item;
    __syncthreads();
    if (item >= bp.total_items) break;
    const long long kfirst = item * bp.chunk;
    int runmin = 0x7fffffff;

    for (int step = 0; step < bp.chunk; ++step) {
      const long long k = kfirst + step;
      const bool inrange = k < kend;
      // ---- words of mask gray(k) into the private buffer (own words only)
      if (inrange) {
        if (step == 0) {
          const long long gk = gray(k);
#pragma unroll 1
          for (int c = 0; c < NWT; c += 4) {
            uint4 acc = make_uint4(0, 0, 0, 0);
            for (int i = 0; i < bp.m; ++i)
              if ((gk >> i) & 1) {
                const uint4 v = *reinterpret_cast<const uint4*>(bp.FT + (long long)i * NWORDS + wbase + c);
                acc.x ^= v.x; acc.y ^= v.y; acc.z ^= v.z; acc.w ^= v.w;
              }
            *reinterpret_cast<uint4*>(gb + wbase + c) = acc;
          }
        } else {
          const int i = __builtin_ctzll((unsigned long long)k);
#pragma unroll 4
          for (int c = 0; c < NWT; c += 4) {
            uint4 acc = *reinterpret_cast<const uint4*>(gb + wbase + c);
            const uint4 v = *reinterpret_cast<const uint4*>(bp.FT + (long long)i * NWORDS + wbase + c);
            acc.x ^= v.x; acc.y ^= v.y; acc.z ^= v.z; acc.w ^= v.w;
            *reinterpret_cast<uint4*>(gb + wbase + c) = acc;
          }
        }
      }
      const bool valid = inrange && k != 0;
      int maskmax = 0;

      for (int ahi = 0; ahi < (1 << L); ++ahi) {
        // ---- phase 1: popcount stages over (x_hi, B low bits), then KB - 1 register stages
        uint32_t R[NR];
        const uint32_t lhi = walsh_mask(ahi << B);
#pragma unroll
        for (int c = 0; c < NWT; c += 4) {
          const uint4 v = inrange ? *reinterpret_cast<const uint4*>(gb + wbase + c) : make_uint4(0, 0, 0, 0);
          const uint32_t g4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t G = g4[q] ^ lhi;
#pragma unroll
            for (int a = 0; a < OPW / 2; ++a) {
              const int c0 = __builtin_popcount(G ^ walsh_mask(a)) - 16;
              const int c1 = __builtin_popcount(G ^ walsh_mask(a | (OPW / 2))) - 16;
              R[((c + q) * (OPW / 2)) + a] = __builtin_amdgcn_perm((uint32_t)c1, (uint32_t)c0, 0x05040100u);
            }
          }
        }
#pragma unroll
        for (int d = B - 1; d < 7; ++d) stage_regs<NR>(R, 1 << d);

        // ---- two-round LDS exchange (as in the n = 16 kernel)
        const int u = (tid & 31) | ((tid >> 6) << 5);
        const int h = (tid >> 5) & 1;
        const int wb6 = (tid >> 6) & 1;
        const int ru = u >> 6;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          if ((r ^ wb6) == 0) {
#pragma unroll
            for (int j = 0; j < 64; ++j) lds[j * kLdsStride + tid] = R[j];
          } else {
#pragma unroll
            for (int j = 0; j < 64; ++j) lds[j * kLdsStride + tid] = R[64 + j];
          }
          __syncthreads();
          const int src = (u & 63) * kLdsStride + h * 128 + ((r ^ ru) << 6);
          if ((r ^ wb6) == 0) {
#pragma unroll
            for (int i = 0; i < 64; ++i) R[i] = lds[src + i];
          } else {
#pragma unroll
            for (int i = 0; i < 64; ++i) R[64 + i] = lds[src + i];
          }
          if (r == 0) __syncthreads();
        }
        // ---- phase 2: K16 packed stages, then int32 chunks: stages, lane swap, last stage
#pragma unroll
        for (int d = 0; d < K16; ++d) stage_regs<NR>(R, 1 << d);
        int hiv = -0x7fffffff, lov = 0x7fffffff;
#pragma unroll
        for (int c = 0; c < (1 << K16); ++c) {
          int lo[NK], hi[NK];
#pragma unroll
          for (int kk = 0; kk < NK; ++kk) {
            const uint32_t v = R[c + (kk << K16)];
            lo[kk] = unpack_lo(v);
            hi[kk] = unpack_hi(v);
          }
#pragma unroll
          for (int hb = 1; hb < NK; hb <<= 1)
#pragma unroll
            for (int kk = 0; kk < NK; ++kk) {
              if (kk & hb) continue;
              const int a0 = lo[kk], a1 = lo[kk | hb];
              lo[kk] = a0 + a1; lo[kk | hb] = a0 - a1;
              const int b0 = hi[kk], b1 = hi[kk | hb];
              hi[kk] = b0 + b1; hi[kk | hb] = b0 - b1;
            }
#pragma unroll
          for (int kk = 0; kk < NK / 2; ++kk) {
            uint32_t x0 = (uint32_t)lo[kk], x1 = (uint32_t)lo[kk + NK / 2];
            swap_halves(x0, x1);
            uint32_t y0 = (uint32_t)hi[kk], y1 = (uint32_t)hi[kk + NK / 2];
            swap_halves(y0, y1);
            const int s0 = (int)x0 + (int)x1, d0 = (int)x0 - (int)x1;
            const int s1 = (int)y0 + (int)y1, d1 = (int)y0 - (int)y1;
            hiv = max(hiv, max(max(s0, d0), max(s1, d1)));
            lov = min(lov, min(min(s0, d0), min(s1, d1)));
          }
        }
        int mx = wave_max(max(hiv, -lov));
        if (lane == 0) red[tid >> 6] = mx;
        __syncthreads();
        mx = max(max(red[0], red[1]), max(red[2], red[3]));
        maskmax = max(maskmax, mx);
        __syncthreads();  // red and lds are rewritten by the next task
      }
      if (tid == 0 && valid) {
        if (bp.maxabs) bp.maxabs[gray(k)] = 2 * maskmax;
        runmin = min(runmin, (1 << (N - 1)) - maskmax);
      }
    }
    if (tid == 0 && runmin != 0x7fffffff) atomicMin(bp.nl, runmin);
  }
}

// ---------------------------------------------------------------------------
// Bit-slicing: F[i][w] = bit i of S[32w + j] at bit j (j < min(32, 2^n)).
// ---------------------------------------------------------------------------
template <int EB>
__device__ __forceinline__ uint32_t load_entry(const void* S, long long x) {
  if constexpr (EB == 1) return reinterpret_cast<const uint8_t*>(S)[x];
  if constexpr (EB == 2) return reinterpret_cast<const uint16_t*>(S)[x];
  return reinterpret_cast<const uint32_t*>(S)[x];
}

template <int EB>
__device__ void bitslice_words(const void* S, int n, int m, uint32_t* F, int nwords, int w) {
  const int bits = (n >= 5) ? 32 : (1 << n);
  uint32_t v[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) v[j] = (j < bits) ? load_entry<EB>(S, (long long)w * 32 + j) : 0u;
  for (int i = 0; i < m; ++i) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) word |= ((v[j] >> i) & 1u) << j;
    F[(long long)i * nwords + w] = word;
  }
}

// Sparse words of the n = 12 fp4 engine: word w holds x = 16 w + j at bit
// 4 (j >> 1) + 1 + (j & 1) (bits 1 and 2 of each nibble, whose e2m1 values
// are 1.0 and 2.0), 16 inputs a word.
template <int EB>
__device__ void bitslice_words_fp4(const void* S, int m, uint32_t* F, int nwords, int w) {
  uint32_t v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = load_entry<EB>(S, (long long)w * 16 + j);
  for (int i = 0; i < m; ++i) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) word |= ((v[j] >> i) & 1u) << (4 * (j >> 1) + 1 + (j & 1));
    F[(long long)i * nwords + w] = word;
  }
}

// Bit-slicing by a whole wave (dense words, tables of at least 64 entries):
// lane l reads entry x0 + l (x0 a multiple of 64; one coalesced load), one
// ballot per output bit gives that bit of all 64 entries, i.e. two words,
// which are selected into lanes 2 ii, 2 ii + 1 of one register and stored
// together.  The same words as bitslice_words, from a single table much
// faster (16 x 16: 8.6 -> 4.4 us); a batch of many small tables stays on
// the word-per-thread form, where the per-bit selects would cost more than
// the loads they save.
template <int EB>
__device__ void bitslice_wave(const void* S, int m, uint32_t* F, int nwords, long long x0) {
  const int lane = tid_x() & 63;
  const uint32_t v = load_entry<EB>(S, x0 + lane);
  const long long w0 = x0 >> 5;
  for (int i0 = 0; i0 < m; i0 += 32) {
    const int nb = min(m - i0, 32);
    uint32_t word = 0;
    for (int ii = 0; ii < nb; ++ii) {
      const unsigned long long mask = __ballot((v >> (i0 + ii)) & 1u);
      word = lane == 2 * ii ? (uint32_t)mask : word;
      word = lane == 2 * ii + 1 ? (uint32_t)(mask >> 32) : word;
    }
    if (lane < 2 * nb) F[(long long)(i0 + (lane >> 1)) * nwords + w0 + (lane & 1)] = word;
  }
}

// The words of one job in its layout.
template <int EB>
__device__ __forceinline__ void bitslice_job(const JobDesc& jd, int w) {
  uint32_t* F = const_cast<uint32_t*>(jd.F);
  if (jd.flags & kWordsFp4) bitslice_words_fp4<EB>(jd.S, jd.m, F, jd.nwords, w);
  else bitslice_words<EB>(jd.S, jd.n, jd.m, F, jd.nwords, w);
}

// Bit-slicing for k_walsh_big: word w = x_lo >> B holds, at bit
// j = x_lo_low + 2^B * x_hi, bit i of S[x_hi * 2^16 + x_lo].
template <int EB>
__global__ __launch_bounds__(256) void k_bitslice_big(const void* S, int L, int m, uint32_t* FT, int nwords) {
  const int w = bid_x() * bdim_x() + tid_x();
  if (w >= nwords) return;
  const int B = 5 - L;
  uint32_t v[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const long long xlo = ((long long)w << B) | (j & ((1 << B) - 1));
    const long long xhi = j >> B;
    v[j] = load_entry<EB>(S, (xhi << 16) | xlo);
  }
  for (int i = 0; i < m; ++i) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) word |= ((v[j] >> i) & 1u) << j;
    FT[(long long)i * nwords + w] = word;
  }
}

// ---------------------------------------------------------------------------
// Per-call initialisation: queue counters, NL start value 2^(n-1),
// maxabs[0] = 2^n, and the b = 0 row / column of a requested spectrum.
// ---------------------------------------------------------------------------
// Entry a of the spectrum's b = 0 row (b-major) or column (a-major).
__device__ __forceinline__ void init_spec_entry(const JobDesc& jd, long long a, int layout) {
  const int v = (a == 0) ? (int)((1LL << jd.n) >> 1) * -jd.wscale : 0;  // 2^n (W) or 2^(n-1) (LAT)
  if (layout == 1) jd.spec[a] = v;
  else jd.spec[a << jd.m] = v;
}

// One workgroup's share: the job's start values (and, if `first`, the queue
// counters); with `spec_row` false the caller writes the b = 0 row / column.
__device__ __forceinline__ void init_job(const JobDesc& jd, bool first, int* queue, int nqueue, int layout,
                                         bool spec_row) {
  if (first) {
    for (int i = tid_x(); i < nqueue; i += bdim_x()) queue[i] = 0;
  }
  if (tid_x() == 0) {
    *jd.nl = 1 << (jd.n - 1);
    if (jd.maxabs) jd.maxabs[0] = 1 << jd.n;
  }
  if (jd.spec && spec_row)
    for (long long a = tid_x(); a < (1LL << jd.n); a += bdim_x()) init_spec_entry(jd, a, layout);
}

// Batched: bid_y() selects the job, threads stride over its words; the
// first workgroup of a job also sets its start values (NL, maxabs[0], the
// b = 0 row or column of a spectrum) and, for the launch's first job, zeroes
// `nqueue` queue counters, so a batch starts with this one launch.
__global__ __launch_bounds__(64) void k_prep_jobs(const JobDesc* jobs, int* queue, int nqueue) {
  const JobDesc jd = jobs[bid_y()];
  if (bid_x() == 0) init_job(jd, bid_y() == 0, queue, nqueue, (jd.flags & kSpecAMajor) ? 2 : 1);
  for (int w = bid_x() * bdim_x() + tid_x(); w < jd.nwords; w += gdim_x() * bdim_x()) {
    if (jd.s_elem_bytes == 1) bitslice_job<1>(jd, w);
    else if (jd.s_elem_bytes == 2) bitslice_job<2>(jd, w);
    else bitslice_job<4>(jd, w);
  }
}


// ---------------------------------------------------------------------------
// Component criteria (n <= 14): balancedness, correlation immunity and the
// autocorrelation spectrum of every nonzero component.  One workgroup
// transforms one mask at a time in LDS (int32, 2^n words):
//   W = H f, then v(a) = (W(a)/2)^2 (int32, wrapping) and V = H v, where
//   V(d) = 2^(n-2) r(d) exactly (Wiener-Khinchin), |V| <= 2^(2n-2) < 2^31,
//   so the wrapping intermediate sums still give the exact V.
// Per-mask results go to the optional arrays; aggregates use atomics into
// crit[]: {NL, #unbalanced, min CI weight, -, abs indicator, min PC weight}.
// ---------------------------------------------------------------------------
struct CritParams {
  const void* S;
  int eb, n, m;
  int32_t* crit;     // 8 ints
  int32_t* w0;       // W(0, b)
  int32_t* minwt;    // min wt(a), a != 0, W(a, b) != 0 (n + 1 if none)
  int32_t* acmax;    // max_{d != 0} |r_b(d)|
  int32_t* pcwt;     // min wt(d), d != 0, r_b(d) != 0 (n + 1 if none)
};

__device__ __forceinline__ void lds_fwht(int32_t* buf, int n) {
  const int half = 1 << (n - 1);
  for (int h = 1; h <= half; h <<= 1) {
    for (int p = tid_x(); p < half; p += bdim_x()) {
      const int i = ((p & ~(h - 1)) << 1) | (p & (h - 1));
      const int32_t u = buf[i], v = buf[i + h];
      buf[i] = (int32_t)((uint32_t)u + (uint32_t)v);
      buf[i + h] = (int32_t)((uint32_t)u - (uint32_t)v);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int block_sum(int v, int* red) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  if ((tid_x() & 63) == 0) red[tid_x() >> 6] = v;
  __syncthreads();
  int r = red[0];
  for (int i = 1; i < (int)(bdim_x() >> 6); ++i) r += red[i];
  __syncthreads();
  return r;
}

template <bool IS_MAX>
__device__ __forceinline__ int block_reduce(int v, int* red) {
  v = group_reduce<64, IS_MAX>(v);
  if ((tid_x() & 63) == 0) red[tid_x() >> 6] = v;
  __syncthreads();
  int r = red[0];
  for (int i = 1; i < (int)(bdim_x() >> 6); ++i) r = IS_MAX ? max(r, red[i]) : min(r, red[i]);
  __syncthreads();
  return r;
}

template <int EB>
__global__ __launch_bounds__(256) void k_criteria(const CritParams p) {
  __shared__ int32_t buf[1 << 14];
  __shared__ int red[4];
  const int n = p.n;
  const int N = 1 << n;
  const long long M = 1LL << p.m;
  // this workgroup's share of the aggregates (thread 0), added once at the end
  int g_nl = N >> 1, g_unb = 0, g_mw = n + 1, g_ac = 0, g_pw = n + 1;
  for (long long b = bid_x() + 1; b < M; b += gdim_x()) {
    for (int x = tid_x(); x < N; x += bdim_x())
      buf[x] = (__builtin_popcount((uint32_t)b & load_entry<EB>(p.S, x)) & 1) ? -1 : 1;
    __syncthreads();
    lds_fwht(buf, n);
    int mx = 0, mw = n + 1, w0 = 0;
    for (int a = tid_x(); a < N; a += bdim_x()) {
      const int v = buf[a];
      mx = max(mx, v < 0 ? -v : v);
      if (a == 0) w0 = v;
      else if (v != 0) mw = min(mw, __builtin_popcount(a));
      const int hv = v / 2;  // every W is even for n >= 1
      buf[a] = (int32_t)((uint32_t)hv * (uint32_t)hv);
    }
    __syncthreads();
    mx = block_reduce<true>(mx, red);
    mw = block_reduce<false>(mw, red);
    lds_fwht(buf, n);
    int ac = 0, pw = n + 1;
    for (int d = tid_x(); d < N; d += bdim_x()) {
      if (d == 0) continue;
      const int r = (int)((uint32_t)buf[d] << 2) >> n;  // 4 V(d) / 2^n, exact
      ac = max(ac, r < 0 ? -r : r);
      if (r != 0) pw = min(pw, __builtin_popcount(d));
    }
    ac = block_reduce<true>(ac, red);
    pw = block_reduce<false>(pw, red);
    if (tid_x() == 0) {
      if (p.w0) p.w0[b] = w0;
      if (p.minwt) p.minwt[b] = mw;
      if (p.acmax) p.acmax[b] = ac;
      if (p.pcwt) p.pcwt[b] = pw;
      g_nl = min(g_nl, (N - mx) >> 1);
      g_unb += w0 != 0;
      g_mw = min(g_mw, mw);
      g_ac = max(g_ac, ac);
      g_pw = min(g_pw, pw);
    }
    __syncthreads();
  }
  if (tid_x() == 0) {
    atomicMin(&p.crit[0], g_nl);
    if (g_unb) atomicAdd(&p.crit[1], g_unb);
    atomicMin(&p.crit[2], g_mw);
    atomicMax(&p.crit[4], g_ac);
    atomicMin(&p.crit[5], g_pw);
  }
}

// ---------------------------------------------------------------------------
// Component criteria, register-blocked (5 <= n <= 12, needs the bit-sliced
// words F; k_crit_wide below takes n = 13 .. 16).  A group of GL = 2^(n-RB)
// lanes owns one mask at a time and each lane holds R = 2^RB int32 values
// (RB = max(5, ceil(n/2))).  Two layouts of the 2^n entries (register j of
// lane l):
//   A: entry (l << RB) | j            bits 0..RB-1 in registers
//   B: entry (j << LB) | l            bits LB..n-1 in registers (LB = n - RB)
// The transforms are products of commuting per-bit stages, so each runs the
// stages of whatever bits its current layout holds in registers:
//   first transform A -> B: popcount stages over bits 0..4 (bias -16: the
//     values are u = -W/2 from the start), then the register stages;
//   v = u^2 = (W/2)^2 (24-bit multiply, |u| <= 2^11);
//   second transform B -> A, giving V(d) = 2^(n-2) r(d).
// Exchanges go through LDS rows of R + 4 words: layout A moves 16-byte quads
// of its own row (the padding puts the rows of consecutive lanes on
// different banks), layout B single words at (lane + a constant per
// register), conflict-free.
// Reductions: max v gives max|W|; for the smallest weight of a nonzero value
// the registers are OR-ed by the weight of their index (a compile-time
// constant) and the lane adds the weight of its own bits.
// ---------------------------------------------------------------------------
constexpr int kCritRegMaxGrid = 4096;  // workgroups (one slot of partial aggregates each)

struct CritRegParams {
  const uint32_t* F;  // [m][2^(n-5)] bit-sliced words
  int m;
  long long chunk;    // Gray indices per group
  int32_t* part;      // [gdim_x()][8] per-workgroup aggregates (nl, unbalanced, minwt, acmax, pcwt)
  int32_t* w0;
  int32_t* minwt;
  int32_t* acmax;
  int32_t* pcwt;
};

// register bits per lane and workgroup size of the register-blocked criteria
// kernels (host and device): k_crit_reg up to n = 12, k_crit_wide (64 values
// per lane, one workgroup of 2^(n-6) lanes per mask) from n = 13
__host__ __device__ constexpr int crit_reg_rb(int n) { return n > 12 ? 6 : ((n + 1) / 2 > 5 ? (n + 1) / 2 : 5); }
__host__ __device__ constexpr int crit_reg_wg(int n) { return n > 12 ? (1 << (n - 6)) : 256; }

template <int N>
struct CritShape {
  static_assert(N >= 5 && N <= 12, "k_crit_wide takes n > 12");
  static constexpr int RB = crit_reg_rb(N);
  static constexpr int LB = N - RB;
  static constexpr int R = 1 << RB;
  static constexpr int GL = 1 << LB;            // lanes per group
  static constexpr int WPL = R / 32;
  static constexpr int WG = crit_reg_wg(N);     // threads per workgroup
  static constexpr int GPB = WG / GL;           // groups per workgroup
  static constexpr int ROW = R + 4;             // padded LDS row (words)
  static constexpr int GWORDS = GL * ROW;       // LDS words per group
};

// Butterflies of one register bit over an array of R values.
template <int R, int BIT>
__device__ __forceinline__ void reg_stage(int32_t* v) {
#pragma unroll
  for (int j = 0; j < R; ++j)
    if (!(j & (1 << BIT))) {
      const int32_t a = v[j], b = v[j | (1 << BIT)];
      v[j] = a + b;
      v[j | (1 << BIT)] = a - b;
    }
}
template <int R, int LO, int HI>
__device__ __forceinline__ void reg_stages(int32_t* v) {
  if constexpr (LO < HI) {
    reg_stage<R, LO>(v);
    reg_stages<R, LO + 1, HI>(v);
  }
}

// Smallest class c (0..C) whose OR-accumulator is nonzero, skipping class 0
// when skip0; 99 if none.
template <int C>
__device__ __forceinline__ int first_class(const uint32_t* acc, bool skip0) {
  int c = 99;
#pragma unroll
  for (int k = C; k >= 1; --k) c = acc[k] ? k : c;
  return (!skip0 && acc[0]) ? 0 : c;
}

template <int GL>
__device__ __forceinline__ void group_sync() {
  if constexpr (GL > 64) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Reduction over the GL lanes of a group; GL > 64 spans GL / 64 <= 16 waves
// that meet in `xr` (one int per wave).
template <int GL, bool IS_MAX>
__device__ __forceinline__ int crit_group_reduce(int v, int* xr, int l) {
  if constexpr (GL <= 64) {
    return group_reduce<GL, IS_MAX>(v);
  } else {
    constexpr int NW = GL / 64;  // waves of the group, <= 16
    v = group_reduce<64, IS_MAX>(v);
    if ((l & 63) == 0) xr[__builtin_amdgcn_readfirstlane(l >> 6)] = v;  // the wave's slot: a scalar offset
    __syncthreads();
    // one wave value per lane, then a reduction inside each row of 16 lanes
    const int r = group_reduce<NW, IS_MAX>(xr[l & (NW - 1)]);
    __syncthreads();
    return r;
  }
}

// Layout A side of an exchange: the lane's own row, 16-byte quads.
template <int R, int ROW>
__device__ __forceinline__ void put_rows(int32_t* buf, int l, const int32_t* v) {
#pragma unroll
  for (int q = 0; q < R / 4; ++q)
    *reinterpret_cast<int4*>(buf + l * ROW + 4 * q) = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}
template <int R, int ROW>
__device__ __forceinline__ void get_rows(const int32_t* buf, int l, int32_t* v) {
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    const int4 t = *reinterpret_cast<const int4*>(buf + l * ROW + 4 * q);
    v[4 * q] = t.x;
    v[4 * q + 1] = t.y;
    v[4 * q + 2] = t.z;
    v[4 * q + 3] = t.w;
  }
}
template <int N>
__global__ __launch_bounds__(crit_reg_wg(N)) void k_crit_reg(const CritRegParams p) {
  using C = CritShape<N>;
  constexpr int RB = C::RB, LB = C::LB, R = C::R, GL = C::GL, WPL = C::WPL, GPB = C::GPB, ROW = C::ROW;
  __shared__ __attribute__((aligned(16))) int32_t lds[GPB * C::GWORDS];
  __shared__ int xr[GPB][GL > 64 ? GL / 64 : 1];
  __shared__ int agg[GPB][5];
  const int tid = tid_x();
  const int grp = tid / GL;
  const int l = tid % GL;
  int32_t* buf = lds + grp * C::GWORDS;
  auto at = [](int e) { return (e >> RB) * ROW + (e & (R - 1)); };  // LDS word of entry e
  const int nwords = 1 << (N - 5);
  const long long kend = 1LL << p.m;
  const long long kfirst = 1 + ((long long)bid_x() * GPB + grp) * p.chunk;
  const int lw = __builtin_popcount(l);

  // this group's share of the aggregates, folded per workgroup at the end
  int g_nl = 1 << (N - 1), g_unb = 0, g_mw = N + 1, g_ac = 0, g_pw = N + 1;

  uint32_t G[WPL], Fn[WPL];
#pragma unroll
  for (int t = 0; t < WPL; ++t) G[t] = Fn[t] = 0;
  if (kfirst < kend) {
    const long long gk = gray(kfirst);
    for (int i = 0; i < p.m; ++i)
      if ((gk >> i) & 1) {
#pragma unroll
        for (int t = 0; t < WPL; ++t) G[t] ^= p.F[(long long)i * nwords + l * WPL + t];
      }
  }
  // every group runs the same number of steps (uniform barriers); steps past
  // the last mask compute on stale words and write nothing
  for (long long step = 0; step < p.chunk; ++step) {
    const long long k = kfirst + step;
    const bool valid = k < kend;
    if (step > 0) {
#pragma unroll
      for (int t = 0; t < WPL; ++t) G[t] ^= Fn[t];
    }
    if (k + 1 < kend && step + 1 < p.chunk) {
      const int i = __builtin_ctzll((unsigned long long)(k + 1));
#pragma unroll
      for (int t = 0; t < WPL; ++t) Fn[t] = p.F[(long long)i * nwords + l * WPL + t];
    }
    int32_t v[R];
    // ---- first transform, layout A: popcounts (bits 0..4), then bits 5..RB-1
#pragma unroll
    for (int t = 0; t < WPL; ++t)
#pragma unroll
      for (int a = 0; a < 32; ++a) v[t * 32 + a] = (int32_t)__builtin_popcount(G[t] ^ walsh_mask(a)) - 16;
    reg_stages<R, 5, RB>(v);
    put_rows<R, ROW>(buf, l, v);
    group_sync<GL>();
    // ---- A -> B: bits RB..n-1 = register bits RB-LB..RB-1
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = buf[at(j << LB) + l];
    group_sync<GL>();
    reg_stages<R, RB - LB, RB>(v);
    // u = -W/2 at a = (j << LB) | l
    const int w0 = -2 * v[0];  // W(0, b) (lane l = 0)
    uint32_t ci[RB + 1];
#pragma unroll
    for (int c = 0; c <= RB; ++c) ci[c] = 0;
    int mxsq = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int32_t s = mul24s(v[j], v[j]);
      mxsq = max(mxsq, s);
      ci[__builtin_popcount(j)] |= (uint32_t)s;
      v[j] = s;
    }
    // group results of the first transform now (a convergent reduction the
    // compiler cannot sink past the second transform with all the squares)
    int mw = first_class<RB>(ci, l == 0) + lw;
    mxsq = crit_group_reduce<GL, true>(mxsq, xr[grp], l);
    mw = crit_group_reduce<GL, false>(mw, xr[grp], l);
    // ---- second transform: all register bits of B (bits LB..n-1)
    reg_stages<R, 0, RB>(v);
#pragma unroll
    for (int j = 0; j < R; ++j) buf[at(j << LB) + l] = v[j];
    group_sync<GL>();
    get_rows<R, ROW>(buf, l, v);
    group_sync<GL>();
    // ---- layout A: the bits not yet done (0..LB-1); V(d) at d = (l << RB) | j
    reg_stages<R, 0, LB>(v);
    if (l == 0) v[0] = 0;  // d = 0 is not a direction
    uint32_t pc[RB + 1];
#pragma unroll
    for (int c = 0; c <= RB; ++c) pc[c] = 0;
    int vmax = 0, vmin = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      vmax = max(vmax, v[j]);
      vmin = min(vmin, v[j]);
      pc[__builtin_popcount(j)] |= (uint32_t)v[j];
    }
    // ---- per-lane results, then the group's
    int pw = first_class<RB>(pc, l == 0) + lw;
    int ac = max(vmax, -vmin) >> (N - 2);  // |V| = 2^(n-2) |r|, exact
    ac = crit_group_reduce<GL, true>(ac, xr[grp], l);
    pw = crit_group_reduce<GL, false>(pw, xr[grp], l);
    if (mw > N) mw = N + 1;
    if (pw > N) pw = N + 1;
    if (l == 0 && valid) {
      const long long b = gray(k);
      const int umax = (int)rintf(sqrtf((float)mxsq));  // mxsq is a perfect square <= 2^22
      if (p.w0) p.w0[b] = w0;
      if (p.minwt) p.minwt[b] = mw;
      if (p.acmax) p.acmax[b] = ac;
      if (p.pcwt) p.pcwt[b] = pw;
      g_nl = min(g_nl, (1 << (N - 1)) - umax);
      g_unb += w0 != 0;
      g_mw = min(g_mw, mw);
      g_ac = max(g_ac, ac);
      g_pw = min(g_pw, pw);
    }
  }
  // the workgroup's aggregates into its slot (no atomics on shared words:
  // thousands of them from every workgroup serialise in L2)
  if (l == 0) {
    agg[grp][0] = g_nl;
    agg[grp][1] = g_unb;
    agg[grp][2] = g_mw;
    agg[grp][3] = g_ac;
    agg[grp][4] = g_pw;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < GPB; ++q) {
      g_nl = min(g_nl, agg[q][0]);
      g_unb += agg[q][1];
      g_mw = min(g_mw, agg[q][2]);
      g_ac = max(g_ac, agg[q][3]);
      g_pw = min(g_pw, agg[q][4]);
    }
    int32_t* o = p.part + 8 * bid_x();
    o[0] = g_nl;
    o[1] = g_unb;
    o[2] = g_mw;
    o[3] = g_ac;
    o[4] = g_pw;
  }
}

// ---------------------------------------------------------------------------
// Component criteria at n = 13 .. 16, register-blocked: one workgroup of
// 2^(n-6) lanes (2 .. 16 waves) per mask, 64 int32 values per lane (the
// whole 2^n entries live in registers), layouts as in k_crit_reg:
//   A: lane l holds entry (l << 6) | j                      bits 0..5
//   M: lane (w, i) = (l >> 6, l & 63) holds (w << 12) | (j << 6) | i   bits 6..11
//   C: lane l holds (P(j) << (n-6)) | l                     bits n-6..n-1
// with P putting register bit 5 on entry bit 11 and bits 0..4 on the other
// five, in order.  A <-> M stays inside each wave (its 2^12 entries): the
// waves take two turns over padded 17 KiB LDS blocks, and the waves of the
// first turn run their stages while the second turn exchanges.  M <-> C
// crosses waves and runs in two rounds of 2^(n-1) entries, split on entry
// bit 11, which is register bit 5 in both M and C, so each round empties and
// refills the same 32 registers.  LDS is 144 / 72 / 36 / 18 KiB for
// n = 16 / 15 / 14 / 13 (exchange blocks plus the Gray-code walk state):
// 16 waves per CU, <= 128 VGPRs each, and nothing that can be rebuilt is
// kept live across the mask loop, so no registers spill.
// ---------------------------------------------------------------------------
// Entry of C register jj (bits 0..4 of the register index; bit 5 is the
// round) without the lane part, with entry bit 11 taken out.
template <int N>
__host__ __device__ constexpr int crit_c_entry(int jj) {
  int x = 0;
  for (int k = 0, off = 0; k < 5; ++k, ++off) {
    if (off == 17 - N) ++off;  // the offset of entry bit 11 belongs to register bit 5
    if ((jj >> k) & 1) x |= 1 << (N - 6 + off);
  }
  return ((x >> 12) << 11) | (x & 0x7FF);
}

template <int N>
__global__ __launch_bounds__(1 << (N - 6), 4) void k_crit_wide(const CritRegParams p) {  // four waves per SIMD
  constexpr int R = 64, ROW = 68;
  constexpr int NWAV = 1 << (N - 12);  // waves per mask
  constexpr int NB = NWAV / 2;         // LDS blocks: waves per turn of the A <-> M exchange
  constexpr int LDS_WORDS = (NB * 64 * ROW > (1 << (N - 1))) ? NB * 64 * ROW : (1 << (N - 1));
  __shared__ __attribute__((aligned(16))) int32_t lds[LDS_WORDS];
  __shared__ int xr[NWAV];
  // the lane's two bit-sliced words of the current mask (the Gray-code walk
  // state), kept here rather than in registers: 1 KiB per wave
  __shared__ uint2 gw[64 * NWAV];
  const int l = tid_x();
  const int w = __builtin_amdgcn_readfirstlane(l >> 6), i = l & 63;  // wave index: uniform, scalar branches
  const bool first_turn = w < NB;
  int32_t* blk = lds + (w % NB) * 64 * ROW;  // this wave's block for A <-> M
  constexpr int nwords = 1 << (N - 5);
  // 32-bit mask counters (m <= 24): their compares stay on the scalar unit
  const int kend = 1 << p.m;
  const int chunk = (int)p.chunk;
  const int kfirst = 1 + (int)bid_x() * chunk;
  // running aggregates (nl, unbalanced, min weight, abs indicator, min PC
  // weight) in LDS, updated by thread 0 only: nothing loop-carried for them
  // in registers
  __shared__ int agg[5];
  if (tid_x() == 0) {
    agg[0] = 1 << (N - 1);
    agg[1] = 0;
    agg[2] = N + 1;
    agg[3] = 0;
    agg[4] = N + 1;
  }
  auto words = [&](int b, int lane) {  // bit slice b, the lane's two words
    return reinterpret_cast<const uint2*>(p.F + b * nwords)[lane];
  };

  {
    uint2 G = make_uint2(0, 0);
    if (kfirst < kend) {
      const int gk = (int)gray(kfirst);
      for (int b = 0; b < p.m; ++b)
        if ((gk >> b) & 1) {
          const uint2 f = words(b, l);
          G.x ^= f.x;
          G.y ^= f.y;
        }
    }
    gw[l] = G;
  }
  // A rows / M words of this wave's block
  auto put_a = [&](const int32_t* v) { put_rows<R, ROW>(blk, i, v); };
  auto get_a = [&](int32_t* v) { get_rows<R, ROW>(blk, i, v); };
  auto put_m = [&](const int32_t* v) {
#pragma unroll
    for (int j = 0; j < R; ++j) blk[j * ROW + i] = v[j];
  };
  auto get_m = [&](int32_t* v) {
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = blk[j * ROW + i];
  };
  auto wsync = []() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  // M <-> C round r (entry bit 11 = r): entries without bit 11, 2^(n-1) words
  auto put_m_round = [&](const int32_t* v, int r) {
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) lds[(w << 11) | (jj << 6) | i] = v[32 * r + jj];
  };
  auto get_m_round = [&](int32_t* v, int r) {
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) v[32 * r + jj] = lds[(w << 11) | (jj << 6) | i];
  };
  auto put_c_round = [&](const int32_t* v, int r) {
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) lds[crit_c_entry<N>(jj) + l] = v[32 * r + jj];
  };
  auto get_c_round = [&](int32_t* v, int r) {
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) v[32 * r + jj] = lds[crit_c_entry<N>(jj) + l];
  };

  for (int step = 0; step < chunk; ++step) {
    const int k = kfirst + step;
    const bool valid = k < kend;
    // the lane index, recomputed per mask: values derived from it (a 64-bit
    // address, its weight) are cheaper to rebuild than to keep in registers
    int lr = l;
    asm volatile("" : "+v"(lr));
    int32_t v[R];
    // ---- first transform: layout A, popcounts (bits 0..4) and bit 5
    {
      const uint2 G = gw[lr];
#pragma unroll
      for (int a = 0; a < 32; ++a) v[a] = (int32_t)__builtin_popcount(G.x ^ walsh_mask(a)) - 16;
#pragma unroll
      for (int a = 0; a < 32; ++a) v[32 + a] = (int32_t)__builtin_popcount(G.y ^ walsh_mask(a)) - 16;
    }
    // the next mask's slice: loaded now, folded into gw after the exchange
    const bool more = k + 1 < kend && step + 1 < chunk;
    uint2 fn = make_uint2(0, 0);
    if (more) fn = words(__builtin_ctz((unsigned)(k + 1)), lr);
    reg_stages<R, 5, 6>(v);
    __syncthreads();  // the previous mask's last reads of the blocks are done
    if (first_turn) { put_a(v); wsync(); get_m(v); }
    __syncthreads();
    if (!first_turn) { put_a(v); wsync(); get_m(v); }
    if (more) {
      uint2 g = gw[lr];
      g.x ^= fn.x;
      g.y ^= fn.y;
      gw[lr] = g;
    }
    reg_stages<R, 0, 6>(v);  // M: bits 6..11
    __syncthreads();
    put_m_round(v, 0);
    __syncthreads();
    get_c_round(v, 0);
    __syncthreads();
    put_m_round(v, 1);
    __syncthreads();
    get_c_round(v, 1);
    reg_stages<R, 17 - N, 5>(v);  // C: bits 12..n-1
    // u = -W/2 at a = (P(j) << (n-6)) | l; entry 0 is lane 0 of wave 0
    const int w0 = __builtin_amdgcn_readfirstlane(-2 * v[0]);
    uint32_t ci[7] = {0, 0, 0, 0, 0, 0, 0};
    int mxsq = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int32_t s = mul24s(v[j], v[j]);
      mxsq = max(mxsq, s);
      ci[__builtin_popcount(j)] |= (uint32_t)s;
      v[j] = s;
    }
    // group results of the first transform now (a convergent reduction the
    // compiler cannot sink past the second transform with all the squares)
    int mw = first_class<6>(ci, l == 0) + __builtin_popcount(lr);
    mxsq = __builtin_amdgcn_readfirstlane(crit_group_reduce<64 * NWAV, true>(mxsq, xr, l));
    mw = __builtin_amdgcn_readfirstlane(crit_group_reduce<64 * NWAV, false>(mw, xr, l));
    // ---- second transform: C bits n-6..n-1, M bits 6..n-7, A bits 0..5
    reg_stages<R, 0, 6>(v);
    __syncthreads();
    put_c_round(v, 0);
    __syncthreads();
    get_m_round(v, 0);
    __syncthreads();
    put_c_round(v, 1);
    __syncthreads();
    get_m_round(v, 1);
    reg_stages<R, 0, N - 12>(v);
    __syncthreads();
    if (first_turn) { put_m(v); wsync(); get_a(v); }
    __syncthreads();
    if (!first_turn) { put_m(v); wsync(); get_a(v); }
    reg_stages<R, 0, 6>(v);
    // V(d) at d = (l << 6) | j
    if (l == 0) v[0] = 0;
    uint32_t pc[7] = {0, 0, 0, 0, 0, 0, 0};
    int vmax = 0, vmin = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      vmax = max(vmax, v[j]);
      vmin = min(vmin, v[j]);
      pc[__builtin_popcount(j)] |= (uint32_t)v[j];
    }
    int pw = first_class<6>(pc, l == 0) + __builtin_popcount(lr);
    int ac = max(vmax, -vmin) >> (N - 2);
    ac = __builtin_amdgcn_readfirstlane(crit_group_reduce<64 * NWAV, true>(ac, xr, l));
    pw = __builtin_amdgcn_readfirstlane(crit_group_reduce<64 * NWAV, false>(pw, xr, l));
    if (mw > N) mw = N + 1;
    if (pw > N) pw = N + 1;
    if (valid && l == 0) {
      const int umax = (int)rintf(sqrtf((float)mxsq));  // mxsq is a perfect square <= 2^30
      const int b = (int)gray(k);
      if (p.w0) p.w0[b] = w0;
      if (p.minwt) p.minwt[b] = mw;
      if (p.acmax) p.acmax[b] = ac;
      if (p.pcwt) p.pcwt[b] = pw;
      agg[0] = min(agg[0], (1 << (N - 1)) - umax);
      agg[1] += w0 != 0;
      agg[2] = min(agg[2], mw);
      agg[3] = max(agg[3], ac);
      agg[4] = min(agg[4], pw);
    }
  }
  if (l == 0) {
    int32_t* o = p.part + 8 * bid_x();
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q] = agg[q];
  }
}

// Aggregates of the register-blocked criteria kernel: the per-workgroup slots
// folded into crit[] (which holds the start values), then the orders as in
// k_criteria_finish.
__global__ __launch_bounds__(256) void k_crit_reg_finish(const int32_t* part, int nwg, int32_t* crit) {
  __shared__ int red[4];
  int nl = 0x7fffffff, unb = 0, mw = 0x7fffffff, ac = 0, pw = 0x7fffffff;
  for (int i = tid_x(); i < nwg; i += bdim_x()) {
    const int32_t* o = part + 8 * i;
    nl = min(nl, o[0]);
    unb += o[1];
    mw = min(mw, o[2]);
    ac = max(ac, o[3]);
    pw = min(pw, o[4]);
  }
  nl = block_reduce<false>(nl, red);
  mw = block_reduce<false>(mw, red);
  ac = block_reduce<true>(ac, red);
  pw = block_reduce<false>(pw, red);
  unb = block_sum(unb, red);
  if (tid_x() == 0) {
    crit[0] = min(crit[0], nl);
    crit[1] += unb;
    crit[2] = min(crit[2], mw) - 1;
    crit[3] = crit[1] == 0 ? crit[2] : -1;
    crit[4] = max(crit[4], ac);
    crit[5] = min(crit[5], pw) - 1;
  }
}

// crit[] start values; per-mask outputs at b = 0 are defined as 0.
__device__ __forceinline__ void criteria_start(int32_t* crit, int n, int32_t* w0, int32_t* minwt, int32_t* acmax,
                                               int32_t* pcwt) {
  if (tid_x() == 0) {
    crit[0] = 1 << (n - 1);
    crit[1] = 0;
    crit[2] = n + 1;
    crit[3] = 0;
    crit[4] = 0;
    crit[5] = n + 1;
    crit[6] = 0;
    crit[7] = 0;
    if (w0) w0[0] = 0;
    if (minwt) minwt[0] = 0;
    if (acmax) acmax[0] = 0;
    if (pcwt) pcwt[0] = 0;
  }
}

__global__ void k_criteria_init(int32_t* crit, int n, int32_t* w0, int32_t* minwt, int32_t* acmax, int32_t* pcwt) {
  criteria_start(crit, n, w0, minwt, acmax, pcwt);
}

// The criteria's start values (workgroup 0) and bit-sliced table (the others)
// in one launch.
template <int EB>
__global__ __launch_bounds__(256) void k_crit_prep(const void* S, int n, int m, uint32_t* F, int nwords, int32_t* crit,
                                                   int32_t* w0, int32_t* minwt, int32_t* acmax, int32_t* pcwt) {
  if (bid_x() == 0) {
    criteria_start(crit, n, w0, minwt, acmax, pcwt);
    return;
  }
  if (n >= 6) {  // a wave per 64 entries
    const long long x0 = ((long long)(bid_x() - 1) * bdim_x() + (tid_x() & ~63));
    if (x0 < (1LL << n)) bitslice_wave<EB>(S, m, F, nwords, x0);
    return;
  }
  const int w = (bid_x() - 1) * bdim_x() + tid_x();
  if (w < nwords) bitslice_words<EB>(S, n, m, F, nwords, w);
}

// Orders from the minimum weights: CI = minwt - 1, resiliency = CI if balanced.
__global__ void k_criteria_finish(int32_t* crit) {
  if (tid_x() == 0) {
    crit[2] = crit[2] - 1;
    crit[3] = crit[1] == 0 ? crit[2] : -1;
    crit[5] = crit[5] - 1;
  }
}
// ---------------------------------------------------------------------------
// a-major spectrum of a large box: the fused kernel (mode kSlab16) writes the
// rows of an aligned block of masks b in [b0, b0 + B) as int16 -W/2 into a
// slab, and this kernel transposes the slab into columns b0 .. b0 + B - 1 of
// the a-major matrix (scaled by wscale: W or W/2) through an LDS tile of 64
// rows by 128 entries read as int16 pairs, so that the slab reads (along a)
// and the spectrum writes (along b) are 256-byte runs.  Column b = 0 is
// written by the init kernel and skipped here.  With `skip` set, the launch
// does nothing when *skip != 0 (the box is a permutation, whose a-major
// matrix the call writes another way).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_transpose_slab16(const int16_t* slab, int n, int32_t* spec, int m,
                                                          long long b0, int B, int wscale, const void* S, int eb,
                                                          const int* skip) {
  if (skip && *skip) return;
  __shared__ int32_t tile[64][65];  // tile[j][p]: entries a0 + 2p, a0 + 2p + 1 of row j
  const long long N = 1LL << n;
  const long long a0 = (long long)bid_x() * 128;
  const int j0 = bid_y() * 64;
  const int tx = tid_x() & 63, ty = tid_x() >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int j = j0 + r;
    if (j < B && a0 + 2 * tx < N) tile[r][tx] = reinterpret_cast<const int32_t*>(slab + (long long)j * N + a0)[tx];
  }
  __syncthreads();
  const int j = j0 + tx;
  const long long b = b0 + j;
  // the one value int16 cannot hold: -W/2 = +2^15, stored as -2^15.  It only
  // occurs for an affine component at n = 16, W(a, b) = 2^16 (-1)^(b . S(0)).
  const uint32_t s0 = eb == 1 ? *reinterpret_cast<const uint8_t*>(S)
                    : eb == 2 ? *reinterpret_cast<const uint16_t*>(S) : *reinterpret_cast<const uint32_t*>(S);
  const bool flip = __builtin_popcount((uint32_t)b & s0) & 1;
  for (int r = ty; r < 128; r += 4) {
    const long long a = a0 + r;
    const uint32_t pair = (uint32_t)tile[tx][r >> 1];
    int v = (int16_t)((r & 1) ? (pair >> 16) : (pair & 0xFFFFu));
    if (v == -32768 && flip) v = 32768;
    // streaming stores: the final spectrum must not evict the slab from the caches
    if (j < B && a < N && b != 0) __builtin_nontemporal_store(wscale * v, &spec[(a << m) + b]);
  }
}

// Start values of a call without its own preparation launch (n > 16).
__global__ __launch_bounds__(256) void k_init_jobs(const JobDesc* jobs, JobDesc job0, int njobs,
                                                   int* queue, int nqueue, int layout) {
  const int j = bid_x();
  if (j >= njobs) return;
  init_job(jobs ? jobs[j] : job0, j == 0, queue, nqueue, layout);
}

// A single box in one launch before its transform: workgroup 0 sets the
// start values, the others bit-slice the table into jd.F (dense words from
// n = 6 on: a wave per 64 entries, which also write those entries of the
// spectrum's b = 0 row or column, a column being one cache line an entry;
// else a word a thread).
template <int EB>
__global__ __launch_bounds__(256) void k_prep_single(JobDesc jd, int* queue, int nqueue, int layout) {
  const bool dense = jd.n >= 6 && !(jd.flags & kWordsFp4);
  if (bid_x() == 0) {
    init_job(jd, true, queue, nqueue, layout, !dense);
    return;
  }
  if (dense) {  // a wave per 64 entries
    const long long x0 = ((long long)(bid_x() - 1) * bdim_x() + (tid_x() & ~63));
    if (x0 < (1LL << jd.n)) {
      if (jd.spec) init_spec_entry(jd, x0 + (tid_x() & 63), layout);
      bitslice_wave<EB>(jd.S, jd.m, const_cast<uint32_t*>(jd.F), jd.nwords, x0);
    }
    return;
  }
  const int w = (bid_x() - 1) * bdim_x() + tid_x();
  if (w < jd.nwords) bitslice_job<EB>(jd, w);
}

// ---------------------------------------------------------------------------
// a-major spectrum of a permutation (n = m).  Substituting y = S(x) in the
// sum of Eq. 1 gives W_{S^-1}(u, v) = W_S(v, u): the spectrum of the inverse
// map is the transpose, so row a of the a-major matrix of S is row a of the
// b-major matrix of S^-1, which the b-major store mode writes as whole rows,
// with no slab and no transpose.  Whether S is a permutation is found on the
// device, so that the call stays asynchronous and capturable: the scatter
// writes inv[S(x)] = x and sets *bij = 1; the check clears *bij if some y
// has S(inv[y]) != y, which (with n = m) happens exactly when S is not onto.
// Later launches of the call read *bij and either run or return at once.
// ---------------------------------------------------------------------------
template <int EB>
__global__ __launch_bounds__(256) void k_perm_scatter(const void* S, int n, uint16_t* inv, int* bij) {
  const uint32_t x = bid_x() * bdim_x() + tid_x();
  if (x == 0) *bij = 1;
  if (x < (1u << n)) inv[load_entry<EB>(S, x) & ((1u << n) - 1)] = (uint16_t)x;
}

// The check, then the start values of the b-major job of S^-1 (workgroup 0:
// its NL start value and row 0, W_{S^-1}(u, 0) = 2^n [u = 0], which is row
// a = 0 of the a-major matrix of S) and its bit-sliced words (the other
// workgroups, a wave per 64 entries of inv).  Row 0 is written either way:
// if S is not a permutation, the transposed slabs overwrite every entry
// but the first, which is 2^n for every S.
template <int EB>
__global__ __launch_bounds__(256) void k_perm_check_prep(const void* S, JobDesc jinv, int* bij, int* queue,
                                                         int nqueue) {
  if (bid_x() == 0) {
    init_job(jinv, true, queue, nqueue, 1);
    return;
  }
  const long long y0 = (long long)(bid_x() - 1) * bdim_x() + (tid_x() & ~63);
  if (y0 >= (1LL << jinv.n)) return;
  const uint32_t y = (uint32_t)y0 + (tid_x() & 63);
  // an entry no x was scattered to holds an old value: masked to stay inside S
  const uint32_t x = reinterpret_cast<const uint16_t*>(jinv.S)[y] & ((1u << jinv.n) - 1);
  if ((load_entry<EB>(S, x) & ((1u << jinv.m) - 1)) != y) *bij = 0;
  bitslice_wave<2>(jinv.S, jinv.m, const_cast<uint32_t*>(jinv.F), jinv.nwords, y0);
}

// Zero `count` ints (queue counters, per-batch maxima) without a memset node.
__global__ __launch_bounds__(256) void k_zero(int* p, long long count) {
  for (long long i = bid_x() * (long long)bdim_x() + tid_x(); i < count;
       i += (long long)gdim_x() * bdim_x())
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// n > 16, second pass: transform over the block index bits [bit0, bit0+R)
// of T[slot][blk][a_lo] (in place), or, on the last pass, fold the maximum
// and write the requested spectrum.
// ---------------------------------------------------------------------------
template <int R, bool LAST>
__global__ __launch_bounds__(256) void k_combine(int32_t* T, long long kcount, int nblk_log, int bit0,
                                                 int* slotmax, int32_t* spec, int layout, int wscale, int m,
                                                 long long kbase, long long mend) {
  const int L = nblk_log;
  const long long per_slot = (1LL << 16) << (L - R);  // threads per slot
  const long long idx = bid_x() * (long long)bdim_x() + tid_x();
  const long long slot = idx / per_slot;
  int mx = 0;
  if (slot < kcount) {
    const long long rem = idx - slot * per_slot;
    const long long alo = rem & 0xFFFF;
    const long long other = rem >> 16;  // block bits outside [bit0, bit0+R)
    const long long lowmask = (1LL << bit0) - 1;
    const long long base_blk = (other & lowmask) | ((other >> bit0) << (bit0 + R));
    int32_t* base = T + (slot << (16 + L)) + alo;
    int v[1 << R];
#pragma unroll
    for (int j = 0; j < (1 << R); ++j) v[j] = base[(base_blk | ((long long)j << bit0)) << 16];
#pragma unroll
    for (int h = 1; h < (1 << R); h <<= 1)
#pragma unroll
      for (int j = 0; j < (1 << R); ++j)
        if (!(j & h)) {
          const int a = v[j], c = v[j | h];
          v[j] = a + c;
          v[j | h] = a - c;
        }
    if constexpr (LAST) {
      const long long k = kbase + slot;
      const bool valid = k != 0 && k < mend;
      const uint32_t b = (uint32_t)gray(k);
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) {
        mx = max(mx, v[j] < 0 ? -v[j] : v[j]);
        if (spec && valid) {
          const long long a = alo | ((base_blk | ((long long)j << bit0)) << 16);
          if (layout == 1) spec[((long long)b << (16 + L)) | a] = wscale * v[j];
          else spec[(a << m) | b] = wscale * v[j];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < (1 << R); ++j) base[(base_blk | ((long long)j << bit0)) << 16] = v[j];
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((tid_x() & 63) == 0 && slot < kcount) atomicMax(&slotmax[slot], mx);
  }
}

// n > 16: per-mask maxima of the batch -> maxabs and NL.
__global__ __launch_bounds__(256) void k_finalize_batch(const int* slotmax, long long kcount, long long kbase,
                                                        long long mend, int n, int32_t* maxabs, int32_t* nl) {
  const long long s = bid_x() * (long long)bdim_x() + tid_x();
  int cand = 0x7fffffff;
  if (s < kcount) {
    const long long k = kbase + s;
    if (k != 0 && k < mend) {
      const int mx = slotmax[s];
      if (maxabs) maxabs[gray(k)] = 2 * mx;
      cand = (1 << (n - 1)) - mx;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) cand = min(cand, __shfl_xor(cand, o, 64));
  if ((tid_x() & 63) == 0 && cand != 0x7fffffff) atomicMin(nl, cand);
}

// ---------------------------------------------------------------------------
// Avalanche and bit independence: the autocorrelation of every component at
// the unit input differences e_i,
//   r_b(e_i) = sum_x (-1)^(b . (S(x) ^ S(x ^ e_i))) = sum_y c_i[y] (-1)^(b . y),
// i.e. the 2^m-point transform over the output masks of the counts
// c_i[y] = #{x : S(x) ^ S(x ^ e_i) = y}.
// ---------------------------------------------------------------------------

// c_i[y] += 2 for each pair {x, x ^ e_i}: one thread per (i, x with bit i clear).
template <int EB>
__global__ __launch_bounds__(256) void k_deriv_count(const void* S, int n, int m, int32_t* cnt) {
  const long long half = 1LL << (n - 1);
  const long long total = (long long)n * half;
  const uint32_t mmask = (m >= 32) ? 0xffffffffu : ((1u << m) - 1u);
  for (long long t = bid_x() * (long long)bdim_x() + tid_x(); t < total;
       t += (long long)gdim_x() * bdim_x()) {
    const int i = (int)(t >> (n - 1));
    const long long j = t & (half - 1);
    const long long x = ((j >> i) << (i + 1)) | (j & ((1LL << i) - 1));
    const uint32_t y = (load_entry<EB>(S, x) ^ load_entry<EB>(S, x | (1LL << i))) & mmask;
    atomicAdd(cnt + ((size_t)i << m) + y, 2);
  }
}

// One pass of an in-place int32 Walsh-Hadamard transform of length 2^mlog
// on each of the vectors: bits [lo, lo + R) through an LDS tile of 2^R rows
// (stride 2^lo) by 2^cwlog consecutive columns, 2^(R + cwlog) <= 4096.
// Every partial sum of a transform of counts is bounded by their total, so
// int32 holds it.
__global__ __launch_bounds__(256) void k_fwht_pass(int32_t* data, int mlog, int lo, int R, int cwlog) {
  __shared__ int32_t t[4096];
  const int tid = tid_x();
  const int CW = 1 << cwlog, TILE = 1 << (R + cwlog);
  long long blk = bid_x();
  const long long ncolb = 1LL << (lo - cwlog);
  const long long colb = blk % ncolb;
  blk /= ncolb;
  const long long nhi = 1LL << (mlog - lo - R);
  const long long hi = blk % nhi;
  const long long vec = blk / nhi;
  int32_t* base = data + (vec << mlog) + (hi << (lo + R)) + (colb << cwlog);
  for (int e = tid; e < TILE; e += 256) t[e] = base[((long long)(e >> cwlog) << lo) | (e & (CW - 1))];
  __syncthreads();
  for (int sb = 0; sb < R; ++sb) {
    for (int e = tid; e < TILE / 2; e += 256) {
      const int col = e & (CW - 1);
      const int rr = e >> cwlog;
      const int r0 = ((rr >> sb) << (sb + 1)) | (rr & ((1 << sb) - 1));
      const int i0 = (r0 << cwlog) | col, i1 = ((r0 | (1 << sb)) << cwlog) | col;
      const int32_t u = t[i0], v = t[i1];
      t[i0] = u + v;
      t[i1] = u - v;
    }
    __syncthreads();
  }
  for (int e = tid; e < TILE; e += 256) base[((long long)(e >> cwlog) << lo) | (e & (CW - 1))] = t[e];
}

// summary[0] = max_{i,j} |r_{e_j}(e_i)|, [1] = max_{i, j<k} |r_{e_j^e_k}(e_i)|
// (-1 if m < 2), [2] = min_{j<k} (2^n - maxabs[e_j ^ e_k]) / 2 (-1 without
// maxabs or if m < 2).  One workgroup.
__global__ __launch_bounds__(256) void k_avalanche_summary(const int32_t* r, int n, int m, const int32_t* maxabs,
                                                           int32_t* summary) {
  __shared__ int s_val[3];
  const int tid = tid_x();
  if (tid == 0) {
    s_val[0] = 0;
    s_val[1] = m >= 2 ? 0 : -1;
    s_val[2] = (m >= 2 && maxabs) ? (1 << (n - 1)) : -1;
  }
  __syncthreads();
  const int npair = m * (m + 1) / 2;  // (j, j) for the unit masks, (j, k > j) for pairs
  int sac = 0, bic = 0, bnl = 0x7fffffff;
  for (int t = tid; t < n * npair; t += 256) {
    const int i = t / npair;
    int q = t % npair, j = 0;
    while (q >= m - j) {
      q -= m - j;
      ++j;
    }
    const int k = j + q;
    const uint32_t b = (1u << j) | (1u << k);
    const int v = r[((size_t)i << m) + b];
    const int av = v < 0 ? -v : v;
    if (k == j) sac = max(sac, av);
    else {
      bic = max(bic, av);
      if (maxabs && i == 0) bnl = min(bnl, ((1 << n) - maxabs[b]) >> 1);
    }
  }
  atomicMax(&s_val[0], sac);
  if (m >= 2) {
    atomicMax(&s_val[1], bic);
    if (maxabs) atomicMin(&s_val[2], bnl);
  }
  __syncthreads();
  if (tid < 3) summary[tid] = s_val[tid];
}

}  // namespace sbw

// sbox_walsh.hip -- host side of libsboxwalsh.so: argument checks, launch
// planning, workspaces, batching and plans.  The kernels live in
// walsh_kernels.hpp; the ABI is declared in include/sbox_walsh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sbox_walsh.h"
#include "walsh_kernels.hpp"

using namespace sbw;

namespace {

// ---------------------------------------------------------------- errors ---
thread_local std::string g_last_error;

sbox_status fail(sbox_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
sbox_status fail(sbox_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(SBOX_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------- kernels ----
using KFn = void (*)(KParams);

constexpr int default_split(int n) { return n <= 8 ? n : (n <= 12 ? 6 : (n <= 14 ? 7 : 8)); }

bool split_valid(int n, int p) {
  if (n <= 8) return p == n;
  return p >= 6 && p <= 8 && n - p >= 1 && n - p <= p;
}

template <int N, int P>
KFn pick_mode(int mode, bool any_p) {
  if (mode == kMax) return &k_walsh<N, P, kMax>;
  if constexpr (P == default_split(N)) {  // the other modes exist for the default split only
    if (any_p) return nullptr;
    if (mode == kStoreB) return &k_walsh<N, P, kStoreB>;
    if (mode == kSlab16) return &k_walsh<N, P, kSlab16>;
    if (mode == kStoreA) return &k_walsh<N, P, kStoreA>;
    if (mode == kHist) return &k_walsh<N, P, kHist>;
    if (mode == kHistBig) return &k_walsh<N, P, kHistBig>;
  }
  return nullptr;
}

template <int N>
KFn pick_big(int p, int mode) {
  constexpr int D = (N <= 12) ? 6 : (N <= 14 ? 7 : 8);
  const bool nd = p != D;
  if constexpr (N <= 12) {
    if (p == 6) return pick_mode<N, 6>(mode, nd);
  }
  if constexpr (N <= 14) {
    if (p == 7) return pick_mode<N, 7>(mode, nd);
  }
  if (p == 8) return pick_mode<N, 8>(mode, nd);
  return nullptr;
}

KFn lookup_kernel(int n, int p, int mode) {
  switch (n) {
    case 1: return pick_mode<1, 1>(mode, false);
    case 2: return pick_mode<2, 2>(mode, false);
    case 3: return pick_mode<3, 3>(mode, false);
    case 4: return pick_mode<4, 4>(mode, false);
    case 5: return pick_mode<5, 5>(mode, false);
    case 6: return pick_mode<6, 6>(mode, false);
    case 7: return pick_mode<7, 7>(mode, false);
    case 8: return pick_mode<8, 8>(mode, false);
    case 9: return pick_big<9>(p, mode);
    case 10: return pick_big<10>(p, mode);
    case 11: return pick_big<11>(p, mode);
    case 12: return pick_big<12>(p, mode);
    case 13: return pick_big<13>(p, mode);
    case 14: return pick_big<14>(p, mode);
    case 15: return pick_big<15>(p, mode);
    case 16:
      if (mode == kBlock) return p == 8 ? &k_walsh<16, 8, kBlock> : nullptr;
      return pick_big<16>(p, mode);
    default: return nullptr;
  }
}

struct DevInfo {
  int cus = 0;
  std::map<const void*, int> occ;
};
std::mutex g_dev_mu;
std::map<int, DevInfo> g_dev;

sbox_status device_info(int* cus) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DevInfo& di = g_dev[dev];
  if (di.cus == 0) HIP_TRY(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
  *cus = di.cus;
  return SBOX_OK;
}

// Measured best residency where it is below what a kernel's resources
// allow: k_walsh_mx12 (120 registers, so four workgroups per CU would fit)
// runs 12 x 20 in 0.41 ms at three workgroups per CU and 0.44 ms at two or
// four.  0: no cap.
int residency_cap(const void* fn) { return fn == (const void*)&k_walsh_mx12 ? 3 : 0; }

// Resident workgroups of `block` threads per CU (each kernel is always
// launched with one block size, so the kernel address keys the cache).
sbox_status occupancy(const void* fn, int* blocks_per_cu, int block = kWG) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DevInfo& di = g_dev[dev];
  auto it = di.occ.find(fn);
  if (it == di.occ.end()) {
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, 0));
    const int cap = residency_cap(fn);
    if (cap && nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    it = di.occ.emplace(fn, nb).first;
  }
  *blocks_per_cu = it->second;
  return SBOX_OK;
}

sbox_status launch(const void* fn, dim3 grid, dim3 block, void** args, hipStream_t st) {
  HIP_TRY(hipLaunchKernel(fn, grid, block, args, 0, st));
  return SBOX_OK;
}

// ------------------------------------------------------------ checking ----
sbox_status check_nm(int n, int m) {
  if (n < 1 || n > 24 || m < 1 || m > 24 || n + m > 40)
    return fail(SBOX_ERR_UNSUPPORTED, "unsupported size n=%d m=%d (need 1<=n,m<=24, n+m<=40)", n, m);
  return SBOX_OK;
}

bool layout_valid(int layout) {
  return layout == SBOX_SPECTRUM_NONE || layout == SBOX_SPECTRUM_B_MAJOR || layout == SBOX_SPECTRUM_A_MAJOR ||
         layout == SBOX_LAT_B_MAJOR || layout == SBOX_LAT_A_MAJOR;
}
int base_layout(int layout) { return layout & 3; }
int wscale_of(int layout) { return (layout & SBOX_SPECTRUM_LAT) ? -1 : -2; }

sbox_status check_layout(int layout, int n, int m, const int32_t* spec) {
  if (!layout_valid(layout)) return fail(SBOX_ERR_INVALID_ARG, "invalid spectrum layout %d", layout);
  if (layout != SBOX_SPECTRUM_NONE) {
    if (!spec) return fail(SBOX_ERR_INVALID_ARG, "spectrum layout %d requested with a null spectrum", layout);
    if (n + m > 34) return fail(SBOX_ERR_UNSUPPORTED, "spectrum of 2^%d coefficients is too large", n + m);
  }
  return SBOX_OK;
}

int elem_bytes_for(int m) { return m <= 8 ? 1 : (m <= 16 ? 2 : 4); }

size_t f_bytes(int n, int m) {
  // n = 12: room for the sparse words of the fp4 engine (16 inputs a word)
  const size_t nwords = n == 12 ? 256 : (n >= 5 ? ((size_t)1 << (n - 5)) : 1);
  return align256((size_t)m * nwords * 4);
}

constexpr size_t kQueueBytes = 256;  // 64 counters

// n > 16: masks per pass that a workspace of `bytes` allows (0: too small).
long long large_batch_for(int n, int m, size_t bytes) {
  const size_t fixed = kQueueBytes + f_bytes(n, m);
  if (bytes < fixed) return 0;
  const size_t per_mask = ((size_t)4 << n) + 4;
  long long b = (long long)((bytes - fixed - 256) / per_mask);
  const long long M = 1LL << m;
  return std::min(b, M);
}

// 17 <= n <= 20 without a spectrum: the recompute kernel k_walsh_big.
constexpr int kBigMaxGrid = 1024;
bool use_big(int n, int layout) { return n > 16 && n <= 20 && layout == 0; }
size_t big_fixed_bytes(int n, int m) { return kQueueBytes + f_bytes(n, m); }
size_t big_per_wg_bytes(int n) { return (size_t)4 << (n - 5); }
size_t big_bytes(int n, int m) { return big_fixed_bytes(n, m) + kBigMaxGrid * big_per_wg_bytes(n); }

long long default_large_batch(int n, int m) {
  const long long b = std::max(1LL, (1LL << 26) >> n);
  return std::min(b, 1LL << m);
}

size_t large_bytes(int n, int m, long long batch) {
  return kQueueBytes + f_bytes(n, m) + align256(4 * (size_t)batch) + ((size_t)batch << n) * 4;
}

long long inverse_gray(long long j) {
  long long r = 0;
  for (; j; j >>= 1) r ^= j;
  return r;
}

// Butterfly engine of the n = 12 and n = 16 fused maximum: the library
// default is variant 3, the fp4 + fp16 matrix-core kernels; variant 2 the
// fp16 matrix-core kernels after popcount stages, variant 1 the packed
// 16-bit VALU ones, variant 4 (n = 12) an int8 first pass in place of the
// fp4 one (plans run their n = 16 boxes on variant 3 then).
constexpr int kDefaultVariant = 3;
// LDS exchange rounds of the n = 16 matrix-core kernel (2: 64 KiB, 4: 32 KiB per workgroup)
#ifndef SBW_MFMA_ROUNDS
#define SBW_MFMA_ROUNDS 4
#endif
constexpr int kMfmaRounds = SBW_MFMA_ROUNDS;
bool mfma_n(int n) { return n == 12 || n == 16; }
int variant_of(const sbox_tuning* tun) { return (tun && tun->variant) ? tun->variant : kDefaultVariant; }
bool use_mfma(int n, const sbox_tuning* tun) { return mfma_n(n) && variant_of(tun) >= 2; }
// n = 16: variant 2 = fp16 passes after popcount stages, 3 = fp4 + fp16
// passes, whose exchange rounds (4 or 8) tuning.split_p selects
#ifndef SBW_MX_ROUNDS
#define SBW_MX_ROUNDS 4
#endif
// The n = 12 fp4 engine reads sparse words (kWordsFp4).
// The int8 engine (variant 4) reads the same words.
bool fp4_words(int n, const sbox_tuning* tun) { return n == 12 && use_mfma(n, tun) && variant_of(tun) >= 3; }
KFn mfma_kernel(int n, const sbox_tuning* tun) {
  if (n == 12) return variant_of(tun) == 4 ? &k_walsh_i8x12 : variant_of(tun) == 3 ? &k_walsh_mx12 : &k_walsh_mfma12;
  if (variant_of(tun) == 2) return &k_walsh_mfma16<kMfmaRounds>;
  const int rounds = (tun && tun->split_p) ? tun->split_p : SBW_MX_ROUNDS;
  return rounds == 8 ? &k_walsh_mx16<1> : &k_walsh_mx16<2>;
}
// masks a workgroup works on at once (thread groups per item slot)
int mfma_groups(int n) { return n == 16 ? 1 : kWG / 64; }

int mode_of(int layout) { return layout == 1 ? kStoreB : (layout == 2 ? kStoreA : kMax); }

// a-major output of a large spectrum (n <= 16, n + m >= 24): rows of a block
// of masks go through a b-major slab that a tiled transpose turns into columns.
bool use_slab(int n, int m, int layout) { return layout == 2 && n <= 16 && n >= 6 && n + m >= 24; }
// slab of 2^SBW_SLAB_LOG int16 entries (256 MiB by default: measured best for
// 16 x 16 a-major among 2^25 .. 2^30; longer runs per spectrum row than 2^26)
#ifndef SBW_SLAB_LOG
#define SBW_SLAB_LOG 27
#endif
long long slab_rows(int n, int m) { return std::min(1LL << m, std::max(64LL, (1LL << SBW_SLAB_LOG) >> n)); }
size_t slab_bytes(int n, int m) { return align256(((size_t)slab_rows(n, m) << n) * 2); }  // int16 rows
// The route for a permutation beside the slabs where there are two or more
// of them (n = m >= 14; at n = m = 12 the one slab costs about what the
// route's extra launches do), and its workspace: the decision flag and a
// spare NL word, the uint16 inverse table and its bit-sliced words.
bool use_perm_route(int n, int m, int layout) { return use_slab(n, m, layout) && n == m && n >= 14; }
size_t perm_route_bytes(int n) { return 256 + align256(size_t(2) << n) + align256(size_t(n) << (n - 3)); }

// Chunk and grid for a kernel with `groups` thread groups per workgroup over
// `masks` masks per job x `njobs` jobs.
void pick_chunk(long long masks_total, int groups, int grid_cap, int chunk_req, int* chunk, int per_wg = 8) {
  if (chunk_req > 0) {
    *chunk = chunk_req;
    return;
  }
  // about `per_wg` items per workgroup; but a new item rebuilds its first
  // mask from up to m slices while each further mask costs one, so small
  // problems still take up to 4 masks per item as long as every CU gets one
  long long c = masks_total / ((long long)groups * grid_cap * per_wg);
  if (c < 4) {
    int cus = 0;
    if (device_info(&cus) != SBOX_OK || cus < 1) cus = 1;
    c = std::max(c, std::min(4LL, masks_total / ((long long)groups * cus)));
  }
  c = std::max(1LL, std::min(64LL, c));
  *chunk = (int)c;
}

// --------------------------------------------- 17 <= n <= 20, max only ----
template <int L>
const void* big_kernel() { return (const void*)&k_walsh_big<L>; }

sbox_status run_big(const void* S, int n, int m, int eb, int32_t* maxabs, int32_t* nl, void* ws, size_t ws_bytes,
                    const sbox_tuning* tun, hipStream_t st, int* queue) {
  int cus = 0;
  sbox_status s = device_info(&cus);
  if (s) return s;
  const int L = n - 16;
  const int nwords = 1 << (n - 5);
  uint32_t* FT = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + kQueueBytes);
  uint32_t* gbuf = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + big_fixed_bytes(n, m));
  {
    const void* S_ = S;
    int L_ = L, m_ = m, nw_ = nwords;
    void* args[] = {(void*)&S_, &L_, &m_, &FT, &nw_};
    const void* fn = eb == 1 ? (const void*)&k_bitslice_big<1> : eb == 2 ? (const void*)&k_bitslice_big<2>
                                                                         : (const void*)&k_bitslice_big<4>;
    s = launch(fn, dim3((nwords + 255) / 256), dim3(256), args, st);
    if (s) return s;
  }
  const void* fn = L == 1 ? big_kernel<1>() : L == 2 ? big_kernel<2>() : L == 3 ? big_kernel<3>() : big_kernel<4>();
  int occ = 1;
  s = occupancy(fn, &occ);
  if (s) return s;
  const long long M = 1LL << m;
  long long grid = (tun && tun->grid) ? tun->grid : (long long)occ * cus;
  grid = std::min<long long>(grid, kBigMaxGrid);
  grid = std::min<long long>(grid, (long long)((ws_bytes - big_fixed_bytes(n, m)) / big_per_wg_bytes(n)));
  int chunk = (tun && tun->chunk) ? tun->chunk : (int)std::max(1LL, std::min(16LL, M / (grid * 16)));
  BigParams bp{};
  bp.FT = FT;
  bp.gbuf = gbuf;
  bp.maxabs = maxabs;
  bp.nl = nl;
  bp.queue = queue;
  bp.total_items = (M + chunk - 1) / chunk;
  bp.m = m;
  bp.chunk = chunk;
  grid = std::min<long long>(grid, bp.total_items);
  void* args[] = {&bp};
  return launch(fn, dim3((unsigned)grid), dim3(kWG), args, st);
}

// One transform launch over all 2^m masks of a single box (n <= 16): the
// matrix-core kernel for the plain maximum where it is the default (or the
// tuning asks for it), else k_walsh in `mode`.  `kp` carries the caller's
// fields (histogram, gate) in and the launched configuration out.
sbox_status launch_transform(const JobDesc& jd, int mode, const sbox_tuning* tun, int cus, int* queue,
                             hipStream_t st, KParams* kp) {
  const int n = jd.n;
  const void* fn = nullptr;
  int groups = 1;
  if (mode == kMax && use_mfma(n, tun)) {
    fn = (const void*)mfma_kernel(n, tun);
    groups = mfma_groups(n);
  } else {
    const int p = (tun && tun->split_p) ? tun->split_p : default_split(n);
    if (n > 8 && !split_valid(n, p)) return fail(SBOX_ERR_INVALID_ARG, "split_p=%d invalid for n=%d", p, n);
    fn = (const void*)lookup_kernel(n, n <= 8 ? n : p, mode);
    if (!fn) return fail(SBOX_ERR_INVALID_ARG, "no kernel for n=%d split_p=%d mode=%d", n, p, mode);
    groups = kWG >> (n <= 8 ? 0 : n - p);
  }
  int occ = 1;
  sbox_status s = occupancy(fn, &occ);
  if (s) return s;
  const long long M = 1LL << jd.m;
  const int grid_cap = (tun && tun->grid) ? tun->grid : occ * cus;
  int chunk = 1;
  // a spectrum store evens out better over more, shorter items (16x16
  // b-major: 2.81 / 2.73 / 2.65 ms at 8 / 16 / 32 items per workgroup)
  const int per_wg = (mode == kStoreB || mode == kStoreA) ? 32 : 8;
  pick_chunk(M, groups, grid_cap, tun ? tun->chunk : 0, &chunk, per_wg);
  const long long per_item = (long long)groups * chunk;
  kp->jobs = nullptr;
  kp->job0 = jd;
  kp->njobs = 1;
  kp->chunk = chunk;
  kp->queue = queue;
  kp->total_items = (M + per_item - 1) / per_item;
  const int grid = (int)std::min<long long>(grid_cap, kp->total_items);
  void* args[] = {kp};
  return launch(fn, dim3(grid), dim3(kWG), args, st);
}

// ------------------------------------------------------- one S-box call ----
sbox_status run_single(const void* S, int n, int m, int eb, int32_t* maxabs, int32_t* nl, int32_t* spec,
                       int layout_arg, void* ws, size_t ws_bytes, const sbox_tuning* tun, hipStream_t st,
                       unsigned long long* hist = nullptr, unsigned long long* hist_over = nullptr) {
  const int layout = base_layout(layout_arg);
  const int wscale = wscale_of(layout_arg);
  int cus = 0;
  sbox_status s = device_info(&cus);
  if (s) return s;
  int* queue = reinterpret_cast<int*>(ws);
  uint32_t* F = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) + kQueueBytes);
  const bool sparse = layout == 0 && !hist && fp4_words(n, tun);
  const int nwords = sparse ? 256 : (n >= 5 ? 1 << (n - 5) : 1);

  if (use_big(n, layout)) {
    // init (NL, maxabs[0], queue), then the x_hi-inner bit-slicing and the kernel
    JobDesc jd{};
    jd.maxabs = maxabs;
    jd.nl = nl;
    jd.n = n;
    jd.m = m;
    jd.wscale = -2;
    const JobDesc* nulljobs = nullptr;
    int one = 1, nq = 64, lay = 0;
    void* args[] = {(void*)&nulljobs, &jd, &one, &queue, &nq, &lay};
    s = launch((const void*)&k_init_jobs, dim3(1), dim3(256), args, st);
    if (s) return s;
    return run_big(S, n, m, eb, maxabs, nl, ws, ws_bytes, tun, st, queue);
  }
  JobDesc jd{};
  jd.S = S;
  jd.F = F;
  jd.maxabs = maxabs;
  jd.nl = nl;
  jd.spec = spec;
  jd.item_begin = 0;
  jd.n = n;
  jd.m = m;
  jd.nwords = nwords;
  jd.s_elem_bytes = eb;
  jd.wscale = wscale;
  jd.flags = sparse ? kWordsFp4 : 0;
  if (n >= 6 && n <= 8 && m <= 8 && !hist) {
    // the transform is one workgroup (a thread a mask), which prepares the
    // box itself: the call is one launch
    jd.flags |= kPrepInline;
  } else {
    // one launch: start values (queue counters, NL, maxabs[0], b = 0 spectrum
    // row) in workgroup 0, bit-sliced component words in the others
    int nq = 64, lay = layout;
    void* args[] = {&jd, &queue, &nq, &lay};
    const void* fn = eb == 1 ? (const void*)&k_prep_single<1> : eb == 2 ? (const void*)&k_prep_single<2>
                                                                        : (const void*)&k_prep_single<4>;
    const long long units = (n >= 6 && !sparse) ? (1LL << n) : nwords;  // entries (a wave per 64) or words
    s = launch(fn, dim3((unsigned)(1 + (units + 255) / 256)), dim3(256), args, st);
    if (s) return s;
  }

  if (n <= 16 && use_slab(n, m, layout)) {
    // A box with n = m may be a permutation: then its a-major matrix is the
    // b-major matrix of the inverse map, written without slabs.  The device
    // decides (*bij); the launches of the route not taken return at once.
    const int* bij = nullptr;
    int qi = 1;
    if (use_perm_route(n, m, layout)) {
      char* extra = reinterpret_cast<char*>(ws) + kQueueBytes + f_bytes(n, m) + slab_bytes(n, m);
      int* flag = reinterpret_cast<int*>(extra);
      int32_t* spare_nl = flag + 1;
      uint16_t* inv = reinterpret_cast<uint16_t*>(extra + 256);
      uint32_t* Finv = reinterpret_cast<uint32_t*>(extra + 256 + align256(size_t(2) << n));
      const void* S_ = S;
      int n_ = n;
      {
        void* args[] = {(void*)&S_, &n_, &inv, &flag};
        const void* fn = eb == 1 ? (const void*)&k_perm_scatter<1> : eb == 2 ? (const void*)&k_perm_scatter<2>
                                                                             : (const void*)&k_perm_scatter<4>;
        s = launch(fn, dim3((unsigned)(((1LL << n) + 255) / 256)), dim3(256), args, st);
        if (s) return s;
      }
      JobDesc ji{};
      ji.S = inv;
      ji.F = Finv;
      ji.maxabs = nullptr;
      ji.nl = maxabs ? spare_nl : nl;  // NL(S^-1) = NL(S) for a permutation
      ji.spec = spec;
      ji.n = n;
      ji.m = m;
      ji.nwords = 1 << (n - 5);
      ji.s_elem_bytes = 2;
      ji.wscale = wscale;
      {
        int* noq = nullptr;
        int nq = 0;
        void* args[] = {(void*)&S_, &ji, &flag, &noq, &nq};
        const void* fn = eb == 1 ? (const void*)&k_perm_check_prep<1> : eb == 2 ? (const void*)&k_perm_check_prep<2>
                                                                                 : (const void*)&k_perm_check_prep<4>;
        s = launch(fn, dim3((unsigned)(1 + ((1LL << n) + 255) / 256)), dim3(256), args, st);
        if (s) return s;
      }
      // for a permutation: the maxima of S per mask b (if asked for) from the
      // fused kernel, and the rows of S^-1 with the NL
      if (maxabs) {
        KParams kp{};
        kp.gate = flag;
        kp.gate_run = 1;
        s = launch_transform(jd, kMax, tun, cus, queue + 1, st, &kp);
        if (s) return s;
      }
      sbox_tuning tb = tun ? *tun : sbox_tuning{};
      tb.split_p = 0;  // the store modes exist for the default split only
      KParams kp{};
      kp.gate = flag;
      kp.gate_run = 1;
      s = launch_transform(ji, kStoreB, &tb, cus, queue + 2, st, &kp);
      if (s) return s;
      bij = flag;
      qi = 3;
    }
    // b-major rows of each aligned block of masks into the slab, then transpose
    const int p = default_split(n);
    KFn fn = lookup_kernel(n, p, kSlab16);
    if (!fn) return fail(SBOX_ERR_INVALID_ARG, "no kernel for n=%d", n);
    int occ = 1;
    s = occupancy((const void*)fn, &occ);
    if (s) return s;
    const int Q = n <= 8 ? 0 : n - p;
    const int groups = kWG >> Q;
    const long long rows = slab_rows(n, m);
    int32_t* slab = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) + kQueueBytes + f_bytes(n, m));
    const int grid_cap = (tun && tun->grid) ? tun->grid : occ * cus;
    int chunk = 1;
    pick_chunk(rows, groups, grid_cap, tun ? tun->chunk : 0, &chunk);
    const long long per_item = (long long)groups * chunk;
    const long long M = 1LL << m;
    for (long long b0 = 0; b0 < M; b0 += rows, ++qi) {
      if (qi >= 64) {
        int* q = queue + 1;
        long long cnt = 63;
        void* za[] = {&q, &cnt};
        s = launch((const void*)&k_zero, dim3(1), dim3(256), za, st);
        if (s) return s;
        qi = 1;
      }
      // Gray indices [g^-1(j) R, g^-1(j) R + R) visit exactly the masks
      // [j R, j R + R): the Gray code maps index block i onto mask block gray(i).
      KParams kp{};
      kp.job0 = jd;
      kp.job0.spec = slab;
      kp.njobs = 1;
      kp.chunk = chunk;
      kp.queue = queue + qi;
      kp.kbase = inverse_gray(b0 / rows) * rows;
      kp.kcount = rows;
      kp.row0 = b0;
      kp.rows = rows;
      kp.total_items = (rows + per_item - 1) / per_item;
      kp.gate = bij;
      kp.gate_run = 0;
      const int grid = (int)std::min<long long>(grid_cap, kp.total_items);
      void* args[] = {&kp};
      s = launch((const void*)fn, dim3(grid), dim3(kWG), args, st);
      if (s) return s;
      int n_ = n, m_ = m, B_ = (int)rows, wsc = jd.wscale, eb_ = jd.s_elem_bytes;
      long long b0_ = b0;
      const int16_t* slab_ = reinterpret_cast<const int16_t*>(slab);
      const void* S_ = jd.S;
      void* targs[] = {(void*)&slab_, &n_, &spec, &m_, &b0_, &B_, &wsc, (void*)&S_, &eb_, (void*)&bij};
      s = launch((const void*)&k_transpose_slab16,
                 dim3((unsigned)(((1LL << n) + 127) / 128), (unsigned)((rows + 63) / 64)), dim3(256), targs, st);
      if (s) return s;
    }
    return SBOX_OK;
  }

  if (layout == 0 && hist && n == 16 && use_mfma(n, tun)) {
    // |W| histogram at n = 16 on the fp4 + fp16 matrix-core transform (LDS
    // bins below kMxHistBins - 1), then the large-value pass for the rest.
    // Eight exchange rounds: with four, the counting spills registers.
    const void* fn = (const void*)&k_walsh_mx16<1, true>;
    int occ = 1;
    s = occupancy(fn, &occ);
    if (s) return s;
    const long long M = 1LL << m;
    const int grid_cap = (tun && tun->grid) ? tun->grid : occ * cus;
    int chunk = 1;
    pick_chunk(M, mfma_groups(n), grid_cap, tun ? tun->chunk : 0, &chunk);
    KParams kp{};
    kp.job0 = jd;
    kp.njobs = 1;
    kp.chunk = chunk;
    kp.queue = queue;
    kp.total_items = (M + chunk - 1) / chunk;
    kp.hist = hist;
    kp.hist_over = hist_over;
    const int grid = (int)std::min<long long>(grid_cap, kp.total_items);
    void* args[] = {&kp};
    s = launch(fn, dim3(grid), dim3(kWG), args, st);
    if (s) return s;
    // the VALU kernel's large-value pass: one thread group per workgroup at
    // n = 16 as well, so the same items cover the same masks
    KFn fnb = lookup_kernel(16, 8, kHistBig);
    if (!fnb) return fail(SBOX_ERR_INVALID_ARG, "no histogram kernel for n=16");
    int occb = 1;
    s = occupancy((const void*)fnb, &occb);
    if (s) return s;
    kp.queue = queue + 1;
    kp.hist_cut = kMxHistBins - 1;
    const int gridb = (int)std::min<long long>((long long)occb * cus, kp.total_items);
    void* argsb[] = {&kp};
    return launch((const void*)fnb, dim3(gridb), dim3(kWG), argsb, st);
  }

  if (n <= 16) {
    KParams kp{};
    kp.hist = hist;
    kp.hist_over = hist_over;
    s = launch_transform(jd, hist ? (int)kHist : mode_of(layout), tun, cus, queue, st, &kp);
    if (s || !hist) return s;
    // the pass for |W|/2 >= kHistBins - 1 (returns at once when there is none)
    const int p = (tun && tun->split_p) ? tun->split_p : default_split(n);
    KFn fnb = lookup_kernel(n, n <= 8 ? n : p, kHistBig);
    if (!fnb) return fail(SBOX_ERR_INVALID_ARG, "no histogram kernel for n=%d", n);
    int occb = 1;
    s = occupancy((const void*)fnb, &occb);
    if (s) return s;
    kp.queue = queue + 1;
    kp.hist_cut = kHistBins - 1;
    const int gridb = (int)std::min<long long>((long long)occb * cus, kp.total_items);
    void* argsb[] = {&kp};
    return launch((const void*)fnb, dim3(gridb), dim3(kWG), argsb, st);
  }

  // ---- n > 16: 2^16-point block transforms, then the block-index stages
  const long long M = 1LL << m;
  long long batch = large_batch_for(n, m, ws_bytes);
  if (batch < 1) return fail(SBOX_ERR_WORKSPACE, "workspace too small for n=%d", n);
  char* base = reinterpret_cast<char*>(ws) + kQueueBytes + f_bytes(n, m);
  int* slotmax = reinterpret_cast<int*>(base);
  int32_t* T = reinterpret_cast<int32_t*>(base + align256(4 * (size_t)batch));
  KFn fnA = lookup_kernel(16, 8, kBlock);
  int occ = 1;
  s = occupancy((const void*)fnA, &occ);
  if (s) return s;
  const int L = n - 16;
  const int chunk = (tun && tun->chunk) ? tun->chunk : 4;
  const int grid_cap = (tun && tun->grid) ? tun->grid : occ * cus;
  for (long long kbase = 0; kbase < M; kbase += batch) {
    const long long kcount = std::min(batch, M - kbase);
    // zero this pass's counter and per-mask maxima
    {
      int* q1 = queue + 1;
      long long one = 1;
      void* a1[] = {&q1, &one};
      s = launch((const void*)&k_zero, dim3(1), dim3(256), a1, st);
      if (s) return s;
      long long cnt = kcount;
      void* a2[] = {&slotmax, &cnt};
      s = launch((const void*)&k_zero, dim3((unsigned)std::min<long long>(1024, (kcount + 255) / 256)), dim3(256), a2, st);
      if (s) return s;
    }
    KParams kp{};
    kp.job0 = jd;
    kp.njobs = 1;
    kp.chunk = chunk;
    kp.queue = queue + 1;
    kp.total_items = ((kcount + chunk - 1) / chunk) << L;
    kp.blockout = T;
    kp.kbase = kbase;
    kp.kcount = kcount;
    kp.nblk_log = L;
    {
      const int grid = (int)std::min<long long>(grid_cap, kp.total_items);
      void* args[] = {&kp};
      s = launch((const void*)fnA, dim3(grid), dim3(kWG), args, st);
      if (s) return s;
    }
    // block-index stages, up to 4 bits per pass
    int bit0 = 0;
    while (bit0 < L) {
      const int r = std::min(4, L - bit0);
      const bool last = bit0 + r == L;
      const long long threads = kcount * ((1LL << 16) << (L - r));
      const unsigned blocks = (unsigned)((threads + 255) / 256);
      int32_t* spec_ = spec;
      int lay = layout, ws_ = wscale, m_ = m, L_ = L, b0 = bit0;
      long long kc = kcount, kb = kbase, mend = M;
      void* args[] = {&T, &kc, &L_, &b0, &slotmax, &spec_, &lay, &ws_, &m_, &kb, &mend};
      const void* fn = nullptr;
      if (last) {
        fn = r == 1 ? (const void*)&k_combine<1, true> : r == 2 ? (const void*)&k_combine<2, true>
           : r == 3 ? (const void*)&k_combine<3, true> : (const void*)&k_combine<4, true>;
      } else {
        fn = (const void*)&k_combine<4, false>;
      }
      s = launch(fn, dim3(blocks), dim3(256), args, st);
      if (s) return s;
      bit0 += r;
    }
    {
      long long kc = kcount, kb = kbase, mend = M;
      int n_ = n;
      int32_t* mx = maxabs;
      int32_t* nl_ = nl;
      void* args[] = {&slotmax, &kc, &kb, &mend, &n_, &mx, &nl_};
      s = launch((const void*)&k_finalize_batch, dim3((unsigned)((kcount + 255) / 256)), dim3(256), args, st);
      if (s) return s;
    }
  }
  return SBOX_OK;
}

// --------------------------------------------------------------- batches ---
struct ClassLaunch {
  int n, layout;
  KFn fn;
  int njobs;
  size_t desc_off;  // byte offset of this class's JobDesc table in the descriptor area
  int chunk;
  long long total_items;
  int grid;
};

struct BatchLayout {
  int count = 0;
  size_t desc_bytes = 0;   // all JobDesc tables
  size_t f_total = 0;      // all bit-sliced words
  size_t ws_bytes = 0;     // queue + descs + F
  std::vector<JobDesc> descs;  // host copy, F pointers relative to the F area (filled at bind)
  std::vector<size_t> f_off;   // per desc, offset inside the F area
  std::vector<ClassLaunch> classes;
};

sbox_status check_job(const sbox_job& j, int idx) {
  if (!j.S || !j.nl) return fail(SBOX_ERR_INVALID_ARG, "job %d: null S or nl", idx);
  if (j.s_elem_bytes != 1 && j.s_elem_bytes != 2 && j.s_elem_bytes != 4)
    return fail(SBOX_ERR_INVALID_ARG, "job %d: s_elem_bytes must be 1, 2 or 4", idx);
  sbox_status s = check_nm(j.n, j.m);
  if (s) return s;
  if (j.n > 16) return fail(SBOX_ERR_UNSUPPORTED, "job %d: batched boxes need n <= 16 (n=%d)", idx, j.n);
  return check_layout(j.layout, j.n, j.m, j.spectrum);
}

sbox_status plan_batch(const sbox_job* jobs, int count, const sbox_tuning* tun, BatchLayout* out) {
  if (count < 0 || (count > 0 && !jobs)) return fail(SBOX_ERR_INVALID_ARG, "bad job array");
  if (count > (1 << 20)) return fail(SBOX_ERR_UNSUPPORTED, "too many jobs (%d)", count);
  for (int i = 0; i < count; ++i) {
    sbox_status s = check_job(jobs[i], i);
    if (s) return s;
  }
  int cus = 0;
  sbox_status s = device_info(&cus);
  if (s) return s;
  BatchLayout L;
  L.count = count;
  // classes keyed by (n desc, layout); jobs inside by descending m (largest work first)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (jobs[a].n != jobs[b].n) return jobs[a].n > jobs[b].n;
    if (jobs[a].layout != jobs[b].layout) return jobs[a].layout < jobs[b].layout;
    return jobs[a].m > jobs[b].m;
  });
  size_t f_off = 0;
  int i = 0;
  while (i < count) {
    const int n = jobs[order[i]].n, layout = jobs[order[i]].layout;
    int jend = i;
    while (jend < count && jobs[order[jend]].n == n && jobs[order[jend]].layout == layout) ++jend;
    ClassLaunch c{};
    c.n = n;
    c.layout = layout;
    const bool mc = layout == 0 && use_mfma(n, tun);
    const int p = (tun && tun->split_p && n > 8 && !mc) ? tun->split_p : default_split(n);
    if (n > 8 && !split_valid(n, p)) return fail(SBOX_ERR_INVALID_ARG, "split_p=%d invalid for n=%d", p, n);
    c.fn = mc ? mfma_kernel(n, tun) : lookup_kernel(n, p, mode_of(base_layout(layout)));
    if (!c.fn) return fail(SBOX_ERR_INVALID_ARG, "no kernel for n=%d split_p=%d layout=%d", n, p, layout);
    int occ = 1;
    s = occupancy((const void*)c.fn, &occ);
    if (s) return s;
    const int Q = n <= 8 ? 0 : n - p;
    const int groups = mc ? mfma_groups(n) : kWG >> Q;
    const int grid_cap = (tun && tun->grid) ? tun->grid : occ * cus;
    long long masks_total = 0;
    for (int k = i; k < jend; ++k) masks_total += 1LL << jobs[order[k]].m;
    pick_chunk(masks_total, groups, grid_cap, tun ? tun->chunk : 0, &c.chunk);
    if (!(tun && tun->chunk) && n > 8 && jend - i >= 32) {
      // a class of many boxes: long items (128 masks per group, a power of two
      // so items tile every box's 2^m masks) as long as the queue still holds
      // an item for every workgroup; each item rebuilds its first mask from up
      // to m slices and takes a queue atomic and a job search (n = 10 class of
      // the 4096-box mix: 0.39 -> 0.21 ms, n = 12: 1.10 -> 0.96 ms; the whole
      // batch at 16 / 32 / 64 / 128 masks: 0.847 / 0.819 / 0.804 / 0.791 ms).
      // A few large boxes keep the balance rule: long items leave a tail there.
      int cb = 128;
      while (cb > 4 && masks_total / ((long long)groups * cb) < grid_cap) cb >>= 1;
      c.chunk = cb;
    }
    c.njobs = jend - i;
    c.desc_off = L.descs.size() * sizeof(JobDesc);
    long long items = 0;
    for (int k = i; k < jend; ++k) {
      const sbox_job& j = jobs[order[k]];
      JobDesc d{};
      d.S = j.S;
      d.maxabs = j.maxabs_per_b;
      d.nl = j.nl;
      d.spec = j.layout ? j.spectrum : nullptr;
      d.item_begin = items;
      d.n = j.n;
      d.m = j.m;
      const bool sparse = mc && fp4_words(j.n, tun);
      d.nwords = sparse ? 256 : (j.n >= 5 ? 1 << (j.n - 5) : 1);
      d.flags = (sparse ? kWordsFp4 : 0) | (base_layout(j.layout) == 2 ? kSpecAMajor : 0);
      d.s_elem_bytes = j.s_elem_bytes;
      d.wscale = wscale_of(j.layout);
      const long long per_item = (long long)groups * c.chunk;
      items += ((1LL << j.m) + per_item - 1) / per_item;
      L.descs.push_back(d);
      L.f_off.push_back(f_off);
      f_off += f_bytes(j.n, j.m);
    }
    c.total_items = items;
    if (items >= (1LL << 31)) return fail(SBOX_ERR_UNSUPPORTED, "batch too large");
    c.grid = (int)std::min<long long>(grid_cap, items);
    L.classes.push_back(c);
    i = jend;
  }
  if (L.classes.size() > 60) return fail(SBOX_ERR_UNSUPPORTED, "too many size classes");
  L.desc_bytes = align256(L.descs.size() * sizeof(JobDesc));
  L.f_total = f_off;
  L.ws_bytes = kQueueBytes + L.desc_bytes + L.f_total;
  *out = std::move(L);
  return SBOX_OK;
}

// Fill F pointers for a workspace at `ws` (descs are copied to ws + kQueueBytes).
void bind_batch(BatchLayout& L, void* ws) {
  char* fbase = reinterpret_cast<char*>(ws) + kQueueBytes + L.desc_bytes;
  for (size_t k = 0; k < L.descs.size(); ++k) L.descs[k].F = reinterpret_cast<const uint32_t*>(fbase + L.f_off[k]);
}

// Streams and events a plan owns so that its size classes run side by side:
// class 0 (the largest n, launched first) stays on the caller's stream, class
// c >= 1 runs on side[c - 1] after `fork` and is joined back through
// join[c - 1].  Streams keep the default priority.
struct ClassStreams {
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
};

sbox_status launch_batch(const BatchLayout& L, void* ws, hipStream_t st, const ClassStreams* cs = nullptr) {
  if (L.count == 0) return SBOX_OK;
  int* queue = reinterpret_cast<int*>(ws);
  const JobDesc* dtab = reinterpret_cast<const JobDesc*>(reinterpret_cast<char*>(ws) + kQueueBytes);
  sbox_status s;
  // bit-slice every table and set every job's start values (grid.y <= 65535
  // jobs per launch; the first launch also zeroes the queue counters): waves
  // of 64 threads striding over a job's words, one per 256 words of the
  // largest job (one up to n = 13); idle workgroups would only cost dispatch
  // time.  (One launch where there were a bit-slicing launch, an init launch
  // per size class and a counter reset.)
  int maxw = 1;
  for (const JobDesc& jd : L.descs) maxw = std::max(maxw, jd.nwords);
  const unsigned gx = (unsigned)std::min(32, (maxw + 255) / 256);
  for (int j0 = 0; j0 < L.count; j0 += 65535) {
    const int nj = std::min(65535, L.count - j0);
    const JobDesc* d = dtab + j0;
    int nq = j0 == 0 ? 64 : 0;
    void* args[] = {(void*)&d, &queue, &nq};
    s = launch((const void*)&k_prep_jobs, dim3(gx, nj), dim3(64), args, st);
    if (s) return s;
  }
  const bool fork = cs && L.classes.size() > 1 && cs->side.size() + 1 >= L.classes.size();
  if (fork) HIP_TRY(hipEventRecord(cs->fork, st));
  int ci = 0;
  for (const ClassLaunch& c : L.classes) {
    KParams kp{};
    kp.jobs = reinterpret_cast<const JobDesc*>(reinterpret_cast<const char*>(dtab) + c.desc_off);
    kp.njobs = c.njobs;
    kp.chunk = c.chunk;
    kp.queue = queue + ci;
    kp.total_items = c.total_items;
    void* args[] = {&kp};
    hipStream_t cst = st;
    if (fork && ci > 0) {
      cst = cs->side[ci - 1];
      HIP_TRY(hipStreamWaitEvent(cst, cs->fork, 0));
    }
    s = launch((const void*)c.fn, dim3(c.grid), dim3(kWG), args, cst);
    if (s) return s;
    if (fork && ci > 0) {
      HIP_TRY(hipEventRecord(cs->join[ci - 1], cst));
      HIP_TRY(hipStreamWaitEvent(st, cs->join[ci - 1], 0));
    }
    ++ci;
  }
  return SBOX_OK;
}

// ------------------------------------------------- pinned staging blocks ---
// sbox_walsh_nl_batched copies its descriptor table to the device from a
// pinned block; a block is taken again only once the event recorded after
// its copy has completed, so calls on different streams never wait on each
// other on the host (only when every block of the pool is still in flight).
struct StageBlock {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t evt = nullptr;
  int dev = -1;
};
constexpr size_t kStageMaxBlocks = 32;
constexpr size_t kStageMinBytes = 64 << 10;
std::mutex g_stage_mu;
std::vector<StageBlock> g_stage;

// A block of at least `bytes` on device `dev` whose last copy has finished
// (waits only when all kStageMaxBlocks blocks are in flight).
sbox_status acquire_stage(int dev, size_t bytes, StageBlock** out) {
  StageBlock* fit = nullptr;    // free and large enough
  StageBlock* spare = nullptr;  // free but too small (replaced when the pool is full)
  size_t mine = 0;
  for (StageBlock& b : g_stage) {
    if (b.dev != dev) continue;
    ++mine;
    const hipError_t q = hipEventQuery(b.evt);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(SBOX_ERR_HIP, "hipEventQuery: %s", hipGetErrorString(q));
    if (b.bytes >= bytes && (!fit || b.bytes < fit->bytes)) fit = &b;
    if (b.bytes < bytes) spare = &b;
  }
  if (!fit && mine >= kStageMaxBlocks) {
    if (!spare) {  // every block is in flight: wait for one of them
      for (StageBlock& b : g_stage)
        if (b.dev == dev) {
          spare = &b;
          break;
        }
      HIP_TRY(hipEventSynchronize(spare->evt));
    }
    if (spare->bytes >= bytes) {
      fit = spare;
    } else {
      HIP_TRY(hipHostFree(spare->host));
      spare->host = nullptr;
      spare->bytes = 0;
      HIP_TRY(hipHostMalloc(&spare->host, std::max(bytes, kStageMinBytes), hipHostMallocDefault));
      spare->bytes = std::max(bytes, kStageMinBytes);
      fit = spare;
    }
  }
  if (!fit) {
    StageBlock b;
    b.dev = dev;
    b.bytes = std::max(bytes, kStageMinBytes);
    HIP_TRY(hipHostMalloc(&b.host, b.bytes, hipHostMallocDefault));
    const hipError_t e = hipEventCreateWithFlags(&b.evt, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipHostFree(b.host);
      return fail(SBOX_ERR_HIP, "hipEventCreateWithFlags: %s", hipGetErrorString(e));
    }
    g_stage.push_back(b);
    fit = &g_stage.back();
  }
  *out = fit;
  return SBOX_OK;
}

sbox_status refuse_capture(hipStream_t st, const char* what) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(SBOX_ERR_INVALID_ARG, "%s cannot be captured into a graph (%s)", what,
                cs == hipStreamCaptureStatusActive ? "the stream is capturing" : "the capture was invalidated");
  return SBOX_OK;
}

// ---------------------------------------- short-form scratch per stream ---
// sbox_walsh_nl takes its scratch (queue counters, bit-sliced words) from a
// buffer reserved ahead of time for its (device, stream) pair; it never
// allocates, and calls on different streams never share scratch.
struct StreamScratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, uintptr_t>, StreamScratch> g_scratch;

// ------------------------------------- static scratch (no allocation) ---
// The scratch of sbox_walsh_nl_static: queue counters and bit-sliced words,
// at most 256 + 24 * 2^13 bytes for n <= 16, m <= 24.  It is part of the
// library's device image, so every GPU holds its own copy from load until
// the process ends.  Host code never uses the name as an address: the
// device address is looked up per GPU (static_scratch_ptr) and passed on.
constexpr size_t kStaticScratchBytes = size_t(256) << 10;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
std::map<int, void*> g_static_ptr;  // device ordinal -> that GPU's copy of `scratch`

// Address of `scratch` on the current device (hipGetSymbolAddress once per
// device, with that device current).
sbox_status static_scratch_ptr(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_static_mu);
  auto it = g_static_ptr.find(dev);
  if (it == g_static_ptr.end()) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    it = g_static_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return SBOX_OK;
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

const char* sbox_last_error(void) { return g_last_error.c_str(); }

const char* sbox_version(void) { return "1.1.0"; }

size_t sbox_walsh_nl_workspace_bytes(int n, int m, int layout) {
  if (n < 1 || n > 24 || m < 1 || m > 24 || n + m > 40) return 0;
  if (!layout_valid(layout)) return 0;
  layout = base_layout(layout);
  if (layout != 0 && n + m > 34) return 0;
  if (n <= 16)
    return kQueueBytes + f_bytes(n, m) + (use_slab(n, m, layout) ? slab_bytes(n, m) : 0) +
           (use_perm_route(n, m, layout) ? perm_route_bytes(n) : 0);
  if (use_big(n, layout)) return big_bytes(n, m);
  return large_bytes(n, m, default_large_batch(n, m));
}

sbox_status sbox_walsh_nl_ex(const void* S, int n, int m, int s_elem_bytes, int32_t* maxabs_per_b,
                             int32_t* nl, int32_t* spectrum, int layout, void* workspace,
                             size_t workspace_bytes, const sbox_tuning* tuning, void* stream) {
  sbox_status s = check_nm(n, m);
  if (s) return s;
  if (!S) return fail(SBOX_ERR_INVALID_ARG, "S is null");
  if (!nl) return fail(SBOX_ERR_INVALID_ARG, "nl is null");
  if (s_elem_bytes != 1 && s_elem_bytes != 2 && s_elem_bytes != 4)
    return fail(SBOX_ERR_INVALID_ARG, "s_elem_bytes must be 1, 2 or 4 (got %d)", s_elem_bytes);
  s = check_layout(layout, n, m, spectrum);
  if (s) return s;
  if (tuning) {
    if (tuning->chunk < 0 || tuning->grid < 0 || tuning->split_p < 0)
      return fail(SBOX_ERR_INVALID_ARG, "negative tuning field");
    if (tuning->variant < 0 || tuning->variant > 4)
      return fail(SBOX_ERR_INVALID_ARG, "tuning variant %d (0 to 4)", tuning->variant);
    if (tuning->variant == 2 && !(mfma_n(n) && layout == 0))
      return fail(SBOX_ERR_INVALID_ARG, "the matrix-core variant covers n = 12 and 16 without a spectrum only");
    if (tuning->variant == 3 && !(mfma_n(n) && layout == 0))
      return fail(SBOX_ERR_INVALID_ARG, "the fp4 matrix-core variant covers n = 12 and 16 without a spectrum only");
    if (tuning->variant == 4 && !(n == 12 && layout == 0))
      return fail(SBOX_ERR_INVALID_ARG, "the int8 matrix-core variant covers n = 12 without a spectrum only");
    if (tuning->variant == 3 && n == 16 && tuning->split_p && tuning->split_p != 4 && tuning->split_p != 8)
      return fail(SBOX_ERR_INVALID_ARG, "the fp4 matrix-core variant takes split_p = 4 or 8 exchange rounds");
    if (tuning->split_p && n > 8 && n <= 16 && !(tuning->variant >= 2 && mfma_n(n) && layout == 0) &&
        !split_valid(n, tuning->split_p))
      return fail(SBOX_ERR_INVALID_ARG, "split_p=%d invalid for n=%d", tuning->split_p, n);
    if (tuning->split_p && n <= 16 && n > 8 && layout != 0 && tuning->split_p != default_split(n))
      return fail(SBOX_ERR_INVALID_ARG, "spectrum output uses split_p=%d for n=%d", default_split(n), n);
  }
  const size_t need = sbox_walsh_nl_workspace_bytes(n, m, layout);
  if (!workspace) return fail(SBOX_ERR_WORKSPACE, "workspace is null (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(SBOX_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (n <= 16 && workspace_bytes < need)
    return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, need);
  if (use_big(n, layout)) {
    if (workspace_bytes < big_fixed_bytes(n, m) + big_per_wg_bytes(n))
      return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes too small for n=%d (need >= %zu)", workspace_bytes, n,
                  big_fixed_bytes(n, m) + big_per_wg_bytes(n));
  } else if (n > 16 && large_batch_for(n, m, workspace_bytes) < 1)
    return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes too small for n=%d (need >= %zu)", workspace_bytes, n,
                large_bytes(n, m, 1));
  return run_single(S, n, m, s_elem_bytes, maxabs_per_b, nl, spectrum, layout, workspace, workspace_bytes,
                    tuning, reinterpret_cast<hipStream_t>(stream));
}

size_t sbox_walsh_nl_static_max_bytes(void) { return kStaticScratchBytes; }

sbox_status sbox_walsh_nl_static(const void* S, int n, int m, int s_elem_bytes, int32_t* maxabs_per_b, int32_t* nl,
                                 int32_t* spectrum, int layout, void* stream) {
  sbox_status s = check_nm(n, m);
  if (s) return s;
  const size_t need = sbox_walsh_nl_workspace_bytes(n, m, layout);
  if (need == 0)  // the full form names what is wrong (layout, spectrum size)
    return sbox_walsh_nl_ex(S, n, m, s_elem_bytes, maxabs_per_b, nl, spectrum, layout, nullptr, 0, nullptr, stream);
  if (need > kStaticScratchBytes)
    return fail(SBOX_ERR_WORKSPACE,
                "n=%d m=%d layout=%d needs %zu bytes of scratch; the static array holds %zu "
                "(n <= 16, and no a-major spectrum with n + m >= 24)",
                n, m, layout, need, kStaticScratchBytes);
  void* ws = nullptr;
  s = static_scratch_ptr(&ws);
  if (s) return s;
  return sbox_walsh_nl_ex(S, n, m, s_elem_bytes, maxabs_per_b, nl, spectrum, layout, ws, kStaticScratchBytes,
                          nullptr, stream);
}

size_t sbox_walsh_histogram_workspace_bytes(int n, int m) {
  if (n < 1 || n > 16 || m < 1 || m > 24) return 0;
  return sbox_walsh_nl_workspace_bytes(n, m, 0) + 256;  // + the large-value count and an NL slot
}

sbox_status sbox_walsh_histogram(const void* S, int n, int m, int s_elem_bytes, uint64_t* hist,
                                 int32_t* maxabs_per_b, int32_t* nl, void* workspace, size_t workspace_bytes,
                                 void* stream) {
  sbox_status s = check_nm(n, m);
  if (s) return s;
  if (n > 16) return fail(SBOX_ERR_UNSUPPORTED, "the |W| histogram needs n <= 16 (n=%d)", n);
  if (!S || !hist) return fail(SBOX_ERR_INVALID_ARG, "S or hist is null");
  if (s_elem_bytes != 1 && s_elem_bytes != 2 && s_elem_bytes != 4)
    return fail(SBOX_ERR_INVALID_ARG, "s_elem_bytes must be 1, 2 or 4 (got %d)", s_elem_bytes);
  const size_t need = sbox_walsh_histogram_workspace_bytes(n, m);
  if (!workspace) return fail(SBOX_ERR_WORKSPACE, "workspace is null (need %zu bytes)", need);
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(SBOX_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  if (workspace_bytes < need) return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* tail = reinterpret_cast<char*>(workspace) + need - 256;
  unsigned long long* over = reinterpret_cast<unsigned long long*>(tail);
  int32_t* nlp = nl ? nl : reinterpret_cast<int32_t*>(tail + 8);
  for (int z = 0; z < 2; ++z) {
    int* h = z ? reinterpret_cast<int*>(over) : reinterpret_cast<int*>(hist);
    long long cnt = z ? 2 : 2 * ((1LL << (n - 1)) + 1);
    void* args[] = {&h, &cnt};
    s = launch((const void*)&k_zero, dim3(64), dim3(256), args, st);
    if (s) return s;
  }
  return run_single(S, n, m, s_elem_bytes, maxabs_per_b, nlp, nullptr, 0, workspace, workspace_bytes, nullptr, st,
                    reinterpret_cast<unsigned long long*>(hist), over);
}

size_t sbox_avalanche_workspace_bytes(int n, int m) {
  if (n < 1 || n > 24 || m < 1 || m > 20 || n + m > 40) return 0;
  return align256((size_t)n << m << 2);
}

sbox_status sbox_avalanche(const void* S, int n, int m, int s_elem_bytes, int32_t* r, int32_t* summary,
                           const int32_t* maxabs_per_b, void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 1 || n > 24 || m < 1 || m > 20 || n + m > 40)
    return fail(SBOX_ERR_UNSUPPORTED, "avalanche needs 1 <= n <= 24, 1 <= m <= 20, n + m <= 40 (n=%d m=%d)", n, m);
  if (!S || !summary) return fail(SBOX_ERR_INVALID_ARG, "S or summary is null");
  if (s_elem_bytes != 1 && s_elem_bytes != 2 && s_elem_bytes != 4)
    return fail(SBOX_ERR_INVALID_ARG, "s_elem_bytes must be 1, 2 or 4 (got %d)", s_elem_bytes);
  int32_t* buf = r;
  if (!buf) {
    const size_t need = sbox_avalanche_workspace_bytes(n, m);
    if (!workspace) return fail(SBOX_ERR_WORKSPACE, "workspace is null (need %zu bytes without r)", need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(SBOX_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (workspace_bytes < need) return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, need);
    buf = reinterpret_cast<int32_t*>(workspace);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long long total = (long long)n << m;
  sbox_status s;
  {
    int* b = buf;
    long long cnt = total;
    void* args[] = {&b, &cnt};
    s = launch((const void*)&k_zero, dim3((unsigned)std::min<long long>(1024, (total + 255) / 256)), dim3(256), args, st);
    if (s) return s;
  }
  {
    const void* S_ = S;
    int n_ = n, m_ = m;
    int32_t* c = buf;
    void* args[] = {(void*)&S_, &n_, &m_, &c};
    const void* fn = s_elem_bytes == 1 ? (const void*)&k_deriv_count<1>
                   : s_elem_bytes == 2 ? (const void*)&k_deriv_count<2> : (const void*)&k_deriv_count<4>;
    const long long threads = (long long)n << (n - 1);
    s = launch(fn, dim3((unsigned)std::min<long long>(4096, (threads + 255) / 256)), dim3(256), args, st);
    if (s) return s;
  }
  // the 2^m-point transforms, in passes of at most 12 bits
  for (int lo = 0; lo < m;) {
    const int cwlog = std::min(lo, 6);
    const int R = std::min(m - lo, 12 - cwlog);
    int32_t* d = buf;
    int mlog = m, lo_ = lo, R_ = R, cw = cwlog;
    void* args[] = {&d, &mlog, &lo_, &R_, &cw};
    const long long blocks = (long long)n << (m - R - cwlog);
    s = launch((const void*)&k_fwht_pass, dim3((unsigned)blocks), dim3(256), args, st);
    if (s) return s;
    lo += R;
  }
  {
    const int32_t* rr = buf;
    int n_ = n, m_ = m;
    const int32_t* mx = maxabs_per_b;
    int32_t* sm = summary;
    void* args[] = {(void*)&rr, &n_, &m_, (void*)&mx, &sm};
    return launch((const void*)&k_avalanche_summary, dim3(1), dim3(256), args, st);
  }
}

sbox_status sbox_scratch_reserve(int n, int m, void* stream) {
  sbox_status s = check_nm(n, m);
  if (s) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  s = refuse_capture(st, "sbox_scratch_reserve");
  if (s) return s;
  const size_t need = sbox_walsh_nl_workspace_bytes(n, m, 0);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  StreamScratch& sc = g_scratch[{dev, reinterpret_cast<uintptr_t>(stream)}];
  if (sc.bytes >= need) return SBOX_OK;
  if (sc.ptr) {
    // earlier calls on this stream may still read the old buffer
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFree(sc.ptr));
    sc.ptr = nullptr;
    sc.bytes = 0;
  }
  HIP_TRY(hipMalloc(&sc.ptr, need));
  sc.bytes = need;
  return SBOX_OK;
}

sbox_status sbox_scratch_release(void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  sbox_status s = refuse_capture(st, "sbox_scratch_release");
  if (s) return s;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find({dev, reinterpret_cast<uintptr_t>(stream)});
  if (it == g_scratch.end()) return SBOX_OK;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipFree(it->second.ptr));
  g_scratch.erase(it);
  return SBOX_OK;
}

sbox_status sbox_walsh_nl(const void* S, int n, int m, int32_t* maxabs_per_b, int32_t* nl, void* stream) {
  sbox_status s = check_nm(n, m);
  if (s) return s;
  if (!S || !nl) return fail(SBOX_ERR_INVALID_ARG, "S or nl is null");
  const size_t need = sbox_walsh_nl_workspace_bytes(n, m, 0);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  StreamScratch sc;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find({dev, reinterpret_cast<uintptr_t>(stream)});
    if (it != g_scratch.end()) sc = it->second;
  }
  if (sc.bytes < need)
    return fail(SBOX_ERR_WORKSPACE,
                "no scratch of %zu bytes reserved for this stream on device %d (have %zu): call "
                "sbox_scratch_reserve(%d, %d, stream) first",
                need, dev, sc.bytes, n, m);
  return sbox_walsh_nl_ex(S, n, m, elem_bytes_for(m), maxabs_per_b, nl, nullptr, 0, sc.ptr, sc.bytes, nullptr,
                          stream);
}

size_t sbox_batched_workspace_bytes(const sbox_job* jobs, int32_t count) {
  BatchLayout L;
  std::string keep = g_last_error;
  if (plan_batch(jobs, count, nullptr, &L) != SBOX_OK) {
    g_last_error = keep;
    return 0;
  }
  return L.ws_bytes;
}

sbox_status sbox_walsh_nl_batched(const sbox_job* jobs, int32_t count, void* workspace, size_t workspace_bytes,
                                  void* stream) {
  BatchLayout L;
  sbox_status s = plan_batch(jobs, count, nullptr, &L);
  if (s) return s;
  if (count == 0) return SBOX_OK;
  if (!workspace || workspace_bytes < L.ws_bytes)
    return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, L.ws_bytes);
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(SBOX_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  s = refuse_capture(st, "sbox_walsh_nl_batched (its descriptors are staged per call; capture sbox_plan_launch)");
  if (s) return s;
  bind_batch(L, workspace);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    const size_t bytes = L.descs.size() * sizeof(JobDesc);
    StageBlock* blk = nullptr;
    s = acquire_stage(dev, bytes, &blk);
    if (s) return s;
    std::memcpy(blk->host, L.descs.data(), bytes);
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(workspace) + kQueueBytes, blk->host, bytes,
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(blk->evt, st));
  }
  return launch_batch(L, workspace, st);
}

size_t sbox_criteria_workspace_bytes(int n, int m) {
  if (n < 1 || n > 16 || m < 1 || m > 24 || n + m > 40) return 0;
  if (n <= 4) return 256;  // unused
  return f_bytes(n, m) + (size_t)kCritRegMaxGrid * 8 * 4;
}

namespace {
// 5 <= n <= 14 with a workspace: bit-sliced words, then the register-blocked
// kernel (one group of lanes per mask, both transforms without leaving the CU).
sbox_status criteria_reg(const void* S, int n, int m, int eb, int32_t* summary, int32_t* w0, int32_t* minwt,
                         int32_t* acmax, int32_t* pcwt, void* ws, hipStream_t st) {
  int cus = 0;
  sbox_status s = device_info(&cus);
  if (s) return s;
  uint32_t* F = reinterpret_cast<uint32_t*>(ws);
  const int nwords = 1 << (n - 5);
  {
    // start values (workgroup 0) and the bit-sliced table, one launch
    const void* S_ = S;
    int n_ = n, m_ = m, nw_ = nwords;
    void* args[] = {(void*)&S_, &n_, &m_, &F, &nw_, &summary, &w0, &minwt, &acmax, &pcwt};
    const void* fn = eb == 1 ? (const void*)&k_crit_prep<1> : eb == 2 ? (const void*)&k_crit_prep<2>
                                                                      : (const void*)&k_crit_prep<4>;
    const long long units = n >= 6 ? (1LL << n) : nwords;  // entries (a wave per 64) or words
    s = launch(fn, dim3((unsigned)(1 + (units + 255) / 256)), dim3(256), args, st);
    if (s) return s;
  }
  static const void* const fns[] = {
      (const void*)&k_crit_reg<5>,  (const void*)&k_crit_reg<6>,  (const void*)&k_crit_reg<7>,
      (const void*)&k_crit_reg<8>,  (const void*)&k_crit_reg<9>,  (const void*)&k_crit_reg<10>,
      (const void*)&k_crit_reg<11>, (const void*)&k_crit_reg<12>, (const void*)&k_crit_wide<13>,
      (const void*)&k_crit_wide<14>, (const void*)&k_crit_wide<15>, (const void*)&k_crit_wide<16>};
  const void* fn = fns[n - 5];
  const int wg = crit_reg_wg(n);
  const int gpb = wg >> (n - crit_reg_rb(n));  // groups (masks in flight) per workgroup
  int occ = 1;
  s = occupancy(fn, &occ, wg);
  if (s) return s;
  const long long masks = (1LL << m) - 1;
  const long long cap = std::min<long long>((long long)std::max(1, occ) * cus, kCritRegMaxGrid) * gpb;
  CritRegParams cp{};
  cp.F = F;
  cp.m = m;
  cp.chunk = (masks + cap - 1) / cap;
  cp.part = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ws) + f_bytes(n, m));
  cp.w0 = w0;
  cp.minwt = minwt;
  cp.acmax = acmax;
  cp.pcwt = pcwt;
  const long long groups = (masks + cp.chunk - 1) / cp.chunk;
  const int grid = (int)((groups + gpb - 1) / gpb);  // <= kCritRegMaxGrid
  {
    void* args[] = {&cp};
    s = launch(fn, dim3((unsigned)grid), dim3(wg), args, st);
    if (s) return s;
  }
  const int32_t* part = cp.part;
  int nwg = grid;
  void* args[] = {(void*)&part, &nwg, &summary};
  return launch((const void*)&k_crit_reg_finish, dim3(1), dim3(256), args, st);
}

}  // namespace

sbox_status sbox_criteria_ex(const void* S, int n, int m, int s_elem_bytes, int32_t* summary, int32_t* w0_per_b,
                             int32_t* minwt_per_b, int32_t* acmax_per_b, int32_t* pcwt_per_b, void* workspace,
                             size_t workspace_bytes, void* stream) {
  if (n < 1 || n > 16 || m < 1 || m > 24 || n + m > 40)
    return fail(SBOX_ERR_UNSUPPORTED, "criteria need 1<=n<=16, 1<=m<=24, n+m<=40 (n=%d m=%d)", n, m);
  if (!S || !summary) return fail(SBOX_ERR_INVALID_ARG, "S or summary is null");
  if (s_elem_bytes != 1 && s_elem_bytes != 2 && s_elem_bytes != 4)
    return fail(SBOX_ERR_INVALID_ARG, "s_elem_bytes must be 1, 2 or 4 (got %d)", s_elem_bytes);
  // n >= 15 needs a workspace; for 5 <= n <= 14 one selects the register-blocked
  // kernels (without one, the LDS kernel runs)
  const bool use_ws = n >= 15 || (n >= 5 && workspace != nullptr);
  if (use_ws) {
    const size_t need = sbox_criteria_workspace_bytes(n, m);
    if (!workspace) return fail(SBOX_ERR_WORKSPACE, "workspace is null (need %zu bytes)", need);
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(SBOX_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (workspace_bytes < need) return fail(SBOX_ERR_WORKSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, need);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int cus = 0;
  sbox_status s = device_info(&cus);
  if (s) return s;
  if (use_ws)  // sets the start values and finishes the summary itself
    return criteria_reg(S, n, m, s_elem_bytes, summary, w0_per_b, minwt_per_b, acmax_per_b, pcwt_per_b,
                        workspace, st);
  {
    int n_ = n;
    void* args[] = {&summary, &n_, &w0_per_b, &minwt_per_b, &acmax_per_b, &pcwt_per_b};
    s = launch((const void*)&k_criteria_init, dim3(1), dim3(64), args, st);
    if (s) return s;
  }
  const void* fn = s_elem_bytes == 1 ? (const void*)&k_criteria<1>
                 : s_elem_bytes == 2 ? (const void*)&k_criteria<2> : (const void*)&k_criteria<4>;
  int occ = 1;
  s = occupancy(fn, &occ);
  if (s) return s;
  CritParams cp{};
  cp.S = S;
  cp.eb = s_elem_bytes;
  cp.n = n;
  cp.m = m;
  cp.crit = summary;
  cp.w0 = w0_per_b;
  cp.minwt = minwt_per_b;
  cp.acmax = acmax_per_b;
  cp.pcwt = pcwt_per_b;
  const long long grid = std::min<long long>((1LL << m) - 1, (long long)occ * cus);
  {
    void* args[] = {&cp};
    s = launch(fn, dim3((unsigned)std::max(1LL, grid)), dim3(256), args, st);
    if (s) return s;
  }
  void* args[] = {&summary};
  return launch((const void*)&k_criteria_finish, dim3(1), dim3(64), args, st);
}

sbox_status sbox_criteria(const void* S, int n, int m, int s_elem_bytes, int32_t* summary, int32_t* w0_per_b,
                          int32_t* minwt_per_b, int32_t* acmax_per_b, int32_t* pcwt_per_b, void* stream) {
  if (n < 1 || n > 14 || m < 1 || m > 24)
    return fail(SBOX_ERR_UNSUPPORTED, "criteria need 1<=n<=14 and 1<=m<=24 without a workspace (n=%d m=%d); "
                "sbox_criteria_ex takes n = 15, 16", n, m);
  return sbox_criteria_ex(S, n, m, s_elem_bytes, summary, w0_per_b, minwt_per_b, acmax_per_b, pcwt_per_b, nullptr,
                          0, stream);
}

struct sbox_plan {
  BatchLayout layout;
  void* dev = nullptr;
  ClassStreams cs;
};

namespace {
void release_streams(ClassStreams& cs) {
  for (hipStream_t s : cs.side) (void)hipStreamDestroy(s);
  for (hipEvent_t e : cs.join) (void)hipEventDestroy(e);
  if (cs.fork) (void)hipEventDestroy(cs.fork);
  cs = ClassStreams{};
}

// One side stream and join event per size class after the first.
sbox_status make_streams(size_t classes, ClassStreams* cs) {
  if (classes < 2) return SBOX_OK;
  HIP_TRY(hipEventCreateWithFlags(&cs->fork, hipEventDisableTiming));
  for (size_t i = 1; i < classes; ++i) {
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    cs->side.push_back(s);
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cs->join.push_back(e);
  }
  return SBOX_OK;
}
}  // namespace

sbox_status sbox_plan_create(const sbox_job* jobs, int32_t count, const sbox_tuning* tuning, sbox_plan** out) {
  if (!out) return fail(SBOX_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  if (tuning && (tuning->chunk < 0 || tuning->grid < 0 || tuning->split_p < 0))
    return fail(SBOX_ERR_INVALID_ARG, "negative tuning field");
  if (tuning && (tuning->variant < 0 || tuning->variant > 4))
    return fail(SBOX_ERR_INVALID_ARG, "tuning variant %d (0 to 4)", tuning->variant);
  sbox_plan* p = new sbox_plan();
  sbox_status s = plan_batch(jobs, count, tuning, &p->layout);
  if (s) {
    delete p;
    return s;
  }
  if (count > 0) {
    hipError_t e = hipMalloc(&p->dev, p->layout.ws_bytes);
    if (e != hipSuccess) {
      delete p;
      return fail(SBOX_ERR_HIP, "hipMalloc(%zu): %s", p->layout.ws_bytes, hipGetErrorString(e));
    }
    bind_batch(p->layout, p->dev);
    e = hipMemcpy(reinterpret_cast<char*>(p->dev) + kQueueBytes, p->layout.descs.data(),
                  p->layout.descs.size() * sizeof(JobDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->dev);
      delete p;
      return fail(SBOX_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    s = make_streams(p->layout.classes.size(), &p->cs);
    if (s) {
      release_streams(p->cs);
      (void)hipFree(p->dev);
      delete p;
      return s;
    }
  }
  *out = p;
  return SBOX_OK;
}

sbox_status sbox_plan_launch(const sbox_plan* plan, void* stream) {
  if (!plan) return fail(SBOX_ERR_INVALID_ARG, "plan is null");
  return launch_batch(plan->layout, plan->dev, reinterpret_cast<hipStream_t>(stream), &plan->cs);
}

void sbox_plan_destroy(sbox_plan* plan) {
  if (!plan) return;
  if (plan->dev) {
    (void)hipDeviceSynchronize();
    (void)hipFree(plan->dev);
  }
  release_streams(plan->cs);
  delete plan;
}

}  // extern "C"

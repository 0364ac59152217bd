/*
 * sbox_walsh.h -- C ABI of the MI355X (gfx950) S-box Walsh spectrum /
 * nonlinearity library (libsboxwalsh.so).
 *
 * What is computed (Khadem & Ghasemi, "Improved Algorithms in Parallel
 * Evaluation of Large Cryptographic S-Box"):
 *   - For an n x m S-box S (a table S[0 .. 2^n) of values whose low m bits
 *     are used; Section 3, the vectorial Boolean function s = (f_1..f_m)),
 *     the Walsh matrix of Eq. 1, with its exponent read as <a,x> + <b,S(x)>:
 *         W(a, b) = sum_x (-1)^( parity(a & x) XOR parity(b & S[x]) ),
 *     a in [0, 2^n), b in [0, 2^m).  Column b is the fast Walsh-Hadamard
 *     transform (Algorithm 1) of the polarity truth table of the component
 *     function x -> parity(b & S[x]) (Eq. 2), 0 -> +1, 1 -> -1, in natural
 *     (Sylvester) order, so output index == a.
 *   - The per-mask maximum maxabs[b] = max_a |W(a, b)| folded into the
 *     transform (Algorithm 3, the "var" array), and the nonlinearity of
 *     Eq. 3 over the nonzero masks (Algorithm 6):
 *         NL = min_{b=1}^{2^m-1} (2^n - maxabs[b]) / 2
 *            = 2^(n-1) - max_{b != 0, a} |W(a, b)| / 2.
 *     maxabs[0] is 2^n by definition (row b = 0 is 2^n at a = 0, else 0).
 *   - Optionally the whole matrix, written as int32 in one of two layouts:
 *     SBOX_SPECTRUM_B_MAJOR: W[b * 2^n + a] (the transposed matrix of
 *     Section 5.1) or SBOX_SPECTRUM_A_MAJOR: W[a * 2^m + b] (Algorithm 1's
 *     matrix), or the same layouts of the linear approximation table W/2
 *     (SBOX_LAT_*).  Without it the 2^(n+m) matrix is never materialised.
 *   Every result is an exact integer; int32 holds all of them for n <= 30.
 *
 * Conventions for every entry point:
 *   - Asynchronous: work is enqueued on `stream` (a hipStream_t; NULL is
 *     the null stream) and results are valid after the stream is
 *     synchronised.  Unless stated otherwise a call performs no host
 *     synchronisation.
 *   - Device pointers: S, maxabs_per_b, nl, spectrum and workspace are
 *     device memory owned by the caller; the library never frees them.
 *     They must be naturally aligned for their element type (workspace:
 *     256 bytes).  S must stay unchanged until the work completes.
 *   - Arguments are validated before anything is enqueued; on any error
 *     nothing is enqueued, outputs are untouched, and the status is
 *     returned with a message available from sbox_last_error().
 *   - Limits: 1 <= n <= 24, 1 <= m <= 24, n + m <= 40.  Requests for a
 *     spectrum need n + m <= 34.  Outside these: SBOX_ERR_UNSUPPORTED.
 *   - Calls that share a workspace must not overlap in time (serialise them
 *     on one stream).
 */
#ifndef SBOX_WALSH_H
#define SBOX_WALSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SBOX_OK = 0,
    SBOX_ERR_INVALID_ARG = 1, /* null pointer, bad element width, bad layout, count < 0 ... */
    SBOX_ERR_UNSUPPORTED = 2, /* n or m outside the limits above */
    SBOX_ERR_WORKSPACE = 3,   /* workspace missing or smaller than the query says */
    SBOX_ERR_HIP = 4          /* a HIP runtime call or kernel launch failed */
} sbox_status;

typedef enum {
    SBOX_SPECTRUM_NONE = 0,
    SBOX_SPECTRUM_B_MAJOR = 1, /* W[b * 2^n + a] */
    SBOX_SPECTRUM_A_MAJOR = 2, /* W[a * 2^m + b] */
    SBOX_SPECTRUM_LAT = 0x10,  /* flag: store the linear approximation table W/2 instead of W */
    SBOX_LAT_B_MAJOR = 0x11,   /* LAT[b * 2^n + a] = W(a, b) / 2 = #{x : a.x = b.S(x)} - 2^(n-1) */
    SBOX_LAT_A_MAJOR = 0x12    /* LAT[a * 2^m + b] */
} sbox_layout;

/*
 * Launch tuning.  Zero fields mean "library default".  Values that do not
 * apply to the (n, m) at hand are rejected with SBOX_ERR_INVALID_ARG.
 *   split_p : bits of x each thread transforms in registers before the
 *             one LDS exchange (6, 7 or 8; n <= 8 uses n and ignores this).
 *   chunk   : consecutive masks (in Gray-code order) one thread group
 *             walks per work item.
 *   grid    : number of persistent workgroups (0: fill every CU).
 *   variant : butterfly engine for the n = 12 and n = 16 fused maximum (no
 *             spectrum): 0 the library's choice (currently 3), 1 packed
 *             16-bit VALU butterflies, 2 matrix cores (fp16 MFMA Hadamard
 *             blocks after popcount stages, exact; split_p does not apply),
 *             3 matrix cores without popcount stages: a first pass on fp4
 *             operands taken straight from the table's bits, then fp16
 *             passes (two at n = 16, where split_p = 4 or 8 picks the LDS
 *             exchange rounds; one at n = 12, one wave per mask); exact.
 *             4 (n = 12 only) as 3 with the first pass on int8 operands
 *             (int32 accumulation), kept for comparison: it issues twice the
 *             matrix-core work of 3.  Other sizes and modes accept 0 or 1
 *             only.  Batched launches and plans apply it to their n = 12
 *             and n = 16 boxes (variant 4 runs n = 16 boxes as 3).
 */
typedef struct sbox_tuning {
    int32_t split_p;
    int32_t chunk;
    int32_t grid;
    int32_t variant;
} sbox_tuning;

/*
 * Fused spectrum + nonlinearity of one S-box (Eq. 1-3, Algorithms 3 and 6).
 *   S            device, 2^n elements; element width inferred from m:
 *                uint8 if m <= 8, uint16 if m <= 16, else uint32.
 *   maxabs_per_b device int32[2^m] receiving max_a |W(a,b)|, or NULL.
 *   nl           device int32[1] receiving NL (required).
 * Takes its scratch from the buffer that sbox_scratch_reserve set aside for
 * this (device, stream) pair and never allocates: with no reservation, or
 * one made for a smaller (n, m), it returns SBOX_ERR_WORKSPACE and enqueues
 * nothing.  Calls on different streams use different scratch, so they may
 * overlap; calls on one stream are ordered by the stream.  Capturable (a
 * captured graph keeps the reserved buffer's address: do not replay it after
 * a reservation on that stream grew or was released).
 */
sbox_status sbox_walsh_nl(const void* S, int n, int m, int32_t* maxabs_per_b, int32_t* nl,
                          void* stream);

/*
 * Scratch for sbox_walsh_nl on `stream` of the current device, large
 * enough for every box up to n x m (the fused path's workspace).  Host
 * call; allocates device memory (hipMalloc) owned by the library, so it is
 * not capturable (SBOX_ERR_INVALID_ARG on a capturing stream).  A
 * reservation that is already large enough is kept as is; a smaller one is
 * replaced after the stream has been synchronised.
 * sbox_scratch_release synchronises the stream and frees its reservation
 * (no-op without one).  Neither may run concurrently with a sbox_walsh_nl
 * call on the same stream from another host thread.
 */
sbox_status sbox_scratch_reserve(int n, int m, void* stream);
sbox_status sbox_scratch_release(void* stream);

/*
 * Full form.
 *   s_elem_bytes  1, 2 or 4: width of the S elements (unsigned).
 *   spectrum      device int32[2^(n+m)] when layout != SBOX_SPECTRUM_NONE,
 *                 else ignored (may be NULL).
 *   workspace     device scratch of at least
 *                 sbox_walsh_nl_workspace_bytes(n, m, layout) bytes
 *                 (256-byte aligned).  When n > 16 a larger workspace lets
 *                 more masks be processed per pass.
 *   tuning        NULL for defaults.
 * Performs no allocation and no host synchronisation; graph-capturable.
 * An a-major spectrum (or LAT) with n = m >= 14 checks on the device
 * whether S is a permutation; if it is, it writes the b-major matrix of
 * S^-1, which is the a-major matrix of S (W_{S^-1}(u, v) = W_S(v, u),
 * Eq. 1 with y = S(x)), instead of transposing slabs (3.6 ms against
 * 6.5 ms at n = m = 16 on one MI355X).  The decision is taken again on
 * every call (and on every replay of a captured call) from the table's
 * contents at that time; a table that is not a permutation costs four
 * short launches more than the slab route alone (the scatter, the check
 * and the two passes of the other route, which return at once).
 */
sbox_status sbox_walsh_nl_ex(const void* S, int n, int m, int s_elem_bytes,
                             int32_t* maxabs_per_b, int32_t* nl,
                             int32_t* spectrum, int layout,
                             void* workspace, size_t workspace_bytes,
                             const sbox_tuning* tuning, void* stream);

/*
 * For callers that cannot allocate device memory or pass a workspace:
 * code under HIP graph capture, tight serving loops, and harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as sbox_walsh_nl_ex
 * with the library's defaults, but the scratch is a static device array of
 * sbox_walsh_nl_static_max_bytes() bytes (256 KiB) compiled into the
 * library, one per GPU, held until the process ends.  The call allocates
 * nothing (no hipMalloc, no hipFree).  It covers every n <= 16 and m <= 24
 * without a spectrum, and spectra except a-major ones with n + m >= 24
 * (those need a slab); larger requests return SBOX_ERR_WORKSPACE.  Every
 * call on a GPU uses that GPU's one array and leaves its last contents
 * behind (each call sets what must start at zero itself): calls that
 * overlap in time on one GPU, e.g. on two streams, race and give wrong
 * results; serialise them on one stream.
 */
sbox_status sbox_walsh_nl_static(const void* S, int n, int m, int s_elem_bytes,
                                 int32_t* maxabs_per_b, int32_t* nl,
                                 int32_t* spectrum, int layout, void* stream);
size_t sbox_walsh_nl_static_max_bytes(void);

/* Minimum workspace for sbox_walsh_nl_ex; 0 if (n, m, layout) is unsupported. */
size_t sbox_walsh_nl_workspace_bytes(int n, int m, int layout);

/*
 * One S-box of a batch.  Same meaning as the arguments of
 * sbox_walsh_nl_ex; batched boxes must have n <= 16.
 */
typedef struct sbox_job {
    const void* S;
    int32_t n, m, s_elem_bytes, layout;
    int32_t* maxabs_per_b;
    int32_t* nl;
    int32_t* spectrum;
} sbox_job;

/*
 * Many S-boxes of mixed sizes in one pass: boxes are grouped by n and each
 * group runs as one persistent launch whose workgroups pull (box, mask
 * range) items from a device work queue.  `jobs` is a host array of
 * `count` entries; its descriptors are copied into the workspace
 * asynchronously from a library-owned pinned block that is taken again only
 * after that copy has completed, so the array may be reused as soon as the
 * call returns and calls on different streams do not wait for each other on
 * the host (the pool holds up to 32 blocks per device; only when all are in
 * flight does a call wait for the oldest).  Each box's results equal those
 * of sbox_walsh_nl_ex on that box alone.  Not capturable, since the copy
 * reads the pinned block at launch time: on a capturing stream it returns
 * SBOX_ERR_INVALID_ARG (capture sbox_plan_launch instead).  Returns
 * SBOX_ERR_UNSUPPORTED if a box has n > 16.
 */
sbox_status sbox_walsh_nl_batched(const sbox_job* jobs, int32_t count,
                                  void* workspace, size_t workspace_bytes, void* stream);

/* Minimum workspace for sbox_walsh_nl_batched on these jobs; 0 if any is unsupported. */
size_t sbox_batched_workspace_bytes(const sbox_job* jobs, int32_t count);

/*
 * Plans: the batch is analysed and its descriptors uploaded once, at
 * creation (host call, synchronous, allocates device memory owned by the
 * plan).  sbox_plan_launch then only enqueues kernels (no allocation, no
 * host synchronisation, no copies), so it can be captured into a HIP graph
 * and replayed; it reads the S tables at launch time.  The job array may
 * be freed after sbox_plan_create returns; the buffers it points to must
 * outlive the plan.  sbox_plan_destroy frees the plan's memory (it
 * synchronises the device first).
 */
typedef struct sbox_plan sbox_plan;
sbox_status sbox_plan_create(const sbox_job* jobs, int32_t count, const sbox_tuning* tuning,
                             sbox_plan** out);
sbox_status sbox_plan_launch(const sbox_plan* plan, void* stream);
void sbox_plan_destroy(sbox_plan* plan);

/*
 * Further criteria of the component functions (the paper's future work,
 * Section 7), computed from the same transforms for every nonzero mask b:
 *   balancedness         W(0, b) == 0;
 *   correlation immunity order t: W(a, b) == 0 for all 1 <= wt(a) <= t,
 *                        resiliency order = t when every component is balanced;
 *   autocorrelation      r_b(d) = sum_x (-1)^(b.S(x) XOR b.S(x XOR d)), obtained
 *                        as 2^-n times the transform of W(., b)^2 (Wiener-Khinchin);
 *   absolute indicator   max_{b != 0, d != 0} |r_b(d)|;
 *   propagation order k: r_b(d) == 0 for all 1 <= wt(d) <= k.
 *   summary      device int32[8] (required): {NL, number of unbalanced masks,
 *                correlation-immunity order, resiliency order (-1 if some
 *                component is unbalanced), absolute indicator, propagation
 *                order, 0, 0}.
 *   w0_per_b, minwt_per_b, acmax_per_b, pcwt_per_b  device int32[2^m] or NULL:
 *                W(0,b); min wt(a) over a != 0 with W(a,b) != 0 (n + 1 if none);
 *                max_{d != 0} |r_b(d)|; min wt(d) over d != 0 with r_b(d) != 0
 *                (n + 1 if none).  Entry b = 0 is written as 0.
 * Limits: 1 <= n <= 14, 1 <= m <= 24 (each mask's transform stays in LDS).
 * No workspace, no allocation, no host synchronisation.
 */
sbox_status sbox_criteria(const void* S, int n, int m, int s_elem_bytes, int32_t* summary,
                          int32_t* w0_per_b, int32_t* minwt_per_b, int32_t* acmax_per_b,
                          int32_t* pcwt_per_b, void* stream);

/*
 * The same criteria up to n = 16 (1 <= n <= 16, 1 <= m <= 24, n + m <= 40).
 * The workspace (device, 256-byte aligned, at least
 * sbox_criteria_workspace_bytes(n, m) bytes: the bit-sliced table and one
 * slot of partial aggregates per workgroup) selects the register-blocked
 * kernel, which keeps both transforms of a mask on one compute unit (a
 * whole 1024-lane workgroup per mask at n = 16).  It is required for
 * n = 15, 16; for 5 <= n <= 14 it is optional and NULL runs the same kernel
 * as sbox_criteria (several times slower).  A workspace that is given must
 * meet the size and alignment above (else SBOX_ERR_WORKSPACE /
 * SBOX_ERR_INVALID_ARG).  For n <= 4 it is not used.  No allocation, no
 * host synchronisation.
 */
sbox_status sbox_criteria_ex(const void* S, int n, int m, int s_elem_bytes, int32_t* summary,
                             int32_t* w0_per_b, int32_t* minwt_per_b, int32_t* acmax_per_b,
                             int32_t* pcwt_per_b, void* workspace, size_t workspace_bytes,
                             void* stream);
size_t sbox_criteria_workspace_bytes(int n, int m);

/*
 * Histogram of |W| over the nonzero masks: the distribution of the entries
 * of the Walsh matrix of Eq. 1 (equivalently of the linear approximation
 * table W/2), counted inside the transform, so the matrix is never stored:
 *   hist[k] = #{(a, b) : 1 <= b < 2^m, |W(a, b)| = 2k},   k = 0 .. 2^(n-1).
 *   hist          device uint64[2^(n-1) + 1], overwritten (no need to clear it).
 *   maxabs_per_b  device int32[2^m] or NULL; nl device int32[1] or NULL: the
 *                 fused per-mask maximum and NL of the same pass.
 *   workspace     at least sbox_walsh_histogram_workspace_bytes(n, m) bytes.
 * Limits: 1 <= n <= 16, 1 <= m <= 24.  No allocation, no host
 * synchronisation.  Costs the fused transform plus one LDS atomic per
 * coefficient (at n = 16 about three times the fused NL call).
 */
sbox_status sbox_walsh_histogram(const void* S, int n, int m, int s_elem_bytes, uint64_t* hist,
                                 int32_t* maxabs_per_b, int32_t* nl, void* workspace,
                                 size_t workspace_bytes, void* stream);
size_t sbox_walsh_histogram_workspace_bytes(int n, int m);

/*
 * Strict avalanche and bit independence (more of the paper's future work,
 * Section 7), from the autocorrelation of every component at the unit input
 * differences e_i = 2^i:
 *   r[i * 2^m + b] = sum_x (-1)^parity(b & (S[x] ^ S[x ^ e_i])),  i < n, b < 2^m,
 * computed as the 2^m-point Walsh-Hadamard transform over the output masks
 * of the counts #{x : S[x] ^ S[x ^ e_i] = y}.  Flipping input bit i flips the
 * component of mask b with probability (1 - r / 2^n) / 2.
 *   r             device int32[n * 2^m], or NULL (then the workspace holds it).
 *   summary       device int32[3] (required):
 *                 [0] max_{i,j} |r_{e_j}(e_i)|: 0 iff every output bit
 *                     satisfies the strict avalanche criterion;
 *                 [1] max_{i, j<k} |r_{e_j ^ e_k}(e_i)|: the same for every XOR
 *                     of two output bits (bit independence), -1 if m < 2;
 *                 [2] min_{j<k} of the NL of the XOR of output bits j and k
 *                     (bit-independence nonlinearity) read from maxabs_per_b,
 *                     -1 if maxabs_per_b is NULL or m < 2.
 *   maxabs_per_b  device int32[2^m] written by sbox_walsh_nl(_ex) for the
 *                 same box (read only), or NULL.
 *   workspace     at least sbox_avalanche_workspace_bytes(n, m) bytes when r
 *                 is NULL; unused (may be NULL) otherwise.
 * Limits: 1 <= n <= 24, 1 <= m <= 20, n + m <= 40.  No allocation, no host
 * synchronisation.
 */
sbox_status sbox_avalanche(const void* S, int n, int m, int s_elem_bytes, int32_t* r, int32_t* summary,
                           const int32_t* maxabs_per_b, void* workspace, size_t workspace_bytes,
                           void* stream);
size_t sbox_avalanche_workspace_bytes(int n, int m);

/* Text describing the last non-OK status returned on this thread ("" if none). */
const char* sbox_last_error(void);

/* Library version, e.g. "1.0.0". */
const char* sbox_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SBOX_WALSH_H */

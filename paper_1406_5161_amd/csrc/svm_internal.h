// svm_internal.h -- types shared by the device kernels and the host driver of
// libsvmhip.so.  Not part of the public C-ABI (include/svmhip.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "svmhip.h"

namespace svm {

// sample layouts inside the library
// LAY_BITS: CSR rows whose values are all 1.0 with d <= BITS_MAX_D (at most 32 words), kept
// as bitsets of wpr 32-bit words per row; a dot product is a popcount of an AND.
enum : int { LAY_DENSE = 0, LAY_CSR_TABLE = 1, LAY_CSR_SLOT = 2, LAY_BITS = 3 };
constexpr int BITS_MAX_D = 1024;
inline int bits_wpr(int d) { return (((d + 31) / 32) + 3) & ~3; }   // words per row, a multiple of 4

// why a persistent-loop launch returned
enum : int { EXIT_NONE = 0, EXIT_CONVERGED = 1, EXIT_MAXITER = 2, EXIT_ABORT = 3 };

constexpr int STEP_BLOCK = 1024;      // threads per workgroup of the persistent step
constexpr int TABLE_MAX_D = 12288;    // CSR: dense float2 pair table in LDS up to this d (96 KB)
constexpr int SLOT_MAX_D = 65536;     // CSR: u16 slot map in LDS up to this d
constexpr int SLOT_MAX_NNZ = 2048;    // CSR slot map: longest row
constexpr int MAX_GRID = 1024;        // records are reduced by one workgroup
constexpr int CTL_BYTES = 512;

// Status byte of a sample: bit 0 = label is +1; bits 1-2 = bound class
// (0: alpha == 0, 1: 0 < alpha < C, 2: alpha == C).
enum : uint8_t { ST_YPOS = 1, ST_FREE = 2, ST_ATC = 4 };

// Selection state and counters of the solver, kept in device memory between
// launches of the persistent loop.
struct Ctl {
    double b_up, b_low;
    double a_up, a_low;       // alpha of the selected pair (carried, never re-read inside a launch)
    int32_t i_up, i_low;
    int64_t iter;
    int64_t counter;          // iterations left until the next shrink pass
    int64_t n_active;
    int64_t shrink_passes;
    int64_t shrunk_total;
    int32_t exit_reason;
    int32_t abort;
    int32_t err;              // validation error bits
    int32_t n_pos, n_neg;
    int32_t max_row_nnz;
    int32_t pad0;
    int64_t cache_both;       // iterations whose two kernel rows both came from the row cache
};
static_assert(sizeof(Ctl) <= 256, "Ctl must fit in its slot");

// One workgroup's partial selection for one iteration, in its own 128-byte line.  Every
// 64-bit word is self-validating: the high half is the iteration tag, the low half a
// 32-bit fragment of (b_up, b_low, i_up, i_low, active count, alpha_up, alpha_low and
// the CSR extents of the two candidates), so readers need no fence or barrier: a
// record is complete when all its words carry the current tag.
constexpr int REC_WORDS = 15;
constexpr int REC_LDS_STRIDE = 17;     // payload words per record in LDS (odd: no bank conflicts)
struct Rec {
    unsigned long long w[16];
};

struct StepArgs {
    int32_t n, d, dpad, lay;
    const float* x;           // dense: internal row-major [n][dpad]
    const int32_t* row_ptr;   // csr
    const int32_t* col;
    const float* val;
    int32_t pattern_only;     // csr values all 1.0: skip reading val
    int32_t max_row_nnz;
    const int8_t* y;
    double* alpha;
    double* f;
    uint8_t* status;
    int32_t* act;             // active ids, segmented by workgroup
    const int32_t* seg_start; // [G+1]
    int32_t* cnt;             // [G] active count of each segment
    Rec* rec;                 // [2*G] partial selections, double-buffered by iteration parity
    Ctl* ctl;
    void* reserved0;          // unused: with the fields below at these offsets the loop's code on bitset
                              // rows measured 3 % faster per iteration (6.2 against 6.4 us)
    double C, gamma, thr;
    int64_t max_iter;
    int64_t H;                // shrink schedule value (0: no shrinking in this launch)
    int64_t trace_cap;
    int32_t* tr_iu;
    int32_t* tr_il;
    double* tr_bu;
    double* tr_bl;
    unsigned long long spin_limit;  // watchdog for one barrier wait (wall-clock ticks)
    unsigned long long* work;       // [G][4] per workgroup in this launch: active rows visited, nonzeros read,
                                    // rows whose payload was read, kernel-row cache values read or written
    // where each workgroup keeps its segment during a launch
    int32_t mode;             // STEP_GLOBAL, STEP_LDS_STATE or STEP_LDS_ALL
    int32_t nseg_max;         // rows of the largest segment
    int32_t lds_meta_off;     // byte offset of the per-row state in dynamic LDS
    int32_t lds_pay_off;      // byte offset of the resident row payload
    int32_t nnz_seg_max;      // CSR: nonzeros of the largest segment
    int32_t lds_rec_off;      // byte offset of the records' payload words in dynamic LDS (G > 1)
    unsigned long long* prof; // [PROF_SLOTS] phase times of workgroup 0 (wall-clock ticks), or NULL
    const uint32_t* bits;     // LAY_BITS: rows as bitsets [n][wpr]
    int32_t wpr;
    int32_t kfull;            // 1: slot s of the cache holds K(s, i) for every sample i (the whole
                              // kernel matrix, cache_rows == n): no tags, no row data, K_ul read from it
    // kernel-row cache (rows streamed from HBM): slot s of `cache` holds K(id, i) for the
    // samples i of every segment, id being the sample named by the workgroup's own tag of slot
    // s; a slot holds sample id % cache_rows.  Values are KT; tags are epoch << 32 | id.
    void* cache;              // [cache_rows][n], or NULL
    unsigned long long* tags; // [G][cache_rows]
    int32_t cache_rows;
    uint32_t epoch;           // tag epoch of this launch (> 0; the host zeroes the tags per solve)
    // CSR rows streamed from HBM as element pairs: row i holds pairs prp[i] .. prp[i+1]-1, each
    // one word of two u16 column ids and two floats (1.0 when all values are 1.0); a row of odd
    // length ends with a zero element (column 0, value 0)
    const uint32_t* col2;     // [prp[n]]
    const float* val2;        // [2 prp[n]], 8-byte aligned
    const int32_t* prp;       // [n + 1] first pair of each row
};

// Residency of a workgroup's segment during one launch of the SMO loop:
// STEP_GLOBAL    per-row state (f, status, active list) and row payload in HBM;
// STEP_LDS_STATE per-row state in LDS, row payload streamed from HBM;
// STEP_LDS_ALL   per-row state and row payload (dense rows, CSR column ids
//                as u16 plus values unless all are 1.0, or bitset rows) in LDS.
enum : int { STEP_GLOBAL = 0, STEP_LDS_STATE = 1, STEP_LDS_ALL = 2 };
constexpr int PROF_SLOTS = 8;
constexpr size_t STEP_LDS_BUDGET = 156 * 1024;

struct StepLds {
    size_t pair_bytes, rec_off, meta_off, pay_off, total;
    int mode;
};
StepLds plan_step_lds(int lay, int d, int dpad, int max_row_nnz, int nseg_max, long long nnz_seg_max,
                      bool pattern_only, int max_mode, int G);

// Kernel sums: out[a] = sum_b coef[b] * K(A_a, B_b) + bias_a, bias_a = -y_a or -beta.
struct SumArgs {
    int32_t lay;              // LAY_DENSE, LAY_CSR_TABLE, LAY_CSR_SLOT or LAY_BITS (A and B share it)
    int32_t d, dpad;
    // A side
    const float* ax;
    const int32_t* arp;
    const int32_t* acol;
    const float* aval;
    const int32_t* alist;     // rows of A to evaluate (na)
    int32_t na;
    // B side
    const float* bx;
    const int32_t* brp;
    const int32_t* bcol;
    const float* bval;
    const int32_t* blist;     // rows of B in the sum (nb), ascending
    const double* coef;       // [nb]
    int32_t nb;
    int32_t nsplit;           // B split across blockIdx.y; partial sums in part[split][a]
    double* part;
    double gamma;
    int32_t rows_per_block;   // A rows held in LDS per workgroup
    // LAY_BITS: both sides as bitsets of wpr words per row
    const uint32_t* abits;
    const uint32_t* bbits;
    int32_t wpr;
    int32_t slot_rows;        // LAY_CSR_SLOT: A rows per group (slot_rows_for)
};
// A rows the wide-CSR kernel sum groups per pass for the longest row max_nnz and d columns:
// the most (at most 8) whose column table fits the LDS next to the slot map.
int slot_rows_for(int d, int max_nnz);

// ---- launch wrappers (device code in svm_kernels.hip)
hipError_t launch_validate(int n, int d, int lay, const float* x, int64_t ldx, int feature_major,
                           const int32_t* rp, const int32_t* col, const float* val, const int8_t* y, Ctl* ctl,
                           hipStream_t s);
hipError_t launch_pack_dense(int n, int d, int dpad, const float* x, int64_t ldx, int feature_major, float* out,
                             hipStream_t s);
hipError_t launch_init_state(int n, const int8_t* y, double C, int warm, double* alpha, double* f, uint8_t* status,
                             hipStream_t s);
hipError_t launch_reset_active(int n, int G, int32_t* seg_start, int32_t* cnt, int32_t* act, hipStream_t s);
hipError_t launch_iota(int n, int32_t* out, hipStream_t s);
hipError_t launch_kmat_sum(int na, const int32_t* alist, int nb, const int32_t* blist, const double* coef,
                           const float* kmat, long long ldk, int nsplit, double* part, hipStream_t s);
hipError_t launch_select(int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act, const double* f,
                         const double* alpha, const int8_t* y, double C, Rec* rec, Ctl* ctl, hipStream_t s);
hipError_t launch_step(const StepArgs& a, int G, int lpr, int kprec, size_t lds, hipStream_t s);
int step_max_blocks(int lay, int lpr, int kprec, int mode, size_t lds, bool cache);
bool step_cache_capable(int lay, int mode);   // layouts and residencies with a kernel-row cache
hipError_t launch_mark_active(int n, int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act,
                              uint8_t* mask, hipStream_t s);
// stable compaction: list = ascending ids i with pred(i); pred: 0 = mask[i]==0, 1 = alpha[i] > 0, 2 = all
hipError_t launch_compact(int n, int pred, const uint8_t* mask, const double* alpha, const int8_t* y,
                          int32_t* blk_cnt, int32_t* list, double* coef, int32_t* count_out, hipStream_t s);
hipError_t launch_kernel_sum(const SumArgs& a, int kprec, hipStream_t s);
bool kernel_sum_uses_mfma(int lay, int dpad, int kprec);   // dense FP32 sums on the matrix cores
constexpr int KSUM_MFMA_ROWS = 64;                         // A rows per workgroup of that kernel
// out[alist[r]] = sum_s part[s][r] + bias (bias: -y[alist[r]] if y != NULL, else -beta)
hipError_t launch_finish_sum(int na, int nsplit, const double* part, const int32_t* alist, const int8_t* y,
                             double beta, double* out, hipStream_t s);
hipError_t launch_refresh_status(int n, const double* alpha, const int8_t* y, double C, uint8_t* status,
                                 hipStream_t s);
// final scalars: [0] sum f over I0, [1] |I0|, [2] sum alpha, [3] sum alpha y (f + y), [4] n_sv, [5] n_bsv
hipError_t launch_summary(int n, const double* alpha, const double* f, const int8_t* y, double C, double* blk,
                          double* out6, hipStream_t s);
hipError_t launch_check_pattern(int nnz, const float* val, int32_t* flag, hipStream_t s);
// CSR columns as u16 and values (1.0 where pattern_only) copied into element pairs for the SMO
// loop's HBM stream: row i from element 2 prp[i], a zero element after a row of odd length
// (d <= 65,536)
hipError_t launch_pack_pairs(int n, const int32_t* rp, const int32_t* prp, const int32_t* col, const float* val,
                             int pattern_only, uint16_t* col16, float* val2, hipStream_t s);

int device_cu_count();

// ---- wide CSR kernel sums with the frequent columns as dense rows (svm_ksum_ht.hip)
constexpr int HT_BLOCK = 512;         // threads per workgroup
constexpr int HT_CHUNK = 64;          // support vectors per sweep step
constexpr int HT_TILE_MAX = 64;       // target rows per workgroup (16, 32 or 64)
constexpr int HT_ENTRIES = 4096;      // tail nonzeros of one tile of target rows (LDS table)
constexpr int HT_SLOTS = 8192;        // LDS hash slots for their columns
constexpr int HT_MAX_D = 65535;       // column ids fit the hash key
constexpr int HT_MAX_WORDS = (HT_MAX_D + 32) / 32;   // head-column bitmap words
constexpr int HT_H_MAX = 128;         // head columns: 32, 64 or 128
constexpr int HT_H_DEFAULT = 128;

struct HtArgs {
    int32_t H, d, na, nb;
    int32_t tile_rows, nsplit;
    // target rows (A): head rows [.][H], CSR for the tail, |x|^2
    const float* a_head;
    const int32_t* a_rp;
    const int32_t* a_col;
    const float* a_val;
    const float* a_nrm;
    const int32_t* alist;     // rows of A to evaluate (na), or NULL for 0..na-1
    // support vectors (B), packed in sweep order by launch_ht_pack
    const float* b_head;      // [nbp][H], nbp = nb rounded up to HT_CHUNK (zero rows beyond nb)
    const float* b_nrm;       // [nbp]
    const int32_t* b_toff;    // [nb + 1] tail offsets
    const uint2* b_tent;      // tail nonzeros: (column << 6 | ordinal % 64, value bits)
    const double* coef;       // [nb]
    const uint32_t* hbits;    // head columns as a bitmap of (d + 31) / 32 words
    double gamma;
    double fx_scale, fx_inv;  // tail dots in 64-bit fixed point: value * fx_scale (a power of two)
    double* part;             // [nsplit][na] partial sums
    // kernel-matrix fill: with kout set, B is every sample in order and the kernel also stores
    // K(a, b) at kout[b * ldk + a] (1.0 where a == b); the sums are then not used
    float* kout;
    int64_t ldk;
};
hipError_t launch_col_count(int64_t nnz, const int32_t* col, int32_t* cnt, hipStream_t s);
hipError_t launch_ht_split(int n, int H, const int32_t* rp, const int32_t* col, const float* val,
                           const int32_t* hmap, float* head, float* nrm, int32_t* tcnt, unsigned* maxn2,
                           hipStream_t s);
hipError_t launch_ht_tiles(int na, const int32_t* alist, const int32_t* tcnt, int32_t* out3, hipStream_t s);
hipError_t launch_ht_pack(int nb, int H, const int32_t* blist, const float* head, const float* nrm, const int32_t* rp,
                          const int32_t* col, const float* val, const int32_t* hmap, const int32_t* tcnt,
                          int32_t* toff, float* bhead, float* bnrm, uint2* tent, hipStream_t s);
hipError_t launch_kernel_sum_ht(const HtArgs& a, hipStream_t s);
size_t ht_lds_bytes(int H);

// ---- several problems over one sample set in lockstep (svm_shared.hip)
constexpr int SHARED_MAX = 8;         // problems per launch
constexpr int SHARED_BLOCK = 512;     // threads per workgroup
constexpr int SHARED_GRID_MAX = 64;   // one wave merges a problem's records

struct SharedProb {
    const int8_t* y;
    double* alpha;
    double* f;
    uint8_t* status;
    Ctl* ctl;                 // state the launch starts from and ends with
    double C, gamma, thr;
    int64_t max_iter;
};
struct SharedArgs {
    int32_t n, d, dpad, lay;  // lay: LAY_DENSE or LAY_BITS
    int32_t wpr, k;           // bitset words per row; problems
    int32_t live_mask;        // problems this launch advances (bit p)
    int32_t seg_max;          // rows of the largest workgroup segment
    int32_t res;              // 1: each workgroup keeps its segment's rows, f and status in LDS
    int32_t pad;
    const float* x;           // dense rows [n][dpad]
    const uint32_t* bits;     // bitset rows [n][wpr]
    Rec* rec;                 // [2][SHARED_MAX][G] exchange records, zeroed before the launch
    unsigned long long spin_limit;
    unsigned long long* work; // [G]: rows read by each workgroup (once per iteration for all problems)
    SharedProb prob[SHARED_MAX];
};
hipError_t launch_shared(const SharedArgs& a, int G, int kprec, hipStream_t s);
int shared_max_blocks(int lay, int kprec, bool res, size_t lds);
// dynamic LDS of the lockstep launch: the pair rows of every problem, and with res the
// segment's rows (bitsets or dense floats), f and status of every problem
size_t shared_lds_bytes(int lay, int d, int seg_max, bool res);

// ---- shape autotuner (svm_tune.cpp): measured shapes per problem class, per process
enum : int { TUNE_GRID = 0, TUNE_TEAM = 1 };
struct TuneClass {
    int target;               // TUNE_GRID (svm_train workgroups) or TUNE_TEAM (batched team size)
    int lay, kprec;
    bool pattern, shrink;
    long long n, d;
};
int tuned_shape(const TuneClass& c);   // 0: not tuned
void set_tuned_shape(const TuneClass& c, int shape);
void clear_tuned_shapes();
// the batched solver's team-size rule for a problem (svm_serve.cpp), and its layout there
int batch_team_rule(const svm_problem_t* p, int nnz, bool pattern);
int batch_layout(const svm_problem_t* p, bool pattern);

// svm_decision on a caller-given device workspace (svm_host.cpp); *need receives the bytes the
// problem needs (SVM_EWORKSPACE when ws_bytes is smaller).
int decision_in_workspace(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                          const svm_problem_t* queries, double* out, int kprec, void* ws, size_t ws_bytes,
                          hipStream_t s, size_t* need);
void set_last_hip_error(hipError_t e);   // reported by svm_strerror(SVM_EHIP)

}  // namespace svm

namespace svm {

// ---- batched / serving solver: a team of workgroups solves one problem

constexpr int BATCH_BLOCK = 512;
constexpr size_t BATCH_LDS_BYTES = 120 * 1024;   // dynamic LDS of a batched workgroup
constexpr int BATCH_SUMR = 8;                     // rows per reconstruction tile
constexpr int TEAM_MAX = 64;                      // workgroups per problem (one wave merges them)

struct BatchResult {
    double beta, b_up, b_low, dual_obj;
    long long iterations;
    int32_t n_sv, n_bsv, n_recon, status;
    long long shrink_passes, shrunk_total;
    unsigned long long t_start, t_end;   // device wall clock (100 MHz) around the solve
    int32_t done;                        // set last (release) when the fields above are final
    int32_t started;                     // set once the whole team has taken its tickets
};

// Outcome of a preparation job (validation, counts, dense packing) run by the serving loop.
struct PrepOut {
    int32_t err;                         // bit 0 malformed input, bit 1 non-finite value
    int32_t n_pos, n_neg, max_row_nnz, nnz, pattern;
    int32_t done;                        // set last (release) when the fields above are final
    int32_t pad;
};

struct BatchDesc {
    int32_t n, d, dpad, lay;             // lay: LAY_DENSE, LAY_CSR_TABLE or LAY_BITS
    const float* x;                      // dense, packed [n][dpad]
    const int32_t* row_ptr;
    const int32_t* col;
    const float* val;
    int32_t pattern_only, lpr;           // lpr: lanes per row (dense and CSR)
    const uint32_t* bits;                // LAY_BITS rows [n][wpr]
    int32_t wpr, pad5;
    const int8_t* y;
    double C, gamma, eps;
    int32_t shrink_mode, kprec;
    long long H, max_iter;
    uint32_t flags;
    int32_t pad;
    int32_t team;                        // workgroups solving this problem together
    int32_t pad2;
    unsigned long long* trec;            // team exchange records [2][team][16], zeroed before the start
    unsigned long long* prof;            // NULL, or 8 device counters rank 0 adds its phase ticks to
    // preparation jobs only (ticket rank -1): the caller's samples, validated and, for dense
    // layouts, packed into x; the team records (TEAM_MAX members) are zeroed
    const float* xsrc;
    int64_t ldx;
    int32_t src_layout;                  // SVM_DENSE_ROW_MAJOR | SVM_DENSE_FEATURE_MAJOR | SVM_CSR
    int32_t pad3;
    PrepOut* prep;                       // pinned host memory
    // per-problem device workspace
    double* alpha;
    double* f;
    uint8_t* status;
    int32_t* act;
    int32_t* list_w;
    int32_t* list_z;                     // [team][n]: each member's support-vector list
    double* coef;                        // [team][n]
    BatchResult* res;                    // device or pinned host memory
};

struct BatchArgs {
    const BatchDesc* descs;              // descriptor ring (device or pinned host)
    int32_t capacity;                    // ring size (power of two)
    int32_t tcapacity;                   // ticket ring size (power of two)
    const int2* tickets;                 // worker ticket -> (descriptor slot, rank in the team; -1: preparation)
    int32_t* head;                       // device counter: next ticket
    const int32_t* tail;                 // number of published tickets (host-written when serving)
    const int32_t* shutdown;             // host sets 1 to stop the loop; set only when no ticket waits
    int32_t* mirror;                     // device [2]: tail and shutdown as last seen by the leader
    int32_t fixed_tail;                  // > 0: a fixed batch (tail is this value, no polling)
    int32_t pad;
};

hipError_t launch_batch(const BatchArgs& a, int workgroups, int kprec, hipStream_t s);
hipError_t launch_pack_bits(int n, int d, int wpr, const int32_t* row_ptr, const int32_t* col, uint32_t* out,
                            hipStream_t s);
unsigned long long* debug_profile_slots();   // per-phase timer slots set by svm_debug_set_profile
int batch_max_workgroups(int kprec);

}  // namespace svm

// svm_host.cpp -- host side of libsvmhip.so: argument checks, workspace plan,
// the phase driver of Alg. 5 (and its multi-reconstruction variant), gradient
// reconstruction (Alg. 6), the classifier of eq:classi and the test hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "svm_internal.h"

using namespace svm;

namespace {

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) {                        \
            last_hip_error() = _e;                     \
            return SVM_EHIP;                           \
        }                                              \
    } while (0)

hipError_t& last_hip_error() {
    static thread_local hipError_t e = hipSuccess;
    return e;
}

struct TraceCfg {
    int64_t cap = 0;
    int32_t* iu = nullptr;
    int32_t* il = nullptr;
    double* bu = nullptr;
    double* bl = nullptr;
};
TraceCfg& trace_cfg() {
    static thread_local TraceCfg t;
    return t;
}
int* last_step_info() {
    static thread_local int v[5] = {0, 0, 0, 0, 0};   // mode, grid, lanes per row, layout, values all 1.0
    return v;
}
unsigned long long*& prof_cfg() {
    static thread_local unsigned long long* p = nullptr;
    return p;
}

constexpr int NSPLIT_MAX = 16;
constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

struct Plan {
    size_t ctl, xpack, bits, fint, status, mask, act, seg, cnt, rec, listw, listz, coef, blkcnt, counts, part,
        sumblk, out6, work, htcnt, hthmap, htbits, hthead, htnrm, httcnt, htmisc, htbhead, htbnrm, httoff, httent,
        kcache, ktags, col16, val2, prp, total;
    int64_t cache_rows;   // slots of the kernel-row cache (0: none)
    int tag_grid;         // workgroups the cache tags are sized for
};

int dpad_of(int d) { return (d + 3) & ~3; }

// Wide CSR (beyond the LDS column table) whose kernel sums can take the dense-head path.
bool ht_capable(const svm_problem_t* p) {
    return p->layout == SVM_CSR && p->d > TABLE_MAX_D && p->d <= HT_MAX_D;
}

// Device buffers of the head/tail kernel sums (svm_ksum_ht.hip).
struct HtBufs {
    int32_t* cnt = nullptr;     // [d] column occurrences
    int32_t* hmap = nullptr;    // [d] head position of a column, -1 for the tail
    uint32_t* hbits = nullptr;  // [HT_MAX_WORDS] head columns as a bitmap
    float* head = nullptr;      // [n][H] head rows of the training set
    float* nrm = nullptr;       // [n] |x|^2
    int32_t* tcnt = nullptr;    // [n] tail nonzeros per row
    int32_t* misc = nullptr;    // [0..2] tile maxima, [3] largest |x|^2 (float bits)
    float* bhead = nullptr;     // support vectors packed in sweep order: head rows [n + 64][H]
    float* bnrm = nullptr;      // [n + 64]
    int32_t* toff = nullptr;    // [n + 1] tail offsets
    uint2* tent = nullptr;      // [nnz] tail nonzeros
};

// Nonzeros of a CSR problem (row_ptr[n], read from the device), 0 for dense rows.
int64_t csr_nnz(const svm_problem_t* p, hipStream_t s) {
    if (p->layout != SVM_CSR || !p->row_ptr || p->n < 1) return 0;
    int32_t v = 0;
    if (hipMemcpyAsync(&v, p->row_ptr + p->n, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return -1;
    if (hipStreamSynchronize(s) != hipSuccess) return -1;
    return v;
}

// Slots of the kernel-row cache for the budget in params (0 when none or fewer than 2 fit).
int64_t cache_rows_for(const svm_problem_t* p, const svm_params_t* q) {
    if (!q || q->cache_mb <= 0 || p->n < 2) return 0;
    const int64_t vb = q->kernel_precision == SVM_KERNEL_FP64 ? 8 : 4;
    const int64_t rows = ((int64_t)q->cache_mb << 20) / ((int64_t)p->n * vb);
    return rows < 2 ? 0 : std::min<int64_t>(rows, p->n);
}

Plan make_plan(const svm_problem_t* p, const svm_params_t* params, int64_t nnz) {
    const size_t n = (size_t)p->n;
    Plan q{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    q.ctl = take(CTL_BYTES);
    q.xpack = take(p->layout == SVM_CSR ? 0 : sizeof(float) * n * (size_t)dpad_of(p->d));
    // binary CSR rows as bitsets (LAY_BITS), reserved for every CSR problem narrow enough
    q.bits = take(p->layout == SVM_CSR && p->d <= BITS_MAX_D ? sizeof(uint32_t) * n * (size_t)bits_wpr(p->d) : 0);
    q.fint = take(sizeof(double) * n);
    q.status = take(n);
    q.mask = take(n);
    q.act = take(sizeof(int32_t) * n);
    q.seg = take(sizeof(int32_t) * (MAX_GRID + 1));
    q.cnt = take(sizeof(int32_t) * MAX_GRID);
    q.rec = take(sizeof(Rec) * 3 * MAX_GRID);   // [0, 2G): tagged step records; [2G, 3G): selection
    q.listw = take(sizeof(int32_t) * n);
    q.listz = take(sizeof(int32_t) * n);
    q.coef = take(sizeof(double) * n);
    q.blkcnt = take(sizeof(int32_t) * (n / 1024 + 4));
    q.counts = take(64);
    q.part = take(sizeof(double) * n * NSPLIT_MAX);
    q.sumblk = take(sizeof(double) * 256 * 6);
    q.out6 = take(64);
    q.work = take(sizeof(unsigned long long) * 4 * MAX_GRID);
    const bool ht = ht_capable(p);
    q.htcnt = take(ht ? sizeof(int32_t) * (size_t)p->d : 0);
    q.hthmap = take(ht ? sizeof(int32_t) * (size_t)p->d : 0);
    q.htbits = take(ht ? sizeof(uint32_t) * HT_MAX_WORDS : 0);
    q.hthead = take(ht ? sizeof(float) * n * HT_H_MAX : 0);
    q.htnrm = take(ht ? sizeof(float) * n : 0);
    q.httcnt = take(ht ? sizeof(int32_t) * n : 0);
    q.htmisc = take(ht ? 64 : 0);
    q.htbhead = take(ht ? sizeof(float) * (n + HT_CHUNK) * HT_H_MAX : 0);
    q.htbnrm = take(ht ? sizeof(float) * (n + HT_CHUNK) : 0);
    q.httoff = take(ht ? sizeof(int32_t) * (n + 1) : 0);
    q.httent = take(ht ? sizeof(uint2) * (size_t)std::max<int64_t>(nnz, 0) : 0);
    q.cache_rows = cache_rows_for(p, params);
    q.tag_grid = std::min(MAX_GRID, std::max(params ? params->grid_blocks : 0, std::max(1, device_cu_count())));
    const size_t vb = params && params->kernel_precision == SVM_KERNEL_FP64 ? 8 : 4;
    q.kcache = take((size_t)q.cache_rows * n * vb);
    q.ktags = take(sizeof(unsigned long long) * (size_t)q.cache_rows * q.tag_grid);
    // CSR rows as element pairs for the loop's HBM stream (u16 columns and a copy of the values,
    // every row from an even element: at most nnz + n elements)
    const size_t npad = p->layout == SVM_CSR ? (size_t)std::max<int64_t>(nnz, 0) + n : 0;
    q.col16 = take(sizeof(uint16_t) * npad);
    q.val2 = take(sizeof(float) * npad);
    q.prp = take(p->layout == SVM_CSR ? sizeof(int32_t) * (n + 1) : 0);
    q.total = o;
    return q;
}

// The H most frequent columns of a CSR training set (ties to the lower column id) become the
// head: hmap / hbits on the device.
// Host staging of the head selection: fixed arrays (the column count is at most HT_MAX_D), so
// choosing a head allocates nothing; one call at a time uses them.
struct HeadStage {
    std::mutex m;
    int32_t cnt[HT_MAX_D + 1];
    int32_t order[HT_MAX_D + 1];
    int32_t hmap[HT_MAX_D + 1];
    uint32_t bits[HT_MAX_WORDS];
};
HeadStage& head_stage() {
    static HeadStage h;
    return h;
}

int ht_choose_head(const svm_problem_t* p, int H, const HtBufs& b, hipStream_t s) {
    if (p->d > HT_MAX_D) return SVM_EUNSUPPORTED;
    int32_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, p->row_ptr + p->n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemsetAsync(b.cnt, 0, sizeof(int32_t) * (size_t)p->d, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(launch_col_count(nnz, p->col, b.cnt, s));
    HeadStage& st = head_stage();
    std::lock_guard<std::mutex> lock(st.m);
    int32_t* cnt = st.cnt;
    HIP_TRY(hipMemcpyAsync(cnt, b.cnt, sizeof(int32_t) * (size_t)p->d, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < p->d; ++c) st.order[c] = c;
    const int h = std::min(H, p->d);
    std::partial_sort(st.order, st.order + h, st.order + p->d,
                      [cnt](int a, int b) { return cnt[a] != cnt[b] ? cnt[a] > cnt[b] : a < b; });
    for (int c = 0; c < p->d; ++c) st.hmap[c] = -1;
    for (int w = 0; w < HT_MAX_WORDS; ++w) st.bits[w] = 0u;
    for (int k = 0; k < h; ++k) {
        st.hmap[st.order[k]] = k;
        st.bits[st.order[k] >> 5] |= 1u << (st.order[k] & 31);
    }
    HIP_TRY(hipMemcpyAsync(b.hmap, st.hmap, sizeof(int32_t) * (size_t)p->d, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b.hbits, st.bits, sizeof(uint32_t) * HT_MAX_WORDS, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SVM_OK;
}

// Fixed-point scale of the tail dots from the largest squared row norm m: every partial sum of
// tail products is at most m <= 2^e in magnitude, kept below 2^62.
void ht_fixed_point(unsigned maxn2_bits, double* scale, double* inv) {
    float m;
    std::memcpy(&m, &maxn2_bits, sizeof(m));
    int e = 0;
    if (m > 0.f && std::isfinite(m)) (void)std::frexp((double)m, &e);
    e = std::max(-900, std::min(900, e));
    *scale = std::ldexp(1.0, 62 - e);
    *inv = std::ldexp(1.0, e - 62);
}

// Rows per tile of the head/tail sum for the target list: the largest of 64, 32, 16 whose
// tiles' tail nonzeros fit the LDS table; 0 if none does.
int ht_tile_rows(int na, const int32_t* alist, const int32_t* tcnt, int32_t* misc, hipStream_t s, int* rows) {
    HIP_TRY(hipMemsetAsync(misc, 0, 3 * sizeof(int32_t), s));
    HIP_TRY(launch_ht_tiles(na, alist, tcnt, misc, s));
    int32_t t[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(t, misc, sizeof(t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *rows = t[0] <= HT_ENTRIES ? 64 : t[1] <= HT_ENTRIES ? 32 : t[2] <= HT_ENTRIES ? 16 : 0;
    return SVM_OK;
}

int ht_nsplit(int na, int rows, int nb) {
    const int blocks = (na + rows - 1) / rows;
    int ns = std::max(1, std::min(NSPLIT_MAX, (512 + blocks - 1) / blocks));
    return std::min(ns, std::max(1, nb / 256));
}

int check_problem(const svm_problem_t* p, bool need_labels) {
    if (!p || p->n < 1 || p->d < 1) return SVM_EINVAL;
    if (need_labels && (!p->y || p->n < 2)) return SVM_EINVAL;
    if (p->layout == SVM_CSR) {
        if (!p->row_ptr || !p->col || !p->val) return SVM_EINVAL;
        if (p->d > SLOT_MAX_D) return SVM_EUNSUPPORTED;
    } else if (p->layout == SVM_DENSE_ROW_MAJOR) {
        if (!p->x || p->ldx < p->d) return SVM_EINVAL;
    } else if (p->layout == SVM_DENSE_FEATURE_MAJOR) {
        if (!p->x || p->ldx < p->n) return SVM_EINVAL;
    } else {
        return SVM_EINVAL;
    }
    return SVM_OK;
}

int check_params(const svm_params_t* q) {
    if (!q) return SVM_EINVAL;
    if (!(q->C > 0) || !(q->gamma > 0) || !(q->eps > 0) || !std::isfinite(q->C) || !std::isfinite(q->gamma) ||
        !std::isfinite(q->eps))
        return SVM_EINVAL;
    if (q->shrink_mode < 0 || q->shrink_mode > 2) return SVM_EINVAL;
    if (q->shrink_mode != SVM_SHRINK_NONE && !(q->shrink_param > 0)) return SVM_EINVAL;
    if (q->shrink_kind < 0 || q->shrink_kind > 1) return SVM_EINVAL;
    if (q->max_iter <= 0) return SVM_EINVAL;
    if (q->kernel_precision != SVM_KERNEL_FP32 && q->kernel_precision != SVM_KERNEL_FP64) return SVM_EINVAL;
    if (q->grid_blocks < 0 || q->grid_blocks > MAX_GRID) return SVM_EINVAL;
    int l = q->lanes_per_row;
    if (l < 0 || l > 64 || (l & (l - 1))) return SVM_EINVAL;
    const int h = q->head_cols;
    if (h != -1 && h != 0 && h != 32 && h != 64 && h != 128) return SVM_EINVAL;
    return SVM_OK;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Everything one training call needs on the device.
struct Solver {
    const svm_problem_t* p;
    const svm_params_t* q;
    hipStream_t s;
    unsigned char* ws;
    Plan plan;
    int n, d, dpad, lay, G, lpr;
    bool pattern_only;
    int max_row_nnz;
    double* alpha;
    double* f;
    Ctl* ctl;
    uint8_t* status;
    uint8_t* mask;
    int32_t* act;
    int32_t* seg;
    int32_t* cnt;
    Rec* rec;
    int32_t* listw;
    int32_t* listz;
    double* coef;
    int32_t* blkcnt;
    int32_t* counts;
    double* part;
    double* sumblk;
    double* out6;
    const float* xin;      // dense values the kernels read (packed)
    uint32_t* bits = nullptr;   // LAY_BITS rows
    uint32_t* col2 = nullptr;   // CSR rows as element pairs (LAY_CSR_TABLE / LAY_CSR_SLOT)
    float* val2 = nullptr;
    int32_t* prp = nullptr;     // first pair of each row
    HtBufs ht{};                // wide CSR: dense head rows for the kernel sums
    int ht_H = 0;               // head columns in use (0: sparse kernel sums only)
    double t_start = 0;         // host clock at the start of the call
    double fx_scale = 1.0, fx_inv = 1.0;
    bool ht_used = false;
    Ctl h{};                // host mirror of ctl
    double ms_step = 0, ms_recon = 0, ms_ksum = 0;
    int64_t recon_pairs = 0;
    int n_launch = 0;
    unsigned long long* work = nullptr;
    StepLds plan_lds{};
    int nseg_max = 0;
    long long nnz_seg_max = 0;
    unsigned long long rows_streamed = 0, nnz_streamed = 0, rows_read = 0, cache_values = 0;
    void* kcache = nullptr;          // kernel-row cache (NULL: off)
    unsigned long long* ktags = nullptr;
    int cache_rows = 0;
    uint32_t epoch = 0;
    int kfull = 0;                   // the cache holds the whole kernel matrix
    double ms_kmatrix = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
    ~Solver() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (ev2) (void)hipEventDestroy(ev2);
        if (ev3) (void)hipEventDestroy(ev3);
    }

    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }

    int read_ctl() {
        HIP_TRY(hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SVM_OK;
    }
    int write_ctl() {
        HIP_TRY(hipMemcpyAsync(ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, s));
        return SVM_OK;
    }

    int select_all() {
        HIP_TRY(launch_select(G, seg, cnt, act, f, alpha, p->y, q->C, rec + 2 * MAX_GRID, ctl, s));
        return read_ctl();
    }

    // The whole kernel matrix into the cache (slot b holds K(b, a) for every a) by the head/tail
    // kernel sums storing their kernel values; left off (the loop computes rows as it goes) when
    // a tile of rows has more tail nonzeros than the kernel's LDS table.
    int fill_kernel_matrix() {
        int rows_t = 0;
        int rc = ht_tile_rows(n, nullptr, ht.tcnt, ht.misc, s, &rows_t);
        if (rc) return rc;
        if (!rows_t) return SVM_OK;
        HIP_TRY(launch_iota(n, listz, s));
        HIP_TRY(hipMemsetAsync(coef, 0, sizeof(double) * (size_t)n, s));
        HtArgs h{};
        h.H = ht_H; h.d = d; h.na = n; h.nb = n;
        h.tile_rows = rows_t;
        h.nsplit = ht_nsplit(n, rows_t, n);
        h.a_head = ht.head;
        h.a_rp = p->row_ptr;
        h.a_col = p->col;
        h.a_val = p->val;
        h.a_nrm = ht.nrm;
        h.alist = nullptr;
        h.b_head = ht.bhead; h.b_nrm = ht.bnrm; h.b_toff = ht.toff; h.b_tent = ht.tent;
        h.coef = coef;
        h.hbits = ht.hbits;
        h.gamma = q->gamma;
        h.fx_scale = fx_scale; h.fx_inv = fx_inv;
        h.part = part;
        h.kout = reinterpret_cast<float*>(kcache);
        h.ldk = n;
        HIP_TRY(hipEventRecord(ev2, s));
        HIP_TRY(launch_ht_pack(n, ht_H, listz, ht.head, ht.nrm, p->row_ptr, p->col, p->val, ht.hmap, ht.tcnt,
                               ht.toff, ht.bhead, ht.bnrm, ht.tent, s));
        HIP_TRY(launch_kernel_sum_ht(h, s));
        HIP_TRY(hipEventRecord(ev3, s));
        HIP_TRY(hipEventSynchronize(ev3));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev2, ev3));
        ms_kmatrix = ms;
        kfull = 1;
        return SVM_OK;
    }

    // f of the rows in `rows` (count from counts[0] or `nrows`) from the support vectors (Alg. 6).
    int kernel_sum_rows(const int32_t* rows, int nrows) {
        if (nrows <= 0) return SVM_OK;
        // support vectors: ascending ids with alpha > 0, coefficient alpha * y
        HIP_TRY(launch_compact(n, 1, mask, alpha, p->y, blkcnt, listz, coef, counts + 1, s));
        int32_t nz = 0;
        HIP_TRY(hipMemcpyAsync(&nz, counts + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (kfull) {
            // the whole kernel matrix is in the cache: the sums read it (the values the loop used)
            const int ns = std::max(1, std::min(NSPLIT_MAX, (1024 + (nrows + 255) / 256 - 1) / ((nrows + 255) / 256)));
            HIP_TRY(hipEventRecord(ev2, s));
            HIP_TRY(launch_kmat_sum(nrows, rows, nz, listz, coef, reinterpret_cast<const float*>(kcache), n, ns, part, s));
            HIP_TRY(hipEventRecord(ev3, s));
            HIP_TRY(launch_finish_sum(nrows, ns, part, rows, p->y, 0.0, f, s));
            HIP_TRY(hipEventSynchronize(ev3));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev2, ev3));
            ms_ksum += ms;
            recon_pairs += (int64_t)nrows * nz;
            return SVM_OK;
        }
        if (ht_H) {
            int rows_t = 0;
            int rc = ht_tile_rows(nrows, rows, ht.tcnt, ht.misc, s, &rows_t);
            if (rc) return rc;
            if (rows_t) {
                HtArgs h{};
                h.H = ht_H; h.d = d; h.na = nrows; h.nb = nz;
                h.tile_rows = rows_t;
                h.nsplit = ht_nsplit(nrows, rows_t, nz);
                h.a_head = ht.head;
                h.a_rp = p->row_ptr;
                h.a_col = p->col;
                h.a_val = p->val;
                h.a_nrm = ht.nrm;
                h.alist = rows;
                h.b_head = ht.bhead; h.b_nrm = ht.bnrm; h.b_toff = ht.toff; h.b_tent = ht.tent;
                h.coef = coef;
                h.hbits = ht.hbits;
                h.gamma = q->gamma;
                h.fx_scale = fx_scale; h.fx_inv = fx_inv;
                h.part = part;
                HIP_TRY(hipEventRecord(ev2, s));
                HIP_TRY(launch_ht_pack(nz, ht_H, listz, ht.head, ht.nrm, p->row_ptr, p->col, p->val, ht.hmap,
                                       ht.tcnt, ht.toff, ht.bhead, ht.bnrm, ht.tent, s));
                HIP_TRY(launch_kernel_sum_ht(h, s));
                HIP_TRY(hipEventRecord(ev3, s));
                HIP_TRY(launch_finish_sum(nrows, h.nsplit, part, rows, p->y, 0.0, f, s));
                HIP_TRY(hipEventSynchronize(ev3));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev2, ev3));
                ms_ksum += ms;
                recon_pairs += (int64_t)nrows * nz;
                ht_used = true;
                return SVM_OK;
            }
            // a tile of 16 rows holds more tail nonzeros than the LDS table: sparse sums below
        }
        SumArgs a{};
        a.lay = lay == LAY_DENSE ? LAY_DENSE : LAY_CSR_TABLE;
        a.d = d;
        a.dpad = dpad;
        a.ax = a.bx = xin;
        a.arp = a.brp = p->row_ptr;
        a.acol = a.bcol = p->col;
        a.aval = a.bval = p->val;
        a.alist = rows;
        a.na = nrows;
        a.blist = listz;
        a.coef = coef;
        a.nb = nz;
        a.gamma = q->gamma;
        const int W = lay == LAY_DENSE ? dpad : d;
        int R = (int)std::min<size_t>(16, (96 * 1024) / (sizeof(float) * (size_t)W));
        int blocks;
        if (lay == LAY_BITS) {
            a.lay = LAY_BITS;
            a.abits = a.bbits = bits;
            a.wpr = bits_wpr(d);
            a.rows_per_block = 16;
            blocks = (nrows + 15) / 16;
        } else if (kernel_sum_uses_mfma(a.lay, dpad, q->kernel_precision)) {
            a.rows_per_block = KSUM_MFMA_ROWS;
            blocks = (nrows + KSUM_MFMA_ROWS - 1) / KSUM_MFMA_ROWS;
        } else if (R < 1) {
            // CSR too wide to stage rows in LDS: slot-map densification, one row per workgroup
            a.lay = LAY_CSR_SLOT;
            a.rows_per_block = max_row_nnz;
            a.slot_rows = slot_rows_for(d, max_row_nnz);
            blocks = std::min((nrows + a.slot_rows - 1) / a.slot_rows, 2048);
        } else {
            a.rows_per_block = R;
            blocks = (nrows + R - 1) / R;
        }
        int ns = std::max(1, std::min(NSPLIT_MAX, (2048 + blocks - 1) / blocks));
        ns = std::min(ns, std::max(1, nz / 256));
        a.nsplit = ns;
        a.part = part;
        HIP_TRY(hipEventRecord(ev2, s));
        HIP_TRY(launch_kernel_sum(a, q->kernel_precision, s));
        HIP_TRY(hipEventRecord(ev3, s));
        HIP_TRY(launch_finish_sum(nrows, ns, part, rows, p->y, 0.0, f, s));
        HIP_TRY(hipEventSynchronize(ev3));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev2, ev3));
        ms_ksum += ms;
        recon_pairs += (int64_t)nrows * nz;
        return SVM_OK;
    }

    int reconstruct_shrunk() {
        double t0 = now_ms();
        HIP_TRY(launch_mark_active(n, G, seg, cnt, act, mask, s));
        HIP_TRY(launch_compact(n, 0, mask, alpha, p->y, blkcnt, listw, nullptr, counts, s));
        int32_t nw = 0;
        HIP_TRY(hipMemcpyAsync(&nw, counts, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int rc = kernel_sum_rows(listw, nw);
        if (rc) return rc;
        HIP_TRY(launch_reset_active(n, G, seg, cnt, act, s));
        HIP_TRY(hipStreamSynchronize(s));
        ms_recon += now_ms() - t0;
        return SVM_OK;
    }

    int recompute_all() {
        double t0 = now_ms();
        int rc = kernel_sum_rows(nullptr, n);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(s));
        ms_recon += now_ms() - t0;
        return SVM_OK;
    }

    int run_loop(double thr, int64_t H) {
        StepArgs a{};
        a.n = n; a.d = d; a.dpad = dpad; a.lay = lay;
        a.x = xin;
        a.bits = bits;
        a.wpr = lay == LAY_BITS ? bits_wpr(d) : 0;
        a.row_ptr = p->row_ptr; a.col = p->col; a.val = p->val;
        a.col2 = col2; a.val2 = val2; a.prp = prp;
        a.pattern_only = pattern_only ? 1 : 0;
        a.max_row_nnz = max_row_nnz;
        a.y = p->y;
        a.alpha = alpha; a.f = f; a.status = status;
        a.act = act; a.seg_start = seg; a.cnt = cnt;
        a.rec = rec; a.ctl = ctl;
        a.C = q->C; a.gamma = q->gamma; a.thr = thr;
        a.max_iter = q->max_iter;
        a.H = H;
        TraceCfg& t = trace_cfg();
        a.trace_cap = t.cap; a.tr_iu = t.iu; a.tr_il = t.il; a.tr_bu = t.bu; a.tr_bl = t.bl;
        a.spin_limit = 500ull * 1000 * 1000;   // 5 s of the 100 MHz wall clock per barrier wait
        a.work = work;
        a.mode = plan_lds.mode;
        a.nseg_max = nseg_max;
        a.nnz_seg_max = (int32_t)nnz_seg_max;
        a.lds_meta_off = (int32_t)plan_lds.meta_off;
        a.lds_pay_off = (int32_t)plan_lds.pay_off;
        a.lds_rec_off = (int32_t)plan_lds.rec_off;
        a.prof = prof_cfg();
        a.cache = kcache;
        a.tags = ktags;
        a.cache_rows = cache_rows;
        a.kfull = kfull;
        a.epoch = ++epoch;   // tags of earlier launches (other active sets) never match
        HIP_TRY(hipEventRecord(ev0, s));
        HIP_TRY(launch_step(a, G, lpr, q->kernel_precision, plan_lds.total, s));
        HIP_TRY(hipEventRecord(ev1, s));
        int rc = read_ctl();
        if (rc) return rc;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
        ms_step += ms;
        std::vector<unsigned long long> w(4 * (size_t)G);
        HIP_TRY(hipMemcpy(w.data(), work, sizeof(unsigned long long) * 4 * G, hipMemcpyDeviceToHost));
        for (int b = 0; b < G; ++b) {
            rows_streamed += w[4 * b];
            nnz_streamed += w[4 * b + 1];
            rows_read += w[4 * b + 2];
            cache_values += w[4 * b + 3];
        }
        ++n_launch;
        return SVM_OK;
    }
};

int64_t heuristic_h(const svm_params_t* q, int n) {
    double h = q->shrink_kind == SVM_KIND_FIXED ? q->shrink_param : std::ceil(q->shrink_param * (double)n);
    if (h < 1) h = 1;
    return (int64_t)h;
}

int finish(Solver& S, int status, int n_recon, svm_result_t* out);

// Everything of a training call before its first loop launch: workspace plan, validation,
// layout (packing, bitsets, head/tail preparation), grid and residency, kernel-row cache, the
// initial state and selection.  S.h then holds the state the loop starts from.
int prepare(Solver& S, const svm_problem_t* p, const svm_params_t* q, double* alpha, double* f_out, void* workspace,
            size_t ws_bytes, hipStream_t s) {
    S.t_start = now_ms();
    S.p = p; S.q = q; S.s = s;
    const int64_t nnz_all = csr_nnz(p, s);
    if (nnz_all < 0) return SVM_EHIP;
    S.plan = make_plan(p, q, nnz_all);
    if (ws_bytes < S.plan.total || ((uintptr_t)workspace & (ALIGN - 1))) return SVM_EWORKSPACE;
    S.ws = (unsigned char*)workspace;
    S.n = p->n; S.d = p->d; S.dpad = dpad_of(p->d);
    S.alpha = alpha;
    S.f = f_out ? f_out : S.at<double>(S.plan.fint);
    S.ctl = S.at<Ctl>(S.plan.ctl);
    S.status = S.at<uint8_t>(S.plan.status);
    S.mask = S.at<uint8_t>(S.plan.mask);
    S.act = S.at<int32_t>(S.plan.act);
    S.seg = S.at<int32_t>(S.plan.seg);
    S.cnt = S.at<int32_t>(S.plan.cnt);
    S.rec = S.at<Rec>(S.plan.rec);
    S.listw = S.at<int32_t>(S.plan.listw);
    S.listz = S.at<int32_t>(S.plan.listz);
    S.coef = S.at<double>(S.plan.coef);
    S.blkcnt = S.at<int32_t>(S.plan.blkcnt);
    S.counts = S.at<int32_t>(S.plan.counts);
    S.part = S.at<double>(S.plan.part);
    S.sumblk = S.at<double>(S.plan.sumblk);
    S.out6 = S.at<double>(S.plan.out6);
    S.work = S.at<unsigned long long>(S.plan.work);
    // records carry iteration tags: clear them so no stale tag of an earlier solve can match
    HIP_TRY(hipMemsetAsync(S.rec, 0, sizeof(Rec) * 2 * MAX_GRID, s));
    HIP_TRY(hipEventCreate(&S.ev0));
    HIP_TRY(hipEventCreate(&S.ev1));
    HIP_TRY(hipEventCreate(&S.ev2));
    HIP_TRY(hipEventCreate(&S.ev3));

    // ---- validate on the device
    HIP_TRY(hipMemsetAsync(S.ctl, 0, CTL_BYTES, s));
    HIP_TRY(launch_validate(p->n, p->d, p->layout, p->x, p->ldx, p->layout == SVM_DENSE_FEATURE_MAJOR, p->row_ptr,
                            p->col, p->val, p->y, S.ctl, s));
    int rc = S.read_ctl();
    if (rc) return rc;
    if (S.h.err & 1) return SVM_EINVAL;
    if (S.h.err & 2) return SVM_ENONFINITE;
    if (S.h.n_pos == 0 || S.h.n_neg == 0) return SVM_EONECLASS;

    if (p->layout == SVM_CSR) {
        S.max_row_nnz = S.h.max_row_nnz;
        int32_t nnz = 0;
        HIP_TRY(hipMemcpyAsync(&nnz, p->row_ptr + p->n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(launch_check_pattern(0, nullptr, S.counts + 2, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(launch_check_pattern(nnz, p->val, S.counts + 2, s));
        int32_t notpat = 1;
        HIP_TRY(hipMemcpyAsync(&notpat, S.counts + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        S.pattern_only = notpat == 0;
        S.lay = p->d <= TABLE_MAX_D ? LAY_CSR_TABLE : LAY_CSR_SLOT;
        if (S.lay == LAY_CSR_SLOT && S.max_row_nnz > SLOT_MAX_NNZ) return SVM_EUNSUPPORTED;
        S.lpr = q->lanes_per_row ? q->lanes_per_row : 1;   // refined with the LDS plan below
        S.xin = nullptr;
        if (S.pattern_only && p->d <= BITS_MAX_D && !(q->flags & SVM_FLAG_NO_BITSETS)) {
            // every value is 1.0: rows as bitsets, dot products as popcounts (exact, so the
            // same values as the column-table path)
            S.lay = LAY_BITS;
            S.lpr = 1;
            S.bits = S.at<uint32_t>(S.plan.bits);
            HIP_TRY(launch_pack_bits(p->n, p->d, bits_wpr(p->d), p->row_ptr, p->col, S.bits, s));
        } else {
            // rows the loop may stream from HBM: u16 column pairs and float2 value pairs (packed
            // below, once the row pointers are on the host)
            S.col2 = S.at<uint32_t>(S.plan.col16);
            S.val2 = S.at<float>(S.plan.val2);
            S.prp = S.at<int32_t>(S.plan.prp);
        }
        if (S.lay == LAY_CSR_SLOT && ht_capable(p) && q->kernel_precision == SVM_KERNEL_FP32 && q->head_cols != -1) {
            // the most frequent columns as dense rows for the matrix cores in the kernel sums
            S.ht_H = q->head_cols ? q->head_cols : HT_H_DEFAULT;
            S.ht.cnt = S.at<int32_t>(S.plan.htcnt);
            S.ht.hmap = S.at<int32_t>(S.plan.hthmap);
            S.ht.hbits = S.at<uint32_t>(S.plan.htbits);
            S.ht.head = S.at<float>(S.plan.hthead);
            S.ht.nrm = S.at<float>(S.plan.htnrm);
            S.ht.tcnt = S.at<int32_t>(S.plan.httcnt);
            S.ht.misc = S.at<int32_t>(S.plan.htmisc);
            S.ht.bhead = S.at<float>(S.plan.htbhead);
            S.ht.bnrm = S.at<float>(S.plan.htbnrm);
            S.ht.toff = S.at<int32_t>(S.plan.httoff);
            S.ht.tent = S.at<uint2>(S.plan.httent);
            if ((rc = ht_choose_head(p, S.ht_H, S.ht, s))) return rc;
            HIP_TRY(hipMemsetAsync(S.ht.misc + 3, 0, sizeof(int32_t), s));
            HIP_TRY(launch_ht_split(p->n, S.ht_H, p->row_ptr, p->col, p->val, S.ht.hmap, S.ht.head, S.ht.nrm,
                                    S.ht.tcnt, (unsigned*)(S.ht.misc + 3), s));
            uint32_t mb = 0;
            HIP_TRY(hipMemcpyAsync(&mb, S.ht.misc + 3, sizeof(mb), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            ht_fixed_point(mb, &S.fx_scale, &S.fx_inv);
        }
    } else {
        S.lay = LAY_DENSE;
        S.lpr = 1;
        S.max_row_nnz = 0;
        float* xp = S.at<float>(S.plan.xpack);
        HIP_TRY(launch_pack_dense(p->n, p->d, S.dpad, p->x, p->ldx, p->layout == SVM_DENSE_FEATURE_MAJOR, xp, s));
        S.xin = xp;
    }

    // ---- grid size and residency: co-resident workgroups (cooperative launch), each owning a
    // segment of about `rows_target` samples, kept in LDS when it fits
    std::vector<int32_t> hrp;
    if (p->layout == SVM_CSR) {
        hrp.resize((size_t)p->n + 1);
        HIP_TRY(hipMemcpyAsync(hrp.data(), p->row_ptr, sizeof(int32_t) * hrp.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (S.col2) {
            // first pair of every row: rows of odd length take one zero element more
            std::vector<int32_t> hprp((size_t)p->n + 1);
            hprp[0] = 0;
            for (int i = 0; i < p->n; ++i) hprp[i + 1] = hprp[i] + (hrp[i + 1] - hrp[i] + 1) / 2;
            HIP_TRY(hipMemcpyAsync(S.prp, hprp.data(), sizeof(int32_t) * hprp.size(), hipMemcpyHostToDevice, s));
            HIP_TRY(launch_pack_pairs(p->n, p->row_ptr, S.prp, p->col, p->val, S.pattern_only ? 1 : 0,
                                      reinterpret_cast<uint16_t*>(S.col2), S.val2, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    const int max_mode = (q->flags & SVM_FLAG_NO_LDS_STATE) ? STEP_GLOBAL
                       : (q->flags & SVM_FLAG_NO_LDS_PAYLOAD) ? STEP_LDS_STATE : STEP_LDS_ALL;
    // Shape rules from per-phase timings of the loop on gfx950: one workgroup (no exchange at
    // all) up to 4096 samples; beyond that about 700 samples per workgroup (at most 11 of the
    // 16 waves hold a row, under three per SIMD), at most one workgroup per CU.  Measured:
    // sparse binary n = 50,000 6.42 / 6.29 us per iteration at G = 63 / 72; whole text-like
    // solves (n = 200,000, row cache) 7.56 / 7.42 / 7.30 / 7.16 / 7.10 s at G = 192 / 208 /
    // 224 / 240 / 256, the records being read in one memory round trip (with two, the exchange
    // grew with G^2 and 224 was best); dense n = 500,000 15.1 us per iteration at G = 245
    // and at 256 (two rows per lane), 16.1 at 224 (three).
    const int cus = std::max(1, device_cu_count());
    int G = q->grid_blocks;
    const TuneClass tclass{TUNE_GRID, S.lay, q->kernel_precision, S.pattern_only, q->shrink_mode != SVM_SHRINK_NONE,
                           p->n, p->d};
    if (!G) G = tuned_shape(tclass);   // measured by svm_autotune for this class
    if (!G) {
        // bitset rows: about 390 samples per workgroup (sparse binary n = 50,000: 5.90 us per
        // iteration and a solve of 0.114 s at G = 128, against 6.18 us and 0.120 s at 71)
        const int per = S.lay == LAY_BITS ? 390 : 700;
        G = p->n <= 4096 ? 1 : std::max(1, std::min(cus, (p->n + per / 2) / per));
    }
    G = std::min(G, p->n);
    const double avg_nnz = p->layout == SVM_CSR ? (double)hrp[p->n] / (double)p->n : 0.0;
    StepLds plan{};
    for (int tries = 0;; ++tries) {
        const int nseg_max = (p->n + G - 1) / G;
        long long nnz_seg_max = 0;
        if (!hrp.empty())
            for (int b = 0; b < G; ++b) {
                const int s0 = (int)(((long long)p->n * b) / G), s1 = (int)(((long long)p->n * (b + 1)) / G);
                nnz_seg_max = std::max<long long>(nnz_seg_max, hrp[s1] - hrp[s0]);
            }
        plan = plan_step_lds(S.lay, S.d, S.dpad, S.max_row_nnz, nseg_max, nnz_seg_max, S.pattern_only, max_mode, G);
        if (plan.total > STEP_LDS_BUDGET) {
            // the records' LDS copy grows with G: where the pair rows leave too little room for
            // it, fewer workgroups (one workgroup has no records at all)
            if (G == 1 || plan.rec_off > STEP_LDS_BUDGET || tries > 8) return SVM_EUNSUPPORTED;
            const size_t rec_room = STEP_LDS_BUDGET - plan.rec_off;
            const int gfit = (int)(rec_room / (sizeof(uint32_t) * REC_LDS_STRIDE)) - 4;
            G = std::max(1, std::min(G - 1, gfit));
            continue;
        }
        if (p->layout == SVM_CSR && S.lay != LAY_BITS && !q->lanes_per_row) {
            // rows in LDS: few lanes per row (short LDS chains, no cross-lane reduction);
            // rows from HBM: enough lanes for coalesced row reads
            int l = 1;
            if (plan.mode == STEP_LDS_ALL) l = avg_nnz < 48 ? 2 : 4;
            else while (l < 32 && 16.0 * l <= avg_nnz) l *= 2;
            S.lpr = l;
        }
        const bool cache = S.plan.cache_rows > 0 && step_cache_capable(S.lay, plan.mode);
        const int maxG = std::min(MAX_GRID, step_max_blocks(S.lay, S.lpr, q->kernel_precision, plan.mode, plan.total,
                                                            cache));
        if (maxG < 1) return SVM_EUNSUPPORTED;
        if (G <= maxG || tries > 4) { G = std::min(G, maxG); break; }
        G = maxG;
    }
    S.G = G;
    S.plan_lds = plan;
    if (S.plan.cache_rows > 0 && step_cache_capable(S.lay, plan.mode) && G <= S.plan.tag_grid) {
        // kernel-row cache: tags zeroed once per solve (launch epochs start at 1)
        S.kcache = S.at<unsigned char>(S.plan.kcache);
        S.ktags = S.at<unsigned long long>(S.plan.ktags);
        S.cache_rows = (int)S.plan.cache_rows;
        HIP_TRY(hipMemsetAsync(S.ktags, 0, sizeof(unsigned long long) * (size_t)S.cache_rows * G, s));
        if ((q->flags & SVM_FLAG_KERNEL_MATRIX) && S.cache_rows == p->n && S.ht_H &&
            q->kernel_precision == SVM_KERNEL_FP32)
            if ((rc = S.fill_kernel_matrix())) return rc;
    }
    last_step_info()[0] = plan.mode;
    last_step_info()[1] = G;
    last_step_info()[2] = S.lpr;
    last_step_info()[3] = S.lay;
    last_step_info()[4] = S.pattern_only ? 1 : 0;
    S.nseg_max = (p->n + G - 1) / G;
    S.nnz_seg_max = 0;
    if (!hrp.empty())
        for (int b = 0; b < G; ++b) {
            const int s0 = (int)(((long long)p->n * b) / G), s1 = (int)(((long long)p->n * (b + 1)) / G);
            S.nnz_seg_max = std::max<long long>(S.nnz_seg_max, hrp[s1] - hrp[s0]);
        }

    // ---- initial state: alpha = 0, f = -y (or the caller's warm start), everything active
    const bool warm = (q->flags & SVM_FLAG_WARM_START) != 0;
    if (warm && !f_out) return SVM_EINVAL;
    HIP_TRY(launch_init_state(p->n, p->y, q->C, warm ? 1 : 0, alpha, S.f, S.status, s));
    HIP_TRY(launch_reset_active(p->n, G, S.seg, S.cnt, S.act, s));
    rc = S.select_all();
    if (rc) return rc;

    const double eps = q->eps;
    bool shrinking = q->shrink_mode != SVM_SHRINK_NONE;
    const int64_t H = shrinking ? heuristic_h(q, p->n) : 0;
    double thr = shrinking ? 20.0 * eps : 2.0 * eps;
    S.h.iter = 0;
    S.h.counter = H;
    S.h.shrink_passes = 0;
    S.h.shrunk_total = 0;
    S.h.abort = 0;
    S.h.cache_both = 0;
    S.h.exit_reason = 0;
    if ((rc = S.write_ctl())) return rc;
    return SVM_OK;
}

int train_impl(const svm_problem_t* p, const svm_params_t* q, double* alpha, double* f_out, svm_result_t* out,
               void* workspace, size_t ws_bytes, hipStream_t s) {
    Solver S{};
    int rc = prepare(S, p, q, alpha, f_out, workspace, ws_bytes, s);
    if (rc) return rc;
    const double eps = q->eps;
    bool shrinking = q->shrink_mode != SVM_SHRINK_NONE;
    const int64_t H = shrinking ? heuristic_h(q, p->n) : 0;
    double thr = shrinking ? 20.0 * eps : 2.0 * eps;
    int status = SVM_OK;
    int n_recon = 0;
    int rechecks = 0;
    const bool final_recompute = q->kernel_precision == SVM_KERNEL_FP32 && !(q->flags & SVM_FLAG_NO_FINAL_RECOMPUTE);
    for (;;) {
        if ((rc = S.run_loop(thr, shrinking ? H : 0))) return rc;
        if (S.h.exit_reason == EXIT_ABORT) return SVM_EABORT;
        if (S.h.exit_reason == EXIT_MAXITER) { status = SVM_NOT_CONVERGED; break; }
        if (shrinking) {
            // the active set meets the tolerance: rebuild f of the shrunk samples (Alg. 6)
            if ((rc = S.reconstruct_shrunk())) return rc;
            ++n_recon;
            Ctl keep = S.h;
            if ((rc = S.select_all())) return rc;
            S.h.iter = keep.iter; S.h.shrink_passes = keep.shrink_passes; S.h.shrunk_total = keep.shrunk_total;
        S.h.cache_both = keep.cache_both;
            S.h.counter = H;
            if (S.h.b_low - S.h.b_up > 2.0 * eps) {
                thr = 2.0 * eps;
                if (q->shrink_mode == SVM_SHRINK_SINGLE) shrinking = false;
                if ((rc = S.write_ctl())) return rc;
                continue;
            }
            if ((rc = S.write_ctl())) return rc;
        }
        if (final_recompute && rechecks < 2) {
            // closing FP64-accumulated recompute of f from alpha (removes FP32 drift), then re-test
            ++rechecks;
            if ((rc = S.recompute_all())) return rc;
            Ctl keep = S.h;
            if ((rc = S.select_all())) return rc;
            S.h.iter = keep.iter; S.h.shrink_passes = keep.shrink_passes; S.h.shrunk_total = keep.shrunk_total;
        S.h.cache_both = keep.cache_both;
            S.h.counter = H;
            if ((rc = S.write_ctl())) return rc;
            if (S.h.b_low - S.h.b_up > 2.0 * eps) {
                thr = 2.0 * eps;
                continue;
            }
        }
        break;
    }
    if (status == SVM_NOT_CONVERGED && S.h.n_active < p->n) {
        if ((rc = S.reconstruct_shrunk())) return rc;
        ++n_recon;
        Ctl keep = S.h;
        if ((rc = S.select_all())) return rc;
        S.h.iter = keep.iter; S.h.shrink_passes = keep.shrink_passes; S.h.shrunk_total = keep.shrunk_total;
        S.h.cache_both = keep.cache_both;
    }

    return finish(S, status, n_recon, out);
}

// ---- several problems over one sample set in lockstep (Alg. 2 for each, rows read once)

struct SharedPlan {
    std::vector<size_t> off, bytes;   // per-problem solver workspaces
    size_t rec = 0, work = 0, total = 0;
};

int shared_plan(const svm_problem_t* x, int k, const int8_t* const* y, const svm_params_t* params, int64_t nnz,
                SharedPlan* P) {
    if (k < 1 || k > SHARED_MAX || !y || !params) return SVM_EINVAL;
    size_t o = 0;
    P->off.assign(k, 0);
    P->bytes.assign(k, 0);
    for (int p = 0; p < k; ++p) {
        svm_problem_t q = *x;
        q.y = y[p];
        int rc = check_problem(&q, true);
        if (rc) return rc;
        if ((rc = check_params(&params[p]))) return rc;
        if (params[p].shrink_mode != SVM_SHRINK_NONE || (params[p].flags & SVM_FLAG_WARM_START) ||
            params[p].kernel_precision != params[0].kernel_precision)
            return SVM_EUNSUPPORTED;
        P->off[p] = o;
        P->bytes[p] = make_plan(&q, &params[p], nnz).total;
        o = align_up(o + P->bytes[p]);
    }
    P->rec = o;
    o = align_up(o + sizeof(Rec) * 2 * SHARED_MAX * SHARED_GRID_MAX);
    P->work = o;
    o = align_up(o + sizeof(unsigned long long) * SHARED_GRID_MAX);
    P->total = o;
    return SVM_OK;
}

int train_shared_impl(const svm_problem_t* x, int k, const int8_t* const* y, const svm_params_t* params,
                      double* const* alpha, double* const* f, svm_result_t* out, unsigned char* ws, size_t ws_bytes,
                      hipStream_t s) {
    const int64_t nnz = csr_nnz(x, s);
    if (nnz < 0) return SVM_EHIP;
    SharedPlan P;
    int rc = shared_plan(x, k, y, params, nnz, &P);
    if (rc) return rc;
    if (ws_bytes < P.total || ((uintptr_t)ws & (ALIGN - 1))) return SVM_EWORKSPACE;
    std::vector<svm_problem_t> probs(k, *x);
    std::vector<std::unique_ptr<Solver>> sv;
    for (int p = 0; p < k; ++p) {
        if (!alpha || !alpha[p]) return SVM_EINVAL;
        probs[p].y = y[p];
        sv.emplace_back(new Solver{});
        if ((rc = prepare(*sv[p], &probs[p], &params[p], alpha[p], f ? f[p] : nullptr, ws + P.off[p], P.bytes[p], s)))
            return rc;
        // rows the shared pass handles: dense, or binary rows kept as bitsets
        if ((sv[p]->lay != LAY_DENSE && sv[p]->lay != LAY_BITS) || sv[p]->lay != sv[0]->lay) return SVM_EUNSUPPORTED;
    }
    const int lay = sv[0]->lay, kprec = params[0].kernel_precision;
    const int n = x->n, d = x->d;
    // about 700 rows per workgroup (at most SHARED_GRID_MAX); each workgroup keeps its segment's
    // rows, f and status in LDS when they fit
    int G = std::max(1, std::min(SHARED_GRID_MAX, n <= 4096 ? 1 : (n + 350) / 700));
    int seg_max = (n + G - 1) / G;
    const size_t lds_res = shared_lds_bytes(lay, d, seg_max, true);
    bool res = lds_res <= STEP_LDS_BUDGET && shared_max_blocks(lay, kprec, true, lds_res) >= G;
    size_t lds = shared_lds_bytes(lay, d, seg_max, res);
    if (lds > STEP_LDS_BUDGET) return SVM_EUNSUPPORTED;
    const int maxG = std::min(SHARED_GRID_MAX, shared_max_blocks(lay, kprec, res, lds));
    if (maxG < 1) return SVM_EUNSUPPORTED;
    if (G > maxG) {   // only without residency, whose LDS does not depend on the segment
        G = maxG;
        seg_max = (n + G - 1) / G;
    }
    Rec* rec = reinterpret_cast<Rec*>(ws + P.rec);
    unsigned long long* work = reinterpret_cast<unsigned long long*>(ws + P.work);
    std::vector<int> status(k, SVM_OK), rechecks(k, 0);
    int running = (1 << k) - 1;
    hipEvent_t e0 = sv[0]->ev0, e1 = sv[0]->ev1;
    while (running) {
        SharedArgs a{};
        a.n = n; a.d = d; a.dpad = dpad_of(d); a.lay = lay;
        a.wpr = lay == LAY_BITS ? bits_wpr(d) : 0;
        a.k = k;
        a.live_mask = running;
        a.seg_max = seg_max;
        a.res = res ? 1 : 0;
        a.x = sv[0]->xin;
        a.bits = sv[0]->bits;
        a.rec = rec;
        a.spin_limit = 500ull * 1000 * 1000;   // 5 s of the 100 MHz wall clock per record wait
        a.work = work;
        for (int p = 0; p < k; ++p) {
            SharedProb& b = a.prob[p];
            b.y = y[p]; b.alpha = alpha[p]; b.f = sv[p]->f; b.status = sv[p]->status; b.ctl = sv[p]->ctl;
            b.C = params[p].C; b.gamma = params[p].gamma; b.thr = 2.0 * params[p].eps; b.max_iter = params[p].max_iter;
        }
        HIP_TRY(hipMemsetAsync(rec, 0, sizeof(Rec) * 2 * SHARED_MAX * G, s));
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(launch_shared(a, G, kprec, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        std::vector<unsigned long long> w(G);
        HIP_TRY(hipMemcpy(w.data(), work, sizeof(unsigned long long) * G, hipMemcpyDeviceToHost));
        unsigned long long rows = 0;
        for (int b = 0; b < G; ++b) rows += w[b];
        const int launched = running;
        for (int p = 0; p < k; ++p) {
            if (!((launched >> p) & 1)) continue;
            Solver& S = *sv[p];
            S.ms_step += ms;
            S.rows_streamed += rows;
            S.rows_read += rows;
            S.G = G;
            ++S.n_launch;
            if ((rc = S.read_ctl())) return rc;
            if (S.h.exit_reason == EXIT_ABORT) return SVM_EABORT;
            if (S.h.exit_reason == EXIT_MAXITER) { status[p] = SVM_NOT_CONVERGED; running &= ~(1 << p); continue; }
            const bool final_recompute = kprec == SVM_KERNEL_FP32 && !(params[p].flags & SVM_FLAG_NO_FINAL_RECOMPUTE);
            if (final_recompute && rechecks[p] < 2) {
                // the closing FP64-accumulated recompute of f and re-test of the single-problem driver
                ++rechecks[p];
                if ((rc = S.recompute_all())) return rc;
                Ctl keep = S.h;
                if ((rc = S.select_all())) return rc;
                S.h.iter = keep.iter; S.h.shrink_passes = keep.shrink_passes; S.h.shrunk_total = keep.shrunk_total;
                S.h.cache_both = keep.cache_both;
                S.h.counter = 0;
                if ((rc = S.write_ctl())) return rc;
                if (S.h.b_low - S.h.b_up > 2.0 * params[p].eps) continue;   // more iterations
            }
            running &= ~(1 << p);
        }
    }
    int first = SVM_OK;
    for (int p = 0; p < k; ++p) {
        rc = finish(*sv[p], status[p], 0, out ? &out[p] : nullptr);
        if (rc && !first) first = rc;
    }
    return first;
}

// The threshold, dual objective and counts of a finished solve into `out` (host struct).
int finish(Solver& S, int status, int n_recon, svm_result_t* out) {
    const svm_problem_t* p = S.p;
    const svm_params_t* q = S.q;
    double* alpha = S.alpha;
    hipStream_t s = S.s;
    const double t_start = S.t_start;
    HIP_TRY(launch_summary(p->n, alpha, S.f, p->y, q->C, S.sumblk, S.out6, s));
    double v6[6];
    HIP_TRY(hipMemcpyAsync(v6, S.out6, sizeof(v6), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (out) {
        memset(out, 0, sizeof(*out));
        out->beta = v6[1] > 0 ? v6[0] / v6[1] : 0.5 * (S.h.b_up + S.h.b_low);
        out->b_up = S.h.b_up;
        out->b_low = S.h.b_low;
        out->dual_obj = v6[2] - 0.5 * v6[3];
        out->iterations = S.h.iter;
        out->n_sv = (int32_t)v6[4];
        out->n_bsv = (int32_t)v6[5];
        out->n_recon = n_recon;
        out->status = status;
        out->shrink_passes = S.h.shrink_passes;
        out->shrunk_total = S.h.shrunk_total;
        out->n_launches = S.n_launch;
        out->grid_blocks = S.G;
        out->ms_total = now_ms() - t_start;
        out->ms_step = S.ms_step;
        out->ms_recon = S.ms_recon;
        out->ms_ksum = S.ms_ksum;
        out->recon_pairs = S.recon_pairs;
        out->ksum_mfma = kernel_sum_uses_mfma(S.lay == LAY_DENSE ? LAY_DENSE : LAY_CSR_TABLE, S.dpad,
                                              q->kernel_precision) ? 1 : S.ht_used ? 2 : 0;
        out->head_cols = S.ht_used ? S.ht_H : 0;
        out->rows_streamed = (int64_t)S.rows_streamed;
        out->rows_read = (int64_t)S.rows_read;
        out->cache_values = (int64_t)S.cache_values;
        out->cache_rows = S.cache_rows;
        out->cache_both = S.h.cache_both;
        out->kernel_matrix = S.kfull;
        out->ms_kmatrix = S.ms_kmatrix;
        out->nnz_streamed = (int64_t)S.nnz_streamed;
        out->pattern_only = S.pattern_only ? 1 : 0;
        out->lanes_per_row = S.lpr;
    }
    return status;
}



// ---- classifier (eq:classi): scratch plan and the kernel sums over the support vectors

int check_decision_args(const svm_problem_t* train, const svm_problem_t* queries, int kprec) {
    int rc = check_problem(train, true);
    if (rc) return rc;
    if ((rc = check_problem(queries, false))) return rc;
    if (queries->d != train->d) return SVM_EINVAL;
    if ((train->layout == SVM_CSR) != (queries->layout == SVM_CSR)) return SVM_EINVAL;
    if (kprec != SVM_KERNEL_FP32 && kprec != SVM_KERNEL_FP64) return SVM_EINVAL;
    return SVM_OK;
}

struct DecPlan {
    size_t ctl, xt, xq, lz, cf, bc, ct, pt, tbits, qbits, htcnt, hthmap, htbits, thead, tnrm, ttcnt, qhead, qnrm, qtcnt,
        htmisc, bhead, bnrm, toff, tent, total;
};

DecPlan make_dec_plan(const svm_problem_t* train, const svm_problem_t* queries, int64_t train_nnz) {
    const size_t n = (size_t)train->n, nq = (size_t)queries->n;
    const int d = train->d, dpad = dpad_of(d);
    const bool dense = train->layout != SVM_CSR;
    const bool bits = !dense && d <= BITS_MAX_D;
    const bool ht = ht_capable(train);
    DecPlan q{};
    size_t o = 0;
    auto take = [&](size_t b) { size_t at = o; o = align_up(o + b); return at; };
    q.ctl = take(2 * CTL_BYTES);
    q.xt = take(dense ? sizeof(float) * n * dpad : 0);
    q.xq = take(dense ? sizeof(float) * nq * dpad : 0);
    q.lz = take(sizeof(int32_t) * n);
    q.cf = take(sizeof(double) * n);
    q.bc = take(sizeof(int32_t) * (n / 1024 + 4));
    q.ct = take(64);
    q.pt = take(sizeof(double) * nq * NSPLIT_MAX);
    q.tbits = take(bits ? sizeof(uint32_t) * n * bits_wpr(d) : 0);
    q.qbits = take(bits ? sizeof(uint32_t) * nq * bits_wpr(d) : 0);
    q.htcnt = take(ht ? sizeof(int32_t) * (size_t)d : 0);
    q.hthmap = take(ht ? sizeof(int32_t) * (size_t)d : 0);
    q.htbits = take(ht ? sizeof(uint32_t) * HT_MAX_WORDS : 0);
    q.thead = take(ht ? sizeof(float) * n * HT_H_DEFAULT : 0);
    q.tnrm = take(ht ? sizeof(float) * n : 0);
    q.ttcnt = take(ht ? sizeof(int32_t) * n : 0);
    q.qhead = take(ht ? sizeof(float) * nq * HT_H_DEFAULT : 0);
    q.qnrm = take(ht ? sizeof(float) * nq : 0);
    q.qtcnt = take(ht ? sizeof(int32_t) * nq : 0);
    q.htmisc = take(ht ? 64 : 0);
    q.bhead = take(ht ? sizeof(float) * (n + HT_CHUNK) * HT_H_DEFAULT : 0);
    q.bnrm = take(ht ? sizeof(float) * (n + HT_CHUNK) : 0);
    q.toff = take(ht ? sizeof(int32_t) * (n + 1) : 0);
    q.tent = take(ht ? sizeof(uint2) * (size_t)std::max<int64_t>(train_nnz, 0) : 0);
    q.total = o;
    return q;
}

// Are all CSR values 1.0 (host result; the flag word is device scratch)?
int csr_pattern_only(const svm_problem_t* p, int32_t* flag, hipStream_t s, bool* yes) {
    int32_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, p->row_ptr + p->n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(launch_check_pattern(nnz, p->val, flag, s));
    int32_t notpat = 1;
    HIP_TRY(hipMemcpyAsync(&notpat, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *yes = notpat == 0;
    return SVM_OK;
}

int decision_impl(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                  const svm_problem_t* queries, double* out, int kprec, unsigned char* ws, size_t ws_bytes,
                  hipStream_t s) {
    const int64_t tnnz = csr_nnz(train, s);
    if (tnnz < 0) return SVM_EHIP;
    const DecPlan P = make_dec_plan(train, queries, tnnz);
    if (ws_bytes < P.total || ((uintptr_t)ws & (ALIGN - 1))) return SVM_EWORKSPACE;
    const int n = train->n, nq = queries->n, d = train->d, dpad = dpad_of(d);
    const bool dense = train->layout != SVM_CSR;
    float* xt = (float*)(ws + P.xt);
    float* xq = (float*)(ws + P.xq);
    int32_t* lz = (int32_t*)(ws + P.lz);
    double* cf = (double*)(ws + P.cf);
    int32_t* bc = (int32_t*)(ws + P.bc);
    int32_t* ct = (int32_t*)(ws + P.ct);
    double* pt = (double*)(ws + P.pt);
    // both sample sets are validated first (labels, CSR structure, finite values)
    Ctl* ctl = (Ctl*)(ws + P.ctl);
    HIP_TRY(hipMemsetAsync(ctl, 0, 2 * CTL_BYTES, s));
    HIP_TRY(launch_validate(n, d, train->layout, train->x, train->ldx, train->layout == SVM_DENSE_FEATURE_MAJOR,
                            train->row_ptr, train->col, train->val, train->y, ctl, s));
    Ctl* ctlq = (Ctl*)(ws + P.ctl + CTL_BYTES);
    HIP_TRY(launch_validate(nq, d, queries->layout, queries->x, queries->ldx,
                            queries->layout == SVM_DENSE_FEATURE_MAJOR, queries->row_ptr, queries->col, queries->val,
                            nullptr, ctlq, s));
    Ctl hv[2];
    HIP_TRY(hipMemcpyAsync(&hv[0], ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hv[1], ctlq, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((hv[0].err | hv[1].err) & 1) return SVM_EINVAL;
    if ((hv[0].err | hv[1].err) & 2) return SVM_ENONFINITE;
    if (dense) {
        HIP_TRY(launch_pack_dense(n, d, dpad, train->x, train->ldx, train->layout == SVM_DENSE_FEATURE_MAJOR, xt, s));
        HIP_TRY(launch_pack_dense(nq, d, dpad, queries->x, queries->ldx, queries->layout == SVM_DENSE_FEATURE_MAJOR,
                                  xq, s));
    }
    // support vectors: ascending ids with alpha > 0, coefficient alpha * y
    HIP_TRY(launch_compact(n, 1, nullptr, alpha, train->y, bc, lz, cf, ct, s));
    int32_t nz = 0;
    HIP_TRY(hipMemcpyAsync(&nz, ct, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    SumArgs a{};
    a.lay = dense ? LAY_DENSE : LAY_CSR_TABLE;
    a.d = d; a.dpad = dpad;
    a.ax = xq; a.arp = queries->row_ptr; a.acol = queries->col; a.aval = queries->val;
    a.alist = nullptr; a.na = nq;
    a.bx = xt; a.brp = train->row_ptr; a.bcol = train->col; a.bval = train->val;
    a.blist = lz; a.coef = cf; a.nb = nz;
    a.gamma = gamma;
    a.part = pt;
    int blocks = 0;
    if (!dense && d <= BITS_MAX_D) {
        // binary rows on both sides: bitsets and popcounts (exact squared distances)
        bool tp = false, qp = false;
        int rc = csr_pattern_only(train, ct + 2, s, &tp);
        if (rc) return rc;
        if (tp && (rc = csr_pattern_only(queries, ct + 3, s, &qp))) return rc;
        if (tp && qp) {
            a.lay = LAY_BITS;
            a.wpr = bits_wpr(d);
            a.abits = (uint32_t*)(ws + P.qbits);
            a.bbits = (uint32_t*)(ws + P.tbits);
            HIP_TRY(launch_pack_bits(nq, d, a.wpr, queries->row_ptr, queries->col, (uint32_t*)a.abits, s));
            HIP_TRY(launch_pack_bits(n, d, a.wpr, train->row_ptr, train->col, (uint32_t*)a.bbits, s));
            a.rows_per_block = 16;
            blocks = (nq + 15) / 16;
        }
    }
    if (!dense && a.lay != LAY_BITS && ht_capable(train) && kprec == SVM_KERNEL_FP32) {
        // wide rows: the most frequent training columns as dense rows on the matrix cores
        HtBufs b{};
        b.cnt = (int32_t*)(ws + P.htcnt);
        b.hmap = (int32_t*)(ws + P.hthmap);
        b.hbits = (uint32_t*)(ws + P.htbits);
        b.misc = (int32_t*)(ws + P.htmisc);
        const int H = HT_H_DEFAULT;
        float* thead = (float*)(ws + P.thead);
        float* tnrm = (float*)(ws + P.tnrm);
        int32_t* ttcnt = (int32_t*)(ws + P.ttcnt);
        float* qhead = (float*)(ws + P.qhead);
        float* qnrm = (float*)(ws + P.qnrm);
        int32_t* qtcnt = (int32_t*)(ws + P.qtcnt);
        int rc = ht_choose_head(train, H, b, s);
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(b.misc + 3, 0, sizeof(int32_t), s));
        HIP_TRY(launch_ht_split(n, H, train->row_ptr, train->col, train->val, b.hmap, thead, tnrm, ttcnt,
                                (unsigned*)(b.misc + 3), s));
        HIP_TRY(launch_ht_split(nq, H, queries->row_ptr, queries->col, queries->val, b.hmap, qhead, qnrm, qtcnt,
                                (unsigned*)(b.misc + 3), s));
        uint32_t mb = 0;
        HIP_TRY(hipMemcpyAsync(&mb, b.misc + 3, sizeof(mb), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int rows_t = 0;
        if ((rc = ht_tile_rows(nq, nullptr, qtcnt, b.misc, s, &rows_t))) return rc;
        if (rows_t) {
            HtArgs h{};
            h.H = H; h.d = d; h.na = nq; h.nb = nz;
            h.tile_rows = rows_t;
            h.nsplit = ht_nsplit(nq, rows_t, nz);
            h.a_head = qhead; h.a_rp = queries->row_ptr; h.a_col = queries->col; h.a_val = queries->val; h.a_nrm = qnrm;
            h.alist = nullptr;
            h.b_head = (float*)(ws + P.bhead); h.b_nrm = (float*)(ws + P.bnrm);
            h.b_toff = (int32_t*)(ws + P.toff); h.b_tent = (uint2*)(ws + P.tent);
            h.coef = cf;
            h.hbits = b.hbits;
            h.gamma = gamma;
            ht_fixed_point(mb, &h.fx_scale, &h.fx_inv);
            h.part = pt;
            HIP_TRY(launch_ht_pack(nz, H, lz, thead, tnrm, train->row_ptr, train->col, train->val, b.hmap, ttcnt,
                                   (int32_t*)h.b_toff, (float*)h.b_head, (float*)h.b_nrm, (uint2*)h.b_tent, s));
            HIP_TRY(launch_kernel_sum_ht(h, s));
            HIP_TRY(launch_finish_sum(nq, h.nsplit, pt, nullptr, nullptr, beta, out, s));
            HIP_TRY(hipStreamSynchronize(s));
            return SVM_OK;
        }
        // a tile of 16 query rows holds more tail nonzeros than the LDS table: sparse sums below
    }
    if (a.lay != LAY_BITS) {
        const int W = dense ? dpad : d;
        const int R = (int)std::min<size_t>(16, (96 * 1024) / (sizeof(float) * (size_t)W));
        if (kernel_sum_uses_mfma(a.lay, dpad, kprec)) {
            a.rows_per_block = KSUM_MFMA_ROWS;
            blocks = (nq + KSUM_MFMA_ROWS - 1) / KSUM_MFMA_ROWS;
        } else if (R < 1) {
            // wide CSR queries: slot-map densification of groups of query rows (longest row from
            // the validation pass)
            const int mx = hv[1].max_row_nnz;
            if (mx > SLOT_MAX_NNZ) return SVM_EUNSUPPORTED;
            a.lay = LAY_CSR_SLOT;
            a.rows_per_block = mx;
            a.slot_rows = slot_rows_for(d, mx);
            blocks = std::min((nq + a.slot_rows - 1) / a.slot_rows, 2048);
        } else {
            a.rows_per_block = R;
            blocks = (nq + R - 1) / R;
        }
    }
    int ns = std::max(1, std::min(NSPLIT_MAX, (2048 + blocks - 1) / blocks));
    ns = std::min(ns, std::max(1, nz / 256));
    a.nsplit = ns;
    HIP_TRY(launch_kernel_sum(a, kprec, s));
    HIP_TRY(launch_finish_sum(nq, ns, pt, nullptr, nullptr, beta, out, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SVM_OK;
}

}  // namespace

unsigned long long* svm::debug_profile_slots() { return prof_cfg(); }

void svm::set_last_hip_error(hipError_t e) { last_hip_error() = e; }

int svm::decision_in_workspace(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                               const svm_problem_t* queries, double* out, int kprec, void* ws, size_t ws_bytes,
                               hipStream_t s, size_t* need) {
    int rc = check_decision_args(train, queries, kprec);
    if (rc) return rc;
    if (!alpha || !out || !ws || !(gamma > 0) || !std::isfinite(gamma)) return SVM_EINVAL;
    const int64_t nnz = csr_nnz(train, s);
    if (nnz < 0) return SVM_EHIP;
    *need = make_dec_plan(train, queries, nnz).total;
    if (*need > ws_bytes) return SVM_EWORKSPACE;
    return decision_impl(train, alpha, beta, gamma, queries, out, kprec, (unsigned char*)ws, ws_bytes, s);
}

extern "C" {

size_t svm_train_workspace_size(const svm_problem_t* prob, const svm_params_t* params) {
    if (check_problem(prob, true) || check_params(params)) return 0;
    const int64_t nnz = csr_nnz(prob, nullptr);
    return nnz < 0 ? 0 : make_plan(prob, params, nnz).total;
}

int svm_train(const svm_problem_t* prob, const svm_params_t* params, double* alpha, double* f, svm_result_t* out,
              void* workspace, size_t ws_bytes, void* stream) {
    int rc = check_problem(prob, true);
    if (rc) return rc;
    if ((rc = check_params(params))) return rc;
    if (!alpha) return SVM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    void* own = nullptr;
    if (!workspace) {
        const int64_t nnz = csr_nnz(prob, s);
        if (nnz < 0) return SVM_EHIP;
        ws_bytes = make_plan(prob, params, nnz).total;
        if (hipMalloc(&own, ws_bytes) != hipSuccess) return SVM_ENOMEM;
        workspace = own;
    }
    rc = train_impl(prob, params, alpha, f, out, workspace, ws_bytes, s);
    if (own) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(own);
    }
    return rc;
}

size_t svm_train_shared_workspace_size(const svm_problem_t* x, int32_t k, const int8_t* const* y,
                                       const svm_params_t* params) {
    if (!x) return 0;
    const int64_t nnz = csr_nnz(x, nullptr);
    SharedPlan P;
    if (nnz < 0 || shared_plan(x, k, y, params, nnz, &P)) return 0;
    return P.total;
}

int svm_train_shared(const svm_problem_t* x, int32_t k, const int8_t* const* y, const svm_params_t* params,
                     double* const* alpha, double* const* f, svm_result_t* out, void* workspace, size_t ws_bytes,
                     void* stream) {
    if (!x) return SVM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (workspace)
        return train_shared_impl(x, k, y, params, alpha, f, out, (unsigned char*)workspace, ws_bytes, s);
    const int64_t nnz = csr_nnz(x, s);
    if (nnz < 0) return SVM_EHIP;
    SharedPlan P;
    int rc = shared_plan(x, k, y, params, nnz, &P);
    if (rc) return rc;
    void* own = nullptr;
    if (hipMalloc(&own, P.total) != hipSuccess) return SVM_ENOMEM;
    rc = train_shared_impl(x, k, y, params, alpha, f, out, (unsigned char*)own, P.total, s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(own);
    return rc;
}

size_t svm_decision_workspace_size(const svm_problem_t* train, const svm_problem_t* queries, int32_t kernel_precision) {
    if (check_decision_args(train, queries, kernel_precision)) return 0;
    const int64_t nnz = csr_nnz(train, nullptr);
    return nnz < 0 ? 0 : make_dec_plan(train, queries, nnz).total;
}

int svm_decision(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                 const svm_problem_t* queries, double* out, int32_t kernel_precision, void* workspace,
                 size_t ws_bytes, void* stream) {
    int rc = check_decision_args(train, queries, kernel_precision);
    if (rc) return rc;
    if (!alpha || !out || !(gamma > 0) || !std::isfinite(gamma)) return SVM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (workspace) return decision_impl(train, alpha, beta, gamma, queries, out, kernel_precision,
                                        (unsigned char*)workspace, ws_bytes, s);
    const int64_t nnz = csr_nnz(train, s);
    if (nnz < 0) return SVM_EHIP;
    const size_t bytes = make_dec_plan(train, queries, nnz).total;
    unsigned char* buf = nullptr;
    HIP_TRY(hipMallocAsync((void**)&buf, bytes, s));
    rc = decision_impl(train, alpha, beta, gamma, queries, out, kernel_precision, buf, bytes, s);
    (void)hipFreeAsync(buf, s);
    (void)hipStreamSynchronize(s);
    return rc;
}

int svm_autotune(const svm_problem_t* prob, const svm_params_t* params, int32_t target, svm_tune_t* out,
                 void* stream) {
    int rc = check_problem(prob, true);
    if (rc) return rc;
    if ((rc = check_params(params))) return rc;
    if ((target != SVM_TUNE_GRID && target != SVM_TUNE_TEAM) || (params->flags & SVM_FLAG_WARM_START))
        return SVM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = prob->n;
    // trial solves: the problem's first iterations, no closing recompute
    svm_params_t q = *params;
    q.max_iter = std::min<int64_t>(params->max_iter, 300);
    q.flags |= SVM_FLAG_NO_FINAL_RECOMPUTE;
    q.cache_mb = 0;
    double* alpha = nullptr;
    double* f = nullptr;
    void* ws = nullptr;
    if (hipMalloc((void**)&alpha, sizeof(double) * n) != hipSuccess) return SVM_ENOMEM;
    if (hipMalloc((void**)&f, sizeof(double) * n) != hipSuccess) { (void)hipFree(alpha); return SVM_ENOMEM; }
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        if (ws) (void)hipFree(ws);
        (void)hipFree(f);
        (void)hipFree(alpha);
    };
    std::vector<int> cand;
    auto add = [&](int v) {
        v = std::max(1, v);
        if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
    };
    svm_result_t r{};
    int lay = 0, pattern = 0;
    if (target == SVM_TUNE_GRID) {
        const int cus = std::max(1, device_cu_count());
        const int g0 = n <= 4096 ? 1 : std::max(1, std::min(cus, (n + 350) / 700));
        for (int v : {g0 / 2, (3 * g0) / 4, g0, std::min(cus, (5 * g0) / 4), std::min(cus, (3 * g0) / 2)})
            if (v <= n) add(v);
        q.grid_blocks = cand.back();
        const size_t bytes = svm_train_workspace_size(prob, &q);
        if (!bytes || hipMalloc(&ws, bytes) != hipSuccess) { cleanup(); return SVM_ENOMEM; }
    } else {
        // the team rule needs the nonzero count and whether every value is 1.0: one trial
        // solve on the automatic team tells the layout
        q.grid_blocks = 0;
        rc = svm_train_batch(1, prob, &q, &alpha, &f, &r, stream);
        if (rc < 0) { cleanup(); return rc; }
        const int64_t nnz = csr_nnz(prob, s);
        bool pat = false;
        if (prob->layout == SVM_CSR && (rc = csr_pattern_only(prob, reinterpret_cast<int32_t*>(f), s, &pat))) {
            cleanup();
            return rc;
        }
        const int t0 = batch_team_rule(prob, (int)std::max<int64_t>(nnz, 0), pat);
        for (int v : {t0 / 2, t0, 2 * t0})
            if (v <= TEAM_MAX) add(v);
        lay = batch_layout(prob, pat);
        pattern = pat ? 1 : 0;
    }
    if (out) {
        memset(out, 0, sizeof(*out));
        out->target = target;
    }
    double best = 0.0;
    int chosen = 0;
    std::vector<std::pair<int, double>> shape_us;
    const int nc = std::min<int>((int)cand.size(), 8);
    for (int c = 0; c < nc; ++c) {
        q.grid_blocks = cand[c];
        double us = 0.0;
        for (int rep = 0; rep < 2; ++rep) {   // the second run is timed
            if (target == SVM_TUNE_GRID) rc = train_impl(prob, &q, alpha, f, &r, ws, svm_train_workspace_size(prob, &q), s);
            else rc = svm_train_batch(1, prob, &q, &alpha, &f, &r, stream);
            if (rc < 0) { cleanup(); return rc; }
            us = r.iterations > 0 ? r.ms_step * 1e3 / (double)r.iterations : 0.0;
        }
        const int used = r.grid_blocks;
        if (target == SVM_TUNE_GRID) {
            lay = last_step_info()[3];
            pattern = last_step_info()[4];
        }
        if (out) { out->shape[c] = used; out->us_per_iter[c] = us; }
        shape_us.push_back({used, us});
        if (!chosen || us < best) { best = us; chosen = used; }
    }
    cleanup();
    if (target == SVM_TUNE_TEAM) {
        // teams share the launch with other problems: the fewest workgroup-microseconds per
        // iteration among the shapes within 1.5x of the fastest one's time per iteration
        double cost = 0.0;
        for (const auto& c : shape_us)
            if (c.second <= 1.5 * best && (cost == 0.0 || c.first * c.second < cost)) {
                cost = c.first * c.second;
                chosen = c.first;
            }
    }
    const TuneClass tc{target == SVM_TUNE_GRID ? TUNE_GRID : TUNE_TEAM, lay, params->kernel_precision, pattern != 0,
                       params->shrink_mode != SVM_SHRINK_NONE, n, prob->d};
    set_tuned_shape(tc, chosen);
    if (out) {
        out->n_candidates = nc;
        out->chosen = chosen;
    }
    return SVM_OK;
}

int svm_autotune_reset(void) {
    clear_tuned_shapes();
    return SVM_OK;
}

int svm_debug_select(int32_t n_active, const int32_t* active, const double* f, const double* alpha, const int8_t* y,
                     double C, int32_t num_blocks, double* b_up, int32_t* i_up, double* b_low, int32_t* i_low,
                     void* stream) {
    if (n_active < 0 || !active || !f || !alpha || !y || !(C > 0) || num_blocks < 0 || num_blocks > MAX_GRID)
        return SVM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int G = num_blocks ? num_blocks : std::max(1, std::min(MAX_GRID, (n_active + 1023) / 1024));
    std::vector<int32_t> seg(G + 1), cnt(G);
    for (int b = 0; b <= G; ++b) seg[b] = (int32_t)(((int64_t)n_active * b) / G);
    for (int b = 0; b < G; ++b) cnt[b] = seg[b + 1] - seg[b];
    size_t bytes = align_up(sizeof(Ctl)) + align_up(sizeof(Rec) * G) + align_up(sizeof(int32_t) * (2 * G + 1));
    unsigned char* buf = nullptr;
    HIP_TRY(hipMallocAsync((void**)&buf, bytes, s));
    Ctl* ctl = (Ctl*)buf;
    Rec* rec = (Rec*)(buf + align_up(sizeof(Ctl)));
    int32_t* dseg = (int32_t*)(buf + align_up(sizeof(Ctl)) + align_up(sizeof(Rec) * G));
    int32_t* dcnt = dseg + G + 1;
    hipError_t e = hipMemcpyAsync(dseg, seg.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcnt, cnt.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_select(G, dseg, dcnt, active, f, alpha, y, C, rec, ctl, s);
    Ctl h{};
    if (e == hipSuccess) e = hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(buf, s);
    (void)hipStreamSynchronize(s);
    if (e != hipSuccess) { last_hip_error() = e; return SVM_EHIP; }
    *b_up = h.b_up; *i_up = h.i_up; *b_low = h.b_low; *i_low = h.i_low;
    return SVM_OK;
}

int svm_debug_set_trace(int64_t cap, int32_t* i_up, int32_t* i_low, double* b_up, double* b_low) {
    if (cap < 0 || (cap > 0 && (!i_up || !i_low || !b_up || !b_low))) return SVM_EINVAL;
    TraceCfg& t = trace_cfg();
    t.cap = cap; t.iu = i_up; t.il = i_low; t.bu = b_up; t.bl = b_low;
    return SVM_OK;
}

int svm_debug_set_profile(uint64_t* slots) {
    prof_cfg() = reinterpret_cast<unsigned long long*>(slots);
    return SVM_OK;
}

int svm_debug_step_info(int32_t* mode, int32_t* grid_blocks, int32_t* lanes_per_row) {
    if (mode) *mode = last_step_info()[0];
    if (grid_blocks) *grid_blocks = last_step_info()[1];
    if (lanes_per_row) *lanes_per_row = last_step_info()[2];
    return SVM_OK;
}

const char* svm_strerror(int code) {
    switch (code) {
        case SVM_OK: return "ok";
        case SVM_NOT_CONVERGED: return "iteration cap reached before the KKT tolerance (state is consistent)";
        case SVM_EINVAL: return "invalid argument (sizes, C/gamma/eps, labels or CSR structure)";
        case SVM_EONECLASS: return "only one class present in the labels";
        case SVM_ENONFINITE: return "NaN or Inf in the sample values";
        case SVM_EWORKSPACE: return "workspace too small or not 256-byte aligned";
        case SVM_EHIP: return hipGetErrorString(last_hip_error());
        case SVM_EUNSUPPORTED: return "problem shape not supported by this library";
        case SVM_ENOMEM: return "device allocation failed or memory budget exhausted";
        case SVM_EBUSY: return "ticket still queued or running";
        case SVM_EABORT: return "device loop stopped by its barrier watchdog";
        case SVM_ESCRATCH: return "the problem needs more scratch than the 96 MiB built-in array of svm_decision_noalloc";
        default: return "unknown status code";
    }
}

int svm_version(void) { return 100; }

}  // extern "C"

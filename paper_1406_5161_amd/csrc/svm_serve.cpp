// svm_serve.cpp -- batched training (svm_train_batch) and the serving loop
// (svm_server_*): continuous batching of SVM training problems on one GPU.
//
// Both run the persistent batched kernel of svm_batch.hip, in which a team of
// one to TEAM_MAX workgroups solves one problem (sized so each member's share
// of the samples fits its LDS when that is possible).  Each
// workgroup takes worker tickets; ticket t names a descriptor slot and a rank
// in that problem's team, and the tickets of one problem are consecutive.  The
// batch entry point hands the kernel a fixed ticket table; the server keeps the
// kernel running and publishes descriptors and tickets into rings in pinned
// host memory as problems are admitted.  Admission needs a free slot (at most
// max_slots problems in flight) and room for the problem's solver state in the
// server's device-memory arena; otherwise the problem waits in a FIFO and is
// admitted when a running one completes.  Prepared problems are published
// largest estimated work first while the kernel has fewer untaken tickets than
// workgroups (see start_solves).  A monitor thread admits waiting problems as
// others complete and parks the kernel after 2 s without work.
//
// Progress of teams: tickets are taken in order and a problem's tickets are
// consecutive, so the oldest partly taken problem always has its missing
// members among the workgroups that finish the problems before it; with at
// least as many workgroups as the largest team, every team fills.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "svm_internal.h"

using namespace svm;

namespace {

constexpr size_t SALIGN = 256;
size_t al(size_t v) { return (v + SALIGN - 1) & ~(SALIGN - 1); }
int dpad4(int d) { return (d + 3) & ~3; }
double al16(double v) { return std::ceil(v / 16.0) * 16.0; }

// ---- shape autotuning: lanes per row of the batched loop.
// Rules measured on gfx950 for one workgroup per problem: enough lanes that a
// row is read with a few 16-byte loads per lane (dense) or about 8 nonzeros per
// lane (CSR); FP64 dense keeps one lane per row so the distance is summed in
// feature order.
int tune_lanes_per_row(const svm_problem_t* p, double avg_nnz, int kprec, int requested) {
    if (requested) return requested;
    int l = 1;
    if (p->layout == SVM_CSR) {
        while (l < 16 && 8.0 * 2 * l <= avg_nnz) l *= 2;
    } else {
        if (kprec == SVM_KERNEL_FP64) return 1;
        const int f4 = dpad4(p->d) / 4;
        while (l < 16 && 8 * 2 * l <= f4) l *= 2;
    }
    return l;
}

// CSR problems narrow enough for bitset rows (used when every value is 1.0).
bool bits_capable(const svm_problem_t* p) { return p->layout == SVM_CSR && p->d <= BITS_MAX_D; }

// Solver state of one problem: a base part that does not depend on the team size (packed
// dense rows, f, status, active and work lists, team records for `rec_members` members) and a
// team part (each member's support-vector list and coefficients).
struct ProbBytes {
    size_t x, bits, f, status, act, lw, trec, base;   // offsets into the base part, its size
    size_t lz, coef, team;                      // offsets into the team part, its size
};

ProbBytes prob_bytes(const svm_problem_t* p, bool need_f, int team, int rec_members) {
    ProbBytes b{};
    const size_t n = (size_t)p->n;
    size_t o = 0;
    auto take = [&](size_t v) { size_t a = o; o = al(o + v); return a; };
    b.x = take(p->layout == SVM_CSR ? 0 : sizeof(float) * n * dpad4(p->d));
    b.bits = take(bits_capable(p) ? sizeof(uint32_t) * n * bits_wpr(p->d) : 0);
    b.f = take(need_f ? sizeof(double) * n : 0);
    b.status = take(n);
    b.act = take(sizeof(int32_t) * n);
    b.lw = take(sizeof(int32_t) * n);
    b.trec = take(sizeof(unsigned long long) * 2 * 16 * rec_members);
    b.base = o;
    o = 0;
    b.lz = take(sizeof(int32_t) * n * team);
    b.coef = take(sizeof(double) * n * team);
    b.team = o;
    return b;
}

int check_batch_problem(const svm_problem_t* p, const svm_params_t* q) {
    if (!p || !q || p->n < 2 || p->d < 1 || !p->y) return SVM_EINVAL;
    if (!(q->C > 0) || !(q->gamma > 0) || !(q->eps > 0) || q->max_iter <= 0) return SVM_EINVAL;
    if (q->shrink_mode < 0 || q->shrink_mode > 2) return SVM_EINVAL;
    if (q->shrink_mode != SVM_SHRINK_NONE && !(q->shrink_param > 0)) return SVM_EINVAL;
    if (q->kernel_precision != SVM_KERNEL_FP32 && q->kernel_precision != SVM_KERNEL_FP64) return SVM_EINVAL;
    int l = q->lanes_per_row;
    if (l < 0 || l > 64 || (l & (l - 1))) return SVM_EINVAL;
    // LDS of a batched workgroup: pair rows (8 B per feature) and the reconstruction tile
    // (BATCH_SUMR densified rows, 4 B per feature)
    const int W = p->layout == SVM_CSR ? p->d : dpad4(p->d);
    if (al16(8.0 * W) + al16(4.0 * BATCH_SUMR * W) + 1024.0 > (double)BATCH_LDS_BYTES) return SVM_EUNSUPPORTED;
    if (p->layout == SVM_CSR) {
        if (!p->row_ptr || !p->col || !p->val) return SVM_EINVAL;
    } else {
        if (!p->x) return SVM_EINVAL;
        if (p->layout == SVM_DENSE_ROW_MAJOR && p->ldx < p->d) return SVM_EINVAL;
        if (p->layout == SVM_DENSE_FEATURE_MAJOR && p->ldx < p->n) return SVM_EINVAL;
    }
    return SVM_OK;
}

// What admission learns about a problem before it allocates anything for it.
struct Inspect {
    int32_t nnz = 0;          // CSR nonzeros
    int32_t pattern = 0;      // CSR values all 1.0
};

// Team size.  The requested one (params.grid_blocks) if set.  Otherwise the smallest team
// whose members can each hold their segment (f, status, active list and rows) in LDS, so the
// loop never reads rows from HBM, when a member then holds at least 512 rows and the team
// needs at most TEAM_MAX workgroups; else about 1500 rows per workgroup (at most TEAM_MAX)
// streamed from HBM.  Never more than the launch's workgroups.
int team_size(const svm_problem_t* p, const Inspect& in, int workers, int requested, int kprec, bool shrink) {
    const int cap = std::max(1, std::min(TEAM_MAX, workers));
    if (requested > 0) return std::min(requested, cap);
    // a team size measured by svm_autotune for this problem's class comes first
    const TuneClass c{TUNE_TEAM, batch_layout(p, in.pattern != 0), kprec, in.pattern != 0, shrink, p->n, p->d};
    if (const int t = tuned_shape(c)) return std::min(t, cap);
    const bool dense = p->layout != SVM_CSR;
    const bool bits = bits_capable(p) && in.pattern;
    const int W = dense ? dpad4(p->d) : bits ? bits_wpr(p->d) : p->d;
    const double fixed = (double)al16(8.0 * W) + al16(4.0 * BATCH_SUMR * W) + 6 * 16;
    const double avail = (double)BATCH_LDS_BYTES - fixed;
    const double avg = dense ? 0.0 : (double)in.nnz / (double)p->n;
    const double per_row = 11.0 + (dense ? 4.0 * dpad4(p->d)
                                   : bits ? 4.0 * bits_wpr(p->d) : 4.0 + avg * (in.pattern ? 2.0 : 6.0));
    // CSR segments vary in length; dense and bitset rows do not
    const double rows_cap = avail / per_row * ((dense || bits) ? 0.97 : 0.85);
    // each member pays a fixed cost per iteration (pair staging, block reduction, team exchange:
    // about 7 us); residency pays off when a member holds at least 512 rows (CSR and narrow
    // dense rows), while wide dense rows stream from HBM at a cost per row close to LDS's
    if (rows_cap >= 512.0) {
        const int b = (int)std::ceil((double)p->n / rows_cap);
        if (b <= cap) return std::max(1, b);
    }
    return std::max(1, std::min(cap, (p->n + 1499) / 1500));
}

int64_t shrink_h(const svm_params_t* q, int n) {
    if (q->shrink_mode == SVM_SHRINK_NONE) return 0;
    double h = q->shrink_kind == SVM_KIND_FIXED ? q->shrink_param : std::ceil(q->shrink_param * (double)n);
    return (int64_t)std::max(1.0, h);
}

// Validate on the device and learn the CSR nonzero count and whether every value is 1.0.
int inspect(const svm_problem_t* p, Ctl* vctl, hipStream_t s, Inspect* out) {
    hipError_t e = hipMemsetAsync(vctl, 0, sizeof(Ctl), s);
    if (e == hipSuccess)
        e = launch_validate(p->n, p->d, p->layout, p->x, p->ldx, p->layout == SVM_DENSE_FEATURE_MAJOR, p->row_ptr,
                            p->col, p->val, p->y, vctl, s);
    Ctl h{};
    int32_t nnz = 0, notpat = 1;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, vctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && p->layout == SVM_CSR)
        e = hipMemcpyAsync(&nnz, p->row_ptr + p->n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return SVM_EHIP;
    if (h.err & 1) return SVM_EINVAL;
    if (h.err & 2) return SVM_ENONFINITE;
    if (h.n_pos == 0 || h.n_neg == 0) return SVM_EONECLASS;
    if (p->layout == SVM_CSR && h.max_row_nnz > 4096) return SVM_EUNSUPPORTED;
    *out = Inspect{};
    if (p->layout == SVM_CSR) {
        int32_t* flag = reinterpret_cast<int32_t*>(vctl) + 40;
        e = launch_check_pattern(nnz, p->val, flag, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&notpat, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return SVM_EHIP;
        out->nnz = nnz;
        out->pattern = notpat == 0;
    }
    return SVM_OK;
}

// Fill the descriptor of a solve (host only).  `base` / `teamp` hold the two parts of
// prob_bytes(p, f_user == nullptr, team, rec_members); dense rows are already packed at
// base + x and the team records zeroed.
void fill_desc(const svm_problem_t* p, const svm_params_t* q, const Inspect& in, int team, int rec_members,
               double* alpha, double* f_user, unsigned char* base, unsigned char* teamp, BatchResult* res,
               BatchDesc* D) {
    const ProbBytes b = prob_bytes(p, f_user == nullptr, team, rec_members);
    memset(D, 0, sizeof(*D));
    D->n = p->n;
    D->d = p->d;
    D->dpad = dpad4(p->d);
    D->y = p->y;
    if (p->layout == SVM_CSR) {
        D->lay = bits_capable(p) && in.pattern ? LAY_BITS : LAY_CSR_TABLE;
        D->row_ptr = p->row_ptr;
        D->col = p->col;
        D->val = p->val;
        D->pattern_only = in.pattern;
        if (bits_capable(p)) {
            D->bits = reinterpret_cast<uint32_t*>(base + b.bits);
            D->wpr = bits_wpr(p->d);
        }
    } else {
        D->lay = LAY_DENSE;
        D->x = reinterpret_cast<float*>(base + b.x);
    }
    const double avg = p->layout == SVM_CSR ? (double)in.nnz / (double)p->n : 0.0;
    D->lpr = D->lay == LAY_BITS ? 1 : tune_lanes_per_row(p, avg, q->kernel_precision, q->lanes_per_row);
    D->C = q->C;
    D->gamma = q->gamma;
    D->eps = q->eps;
    D->shrink_mode = q->shrink_mode;
    D->kprec = q->kernel_precision;
    D->H = shrink_h(q, p->n);
    D->max_iter = q->max_iter;
    D->flags = q->flags;
    D->alpha = alpha;
    D->f = f_user ? f_user : reinterpret_cast<double*>(base + b.f);
    D->status = base + b.status;
    D->act = reinterpret_cast<int32_t*>(base + b.act);
    D->list_w = reinterpret_cast<int32_t*>(base + b.lw);
    D->list_z = reinterpret_cast<int32_t*>(teamp + b.lz);
    D->coef = reinterpret_cast<double*>(teamp + b.coef);
    D->team = team;
    D->trec = reinterpret_cast<unsigned long long*>(base + b.trec);
    D->prof = debug_profile_slots();
    D->res = res;
}

// Batch entry: pack dense rows and zero the team records with kernels on `s` (no loop is
// running yet), then fill the descriptor.  `ws` holds the base part followed by the team part.
int prepare(const svm_problem_t* p, const svm_params_t* q, const Inspect& in, int team, double* alpha,
            double* f_user, unsigned char* ws, BatchResult* res, hipStream_t s, BatchDesc* D) {
    const ProbBytes b = prob_bytes(p, f_user == nullptr, team, team);
    hipError_t e = hipSuccess;
    if (p->layout != SVM_CSR)
        e = launch_pack_dense(p->n, p->d, dpad4(p->d), p->x, p->ldx, p->layout == SVM_DENSE_FEATURE_MAJOR,
                              reinterpret_cast<float*>(ws + b.x), s);
    if (e == hipSuccess && bits_capable(p) && in.pattern)
        e = launch_pack_bits(p->n, p->d, bits_wpr(p->d), p->row_ptr, p->col, reinterpret_cast<uint32_t*>(ws + b.bits),
                             s);
    if (e == hipSuccess) e = hipMemsetAsync(ws + b.trec, 0, sizeof(unsigned long long) * 2 * 16 * team, s);
    if (e != hipSuccess) return SVM_EHIP;
    fill_desc(p, q, in, team, team, alpha, f_user, ws, ws + b.base, res, D);
    return SVM_OK;
}

void fill_result(const BatchResult& r, int team, svm_result_t* out) {
    memset(out, 0, sizeof(*out));
    out->beta = r.beta;
    out->b_up = r.b_up;
    out->b_low = r.b_low;
    out->dual_obj = r.dual_obj;
    out->iterations = r.iterations;
    out->n_sv = r.n_sv;
    out->n_bsv = r.n_bsv;
    out->n_recon = r.n_recon;
    out->status = r.status;
    out->shrink_passes = r.shrink_passes;
    out->shrunk_total = r.shrunk_total;
    out->n_launches = 1;
    out->grid_blocks = team;
    out->ms_step = (double)(r.t_end - r.t_start) * 1e-5;   // 100 MHz device wall clock
    out->ms_total = out->ms_step;
}

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ server

struct Arena {
    // first-fit free list over [0, size)
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> bytes
    void init(size_t s) { size = s; free_.clear(); if (s) free_[0] = s; }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

constexpr int RING = 4096;          // descriptor slots
constexpr int TRING = RING * 32;    // worker tickets

struct Pending {
    int64_t ticket;
    svm_problem_t prob;
    svm_params_t params;
    double* alpha;
};

// A problem between admission and completion.
struct Job {
    Pending w;
    double ready_ms = 0.0;            // when it became ready to solve
    double cost = 0.0;                // estimated work: n^2 x bytes per row
    int32_t slot = -1;                // descriptor slot of its current job (preparation, then solve)
    size_t base_off = 0, base_bytes = 0, team_off = 0, team_bytes = 0;
    Inspect in;
    int team = 1;
    bool counted_deferred = false;
};

struct Server {
    size_t budget = 0;
    int max_slots = 0;
    int workgroups = 0;
    hipStream_t ks = nullptr;
    unsigned char* arena_mem = nullptr;
    Arena arena;
    BatchDesc* ring = nullptr;        // pinned
    int2* tickets = nullptr;          // pinned
    BatchResult* results = nullptr;   // pinned, per descriptor slot
    PrepOut* preps = nullptr;         // pinned, per descriptor slot
    int32_t* tail = nullptr;          // pinned
    int32_t* shutdown = nullptr;      // pinned
    int32_t* head = nullptr;          // device: [0] next ticket, [16..17] tail / shutdown mirrors
    int32_t published = 0;            // descriptors
    int32_t published_tickets = 0;    // worker tickets
    bool kernel_live = false;
    bool stop_monitor = false;
    double last_busy_ms = 0.0;
    std::thread monitor;
    std::mutex mu;
    std::deque<Pending> waiting;      // not admitted yet (slots or memory)
    std::map<int64_t, Job> prepping;  // preparation job published
    std::vector<Job> ready;           // prepared, waiting for the loop to need work and for memory
    std::map<int64_t, Job> live;      // solve published, not yet observed done
    std::map<int64_t, svm_result_t> done;
    std::map<int64_t, int> failed;    // ticket -> error code
    int64_t next_ticket = 0;
    int64_t n_admitted = 0, n_deferred = 0, n_completed = 0;

    int in_flight() const { return (int)(prepping.size() + ready.size() + live.size()); }

    // The loop is stopped only by the host (park or destroy), and only when no published ticket
    // is waiting, so a new launch starts its tickets at the published count.
    void ensure_running() {
        if (kernel_live) return;
        // head, then the mirrors of tail and shutdown (64 bytes on)
        int32_t init[18] = {published_tickets};
        init[16] = published_tickets;
        if (hipMemcpyAsync(head, init, sizeof(init), hipMemcpyHostToDevice, ks) != hipSuccess) return;
        BatchArgs a{};
        a.descs = ring;
        a.capacity = RING;
        a.tickets = tickets;
        a.tcapacity = TRING;
        a.head = head;
        a.tail = tail;
        a.shutdown = shutdown;
        a.mirror = head + 16;
        a.fixed_tail = 0;
        if (launch_batch(a, workgroups, SVM_KERNEL_FP32, ks) == hipSuccess) kernel_live = true;
    }

    // stop the loop once nothing is in flight (its workgroups return to the GPU)
    void park() {
        if (!kernel_live || in_flight() || !waiting.empty()) return;
        __atomic_store_n(shutdown, 1, __ATOMIC_RELEASE);
        (void)hipStreamSynchronize(ks);
        __atomic_store_n(shutdown, 0, __ATOMIC_RELEASE);
        kernel_live = false;
    }

    // hand descriptor D and `team` tickets (rank -1: one preparation ticket) to the loop
    int32_t publish(const BatchDesc& D, int team, bool prep) {
        const int32_t slot = published & (RING - 1);
        ring[slot] = D;
        if (prep) {
            tickets[published_tickets & (TRING - 1)] = make_int2(slot, -1);
        } else {
            for (int r = 0; r < team; ++r) tickets[(published_tickets + r) & (TRING - 1)] = make_int2(slot, r);
        }
        std::atomic_thread_fence(std::memory_order_release);
        ++published;
        published_tickets += prep ? 1 : team;
        __atomic_store_n(tail, published_tickets, __ATOMIC_RELEASE);
        ensure_running();
        return slot;
    }

    // waiting -> prepping: needs a slot and the base part of the solver state
    bool start_prep(const Pending& w) {
        if (in_flight() >= max_slots) return false;
        Job j;
        j.w = w;
        j.base_bytes = prob_bytes(&w.prob, true, 1, TEAM_MAX).base;
        if (!arena.alloc(j.base_bytes, &j.base_off)) return false;
        const ProbBytes b = prob_bytes(&w.prob, true, 1, TEAM_MAX);
        unsigned char* base = arena_mem + j.base_off;
        const int32_t slot = published & (RING - 1);
        memset(&preps[slot], 0, sizeof(PrepOut));
        BatchDesc D;
        memset(&D, 0, sizeof(D));
        D.n = w.prob.n;
        D.d = w.prob.d;
        D.dpad = dpad4(w.prob.d);
        D.lay = w.prob.layout == SVM_CSR ? LAY_CSR_TABLE : LAY_DENSE;
        D.y = w.prob.y;
        D.row_ptr = w.prob.row_ptr;
        D.col = w.prob.col;
        D.val = w.prob.val;
        D.x = w.prob.layout == SVM_CSR ? nullptr : reinterpret_cast<float*>(base + b.x);
        D.xsrc = w.prob.x;
        D.ldx = w.prob.ldx;
        D.src_layout = w.prob.layout;
        D.trec = reinterpret_cast<unsigned long long*>(base + b.trec);
        D.prep = &preps[slot];
        if (bits_capable(&w.prob)) {
            D.bits = reinterpret_cast<uint32_t*>(base + b.bits);
            D.wpr = bits_wpr(w.prob.d);
        }
        j.slot = publish(D, 1, true);
        prepping.emplace(w.ticket, j);
        return true;
    }

    // prepping -> ready or failed
    void scan_prep() {
        for (auto it = prepping.begin(); it != prepping.end();) {
            const PrepOut& o = preps[it->second.slot];
            if (!__atomic_load_n(&o.done, __ATOMIC_ACQUIRE)) {
                ++it;
                continue;
            }
            Job j = it->second;
            it = prepping.erase(it);
            int rc = SVM_OK;
            if (o.err & 1) rc = SVM_EINVAL;
            else if (o.err & 2) rc = SVM_ENONFINITE;
            else if (o.n_pos == 0 || o.n_neg == 0) rc = SVM_EONECLASS;
            else if (j.w.prob.layout == SVM_CSR && o.max_row_nnz > 4096) rc = SVM_EUNSUPPORTED;
            if (rc) {
                arena.release(j.base_off, j.base_bytes);
                failed[j.w.ticket] = rc;
                continue;
            }
            j.in.nnz = o.nnz;
            j.in.pattern = o.pattern;
            j.team = team_size(&j.w.prob, j.in, workgroups, j.w.params.grid_blocks, j.w.params.kernel_precision,
                               j.w.params.shrink_mode != SVM_SHRINK_NONE);
            while (j.team > 1 && j.base_bytes + prob_bytes(&j.w.prob, true, j.team, TEAM_MAX).team > budget) j.team /= 2;
            j.team_bytes = prob_bytes(&j.w.prob, true, j.team, TEAM_MAX).team;
            const double row = j.w.prob.layout == SVM_CSR ? (bits_capable(&j.w.prob) && j.in.pattern
                                                                 ? 4.0 * bits_wpr(j.w.prob.d)
                                                                 : 6.0 * (double)j.in.nnz / j.w.prob.n)
                                                          : 4.0 * dpad4(j.w.prob.d);
            j.cost = (double)j.w.prob.n * (double)j.w.prob.n * row;
            j.ready_ms = now_ms();
            ready.push_back(j);
        }
    }

    // tickets published for solves whose team has not gathered yet
    int64_t unstarted_tickets() const {
        int64_t t = 0;
        for (const auto& kv : live)
            if (!__atomic_load_n(&results[kv.second.slot].started, __ATOMIC_ACQUIRE) &&
                !__atomic_load_n(&results[kv.second.slot].done, __ATOMIC_ACQUIRE))
                t += kv.second.team;
        return t;
    }

    // ready -> live.  Solves are published only while the loop has fewer untaken tickets than
    // workgroups, largest estimated work first (problems ready for more than 3 s first, in
    // order), so a burst runs longest-first and the loop is never short of work.  Needs the
    // team part of the solver state.
    void start_solves() {
        int64_t pending = unstarted_tickets();
        while (!ready.empty() && pending < workgroups) {
            const double now = now_ms();
            size_t pick = 0;
            for (size_t k = 1; k < ready.size(); ++k) {
                const bool ak = now - ready[k].ready_ms > 3000.0, ap = now - ready[pick].ready_ms > 3000.0;
                if (ak != ap ? ak : (ak ? ready[k].ready_ms < ready[pick].ready_ms : ready[k].cost > ready[pick].cost))
                    pick = k;
            }
            Job& j = ready[pick];
            if (!arena.alloc(j.team_bytes, &j.team_off)) {
                if (!j.counted_deferred) {
                    j.counted_deferred = true;
                    ++n_deferred;
                }
                return;
            }
            const int32_t slot = published & (RING - 1);
            memset(&results[slot], 0, sizeof(BatchResult));
            BatchDesc D;
            fill_desc(&j.w.prob, &j.w.params, j.in, j.team, TEAM_MAX, j.w.alpha, nullptr, arena_mem + j.base_off,
                      arena_mem + j.team_off, &results[slot], &D);
            j.slot = publish(D, j.team, false);
            ++n_admitted;
            pending += j.team;
            live.emplace(j.w.ticket, j);
            ready.erase(ready.begin() + (long)pick);
        }
    }

    // live -> done
    void scan_done() {
        for (auto it = live.begin(); it != live.end();) {
            BatchResult& r = results[it->second.slot];
            if (__atomic_load_n(&r.done, __ATOMIC_ACQUIRE)) {
                svm_result_t out;
                fill_result(r, it->second.team, &out);
                done[it->first] = out;
                arena.release(it->second.base_off, it->second.base_bytes);
                arena.release(it->second.team_off, it->second.team_bytes);
                ++n_completed;
                it = live.erase(it);
            } else {
                ++it;
            }
        }
    }

    void harvest() {
        scan_done();
        scan_prep();
        start_solves();
        while (!waiting.empty() && start_prep(waiting.front())) waiting.pop_front();
        if (in_flight() || !waiting.empty()) last_busy_ms = now_ms();
    }

    void monitor_loop() {
        for (;;) {
            std::this_thread::sleep_for(std::chrono::milliseconds(2));
            std::lock_guard<std::mutex> lk(mu);
            if (stop_monitor) return;
            harvest();
            if (kernel_live && !in_flight() && waiting.empty() && now_ms() - last_busy_ms > 2000.0) park();
        }
    }
};

}  // namespace

int svm::batch_team_rule(const svm_problem_t* p, int nnz, bool pattern) {
    Inspect in;
    in.nnz = nnz;
    in.pattern = pattern ? 1 : 0;
    return team_size(p, in, std::max(1, batch_max_workgroups(SVM_KERNEL_FP32)), 0, -1, false);
}

int svm::batch_layout(const svm_problem_t* p, bool pattern) {
    return p->layout != SVM_CSR ? LAY_DENSE : (bits_capable(p) && pattern) ? LAY_BITS : LAY_CSR_TABLE;
}

extern "C" {

int svm_train_batch(int32_t k, const svm_problem_t* probs, const svm_params_t* params, double* const* alpha,
                    double* const* f, svm_result_t* out, void* stream) {
    if (k < 0 || (k > 0 && (!probs || !params || !alpha || !out))) return SVM_EINVAL;
    if (k == 0) return SVM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int kprec = params[0].kernel_precision;
    for (int p = 0; p < k; ++p) {
        int rc = check_batch_problem(&probs[p], &params[p]);
        if (rc) return rc;
        if (!alpha[p] || params[p].kernel_precision != kprec) return SVM_EINVAL;
    }
    // one buffer for every problem's solver state, descriptors and results
    const int wg = std::max(1, batch_max_workgroups(kprec));
    std::vector<int> team(k);
    std::vector<Inspect> ins(k);
    int64_t nt = 0;
    Ctl* ictl = nullptr;
    if (hipMalloc(&ictl, sizeof(Ctl) + 256) != hipSuccess) return SVM_ENOMEM;
    for (int p = 0; p < k; ++p) {
        const int rc = inspect(&probs[p], ictl, s, &ins[p]);
        if (rc) {
            (void)hipFree(ictl);
            return rc;
        }
        team[p] = team_size(&probs[p], ins[p], wg, params[p].grid_blocks, params[p].kernel_precision,
                            params[p].shrink_mode != SVM_SHRINK_NONE);
        nt += team[p];
    }
    (void)hipFree(ictl);
    std::vector<size_t> off(k);
    size_t o = al(sizeof(BatchDesc) * k) + al(sizeof(BatchResult) * k) + al(sizeof(Ctl) + 256) + al(64) +
               al(sizeof(int2) * nt);
    for (int p = 0; p < k; ++p) {
        off[p] = o;
        const ProbBytes b = prob_bytes(&probs[p], !(f && f[p]), team[p], team[p]);
        o += b.base + b.team;
    }
    unsigned char* buf = nullptr;
    if (hipMalloc(&buf, o) != hipSuccess) return SVM_ENOMEM;
    BatchDesc* ddesc = reinterpret_cast<BatchDesc*>(buf);
    BatchResult* dres = reinterpret_cast<BatchResult*>(buf + al(sizeof(BatchDesc) * k));
    int32_t* head = reinterpret_cast<int32_t*>(buf + al(sizeof(BatchDesc) * k) + al(sizeof(BatchResult) * k) +
                                               al(sizeof(Ctl) + 256));
    int2* dtk = reinterpret_cast<int2*>(buf + al(sizeof(BatchDesc) * k) + al(sizeof(BatchResult) * k) +
                                        al(sizeof(Ctl) + 256) + al(64));
    std::vector<BatchDesc> hd(k);
    int rc = SVM_OK;
    for (int p = 0; p < k && rc == SVM_OK; ++p)
        rc = prepare(&probs[p], &params[p], ins[p], team[p], alpha[p], f ? f[p] : nullptr, buf + off[p], dres + p, s,
                     &hd[p]);
    if (rc) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        return rc;
    }
    // largest problems first (longest-processing-time order) so the tail of the launch is short
    std::vector<int> order(k);
    for (int p = 0; p < k; ++p) order[p] = p;
    auto cost = [&](int p) {
        const double row = hd[p].lay == LAY_DENSE ? 4.0 * hd[p].dpad : 40.0;
        return (double)hd[p].n * (double)hd[p].n * row;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<BatchDesc> sorted(k);
    std::vector<int2> tk;
    tk.reserve(nt);
    for (int t = 0; t < k; ++t) {
        sorted[t] = hd[order[t]];
        for (int r = 0; r < sorted[t].team; ++r) tk.push_back(make_int2(t, r));
    }
    // a fixed batch: tickets run 0..nt-1, so a mask wider than any ticket indexes the arrays directly
    const int cap = 1 << 30;
    BatchDesc* dring = ddesc;
    hipError_t e = hipMemcpyAsync(dring, sorted.data(), sizeof(BatchDesc) * k, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dtk, tk.data(), sizeof(int2) * nt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(dres, 0, sizeof(BatchResult) * k, s);
    if (e == hipSuccess) e = hipMemsetAsync(head, 0, sizeof(int32_t), s);
    BatchArgs a{};
    a.descs = dring;
    a.capacity = cap;
    a.tickets = dtk;
    a.tcapacity = cap;
    a.head = head;
    a.tail = head;
    a.shutdown = head;
    a.mirror = head;
    a.fixed_tail = (int32_t)nt;
    if (e == hipSuccess) e = launch_batch(a, (int)std::min<int64_t>(wg, nt), kprec, s);
    std::vector<BatchResult> hr(k);
    if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), dres, sizeof(BatchResult) * k, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(buf);
    if (e != hipSuccess) return SVM_EHIP;
    int worst = SVM_OK;
    for (int p = 0; p < k; ++p) {
        fill_result(hr[p], team[p], &out[p]);
        if (hr[p].status != SVM_OK) worst = hr[p].status;
    }
    return worst;
}

int svm_server_create(size_t hbm_budget, int32_t max_slots, void** server) {
    if (!server || max_slots < 1 || max_slots > RING / 4 || hbm_budget < 4096) return SVM_EINVAL;
    Server* S = new Server();
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    // the loop leaves 8 compute units free for the caller's other work (copies, kernels); its own
    // admission work (validation, packing) runs inside the loop
    const int cus = device_cu_count(), per_cu = cus > 0 ? batch_max_workgroups(SVM_KERNEL_FP32) / cus : 0;
    S->workgroups = std::max(1, per_cu * std::max(1, cus - 8));
    bool ok = S->workgroups >= TEAM_MAX &&
              hipStreamCreateWithFlags(&S->ks, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&S->arena_mem, hbm_budget) == hipSuccess &&
              hipHostMalloc((void**)&S->ring, sizeof(BatchDesc) * RING, hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc((void**)&S->tickets, sizeof(int2) * TRING, hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc((void**)&S->results, sizeof(BatchResult) * RING, hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc((void**)&S->preps, sizeof(PrepOut) * RING, hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc((void**)&S->tail, 64, hipHostMallocCoherent) == hipSuccess &&
              hipHostMalloc((void**)&S->shutdown, 64, hipHostMallocCoherent) == hipSuccess &&
              hipMalloc(&S->head, 256) == hipSuccess;
    if (!ok) {
        svm_server_destroy(S);
        return SVM_ENOMEM;
    }
    S->arena.init(hbm_budget);
    *S->tail = 0;
    *S->shutdown = 0;
    memset(S->results, 0, sizeof(BatchResult) * RING);
    memset(S->preps, 0, sizeof(PrepOut) * RING);
    S->ensure_running();
    if (!S->kernel_live) {
        svm_server_destroy(S);
        return SVM_EHIP;
    }
    S->last_busy_ms = now_ms();
    S->monitor = std::thread([S] { S->monitor_loop(); });
    *server = S;
    return SVM_OK;
}

int svm_server_submit(void* server, const svm_problem_t* prob, const svm_params_t* params, double* alpha,
                      int64_t* ticket) {
    Server* S = (Server*)server;
    if (!S || !ticket || !alpha) return SVM_EINVAL;
    int rc = check_batch_problem(prob, params);
    if (rc) return rc;
    if (params->kernel_precision != SVM_KERNEL_FP32) return SVM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    Pending w{S->next_ticket++, *prob, *params, alpha};
    *ticket = w.ticket;
    const ProbBytes b = prob_bytes(prob, true, 1, TEAM_MAX);
    if (b.base + b.team > S->budget) {      // reported by svm_server_poll for this ticket
        S->failed[w.ticket] = SVM_ENOMEM;
        return SVM_OK;
    }
    S->harvest();
    if (!S->waiting.empty() || !S->start_prep(w)) {
        S->waiting.push_back(w);
        ++S->n_deferred;
    }
    S->last_busy_ms = now_ms();
    return SVM_OK;
}

int svm_server_poll(void* server, int64_t ticket, svm_result_t* out) {
    Server* S = (Server*)server;
    if (!S || ticket < 0) return SVM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->harvest();
    auto f = S->failed.find(ticket);
    if (f != S->failed.end()) return f->second;
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return ticket < S->next_ticket ? SVM_EBUSY : SVM_EINVAL;
    if (out) *out = it->second;
    return it->second.status;
}

int svm_server_drain(void* server) {
    Server* S = (Server*)server;
    if (!S) return SVM_EINVAL;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->harvest();
            if (!S->in_flight() && S->waiting.empty()) return SVM_OK;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

int svm_server_stats(void* server, int64_t* admitted, int64_t* deferred, int64_t* completed, int64_t* in_flight) {
    Server* S = (Server*)server;
    if (!S) return SVM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->harvest();
    if (admitted) *admitted = S->n_admitted;
    if (deferred) *deferred = S->n_deferred;
    if (completed) *completed = S->n_completed;
    if (in_flight) *in_flight = (int64_t)S->in_flight();
    return SVM_OK;
}

int svm_server_destroy(void* server) {
    Server* S = (Server*)server;
    if (!S) return SVM_EINVAL;
    if (S->monitor.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop_monitor = true;
        }
        S->monitor.join();
    }
    if (S->shutdown) __atomic_store_n(S->shutdown, 1, __ATOMIC_RELEASE);
    if (S->ks) (void)hipStreamSynchronize(S->ks);
    if (S->arena_mem) (void)hipFree(S->arena_mem);
    if (S->head) (void)hipFree(S->head);
    if (S->ring) (void)hipHostFree(S->ring);
    if (S->tickets) (void)hipHostFree(S->tickets);
    if (S->results) (void)hipHostFree(S->results);
    if (S->preps) (void)hipHostFree(S->preps);
    if (S->tail) (void)hipHostFree(S->tail);
    if (S->shutdown) (void)hipHostFree(S->shutdown);
    if (S->ks) (void)hipStreamDestroy(S->ks);
    delete S;
    return SVM_OK;
}

}  // extern "C"

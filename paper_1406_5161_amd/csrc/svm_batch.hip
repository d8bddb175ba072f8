// svm_batch.hip -- many independent training problems in one persistent launch.
//
// Each problem is solved by its own team of 1 to 64 workgroups, each member owning a
// contiguous segment of the samples: the SMO loop of Alg. 2 / Alg. 4, the shrinking
// driver of Alg. 5 (or its multi-reconstruction variant), gradient reconstruction
// (Alg. 6), the closing FP64-accumulated recompute of f and the threshold of the
// paper's Sec. 3.1 all run inside the team, whose members meet only in tag-validated
// record exchanges with an exact merge, so problems never wait for each other and a
// problem's result depends neither on its team size nor on what else is resident.
// Workgroups take worker tickets (problem, rank in its team) in order; when serving,
// the host keeps publishing descriptors and tickets into pinned memory while the loop
// runs (continuous batching) and the loop ends once the host asks it to and the rings
// are drained.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "svm_device.h"
#include "svm_internal.h"

namespace svm {

constexpr int BB = BATCH_BLOCK;
constexpr int BNW = BB / 64;
constexpr int SUMR = BATCH_SUMR;          // rows per tile in block-local kernel sums
constexpr size_t BATCH_LDS = BATCH_LDS_BYTES;

struct BatchShared {
    BatchDesc P;
    double v[SEL_LDS(BB)];
    int i[SEL_LDS(BB)];
    int wc[BNW];
    double pair[4];
    double red[BNW][SUMR];
    double na[SUMR];
    long long cnt;
    int ticket;
    int rank;
    double tsel[4];
    int tseli[2];
    long long tcnt;
    int tok;
    double tsum[6];
    unsigned long long pt[9];   // per-phase timer of rank 0 (slots as in svm_debug_set_profile's batch use)
    int pr[5];                  // preparation job: err, n_pos, n_neg, max_row_nnz, not-pattern
};

// Descriptor fields made wave-uniform (scalar registers) after the LDS broadcast.
template <typename T>
DEV T* uptr(T* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffull));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}
DEV int ui(int v) { return __builtin_amdgcn_readfirstlane(v); }
DEV size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }
DEV long long ull_(long long v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffll));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
DEV double ud(double v) { return __longlong_as_double(ull_(__double_as_longlong(v))); }

DEV BatchDesc uniform_desc(const BatchDesc& S) {
    BatchDesc P;
    P.n = ui(S.n); P.d = ui(S.d); P.dpad = ui(S.dpad); P.lay = ui(S.lay);
    P.x = uptr(S.x); P.row_ptr = uptr(S.row_ptr); P.col = uptr(S.col); P.val = uptr(S.val);
    P.pattern_only = ui(S.pattern_only); P.lpr = ui(S.lpr);
    P.y = uptr(S.y);
    P.C = ud(S.C); P.gamma = ud(S.gamma); P.eps = ud(S.eps);
    P.shrink_mode = ui(S.shrink_mode); P.kprec = ui(S.kprec);
    P.H = ull_(S.H); P.max_iter = ull_(S.max_iter);
    P.flags = (uint32_t)ui((int)S.flags); P.pad = 0;
    P.alpha = uptr(S.alpha); P.f = uptr(S.f); P.status = uptr(S.status); P.act = uptr(S.act);
    P.list_w = uptr(S.list_w); P.list_z = uptr(S.list_z); P.coef = uptr(S.coef); P.res = uptr(S.res);
    return P;
}

// group sum over `lpr` consecutive lanes (lpr a power of two <= 64)
template <typename T>
DEV T group_sum(T v, int lpr) {
    for (int off = 1; off < lpr; off <<= 1) v += __shfl_xor(v, off);
    return v;
}

// Stable in-place-compatible block scan of keep flags for one chunk; returns the
// position of this thread's kept entry relative to `base_out` and the chunk total.
DEV int block_scan_keep(bool keep, int* s_wc, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(keep);
    const int wpre = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_wc[wid] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < BNW; ++w) {
        const int c = s_wc[w];
        off += (w < wid) ? c : 0;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return off + wpre;
}

// Distances of RPT rows at once: the rows' loads are interleaved so a lane keeps several
// rows in flight instead of walking one dependent chain after another.  Row r of the call is
// ri[r] in the row source: dense rows at xb + ri * dpad; CSR rows [off[ri], off[ri + 1]) of
// cols / vals.  The source is the problem's arrays in HBM or the member's copy in LDS.
template <typename KT, int RPT, typename OT, typename CT>
DEV void rows_dist(bool dense, int dpad, const float* xb, const OT* off, const CT* cols, const float* vals,
                   bool pattern, const float2* pairv, const int* ri, const bool* vv, int gl, int lpr, KT nuu,
                   KT nll, KT* du2, KT* dl2) {
    if (dense) {
        // DU k-steps of every row are loaded before any is used: a chunk read from HBM costs
        // one memory latency per DU k-steps
        constexpr int DU = 2;
        const float4* p4 = reinterpret_cast<const float4*>(pairv);
        const int n4 = dpad / 4;
        KT a[RPT], b[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) { a[r] = 0; b[r] = 0; }
        for (int k0 = gl; k0 < n4; k0 += DU * lpr) {
            float4 v[DU][RPT];
#pragma unroll
            for (int u = 0; u < DU; ++u) {
                const int k4 = k0 + u * lpr;
#pragma unroll
                for (int r = 0; r < RPT; ++r)
                    v[u][r] = (vv[r] && k4 < n4) ? reinterpret_cast<const float4*>(xb + (size_t)ri[r] * dpad)[k4]
                                                 : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < DU; ++u) {
                const int k4 = k0 + u * lpr;
                if (k4 >= n4) break;
                const float4 q0 = p4[2 * k4], q1 = p4[2 * k4 + 1];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const float4 w = v[u][r];
                    if constexpr (std::is_same<KT, double>::value) {
#pragma clang fp contract(off)
                        double t, x = a[r], y = b[r];
                        t = (double)w.x - (double)q0.x; x = x + t * t;
                        t = (double)w.x - (double)q0.y; y = y + t * t;
                        t = (double)w.y - (double)q0.z; x = x + t * t;
                        t = (double)w.y - (double)q0.w; y = y + t * t;
                        t = (double)w.z - (double)q1.x; x = x + t * t;
                        t = (double)w.z - (double)q1.y; y = y + t * t;
                        t = (double)w.w - (double)q1.z; x = x + t * t;
                        t = (double)w.w - (double)q1.w; y = y + t * t;
                        a[r] = x; b[r] = y;
                    } else {
                        float t, x = a[r], y = b[r];
                        t = w.x - q0.x; x = fmaf(t, t, x);
                        t = w.x - q0.y; y = fmaf(t, t, y);
                        t = w.y - q0.z; x = fmaf(t, t, x);
                        t = w.y - q0.w; y = fmaf(t, t, y);
                        t = w.z - q1.x; x = fmaf(t, t, x);
                        t = w.z - q1.y; y = fmaf(t, t, y);
                        t = w.w - q1.z; x = fmaf(t, t, x);
                        t = w.w - q1.w; y = fmaf(t, t, y);
                        a[r] = x; b[r] = y;
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            du2[r] = group_sum(a[r], lpr);
            dl2[r] = group_sum(b[r], lpr);
        }
    } else {
        int p0[RPT], p1[RPT], len = 0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            p0[r] = vv[r] ? (int)off[ri[r]] : 0;
            p1[r] = vv[r] ? (int)off[ri[r] + 1] : 0;
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) len = max(len, p1[r] - p0[r]);
        KT nn[RPT], su[RPT], sl[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) { nn[r] = 0; su[r] = 0; sl[r] = 0; }
        for (int k = gl; k < len; k += lpr) {
            int c[RPT];
            float fv[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int p = p0[r] + k;
                const bool in = p < p1[r];
                c[r] = in ? (int)cols[p] : -1;
                fv[r] = in ? (pattern ? 1.f : vals[p]) : 0.f;
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (c[r] >= 0) {
                    const float2 ul = pairv[c[r]];
                    const KT v = (KT)fv[r];
                    nn[r] += v * v;
                    su[r] += v * (KT)ul.x;
                    sl[r] += v * (KT)ul.y;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const KT n2 = group_sum(nn[r], lpr), s1 = group_sum(su[r], lpr), s2 = group_sum(sl[r], lpr);
            KT a = n2 + nuu - (KT)2 * s1, b = n2 + nll - (KT)2 * s2;
            du2[r] = a < (KT)0 ? (KT)0 : a;
            dl2[r] = b < (KT)0 ? (KT)0 : b;
        }
    }
}

// Distances of RPT bitset rows (LAY_BITS, one lane per row) to the two pair rows held at pb
// (pair row u in words [0, wpr), row l in [wpr, 2 wpr)).  Counts are exact integers, so the
// values equal the CSR path's sums of 1.0 in either precision.
template <typename KT, int RPT>
DEV void rows_dist_bits(int wpr, const uint32_t* src, const uint32_t* pb, const int* ri, const bool* vv, KT nuu,
                        KT nll, KT* du2, KT* dl2) {
    const uint4* pu = reinterpret_cast<const uint4*>(pb);
    const uint4* pl = reinterpret_cast<const uint4*>(pb + wpr);
    int nn[RPT], su[RPT], sl[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) { nn[r] = 0; su[r] = 0; sl[r] = 0; }
    for (int w4 = 0; w4 < wpr / 4; ++w4) {
        const uint4 a = pu[w4], b = pl[w4];
        uint4 v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            v[r] = vv[r] ? reinterpret_cast<const uint4*>(src + (size_t)ri[r] * wpr)[w4] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            nn[r] += __popc(v[r].x) + __popc(v[r].y) + __popc(v[r].z) + __popc(v[r].w);
            su[r] += __popc(v[r].x & a.x) + __popc(v[r].y & a.y) + __popc(v[r].z & a.z) + __popc(v[r].w & a.w);
            sl[r] += __popc(v[r].x & b.x) + __popc(v[r].y & b.y) + __popc(v[r].z & b.z) + __popc(v[r].w & b.w);
        }
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        KT a = (KT)nn[r] + nuu - (KT)2 * (KT)su[r], b = (KT)nn[r] + nll - (KT)2 * (KT)sl[r];
        du2[r] = a < (KT)0 ? (KT)0 : a;
        dl2[r] = b < (KT)0 ? (KT)0 : b;
    }
}

// Local selection over this member's active list from (f, alpha, y) in global memory; every
// thread gets the result.
DEV void select_block(const BatchDesc& P, const int32_t* act, int nact, BatchShared& sh, double& bu, int& iu,
                      double& bl, int& il) {
    bu = INFINITY; bl = -INFINITY; iu = IDX_NONE; il = IDX_NONE;
    for (int t = threadIdx.x; t < nact; t += BB) {
        const int i = act[t];
        const uint8_t st = st_make(P.y[i] > 0, ld_agent(P.alpha + i), P.C);
        const double fi = P.f[i];
        if (st_in_up(st) && better_up(fi, i, bu, iu)) { bu = fi; iu = i; }
        if (st_in_low(st) && better_low(fi, i, bl, il)) { bl = fi; il = i; }
    }
    block_reduce_sel_all<BB>(bu, iu, bl, il, sh.v, sh.i);
    __syncthreads();
}

// ---- team exchanges: the B workgroups of one problem publish tag-validated records
// (high half of each 64-bit word = exchange sequence number) and read each other's.

// Watchdogs (device wall clock, 100 MHz): the first exchange of a problem waits for the team to
// gather (members start as workgroups finish earlier problems); later exchanges wait only for
// members doing the same step.  An expired wait ends the solve with SVM_EABORT.
constexpr unsigned long long TEAM_GATHER_TICKS = 120ull * 100 * 1000 * 1000;
constexpr unsigned long long TEAM_WAIT_TICKS = 30ull * 100 * 1000 * 1000;

struct TeamSel {
    double bu, bl, au, al;
    int iu, il;
    long long cnt;
    int ok;
};

// Wave 0 of the calling workgroup waits for all B records of exchange `seq` and returns them
// decoded in lanes < B; false if the watchdog fired.
DEV bool team_read(const unsigned long long* trec, int B, unsigned seq, unsigned* v,
                   unsigned long long spin_limit) {
    const int lane = threadIdx.x & 63;
    bool ok = true;
    if (lane < B) {
        const unsigned long long* w = trec + ((size_t)(seq & 1) * B + lane) * 16;
        const unsigned long long t0 = wall_clock64();
        while ((unsigned)(ld_agent(w + REC_WORDS - 1) >> 32) != seq) {
            if (wall_clock64() - t0 > spin_limit) { ok = false; break; }
            __builtin_amdgcn_s_sleep(1);
        }
        for (; ok;) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < REC_WORDS; ++k) {
                const unsigned long long x = ld_agent(w + k);
                v[k] = (unsigned)(x & 0xffffffffull);
                all = all && (unsigned)(x >> 32) == seq;
            }
            if (all) break;
            if (wall_clock64() - t0 > spin_limit) { ok = false; break; }
        }
    }
    return __all(ok);
}

// Called by every lane of wave 0 with the same v: lane k < REC_WORDS stores word k, so the
// record leaves in one store instruction.
DEV void team_write(unsigned long long* trec, int B, int rank, unsigned seq, const unsigned* v) {
    const int lane = threadIdx.x & 63;
    unsigned x = v[0];
#pragma unroll
    for (int k = 1; k < REC_WORDS; ++k)
        if (lane == k) x = v[k];
    if (lane < REC_WORDS) {
        unsigned long long* w = trec + ((size_t)(seq & 1) * B + rank) * 16;
        st_agent(w + lane, ((unsigned long long)seq << 32) | x);
    }
}

// Int sum over the wave by DPP (row sums, then rows 0-3 into lane 63), returned in every lane.
DEV int wave_sum_i32_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, DPP_XOR1, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_XOR2, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_ROR4, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_ROR8, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_BCAST15, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_BCAST31, 0xC, 0xF, false);
    return __builtin_amdgcn_readlane(v, 63);
}

DEV void pack_d(unsigned* v, int k, double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    v[k] = (unsigned)(b & 0xffffffffull);
    v[k + 1] = (unsigned)(b >> 32);
}
DEV double unpack_d(const unsigned* v, int k) {
    return __longlong_as_double((long long)(((unsigned long long)v[k + 1] << 32) | v[k]));
}

// Merge the members' candidates (called by every thread; every lane of wave 0 holds this
// member's values).
DEV TeamSel team_select(const BatchDesc& P, int rank, unsigned seq, double bu, int iu, double au, double bl,
                        int il, double al, long long cnt, BatchShared& sh) {
    const int tid = threadIdx.x;
    TeamSel r;
    if (P.team == 1) {
        if (tid == 0) {
            sh.tsel[0] = bu; sh.tsel[1] = bl; sh.tsel[2] = au; sh.tsel[3] = al;
            sh.tseli[0] = iu; sh.tseli[1] = il; sh.tcnt = cnt; sh.tok = 1;
        }
    } else {
        if (tid < 64) {
            unsigned v[REC_WORDS];
            pack_d(v, 0, bu); pack_d(v, 2, bl); pack_d(v, 4, au); pack_d(v, 6, al);
            v[8] = (unsigned)iu; v[9] = (unsigned)il;
            v[10] = (unsigned)(cnt & 0xffffffffll); v[11] = (unsigned)((unsigned long long)cnt >> 32);
            v[12] = v[13] = v[14] = 0;
            team_write(P.trec, P.team, rank, seq, v);
        }
        if (tid < 64) {
            unsigned v[REC_WORDS];
            const bool ok = team_read(P.trec, P.team, seq, v, seq == 1 ? TEAM_GATHER_TICKS : TEAM_WAIT_TICKS);
            const int lane = tid;
            double xbu = INFINITY, xbl = -INFINITY, xau = 0.0, xal = 0.0;
            int xiu = IDX_NONE, xil = IDX_NONE;
            long long xc = 0;
            if (lane < P.team && ok) {
                xbu = unpack_d(v, 0); xbl = unpack_d(v, 2); xau = unpack_d(v, 4); xal = unpack_d(v, 6);
                xiu = (int)v[8]; xil = (int)v[9];
                xc = (long long)(((unsigned long long)v[11] << 32) | v[10]);
            }
            const int myiu = xiu, myil = xil;
            // active-row counts: the team's total is at most n < 2^31
            const long long tot = wave_sum_i32_dpp((int)xc);
            wave_reduce_sel(xbu, xiu, xbl, xil);
            if (lane < P.team && myiu == xiu && xiu != IDX_NONE) sh.tsel[2] = xau;
            if (lane < P.team && myil == xil && xil != IDX_NONE) sh.tsel[3] = xal;
            if (lane == 0) {
                sh.tsel[0] = xbu; sh.tsel[1] = xbl; sh.tseli[0] = xiu; sh.tseli[1] = xil; sh.tcnt = tot;
                sh.tok = ok ? 1 : 0;
                if (xiu == IDX_NONE) sh.tsel[2] = 0.0;
                if (xil == IDX_NONE) sh.tsel[3] = 0.0;
            }
        }
    }
    __syncthreads();
    r.bu = sh.tsel[0]; r.bl = sh.tsel[1]; r.au = sh.tsel[2]; r.al = sh.tsel[3];
    r.iu = sh.tseli[0] == IDX_NONE ? -1 : sh.tseli[0];
    r.il = sh.tseli[1] == IDX_NONE ? -1 : sh.tseli[1];
    r.cnt = sh.tcnt;
    r.ok = sh.tok;
    __syncthreads();
    return r;
}

// Sum 6 doubles over the team (every lane of wave 0 holds this member's values; thread 0 is
// enough for a team of one); every thread gets the totals.
// With fence = true the exchange also publishes every global write made before it (alpha of the
// pair rows) to the other members.
DEV bool team_sum(const BatchDesc& P, int rank, unsigned seq, const double* x6, double* out6, bool fence,
                  BatchShared& sh) {
    const int tid = threadIdx.x;
    if (P.team == 1) {
        if (tid == 0) {
            for (int k = 0; k < 6; ++k) sh.tsum[k] = x6[k];
            sh.tok = 1;
        }
    } else {
        if (fence) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid < 64) {
            unsigned v[REC_WORDS];
            for (int k = 0; k < 6; ++k) pack_d(v, 2 * k, x6[k]);
            v[12] = v[13] = v[14] = 0;
            team_write(P.trec, P.team, rank, seq, v);
        }
        if (tid < 64) {
            unsigned v[REC_WORDS];
            const bool ok = team_read(P.trec, P.team, seq, v, TEAM_WAIT_TICKS);
            double t[6] = {0, 0, 0, 0, 0, 0};
            if (tid < P.team && ok)
                for (int k = 0; k < 6; ++k) t[k] = unpack_d(v, 2 * k);
            // sum in member order for the same result in every member
            for (int k = 0; k < 6; ++k) {
                double acc = 0.0;
                for (int m = 0; m < P.team; ++m) acc += __shfl(t[k], m);
                if (tid == 0) sh.tsum[k] = acc;
            }
            if (tid == 0) sh.tok = ok ? 1 : 0;
        }
    }
    __syncthreads();
    if (fence && P.team > 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int k = 0; k < 6; ++k) out6[k] = sh.tsum[k];
    const bool ok = sh.tok != 0;
    __syncthreads();
    return ok;
}

// Stable compaction over ids lo..hi-1: list = ids with pred(i) (0: shrunk, i.e. status bit 3
// set; 1: alpha > 0, with coefficient alpha * y).  Returns the count (all threads).
template <int PRED>
DEV int compact_block(const BatchDesc& P, int lo, int hi, int32_t* list, double* coef, BatchShared& sh) {
    int out = 0;
    for (int base = lo; base < hi; base += BB) {
        const int i = base + threadIdx.x;
        bool k = false;
        if (i < hi) {
            if (PRED == 0) k = (P.status[i] & 8) != 0;
            else k = ld_agent(P.alpha + i) > 0.0;
        }
        int tot;
        const int pos = block_scan_keep(k, sh.wc, tot);
        if (k) {
            list[out + pos] = i;
            if (coef) coef[out + pos] = ld_agent(P.alpha + i) * (P.y[i] > 0 ? 1.0 : -1.0);
        }
        out += tot;
    }
    __syncthreads();
    return out;
}

// f[a] = sum_j coef_j K(x_a, x_{z_j}) - y_a for the rows in `rows` (or 0..na-1), block-local (Alg. 6).
template <typename KT>
__device__ __attribute__((noinline)) void kernel_sum_block(const BatchDesc& P, const int32_t* rows, int row0, int na,
                                                          const int32_t* lz, const double* lcoef, int nz, float* tile,
                                                          BatchShared& sh) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool dense = P.lay == LAY_DENSE;
    const KT gam = (KT)P.gamma;
    if (P.lay == LAY_BITS) {
        // target rows' bitsets in LDS; one support vector per lane and step
        const int wpr = P.wpr;
        uint32_t* tb = reinterpret_cast<uint32_t*>(tile);
        for (int r0 = 0; r0 < na; r0 += SUMR) {
            const int nr = min(SUMR, na - r0);
            for (int e = tid; e < SUMR * wpr; e += BB) {
                const int r = e / wpr, k = e % wpr;
                const int a = r < nr ? (rows ? rows[r0 + r] : row0 + r0 + r) : -1;
                tb[e] = a >= 0 ? P.bits[(size_t)a * wpr + k] : 0u;
            }
            __syncthreads();
            if (tid < SUMR) {
                int c = 0;
                for (int k = 0; k < wpr; ++k) c += __popc(tb[tid * wpr + k]);
                sh.na[tid] = (double)c;
            }
            __syncthreads();
            double acc[SUMR];
#pragma unroll
            for (int r = 0; r < SUMR; ++r) acc[r] = 0.0;
            for (int jb = tid; jb < nz; jb += BB) {
                const int j = lz[jb];
                const double cj = lcoef[jb];
                const uint4* xb = reinterpret_cast<const uint4*>(P.bits + (size_t)j * wpr);
                int nb = 0, dot[SUMR];
#pragma unroll
                for (int r = 0; r < SUMR; ++r) dot[r] = 0;
                for (int w4 = 0; w4 < wpr / 4; ++w4) {
                    const uint4 v = xb[w4];
                    nb += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
#pragma unroll
                    for (int r = 0; r < SUMR; ++r) {
                        const uint4 t = reinterpret_cast<const uint4*>(tb + r * wpr)[w4];
                        dot[r] += __popc(v.x & t.x) + __popc(v.y & t.y) + __popc(v.z & t.z) + __popc(v.w & t.w);
                    }
                }
#pragma unroll
                for (int r = 0; r < SUMR; ++r) {
                    if (r < nr) {
                        KT d2 = (KT)sh.na[r] + (KT)nb - (KT)2 * (KT)dot[r];
                        if (d2 < (KT)0) d2 = (KT)0;
                        acc[r] += cj * (double)kexp(-gam * d2);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < SUMR; ++r) {
                const double v = wave_sum(acc[r]);
                if (lane == 0) sh.red[wid][r] = v;
            }
            __syncthreads();
            if (tid < nr) {
                double v = 0.0;
                for (int w = 0; w < BNW; ++w) v += sh.red[w][tid];
                const int a = rows ? rows[r0 + tid] : row0 + r0 + tid;
                P.f[a] = v - (P.y[a] > 0 ? 1.0 : -1.0);
            }
            __syncthreads();
        }
        return;
    }
    const int W = dense ? P.dpad : P.d;
    for (int r0 = 0; r0 < na; r0 += SUMR) {
        const int nr = min(SUMR, na - r0);
        for (int e = tid; e < SUMR * W; e += BB) tile[e] = 0.f;
        __syncthreads();
        if (dense) {
            for (int e = tid; e < nr * W; e += BB) {
                const int r = e / W, k = e % W;
                const int a = rows ? rows[r0 + r] : row0 + r0 + r;
                tile[e] = P.x[(size_t)a * P.dpad + k];
            }
        } else {
            for (int r = 0; r < nr; ++r) {
                const int a = rows ? rows[r0 + r] : row0 + r0 + r;
                for (int p = P.row_ptr[a] + tid; p < P.row_ptr[a + 1]; p += BB)
                    tile[r * W + P.col[p]] = P.pattern_only ? 1.f : P.val[p];
            }
        }
        __syncthreads();
        if (!dense) {
            for (int r = wid; r < nr; r += BNW) {
                KT s = 0;
                for (int k = lane; k < W; k += 64) {
                    const KT v = (KT)tile[r * W + k];
                    s += v * v;
                }
                s = wave_sum(s);
                if (lane == 0) sh.na[r] = (double)s;
            }
            __syncthreads();
        }
        double acc[SUMR];
#pragma unroll
        for (int r = 0; r < SUMR; ++r) acc[r] = 0.0;
        for (int jb = tid; jb < nz; jb += BB) {
            const int j = lz[jb];
            const double cj = lcoef[jb];
            KT dist[SUMR];
#pragma unroll
            for (int r = 0; r < SUMR; ++r) dist[r] = 0;
            if (dense) {
                const float4* xb = reinterpret_cast<const float4*>(P.x + (size_t)j * P.dpad);
                for (int k4 = 0; k4 < P.dpad / 4; ++k4) {
                    const float4 v = xb[k4];
#pragma unroll
                    for (int r = 0; r < SUMR; ++r) {
                        if (r < nr) {
                            const float4 q = reinterpret_cast<const float4*>(tile + r * W)[k4];
                            if constexpr (std::is_same<KT, double>::value) {
#pragma clang fp contract(off)
                                double t, s = dist[r];
                                t = (double)q.x - (double)v.x; s = s + t * t;
                                t = (double)q.y - (double)v.y; s = s + t * t;
                                t = (double)q.z - (double)v.z; s = s + t * t;
                                t = (double)q.w - (double)v.w; s = s + t * t;
                                dist[r] = s;
                            } else {
                                float t, s = dist[r];
                                t = q.x - v.x; s = fmaf(t, t, s);
                                t = q.y - v.y; s = fmaf(t, t, s);
                                t = q.z - v.z; s = fmaf(t, t, s);
                                t = q.w - v.w; s = fmaf(t, t, s);
                                dist[r] = s;
                            }
                        }
                    }
                }
            } else {
                KT nb = 0;
                for (int p = P.row_ptr[j]; p < P.row_ptr[j + 1]; ++p) {
                    const int c = P.col[p];
                    const KT v = P.pattern_only ? (KT)1 : (KT)P.val[p];
                    nb += v * v;
#pragma unroll
                    for (int r = 0; r < SUMR; ++r)
                        if (r < nr) dist[r] += v * (KT)tile[r * W + c];
                }
#pragma unroll
                for (int r = 0; r < SUMR; ++r) {
                    KT d2 = (KT)sh.na[r < nr ? r : 0] + nb - (KT)2 * dist[r];
                    dist[r] = d2 < (KT)0 ? (KT)0 : d2;
                }
            }
#pragma unroll
            for (int r = 0; r < SUMR; ++r)
                if (r < nr) acc[r] += cj * (double)kexp(-gam * dist[r]);
        }
#pragma unroll
        for (int r = 0; r < SUMR; ++r) {
            const double v = wave_sum(acc[r]);
            if (lane == 0) sh.red[wid][r] = v;
        }
        __syncthreads();
        if (tid < nr) {
            double v = 0.0;
            for (int w = 0; w < BNW; ++w) v += sh.red[w][tid];
            const int a = rows ? rows[r0 + tid] : row0 + r0 + tid;
            P.f[a] = v - (P.y[a] > 0 ? 1.0 : -1.0);
        }
        __syncthreads();
    }
}

// One member (rank) of the team of P.team workgroups solving problem P.  Member b owns rows
// [n b / B, n (b+1) / B); the members run the same driver, take the same decisions from the
// merged selections, and meet only in team exchanges.
// (one instance per kernel precision and row layout, each with its own register allocation)
template <typename KT, int LAYK>
__device__ __attribute__((noinline)) void solve_team(BatchShared& sh, unsigned char* dyn) {
    const BatchDesc& P = sh.P;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = P.n, B = P.team, rank = sh.rank;
    const int seg0 = (int)(((long long)n * rank) / B), seg1 = (int)(((long long)n * (rank + 1)) / B);
    const int lpr = P.lpr;
    const int NG = BB / lpr, g = tid / lpr, gl = tid % lpr;
    const double C = P.C;
    constexpr bool dense = LAYK == LAY_DENSE;
    constexpr bool bits = LAYK == LAY_BITS;
    int32_t* act = P.act + seg0;
    int32_t* lw = P.list_w + seg0;
    int32_t* lz = P.list_z + (size_t)rank * n;
    double* lcoef = P.coef + (size_t)rank * n;
    // dynamic LDS: pair rows (float2 per feature), the reconstruction tile (SUMR rows), then,
    // when it fits, this member's segment: f, status, active list and its rows
    const int W = dense ? P.dpad : bits ? P.wpr : P.d;
    float2* pairv = reinterpret_cast<float2*>(dyn);
    uint32_t* pairb = reinterpret_cast<uint32_t*>(dyn);   // LAY_BITS: the two pair rows' bitsets
    const size_t tile_off = al16(sizeof(float2) * (size_t)W);
    float* tile = reinterpret_cast<float*>(dyn + tile_off);
    unsigned char* segmem = dyn + tile_off + al16(sizeof(float) * SUMR * (size_t)W);
    const int m = seg1 - seg0;
    const int nnz0 = (dense || bits) ? 0 : P.row_ptr[seg0];
    const int nnz_seg = (dense || bits) ? 0 : P.row_ptr[seg1] - nnz0;
    const bool pat = P.pattern_only != 0;
    // this member's state (f, status, active list) lives in LDS when it fits (`res`), and its
    // rows too when they also fit (`rres`); otherwise the rows stream from HBM
    const size_t state_bytes = al16(sizeof(double) * (size_t)m) + al16((size_t)m) + al16(sizeof(uint16_t) * (size_t)m);
    size_t rows_bytes;
    if (dense) {
        rows_bytes = al16(sizeof(float) * (size_t)m * P.dpad);
    } else if (bits) {
        rows_bytes = al16(sizeof(uint32_t) * (size_t)m * P.wpr);
    } else {
        rows_bytes = al16(sizeof(uint32_t) * (size_t)(m + 1)) + al16(sizeof(uint16_t) * (size_t)nnz_seg) +
                     (pat ? 0 : al16(sizeof(float) * (size_t)nnz_seg));
    }
    const size_t seg_room = BATCH_LDS - (size_t)(segmem - dyn);
    const bool res = state_bytes <= seg_room && m <= 65535;
    const bool rres = res && state_bytes + rows_bytes <= seg_room && (dense || P.d <= 65536);
    size_t so = al16(sizeof(double) * (size_t)m);
    double* f_l = reinterpret_cast<double*>(segmem);
    uint8_t* st_l = segmem + so;
    so += al16((size_t)m);
    uint16_t* act_l = reinterpret_cast<uint16_t*>(segmem + so);
    so += al16(sizeof(uint16_t) * (size_t)m);
    float* x_l = reinterpret_cast<float*>(segmem + so);
    uint32_t* bits_l = reinterpret_cast<uint32_t*>(segmem + so);
    uint32_t* off_l = reinterpret_cast<uint32_t*>(segmem + so);
    if (!dense && !bits) so += al16(sizeof(uint32_t) * (size_t)(m + 1));
    uint16_t* cols_l = reinterpret_cast<uint16_t*>(segmem + so);
    if (!dense && !bits) so += al16(sizeof(uint16_t) * (size_t)nnz_seg);
    float* vals_l = reinterpret_cast<float*>(segmem + so);
    const unsigned long long t_start = wall_clock64();
    unsigned seq = 1;
    bool alive = true;
    // rank 0's per-phase timer: [0] pair staging and K(up, low), [1] f update / selection / shrink
    // stream, [2] block reduction, [3] team selection exchange, [4] reconstruction and recompute,
    // [5] iterations, [6] start-up to the first selection, [7] summary and completion
    const bool prof_on = P.prof != nullptr && rank == 0 && tid == 0;
    if (prof_on) {
        for (int k = 0; k < 8; ++k) sh.pt[k] = 0;
        sh.pt[8] = t_start;
    }
    auto lap = [&](int k) {
        if (prof_on) {
            const unsigned long long t = wall_clock64();
            sh.pt[k] += t - sh.pt[8];
            sh.pt[8] = t;
        }
    };

    // initial state of this member's rows: alpha = 0, f = -y, active (status bit 3 = shrunk)
    for (int i = seg0 + tid; i < seg1; i += BB) {
        const bool yp = P.y[i] > 0;
        st_agent(P.alpha + i, 0.0);
        P.f[i] = yp ? -1.0 : 1.0;
        P.status[i] = st_make(yp, 0.0, C);
        act[i - seg0] = i;
    }
    __syncthreads();

    int nact = seg1 - seg0;
    long long nact_total = n;
    double bu, bl, au = 0.0, al = 0.0;
    int iu, il;
    // merge this member's candidates; (ju, aju), (jl, ajl): rows whose alpha this workgroup has
    // just changed, with their new values (the only alphas not yet settled in memory)
    auto merge = [&](double cbu, int ciu, double cbl, int cil, long long cnt, int ju, double aju, int jl,
                     double ajl) {
        double cau = 0.0, cal = 0.0;
        if (tid < 64) {
            if (ciu != IDX_NONE) cau = ciu == ju ? aju : ciu == jl ? ajl : ld_agent(P.alpha + ciu);
            if (cil != IDX_NONE) cal = cil == ju ? aju : cil == jl ? ajl : ld_agent(P.alpha + cil);
        }
        const TeamSel t = team_select(P, rank, seq++, cbu, ciu, cau, cbl, cil, cal, cnt, sh);
        bu = t.bu; bl = t.bl; au = t.au; al = t.al; iu = t.iu; il = t.il;
        if (!t.ok) alive = false;
        return t.cnt;
    };
    {
        double cbu, cbl;
        int ciu, cil;
        select_block(P, act, nact, sh, cbu, ciu, cbl, cil);
        merge(cbu, ciu, cbl, cil, nact, -1, 0.0, -1, 0.0);
    }
    // f, status and active list between HBM and the LDS copy (resident members only)
    auto to_global = [&]() {
        for (int r = tid; r < m; r += BB) {
            P.f[seg0 + r] = f_l[r];
            P.status[seg0 + r] = st_l[r];
        }
        __syncthreads();
    };
    auto from_global = [&]() {
        for (int r = tid; r < m; r += BB) {
            f_l[r] = P.f[seg0 + r];
            st_l[r] = P.status[seg0 + r];
            act_l[r] = (uint16_t)r;
        }
        __syncthreads();
    };
    if (rres) {
        if (dense) {
            const float4* src = reinterpret_cast<const float4*>(P.x + (size_t)seg0 * P.dpad);
            float4* dst = reinterpret_cast<float4*>(x_l);
            for (int k = tid; k < m * (P.dpad / 4); k += BB) dst[k] = src[k];
        } else if (bits) {
            const uint4* src = reinterpret_cast<const uint4*>(P.bits + (size_t)seg0 * P.wpr);
            uint4* dst = reinterpret_cast<uint4*>(bits_l);
            for (int k = tid; k < m * (P.wpr / 4); k += BB) dst[k] = src[k];
        } else {
            for (int r = tid; r <= m; r += BB) off_l[r] = (uint32_t)(P.row_ptr[seg0 + r] - nnz0);
            for (int k = tid; k < nnz_seg; k += BB) {
                cols_l[k] = (uint16_t)P.col[nnz0 + k];
                if (!pat) vals_l[k] = P.val[nnz0 + k];
            }
        }
    }
    if (res) from_global();
    // the first exchange gathered the whole team: its tickets are all taken
    if (rank == 0 && tid == 0) __hip_atomic_store(&P.res->started, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    lap(6);
    bool shrinking = P.shrink_mode != SVM_SHRINK_NONE;
    double thr = shrinking ? 20.0 * P.eps : 2.0 * P.eps;
    const long long H = shrinking ? P.H : 0;
    long long counter = H, iter = 0, passes = 0, shrunk = 0;
    int n_recon = 0, rechecks = 0, status = SVM_OK;
    const bool final_recompute = P.kprec == SVM_KERNEL_FP32 && !(P.flags & SVM_FLAG_NO_FINAL_RECOMPUTE);

    // f of this member's shrunk rows (all its rows when `all`) from the current support vectors
    auto rebuild = [&](bool all) {
        const double zero6[6] = {0, 0, 0, 0, 0, 0};
        double t6[6];
        if (res) to_global();
        if (!team_sum(P, rank, seq++, zero6, t6, true, sh)) { alive = false; return; }   // publishes alpha
        const int nz = compact_block<1>(P, 0, n, lz, lcoef, sh);
        if (all) {
            kernel_sum_block<KT>(P, nullptr, seg0, seg1 - seg0, lz, lcoef, nz, tile, sh);
        } else {
            const int nw = compact_block<0>(P, seg0, seg1, lw, nullptr, sh);
            if (nw > 0) kernel_sum_block<KT>(P, lw, 0, nw, lz, lcoef, nz, tile, sh);
        }
        for (int i = seg0 + tid; i < seg1; i += BB) {
            P.status[i] &= 7;
            act[i - seg0] = i;
        }
        __syncthreads();
        nact = seg1 - seg0;
        nact_total = n;
        double cbu, cbl;
        int ciu, cil;
        select_block(P, act, nact, sh, cbu, ciu, cbl, cil);
        merge(cbu, ciu, cbl, cil, nact, -1, 0.0, -1, 0.0);
        if (res) from_global();
    };

    while (alive) {
        // ---- SMO iterations of this phase
        while (alive && bl - bu > thr) {
            if (iter >= P.max_iter) { status = SVM_NOT_CONVERGED; break; }
            const int yu = P.y[iu] > 0 ? 1 : -1, yl = P.y[il] > 0 ? 1 : -1;
            if (dense) {
                const float* xu = P.x + (size_t)iu * P.dpad;
                const float* xl = P.x + (size_t)il * P.dpad;
                if constexpr (std::is_same<KT, double>::value) {
                    for (int k = tid; k < P.dpad; k += BB) pairv[k] = make_float2(xu[k], xl[k]);
                    __syncthreads();
                    if (tid == 0) {
                        // sequential in k: the same rounding as the FP64 reference
#pragma clang fp contract(off)
                        double a = 0.0;
                        for (int k = 0; k < P.dpad; ++k) {
                            const double t = (double)pairv[k].x - (double)pairv[k].y;
                            a = a + t * t;
                        }
                        sh.pair[0] = exp(-P.gamma * a);
                    }
                } else if (wid == 0) {
                    // wave 0 alone stages the rows and sums the squared differences
                    float a = 0.f;
                    for (int k = lane; k < P.dpad; k += 64) {
                        const float u = xu[k], l = xl[k];
                        pairv[k] = make_float2(u, l);
                        const float t = u - l;
                        a = fmaf(t, t, a);
                    }
                    a = wave_sum_dpp(a);
                    if (lane == 0) sh.pair[0] = (double)kexp(-(float)P.gamma * a);
                }
            } else if (bits) {
                // wave 0 alone: lane k < wpr (at most 32) stages word k of both rows and counts its
                // bits; |u| and |l| travel packed 16 bits apart (each at most d <= 1024)
                if (wid == 0) {
                    const int wpr = P.wpr;
                    uint32_t wu = 0, wl = 0;
                    if (lane < wpr) {
                        wu = P.bits[(size_t)iu * wpr + lane];
                        wl = P.bits[(size_t)il * wpr + lane];
                        pairb[lane] = wu;
                        pairb[wpr + lane] = wl;
                    }
                    int c2 = __popc(wu) | (__popc(wl) << 16), cd = __popc(wu & wl);
                    sum2_lanes32(c2, cd);
                    const int cu = c2 & 0xffff, cl = c2 >> 16;
                    if (lane == 0) {
                        KT d2 = (KT)cu + (KT)cl - (KT)2 * (KT)cd;
                        if (d2 < (KT)0) d2 = (KT)0;
                        sh.pair[0] = (double)kexp((KT)(-(KT)P.gamma * d2));
                        sh.pair[1] = (double)cu;
                        sh.pair[2] = (double)cl;
                    }
                }
            } else {
                const int pu0 = P.row_ptr[iu], pu1 = P.row_ptr[iu + 1];
                const int pl0 = P.row_ptr[il], pl1 = P.row_ptr[il + 1];
                const int nu = pu1 - pu0, nl = pl1 - pl0;
                for (int k = tid; k < P.d; k += BB) pairv[k] = make_float2(0.f, 0.f);
                __syncthreads();
                float* pf = reinterpret_cast<float*>(pairv);
                for (int p = tid; p < nu; p += BB) pf[2 * P.col[pu0 + p]] = pat ? 1.f : P.val[pu0 + p];
                for (int p = tid; p < nl; p += BB) pf[2 * P.col[pl0 + p] + 1] = pat ? 1.f : P.val[pl0 + p];
                __syncthreads();
                if (wid == 0) {
                    KT su = 0, sl = 0, dot = 0;
                    for (int p = lane; p < nu; p += 64) {
                        const KT v = P.pattern_only ? (KT)1 : (KT)P.val[pu0 + p];
                        su += v * v;
                    }
                    for (int p = lane; p < nl; p += 64) {
                        const KT v = P.pattern_only ? (KT)1 : (KT)P.val[pl0 + p];
                        sl += v * v;
                        dot += v * (KT)pairv[P.col[pl0 + p]].x;
                    }
                    su = wave_sum(su);
                    sl = wave_sum(sl);
                    dot = wave_sum(dot);
                    if (lane == 0) {
                        KT d2 = su + sl - (KT)2 * dot;
                        if (d2 < (KT)0) d2 = (KT)0;
                        sh.pair[0] = (double)kexp((KT)(-(KT)P.gamma * d2));
                        sh.pair[1] = (double)su;
                        sh.pair[2] = (double)sl;
                    }
                }
            }
            __syncthreads();
            lap(0);
            const PairNew pn = pair_update(au, al, yu, yl, bu, bl, sh.pair[0], C);
            const KT gam = (KT)P.gamma;
            const KT nuu = dense ? (KT)0 : (KT)sh.pair[1], nll = dense ? (KT)0 : (KT)sh.pair[2];
            bool do_shrink = false;
            if (shrinking) {
                --counter;
                do_shrink = counter == 0;
            }
            double cbu = INFINITY, cbl = -INFINITY;
            int ciu = IDX_NONE, cil = IDX_NONE;
            int newcount = 0;
            constexpr int RPT = 4;
            for (int base = 0; base < nact; base += NG * RPT) {
                int ii[RPT], rr[RPT];
                bool vv[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const int t = base + r * NG + g;
                    vv[r] = t < nact;
                    rr[r] = vv[r] ? (res ? (int)act_l[t] : act[t] - seg0) : 0;
                    ii[r] = seg0 + rr[r];
                }
                KT du2[RPT], dl2[RPT];
                if (bits)
                    rows_dist_bits<KT, RPT>(P.wpr, rres ? bits_l : P.bits, pairb, rres ? rr : ii, vv, nuu, nll, du2,
                                            dl2);
                else if (rres)
                    rows_dist<KT, RPT>(dense, P.dpad, x_l, off_l, cols_l, vals_l, pat, pairv, rr, vv, gl, lpr, nuu,
                                       nll, du2, dl2);
                else
                    rows_dist<KT, RPT>(dense, P.dpad, P.x, P.row_ptr, P.col, P.val, pat, pairv, ii, vv, gl, lpr,
                                       nuu, nll, du2, dl2);
                bool keep[RPT];
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    keep[r] = false;
                    const int i = ii[r];
                    if (vv[r] && gl == 0) {
                        const double ku = (i == iu) ? 1.0 : (double)kexp(-gam * du2[r]);
                        const double kl = (i == il) ? 1.0 : (double)kexp(-gam * dl2[r]);
                        double* fp = res ? f_l + rr[r] : P.f + i;
                        uint8_t* sp = res ? st_l + rr[r] : P.status + i;
                        double fi;
                        {
#pragma clang fp contract(off)
                            fi = *fp + (pn.cu * ku + pn.cl * kl);
                        }
                        *fp = fi;
                        uint8_t st = *sp;
                        if (i == iu) {
                            st = st_make(yu > 0, pn.au, C);
                            *sp = st;
                            st_agent(P.alpha + i, pn.au);
                        } else if (i == il) {
                            st = st_make(yl > 0, pn.al, C);
                            *sp = st;
                            st_agent(P.alpha + i, pn.al);
                        }
                        keep[r] = !(do_shrink && shrink_rule(st, fi, bu, bl));
                        if (!keep[r]) *sp = st | 8;
                        if (keep[r]) {
                            if (st_in_up(st) && better_up(fi, i, cbu, ciu)) { cbu = fi; ciu = i; }
                            if (st_in_low(st) && better_low(fi, i, cbl, cil)) { cbl = fi; cil = i; }
                        }
                    }
                }
            }
            if (do_shrink) {
                // rows the rule removed carry the shrunk bit: one stable in-place compaction of
                // the list after the pass (each chunk is read before its first barrier and
                // written only below its own start)
                __syncthreads();
                for (int b0 = 0; b0 < nact; b0 += BB) {
                    const int t = b0 + (int)threadIdx.x;
                    int r = 0;
                    bool k = false;
                    if (t < nact) {
                        r = res ? (int)act_l[t] : act[t] - seg0;
                        k = !((res ? st_l[r] : P.status[seg0 + r]) & 8);
                    }
                    int tot;
                    const int pos = block_scan_keep(k, sh.wc, tot);
                    if (k) {
                        if (res) act_l[newcount + pos] = (uint16_t)r;
                        else act[newcount + pos] = seg0 + r;
                    }
                    newcount += tot;
                }
            }
            lap(1);
            block_reduce_sel_all<BB>(cbu, ciu, cbl, cil, sh.v, sh.i);
            __syncthreads();
            lap(2);
            if (do_shrink) nact = newcount;
            const long long tot = merge(cbu, ciu, cbl, cil, nact, iu, pn.au, il, pn.al);
            lap(3);
            if (prof_on) sh.pt[5] += 1;
            if (do_shrink) {
                shrunk += nact_total - tot;
                nact_total = tot;
                ++passes;
                counter = tot < H ? tot : H;
                if (counter < 1) counter = 1;
            }
            ++iter;
        }
        if (!alive || status != SVM_OK) break;
        if (shrinking) {
            rebuild(false);                     // the active set meets the tolerance: Alg. 6
            lap(4);
            ++n_recon;
            if (!alive) break;
            if (bl - bu > 2.0 * P.eps) {
                thr = 2.0 * P.eps;
                if (P.shrink_mode == SVM_SHRINK_SINGLE) shrinking = false;
                counter = H;
                continue;
            }
        }
        if (final_recompute && rechecks < 2) {
            ++rechecks;
            rebuild(true);
            lap(4);
            if (!alive) break;
            if (bl - bu > 2.0 * P.eps) {
                thr = 2.0 * P.eps;
                counter = H;
                continue;
            }
        }
        break;
    }
    if (alive && status == SVM_NOT_CONVERGED && nact_total < n) {
        rebuild(false);
        ++n_recon;
    }
    lap(4);
    // ---- threshold and summary over the team
    if (res) to_global();
    double x6[6] = {0, 0, 0, 0, 0, 0}, s6[6];
    if (alive) {
        double v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0;
        for (int i = seg0 + tid; i < seg1; i += BB) {
            const double a = ld_agent(P.alpha + i);
            const double yi = P.y[i] > 0 ? 1.0 : -1.0;
            if (a > 0.0 && a < C) { v0 += P.f[i]; v1 += 1.0; }
            v2 += a;
            v3 += a * yi * (P.f[i] + yi);
            if (a > 0.0) v4 += 1.0;
            if (a >= C) v5 += 1.0;
        }
        v0 = wave_sum(v0); v1 = wave_sum(v1); v2 = wave_sum(v2);
        v3 = wave_sum(v3); v4 = wave_sum(v4); v5 = wave_sum(v5);
        if (lane == 0) {
            sh.red[wid][0] = v0; sh.red[wid][1] = v1; sh.red[wid][2] = v2;
            sh.red[wid][3] = v3; sh.red[wid][4] = v4; sh.red[wid][5] = v5;
        }
        __syncthreads();
        if (tid < 64)
            for (int w = 0; w < BNW; ++w)
                for (int k = 0; k < 6; ++k) x6[k] += sh.red[w][k];
        __syncthreads();
        if (!team_sum(P, rank, seq++, x6, s6, true, sh)) alive = false;
    }
    // ---- completion: every member posts an acknowledgement and leaves; rank 0 waits for all of
    // them before it publishes the result (after which the host may reuse the team records)
    if (P.team > 1) {
        if (tid < 64) {
            unsigned v[REC_WORDS];
            for (int k = 0; k < REC_WORDS; ++k) v[k] = 0;
            team_write(P.trec, P.team, rank, seq, v);
        }
        if (rank == 0) {                  // rank is uniform in the workgroup
            if (tid == 0) sh.tok = 1;
            __syncthreads();
            if (tid < 64) {
                unsigned v[REC_WORDS];
                const bool ok = team_read(P.trec, P.team, seq, v, TEAM_WAIT_TICKS);
                if (tid == 0 && !ok) sh.tok = 0;
            }
            __syncthreads();
            if (!sh.tok) alive = false;
        }
    }
    if (prof_on) {
        lap(7);
        for (int k = 0; k < 8; ++k) atomicAdd(P.prof + k, sh.pt[k]);
    }
    if (rank == 0 && tid == 0) {
        BatchResult* R = P.res;
        if (!alive) status = SVM_EABORT;
        const double beta = alive && s6[1] > 0 ? s6[0] / s6[1] : 0.5 * (bu + bl);
        __hip_atomic_store(&R->beta, beta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->b_up, bu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->b_low, bl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->dual_obj, alive ? s6[2] - 0.5 * s6[3] : 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->iterations, iter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->n_sv, alive ? (int32_t)s6[4] : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->n_bsv, alive ? (int32_t)s6[5] : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->n_recon, n_recon, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->status, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->shrink_passes, passes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->shrunk_total, shrunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->t_start, t_start, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->t_end, wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&R->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
}

// Preparation job of the serving loop (one workgroup): the checks of the one-problem entry
// point's validation (labels +-1, finite values, CSR rows with increasing in-range columns),
// class counts, the largest CSR row, whether every CSR value is 1.0, dense packing into
// [n][dpad] rows, and zeroed team records.  The host reads the outcome from pinned memory, so
// admission never needs a kernel of its own while the loop holds the GPU.
DEV void prep_job(BatchShared& sh) {
    const BatchDesc& P = sh.P;
    const int tid = threadIdx.x;
    const int n = P.n, d = P.d;
    if (tid < 5) sh.pr[tid] = 0;
    __syncthreads();
    int err = 0, npos = 0, nneg = 0, maxnnz = 0, notpat = 0;
    for (int i = tid; i < n; i += BB) {
        const int8_t v = P.y[i];
        if (v == 1) ++npos;
        else if (v == -1) ++nneg;
        else err |= 1;
    }
    if (P.src_layout == SVM_CSR) {
        for (int i = tid; i < n; i += BB) {
            const int p0 = P.row_ptr[i], p1 = P.row_ptr[i + 1];
            if (i == 0 && p0 != 0) err |= 1;
            if (p1 < p0) {
                err |= 1;
                continue;
            }
            maxnnz = max(maxnnz, p1 - p0);
            for (int p = p0; p < p1; ++p) {
                const int c = P.col[p];
                if (c < 0 || c >= d) err |= 1;
                if (p > p0 && c <= P.col[p - 1]) err |= 1;
                const float v = P.val[p];
                if (!isfinite(v)) err |= 2;
                if (v != 1.f) notpat = 1;
            }
        }
    } else {
        const bool fm = P.src_layout == SVM_DENSE_FEATURE_MAJOR;
        const size_t tot = (size_t)n * P.dpad;
        float* out = const_cast<float*>(P.x);
        for (size_t e = tid; e < tot; e += BB) {
            const int i = (int)(e / P.dpad), k = (int)(e % P.dpad);
            float v = 0.f;
            if (k < d) v = fm ? P.xsrc[(size_t)k * P.ldx + i] : P.xsrc[(size_t)i * P.ldx + k];
            if (!isfinite(v)) err |= 2;
            out[e] = v;
        }
    }
    if (P.bits) {   // bitset rows for the LAY_BITS path (used only if every value is 1.0)
        uint32_t* out = const_cast<uint32_t*>(P.bits);
        const int wpr = P.wpr;
        for (size_t e = tid; e < (size_t)n * wpr; e += BB) out[e] = 0u;
        __syncthreads();
        for (int i = tid; i < n; i += BB) {
            const int p0 = P.row_ptr[i], p1 = P.row_ptr[i + 1];
            int cw = -1;
            uint32_t acc = 0u;
            for (int p = p0; p < p1; ++p) {
                const int c = P.col[p];
                if (c < 0 || c >= d) continue;
                if ((c >> 5) != cw) {
                    if (cw >= 0) out[(size_t)i * wpr + cw] |= acc;
                    cw = c >> 5;
                    acc = 0u;
                }
                acc |= 1u << (c & 31);
            }
            if (cw >= 0) out[(size_t)i * wpr + cw] |= acc;
        }
    }
    for (int k = tid; k < 2 * 16 * TEAM_MAX; k += BB) P.trec[k] = 0ull;
    if (err) atomicOr(&sh.pr[0], err);
    if (npos) atomicAdd(&sh.pr[1], npos);
    if (nneg) atomicAdd(&sh.pr[2], nneg);
    if (maxnnz) atomicMax(&sh.pr[3], maxnnz);
    if (notpat) atomicOr(&sh.pr[4], 1);
    __syncthreads();
    if (tid == 0) {
        PrepOut* o = P.prep;
        __hip_atomic_store(&o->err, sh.pr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&o->n_pos, sh.pr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&o->n_neg, sh.pr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&o->max_row_nnz, sh.pr[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&o->nnz, P.src_layout == SVM_CSR ? P.row_ptr[n] : 0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&o->pattern, sh.pr[4] ? 0 : 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // every thread's packed rows and zeroed records are released before the flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&P.prep->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
}

template <typename KT>
__global__ __launch_bounds__(BB) void smo_batch_kernel(BatchArgs A) {
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ BatchShared sh;
    const int tid = threadIdx.x;
    for (;;) {
        // ---- take a worker ticket (a problem and a rank in its team); wait until it is
        // published or the host stops the loop
        if (tid == 0) {
            const int t = atomicAdd(A.head, 1);
            int ok = 0;
            if (A.fixed_tail > 0) {
                ok = t < A.fixed_tail;
            } else {
                // Only the workgroup holding the lowest unpublished ticket (the leader) polls the
                // host-written tail and shutdown flag; it mirrors them into device memory, where
                // the other waiting workgroups poll.
                for (;;) {
                    const int m = __hip_atomic_load(A.mirror, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    if (t < m) { ok = 1; break; }
                    if (__hip_atomic_load(A.mirror + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) break;
                    if (t == m) {
                        const int tail = __hip_atomic_load(A.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                        if (tail > m) {
                            __hip_atomic_store(A.mirror, tail, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            continue;
                        }
                        if (__hip_atomic_load(A.shutdown, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) {
                            __hip_atomic_store(A.mirror + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(127);
                }
            }
            sh.ticket = ok ? t : -1;
            if (ok) {
                const int2 tk = A.tickets[t & (A.tcapacity - 1)];
                sh.rank = tk.y;
                sh.P = A.descs[tk.x & (A.capacity - 1)];
            }
        }
        __syncthreads();
        if (sh.ticket < 0) break;
        if (sh.rank < 0) prep_job(sh);
        else if (sh.P.lay == LAY_DENSE) solve_team<KT, LAY_DENSE>(sh, dyn);
        else if (sh.P.lay == LAY_BITS) solve_team<KT, LAY_BITS>(sh, dyn);
        else solve_team<KT, LAY_CSR_TABLE>(sh, dyn);
    }
}

// Bitset rows from CSR columns (one thread per row; columns increasing, as validated).
__global__ void pack_bits_kernel(int n, int d, int wpr, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 uint32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t* o = out + (size_t)i * wpr;
    for (int k = 0; k < wpr; ++k) o[k] = 0u;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int c = col[p];
        if (c >= 0 && c < d) o[c >> 5] |= 1u << (c & 31);
    }
}

hipError_t launch_pack_bits(int n, int d, int wpr, const int32_t* row_ptr, const int32_t* col, uint32_t* out,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    pack_bits_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, d, wpr, row_ptr, col, out);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int workgroups, int kprec, hipStream_t s) {
    BatchArgs c = a;
    if (kprec == SVM_KERNEL_FP64) {
        (void)hipFuncSetAttribute((const void*)smo_batch_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)BATCH_LDS);
        smo_batch_kernel<double><<<workgroups, BB, BATCH_LDS, s>>>(c);
    } else {
        (void)hipFuncSetAttribute((const void*)smo_batch_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)BATCH_LDS);
        smo_batch_kernel<float><<<workgroups, BB, BATCH_LDS, s>>>(c);
    }
    return hipGetLastError();
}

int batch_max_workgroups(int kprec) {
    const void* fn = kprec == SVM_KERNEL_FP64 ? (const void*)smo_batch_kernel<double>
                                              : (const void*)smo_batch_kernel<float>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BATCH_LDS);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, BB, BATCH_LDS) != hipSuccess) return 0;
    return nb * device_cu_count();
}

}  // namespace svm

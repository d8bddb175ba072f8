// svm_step.hip -- the persistent SMO loop of libsvmhip.so for gfx950.
//
// One cooperative launch runs the inner loop of Alg. 5 (Alg. 2 when shrinking
// is off) until the gap b_low - b_up drops to the phase tolerance or the
// iteration cap is reached.  Every iteration:
//   1. each workgroup stages the working pair (x_up, x_low) in LDS -- the
//      paper's broadcast -- and computes the FP64 pair update (eq:alphaup /
//      eq:rho) redundantly, as every MPI rank does;
//   2. it updates f (eq:fup) over the active rows of its segment, applies the
//      shrink rule (eq:shrink) on shrink iterations and compacts its active
//      list in place (Alg. 4), and reduces the two-threshold candidates
//      (eq:bminmax, lowest sample id on ties);
//   3. the workgroups exchange one record each -- the paper's Allreduce, here
//      tag-validated words in memory with no grid barrier -- after which every
//      workgroup merges all records identically and holds the next pair.
// A workgroup owns a fixed segment of the samples for the whole launch and,
// when it fits, keeps the segment's per-row state (f, status, active list,
// CSR offsets) and even its row payload in LDS, so an iteration reads HBM
// only for the working pair and the records.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "svm_device.h"
#include "svm_internal.h"

namespace svm {

static size_t al16(size_t v) { return (v + 15) & ~(size_t)15; }

// Dynamic LDS of one workgroup: the working pair, the payload words of the G records (G > 1),
// then, by mode, the segment's per-row state and its rows.
StepLds plan_step_lds(int lay, int d, int dpad, int max_row_nnz, int nseg_max, long long nnz_seg_max,
                      bool pattern_only, int max_mode, int G) {
    StepLds p{};
    const size_t rec = G > 1 ? sizeof(uint32_t) * REC_LDS_STRIDE * (size_t)G : 0;
    if (lay == LAY_BITS) {
        const int wpr = bits_wpr(d);
        p.pair_bytes = sizeof(uint32_t) * 2 * (size_t)wpr;
        p.rec_off = al16(p.pair_bytes);
        p.meta_off = p.rec_off + al16(rec);
        p.pay_off = p.meta_off + al16(2 * sizeof(double) * (size_t)nseg_max + sizeof(int) * (size_t)nseg_max +
                                      (size_t)nseg_max);
        const size_t pay = sizeof(uint32_t) * (size_t)wpr * nseg_max;
        if (max_mode >= STEP_LDS_ALL && p.pay_off + pay <= STEP_LDS_BUDGET) {
            p.mode = STEP_LDS_ALL;
            p.total = p.pay_off + pay;
        } else if (max_mode >= STEP_LDS_STATE && p.pay_off <= STEP_LDS_BUDGET) {
            p.mode = STEP_LDS_STATE;
            p.total = p.pay_off;
        } else {
            p.mode = STEP_GLOBAL;
            p.total = p.meta_off;
        }
        return p;
    }
    if (lay == LAY_DENSE) p.pair_bytes = sizeof(float2) * (size_t)dpad;
    else if (lay == LAY_CSR_TABLE) p.pair_bytes = sizeof(float2) * (size_t)d + sizeof(int) * 2 * (size_t)max_row_nnz;
    else
        p.pair_bytes = sizeof(float2) * (1 + 2 * (size_t)max_row_nnz) + al16(sizeof(uint16_t) * (size_t)d) +
                       sizeof(int) * 2 * (size_t)max_row_nnz;
    const bool csr = lay != LAY_DENSE;
    p.rec_off = al16(p.pair_bytes);
    p.meta_off = p.rec_off + al16(rec);
    const size_t meta = al16(2 * sizeof(double) * (size_t)nseg_max + sizeof(int) * (size_t)nseg_max +
                             (csr ? 2 * sizeof(int) * ((size_t)nseg_max + 1) : 0) + (size_t)nseg_max);
    p.pay_off = p.meta_off + meta;
    size_t pay;
    if (csr) pay = al16(sizeof(uint16_t) * (size_t)nnz_seg_max) + (pattern_only ? 0 : sizeof(float) * (size_t)nnz_seg_max);
    else pay = sizeof(float) * (size_t)dpad * (size_t)nseg_max;
    if (max_mode >= STEP_LDS_ALL && (!csr || d <= 65536) && p.pay_off + pay <= STEP_LDS_BUDGET) {
        p.mode = STEP_LDS_ALL;
        p.total = p.pay_off + pay;
    } else if (max_mode >= STEP_LDS_STATE && p.pay_off <= STEP_LDS_BUDGET) {
        p.mode = STEP_LDS_STATE;
        p.total = p.pay_off;
    } else {
        p.mode = STEP_GLOBAL;
        p.total = p.meta_off;
    }
    return p;
}

// element pairs per lane in one load batch of a CSR row streamed from HBM
constexpr int STREAM_CB2 = 6;

template <int LAY, typename KT, int LPR, int MODE, bool CACHE>
__global__ __launch_bounds__(STEP_BLOCK) void smo_loop_kernel(StepArgs A) {
    constexpr int BLOCK = STEP_BLOCK;
    constexpr int NW = BLOCK / 64;
    constexpr int NG = BLOCK / LPR;
    constexpr bool BITS = LAY == LAY_BITS;
    constexpr bool CSR = LAY == LAY_CSR_TABLE || LAY == LAY_CSR_SLOT;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_v[SEL_LDS(BLOCK)];
    __shared__ int s_i[SEL_LDS(BLOCK)];
    __shared__ int s_wc[NW];
    __shared__ double s_pair[4];     // K_ul, |u|^2, |l|^2
    __shared__ double s_sel[4];
    __shared__ int s_seli[3];
    __shared__ int s_prev_n;
    __shared__ unsigned long long s_ext[2];
    __shared__ int s_cache[4];       // kernel-row cache: slot of i_up, slot of i_low, hit up, hit low

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int g = tid / LPR, gl = tid % LPR;
    const int blk = blockIdx.x, G = gridDim.x;
    const double C = A.C;

    // ---- LDS: the working pair first
    float2* pairv = reinterpret_cast<float2*>(smem);
    uint32_t* pairb = reinterpret_cast<uint32_t*>(smem);   // LAY_BITS: pair rows' bitsets
    uint16_t* slot = nullptr;
    int* prev_cols = nullptr;
    if (LAY == LAY_CSR_TABLE) {
        prev_cols = reinterpret_cast<int*>(smem + sizeof(float2) * (size_t)A.d);
        for (int k = tid; k < A.d; k += BLOCK) pairv[k] = make_float2(0.f, 0.f);
    } else if (LAY == LAY_CSR_SLOT) {
        const int nv = 1 + 2 * A.max_row_nnz;
        slot = reinterpret_cast<uint16_t*>(smem + sizeof(float2) * (size_t)nv);
        prev_cols = reinterpret_cast<int*>(smem + sizeof(float2) * (size_t)nv + ((sizeof(uint16_t) * (size_t)A.d + 15) & ~(size_t)15));
        for (int k = tid; k < A.d; k += BLOCK) slot[k] = 0;
        if (tid == 0) pairv[0] = make_float2(0.f, 0.f);
    }
    if (tid == 0) s_prev_n = 0;

    // ---- this workgroup's segment and where its rows live during the launch
    const int seg0 = A.seg_start[blk];
    const int nseg = A.seg_start[blk + 1] - seg0;
    int nrows = A.cnt[blk];
    const int gbase = CSR ? A.row_ptr[seg0] : 0;
    const int pbase = (CSR && MODE != STEP_LDS_ALL) ? A.prp[seg0] : 0;
    double* F;
    double* AL = nullptr;   // alpha of the segment's rows (LDS modes)
    uint8_t* ST;
    int* L;           // active list: global ids (STEP_GLOBAL) or segment-local indices
    int* OFF = nullptr;
    int* OFF2 = nullptr;      // CSR rows from HBM: first element pair of each row, segment-relative
    float* XL = nullptr;
    uint32_t* XB = nullptr;   // LAY_BITS rows in LDS
    uint16_t* COLL = nullptr;
    float* VALL = nullptr;
    if constexpr (MODE == STEP_GLOBAL) {
        F = A.f + seg0;
        ST = A.status + seg0;
        L = A.act + seg0;
    } else {
        F = reinterpret_cast<double*>(smem + A.lds_meta_off);
        AL = F + A.nseg_max;
        L = reinterpret_cast<int*>(AL + A.nseg_max);
        OFF = L + A.nseg_max;
        OFF2 = OFF + (CSR ? A.nseg_max + 1 : 0);
        ST = reinterpret_cast<uint8_t*>(OFF2 + (CSR ? A.nseg_max + 1 : 0));
        for (int li = tid; li < nseg; li += BLOCK) {
            F[li] = A.f[seg0 + li];
            AL[li] = A.alpha[seg0 + li];
            ST[li] = A.status[seg0 + li];
        }
        if (!(CSR && MODE == STEP_LDS_STATE))
            for (int t = tid; t < nrows; t += BLOCK) L[t] = A.act[seg0 + t] - seg0;
        if (CSR)
            for (int li = tid; li <= nseg; li += BLOCK) OFF[li] = A.row_ptr[seg0 + li] - gbase;
        if (CSR && MODE != STEP_LDS_ALL)
            for (int li = tid; li <= nseg; li += BLOCK) OFF2[li] = A.prp[seg0 + li] - pbase;
        if constexpr (CSR && MODE == STEP_LDS_STATE) {
            // rows that take more than one load batch first, so that every lane group gets about
            // as many of them (the list's order changes no result: the selection is exact)
            __syncthreads();
            const int longp = LPR * STREAM_CB2;
            int nlong = 0;
            for (int pass = 0; pass < 2; ++pass) {
                int at_long = 0, at_short = 0;
                for (int base = 0; base < nrows; base += BLOCK) {
                    const int t = base + tid;
                    const int li = t < nrows ? A.act[seg0 + t] - seg0 : 0;
                    const bool lg = t < nrows && OFF2[li + 1] - OFF2[li] > longp;
                    const unsigned long long ml = __ballot(lg), ms = __ballot(t < nrows && !lg);
                    if (lane == 0) { s_wc[wid] = __popcll(ml); s_i[wid] = __popcll(ms); }
                    __syncthreads();
                    int offl = 0, offs = 0, totl = 0, tots = 0;
                    for (int w = 0; w < NW; ++w) {
                        const int cl = s_wc[w], cs = s_i[w];
                        offl += (w < wid) ? cl : 0;
                        offs += (w < wid) ? cs : 0;
                        totl += cl;
                        tots += cs;
                    }
                    const unsigned long long below = (1ull << lane) - 1ull;
                    if (pass == 1 && t < nrows) {
                        if (lg) L[at_long + offl + __popcll(ml & below)] = li;
                        else L[nlong + at_short + offs + __popcll(ms & below)] = li;
                    }
                    at_long += totl;
                    at_short += tots;
                    __syncthreads();
                }
                nlong = at_long;
            }
        }
        if constexpr (MODE == STEP_LDS_ALL) {
            if (BITS) {
                XB = reinterpret_cast<uint32_t*>(smem + A.lds_pay_off);
                const uint4* src = reinterpret_cast<const uint4*>(A.bits + (size_t)seg0 * A.wpr);
                uint4* dst = reinterpret_cast<uint4*>(XB);
                const int n4 = nseg * (A.wpr / 4);
                for (int e = tid; e < n4; e += BLOCK) dst[e] = src[e];
            } else if (CSR) {
                const int nnz = A.row_ptr[seg0 + nseg] - gbase;
                COLL = reinterpret_cast<uint16_t*>(smem + A.lds_pay_off);
                VALL = reinterpret_cast<float*>(smem + A.lds_pay_off + ((sizeof(uint16_t) * (size_t)A.nnz_seg_max + 15) & ~(size_t)15));
                for (int p = tid; p < nnz; p += BLOCK) {
                    COLL[p] = (uint16_t)A.col[gbase + p];
                    if (!A.pattern_only) VALL[p] = A.val[gbase + p];
                }
            } else {
                XL = reinterpret_cast<float*>(smem + A.lds_pay_off);
                const float4* src = reinterpret_cast<const float4*>(A.x + (size_t)seg0 * A.dpad);
                float4* dst = reinterpret_cast<float4*>(XL);
                const int n4 = nseg * A.dpad / 4;
                for (int e = tid; e < n4; e += BLOCK) dst[e] = src[e];
            }
        }
    }

    // ---- solver state (identical in every workgroup)
    Ctl* ctl = A.ctl;
    double bu = ctl->b_up, bl = ctl->b_low;
    double au = ctl->a_up, al = ctl->a_low;
    int iu = ctl->i_up, il = ctl->i_low;
    unsigned long long ext_u = 0, ext_l = 0;   // CSR extents of the pair rows (0: read row_ptr)
    long long iter = ctl->iter, counter = ctl->counter, n_act_total = ctl->n_active;
    long long passes = ctl->shrink_passes, shrunk = ctl->shrunk_total;
    int exit_reason = EXIT_NONE;
    unsigned long long work_rows = 0, work_nnz = 0, work_payload = 0, work_cache = 0;   // payload, cache: CACHE only
    long long cache_both = 0;
    if constexpr (CACHE) cache_both = ctl->cache_both;
    // per-phase timer of workgroup 0, kept in LDS so it costs no registers
    __shared__ unsigned long long s_pt[PROF_SLOTS + 1];
    const bool prof_on = A.prof != nullptr && blk == 0 && tid == 0;
    if (prof_on) {
        for (int k = 0; k < PROF_SLOTS; ++k) s_pt[k] = 0;
        s_pt[PROF_SLOTS] = wall_clock64();
    }
    auto lap = [&](int k) {
        if (prof_on) {
            const unsigned long long t = wall_clock64();
            s_pt[k] += t - s_pt[PROF_SLOTS];
            s_pt[PROF_SLOTS] = t;
        }
    };
    const bool kfull = CACHE && A.kfull;
    __syncthreads();
    lap(6);

    for (;;) {
        if (!(bl - bu > A.thr)) { exit_reason = EXIT_CONVERGED; break; }
        if (iter >= A.max_iter) { exit_reason = EXIT_MAXITER; break; }
        if (blk == 0 && tid == 0 && iter < A.trace_cap) {
            A.tr_iu[iter] = iu; A.tr_il[iter] = il; A.tr_bu[iter] = bu; A.tr_bl[iter] = bl;
        }
        // ---- 1. the working pair: labels, rows into LDS (alpha came with the records)
        if constexpr (CACHE) {
            // kernel rows of the pair from the cache: this workgroup's tags name the sample whose
            // row (over this segment) each slot holds; looked up by wave 1 while wave 0 (or the
            // whole workgroup) stages the rows.  With the whole kernel matrix in the cache every
            // row is there and K_ul too: nothing is staged.
            if (tid == 64) {
                if (kfull) {
                    s_cache[0] = iu;
                    s_cache[1] = il;
                    s_cache[2] = 1;
                    s_cache[3] = 1;
                } else {
                    const int S = A.cache_rows;
                    const int su = iu % S, sl = il % S;
                    const unsigned long long* tg = A.tags + (size_t)blk * S;
                    const unsigned long long ep = (unsigned long long)A.epoch << 32;
                    s_cache[0] = su;
                    s_cache[1] = sl;
                    s_cache[2] = ld_agent(tg + su) == (ep | (unsigned)iu);
                    s_cache[3] = ld_agent(tg + sl) == (ep | (unsigned)il);
                }
            }
            if (kfull && tid == 0) s_pair[0] = (double)reinterpret_cast<const KT*>(A.cache)[(size_t)iu * A.n + il];
        }
        const int yu = A.y[iu] > 0 ? 1 : -1;
        const int yl = A.y[il] > 0 ? 1 : -1;
        if (kfull) {
        } else if (LAY == LAY_DENSE) {
            const float* xu = A.x + (size_t)iu * A.dpad;
            const float* xl = A.x + (size_t)il * A.dpad;
            if constexpr (std::is_same<KT, float>::value) {
                // wave 0 alone stages the rows and sums the squared differences
                if (wid == 0) {
                    float a = 0.f;
                    for (int k = lane; k < A.dpad; k += 64) {
                        const float u = xu[k], l = xl[k];
                        pairv[k] = make_float2(u, l);
                        const float t = u - l;
                        a = fmaf(t, t, a);
                    }
                    a = wave_sum_dpp(a);
                    if (lane == 0) s_pair[0] = (double)kexp(-(float)A.gamma * a);
                }
            } else {
                for (int k = tid; k < A.dpad; k += BLOCK) pairv[k] = make_float2(xu[k], xl[k]);
                __syncthreads();
                // sequential in k: the same rounding as the FP64 reference
                if (tid == 0) {
#pragma clang fp contract(off)
                    double a = 0.0;
                    for (int k = 0; k < A.dpad; ++k) {
                        double t = (double)pairv[k].x - (double)pairv[k].y;
                        a = a + t * t;
                    }
                    s_pair[0] = exp(-A.gamma * a);
                }
            }
        } else if constexpr (BITS) {
            // wave 0 alone: lane k < wpr (at most 32) stages word k of both rows and counts its
            // bits; |u| and |l| travel packed 16 bits apart (each at most d <= 1024)
            if (wid == 0) {
                const int wpr = A.wpr;
                uint32_t wu = 0, wl = 0;
                if (lane < wpr) {
                    wu = A.bits[(size_t)iu * wpr + lane];
                    wl = A.bits[(size_t)il * wpr + lane];
                    pairb[lane] = wu;
                    pairb[wpr + lane] = wl;
                }
                int c2 = __popc(wu) | (__popc(wl) << 16), cd = __popc(wu & wl);
                sum2_lanes32(c2, cd);
                const int cu = c2 & 0xffff, cl = c2 >> 16;
                if (lane == 0) {
                    KT d2 = (KT)cu + (KT)cl - (KT)2 * (KT)cd;
                    if (d2 < (KT)0) d2 = (KT)0;
                    s_pair[0] = (double)kexp((KT)(-(KT)A.gamma * d2));
                    s_pair[1] = (double)cu;
                    s_pair[2] = (double)cl;
                }
            }
        } else {
            int pu0, pu1, pl0, pl1;
            if (ext_u) { pu0 = (int)(unsigned)(ext_u & 0xffffffffull); pu1 = (int)(unsigned)(ext_u >> 32); }
            else { pu0 = A.row_ptr[iu]; pu1 = A.row_ptr[iu + 1]; }
            if (ext_l) { pl0 = (int)(unsigned)(ext_l & 0xffffffffull); pl1 = (int)(unsigned)(ext_l >> 32); }
            else { pl0 = A.row_ptr[il]; pl1 = A.row_ptr[il + 1]; }
            const int nu = pu1 - pu0, nl = pl1 - pl0;
            // each thread's first element of both rows is loaded before the LDS clear, so the
            // two rows cost one memory round trip
            int cu0 = 0, cl0 = 0;
            float vu0 = 0.f, vl0 = 0.f;
            if (tid < nu) { cu0 = A.col[pu0 + tid]; vu0 = A.pattern_only ? 1.f : A.val[pu0 + tid]; }
            if (tid < nl) { cl0 = A.col[pl0 + tid]; vl0 = A.pattern_only ? 1.f : A.val[pl0 + tid]; }
            const int npv = s_prev_n;
            if (LAY == LAY_CSR_TABLE) {
                for (int j = tid; j < npv; j += BLOCK) pairv[prev_cols[j]] = make_float2(0.f, 0.f);
            } else {
                for (int j = tid; j < npv; j += BLOCK) slot[prev_cols[j]] = 0;
            }
            __syncthreads();
            float* pf = reinterpret_cast<float*>(pairv);
            auto stage_u = [&](int p, int c, float v) {
                if (LAY == LAY_CSR_TABLE) {
                    pf[2 * c] = v;
                } else {
                    slot[c] = (uint16_t)(1 + p);
                    pairv[1 + p] = make_float2(v, 0.f);
                }
                prev_cols[p] = c;
            };
            auto stage_l = [&](int p, int c, float v) {
                if (LAY == LAY_CSR_TABLE) {
                    pf[2 * c + 1] = v;
                } else {
                    const int sl = slot[c];
                    if (sl) {
                        pf[2 * sl + 1] = v;
                    } else {
                        slot[c] = (uint16_t)(1 + nu + p);
                        pairv[1 + nu + p] = make_float2(0.f, v);
                    }
                }
                prev_cols[nu + p] = c;
            };
            if (tid < nu) stage_u(tid, cu0, vu0);
            for (int p = tid + BLOCK; p < nu; p += BLOCK)
                stage_u(p, A.col[pu0 + p], A.pattern_only ? 1.f : A.val[pu0 + p]);
            // the slot map needs every column of the up row before the low row looks it up
            if (LAY == LAY_CSR_SLOT) __syncthreads();
            if (tid < nl) stage_l(tid, cl0, vl0);
            for (int p = tid + BLOCK; p < nl; p += BLOCK)
                stage_l(p, A.col[pl0 + p], A.pattern_only ? 1.f : A.val[pl0 + p]);
            __syncthreads();
            if (tid == 0) s_prev_n = nu + nl;
            if (wid == 0) {
                // |u|^2, |l|^2 and u.l from the staged rows (the values as loaded, lane-strided)
                KT su = 0, sl2 = 0, dot = 0;
                for (int p = lane; p < nu; p += 64) {
                    const KT v = (KT)((LAY == LAY_CSR_TABLE) ? pf[2 * prev_cols[p]] : pairv[1 + p].x);
                    su += v * v;
                }
                for (int p = lane; p < nl; p += 64) {
                    const int c = prev_cols[nu + p];
                    const float2 e = (LAY == LAY_CSR_TABLE) ? pairv[c] : pairv[slot[c]];
                    const KT v = (KT)e.y;
                    sl2 += v * v;
                    dot += v * (KT)e.x;
                }
                su = wave_sum(su);
                sl2 = wave_sum(sl2);
                dot = wave_sum(dot);
                if (lane == 0) {
                    KT d2 = su + sl2 - (KT)2 * dot;
                    if (d2 < (KT)0) d2 = (KT)0;
                    s_pair[0] = (double)kexp((KT)(-(KT)A.gamma * d2));
                    s_pair[1] = (double)su;
                    s_pair[2] = (double)sl2;
                }
            }
        }
        __syncthreads();
        const PairNew pn = pair_update(au, al, yu, yl, bu, bl, s_pair[0], C);
        // kernel-row cache of this iteration: hits, and which missing rows get stored (when both
        // rows map to one slot, only the up row may take it)
        const int c_su = CACHE ? s_cache[0] : 0, c_sl = CACHE ? s_cache[1] : 0;
        const bool c_hu = CACHE && s_cache[2], c_hl = CACHE && s_cache[3];
        const bool c_stu = CACHE && !c_hu, c_stl = CACHE && !c_hl && c_sl != c_su;
        const bool need_row = !(c_hu && c_hl);
        const KT gam = (KT)A.gamma;
        const KT nuu = (CSR || BITS) ? (KT)s_pair[1] : (KT)0, nll = (CSR || BITS) ? (KT)s_pair[2] : (KT)0;

        bool do_shrink = false;
        if (A.H > 0) {
            --counter;
            do_shrink = counter == 0;
        }
        lap(0);

        // ---- 2. f update over the active rows of this segment, candidates, shrink rule
        double cbu = INFINITY, cbl = -INFINITY;
        int ciu = IDX_NONE, cil = IDX_NONE;
        work_rows += (unsigned long long)nrows;
        if constexpr (CACHE) {
            if (need_row) work_payload += (unsigned long long)nrows;
            work_cache += (unsigned long long)nrows * ((int)c_hu + (int)c_hl + (int)c_stu + (int)c_stl);
        }
        // f update (eq:fup), the pair's alpha and status, the shrink rule and the candidates of
        // one active row; returns whether the row stays active
        auto update_row = [&](int li, int i, double ku, double kl) -> bool {
            double fi;
            {
#pragma clang fp contract(off)
                fi = F[li] + (pn.cu * ku + pn.cl * kl);
            }
            F[li] = fi;
            uint8_t st = ST[li];
            if (i == iu) {
                st = st_make(yu > 0, pn.au, C);
                ST[li] = st;
                if constexpr (MODE == STEP_GLOBAL) st_agent(A.alpha + i, pn.au);
                else AL[li] = pn.au;
            } else if (i == il) {
                st = st_make(yl > 0, pn.al, C);
                ST[li] = st;
                if constexpr (MODE == STEP_GLOBAL) st_agent(A.alpha + i, pn.al);
                else AL[li] = pn.al;
            }
            const bool keep = !(do_shrink && shrink_rule(st, fi, bu, bl));
            if (keep) {
                if (st_in_up(st) && better_up(fi, i, cbu, ciu)) { cbu = fi; ciu = i; }
                if (st_in_low(st) && better_low(fi, i, cbl, cil)) { cbl = fi; cil = i; }
            }
            return keep;
        };
        // a row the shrink rule removes is marked in its own entry of the active list (-1); the
        // list is compacted once at the end of the pass, so the stream has no barriers
        bool rows_done = false;
        if constexpr (CACHE) {
            if (!need_row) {
                // both kernel rows come from the cache: no row data, one thread per active row
                const KT* cu = reinterpret_cast<const KT*>(A.cache) + (size_t)c_su * A.n;
                const KT* cl = reinterpret_cast<const KT*>(A.cache) + (size_t)c_sl * A.n;
                for (int base = 0; base < nrows; base += BLOCK) {
                    const int t = base + tid;
                    const bool valid = t < nrows;
                    const int li = valid ? (MODE == STEP_GLOBAL ? L[t] - seg0 : L[t]) : 0;
                    const int i = seg0 + li;
                    bool keep = false;
                    if (valid) keep = update_row(li, i, (double)cu[i], (double)cl[i]);
                    if (do_shrink && valid && !keep) L[t] = -1;
                }
                rows_done = true;
            }
        }
        for (int base = 0; base < (rows_done ? 0 : nrows); base += NG) {
            const int t = base + g;
            const bool valid = t < nrows;
            const int li = valid ? (MODE == STEP_GLOBAL ? L[t] - seg0 : L[t]) : 0;
            const int i = seg0 + li;
            bool keep = false;
            if (valid) {
                KT du2 = (KT)0, dl2 = (KT)0;
                if constexpr (LAY == LAY_DENSE) {
                    const float* xr = (MODE == STEP_LDS_ALL) ? XL + (size_t)li * A.dpad : A.x + (size_t)i * A.dpad;
                    dense_dist<KT>(xr, pairv, A.dpad, du2, dl2);
                } else if constexpr (BITS) {
                    // one lane per row: popcounts of the row's bitset against the pair's
                    const uint4* xr = reinterpret_cast<const uint4*>(
                        (MODE == STEP_LDS_ALL) ? XB + (size_t)li * A.wpr : A.bits + (size_t)i * A.wpr);
                    const uint4* pu = reinterpret_cast<const uint4*>(pairb);
                    const uint4* pl = reinterpret_cast<const uint4*>(pairb + A.wpr);
                    int nn = 0, su = 0, sl2 = 0;
                    for (int w4 = 0; w4 < A.wpr / 4; ++w4) {
                        const uint4 v = xr[w4], a = pu[w4], b = pl[w4];
                        nn += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
                        su += __popc(v.x & a.x) + __popc(v.y & a.y) + __popc(v.z & a.z) + __popc(v.w & a.w);
                        sl2 += __popc(v.x & b.x) + __popc(v.y & b.y) + __popc(v.z & b.z) + __popc(v.w & b.w);
                    }
                    work_nnz += (unsigned long long)nn;
                    du2 = (KT)nn + nuu - (KT)2 * (KT)su;
                    dl2 = (KT)nn + nll - (KT)2 * (KT)sl2;
                    if (du2 < (KT)0) du2 = (KT)0;
                    if (dl2 < (KT)0) dl2 = (KT)0;
                } else {
                    int p0, p1;
                    if constexpr (MODE == STEP_GLOBAL) {
                        p0 = A.row_ptr[i] - gbase;
                        p1 = A.row_ptr[i + 1] - gbase;
                    } else {
                        p0 = OFF[li];
                        p1 = OFF[li + 1];
                    }
                    if (gl == 0) work_nnz += (unsigned long long)(p1 - p0);
                    KT nn = 0, su = 0, sl2 = 0;
                    if constexpr (MODE == STEP_LDS_ALL) {
                        for (int p = p0 + gl; p < p1; p += LPR) {
                            const int c = COLL[p];
                            const KT v = A.pattern_only ? (KT)1 : (KT)VALL[p];
                            const float2 ul = (LAY == LAY_CSR_TABLE) ? pairv[c] : pairv[slot[c]];
                            nn += v * v;
                            su += v * (KT)ul.x;
                            sl2 += v * (KT)ul.y;
                        }
                    } else {
                        // columns and values from HBM as the row's element pairs: one word of two
                        // u16 ids and one float2 per pair, CB2 pairs loaded before any is used (a
                        // row of odd length ends with a zero element, which adds nothing)
                        constexpr int CB2 = STREAM_CB2;
                        int q0, q1;
                        if constexpr (MODE == STEP_GLOBAL) {
                            q0 = A.prp[i];
                            q1 = A.prp[i + 1];
                        } else {
                            q0 = pbase + OFF2[li];
                            q1 = pbase + OFF2[li + 1];
                        }
                        const float2* v2 = reinterpret_cast<const float2*>(A.val2);
                        for (int qb = q0 + gl; qb < q1; qb += LPR * CB2) {
                            uint32_t cc[CB2];
                            float2 vv[CB2];
#pragma unroll
                            for (int u = 0; u < CB2; ++u) {
                                const int q = qb + u * LPR;
                                cc[u] = q < q1 ? A.col2[q] : 0u;
                                vv[u] = q < q1 ? v2[q] : make_float2(0.f, 0.f);
                            }
#pragma unroll
                            for (int u = 0; u < CB2; ++u) {
                                if (qb + u * LPR >= q1) break;
                                const KT va = (KT)vv[u].x, vb = (KT)vv[u].y;
                                const int ca = (int)(cc[u] & 0xffffu), cb = (int)(cc[u] >> 16);
                                const float2 ua = (LAY == LAY_CSR_TABLE) ? pairv[ca] : pairv[slot[ca]];
                                const float2 ub = (LAY == LAY_CSR_TABLE) ? pairv[cb] : pairv[slot[cb]];
                                nn += va * va;
                                su += va * (KT)ua.x;
                                sl2 += va * (KT)ua.y;
                                nn += vb * vb;
                                su += vb * (KT)ub.x;
                                sl2 += vb * (KT)ub.y;
                            }
                        }
                    }
#pragma unroll
                    for (int off = LPR / 2; off > 0; off >>= 1) {
                        nn += __shfl_xor(nn, off);
                        su += __shfl_xor(su, off);
                        sl2 += __shfl_xor(sl2, off);
                    }
                    du2 = nn + nuu - (KT)2 * su;
                    dl2 = nn + nll - (KT)2 * sl2;
                    if (du2 < (KT)0) du2 = (KT)0;
                    if (dl2 < (KT)0) dl2 = (KT)0;
                }
                if (gl == 0) {
                    double ku, kl;
                    if constexpr (CACHE) {
                        KT* cv = reinterpret_cast<KT*>(A.cache);
                        KT* cu = cv + (size_t)c_su * A.n + i;
                        KT* cl = cv + (size_t)c_sl * A.n + i;
                        ku = c_hu ? (double)*cu : (i == iu) ? 1.0 : (double)kexp(-gam * du2);
                        kl = c_hl ? (double)*cl : (i == il) ? 1.0 : (double)kexp(-gam * dl2);
                        if (c_stu) *cu = (KT)ku;
                        if (c_stl) *cl = (KT)kl;
                    } else {
                        ku = (i == iu) ? 1.0 : (double)kexp(-gam * du2);
                        kl = (i == il) ? 1.0 : (double)kexp(-gam * dl2);
                    }
                    keep = update_row(li, i, ku, kl);
                }
            }
            if (do_shrink && valid && gl == 0 && !keep) L[t] = -1;
        }
        if (do_shrink) {
            // stable in-place compaction of the marked list: every chunk is read before its
            // first barrier and written only below its own start
            __syncthreads();
            int newcount = 0;
            for (int base = 0; base < nrows; base += BLOCK) {
                const int t = base + tid;
                const int v = t < nrows ? L[t] : -1;
                const unsigned long long m = __ballot(v >= 0);
                if (lane == 0) s_wc[wid] = __popcll(m);
                __syncthreads();
                int off = 0, tot = 0;
                for (int w = 0; w < NW; ++w) {
                    const int c = s_wc[w];
                    off += (w < wid) ? c : 0;
                    tot += c;
                }
                if (v >= 0) L[newcount + off + __popcll(m & ((1ull << lane) - 1ull))] = v;
                newcount += tot;
                __syncthreads();
            }
            nrows = newcount;
        }
        if constexpr (CACHE) {
            if (tid == 0) {
                unsigned long long* tg = A.tags + (size_t)A.cache_rows * blk;
                const unsigned long long ep = (unsigned long long)A.epoch << 32;
                if (c_stu) st_agent(tg + c_su, ep | (unsigned)iu);
                if (c_stl) st_agent(tg + c_sl, ep | (unsigned)il);
                if (c_hu && c_hl) ++cache_both;
            }
        }
        lap(1);

        block_reduce_sel_wave0<BLOCK>(cbu, ciu, cbl, cil, s_v, s_i);   // wave 0 publishes
        // alpha and CSR extent of this workgroup's candidates: its own rows, which no other
        // workgroup writes, so they travel in the records instead of being re-read later
        double cau = 0.0, cal = 0.0;
        unsigned long long ceu = 0, cel = 0;
        if (wid == 0) {   // every lane of wave 0: the record's words are stored one per lane
            if (ciu != IDX_NONE) {
                if constexpr (MODE == STEP_GLOBAL) cau = ld_agent(A.alpha + ciu);
                else cau = AL[ciu - seg0];
                if constexpr (CSR) {
                    unsigned p0, p1;
                    if constexpr (MODE == STEP_GLOBAL) { p0 = (unsigned)A.row_ptr[ciu]; p1 = (unsigned)A.row_ptr[ciu + 1]; }
                    else { p0 = (unsigned)(gbase + OFF[ciu - seg0]); p1 = (unsigned)(gbase + OFF[ciu - seg0 + 1]); }
                    ceu = (unsigned long long)p0 | ((unsigned long long)p1 << 32);
                }
            }
            if (cil != IDX_NONE) {
                if constexpr (MODE == STEP_GLOBAL) cal = ld_agent(A.alpha + cil);
                else cal = AL[cil - seg0];
                if constexpr (CSR) {
                    unsigned p0, p1;
                    if constexpr (MODE == STEP_GLOBAL) { p0 = (unsigned)A.row_ptr[cil]; p1 = (unsigned)A.row_ptr[cil + 1]; }
                    else { p0 = (unsigned)(gbase + OFF[cil - seg0]); p1 = (unsigned)(gbase + OFF[cil - seg0 + 1]); }
                    cel = (unsigned long long)p0 | ((unsigned long long)p1 << 32);
                }
            }
        }
        // ---- 3. exchange (the paper's Allreduce of the b's): every workgroup stores its record
        // as tag-validated words and reads everybody's record; no barrier, no fence, no atomic RMW
        if (G > 1) {
            const int par = (int)(iter & 1);
            const unsigned tg = (unsigned)(iter + 1);
            const unsigned long long TAG = (unsigned long long)tg << 32;
            if (wid == 0 && lane < REC_WORDS) {   // word `lane` of the record, one store per lane
                const unsigned long long bub = (unsigned long long)__double_as_longlong(cbu);
                const unsigned long long blb = (unsigned long long)__double_as_longlong(cbl);
                const unsigned long long aub = (unsigned long long)__double_as_longlong(cau);
                const unsigned long long alb = (unsigned long long)__double_as_longlong(cal);
                unsigned long long x;
                switch (lane) {
                    case 0: x = bub; break;
                    case 1: x = bub >> 32; break;
                    case 2: x = blb; break;
                    case 3: x = blb >> 32; break;
                    case 4: x = (unsigned)ciu; break;
                    case 5: x = (unsigned)cil; break;
                    case 6: x = (unsigned)nrows; break;
                    case 7: x = aub; break;
                    case 8: x = aub >> 32; break;
                    case 9: x = alb; break;
                    case 10: x = alb >> 32; break;
                    case 11: x = ceu; break;
                    case 12: x = ceu >> 32; break;
                    case 13: x = cel; break;
                    default: x = cel >> 32; break;
                }
                st_agent(A.rec[par * G + blk].w + lane, TAG | (x & 0xffffffffull));
            }
            lap(2);
            double rbu = INFINITY, rbl = -INFINITY, rau = 0.0, ral = 0.0;
            int riu = IDX_NONE, ril = IDX_NONE;
            unsigned long long reu = 0, rel = 0;
            long long rcnt = 0;
            int ab = 0;
            // every wave polls whole records, four per load instruction (16 lanes per record,
            // one 128-byte line each; a lane re-reads its word until it carries the tag), and
            // puts their payload halves into LDS; a wave issues the loads of up to QW groups
            // of four records before it waits, so the exchange is one memory round trip
            {
                constexpr int QW = 4;
                uint32_t* RW = reinterpret_cast<uint32_t*>(smem + A.lds_rec_off);
                const int sub = lane >> 4, wd = lane & 15;
                const unsigned long long t0 = wall_clock64();
                for (int q0 = wid; 4 * q0 < G && !ab; q0 += NW * QW) {
                    unsigned x[QW];
                    bool ok[QW];
#pragma unroll
                    for (int j = 0; j < QW; ++j) {
                        const int r = 4 * (q0 + NW * j) + sub;
                        ok[j] = !(r < G && wd < REC_WORDS);
                        x[j] = 0u;
                    }
                    for (;;) {
                        bool all = true;
#pragma unroll
                        for (int j = 0; j < QW; ++j) {
                            if (!ok[j]) {
                                const int r = 4 * (q0 + NW * j) + sub;
                                const unsigned long long y = ld_agent(A.rec[par * G + r].w + wd);
                                ok[j] = (unsigned)(y >> 32) == tg;
                                x[j] = (unsigned)(y & 0xffffffffull);
                            }
                            all = all && ok[j];
                        }
                        if (__all(all)) break;
                        if (wall_clock64() - t0 > A.spin_limit) { ab = 1; break; }
                        __builtin_amdgcn_s_sleep(1);
                    }
#pragma unroll
                    for (int j = 0; j < QW; ++j) {
                        const int r = 4 * (q0 + NW * j) + sub;
                        if (r < G && wd < REC_WORDS) RW[r * REC_LDS_STRIDE + wd] = x[j];
                    }
                }
            }
            if (__syncthreads_or(ab)) {
                if (tid == 0) __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                exit_reason = EXIT_ABORT;
                break;
            }
            if (tid < G) {
                const uint32_t* RW = reinterpret_cast<const uint32_t*>(smem + A.lds_rec_off) + tid * REC_LDS_STRIDE;
                unsigned v[REC_WORDS];
#pragma unroll
                for (int k = 0; k < REC_WORDS; ++k) v[k] = RW[k];
                rbu = __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
                rbl = __longlong_as_double((long long)(((unsigned long long)v[3] << 32) | v[2]));
                riu = (int)v[4];
                ril = (int)v[5];
                rcnt = (long long)v[6];
                rau = __longlong_as_double((long long)(((unsigned long long)v[8] << 32) | v[7]));
                ral = __longlong_as_double((long long)(((unsigned long long)v[10] << 32) | v[9]));
                reu = ((unsigned long long)v[12] << 32) | v[11];
                rel = ((unsigned long long)v[14] << 32) | v[13];
            }
            lap(3);
            // reduce (value, id) and the record holding each winner publishes its payload
            // (alpha, CSR extent); with at most 64 records wave 0 holds them all
            const int myiu = riu, myil = ril;
            if (G <= 64) {
                if (wid == 0) {
                    const long long csum = do_shrink ? wave_sum(rcnt) : 0;
                    wave_reduce_sel(rbu, riu, rbl, ril);
                    if (tid < G) {
                        if (myiu != IDX_NONE && myiu == riu) { s_sel[2] = rau; s_ext[0] = reu; }
                        if (myil != IDX_NONE && myil == ril) { s_sel[3] = ral; s_ext[1] = rel; }
                    }
                    if (tid == 0) {
                        s_sel[0] = rbu; s_sel[1] = rbl;
                        s_seli[0] = riu; s_seli[1] = ril;
                        if (do_shrink) s_seli[2] = (int)csum;
                    }
                }
            } else {
                // waves 0 .. NR-1 hold 64 records each: reduce within them, then combine NR values
                const int NR = (G + 63) / 64;
                if (wid < NR) {
                    const long long csum = do_shrink ? wave_sum(rcnt) : 0;
                    wave_reduce_sel(rbu, riu, rbl, ril);
                    if (lane == 0) {
                        s_v[wid] = rbu; s_i[wid] = riu;
                        s_v[NW + wid] = rbl; s_i[NW + wid] = ril;
                        s_wc[wid] = (int)csum;
                    }
                }
                __syncthreads();
                double xbu = s_v[0], xbl = s_v[NW];
                int xiu = s_i[0], xil = s_i[NW];
                for (int w = 1; w < NR; ++w) {
                    if (better_up(s_v[w], s_i[w], xbu, xiu)) { xbu = s_v[w]; xiu = s_i[w]; }
                    if (better_low(s_v[NW + w], s_i[NW + w], xbl, xil)) { xbl = s_v[NW + w]; xil = s_i[NW + w]; }
                }
                if (tid < G) {
                    if (myiu != IDX_NONE && myiu == xiu) { s_sel[2] = rau; s_ext[0] = reu; }
                    if (myil != IDX_NONE && myil == xil) { s_sel[3] = ral; s_ext[1] = rel; }
                }
                if (tid == 0) {
                    s_sel[0] = xbu; s_sel[1] = xbl;
                    s_seli[0] = xiu; s_seli[1] = xil;
                    if (do_shrink) {
                        long long c = 0;
                        for (int w = 0; w < NR; ++w) c += s_wc[w];
                        s_seli[2] = (int)c;
                    }
                }
            }
        } else {
            if (tid == 0) {
                s_sel[0] = cbu; s_sel[1] = cbl; s_sel[2] = cau; s_sel[3] = cal;
                s_seli[0] = ciu; s_seli[1] = cil;
                s_seli[2] = nrows;
                s_ext[0] = ceu; s_ext[1] = cel;
            }
            lap(2);
        }
        __syncthreads();
        bu = s_sel[0];
        bl = s_sel[1];
        au = s_sel[2];
        al = s_sel[3];
        ext_u = s_ext[0];
        ext_l = s_ext[1];
        iu = s_seli[0] == IDX_NONE ? -1 : s_seli[0];
        il = s_seli[1] == IDX_NONE ? -1 : s_seli[1];
        if (do_shrink) {
            const long long tot = s_seli[2];
            shrunk += n_act_total - tot;
            n_act_total = tot;
            ++passes;
            counter = tot < A.H ? tot : A.H;
            if (counter < 1) counter = 1;
        }
        ++iter;
        lap(4);
        if (prof_on) s_pt[5] += 1;
    }

    // ---- write the segment back for the host-side phases (reconstruction, selection)
    if constexpr (MODE != STEP_GLOBAL) {
        for (int li = tid; li < nseg; li += BLOCK) {
            A.f[seg0 + li] = F[li];
            A.alpha[seg0 + li] = AL[li];
            A.status[seg0 + li] = ST[li];
        }
        for (int t = tid; t < nrows; t += BLOCK) A.act[seg0 + t] = seg0 + L[t];
    }
    if (tid == 0) A.cnt[blk] = nrows;
    if (A.work) {
        unsigned long long wn = wave_sum(work_nnz);
        __syncthreads();
        if (lane == 0) s_v[wid] = __longlong_as_double((long long)wn);
        __syncthreads();
        if (tid == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < NW; ++w) t += (unsigned long long)__double_as_longlong(s_v[w]);
            A.work[4 * blk] = work_rows;
            A.work[4 * blk + 1] = t;
            A.work[4 * blk + 2] = CACHE ? work_payload : work_rows;
            A.work[4 * blk + 3] = work_cache;
        }
    }
    if (prof_on) {
        lap(7);
        for (int k = 0; k < PROF_SLOTS; ++k) A.prof[k] += s_pt[k];
    }
    if (blk == 0 && tid == 0) {
        ctl->b_up = bu; ctl->b_low = bl; ctl->i_up = iu; ctl->i_low = il;
        ctl->a_up = au; ctl->a_low = al;
        ctl->iter = iter; ctl->counter = counter; ctl->n_active = n_act_total;
        ctl->shrink_passes = passes; ctl->shrunk_total = shrunk;
        if constexpr (CACHE) ctl->cache_both = cache_both;
        ctl->exit_reason = exit_reason;
    }
}

// ------------------------------------------------------------------ dispatch

bool step_cache_capable(int lay, int mode) { return lay != LAY_BITS && mode != STEP_LDS_ALL; }

template <int LAY, typename KT, int LPR, int MODE>
static const void* loop_fn(bool cache) {
    if constexpr (LAY != LAY_BITS && MODE != STEP_LDS_ALL) {
        if (cache) return (const void*)smo_loop_kernel<LAY, KT, LPR, MODE, true>;
    }
    return (const void*)smo_loop_kernel<LAY, KT, LPR, MODE, false>;
}

template <int LAY, typename KT, int MODE>
static const void* pick_lpr(int lpr, bool cache) {
    if constexpr (LAY == LAY_DENSE || LAY == LAY_BITS) {
        return loop_fn<LAY, KT, 1, MODE>(cache);
    } else {
        switch (lpr) {
            case 1: return loop_fn<LAY, KT, 1, MODE>(cache);
            case 2: return loop_fn<LAY, KT, 2, MODE>(cache);
            case 4: return loop_fn<LAY, KT, 4, MODE>(cache);
            case 8: return loop_fn<LAY, KT, 8, MODE>(cache);
            case 16: return loop_fn<LAY, KT, 16, MODE>(cache);
            default: return loop_fn<LAY, KT, 32, MODE>(cache);
        }
    }
}

template <int LAY, typename KT>
static const void* pick_mode(int mode, int lpr, bool cache) {
    if (mode == STEP_LDS_ALL) return pick_lpr<LAY, KT, STEP_LDS_ALL>(lpr, false);
    if (mode == STEP_LDS_STATE) return pick_lpr<LAY, KT, STEP_LDS_STATE>(lpr, cache);
    return pick_lpr<LAY, KT, STEP_GLOBAL>(lpr, cache);
}

static const void* pick(int lay, int kprec, int mode, int lpr, bool cache) {
    if (kprec == SVM_KERNEL_FP64) {
        if (lay == LAY_DENSE) return pick_mode<LAY_DENSE, double>(mode, lpr, cache);
        if (lay == LAY_BITS) return pick_mode<LAY_BITS, double>(mode, lpr, false);
        if (lay == LAY_CSR_TABLE) return pick_mode<LAY_CSR_TABLE, double>(mode, lpr, cache);
        return pick_mode<LAY_CSR_SLOT, double>(mode, lpr, cache);
    }
    if (lay == LAY_DENSE) return pick_mode<LAY_DENSE, float>(mode, lpr, cache);
    if (lay == LAY_BITS) return pick_mode<LAY_BITS, float>(mode, lpr, false);
    if (lay == LAY_CSR_TABLE) return pick_mode<LAY_CSR_TABLE, float>(mode, lpr, cache);
    return pick_mode<LAY_CSR_SLOT, float>(mode, lpr, cache);
}

hipError_t launch_step(const StepArgs& a, int G, int lpr, int kprec, size_t lds, hipStream_t s) {
    const void* fn = pick(a.lay, kprec, a.mode, lpr, a.cache != nullptr);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    StepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(STEP_BLOCK), args, (unsigned)lds, s);
}

int step_max_blocks(int lay, int lpr, int kprec, int mode, size_t lds, bool cache) {
    const void* fn = pick(lay, kprec, mode, lpr, cache);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, STEP_BLOCK, lds) != hipSuccess) return 0;
    return nb * device_cu_count();
}

}  // namespace svm

// svm_kernels.hip -- device code of libsvmhip.so for gfx950 (CDNA4, wave64).
//
// The SMO step of the paper (Alg. 2 / Alg. 4: pair update, f update of eq:fup
// over the active set, two-threshold selection of eq:bminmax, shrink rule of
// eq:shrink) runs as ONE persistent cooperative launch per driver phase:
// every workgroup owns a fixed slice of the samples, keeps its active list
// compacted in place, and the workgroups meet once per iteration at a grid
// barrier to merge their (b_up, i_up, b_low, i_low) records.  Everything the
// paper does with MPI_Bcast / MPI_Allreduce / GA get-put becomes LDS staging
// of the working pair, wave64 shuffle reductions and one barrier.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "svm_internal.h"

namespace svm {

#define DEV __device__ __forceinline__

constexpr double PAIR_TAU = 1e-12;    // floor for eta = K_uu + K_ll - 2 K_ul
constexpr double PAIR_DELTA = 1e-12;  // alpha within DELTA*C of 0 or C is put on the bound
constexpr int IDX_NONE = 0x7fffffff;  // empty side of a reduction

// ------------------------------------------------------------------ small helpers

DEV bool st_in_up(uint8_t s) {       // I0 u I1 u I2
    return (s & ST_FREE) || ((s & ST_YPOS) ? !(s & ST_ATC) : (s & ST_ATC));
}
DEV bool st_in_low(uint8_t s) {      // I0 u I3 u I4
    return (s & ST_FREE) || ((s & ST_YPOS) ? (s & ST_ATC) : !(s & ST_ATC));
}
DEV uint8_t st_make(bool ypos, double a, double C) {
    uint8_t s = ypos ? ST_YPOS : 0;
    if (a >= C) s |= ST_ATC;
    else if (a > 0.0) s |= ST_FREE;
    return s;
}
// eq:shrink: bound samples in I3 u I4 below b_up, or in I1 u I2 above b_low
DEV bool shrink_rule(uint8_t s, double fi, double bu, double bl) {
    if (s & ST_FREE) return false;
    return (st_in_low(s) && fi < bu) || (st_in_up(s) && fi > bl);
}

DEV bool better_up(double v, int i, double bv, int bi) { return v < bv || (v == bv && i < bi); }
DEV bool better_low(double v, int i, double bv, int bi) { return v > bv || (v == bv && i < bi); }

DEV void wave_reduce_sel(double& bu, int& iu, double& bl, int& il) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ou = __shfl_xor(bu, off);
        int oiu = __shfl_xor(iu, off);
        double ol = __shfl_xor(bl, off);
        int oil = __shfl_xor(il, off);
        if (better_up(ou, oiu, bu, iu)) { bu = ou; iu = oiu; }
        if (better_low(ol, oil, bl, il)) { bl = ol; il = oil; }
    }
}

template <typename T>
DEV T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

DEV float kexp(float v) { return expf(v); }
DEV double kexp(double v) { return exp(v); }

DEV double ld_agent(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV void st_agent(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV unsigned long long ld_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void st_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide reduction of the selection candidates; result valid in thread 0.
template <int BLOCK>
DEV void block_reduce_sel(double& bu, int& iu, double& bl, int& il, double* s_v, int* s_i) {
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_reduce_sel(bu, iu, bl, il);
    if (lane == 0) {
        s_v[wid] = bu; s_i[wid] = iu;
        s_v[NW + wid] = bl; s_i[NW + wid] = il;
    }
    __syncthreads();
    if (wid == 0) {
        bu = lane < NW ? s_v[lane] : INFINITY;
        iu = lane < NW ? s_i[lane] : IDX_NONE;
        bl = lane < NW ? s_v[NW + lane] : -INFINITY;
        il = lane < NW ? s_i[NW + lane] : IDX_NONE;
        wave_reduce_sel(bu, iu, bl, il);
    }
    __syncthreads();
}

// ------------------------------------------------------------------ pair update (eq:alphaup, eq:rho)

struct PairNew {
    double au, al;            // new alpha of the pair
    double cu, cl;            // y_up * d_alpha_up, y_low * d_alpha_low
};

DEV double snap_bound(double a, double C) {
    if (a < PAIR_DELTA * C) return 0.0;
    if (a > C - PAIR_DELTA * C) return C;
    return a;
}

// K(up,up) = K(low,low) = 1 for the Gaussian kernel, so eta = 2 - 2 K_ul (= -rho).
DEV PairNew pair_update(double au, double al, int yu, int yl, double bu, double bl, double Kul, double C) {
    double eta = 2.0 - 2.0 * Kul;
    if (eta < PAIR_TAU) eta = PAIR_TAU;
    const double s = (double)(yu * yl);
    double L, H;
    if (yu != yl) {
        L = fmax(0.0, al - au);
        H = fmin(C, C + al - au);
    } else {
        L = fmax(0.0, al + au - C);
        H = fmin(C, al + au);
    }
    double nl = al + (double)yl * (bu - bl) / eta;
    nl = fmin(fmax(nl, L), H);
    double nu = au + s * (al - nl);
    PairNew p;
    p.al = snap_bound(nl, C);
    p.au = snap_bound(nu, C);
    p.cu = (double)yu * (p.au - au);
    p.cl = (double)yl * (p.al - al);
    return p;
}

// ------------------------------------------------------------------ grid barrier

// Monotone counter barrier across the co-resident workgroups of a cooperative
// launch.  Release/acquire at agent scope publish the records and alpha writes.
DEV bool grid_barrier(unsigned long long* bar, unsigned long long target, int* abort_flag,
                      unsigned long long spin_limit, int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long t0 = wall_clock64();
        int ab = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ab = 1; break; }
            if (wall_clock64() - t0 > spin_limit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
        }
        *s_flag = ab;
    }
    __syncthreads();
    return *s_flag == 0;
}

// ------------------------------------------------------------------ kernel rows of the pair

// Dense: squared distances of row xr to the pair (u, l) held in LDS as float2,
// by direct difference in the order k = 0..dpad-1 (padding contributes 0).
template <typename KT>
DEV void dense_dist(const float* __restrict__ xr, const float2* __restrict__ pair, int dpad, KT& su, KT& sl) {
    const float4* x4 = reinterpret_cast<const float4*>(xr);
    const float4* p4 = reinterpret_cast<const float4*>(pair);
    if constexpr (std::is_same<KT, double>::value) {
#pragma clang fp contract(off)
        double a = 0.0, b = 0.0;
        for (int k4 = 0; k4 < dpad / 4; ++k4) {
            float4 v = x4[k4];
            float4 q0 = p4[2 * k4], q1 = p4[2 * k4 + 1];   // (u0 l0 u1 l1) (u2 l2 u3 l3)
            double t;
            t = (double)v.x - (double)q0.x; a = a + t * t;
            t = (double)v.x - (double)q0.y; b = b + t * t;
            t = (double)v.y - (double)q0.z; a = a + t * t;
            t = (double)v.y - (double)q0.w; b = b + t * t;
            t = (double)v.z - (double)q1.x; a = a + t * t;
            t = (double)v.z - (double)q1.y; b = b + t * t;
            t = (double)v.w - (double)q1.z; a = a + t * t;
            t = (double)v.w - (double)q1.w; b = b + t * t;
        }
        su = a; sl = b;
    } else {
        float a = 0.f, b = 0.f;
        for (int k4 = 0; k4 < dpad / 4; ++k4) {
            float4 v = x4[k4];
            float4 q0 = p4[2 * k4], q1 = p4[2 * k4 + 1];
            float t;
            t = v.x - q0.x; a = fmaf(t, t, a);
            t = v.x - q0.y; b = fmaf(t, t, b);
            t = v.y - q0.z; a = fmaf(t, t, a);
            t = v.y - q0.w; b = fmaf(t, t, b);
            t = v.z - q1.x; a = fmaf(t, t, a);
            t = v.z - q1.y; b = fmaf(t, t, b);
            t = v.w - q1.z; a = fmaf(t, t, a);
            t = v.w - q1.w; b = fmaf(t, t, b);
        }
        su = a; sl = b;
    }
}

// ------------------------------------------------------------------ the persistent SMO loop

template <int LAY, typename KT, int LPR>
__global__ __launch_bounds__(STEP_BLOCK) void smo_loop_kernel(StepArgs A) {
    constexpr int BLOCK = STEP_BLOCK;
    constexpr int NW = BLOCK / 64;
    constexpr int NG = BLOCK / LPR;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_v[2 * NW];
    __shared__ int s_i[2 * NW];
    __shared__ int s_wc[NW];
    __shared__ int s_flag;
    __shared__ double s_pair[4];     // K_ul, |u|^2, |l|^2
    __shared__ double s_sel[2];
    __shared__ int s_seli[3];
    __shared__ int s_prev_n;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int g = tid / LPR, gl = tid % LPR;
    const int blk = blockIdx.x, G = gridDim.x;
    const double C = A.C;

    // LDS carve-up: pair staging area, then the previous pair's columns (CSR)
    float2* pairv = reinterpret_cast<float2*>(smem);
    uint16_t* slot = nullptr;
    int* prev_cols = nullptr;
    if (LAY == LAY_DENSE) {
        // pairv[dpad]
    } else if (LAY == LAY_CSR_TABLE) {
        prev_cols = reinterpret_cast<int*>(smem + sizeof(float2) * (size_t)A.d);
        for (int k = tid; k < A.d; k += BLOCK) pairv[k] = make_float2(0.f, 0.f);
    } else {
        // vals[1 + 2*maxnnz] float2, slot[d] u16, prev_cols[2*maxnnz]
        const int nv = 1 + 2 * A.max_row_nnz;
        slot = reinterpret_cast<uint16_t*>(smem + sizeof(float2) * (size_t)nv);
        prev_cols = reinterpret_cast<int*>(smem + sizeof(float2) * (size_t)nv + ((sizeof(uint16_t) * (size_t)A.d + 15) & ~(size_t)15));
        for (int k = tid; k < A.d; k += BLOCK) slot[k] = 0;
        if (tid == 0) pairv[0] = make_float2(0.f, 0.f);
    }
    if (tid == 0) s_prev_n = 0;

    // solver state (identical in every workgroup)
    Ctl* ctl = A.ctl;
    double bu = ctl->b_up, bl = ctl->b_low;
    int iu = ctl->i_up, il = ctl->i_low;
    long long iter = ctl->iter, counter = ctl->counter, n_act_total = ctl->n_active;
    long long passes = ctl->shrink_passes, shrunk = ctl->shrunk_total;
    const int seg0 = A.seg_start[blk];
    int nrows = A.cnt[blk];
    int32_t* lst = A.act + seg0;
    int exit_reason = EXIT_NONE;
    unsigned long long bar_target = 0;
    unsigned long long work_rows = 0, work_nnz = 0;
    __syncthreads();

    for (;;) {
        if (!(bl - bu > A.thr)) { exit_reason = EXIT_CONVERGED; break; }
        if (iter >= A.max_iter) { exit_reason = EXIT_MAXITER; break; }
        if (blk == 0 && tid == 0 && iter < A.trace_cap) {
            A.tr_iu[iter] = iu; A.tr_il[iter] = il; A.tr_bu[iter] = bu; A.tr_bl[iter] = bl;
        }
        // ---- the working pair: alpha, labels, rows into LDS (the paper's broadcast of x_up, x_low)
        const double au = ld_agent(A.alpha + iu);
        const double al = ld_agent(A.alpha + il);
        const int yu = A.y[iu] > 0 ? 1 : -1;
        const int yl = A.y[il] > 0 ? 1 : -1;
        if (LAY == LAY_DENSE) {
            const float* xu = A.x + (size_t)iu * A.dpad;
            const float* xl = A.x + (size_t)il * A.dpad;
            for (int k = tid; k < A.dpad; k += BLOCK) pairv[k] = make_float2(xu[k], xl[k]);
            __syncthreads();
            if (tid == 0) {
                double s;
                if constexpr (std::is_same<KT, double>::value) {
#pragma clang fp contract(off)
                    double a = 0.0;
                    for (int k = 0; k < A.dpad; ++k) {
                        double t = (double)pairv[k].x - (double)pairv[k].y;
                        a = a + t * t;
                    }
                    s = a;
                } else {
                    float a = 0.f;
                    for (int k = 0; k < A.dpad; ++k) {
                        float t = pairv[k].x - pairv[k].y;
                        a = fmaf(t, t, a);
                    }
                    s = (double)a;
                }
                s_pair[0] = (double)kexp((KT)(-(KT)A.gamma * (KT)s));
            }
        } else {
            const int pu0 = A.row_ptr[iu], pu1 = A.row_ptr[iu + 1];
            const int pl0 = A.row_ptr[il], pl1 = A.row_ptr[il + 1];
            const int nu = pu1 - pu0, nl = pl1 - pl0;
            const int pn = s_prev_n;
            // clear the previous pair
            if (LAY == LAY_CSR_TABLE) {
                for (int j = tid; j < pn; j += BLOCK) pairv[prev_cols[j]] = make_float2(0.f, 0.f);
            } else {
                for (int j = tid; j < pn; j += BLOCK) slot[prev_cols[j]] = 0;
            }
            __syncthreads();
            float* pf = reinterpret_cast<float*>(pairv);
            if (LAY == LAY_CSR_TABLE) {
                for (int p = tid; p < nu; p += BLOCK) {
                    int c = A.col[pu0 + p];
                    pf[2 * c] = A.pattern_only ? 1.f : A.val[pu0 + p];
                    prev_cols[p] = c;
                }
                for (int p = tid; p < nl; p += BLOCK) {
                    int c = A.col[pl0 + p];
                    pf[2 * c + 1] = A.pattern_only ? 1.f : A.val[pl0 + p];
                    prev_cols[nu + p] = c;
                }
            } else {
                for (int p = tid; p < nu; p += BLOCK) {
                    int c = A.col[pu0 + p];
                    slot[c] = (uint16_t)(1 + p);
                    pairv[1 + p] = make_float2(A.pattern_only ? 1.f : A.val[pu0 + p], 0.f);
                    prev_cols[p] = c;
                }
                __syncthreads();
                for (int p = tid; p < nl; p += BLOCK) {
                    int c = A.col[pl0 + p];
                    float v = A.pattern_only ? 1.f : A.val[pl0 + p];
                    int sl = slot[c];
                    if (sl) {
                        pf[2 * sl + 1] = v;
                    } else {
                        slot[c] = (uint16_t)(1 + nu + p);
                        pairv[1 + nu + p] = make_float2(0.f, v);
                    }
                    prev_cols[nu + p] = c;
                }
            }
            __syncthreads();
            if (tid == 0) s_prev_n = nu + nl;
            if (wid == 0) {
                KT su = 0, sl2 = 0, dot = 0;
                for (int p = lane; p < nu; p += 64) {
                    KT v = A.pattern_only ? (KT)1 : (KT)A.val[pu0 + p];
                    su += v * v;
                }
                for (int p = lane; p < nl; p += 64) {
                    int c = A.col[pl0 + p];
                    KT v = A.pattern_only ? (KT)1 : (KT)A.val[pl0 + p];
                    float uv = (LAY == LAY_CSR_TABLE) ? pairv[c].x : pairv[slot[c]].x;
                    sl2 += v * v;
                    dot += v * (KT)uv;
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
        const KT gam = (KT)A.gamma;
        const KT nuu = (KT)s_pair[1], nll = (KT)s_pair[2];

        bool do_shrink = false;
        if (A.H > 0) {
            --counter;
            do_shrink = counter == 0;
        }

        // ---- f update over this workgroup's active rows, selection candidates, shrink rule
        double cbu = INFINITY, cbl = -INFINITY;
        int ciu = IDX_NONE, cil = IDX_NONE;
        int newcount = 0;
        work_rows += (unsigned long long)nrows;
        for (int base = 0; base < nrows; base += NG) {
            const int t = base + g;
            const bool valid = t < nrows;
            const int i = valid ? lst[t] : 0;
            bool keep = false;
            if (valid) {
                KT du2, dl2;
                if (LAY == LAY_DENSE) {
                    dense_dist<KT>(A.x + (size_t)i * A.dpad, pairv, A.dpad, du2, dl2);
                } else {
                    const int p0 = A.row_ptr[i], p1 = A.row_ptr[i + 1];
                    if (gl == 0) work_nnz += (unsigned long long)(p1 - p0);
                    KT nn = 0, su = 0, sl2 = 0;
                    for (int p = p0 + gl; p < p1; p += LPR) {
                        const int c = A.col[p];
                        const KT v = A.pattern_only ? (KT)1 : (KT)A.val[p];
                        const float2 ul = (LAY == LAY_CSR_TABLE) ? pairv[c] : pairv[slot[c]];
                        nn += v * v;
                        su += v * (KT)ul.x;
                        sl2 += v * (KT)ul.y;
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
                    double ku = (i == iu) ? 1.0 : (double)kexp(-gam * du2);
                    double kl = (i == il) ? 1.0 : (double)kexp(-gam * dl2);
                    double fi;
                    {
#pragma clang fp contract(off)
                        fi = A.f[i] + (pn.cu * ku + pn.cl * kl);
                    }
                    A.f[i] = fi;
                    uint8_t st = A.status[i];
                    if (i == iu) {
                        st = st_make(yu > 0, pn.au, C);
                        A.status[i] = st;
                        st_agent(A.alpha + i, pn.au);
                    } else if (i == il) {
                        st = st_make(yl > 0, pn.al, C);
                        A.status[i] = st;
                        st_agent(A.alpha + i, pn.al);
                    }
                    keep = !(do_shrink && shrink_rule(st, fi, bu, bl));
                    if (keep) {
                        if (st_in_up(st) && better_up(fi, i, cbu, ciu)) { cbu = fi; ciu = i; }
                        if (st_in_low(st) && better_low(fi, i, cbl, cil)) { cbl = fi; cil = i; }
                    }
                }
            }
            if (do_shrink) {   // stable in-place compaction of this chunk of the active list
                const unsigned long long m = __ballot(keep);
                const int wpre = __popcll(m & ((1ull << lane) - 1ull));
                if (lane == 0) s_wc[wid] = __popcll(m);
                __syncthreads();
                int off = 0, tot = 0;
                for (int w = 0; w < NW; ++w) {
                    int c = s_wc[w];
                    off += (w < wid) ? c : 0;
                    tot += c;
                }
                if (keep) lst[newcount + off + wpre] = i;
                newcount += tot;
                __syncthreads();
            }
        }
        if (do_shrink) nrows = newcount;

        block_reduce_sel<BLOCK>(cbu, ciu, cbl, cil, s_v, s_i);
        // ---- merge the workgroups' records (the paper's Allreduce of the b's)
        if (G > 1) {
            const int par = (int)(iter & 1);
            if (tid == 0) {
                Rec* r = A.rec + par * G + blk;
                st_agent(&r->w[0], (unsigned long long)__double_as_longlong(cbu));
                st_agent(&r->w[1], (unsigned long long)__double_as_longlong(cbl));
                st_agent(&r->w[2], (unsigned long long)(unsigned)ciu | ((unsigned long long)(unsigned)cil << 32));
                st_agent(&r->w[3], (unsigned long long)(unsigned)nrows);
            }
            bar_target += (unsigned long long)G;
            if (!grid_barrier(A.bar, bar_target, &ctl->abort, A.spin_limit, &s_flag)) {
                exit_reason = EXIT_ABORT;
                break;
            }
            double rbu = INFINITY, rbl = -INFINITY;
            int riu = IDX_NONE, ril = IDX_NONE;
            long long rcnt = 0;
            if (tid < G) {
                const Rec* r = A.rec + par * G + tid;
                rbu = __longlong_as_double((long long)ld_agent(&r->w[0]));
                rbl = __longlong_as_double((long long)ld_agent(&r->w[1]));
                unsigned long long w2 = ld_agent(&r->w[2]);
                riu = (int)(unsigned)(w2 & 0xffffffffull);
                ril = (int)(unsigned)(w2 >> 32);
                rcnt = (long long)ld_agent(&r->w[3]);
            }
            if (do_shrink) {
                long long c = wave_sum(rcnt);
                if (lane == 0) s_wc[wid] = (int)c;
            }
            block_reduce_sel<BLOCK>(rbu, riu, rbl, ril, s_v, s_i);
            if (tid == 0) {
                s_sel[0] = rbu; s_sel[1] = rbl; s_seli[0] = riu; s_seli[1] = ril;
                if (do_shrink) {
                    long long c = 0;
                    for (int w = 0; w < NW; ++w) c += s_wc[w];
                    s_seli[2] = (int)c;
                }
            }
        } else {
            if (tid == 0) {
                s_sel[0] = cbu; s_sel[1] = cbl; s_seli[0] = ciu; s_seli[1] = cil;
                s_seli[2] = nrows;
            }
        }
        __syncthreads();
        bu = s_sel[0];
        bl = s_sel[1];
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
        __syncthreads();
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
            A.work[2 * blk] = work_rows;
            A.work[2 * blk + 1] = t;
        }
    }
    if (blk == 0 && tid == 0) {
        ctl->b_up = bu; ctl->b_low = bl; ctl->i_up = iu; ctl->i_low = il;
        ctl->iter = iter; ctl->counter = counter; ctl->n_active = n_act_total;
        ctl->shrink_passes = passes; ctl->shrunk_total = shrunk;
        ctl->exit_reason = exit_reason;
    }
}

template <int LAY, typename KT, int LPR>
static hipError_t launch_loop_t(const StepArgs& a, int G, size_t lds, hipStream_t s) {
    auto fn = smo_loop_kernel<LAY, KT, LPR>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    StepArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel((const void*)fn, dim3(G), dim3(STEP_BLOCK), args, (unsigned)lds, s);
}

size_t step_lds_bytes(int lay, int d, int dpad, int max_row_nnz) {
    if (lay == LAY_DENSE) return sizeof(float2) * (size_t)dpad;
    if (lay == LAY_CSR_TABLE) return sizeof(float2) * (size_t)d + sizeof(int) * 2 * (size_t)max_row_nnz;
    size_t nv = 1 + 2 * (size_t)max_row_nnz;
    return sizeof(float2) * nv + ((sizeof(uint16_t) * (size_t)d + 15) & ~(size_t)15) + sizeof(int) * 2 * (size_t)max_row_nnz;
}

template <int LAY, typename KT>
static hipError_t dispatch_lpr(const StepArgs& a, int G, int lpr, size_t lds, hipStream_t s) {
    if constexpr (LAY == LAY_DENSE) return launch_loop_t<LAY, KT, 1>(a, G, lds, s);
    else switch (lpr) {
        case 1: return launch_loop_t<LAY, KT, 1>(a, G, lds, s);
        case 2: return launch_loop_t<LAY, KT, 2>(a, G, lds, s);
        case 4: return launch_loop_t<LAY, KT, 4>(a, G, lds, s);
        case 8: return launch_loop_t<LAY, KT, 8>(a, G, lds, s);
        case 16: return launch_loop_t<LAY, KT, 16>(a, G, lds, s);
        case 32: return launch_loop_t<LAY, KT, 32>(a, G, lds, s);
        default: return launch_loop_t<LAY, KT, 64>(a, G, lds, s);
    }
}

hipError_t launch_step(const StepArgs& a, int G, int lpr, int kprec, hipStream_t s) {
    size_t lds = step_lds_bytes(a.lay, a.d, a.dpad, a.max_row_nnz);
    if (kprec == SVM_KERNEL_FP64) {
        if (a.lay == LAY_DENSE) return dispatch_lpr<LAY_DENSE, double>(a, G, lpr, lds, s);
        if (a.lay == LAY_CSR_TABLE) return dispatch_lpr<LAY_CSR_TABLE, double>(a, G, lpr, lds, s);
        return dispatch_lpr<LAY_CSR_SLOT, double>(a, G, lpr, lds, s);
    }
    if (a.lay == LAY_DENSE) return dispatch_lpr<LAY_DENSE, float>(a, G, lpr, lds, s);
    if (a.lay == LAY_CSR_TABLE) return dispatch_lpr<LAY_CSR_TABLE, float>(a, G, lpr, lds, s);
    return dispatch_lpr<LAY_CSR_SLOT, float>(a, G, lpr, lds, s);
}

template <int LAY, typename KT, int LPR>
static int max_blocks_t(size_t lds) {
    int nb = 0;
    auto fn = smo_loop_kernel<LAY, KT, LPR>;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, STEP_BLOCK, lds) != hipSuccess) return 0;
    return nb;
}

template <int LAY, typename KT>
static int max_blocks_lpr(int lpr, size_t lds) {
    if constexpr (LAY == LAY_DENSE) return max_blocks_t<LAY, KT, 1>(lds);
    else switch (lpr) {
        case 1: return max_blocks_t<LAY, KT, 1>(lds);
        case 2: return max_blocks_t<LAY, KT, 2>(lds);
        case 4: return max_blocks_t<LAY, KT, 4>(lds);
        case 8: return max_blocks_t<LAY, KT, 8>(lds);
        case 16: return max_blocks_t<LAY, KT, 16>(lds);
        case 32: return max_blocks_t<LAY, KT, 32>(lds);
        default: return max_blocks_t<LAY, KT, 64>(lds);
    }
}

int step_max_blocks(int lay, int lpr, int kprec, size_t lds) {
    int per_cu;
    if (kprec == SVM_KERNEL_FP64) {
        per_cu = lay == LAY_DENSE ? max_blocks_lpr<LAY_DENSE, double>(lpr, lds)
               : lay == LAY_CSR_TABLE ? max_blocks_lpr<LAY_CSR_TABLE, double>(lpr, lds)
                                      : max_blocks_lpr<LAY_CSR_SLOT, double>(lpr, lds);
    } else {
        per_cu = lay == LAY_DENSE ? max_blocks_lpr<LAY_DENSE, float>(lpr, lds)
               : lay == LAY_CSR_TABLE ? max_blocks_lpr<LAY_CSR_TABLE, float>(lpr, lds)
                                      : max_blocks_lpr<LAY_CSR_SLOT, float>(lpr, lds);
    }
    return per_cu * device_cu_count();
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

// ------------------------------------------------------------------ set-up kernels

__global__ void validate_kernel(int n, int d, int lay, const float* __restrict__ x, int64_t ldx, int feature_major,
                                const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const float* __restrict__ val, const int8_t* __restrict__ y, Ctl* ctl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int err = 0;
    if (y) {
        int8_t v = y[i];
        if (v == 1) atomicAdd(&ctl->n_pos, 1);
        else if (v == -1) atomicAdd(&ctl->n_neg, 1);
        else err |= 1;
    }
    if (lay == SVM_CSR) {
        int p0 = rp[i], p1 = rp[i + 1];
        if (i == 0 && p0 != 0) err |= 1;
        if (p1 < p0) err |= 1;
        else {
            atomicMax(&ctl->max_row_nnz, p1 - p0);
            for (int p = p0; p < p1; ++p) {
                int c = col[p];
                if (c < 0 || c >= d) err |= 1;
                if (p > p0 && c <= col[p - 1]) err |= 1;
                if (!isfinite(val[p])) err |= 2;
            }
        }
    } else {
        for (int k = 0; k < d; ++k) {
            float v = feature_major ? x[(size_t)k * ldx + i] : x[(size_t)i * ldx + k];
            if (!isfinite(v)) err |= 2;
        }
    }
    if (err) atomicOr(&ctl->err, err);
}

hipError_t launch_validate(int n, int d, int lay, const float* x, int64_t ldx, int feature_major, const int32_t* rp,
                           const int32_t* col, const float* val, const int8_t* y, Ctl* ctl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    validate_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, d, lay, x, ldx, feature_major, rp, col, val, y, ctl);
    return hipGetLastError();
}

__global__ void pack_dense_kernel(int n, int d, int dpad, const float* __restrict__ x, int64_t ldx, int feature_major,
                                  float* __restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * dpad) return;
    const int i = (int)(e / dpad), k = (int)(e % dpad);
    float v = 0.f;
    if (k < d) v = feature_major ? x[(size_t)k * ldx + i] : x[(size_t)i * ldx + k];
    out[e] = v;
}

hipError_t launch_pack_dense(int n, int d, int dpad, const float* x, int64_t ldx, int feature_major, float* out,
                             hipStream_t s) {
    size_t tot = (size_t)n * dpad;
    if (!tot) return hipSuccess;
    pack_dense_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(n, d, dpad, x, ldx, feature_major, out);
    return hipGetLastError();
}

__global__ void init_state_kernel(int n, const int8_t* __restrict__ y, double C, int warm, double* alpha, double* f,
                                  uint8_t* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool yp = y[i] > 0;
    double a = 0.0;
    if (warm) a = alpha[i];
    else {
        alpha[i] = 0.0;
        f[i] = yp ? -1.0 : 1.0;
    }
    status[i] = st_make(yp, a, C);
}

hipError_t launch_init_state(int n, const int8_t* y, double C, int warm, double* alpha, double* f, uint8_t* status,
                             hipStream_t s) {
    init_state_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, y, C, warm, alpha, f, status);
    return hipGetLastError();
}

__global__ void refresh_status_kernel(int n, const double* __restrict__ alpha, const int8_t* __restrict__ y, double C,
                                      uint8_t* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) status[i] = st_make(y[i] > 0, alpha[i], C);
}

hipError_t launch_refresh_status(int n, const double* alpha, const int8_t* y, double C, uint8_t* status,
                                 hipStream_t s) {
    refresh_status_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, alpha, y, C, status);
    return hipGetLastError();
}

__global__ void reset_active_kernel(int n, int G, int32_t* seg_start, int32_t* cnt, int32_t* act) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) act[i] = i;
    if (i <= G) {
        const int s = (int)(((long long)n * i) / G);
        seg_start[i] = s;
        if (i < G) cnt[i] = (int)(((long long)n * (i + 1)) / G) - s;
    }
}

hipError_t launch_reset_active(int n, int G, int32_t* seg_start, int32_t* cnt, int32_t* act, hipStream_t s) {
    int m = n > G + 1 ? n : G + 1;
    reset_active_kernel<<<(m + 255) / 256, 256, 0, s>>>(n, G, seg_start, cnt, act);
    return hipGetLastError();
}

__global__ void mark_active_kernel(int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act,
                                   uint8_t* mask) {
    const int b = blockIdx.x;
    const int s0 = seg_start[b], c = cnt[b];
    for (int t = threadIdx.x; t < c; t += blockDim.x) mask[act[s0 + t]] = 1;
}

hipError_t launch_mark_active(int n, int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act,
                              uint8_t* mask, hipStream_t s) {
    hipError_t e = hipMemsetAsync(mask, 0, (size_t)n, s);
    if (e != hipSuccess) return e;
    mark_active_kernel<<<G, 256, 0, s>>>(G, seg_start, cnt, act, mask);
    return hipGetLastError();
}

// ------------------------------------------------------------------ selection (set-up and test hook)

// Each workgroup reduces one segment of the active lists to a record; a
// second one-workgroup kernel merges the records into ctl.  Membership comes
// from (alpha, y, C) directly.
__global__ __launch_bounds__(256) void select_partial_kernel(const int32_t* seg_start, const int32_t* cnt,
                                                             const int32_t* act, const double* __restrict__ f,
                                                             const double* __restrict__ alpha,
                                                             const int8_t* __restrict__ y, double C, Rec* rec) {
    __shared__ double s_v[8];
    __shared__ int s_i[8];
    const int b = blockIdx.x;
    const int s0 = seg_start[b], c = cnt[b];
    double bu = INFINITY, bl = -INFINITY;
    int iu = IDX_NONE, il = IDX_NONE;
    for (int t = threadIdx.x; t < c; t += blockDim.x) {
        const int i = act[s0 + t];
        const uint8_t st = st_make(y[i] > 0, alpha[i], C);
        const double fi = f[i];
        if (st_in_up(st) && better_up(fi, i, bu, iu)) { bu = fi; iu = i; }
        if (st_in_low(st) && better_low(fi, i, bl, il)) { bl = fi; il = i; }
    }
    block_reduce_sel<256>(bu, iu, bl, il, s_v, s_i);
    if (threadIdx.x == 0) {
        rec[b].w[0] = (unsigned long long)__double_as_longlong(bu);
        rec[b].w[1] = (unsigned long long)__double_as_longlong(bl);
        rec[b].w[2] = (unsigned long long)(unsigned)iu | ((unsigned long long)(unsigned)il << 32);
        rec[b].w[3] = (unsigned long long)(unsigned)c;
    }
}

__global__ __launch_bounds__(1024) void select_merge_kernel(int G, const Rec* rec, Ctl* ctl) {
    __shared__ double s_v[32];
    __shared__ int s_i[32];
    __shared__ long long s_c[16];
    double bu = INFINITY, bl = -INFINITY;
    int iu = IDX_NONE, il = IDX_NONE;
    long long c = 0;
    for (int t = threadIdx.x; t < G; t += blockDim.x) {
        double v = __longlong_as_double((long long)rec[t].w[0]);
        double w = __longlong_as_double((long long)rec[t].w[1]);
        int a = (int)(unsigned)(rec[t].w[2] & 0xffffffffull);
        int b2 = (int)(unsigned)(rec[t].w[2] >> 32);
        if (better_up(v, a, bu, iu)) { bu = v; iu = a; }
        if (better_low(w, b2, bl, il)) { bl = w; il = b2; }
        c += (long long)rec[t].w[3];
    }
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    block_reduce_sel<1024>(bu, iu, bl, il, s_v, s_i);
    if (threadIdx.x == 0) {
        long long tot = 0;
        for (int w = 0; w < 16; ++w) tot += s_c[w];
        ctl->b_up = bu; ctl->b_low = bl;
        ctl->i_up = iu == IDX_NONE ? -1 : iu;
        ctl->i_low = il == IDX_NONE ? -1 : il;
        ctl->n_active = tot;
    }
}

hipError_t launch_select(int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act, const double* f,
                         const double* alpha, const int8_t* y, double C, Rec* rec, Ctl* ctl, hipStream_t s) {
    select_partial_kernel<<<G, 256, 0, s>>>(seg_start, cnt, act, f, alpha, y, C, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    select_merge_kernel<<<1, 1024, 0, s>>>(G, rec, ctl);
    return hipGetLastError();
}

// ------------------------------------------------------------------ stable compaction (flags -> sorted id list)

template <int PRED>
DEV bool pred_at(int i, const uint8_t* mask, const double* alpha) {
    if (PRED == 0) return mask[i] == 0;
    if (PRED == 1) return alpha[i] > 0.0;
    return true;
}

constexpr int CMP_BLOCK = 1024;

template <int PRED>
__global__ __launch_bounds__(CMP_BLOCK) void compact_count_kernel(int n, const uint8_t* mask, const double* alpha,
                                                                  int32_t* blk_cnt) {
    __shared__ int s_c[CMP_BLOCK / 64];
    const int i = blockIdx.x * CMP_BLOCK + threadIdx.x;
    const bool p = i < n && pred_at<PRED>(i, mask, alpha);
    const unsigned long long m = __ballot(p);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < CMP_BLOCK / 64; ++w) t += s_c[w];
        blk_cnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void compact_scan_kernel(int nb, int32_t* blk_cnt, int32_t* count_out) {
    // exclusive scan of nb block counts by one workgroup, in chunks of 1024
    __shared__ int s_w[16];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int t = base + threadIdx.x;
        const int v = t < nb ? blk_cnt[t] : 0;
        // inclusive scan within the wave
        int x = v;
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int o = __shfl_up(x, off);
            if (lane >= off) x += o;
        }
        if (lane == 63) s_w[wid] = x;
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            woff += (w < wid) ? s_w[w] : 0;
            tot += s_w[w];
        }
        const int carry = s_carry;
        if (t < nb) blk_cnt[t] = carry + woff + x - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count_out = s_carry;
}

template <int PRED>
__global__ __launch_bounds__(CMP_BLOCK) void compact_write_kernel(int n, const uint8_t* mask, const double* alpha,
                                                                  const int8_t* y, const int32_t* blk_off,
                                                                  int32_t* list, double* coef) {
    __shared__ int s_c[CMP_BLOCK / 64];
    const int i = blockIdx.x * CMP_BLOCK + threadIdx.x;
    const bool p = i < n && pred_at<PRED>(i, mask, alpha);
    const unsigned long long m = __ballot(p);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_c[wid] = __popcll(m);
    __syncthreads();
    int off = blk_off[blockIdx.x];
    for (int w = 0; w < wid; ++w) off += s_c[w];
    off += __popcll(m & ((1ull << lane) - 1ull));
    if (p) {
        list[off] = i;
        if (coef) coef[off] = alpha[i] * (y[i] > 0 ? 1.0 : -1.0);
    }
}

hipError_t launch_compact(int n, int pred, const uint8_t* mask, const double* alpha, const int8_t* y,
                          int32_t* blk_cnt, int32_t* list, double* coef, int32_t* count_out, hipStream_t s) {
    const int nb = (n + CMP_BLOCK - 1) / CMP_BLOCK;
    if (nb == 0) return hipMemsetAsync(count_out, 0, sizeof(int32_t), s);
    if (pred == 0) compact_count_kernel<0><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, blk_cnt);
    else if (pred == 1) compact_count_kernel<1><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, blk_cnt);
    else compact_count_kernel<2><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, blk_cnt);
    compact_scan_kernel<<<1, 1024, 0, s>>>(nb, blk_cnt, count_out);
    if (pred == 0) compact_write_kernel<0><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, y, blk_cnt, list, coef);
    else if (pred == 1) compact_write_kernel<1><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, y, blk_cnt, list, coef);
    else compact_write_kernel<2><<<nb, CMP_BLOCK, 0, s>>>(n, mask, alpha, y, blk_cnt, list, coef);
    return hipGetLastError();
}

// ------------------------------------------------------------------ kernel sums (reconstruction, decision)

// Workgroup = 256 threads, holding R rows of A in LDS (dense: [R][dpad];
// CSR: densified [R][d]).  Threads stride over this split's part of the B
// list; each keeps R distances and R FP64 partial sums.  Partial sums per
// split go to part[split][a]; launch_finish_sum adds the splits in order.
constexpr int SUM_BLOCK = 256;
constexpr int SUM_RMAX = 16;

template <int LAY, typename KT>
__global__ __launch_bounds__(SUM_BLOCK) void kernel_sum_kernel(SumArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_red[SUM_BLOCK / 64][SUM_RMAX];
    __shared__ double s_na[SUM_RMAX];
    float* at = reinterpret_cast<float*>(smem);
    const int R = A.rows_per_block;
    const int r0 = blockIdx.x * R;
    const int nr = min(R, A.na - r0);
    const int W = (LAY == LAY_DENSE) ? A.dpad : A.d;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

    // stage the A rows
    for (int e = tid; e < R * W; e += SUM_BLOCK) at[e] = 0.f;
    __syncthreads();
    if (LAY == LAY_DENSE) {
        for (int e = tid; e < nr * W; e += SUM_BLOCK) {
            const int r = e / W, k = e % W;
            const int a = A.alist ? A.alist[r0 + r] : r0 + r;
            at[e] = A.ax[(size_t)a * A.dpad + k];
        }
    } else {
        for (int r = 0; r < nr; ++r) {
            const int a = A.alist ? A.alist[r0 + r] : r0 + r;
            const int p0 = A.arp[a], p1 = A.arp[a + 1];
            for (int p = p0 + tid; p < p1; p += SUM_BLOCK) at[r * W + A.acol[p]] = A.aval[p];
        }
    }
    __syncthreads();
    if (LAY != LAY_DENSE) {
        // |a|^2 of each staged row
        for (int r = wid; r < nr; r += SUM_BLOCK / 64) {
            KT s = 0;
            for (int k = lane; k < W; k += 64) {
                KT v = (KT)at[r * W + k];
                s += v * v;
            }
            s = wave_sum(s);
            if (lane == 0) s_na[r] = (double)s;
        }
        __syncthreads();
    }

    double acc[SUM_RMAX];
#pragma unroll
    for (int r = 0; r < SUM_RMAX; ++r) acc[r] = 0.0;
    const KT gam = (KT)A.gamma;
    const int nb = A.nb;
    const int per = (nb + A.nsplit - 1) / A.nsplit;
    const int b0 = blockIdx.y * per, b1 = min(nb, b0 + per);
    for (int jb = b0 + tid; jb < b1; jb += SUM_BLOCK) {
        const int j = A.blist[jb];
        const double cj = A.coef[jb];
        KT dist[SUM_RMAX];
#pragma unroll
        for (int r = 0; r < SUM_RMAX; ++r) dist[r] = 0;
        if (LAY == LAY_DENSE) {
            const float4* xb = reinterpret_cast<const float4*>(A.bx + (size_t)j * A.dpad);
            for (int k4 = 0; k4 < A.dpad / 4; ++k4) {
                const float4 v = xb[k4];
#pragma unroll
                for (int r = 0; r < SUM_RMAX; ++r) {
                    if (r < nr) {
                        const float4 q = reinterpret_cast<const float4*>(at + r * W)[k4];
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
            const int p0 = A.brp[j], p1 = A.brp[j + 1];
            KT nbn = 0;
            for (int p = p0; p < p1; ++p) {
                const int c = A.bcol[p];
                const KT v = (KT)A.bval[p];
                nbn += v * v;
#pragma unroll
                for (int r = 0; r < SUM_RMAX; ++r)
                    if (r < nr) dist[r] += v * (KT)at[r * W + c];
            }
#pragma unroll
            for (int r = 0; r < SUM_RMAX; ++r) {
                KT d2 = (KT)s_na[r < nr ? r : 0] + nbn - (KT)2 * dist[r];
                dist[r] = d2 < (KT)0 ? (KT)0 : d2;
            }
        }
#pragma unroll
        for (int r = 0; r < SUM_RMAX; ++r) {
            if (r < nr) {
                const double k = (double)kexp(-gam * dist[r]);
                acc[r] += cj * k;
            }
        }
    }
    // reduce acc[r] over the workgroup
#pragma unroll
    for (int r = 0; r < SUM_RMAX; ++r) {
        double v = wave_sum(acc[r]);
        if (lane == 0) s_red[wid][r] = v;
    }
    __syncthreads();
    if (tid < nr) {
        double v = 0.0;
        for (int w = 0; w < SUM_BLOCK / 64; ++w) v += s_red[w][tid];
        A.part[(size_t)blockIdx.y * A.na + r0 + tid] = v;
    }
}

// Large-d CSR: one A row at a time per workgroup, densified through a u16 slot
// map over the d columns (zeroed once, cleared sparsely after each row).
template <typename KT>
__global__ __launch_bounds__(SUM_BLOCK) void kernel_sum_slot_kernel(SumArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_red[SUM_BLOCK / 64];
    __shared__ double s_na;
    float* av = reinterpret_cast<float*>(smem);                       // [1 + max_row_nnz]
    uint16_t* slot = reinterpret_cast<uint16_t*>(smem + ((sizeof(float) * (size_t)(1 + A.rows_per_block) + 15) & ~(size_t)15));
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int k = tid; k < A.d; k += SUM_BLOCK) slot[k] = 0;
    if (tid == 0) av[0] = 0.f;
    __syncthreads();
    const KT gam = (KT)A.gamma;
    const int per = (A.nb + A.nsplit - 1) / A.nsplit;
    const int b0 = blockIdx.y * per, b1 = min(A.nb, b0 + per);
    for (int r = blockIdx.x; r < A.na; r += gridDim.x) {
        const int a = A.alist ? A.alist[r] : r;
        const int p0 = A.arp[a], p1 = A.arp[a + 1];
        KT nn = 0;
        for (int p = p0 + tid; p < p1; p += SUM_BLOCK) {
            slot[A.acol[p]] = (uint16_t)(1 + p - p0);
            const float v = A.aval[p];
            av[1 + p - p0] = v;
            nn += (KT)v * (KT)v;
        }
        nn = wave_sum(nn);
        if (lane == 0) s_red[wid] = (double)nn;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < SUM_BLOCK / 64; ++w) t += s_red[w];
            s_na = t;
        }
        __syncthreads();
        const KT na = (KT)s_na;
        double acc = 0.0;
        for (int jb = b0 + tid; jb < b1; jb += SUM_BLOCK) {
            const int j = A.blist[jb];
            const int q0 = A.brp[j], q1 = A.brp[j + 1];
            KT nb = 0, dot = 0;
            for (int q = q0; q < q1; ++q) {
                const KT v = (KT)A.bval[q];
                nb += v * v;
                dot += v * (KT)av[slot[A.bcol[q]]];
            }
            KT d2 = na + nb - (KT)2 * dot;
            if (d2 < (KT)0) d2 = (KT)0;
            acc += A.coef[jb] * (double)kexp(-gam * d2);
        }
        acc = wave_sum(acc);
        __syncthreads();
        if (lane == 0) s_red[wid] = acc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < SUM_BLOCK / 64; ++w) t += s_red[w];
            A.part[(size_t)blockIdx.y * A.na + r] = t;
        }
        for (int p = p0 + tid; p < p1; p += SUM_BLOCK) slot[A.acol[p]] = 0;
        __syncthreads();
    }
}

hipError_t launch_kernel_sum(const SumArgs& a, int kprec, hipStream_t s) {
    if (a.na <= 0) return hipSuccess;
    if (a.lay == LAY_CSR_SLOT) {
        // rows_per_block carries the longest A row here
        const size_t lds = ((sizeof(float) * (size_t)(1 + a.rows_per_block) + 15) & ~(size_t)15) +
                           sizeof(uint16_t) * (size_t)a.d;
        dim3 grid(std::min(a.na, 2048), a.nsplit);
        SumArgs c = a;
        if (kprec == SVM_KERNEL_FP64) {
            (void)hipFuncSetAttribute((const void*)kernel_sum_slot_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_slot_kernel<double><<<grid, SUM_BLOCK, lds, s>>>(c);
        } else {
            (void)hipFuncSetAttribute((const void*)kernel_sum_slot_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_slot_kernel<float><<<grid, SUM_BLOCK, lds, s>>>(c);
        }
        return hipGetLastError();
    }
    const int W = a.lay == LAY_DENSE ? a.dpad : a.d;
    const size_t lds = sizeof(float) * (size_t)a.rows_per_block * W;
    dim3 grid((a.na + a.rows_per_block - 1) / a.rows_per_block, a.nsplit);
    SumArgs c = a;
    if (kprec == SVM_KERNEL_FP64) {
        if (a.lay == LAY_DENSE) {
            if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel_sum_kernel<LAY_DENSE, double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_kernel<LAY_DENSE, double><<<grid, SUM_BLOCK, lds, s>>>(c);
        } else {
            if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel_sum_kernel<LAY_CSR_TABLE, double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_kernel<LAY_CSR_TABLE, double><<<grid, SUM_BLOCK, lds, s>>>(c);
        }
    } else {
        if (a.lay == LAY_DENSE) {
            if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel_sum_kernel<LAY_DENSE, float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_kernel<LAY_DENSE, float><<<grid, SUM_BLOCK, lds, s>>>(c);
        } else {
            if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kernel_sum_kernel<LAY_CSR_TABLE, float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_kernel<LAY_CSR_TABLE, float><<<grid, SUM_BLOCK, lds, s>>>(c);
        }
    }
    return hipGetLastError();
}

__global__ void finish_sum_kernel(int na, int nsplit, const double* __restrict__ part, const int32_t* __restrict__ alist,
                                  const int8_t* __restrict__ y, double beta, double* out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    double v = 0.0;
    for (int s = 0; s < nsplit; ++s) v += part[(size_t)s * na + r];
    const int a = alist ? alist[r] : r;
    out[a] = v - (y ? (y[a] > 0 ? 1.0 : -1.0) : beta);
}

hipError_t launch_finish_sum(int na, int nsplit, const double* part, const int32_t* alist, const int8_t* y, double beta,
                             double* out, hipStream_t s) {
    if (na <= 0) return hipSuccess;
    finish_sum_kernel<<<(na + 255) / 256, 256, 0, s>>>(na, nsplit, part, alist, y, beta, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ closing reductions

__global__ __launch_bounds__(256) void summary_partial_kernel(int n, const double* __restrict__ alpha,
                                                              const double* __restrict__ f,
                                                              const int8_t* __restrict__ y, double C, double* blk) {
    __shared__ double s[6][4];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double a = alpha[i];
        const double yi = y[i] > 0 ? 1.0 : -1.0;
        if (a > 0.0 && a < C) { v[0] += f[i]; v[1] += 1.0; }
        v[2] += a;
        v[3] += a * yi * (f[i] + yi);
        if (a > 0.0) v[4] += 1.0;
        if (a >= C) v[5] += 1.0;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double t = wave_sum(v[k]);
        if (lane == 0) s[k][wid] = t;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double t = 0.0;
        for (int w = 0; w < 4; ++w) t += s[threadIdx.x][w];
        blk[blockIdx.x * 6 + threadIdx.x] = t;
    }
}

__global__ void summary_final_kernel(int nb, const double* blk, double* out6) {
    if (threadIdx.x < 6) {
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += blk[b * 6 + threadIdx.x];
        out6[threadIdx.x] = t;
    }
}

hipError_t launch_summary(int n, const double* alpha, const double* f, const int8_t* y, double C, double* blk,
                          double* out6, hipStream_t s) {
    const int nb = 256;
    summary_partial_kernel<<<nb, 256, 0, s>>>(n, alpha, f, y, C, blk);
    summary_final_kernel<<<1, 64, 0, s>>>(nb, blk, out6);
    return hipGetLastError();
}

__global__ void check_pattern_kernel(int nnz, const float* __restrict__ val, int32_t* flag) {
    int bad = 0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += gridDim.x * blockDim.x)
        if (val[p] != 1.0f) bad = 1;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_check_pattern(int nnz, const float* val, int32_t* flag, hipStream_t s) {
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), s);
    if (e != hipSuccess || nnz <= 0) return e;
    check_pattern_kernel<<<512, 256, 0, s>>>(nnz, val, flag);
    return hipGetLastError();
}

}  // namespace svm

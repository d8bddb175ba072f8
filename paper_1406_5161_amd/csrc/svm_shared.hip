// svm_shared.hip -- several training problems over one sample set in lockstep (one-vs-rest
// labelings of a dataset, a C / gamma grid): one persistent cooperative launch advances every
// live problem by one SMO iteration (Alg. 2) per pass over the rows, and each row is read once
// per pass for all of them.  Every problem's arithmetic is the single-problem loop's (the same
// pair staging and K(up, low), the same distance, kernel value and eq:fup update, the exact
// two-threshold selection of eq:bminmax), so each problem follows its own run's trajectory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "svm_device.h"
#include "svm_internal.h"

namespace svm {

// bytes of the pair rows of SHARED_MAX problems at the start of the dynamic LDS (16-aligned)
__host__ __device__ inline size_t shared_pair_bytes(int lay, int wpr, int dpad) {
    const size_t per = lay == LAY_BITS ? sizeof(uint32_t) * 2 * (size_t)wpr : sizeof(float2) * (size_t)dpad;
    return (per * SHARED_MAX + 15) & ~(size_t)15;
}

template <int LAY, typename KT, bool RES>
__global__ __launch_bounds__(SHARED_BLOCK) void smo_shared_kernel(SharedArgs A) {
    constexpr int BLOCK = SHARED_BLOCK;
    constexpr int KM = SHARED_MAX;
    constexpr bool BITS = LAY == LAY_BITS;
    extern __shared__ __align__(16) unsigned char smem[];   // the pair rows of every problem
    __shared__ double s_v[KM][SEL_LDS(BLOCK)];
    __shared__ int s_i[KM][SEL_LDS(BLOCK)];
    __shared__ double s_kul[KM], s_cu[KM], s_cl[KM], s_nau[KM], s_nal[KM];
    __shared__ double s_bu[KM], s_bl[KM], s_au[KM], s_al[KM];
    __shared__ int s_iu[KM], s_il[KM], s_yu[KM], s_yl[KM], s_nuu[KM], s_nll[KM];
    __shared__ int s_live[KM], s_exit[KM];
    __shared__ long long s_iter[KM];
    __shared__ int s_abort;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int blk = blockIdx.x, G = gridDim.x, k = A.k;
    const int seg0 = (int)((long long)A.n * blk / G), seg1 = (int)((long long)A.n * (blk + 1) / G);
    uint32_t* pairb = reinterpret_cast<uint32_t*>(smem);   // LAY_BITS: problem p at 2 wpr p
    float2* pairv = reinterpret_cast<float2*>(smem);       // dense: problem p at dpad p
    if (tid < KM) {
        const int p = tid;
        int live = 0;
        if (p < k && ((A.live_mask >> p) & 1)) {
            const Ctl* c = A.prob[p].ctl;
            s_bu[p] = c->b_up; s_bl[p] = c->b_low;
            s_au[p] = c->a_up; s_al[p] = c->a_low;
            s_iu[p] = c->i_up; s_il[p] = c->i_low;
            s_iter[p] = c->iter;
            live = 1;
        }
        s_live[p] = live;
        s_exit[p] = EXIT_NONE;
    }
    // RES: this segment's rows, and f and status of every problem, live in LDS for the launch
    const int segn = seg1 - seg0, smax = A.seg_max;
    const uint32_t* XB = nullptr;
    const float* XL = nullptr;
    double* FL = nullptr;
    uint8_t* SL = nullptr;
    if constexpr (RES) {
        const size_t pair = shared_pair_bytes(LAY, A.wpr, A.dpad);
        const size_t rows = BITS ? sizeof(uint32_t) * (size_t)smax * A.wpr : sizeof(float) * (size_t)smax * A.dpad;
        unsigned char* base = smem + pair;
        FL = reinterpret_cast<double*>(base + ((rows + 15) & ~(size_t)15));
        SL = reinterpret_cast<uint8_t*>(FL + (size_t)KM * smax);
        if constexpr (BITS) {
            uint4* dst = reinterpret_cast<uint4*>(base);
            const uint4* src = reinterpret_cast<const uint4*>(A.bits + (size_t)seg0 * A.wpr);
            for (int e = tid; e < segn * (A.wpr / 4); e += BLOCK) dst[e] = src[e];
            XB = reinterpret_cast<const uint32_t*>(base);
        } else {
            float4* dst = reinterpret_cast<float4*>(base);
            const float4* src = reinterpret_cast<const float4*>(A.x + (size_t)seg0 * A.dpad);
            for (int e = tid; e < segn * (A.dpad / 4); e += BLOCK) dst[e] = src[e];
            XL = reinterpret_cast<const float*>(base);
        }
        for (int p = 0; p < k; ++p) {
            if (!((A.live_mask >> p) & 1)) continue;
            for (int li = tid; li < segn; li += BLOCK) {
                FL[(size_t)p * smax + li] = A.prob[p].f[seg0 + li];
                SL[(size_t)p * smax + li] = A.prob[p].status[seg0 + li];
            }
        }
    }
    if (tid == 0) s_abort = 0;
    unsigned long long work_rows = 0;
    long long lit = 0;   // iterations of this launch: the records' tags and parity
    __syncthreads();

    for (;;) {
        // ---- stop tests, identical in every workgroup (eq:kktterm, the iteration cap)
        if (tid < KM && s_live[tid]) {
            const int p = tid;
            if (!(s_bl[p] - s_bu[p] > A.prob[p].thr)) { s_live[p] = 0; s_exit[p] = EXIT_CONVERGED; }
            else if (s_iter[p] >= A.prob[p].max_iter) { s_live[p] = 0; s_exit[p] = EXIT_MAXITER; }
        }
        __syncthreads();
        int any = 0;
#pragma unroll
        for (int p = 0; p < KM; ++p) any |= s_live[p];
        if (!any) break;

        // ---- 1. every live problem's pair: wave p stages its two rows and forms K(up, low)
        if (wid < k && s_live[wid]) {
            const int p = wid;
            const int iu = s_iu[p], il = s_il[p];
            if constexpr (BITS) {
                const int wpr = A.wpr;
                uint32_t* pb = pairb + (size_t)2 * wpr * p;
                uint32_t wu = 0, wl = 0;
                if (lane < wpr) {
                    wu = A.bits[(size_t)iu * wpr + lane];
                    wl = A.bits[(size_t)il * wpr + lane];
                    pb[lane] = wu;
                    pb[wpr + lane] = wl;
                }
                int c2 = __popc(wu) | (__popc(wl) << 16), cd = __popc(wu & wl);
                sum2_lanes32(c2, cd);
                const int cu = c2 & 0xffff, cl = c2 >> 16;
                if (lane == 0) {
                    KT d2 = (KT)cu + (KT)cl - (KT)2 * (KT)cd;
                    if (d2 < (KT)0) d2 = (KT)0;
                    s_kul[p] = (double)kexp((KT)(-(KT)A.prob[p].gamma * d2));
                    s_nuu[p] = cu;
                    s_nll[p] = cl;
                }
            } else {
                float2* pv = pairv + (size_t)A.dpad * p;
                const float* xu = A.x + (size_t)iu * A.dpad;
                const float* xl = A.x + (size_t)il * A.dpad;
                if constexpr (std::is_same<KT, float>::value) {
                    float a = 0.f;
                    for (int j = lane; j < A.dpad; j += 64) {
                        const float u = xu[j], l = xl[j];
                        pv[j] = make_float2(u, l);
                        const float t = u - l;
                        a = fmaf(t, t, a);
                    }
                    a = wave_sum_dpp(a);
                    if (lane == 0) s_kul[p] = (double)kexp(-(float)A.prob[p].gamma * a);
                } else {
                    for (int j = lane; j < A.dpad; j += 64) pv[j] = make_float2(xu[j], xl[j]);
                    if (lane == 0) {
                        // sequential in the feature index: the rounding of the FP64 reference
#pragma clang fp contract(off)
                        double a = 0.0;
                        for (int j = 0; j < A.dpad; ++j) {
                            const double t = (double)xu[j] - (double)xl[j];
                            a = a + t * t;
                        }
                        s_kul[p] = exp(-A.prob[p].gamma * a);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < KM && s_live[tid]) {
            const int p = tid;
            const int yu = A.prob[p].y[s_iu[p]] > 0 ? 1 : -1, yl = A.prob[p].y[s_il[p]] > 0 ? 1 : -1;
            const PairNew pn = pair_update(s_au[p], s_al[p], yu, yl, s_bu[p], s_bl[p], s_kul[p], A.prob[p].C);
            s_cu[p] = pn.cu; s_cl[p] = pn.cl;
            s_nau[p] = pn.au; s_nal[p] = pn.al;
            s_yu[p] = yu; s_yl[p] = yl;
        }
        __syncthreads();

        // ---- 2. one pass over this segment's rows: each row serves every live problem
        double cbu[KM], cbl[KM];
        int ciu[KM], cil[KM];
#pragma unroll
        for (int p = 0; p < KM; ++p) { cbu[p] = INFINITY; cbl[p] = -INFINITY; ciu[p] = IDX_NONE; cil[p] = IDX_NONE; }
        for (int i = seg0 + tid; i < seg1; i += BLOCK) {
            ++work_rows;
            // a bitset row is loaded once into registers and serves every live problem
            constexpr int XW = BITS ? BITS_MAX_D / 128 : 1;   // uint4 words of the widest bitset row
            uint4 xv[XW];
            int nn = 0;
            if constexpr (BITS) {
                const uint4* xr = reinterpret_cast<const uint4*>(RES ? XB + (size_t)(i - seg0) * A.wpr
                                                                     : A.bits + (size_t)i * A.wpr);
#pragma unroll
                for (int w4 = 0; w4 < XW; ++w4) {
                    if (w4 >= A.wpr / 4) break;
                    xv[w4] = xr[w4];
                    nn += __popc(xv[w4].x) + __popc(xv[w4].y) + __popc(xv[w4].z) + __popc(xv[w4].w);
                }
            }
#pragma unroll
            for (int p = 0; p < KM; ++p) {
                if (p >= k || !s_live[p]) continue;
                KT du2, dl2;
                if constexpr (BITS) {
                    const int wpr = A.wpr;
                    const uint4* pu = reinterpret_cast<const uint4*>(pairb + (size_t)2 * wpr * p);
                    const uint4* pl = reinterpret_cast<const uint4*>(pairb + (size_t)2 * wpr * p + wpr);
                    int su = 0, sl2 = 0;
#pragma unroll
                    for (int w4 = 0; w4 < XW; ++w4) {
                        if (w4 >= wpr / 4) break;
                        const uint4 v = xv[w4], a = pu[w4], b = pl[w4];
                        su += __popc(v.x & a.x) + __popc(v.y & a.y) + __popc(v.z & a.z) + __popc(v.w & a.w);
                        sl2 += __popc(v.x & b.x) + __popc(v.y & b.y) + __popc(v.z & b.z) + __popc(v.w & b.w);
                    }
                    du2 = (KT)nn + (KT)s_nuu[p] - (KT)2 * (KT)su;
                    dl2 = (KT)nn + (KT)s_nll[p] - (KT)2 * (KT)sl2;
                    if (du2 < (KT)0) du2 = (KT)0;
                    if (dl2 < (KT)0) dl2 = (KT)0;
                } else {
                    dense_dist<KT>(RES ? XL + (size_t)(i - seg0) * A.dpad : A.x + (size_t)i * A.dpad,
                                   pairv + (size_t)A.dpad * p, A.dpad, du2, dl2);
                }
                const SharedProb& P = A.prob[p];
                const int iu = s_iu[p], il = s_il[p];
                const KT gam = (KT)P.gamma;
                const double ku = (i == iu) ? 1.0 : (double)kexp(-gam * du2);
                const double kl = (i == il) ? 1.0 : (double)kexp(-gam * dl2);
                double* fp = RES ? FL + (size_t)p * smax + (i - seg0) : P.f + i;
                uint8_t* sp = RES ? SL + (size_t)p * smax + (i - seg0) : P.status + i;
                double fi;
                {
#pragma clang fp contract(off)
                    fi = *fp + (s_cu[p] * ku + s_cl[p] * kl);
                }
                *fp = fi;
                uint8_t st = *sp;
                if (i == iu) {
                    st = st_make(s_yu[p] > 0, s_nau[p], P.C);
                    *sp = st;
                    st_agent(P.alpha + i, s_nau[p]);
                } else if (i == il) {
                    st = st_make(s_yl[p] > 0, s_nal[p], P.C);
                    *sp = st;
                    st_agent(P.alpha + i, s_nal[p]);
                }
                if (st_in_up(st) && better_up(fi, i, cbu[p], ciu[p])) { cbu[p] = fi; ciu[p] = i; }
                if (st_in_low(st) && better_low(fi, i, cbl[p], cil[p])) { cbl[p] = fi; cil[p] = i; }
            }
        }
        // ---- 3. per problem: wave results into LDS, then wave p holds the workgroup's winners
#pragma unroll
        for (int p = 0; p < KM; ++p)
            if (p < k && s_live[p]) waves_to_lds<BLOCK>(cbu[p], ciu[p], cbl[p], cil[p], s_v[p], s_i[p]);
        __syncthreads();
        const int pw = wid;   // the problem this wave reduces and exchanges
        const bool pw_live = pw < k && s_live[pw];
        double bu = INFINITY, bl = -INFINITY, au = 0.0, al = 0.0;
        int iu = IDX_NONE, il = IDX_NONE;
        if (pw_live) {
            wave_reduce_waves<BLOCK>(bu, iu, bl, il, s_v[pw], s_i[pw]);
            // alpha of the candidates: this workgroup's own rows
            if (iu != IDX_NONE) au = ld_agent(A.prob[pw].alpha + iu);
            if (il != IDX_NONE) al = ld_agent(A.prob[pw].alpha + il);
        }
        // ---- 4. exchange: one tag-validated record per workgroup and problem, merged by wave p
        if (G > 1) {
            const int par = (int)(lit & 1);
            const unsigned tg = (unsigned)(lit + 1);
            const unsigned long long TAG = (unsigned long long)tg << 32;
            Rec* rec = A.rec + ((size_t)par * KM + pw) * G;
            if (pw_live && lane < 10) {
                const unsigned long long bub = (unsigned long long)__double_as_longlong(bu);
                const unsigned long long blb = (unsigned long long)__double_as_longlong(bl);
                const unsigned long long aub = (unsigned long long)__double_as_longlong(au);
                const unsigned long long alb = (unsigned long long)__double_as_longlong(al);
                unsigned long long x;
                switch (lane) {
                    case 0: x = bub; break;
                    case 1: x = bub >> 32; break;
                    case 2: x = blb; break;
                    case 3: x = blb >> 32; break;
                    case 4: x = (unsigned)iu; break;
                    case 5: x = (unsigned)il; break;
                    case 6: x = aub; break;
                    case 7: x = aub >> 32; break;
                    case 8: x = alb; break;
                    default: x = alb >> 32; break;
                }
                st_agent(rec[blk].w + lane, TAG | (x & 0xffffffffull));
            }
            int ab = 0;
            double rbu = INFINITY, rbl = -INFINITY, rau = 0.0, ral = 0.0;
            int riu = IDX_NONE, ril = IDX_NONE;
            if (pw_live && lane < G) {
                const unsigned long long* w = rec[lane].w;
                unsigned v[10];
                const unsigned long long t0 = wall_clock64();
                for (;;) {
                    bool ok = true;
#pragma unroll
                    for (int j = 0; j < 10; ++j) {
                        const unsigned long long x = ld_agent(w + j);
                        v[j] = (unsigned)(x & 0xffffffffull);
                        ok = ok && (unsigned)(x >> 32) == tg;
                    }
                    if (ok) break;
                    if (wall_clock64() - t0 > A.spin_limit) { ab = 1; break; }
                    __builtin_amdgcn_s_sleep(1);
                }
                rbu = __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
                rbl = __longlong_as_double((long long)(((unsigned long long)v[3] << 32) | v[2]));
                riu = (int)v[4];
                ril = (int)v[5];
                rau = __longlong_as_double((long long)(((unsigned long long)v[7] << 32) | v[6]));
                ral = __longlong_as_double((long long)(((unsigned long long)v[9] << 32) | v[8]));
            }
            if (ab) s_abort = 1;
            if (pw_live) {
                const int myiu = riu, myil = ril;
                wave_reduce_sel(rbu, riu, rbl, ril);
                // the record holding each winner carries its alpha
                if (lane < G && myiu != IDX_NONE && myiu == riu) s_au[pw] = rau;
                if (lane < G && myil != IDX_NONE && myil == ril) s_al[pw] = ral;
                if (lane == 0) {
                    s_bu[pw] = rbu; s_bl[pw] = rbl;
                    s_iu[pw] = riu == IDX_NONE ? -1 : riu;
                    s_il[pw] = ril == IDX_NONE ? -1 : ril;
                }
            }
        } else if (pw_live && lane == 0) {
            s_bu[pw] = bu; s_bl[pw] = bl; s_au[pw] = au; s_al[pw] = al;
            s_iu[pw] = iu == IDX_NONE ? -1 : iu;
            s_il[pw] = il == IDX_NONE ? -1 : il;
        }
        __syncthreads();
        if (s_abort) {
            if (tid < KM && s_live[tid]) { s_exit[tid] = EXIT_ABORT; s_live[tid] = 0; }
            break;
        }
        if (tid < KM && s_live[tid]) ++s_iter[tid];
        ++lit;
        __syncthreads();
    }
    __syncthreads();
    if constexpr (RES) {
        // the segment's f and status back for the host phases (recompute, summary)
        for (int p = 0; p < k; ++p) {
            if (!((A.live_mask >> p) & 1)) continue;
            for (int li = tid; li < segn; li += BLOCK) {
                A.prob[p].f[seg0 + li] = FL[(size_t)p * smax + li];
                A.prob[p].status[seg0 + li] = SL[(size_t)p * smax + li];
            }
        }
    }
    if (A.work && tid == 0) A.work[blk] = 0;
    __syncthreads();
    if (A.work) atomicAdd(A.work + blk, work_rows);
    if (blk == 0 && tid < k && ((A.live_mask >> tid) & 1)) {
        Ctl* c = A.prob[tid].ctl;
        c->b_up = s_bu[tid]; c->b_low = s_bl[tid];
        c->a_up = s_au[tid]; c->a_low = s_al[tid];
        c->i_up = s_iu[tid]; c->i_low = s_il[tid];
        c->iter = s_iter[tid];
        c->exit_reason = s_exit[tid];
        if (s_exit[tid] == EXIT_ABORT) c->abort = 1;
    }
}

size_t shared_lds_bytes(int lay, int d, int seg_max, bool res) {
    const int wpr = lay == LAY_BITS ? bits_wpr(d) : 0, dpad = (d + 3) & ~3;
    size_t b = shared_pair_bytes(lay, wpr, dpad);
    if (res) {
        const size_t rows = lay == LAY_BITS ? sizeof(uint32_t) * (size_t)seg_max * wpr
                                            : sizeof(float) * (size_t)seg_max * dpad;
        b += ((rows + 15) & ~(size_t)15) + (sizeof(double) + 1) * (size_t)SHARED_MAX * seg_max;
    }
    return b;
}

static const void* shared_fn(int lay, int kprec, bool res) {
    if (lay == LAY_BITS) {
        if (res)
            return kprec == SVM_KERNEL_FP64 ? (const void*)smo_shared_kernel<LAY_BITS, double, true>
                                            : (const void*)smo_shared_kernel<LAY_BITS, float, true>;
        return kprec == SVM_KERNEL_FP64 ? (const void*)smo_shared_kernel<LAY_BITS, double, false>
                                        : (const void*)smo_shared_kernel<LAY_BITS, float, false>;
    }
    if (res)
        return kprec == SVM_KERNEL_FP64 ? (const void*)smo_shared_kernel<LAY_DENSE, double, true>
                                        : (const void*)smo_shared_kernel<LAY_DENSE, float, true>;
    return kprec == SVM_KERNEL_FP64 ? (const void*)smo_shared_kernel<LAY_DENSE, double, false>
                                    : (const void*)smo_shared_kernel<LAY_DENSE, float, false>;
}

int shared_max_blocks(int lay, int kprec, bool res, size_t lds) {
    const void* fn = shared_fn(lay, kprec, res);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, SHARED_BLOCK, lds) != hipSuccess) return 0;
    return nb * device_cu_count();
}

hipError_t launch_shared(const SharedArgs& a, int G, int kprec, hipStream_t s) {
    const void* fn = shared_fn(a.lay, kprec, a.res != 0);
    const size_t lds = shared_lds_bytes(a.lay, a.d, a.seg_max, a.res != 0);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    SharedArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(SHARED_BLOCK), args, (unsigned)lds, s);
}

}  // namespace svm

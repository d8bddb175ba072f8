// svm_kernels.hip -- set-up and support kernels of libsvmhip.so for gfx950:
// input validation, dense packing, state initialisation, the initial and
// post-reconstruction selection, stable compaction of id lists, the kernel
// sums behind gradient reconstruction (Alg. 6) and the classifier
// (eq:classi), and the closing reductions (threshold, dual objective).
// The persistent SMO loop itself is in svm_step.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "svm_device.h"
#include "svm_internal.h"

namespace svm {

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

__global__ void iota_kernel(int n, int32_t* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = i;
}

hipError_t launch_iota(int n, int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    iota_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, out);
    return hipGetLastError();
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
    __shared__ double s_v[SEL_LDS(256)];
    __shared__ int s_i[SEL_LDS(256)];
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

__global__ __launch_bounds__(1024) void select_merge_kernel(int G, const Rec* rec, const double* alpha, Ctl* ctl) {
    __shared__ double s_v[SEL_LDS(1024)];
    __shared__ int s_i[SEL_LDS(1024)];
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
        ctl->a_up = iu == IDX_NONE ? 0.0 : alpha[iu];
        ctl->a_low = il == IDX_NONE ? 0.0 : alpha[il];
        ctl->n_active = tot;
    }
}

hipError_t launch_select(int G, const int32_t* seg_start, const int32_t* cnt, const int32_t* act, const double* f,
                         const double* alpha, const int8_t* y, double C, Rec* rec, Ctl* ctl, hipStream_t s) {
    select_partial_kernel<<<G, 256, 0, s>>>(seg_start, cnt, act, f, alpha, y, C, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    select_merge_kernel<<<1, 1024, 0, s>>>(G, rec, alpha, ctl);
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
constexpr int SLOT_R_MAX = 8;

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

// Large-d CSR: a few A rows at a time per workgroup, densified through a u16 slot map over
// the d columns (zeroed once, cleared sparsely after each group).
template <typename KT>
__global__ __launch_bounds__(SUM_BLOCK) void kernel_sum_slot_kernel(SumArgs A) {
    // R = A.slot_rows target rows at a time: slot[c] numbers the columns of their union
    // (1-based; 0 = in none of them) and tab[slot][r] holds row r's value there, so one pass
    // over a support vector's nonzeros serves all R rows
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_red[SUM_BLOCK / 64][SLOT_R_MAX];
    __shared__ double s_na[SLOT_R_MAX];
    __shared__ int s_u;
    const int R = A.slot_rows;
    uint16_t* slot = reinterpret_cast<uint16_t*>(smem);
    float* tab = reinterpret_cast<float*>(smem + ((sizeof(uint16_t) * (size_t)A.d + 15) & ~(size_t)15));
    const int tab_rows = 1 + R * A.rows_per_block;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int k = tid; k < A.d; k += SUM_BLOCK) slot[k] = 0;
    for (int e = tid; e < tab_rows * R; e += SUM_BLOCK) tab[e] = 0.f;
    __syncthreads();
    const KT gam = (KT)A.gamma;
    const int per = (A.nb + A.nsplit - 1) / A.nsplit;
    const int b0 = blockIdx.y * per, b1 = min(A.nb, b0 + per);
    const int ngroups = (A.na + R - 1) / R;
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int r0 = grp * R, nr = min(R, A.na - r0);
        // union of the group's columns: one thread per row claims slots in row order
        if (tid == 0) {
            int u = 0;
            for (int r = 0; r < nr; ++r) {
                const int a = A.alist ? A.alist[r0 + r] : r0 + r;
                for (int p = A.arp[a]; p < A.arp[a + 1]; ++p) {
                    const int c = A.acol[p];
                    int sl = slot[c];
                    if (!sl) { sl = ++u; slot[c] = (uint16_t)sl; }
                    tab[sl * R + r] = A.aval[p];
                }
            }
            s_u = u;
        }
        __syncthreads();
        if (tid < nr) {
            const int a = A.alist ? A.alist[r0 + tid] : r0 + tid;
            KT nn = 0;
            for (int p = A.arp[a]; p < A.arp[a + 1]; ++p) {
                const KT v = (KT)A.aval[p];
                nn += v * v;
            }
            s_na[tid] = (double)nn;
        }
        __syncthreads();
        double acc[SLOT_R_MAX];
#pragma unroll
        for (int r = 0; r < SLOT_R_MAX; ++r) acc[r] = 0.0;
        for (int jb = b0 + tid; jb < b1; jb += SUM_BLOCK) {
            const int j = A.blist[jb];
            const int q0 = A.brp[j], q1 = A.brp[j + 1];
            KT nb = 0, dot[SLOT_R_MAX];
#pragma unroll
            for (int r = 0; r < SLOT_R_MAX; ++r) dot[r] = 0;
            for (int q = q0; q < q1; ++q) {
                const KT v = (KT)A.bval[q];
                nb += v * v;
                const float* t = tab + (int)slot[A.bcol[q]] * R;
#pragma unroll
                for (int r = 0; r < SLOT_R_MAX; ++r)
                    if (r < R) dot[r] += v * (KT)t[r];
            }
#pragma unroll
            for (int r = 0; r < SLOT_R_MAX; ++r) {
                if (r < nr) {
                    KT d2 = (KT)s_na[r] + nb - (KT)2 * dot[r];
                    if (d2 < (KT)0) d2 = (KT)0;
                    acc[r] += A.coef[jb] * (double)kexp(-gam * d2);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < SLOT_R_MAX; ++r) {
            const double v = wave_sum(acc[r]);
            if (lane == 0) s_red[wid][r] = v;
        }
        __syncthreads();
        if (tid < nr) {
            double t = 0.0;
            for (int w = 0; w < SUM_BLOCK / 64; ++w) t += s_red[w][tid];
            A.part[(size_t)blockIdx.y * A.na + r0 + tid] = t;
        }
        // clear the group's slots and table rows for the next group
        if (tid == 0) {
            for (int r = 0; r < nr; ++r) {
                const int a = A.alist ? A.alist[r0 + r] : r0 + r;
                for (int p = A.arp[a]; p < A.arp[a + 1]; ++p) slot[A.acol[p]] = 0;
            }
        }
        for (int e = tid; e < (1 + s_u) * R; e += SUM_BLOCK) tab[e] = 0.f;
        __syncthreads();
    }
}

// Dense rows, FP32 kernel values: the distance terms come from matrix-core products.  A
// workgroup (4 waves) holds 64 A rows in LDS and sweeps its split of the B list 64 rows at a
// time; wave w forms the 16 x 64 block of dot products of A rows 16w.. with the chunk through
// v_mfma_f32_16x16x4f32 (a 16x4 by 4x16 product per instruction, K = dpad in steps of 4), then
// applies the epilogue d2 = |a|^2 + |b|^2 - 2 a.b (clamped at 0), exp(-gamma d2), and adds
// coef_b * K into FP64 row sums.  Operand lanes: A[row][k] and B[k][col] sit in lane
// (row or col) + 16 k; output C[row][col] in lane col + 16 (row / 4), register row % 4.
constexpr int MF_T = 64;              // A rows per workgroup, B rows per chunk
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MF_MAX_DPAD = 240;      // LDS: 2 x 64 rows x (dpad + 1) floats

__global__ __launch_bounds__(SUM_BLOCK) void kernel_sum_mfma_kernel(SumArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float s_na[MF_T], s_nb[MF_T];
    __shared__ double s_cb[MF_T];
    const int dpad = A.dpad, S = dpad + 1;       // odd row stride: column reads hit distinct banks
    float* at = reinterpret_cast<float*>(smem);
    float* bt = at + MF_T * S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r0 = blockIdx.x * MF_T;
    const int nr = min(MF_T, A.na - r0);
    for (int e = tid; e < MF_T * dpad; e += SUM_BLOCK) {
        const int r = e / dpad, k = e % dpad;
        float v = 0.f;
        if (r < nr) v = A.ax[(size_t)(A.alist ? A.alist[r0 + r] : r0 + r) * dpad + k];
        at[r * S + k] = v;
    }
    __syncthreads();
    if (tid < MF_T) {
        float sq = 0.f;
        for (int k = 0; k < dpad; ++k) sq = fmaf(at[tid * S + k], at[tid * S + k], sq);
        s_na[tid] = sq;
    }
    const float gam = (float)A.gamma;
    const int per = (A.nb + A.nsplit - 1) / A.nsplit;
    const int b0 = blockIdx.y * per, b1 = min(A.nb, b0 + per);
    const int mrow = lane & 15, mk = lane >> 4;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = b0; c0 < b1; c0 += MF_T) {
        const int nc = min(MF_T, b1 - c0);
        __syncthreads();                          // the previous chunk is no longer read
        for (int e = tid; e < MF_T * dpad; e += SUM_BLOCK) {
            const int c = e / dpad, k = e % dpad;
            bt[c * S + k] = c < nc ? A.bx[(size_t)A.blist[c0 + c] * dpad + k] : 0.f;
        }
        if (tid < MF_T) s_cb[tid] = tid < nc ? A.coef[c0 + tid] : 0.0;
        __syncthreads();
        if (tid < MF_T) {
            float sq = 0.f;
            for (int k = 0; k < dpad; ++k) sq = fmaf(bt[tid * S + k], bt[tid * S + k], sq);
            s_nb[tid] = sq;
        }
        __syncthreads();
        const float* arow = at + (16 * wid + mrow) * S + mk;
        for (int cb = 0; cb < 4; ++cb) {
            const float* brow = bt + (16 * cb + mrow) * S + mk;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            for (int k4 = 0; k4 < dpad; k4 += 4)
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[k4], brow[k4], d, 0, 0, 0);
            const int col = 16 * cb + mrow;
            const float nbc = s_nb[col];
            const double cbv = s_cb[col];
            const float dv[4] = {d[0], d[1], d[2], d[3]};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * wid + 4 * mk + i;
                float d2 = s_na[row] + nbc - 2.f * dv[i];
                d2 = d2 < 0.f ? 0.f : d2;
                acc[i] += cbv * (double)kexp(-gam * d2);
            }
        }
    }
    // rows 16 wid + 4 mk + i: add the 16 lanes (columns) that share mk
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double v = acc[i];
        for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
        const int row = 16 * wid + 4 * mk + i;
        if (mrow == 0 && row < nr) A.part[(size_t)blockIdx.y * A.na + r0 + row] = v;
    }
}

// Binary rows as bitsets (LAY_BITS): a workgroup holds R = 16 A rows' bitsets in LDS and
// sweeps its split of the B list, one B row per thread and step; the squared distance is
// |a| + |b| - 2 |a & b| from popcounts (exact integers), then exp and FP64 sums as above.
constexpr int BITS_R = 16;

template <typename KT>
__global__ __launch_bounds__(SUM_BLOCK) void kernel_sum_bits_kernel(SumArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_red[SUM_BLOCK / 64][BITS_R];
    __shared__ int s_na[BITS_R];
    uint32_t* at = reinterpret_cast<uint32_t*>(smem);   // [BITS_R][wpr]
    const int wpr = A.wpr;
    const int r0 = blockIdx.x * BITS_R;
    const int nr = min(BITS_R, A.na - r0);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int e = tid; e < BITS_R * wpr; e += SUM_BLOCK) {
        const int r = e / wpr, k = e % wpr;
        at[e] = r < nr ? A.abits[(size_t)(A.alist ? A.alist[r0 + r] : r0 + r) * wpr + k] : 0u;
    }
    __syncthreads();
    if (tid < BITS_R) {
        int c = 0;
        for (int k = 0; k < wpr; ++k) c += __popc(at[tid * wpr + k]);
        s_na[tid] = c;
    }
    __syncthreads();
    double acc[BITS_R];
#pragma unroll
    for (int r = 0; r < BITS_R; ++r) acc[r] = 0.0;
    const KT gam = (KT)A.gamma;
    const int per = (A.nb + A.nsplit - 1) / A.nsplit;
    const int b0 = blockIdx.y * per, b1 = min(A.nb, b0 + per);
    for (int jb = b0 + tid; jb < b1; jb += SUM_BLOCK) {
        const int j = A.blist[jb];
        const double cj = A.coef[jb];
        const uint4* xb = reinterpret_cast<const uint4*>(A.bbits + (size_t)j * wpr);
        int nb = 0, dot[BITS_R];
#pragma unroll
        for (int r = 0; r < BITS_R; ++r) dot[r] = 0;
        for (int w4 = 0; w4 < wpr / 4; ++w4) {
            const uint4 v = xb[w4];
            nb += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
#pragma unroll
            for (int r = 0; r < BITS_R; ++r) {
                const uint4 t = reinterpret_cast<const uint4*>(at + r * wpr)[w4];
                dot[r] += __popc(v.x & t.x) + __popc(v.y & t.y) + __popc(v.z & t.z) + __popc(v.w & t.w);
            }
        }
#pragma unroll
        for (int r = 0; r < BITS_R; ++r) {
            if (r < nr) {
                KT d2 = (KT)s_na[r] + (KT)nb - (KT)2 * (KT)dot[r];
                if (d2 < (KT)0) d2 = (KT)0;
                acc[r] += cj * (double)kexp(-gam * d2);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < BITS_R; ++r) {
        const double v = wave_sum(acc[r]);
        if (lane == 0) s_red[wid][r] = v;
    }
    __syncthreads();
    if (tid < nr) {
        double v = 0.0;
        for (int w = 0; w < SUM_BLOCK / 64; ++w) v += s_red[w][tid];
        A.part[(size_t)blockIdx.y * A.na + r0 + tid] = v;
    }
}

int slot_rows_for(int d, int max_nnz) {
    const size_t budget = 150 * 1024;
    const size_t base = (sizeof(uint16_t) * (size_t)d + 15) & ~(size_t)15;
    for (int r = SLOT_R_MAX; r > 1; r /= 2)
        if (base + sizeof(float) * (size_t)(1 + r * max_nnz) * r <= budget) return r;
    return 1;
}

bool kernel_sum_uses_mfma(int lay, int dpad, int kprec) {
    return lay == LAY_DENSE && kprec == SVM_KERNEL_FP32 && dpad <= MF_MAX_DPAD;
}

hipError_t launch_kernel_sum(const SumArgs& a, int kprec, hipStream_t s) {
    if (a.na <= 0) return hipSuccess;
    if (a.lay == LAY_BITS) {
        const size_t lds = sizeof(uint32_t) * BITS_R * (size_t)a.wpr;
        dim3 grid((a.na + BITS_R - 1) / BITS_R, a.nsplit);
        SumArgs c = a;
        if (kprec == SVM_KERNEL_FP64) kernel_sum_bits_kernel<double><<<grid, SUM_BLOCK, lds, s>>>(c);
        else kernel_sum_bits_kernel<float><<<grid, SUM_BLOCK, lds, s>>>(c);
        return hipGetLastError();
    }
    if (kernel_sum_uses_mfma(a.lay, a.dpad, kprec)) {
        const size_t lds = sizeof(float) * 2 * MF_T * (size_t)(a.dpad + 1);
        dim3 grid((a.na + MF_T - 1) / MF_T, a.nsplit);
        SumArgs c = a;
        (void)hipFuncSetAttribute((const void*)kernel_sum_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        kernel_sum_mfma_kernel<<<grid, SUM_BLOCK, lds, s>>>(c);
        return hipGetLastError();
    }
    if (a.lay == LAY_CSR_SLOT) {
        // rows_per_block carries the longest A row here, slot_rows the rows per group
        const size_t lds = ((sizeof(uint16_t) * (size_t)a.d + 15) & ~(size_t)15) +
                           sizeof(float) * (size_t)(1 + a.slot_rows * a.rows_per_block) * a.slot_rows;
        dim3 grid(std::min((a.na + a.slot_rows - 1) / a.slot_rows, 2048), a.nsplit);
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

// Kernel sums from the whole kernel matrix in memory (K(b, a) at kmat[b * ldk + a]): one thread
// per target row a, its split of the B list in order, eight matrix rows in flight per thread.
// The rows of B are read contiguously along a, so a workgroup reads 1 KB per support vector.
__global__ __launch_bounds__(256) void kmat_sum_kernel(int na, const int32_t* __restrict__ alist, int nb,
                                                       const int32_t* __restrict__ blist,
                                                       const double* __restrict__ coef,
                                                       const float* __restrict__ kmat, long long ldk, double* part) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = (nb + gridDim.y - 1) / gridDim.y;
    const int b0 = blockIdx.y * per, b1 = min(nb, b0 + per);
    if (r >= na) return;
    const int a = alist ? alist[r] : r;
    double acc = 0.0;
    int j = b0;
    for (; j + 8 <= b1; j += 8) {
        float k[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) k[u] = kmat[(size_t)blist[j + u] * ldk + a];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += coef[j + u] * (double)k[u];
    }
    for (; j < b1; ++j) acc += coef[j] * (double)kmat[(size_t)blist[j] * ldk + a];
    part[(size_t)blockIdx.y * na + r] = acc;
}

hipError_t launch_kmat_sum(int na, const int32_t* alist, int nb, const int32_t* blist, const double* coef,
                           const float* kmat, long long ldk, int nsplit, double* part, hipStream_t s) {
    if (na <= 0) return hipSuccess;
    const dim3 grid((na + 255) / 256, nsplit);
    kmat_sum_kernel<<<grid, 256, 0, s>>>(na, alist, nb, blist, coef, kmat, ldk, part);
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

__global__ __launch_bounds__(256) void pack_pairs_kernel(int n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ prp,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ val, int pattern_only,
                                                         uint16_t* col16, float* val2) {
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4), sub = threadIdx.x & 15;   // 16 threads per row
    if (i >= n) return;
    const int p0 = rp[i], len = rp[i + 1] - p0;
    const int64_t o = 2 * (int64_t)prp[i];
    for (int k = sub; k < len; k += 16) {
        col16[o + k] = (uint16_t)col[p0 + k];
        val2[o + k] = pattern_only ? 1.f : val[p0 + k];
    }
    if ((len & 1) && sub == 0) {
        col16[o + len] = (uint16_t)0;
        val2[o + len] = 0.f;
    }
}

hipError_t launch_pack_pairs(int n, const int32_t* rp, const int32_t* prp, const int32_t* col, const float* val,
                             int pattern_only, uint16_t* col16, float* val2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    pack_pairs_kernel<<<(n + 15) / 16, 256, 0, s>>>(n, rp, prp, col, val, pattern_only, col16, val2);
    return hipGetLastError();
}

}  // namespace svm

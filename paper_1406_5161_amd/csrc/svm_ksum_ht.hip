// svm_ksum_ht.hip -- kernel sums over wide sparse rows (Alg. 6 gradient reconstruction, the
// closing recompute and the classifier of eq:classi) with the dot products split by column
// frequency: the H most frequent columns of the training set form a dense "head" row per
// sample, multiplied on the matrix cores; the remaining "tail" nonzeros are matched through a
// hash table of the target rows' tail columns in LDS.  Both parts are sums of FP32 products:
// the head on the matrix cores, the tail exactly in 64-bit fixed point (so its sum does not
// depend on the order in which threads add); the squared distance is
// |a|^2 + |b|^2 - 2 (a_h.b_h + a_t.b_t) as in the other FP32 kernel sums.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "svm_device.h"
#include "svm_internal.h"

namespace svm {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ preparation

// Occurrences of every column over the nonzeros of a CSR matrix (cnt zeroed by the caller).
__global__ void col_count_kernel(int64_t nnz, const int32_t* __restrict__ col, int32_t* cnt) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[p]], 1);
}

hipError_t launch_col_count(int64_t nnz, const int32_t* col, int32_t* cnt, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nnz + 255) / 256, 4096);
    col_count_kernel<<<(unsigned)blocks, 256, 0, s>>>(nnz, col, cnt);
    return hipGetLastError();
}

// Per row i (16 threads): head[i][0..H) = the row's values in the head columns (hmap[c] >= 0
// gives the position), zero elsewhere; nrm[i] = |x_i|^2 summed in CSR order in FP32; tcnt[i] =
// its tail nonzeros.  maxn2 receives the largest |x_i|^2 (bits of a non-negative float).
__global__ __launch_bounds__(256) void ht_split_kernel(int n, int H, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const int32_t* __restrict__ hmap, float* head, float* nrm,
                                                       int32_t* tcnt, unsigned* maxn2) {
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4), sub = threadIdx.x & 15;
    const bool ok = i < n;
    float* h = head + (size_t)i * H;
    if (ok)
        for (int k = sub; k < H; k += 16) h[k] = 0.f;
    __syncthreads();   // zeros before values
    if (!ok) return;
    const int p0 = rp[i], p1 = rp[i + 1];
    for (int p = p0 + sub; p < p1; p += 16) {
        const int k = hmap[col[p]];
        if (k >= 0) h[k] = val[p];
    }
    if (sub == 0) {
        float s = 0.f;
        int t = 0;
        for (int p = p0; p < p1; ++p) {
            const float v = val[p];
            s += v * v;
            t += hmap[col[p]] < 0 ? 1 : 0;
        }
        nrm[i] = s;
        tcnt[i] = t;
        atomicMax(maxn2, __float_as_uint(s));
    }
}

hipError_t launch_ht_split(int n, int H, const int32_t* rp, const int32_t* col, const float* val,
                           const int32_t* hmap, float* head, float* nrm, int32_t* tcnt, unsigned* maxn2,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    ht_split_kernel<<<(n + 15) / 16, 256, 0, s>>>(n, H, rp, col, val, hmap, head, nrm, tcnt, maxn2);
    return hipGetLastError();
}

// Largest number of tail nonzeros in any tile of 64, 32 and 16 consecutive target rows
// (out3[0..2], zeroed by the caller): the host takes the largest tile whose tail fits the
// kernel's LDS table.
__global__ void ht_tiles_kernel(int na, const int32_t* __restrict__ alist, const int32_t* __restrict__ tcnt,
                                int32_t* out3) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;   // one tile of 64 rows
    if (t * 64 >= na) return;
    int s16[4] = {0, 0, 0, 0};
    for (int r = 0; r < 64; ++r) {
        const int k = t * 64 + r;
        if (k >= na) break;
        s16[r >> 4] += tcnt[alist ? alist[k] : k];
    }
    atomicMax(&out3[0], s16[0] + s16[1] + s16[2] + s16[3]);
    atomicMax(&out3[1], max(s16[0] + s16[1], s16[2] + s16[3]));
    atomicMax(&out3[2], max(max(s16[0], s16[1]), max(s16[2], s16[3])));
}

hipError_t launch_ht_tiles(int na, const int32_t* alist, const int32_t* tcnt, int32_t* out3, hipStream_t s) {
    if (na <= 0) return hipSuccess;
    const int tiles = (na + 63) / 64;
    ht_tiles_kernel<<<(tiles + 255) / 256, 256, 0, s>>>(na, alist, tcnt, out3);
    return hipGetLastError();
}

// The support vectors in sweep order, packed once per kernel sum so the sweep reads them
// contiguously: head rows [nbp][H] and |x|^2 (rows nb..nbp-1 zero), and the tail nonzeros of
// support vector j (in its column order) as (column << 6 | j % 64, value bits) from toff[j].
// toff is the exclusive scan of the tail counts, by one workgroup in chunks of 1024.
__global__ __launch_bounds__(1024) void ht_tail_offsets_kernel(int nb, const int32_t* __restrict__ blist,
                                                               const int32_t* __restrict__ tcnt, int32_t* toff) {
    __shared__ int s_w[16];
    __shared__ int s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int base = 0; base < nb; base += 1024) {
        const int t = base + threadIdx.x;
        const int v = t < nb ? tcnt[blist[t]] : 0;
        int x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(x, off);
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
        if (t < nb) toff[t] = carry + woff + x - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) toff[nb] = s_carry;
}

__global__ __launch_bounds__(256) void ht_pack_kernel(int nb, int nbp, int H, const int32_t* __restrict__ blist,
                                                      const float* __restrict__ head, const float* __restrict__ nrm,
                                                      const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const float* __restrict__ val, const int32_t* __restrict__ hmap,
                                                      const int32_t* __restrict__ toff, float* bhead, float* bnrm,
                                                      uint2* tent) {
    const int j = blockIdx.x * 16 + (threadIdx.x >> 4), sub = threadIdx.x & 15;
    if (j >= nbp) return;
    float* dst = bhead + (size_t)j * H;
    if (j >= nb) {
        for (int k = sub; k < H; k += 16) dst[k] = 0.f;
        if (sub == 0) bnrm[j] = 0.f;
        return;
    }
    const int a = blist[j];
    const float* src = head + (size_t)a * H;
    for (int k = sub; k < H; k += 16) dst[k] = src[k];
    if (sub == 0) {
        bnrm[j] = nrm[a];
        int e = toff[j];
        const unsigned tag = (unsigned)(j & 63);
        for (int p = rp[a]; p < rp[a + 1]; ++p) {
            const int c = col[p];
            if (hmap[c] < 0) tent[e++] = make_uint2(((unsigned)c << 6) | tag, __float_as_uint(val[p]));
        }
    }
}

hipError_t launch_ht_pack(int nb, int H, const int32_t* blist, const float* head, const float* nrm, const int32_t* rp,
                          const int32_t* col, const float* val, const int32_t* hmap, const int32_t* tcnt,
                          int32_t* toff, float* bhead, float* bnrm, uint2* tent, hipStream_t s) {
    const int nbp = (nb + HT_CHUNK - 1) / HT_CHUNK * HT_CHUNK;
    ht_tail_offsets_kernel<<<1, 1024, 0, s>>>(nb, blist, tcnt, toff);
    if (nbp > 0)
        ht_pack_kernel<<<(nbp + 15) / 16, 256, 0, s>>>(nb, nbp, H, blist, head, nrm, rp, col, val, hmap, toff, bhead,
                                                         bnrm, tent);
    return hipGetLastError();
}

// ------------------------------------------------------------------ the kernel sum

// LDS table of the tile's tail nonzeros grouped by column: an open-addressing hash over the
// columns, slot word (column + 1) << 13 | first entry, slot count in a byte array, and the
// entries (target row, value) of one column contiguous, so a lookup reads its matches with
// independent loads.
DEV uint32_t ht_slot0(int c) { return ((uint32_t)c * 2654435761u) >> (32 - 13); }
static_assert(HT_SLOTS == 1 << 13, "hash width");
static_assert(HT_ENTRIES <= (1 << 13), "first-entry field");
static_assert(HT_TILE_MAX <= 255, "row byte and count byte");

template <int H>
struct HtLds {
    static constexpr int HS = H + 4;   // row stride of the staged head rows (b128 reads without conflicts)
    // tail-dot tile, support vector major: the atomics of one support vector's nonzeros go to
    // consecutive target rows (distinct banks); the odd stride spreads the epilogue's reads
    static constexpr int CS = HT_TILE_MAX + 1;
    static constexpr size_t bits = 0;
    static constexpr size_t hkey = bits + sizeof(uint32_t) * HT_MAX_WORDS;
    static constexpr size_t hcnt = hkey + sizeof(uint32_t) * HT_SLOTS;
    static constexpr size_t erow = hcnt + sizeof(uint8_t) * HT_SLOTS;
    static constexpr size_t eval = erow + sizeof(uint8_t) * HT_ENTRIES;
    static constexpr size_t bt = eval + sizeof(float) * HT_ENTRIES;
    static constexpr size_t corr = bt + sizeof(float) * HT_CHUNK * HS;
    static constexpr size_t cb = corr + sizeof(unsigned long long) * HT_CHUNK * CS;
    static constexpr size_t nb = cb + sizeof(double) * HT_CHUNK;
    static constexpr size_t na = nb + sizeof(float) * HT_CHUNK;
    static constexpr size_t red = na + sizeof(float) * HT_TILE_MAX;
    static constexpr size_t misc = red + sizeof(double) * 4 * HT_TILE_MAX;
    static constexpr size_t total = misc + 64;
    // the tail-dot tile doubles as the table builder's per-slot counters
    static_assert(sizeof(unsigned long long) * HT_CHUNK * CS >= sizeof(uint32_t) * HT_SLOTS, "builder scratch");
};

// Workgroup = 8 waves and one tile of R (16, 32 or 64) target rows; it sweeps its split (whole
// chunks) of the packed support vectors HT_CHUNK at a time.  Per chunk: the head rows are
// staged in LDS, and the chunk's tail nonzeros, spread evenly over the threads, are looked up
// in the tile's column table; each match adds a value product into a 64 x 64 tile of 64-bit
// fixed-point tail dots (stored support vector major, so the adds of one support vector's
// nonzeros fall in distinct LDS banks).  The next chunk's data are loaded into registers meanwhile.
// Then the waves form the head dots of their 16 x 16 blocks on the matrix cores
// (v_mfma_f32_16x16x4f32; K = H, where for instruction t lane q of a 16-lane group supplies
// column (H/4) q + t of both operands, so each lane reads H/4 consecutive values), add the tail
// dot, and apply d2 = |a|^2 + |b|^2 - 2 dot (clamped at 0), exp(-gamma d2), coef_b K into FP64
// row sums.  Block k of the tile is (row block k % RB, column block k / RB), RB = R / 16, and
// wave w takes blocks w and w + 8, so its row block is fixed for the whole sweep and its A
// operands stay in registers.
template <int H>
__global__ __launch_bounds__(HT_BLOCK) void kernel_sum_ht_kernel(HtArgs A) {
    using L = HtLds<H>;
    constexpr int KQ = H / 4;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* s_bits = reinterpret_cast<uint32_t*>(smem + L::bits);
    uint32_t* s_hkey = reinterpret_cast<uint32_t*>(smem + L::hkey);
    uint8_t* s_hcnt = reinterpret_cast<uint8_t*>(smem + L::hcnt);
    uint8_t* s_erow = reinterpret_cast<uint8_t*>(smem + L::erow);
    float* s_eval = reinterpret_cast<float*>(smem + L::eval);
    float* s_bt = reinterpret_cast<float*>(smem + L::bt);
    unsigned long long* s_corr = reinterpret_cast<unsigned long long*>(smem + L::corr);
    uint32_t* s_slotc = reinterpret_cast<uint32_t*>(smem + L::corr);   // builder counters
    double* s_cb = reinterpret_cast<double*>(smem + L::cb);
    float* s_nb = reinterpret_cast<float*>(smem + L::nb);
    float* s_na = reinterpret_cast<float*>(smem + L::na);
    double* s_red = reinterpret_cast<double*>(smem + L::red);
    int* s_scan = reinterpret_cast<int*>(smem + L::misc);               // [HT_BLOCK / 64]

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int R = A.tile_rows, RB = R >> 4;
    const int r0 = blockIdx.x * R;
    const int nr = min(R, A.na - r0);
    const int nwords = (A.d + 31) >> 5;
    for (int k = tid; k < nwords; k += HT_BLOCK) s_bits[k] = A.hbits[k];
    for (int k = tid; k < HT_SLOTS; k += HT_BLOCK) { s_hkey[k] = 0u; s_slotc[k] = 0u; }
    __syncthreads();

    // the tile's rows (8 threads per row): norms; every tail nonzero claims its column's slot
    // and counts itself there
    const int tr = tid >> 3, tsub = tid & 7;
    const int ta = tr < nr ? (A.alist ? A.alist[r0 + tr] : r0 + tr) : 0;
    auto find_slot = [&](int c, bool insert) -> uint32_t {
        const uint32_t key = (uint32_t)(c + 1) << 13;
        uint32_t slot = ht_slot0(c);
        for (;;) {
            uint32_t w = __hip_atomic_load(&s_hkey[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (insert && w == 0u) {
                w = atomicCAS(&s_hkey[slot], 0u, key);
                if (w == 0u) return slot;
            }
            if ((w & ~0x1FFFu) == key) return slot;
            slot = (slot + 1) & (HT_SLOTS - 1);
        }
    };
    if (tr < nr) {
        if (tsub == 0) s_na[tr] = A.a_nrm[ta];
        const int p1 = A.a_rp[ta + 1];
        for (int p = A.a_rp[ta] + tsub; p < p1; p += 8) {
            const int c = A.a_col[p];
            if ((s_bits[c >> 5] >> (c & 31)) & 1u) continue;
            atomicAdd(&s_slotc[find_slot(c, true)], 1u);
        }
    }
    __syncthreads();
    // first entry of every slot: exclusive scan of the counts (16 slots per thread)
    {
        constexpr int PER = HT_SLOTS / HT_BLOCK;
        int loc = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) loc += (int)s_slotc[tid * PER + k];
        int x = loc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(x, off);
            if (lane >= off) x += o;
        }
        if (lane == 63) s_scan[wid] = x;
        __syncthreads();
        int run = x - loc;
        for (int w = 0; w < wid; ++w) run += s_scan[w];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int sl = tid * PER + k;
            const uint32_t cnt = s_slotc[sl];
            s_hcnt[sl] = (uint8_t)cnt;
            if (cnt) s_hkey[sl] |= (uint32_t)run;
            run += (int)cnt;
            s_slotc[sl] = 0u;   // from here on the fill cursor of the slot
        }
    }
    __syncthreads();
    // the entries themselves, contiguous per column (their order within a column is free:
    // the tail dots are exact fixed-point sums)
    if (tr < nr) {
        const int p1 = A.a_rp[ta + 1];
        for (int p = A.a_rp[ta] + tsub; p < p1; p += 8) {
            const int c = A.a_col[p];
            if ((s_bits[c >> 5] >> (c & 31)) & 1u) continue;
            const uint32_t sl = find_slot(c, false);
            const int e = (int)(s_hkey[sl] & 0x1FFFu) + (int)atomicAdd(&s_slotc[sl], 1u);
            s_erow[e] = (uint8_t)tr;
            s_eval[e] = A.a_val[p];
        }
    }
    __syncthreads();
    for (int k = tid; k < HT_CHUNK * L::CS; k += HT_BLOCK) s_corr[k] = 0ull;
    // head values of this wave's 16 target rows: lane (row + 16 q) holds columns (H/4) q ..
    const int rb = wid % RB;
    const int q = lane >> 4, l16 = lane & 15;
    const bool mwave = wid < 4 * RB;
    float areg[KQ];
    {
        const int r = 16 * rb + l16;
#pragma unroll
        for (int t = 0; t < KQ; ++t) areg[t] = 0.f;
        if (mwave && r < nr) {
            const int a = A.alist ? A.alist[r0 + r] : r0 + r;
            const float4* src = reinterpret_cast<const float4*>(A.a_head + (size_t)a * H + KQ * q);
#pragma unroll
            for (int t4 = 0; t4 < KQ / 4; ++t4) {
                const float4 v = src[t4];
                areg[4 * t4] = v.x; areg[4 * t4 + 1] = v.y; areg[4 * t4 + 2] = v.z; areg[4 * t4 + 3] = v.w;
            }
        }
    }
    __syncthreads();   // hash and entries complete

    const float gam = (float)A.gamma;
    const double fx_scale = A.fx_scale, fx_inv = A.fx_inv;
    // splits are whole chunks, so chunk rows are support-vector ordinals modulo 64
    const int per = (A.nb + A.nsplit * HT_CHUNK - 1) / (A.nsplit * HT_CHUNK) * HT_CHUNK;
    const int b0 = blockIdx.y * per, b1 = min(A.nb, b0 + per);
    constexpr int HV = HT_CHUNK * (H / 4) / HT_BLOCK;   // float4 of head rows per thread and chunk
    constexpr int PE = 8;                               // tail entries per thread held ahead
    static_assert(HV >= 1, "head tile");
    double racc[4] = {0.0, 0.0, 0.0, 0.0};
    // the next chunk's head values, tail entries, norm and coefficient are loaded one chunk
    // ahead into registers (the end offset of its tail two chunks ahead)
    float4 hv[HV];
    uint2 pe[PE];
    float pnrm = 0.f;
    double pcf = 0.0;
    int e_lo = 0, e_hi = 0, e_next = 0;
    auto prefetch = [&](int c0, int lo, int hi) {
        const float4* src = reinterpret_cast<const float4*>(A.b_head + (size_t)c0 * H);
#pragma unroll
        for (int v = 0; v < HV; ++v) hv[v] = src[tid + HT_BLOCK * v];
#pragma unroll
        for (int m = 0; m < PE; ++m) {
            const int e = lo + tid + HT_BLOCK * m;
            pe[m] = e < hi ? A.b_tent[e] : make_uint2(0xffffffffu, 0u);
        }
        if (tid < HT_CHUNK) {
            pnrm = A.b_nrm[c0 + tid];
            pcf = c0 + tid < b1 ? A.coef[c0 + tid] : 0.0;
        }
    };
    if (b0 < b1) {
        e_lo = A.b_toff[b0];
        e_hi = A.b_toff[min(b0 + HT_CHUNK, b1)];
        e_next = A.b_toff[min(b0 + 2 * HT_CHUNK, b1)];
        prefetch(b0, e_lo, e_hi);
    }
    for (int c0 = b0; c0 < b1; c0 += HT_CHUNK) {
        const int nc = min(HT_CHUNK, b1 - c0);
        // this chunk: head rows into LDS, norms and coefficients, tail products into the tile
#pragma unroll
        for (int v = 0; v < HV; ++v) {
            const int e = tid + HT_BLOCK * v;
            *reinterpret_cast<float4*>(s_bt + (e / (H / 4)) * L::HS + 4 * (e % (H / 4))) = hv[v];
        }
        if (tid < HT_CHUNK) {
            s_nb[tid] = pnrm;
            s_cb[tid] = pcf;
        }
        // a support-vector tail nonzero: each of its column's entries in the table adds the
        // product as a 64-bit integer (the product of two FP32 values is exact in FP64, the
        // scale a power of two, the conversion rounds to nearest)
        auto tail = [&](uint2 t) {
            const uint32_t key = (t.x >> 6) + 1u;   // a tail column by construction
            uint32_t slot = ht_slot0((int)(t.x >> 6)), w;
            while ((w = s_hkey[slot]) != 0u && (w >> 13) != key) slot = (slot + 1) & (HT_SLOTS - 1);
            if (!w) return;
            const int e0 = (int)(w & 0x1FFFu), ne = s_hcnt[slot];
            const double vb = (double)__uint_as_float(t.y) * fx_scale;
            unsigned long long* col = s_corr + (int)(t.x & 63u) * L::CS;
            for (int k = 0; k < ne; ++k) {
                const long long v = __double2ll_rn((double)s_eval[e0 + k] * vb);
                atomicAdd(&col[s_erow[e0 + k]], (unsigned long long)v);
            }
        };
#pragma unroll
        for (int m = 0; m < PE; ++m)
            if (pe[m].x != 0xffffffffu) tail(pe[m]);
        for (int e = e_lo + tid + HT_BLOCK * PE; e < e_hi; e += HT_BLOCK) tail(A.b_tent[e]);
        // the next chunk's loads are in flight while this one is reduced
        if (c0 + HT_CHUNK < b1) {
            const int c2 = c0 + HT_CHUNK;
            const int lo = e_hi, hi = e_next;
            e_lo = lo;
            e_hi = hi;
            prefetch(c2, lo, hi);
            e_next = A.b_toff[min(c2 + 2 * HT_CHUNK, b1)];
        }
        __syncthreads();
        if (mwave) {
            for (int k = wid; k < 4 * RB; k += 8) {
                const int cbk = k / RB;
                const int col = 16 * cbk + l16;
                const float* brow = s_bt + col * L::HS + KQ * q;
                float bv[KQ];
#pragma unroll
                for (int t4 = 0; t4 < KQ / 4; ++t4) {
                    const float4 v = *reinterpret_cast<const float4*>(brow + 4 * t4);
                    bv[4 * t4] = v.x; bv[4 * t4 + 1] = v.y; bv[4 * t4 + 2] = v.z; bv[4 * t4 + 3] = v.w;
                }
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < KQ; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[t], bv[t], acc, 0, 0, 0);
                const float nbc = s_nb[col];
                const double cbv = s_cb[col];
                const float dv[4] = {acc[0], acc[1], acc[2], acc[3]};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * rb + 4 * q + i;
                    unsigned long long* cell = &s_corr[col * L::CS + row];
                    const long long tv = (long long)*cell;
                    *cell = 0ull;
                    if (row < nr && col < nc) {
                        const float dot = dv[i] + (float)((double)tv * fx_inv);
                        float d2 = s_na[row] + nbc - 2.f * dot;
                        d2 = d2 < 0.f ? 0.f : d2;
                        const float kv = kexp(-gam * d2);
                        racc[i] += cbv * (double)kv;
                        if (A.kout) {
                            const int a = A.alist ? A.alist[r0 + row] : r0 + row;
                            const int b = c0 + col;
                            A.kout[(size_t)b * A.ldk + a] = a == b ? 1.f : kv;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    // rows 16 rb + 4 q + i: add the 16 lanes (columns) of each q, then the waves of each row block
    if (mwave) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v = racc[i];
            for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
            if (l16 == 0) s_red[(wid / RB) * HT_TILE_MAX + 16 * rb + 4 * q + i] = v;
        }
    }
    __syncthreads();
    if (tid < nr) {
        const int groups = RB == 4 ? 2 : 4;
        double v = 0.0;
        for (int g = 0; g < groups; ++g) v += s_red[g * HT_TILE_MAX + tid];
        A.part[(size_t)blockIdx.y * A.na + r0 + tid] = v;
    }
}

size_t ht_lds_bytes(int H) {
    switch (H) {
        case 32: return HtLds<32>::total;
        case 64: return HtLds<64>::total;
        case 128: return HtLds<128>::total;
        default: return 0;
    }
}

hipError_t launch_kernel_sum_ht(const HtArgs& a, hipStream_t s) {
    if (a.na <= 0) return hipSuccess;
    const size_t lds = ht_lds_bytes(a.H);
    if (!lds || (a.tile_rows != 16 && a.tile_rows != 32 && a.tile_rows != 64)) return hipErrorInvalidValue;
    dim3 grid((a.na + a.tile_rows - 1) / a.tile_rows, a.nsplit);
    HtArgs c = a;
    switch (a.H) {
        case 32:
            (void)hipFuncSetAttribute((const void*)kernel_sum_ht_kernel<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_ht_kernel<32><<<grid, HT_BLOCK, lds, s>>>(c);
            break;
        case 64:
            (void)hipFuncSetAttribute((const void*)kernel_sum_ht_kernel<64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_ht_kernel<64><<<grid, HT_BLOCK, lds, s>>>(c);
            break;
        default:
            (void)hipFuncSetAttribute((const void*)kernel_sum_ht_kernel<128>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            kernel_sum_ht_kernel<128><<<grid, HT_BLOCK, lds, s>>>(c);
            break;
    }
    return hipGetLastError();
}

}  // namespace svm

// svm_device.h -- device helpers shared by the kernels of libsvmhip.so:
// index-set tests on the status byte, the two-threshold reduction with its
// lowest-index tie-break, the FP64 pair update, the agent-scope loads and
// stores of the record exchanges and the dense distance of a row to the
// working pair.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

// DPP lane moves (gfx9 encodings): xor 1 and 2 inside a quad, rotate by 4 and 8 inside a
// 16-lane row, then lane 15 -> next row and lane 31 -> rows 2-3.
constexpr int DPP_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROR4 = 0x124;     // row_ror:4
constexpr int DPP_ROR8 = 0x128;     // row_ror:8
constexpr int DPP_BCAST15 = 0x142;  // row_bcast:15
constexpr int DPP_BCAST31 = 0x143;  // row_bcast:31

// Exact two-threshold reductions (eq:bminmax): the up side keeps the least f, the low side the
// largest, ties to the lowest sample id.  Values are only compared, never combined, so any
// order of reduction picks the same winner.  Each runs in two passes over the lanes: first
// the extreme value, then the lowest id among the lanes holding it; the winner keeps its own
// value (an f equal to the extreme can differ from it only in the sign of a zero).  Lanes
// without a candidate hold (+inf, IDX_NONE) on the up side and (-inf, IDX_NONE) on the low side.
//
// Lane moves: quad swaps and row rotations by 4 and 8 leave every lane of a 16-lane row with
// the row's result; the two row broadcasts then carry it to lane 63 only (the other lanes of
// rows the broadcast does not write end with unspecified values, which nothing reads).
template <int CTRL, int ROWS>
DEV int mov_dpp(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
DEV double mov_dpp_d(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = mov_dpp<CTRL, ROWS>((int)(unsigned)(x & 0xffffffffll));
    const int hi = mov_dpp<CTRL, ROWS>((int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWS>
DEV void ext_step(double& mu, double& ml) {
    const double ou = mov_dpp_d<CTRL, ROWS>(mu), ol = mov_dpp_d<CTRL, ROWS>(ml);
    mu = ou < mu ? ou : mu;
    ml = ol > ml ? ol : ml;
}
// (ids: the move's unwritten lanes hold IDX_NONE, so the min folds into one DPP instruction)
template <int CTRL, int ROWS>
DEV void idx_step(int& ju, int& jl) {
    ju = min(ju, __builtin_amdgcn_update_dpp(IDX_NONE, ju, CTRL, ROWS, 0xF, false));
    jl = min(jl, __builtin_amdgcn_update_dpp(IDX_NONE, jl, CTRL, ROWS, 0xF, false));
}

DEV double readlane_d(double v, int lane) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(x & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave-wide two-threshold reduction; every lane returns the winners.  DPP moves and lane
// reads only: no LDS traffic.  Needs the whole wave active.  With LANES = 16 only lanes 0-15
// may hold candidates (the others must hold the empty entries), and the broadcasts between
// rows are skipped.
template <int LANES = 64>
DEV void wave_reduce_sel(double& bu, int& iu, double& bl, int& il) {
    static_assert(LANES == 16 || LANES == 64, "a row or the whole wave");
    constexpr int LAST = LANES - 1;   // a lane that ends with the result
    double mu = bu, ml = bl;
    ext_step<DPP_XOR1, 0xF>(mu, ml);
    ext_step<DPP_XOR2, 0xF>(mu, ml);
    ext_step<DPP_ROR4, 0xF>(mu, ml);
    ext_step<DPP_ROR8, 0xF>(mu, ml);
    if constexpr (LANES == 64) {
        ext_step<DPP_BCAST15, 0xA>(mu, ml);
        ext_step<DPP_BCAST31, 0xC>(mu, ml);
    }
    mu = readlane_d(mu, LAST);
    ml = readlane_d(ml, LAST);
    int ju = bu == mu ? iu : IDX_NONE, jl = bl == ml ? il : IDX_NONE;
    idx_step<DPP_XOR1, 0xF>(ju, jl);
    idx_step<DPP_XOR2, 0xF>(ju, jl);
    idx_step<DPP_ROR4, 0xF>(ju, jl);
    idx_step<DPP_ROR8, 0xF>(ju, jl);
    if constexpr (LANES == 64) {
        idx_step<DPP_BCAST15, 0xA>(ju, jl);
        idx_step<DPP_BCAST31, 0xC>(ju, jl);
    }
    ju = __builtin_amdgcn_readlane(ju, LAST);
    jl = __builtin_amdgcn_readlane(jl, LAST);
    // the lanes holding the winners (in an empty side every lane holds the same empty entry)
    const int wu = __builtin_ctzll(__ballot(iu == ju && bu == mu));
    const int wl = __builtin_ctzll(__ballot(il == jl && bl == ml));
    bu = readlane_d(bu, wu);
    bl = readlane_d(bl, wl);
    iu = ju;
    il = jl;
}

// Sums of two ints over lanes 0-31 (lanes 32-63 ignored), returned in every lane: row sums by
// DPP (quad swaps, rotations by 4 and 8), then row 0 added into row 1 and read from lane 31.
DEV void sum2_lanes32(int& a, int& b) {
    a += __builtin_amdgcn_update_dpp(0, a, DPP_XOR1, 0xF, 0xF, false);
    b += __builtin_amdgcn_update_dpp(0, b, DPP_XOR1, 0xF, 0xF, false);
    a += __builtin_amdgcn_update_dpp(0, a, DPP_XOR2, 0xF, 0xF, false);
    b += __builtin_amdgcn_update_dpp(0, b, DPP_XOR2, 0xF, 0xF, false);
    a += __builtin_amdgcn_update_dpp(0, a, DPP_ROR4, 0xF, 0xF, false);
    b += __builtin_amdgcn_update_dpp(0, b, DPP_ROR4, 0xF, 0xF, false);
    a += __builtin_amdgcn_update_dpp(0, a, DPP_ROR8, 0xF, 0xF, false);
    b += __builtin_amdgcn_update_dpp(0, b, DPP_ROR8, 0xF, 0xF, false);
    a += __builtin_amdgcn_update_dpp(0, a, DPP_BCAST15, 0xA, 0xF, false);
    b += __builtin_amdgcn_update_dpp(0, b, DPP_BCAST15, 0xA, 0xF, false);
    a = __builtin_amdgcn_readlane(a, 31);
    b = __builtin_amdgcn_readlane(b, 31);
}

// Float sum over the wave by DPP (row sums, then rows 0-3 into lane 63), returned in every lane.
DEV float wave_sum_dpp(float v) {
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_XOR1, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_XOR2, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_ROR4, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_ROR8, 0xF, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_BCAST15, 0xA, 0xF, false));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), DPP_BCAST31, 0xC, 0xF, false));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <typename T>
DEV T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// FP32 kernel values: e^v as 2^(v log2 e) on the hardware base-2 exponential (about 1 ulp; the
// product adds one rounding, an error of the same order as forming v = -gamma d^2 in FP32).
// Results below the smallest normal float may flush to 0.
DEV float kexp(float v) { return __builtin_amdgcn_exp2f(v * 1.44269504088896341f); }
DEV double kexp(double v) { return exp(v); }

DEV double ld_agent(const double* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV void st_agent(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV unsigned long long ld_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void st_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS the block reductions below need: SEL_LDS(BLOCK) doubles and as many ints.
constexpr int SEL_LDS(int block) { return block / 32; }

// Each wave's winners into LDS: s_v / s_i [wave] up side, [BLOCK/64 + wave] low side.
template <int BLOCK>
DEV void waves_to_lds(double bu, int iu, double bl, int il, double* s_v, int* s_i) {
    constexpr int NW = BLOCK / 64;
    const int wid = threadIdx.x >> 6;
    // a wave without candidates holds the empty entries in every lane already
    if (__ballot(iu != IDX_NONE || il != IDX_NONE)) wave_reduce_sel(bu, iu, bl, il);
    if ((threadIdx.x & 63) == 0) {
        s_v[wid] = bu; s_i[wid] = iu;
        s_v[NW + wid] = bl; s_i[NW + wid] = il;
    }
}

// The wave results of waves_to_lds reduced by one wave (every lane of it gets the winners).
template <int BLOCK>
DEV void wave_reduce_waves(double& bu, int& iu, double& bl, int& il, const double* s_v, const int* s_i) {
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    bu = lane < NW ? s_v[lane] : INFINITY;
    iu = lane < NW ? s_i[lane] : IDX_NONE;
    bl = lane < NW ? s_v[NW + lane] : -INFINITY;
    il = lane < NW ? s_i[NW + lane] : IDX_NONE;
    wave_reduce_sel<(NW <= 16 ? 16 : 64)>(bu, iu, bl, il);
}

// Block-wide reduction whose result every thread holds on return; one barrier.  The
// caller must not overwrite s_v / s_i before the next barrier.
template <int BLOCK>
DEV void block_reduce_sel_all(double& bu, int& iu, double& bl, int& il, double* s_v, int* s_i) {
    waves_to_lds<BLOCK>(bu, iu, bl, il, s_v, s_i);
    __syncthreads();
    wave_reduce_waves<BLOCK>(bu, iu, bl, il, s_v, s_i);
}

// Block-wide reduction of the selection candidates; result valid in every thread, and s_v /
// s_i free again on return.
template <int BLOCK>
DEV void block_reduce_sel(double& bu, int& iu, double& bl, int& il, double* s_v, int* s_i) {
    block_reduce_sel_all<BLOCK>(bu, iu, bl, il, s_v, s_i);
    __syncthreads();
}

// Block-wide reduction whose result only wave 0 needs: the wave results go to LDS, one
// barrier, then wave 0 alone reduces them; the other waves return at once.  Every lane of
// wave 0 holds the result; other lanes keep their own candidates.  The caller must not
// overwrite s_v / s_i before the next barrier.
template <int BLOCK>
DEV void block_reduce_sel_wave0(double& bu, int& iu, double& bl, int& il, double* s_v, int* s_i) {
    waves_to_lds<BLOCK>(bu, iu, bl, il, s_v, s_i);
    __syncthreads();
    if ((threadIdx.x >> 6) == 0) wave_reduce_waves<BLOCK>(bu, iu, bl, il, s_v, s_i);
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

// ------------------------------------------------------------------ kernel rows of the pair

// Dense: squared distances of row xr to the pair (u, l) held in LDS as float2,
// by direct difference in the order k = 0..dpad-1 (padding contributes 0).
template <typename KT>
DEV void dense_dist(const float* __restrict__ xr, const float2* __restrict__ pair, int dpad, KT& su, KT& sl) {
    // the row's loads are issued in blocks of DB float4 before any of them is used, so a row
    // read from HBM costs about one memory latency per block instead of one per float4
    constexpr int DB = 8;
    const float4* x4 = reinterpret_cast<const float4*>(xr);
    const float4* p4 = reinterpret_cast<const float4*>(pair);
    const int n4 = dpad / 4;
    KT a = 0, b = 0;
    for (int k0 = 0; k0 < n4; k0 += DB) {
        float4 v[DB];
#pragma unroll
        for (int j = 0; j < DB; ++j)
            if (k0 + j < n4) v[j] = x4[k0 + j];
#pragma unroll
        for (int j = 0; j < DB; ++j) {
            if (k0 + j < n4) {
                const float4 q0 = p4[2 * (k0 + j)], q1 = p4[2 * (k0 + j) + 1];   // (u0 l0 u1 l1) (u2 l2 u3 l3)
                if constexpr (std::is_same<KT, double>::value) {
#pragma clang fp contract(off)
                    double t;
                    t = (double)v[j].x - (double)q0.x; a = a + t * t;
                    t = (double)v[j].x - (double)q0.y; b = b + t * t;
                    t = (double)v[j].y - (double)q0.z; a = a + t * t;
                    t = (double)v[j].y - (double)q0.w; b = b + t * t;
                    t = (double)v[j].z - (double)q1.x; a = a + t * t;
                    t = (double)v[j].z - (double)q1.y; b = b + t * t;
                    t = (double)v[j].w - (double)q1.z; a = a + t * t;
                    t = (double)v[j].w - (double)q1.w; b = b + t * t;
                } else {
                    float t;
                    t = v[j].x - q0.x; a = fmaf(t, t, a);
                    t = v[j].x - q0.y; b = fmaf(t, t, b);
                    t = v[j].y - q0.z; a = fmaf(t, t, a);
                    t = v[j].y - q0.w; b = fmaf(t, t, b);
                    t = v[j].z - q1.x; a = fmaf(t, t, a);
                    t = v[j].z - q1.y; b = fmaf(t, t, b);
                    t = v[j].w - q1.z; a = fmaf(t, t, a);
                    t = v[j].w - q1.w; b = fmaf(t, t, b);
                }
            }
        }
    }
    su = a;
    sl = b;
}


}  // namespace svm

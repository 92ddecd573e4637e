// tiles.hpp -- device building blocks shared by the per-level kernels and the
// persistent sweep: one output tile of the grouped MFMA GEMM and one tile of
// the gather.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_types.hpp"

namespace selinv {

// Global-memory views of generic pointers.  Pointers read from records in
// memory are generic (flat) to the compiler; flat loads also count against
// the LDS wait counter, so a wait for LDS data would wait for every global
// load in flight.  Casting to the global address space gives global loads and
// stores that keep the two counters apart.
#define SELINV_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const SELINV_GLOBAL T *gptr(const T *p) {
    return (const SELINV_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ SELINV_GLOBAL T *gptr_w(T *p) {
    return (SELINV_GLOBAL T *)p;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int MODE>
struct Mode;
template <>
struct Mode<CMP_F64> {
    typedef double T;
    typedef v4d Acc;
    static constexpr int BK = 16;
};
template <>
struct Mode<CMP_F32> {
    typedef float T;
    typedef v4f Acc;
    static constexpr int BK = 16;
};
template <>
struct Mode<CMP_BF16X3> {
    typedef float T;
    typedef v4f Acc;
    static constexpr int BK = 32;
};

// LDS layouts.  F64/F32: [k][m] (m contiguous: the 16 lanes of a row group
// read 16 consecutive m of one k).  BF16X3: [m][k] (k contiguous: a lane reads
// its 8 consecutive k of one m with one 16-byte load).
// k chunk of a BM-row tile: 32 for the 32x32 FP64 / FP32 tiles (the launches
// that cannot fill the device, where each workgroup's time is its chain of
// chunks: half the chunks, half the barriers), Mode::BK otherwise (wider tiles
// keep 16, whose LDS lets four workgroups share a compute unit).  Measured on
// MI355X: 32 everywhere gave 2D 256^2 0.374 ms instead of 0.385 ms but 3D 64^3
// 51.6 ms instead of 45.5 ms.
template <int MODE, int BM>
struct ChunkK {
    static constexpr int value = (BM == 32 && MODE != CMP_BF16X3) ? 32 : Mode<MODE>::BK;
};

// Rows of FP64 chunks are padded by one element: the staging stores of the
// k-contiguous operands (16 lanes along k, one 8-byte element each) then fall
// on 16 distinct bank pairs, where a stride of BM + 2 elements put k and
// k + 8 on the same pair.
template <int MODE, int BM, int BN, int BK = ChunkK<MODE, BM>::value>
struct Smem {
    typedef typename Mode<MODE>::T T;
    static constexpr int PAD = sizeof(T) == 8 ? 1 : 2;
    T a[2][BK][BM + PAD];
    T b[2][BK][BN + PAD];
};
template <int BM, int BN, int BK>
struct Smem<CMP_BF16X3, BM, BN, BK> {
    static constexpr int P = BK + 8;
    __bf16 ah[2][BM][P], al[2][BM][P];
    __bf16 bh[2][BN][P], bl[2][BN][P];
};

// An operand of the split-BF16 form that is contiguous along k (A with
// op = T, B with op = N): each thread moves 4 consecutive k of R / 32 rows of
// every 32-wide chunk, with one 16-byte load (two for FP64 operands) per row
// and one 8-byte LDS store per plane and row.  The split and the zero padding
// are those of the scalar path: v = (float) x, hi = bf16(v), lo = bf16(v - hi).
template <int R, typename TA>
struct SplitKRows {
    static constexpr int NT = R / 32;
    typedef TA v4 __attribute__((ext_vector_type(4), aligned(sizeof(TA))));
    typedef __bf16 v4b __attribute__((ext_vector_type(4)));
    struct Regs {  // one chunk in flight
        v4 reg[NT];
    };
    const SELINV_GLOBAL TA *ptr[NT];
    // Row of element t: the 8-lane groups of one 16-lane store phase take
    // rows 4 apart (group 8p + q -> row 8p + q / 2 + 4 (q & 1)), whose 64-byte
    // spans of the 80-byte padded rows fall on disjoint banks; consecutive
    // rows (one group each) would overlap on four banks.
    __device__ __forceinline__ int row(int t) const {
        const int g = (int)(threadIdx.x >> 3), q = g & 7;
        return (g & ~7) + (q >> 1) + 4 * (q & 1) + 32 * t;
    }
    static __device__ __forceinline__ int swz(int) { return 0; }  // k blocks in their own order
    __device__ __forceinline__ int kk() const { return 4 * (int)(threadIdx.x & 7); }
    // row r of the operand starts at base + r ld (rows clamped into [0, rows))
    __device__ __forceinline__ void init(const void *base, int64_t ld, int r0, int rows) {
        const SELINV_GLOBAL TA *B = gptr((const TA *)base);
#pragma unroll
        for (int t = 0; t < NT; t++) ptr[t] = B + (int64_t)min(r0 + row(t), rows - 1) * ld + kk();
    }
    __device__ __forceinline__ void load(Regs &g, int k0, int K) const {
        if (k0 + 32 <= K) {
#pragma unroll
            for (int t = 0; t < NT; t++) g.reg[t] = *(const SELINV_GLOBAL v4 *)(ptr[t] + k0);
        } else {
            // last, partial chunk: k clamped into the operand
#pragma unroll
            for (int t = 0; t < NT; t++)
#pragma unroll
                for (int e = 0; e < 4; e++) g.reg[t][e] = ptr[t][min(k0 + kk() + e, K - 1) - kk()];
        }
    }
    template <int P>
    __device__ __forceinline__ void store(const Regs &g, __bf16 (&hi)[R][P], __bf16 (&lo)[R][P], int r0, int rows,
                                          int k0, int K) const {
        const v4(&reg)[NT] = g.reg;
#pragma unroll
        for (int t = 0; t < NT; t++) {
            v4b h4, l4;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float v = (r0 + row(t) < rows && k0 + kk() + e < K) ? (float)reg[t][e] : 0.0f;
                const __bf16 h = (__bf16)v;
                h4[e] = h;
                l4[e] = (__bf16)(v - (float)h);
            }
            *(v4b *)&hi[row(t)][kk()] = h4;
            *(v4b *)&lo[row(t)][kk()] = l4;
        }
    }
};

// An operand of the split-BF16 form that is contiguous along its rows (A with
// op = N, B with op = T): each thread owns a block of 4 consecutive rows by
// KB = R / 32 consecutive k (4, 2 or 1) of every 32-wide chunk, loads it as KB
// 16-byte row quads (one per k) and writes it transposed, one store of KB
// values per row and plane.
// The lanes of one store write rows 4 apart, which fall on only two bank
// groups of the padded rows; row r therefore keeps its 8-wide k blocks in
// the order kb ^ swz(r) (swz(r) = 8 ((r >> 3) & 3)), which spreads one
// store over eight bank groups and leaves the MFMA operand reads (8
// consecutive rows, one k block) as they were.  The readers of such a tile
// apply the same order (gemm_tile_op).
template <int R, typename TA>
struct SplitMRows {
    static constexpr int KB = R / 32;
    static constexpr int TPK = R / 4;  // threads along the rows
    typedef TA v4 __attribute__((ext_vector_type(4), aligned(sizeof(TA))));
    typedef __bf16 vkb __attribute__((ext_vector_type(KB)));
    const SELINV_GLOBAL TA *ptr;  // row r0 + r4 (0 when the quad is not whole) of k = kq
    int64_t ld;
    int r0, rows;
    bool full;  // all 4 rows of the quad inside the operand
    struct Regs {  // one chunk in flight
        v4 reg[KB];
    };
    // R = 128: each 16-lane store phase takes 8 row quads at two k offsets 4
    // apart (lane bits 0-2 and 4-5: the row quad, bit 3 and 6-7: the k group),
    // so that its 16 eight-byte stores fall on 16 distinct bank pairs; with
    // 16 row quads at one k they met in pairs (rows 32 apart).
    __device__ __forceinline__ int r4() const {
        const int t = (int)threadIdx.x;
        if constexpr (R == 128) return 4 * ((t & 7) | (((t >> 4) & 3) << 3));
        return 4 * (t % TPK);
    }
    static __device__ __forceinline__ int swz(int r) { return 8 * ((r >> 3) & 3); }
    __device__ __forceinline__ int kq() const {
        const int t = (int)threadIdx.x;
        if constexpr (R == 128) return KB * (((t >> 3) & 1) | ((t >> 6) << 1));
        return KB * (t / TPK);
    }
    // element (r, k) of the operand at base + r + k ld
    __device__ __forceinline__ void init(const void *base, int64_t ld_, int r0_, int rows_) {
        ld = ld_;
        r0 = r0_;
        rows = rows_;
        full = r0 + r4() + 3 < rows;
        ptr = gptr((const TA *)base) + (full ? r0 + r4() : 0) + (int64_t)kq() * ld;
    }
    __device__ __forceinline__ void load(Regs &g, int k0, int K) const {
        v4(&reg)[KB] = g.reg;
        const bool kin = k0 + 32 <= K;
#pragma unroll
        for (int e = 0; e < KB; e++) {
            // k offset from kq; the last, partial chunk clamps k into the operand
            const int64_t kc = kin ? (int64_t)(k0 + e) : (int64_t)(min(k0 + kq() + e, K - 1) - kq());
            if (full) {
                reg[e] = *(const SELINV_GLOBAL v4 *)(ptr + kc * ld);
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++) reg[e][q] = ptr[min(r0 + r4() + q, rows - 1) + kc * ld];
            }
        }
    }
    template <int P>
    __device__ __forceinline__ void store(const Regs &g, __bf16 (&hi)[R][P], __bf16 (&lo)[R][P], int k0,
                                          int K) const {
        const v4(&reg)[KB] = g.reg;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            vkb h, l;
#pragma unroll
            for (int e = 0; e < KB; e++) {
                const float v = (r0 + r4() + q < rows && k0 + kq() + e < K) ? (float)reg[e][q] : 0.0f;
                const __bf16 b = (__bf16)v;
                h[e] = b;
                l[e] = (__bf16)(v - (float)b);
            }
            const int r = r4() + q, kp = kq() ^ swz(r);
            *(vkb *)&hi[r][kp] = h;
            *(vkb *)&lo[r][kp] = l;
        }
    }
};

// One BM x BN output tile of C = alpha op(A) op(B) + beta Cin, computed by
// the 256 threads of the calling workgroup (see gemm.hip for the design),
// for fixed operand forms OPA, OPB (0: N, 1: T).
// Each thread owns LA elements of every A chunk and LB of every B chunk; their
// addresses are formed once (rows clamped into the operand) and advanced by a
// uniform step per chunk, so that the loop issues its loads without per
// element address arithmetic.  Only the last, partial chunk clamps k.  Values
// outside the operands are loaded from a clamped address and replaced by zero
// when staged into LDS, so that no load is tied to a branch.
// CIN: the problem may carry an input matrix (beta Cin); without it Cin is
// ignored and its registers are not reserved.
// PUSH: a step-4 product with push_sn >= 0 also writes its final entries of
// A^{-T}(P,P) into G of each child of P (converted to the storage type TG,
// as the gather would), so that the children's gather can run beside it.
// GA: op(A) is G_K, taken from its sources through its codes (GemmProb::gcode)
// instead of a stored G.  The codes of chunk c + 1 are loaded with the values
// of chunk c, so that the values' addresses are in registers one chunk ahead
// and the loop keeps one round trip per chunk in flight, as for a stored
// operand.  The staged values equal those the gather would have stored.
template <int MODE, int BM, int BN, typename TA, typename TC, bool CIN, int BK, int OPA, int OPB, bool PUSH,
          typename TG, bool GA = false>
__device__ __forceinline__ void gemm_tile_op(const GemmProb &p, const int m0, const int n0,
                                             Smem<MODE, BM, BN, BK> &sm, const MatDev *mats) {
    typedef typename Mode<MODE>::T T;
    typedef typename Mode<MODE>::Acc Acc;
    static_assert(MODE != CMP_BF16X3 || BK % 32 == 0, "split-BF16 chunks are multiples of 32");
    static_assert(256 % BM == 0 && 256 % BN == 0 && 256 % BK == 0, "thread-to-element maps assume divisors of 256");
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = p.M, N = p.N, K = p.K;
    const int64_t lda = p.lda, ldb = p.ldb;

    // (row, k) of element t of this thread's share of an A chunk, (k, col) of B;
    // the contiguous dimension of the operand runs along consecutive threads
    // (measured: reading an in-place G_K along k for op = N as well, which
    // would coalesce its U-panel entries, made C4's products slower)
    auto ai = [&](int t) { return OPA == 0 ? tid % BM : tid / BK + t * (256 / BK); };
    auto ak = [&](int t) { return OPA == 0 ? tid / BM + t * (256 / BM) : tid % BK; };
    auto bj = [&](int t) { return OPB == 0 ? tid / BK + t * (256 / BK) : tid % BN; };
    auto bk = [&](int t) { return OPB == 0 ? tid % BK : tid / BN + t * (256 / BN); };
    const int64_t ksa = OPA == 0 ? lda : 1;  // address step per unit of k
    const int64_t ksb = OPB == 0 ? 1 : ldb;

    // split-BF16 operands take the vector paths: along k (A with op = T, B
    // with op = N) or along the rows (A with op = N, B with op = T)
    constexpr bool VA = MODE == CMP_BF16X3 && !GA, VB = MODE == CMP_BF16X3;
    typedef std::conditional_t<OPA == 1, SplitKRows<BM, TA>, SplitMRows<BM, TA>> VecA;
    typedef std::conditional_t<OPB == 0, SplitKRows<BN, TA>, SplitMRows<BN, TA>> VecB;
    VecA va;
    VecB vb;
    if constexpr (VA) va.init(p.A, lda, m0, M);
    if constexpr (VB) vb.init(p.B, ldb, n0, N);

    const SELINV_GLOBAL TA *pa[GA ? 1 : LA];
    const SELINV_GLOBAL uint32_t *pc[GA ? LA : 1];  // GA: codes of this thread's A elements
    const SELINV_GLOBAL TA *pb[LB];
    {
        const SELINV_GLOBAL TA *B = gptr((const TA *)p.B);
        if constexpr (GA) {
            // G_K is c_L x c_U with ld = lda = c_L, laid out as a stored G would be
            const SELINV_GLOBAL uint32_t *Cd = gptr(mats[p.gmat].gcA) + p.gcode;
#pragma unroll
            for (int t = 0; t < LA; t++) {
                const int64_t r = min(m0 + ai(t), M - 1);
                pc[t] = Cd + (OPA == 0 ? r : r * lda) + ak(t) * ksa;
            }
        } else {
            const SELINV_GLOBAL TA *A = gptr((const TA *)p.A);
#pragma unroll
            for (int t = 0; t < LA; t++) {
                const int64_t r = min(m0 + ai(t), M - 1);
                pa[t] = A + (OPA == 0 ? r : r * lda) + ak(t) * ksa;
            }
        }
#pragma unroll
        for (int t = 0; t < LB; t++) {
            const int64_t c = min(n0 + bj(t), N - 1);
            pb[t] = B + (OPB == 0 ? c * ldb : c) + bk(t) * ksb;
        }
    }

    Acc acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = Acc{0, 0, 0, 0};

    const int nch = (K + BK - 1) / BK;
    // GA: the source arrays of matrix gmat, and the code of every A element
    // of the next chunk to load
    const SELINV_GLOBAL double *gZd = nullptr;
    const SELINV_GLOBAL TA *gZL = nullptr, *gZU = nullptr;
    if constexpr (GA) {
        const MatDev &Md = mats[p.gmat];
        gZd = gptr(Md.Zd);
        gZL = gptr((const TA *)Md.ZL);
        gZU = gptr((const TA *)Md.ZU);
    }
    uint32_t code[GA ? LA : 1];
    auto cload = [&](int c) {
        const int k0 = c * BK;
        if (k0 + BK <= K) {
#pragma unroll
            for (int t = 0; t < LA; t++) code[t] = pc[t][k0 * ksa];
        } else {
#pragma unroll
            for (int t = 0; t < LA; t++) code[t] = pc[t][(int64_t)(min(k0 + ak(t), K - 1) - ak(t)) * ksa];
        }
    };
    // value named by a code (array << 30 | offset; 1 Zd, 2 ZL, 3 ZU): in the
    // mixed forms a diagonal-block entry is rounded to TA as the gather
    // rounds it
    auto gval = [&](uint32_t cd) -> TA {
        const uint32_t kd = cd >> GCODE_SHIFT, off = cd & GCODE_MASK;
        if constexpr (sizeof(TA) == sizeof(double)) {
            const SELINV_GLOBAL TA *src = kd == 1 ? (const SELINV_GLOBAL TA *)gZd : kd == 3 ? gZU : gZL;
            return src[off];
        } else {
            const double vd = gZd[kd == 1 ? off : 0];
            const TA v = (kd == 3 ? gZU : gZL)[kd == 1 ? 0 : off];
            return kd == 1 ? (TA)vd : v;
        }
    };

    // Register slots of the chunks loaded ahead of their LDS stage: PF = 2
    // for the 32-wide tiles, which serve the launches that cannot fill the
    // device, where each workgroup waits on the latency of every chunk's
    // loads (two chunks in flight halve that wait), and for the FP64 64-wide
    // products (within 128 VGPRs, see gemm.hip); 1 for the other tiles, whose
    // launches hide it behind other workgroups (and whose registers would
    // cost occupancy; measured: two slots on the 128-wide split-BF16
    // steps-3/5 tile left C4 at 15.9 ms).
    constexpr int PF = (BM == 32 || (MODE == CMP_F64 && BM == 64 && !GA && !PUSH)) ? 2 : 1;
    TA ra[PF][VA ? 1 : LA], rb[PF][VB ? 1 : LB];
    typename VecA::Regs rva[PF];
    typename VecB::Regs rvb[PF];
    // chunk c into slot S
    auto gload = [&](int c, auto S_) {
        constexpr int S = decltype(S_)::value;
        const int k0 = c * BK;
        if constexpr (VA) va.load(rva[S], k0, K);
        if constexpr (VB) vb.load(rvb[S], k0, K);
        if constexpr (GA) {
#pragma unroll
            for (int t = 0; t < LA; t++) ra[S][t] = gval(code[t]);
            if (c + 1 < nch) cload(c + 1);
        }
        if (k0 + BK <= K) {
            if constexpr (!VA && !GA) {
#pragma unroll
                for (int t = 0; t < LA; t++) ra[S][t] = pa[t][k0 * ksa];
            }
            if constexpr (!VB) {
#pragma unroll
                for (int t = 0; t < LB; t++) rb[S][t] = pb[t][k0 * ksb];
            }
        } else {
            // last, partial chunk: k clamped into the operand
            if constexpr (!VA && !GA) {
#pragma unroll
                for (int t = 0; t < LA; t++) ra[S][t] = pa[t][(int64_t)(min(k0 + ak(t), K - 1) - ak(t)) * ksa];
            }
            if constexpr (!VB) {
#pragma unroll
                for (int t = 0; t < LB; t++) rb[S][t] = pb[t][(int64_t)(min(k0 + bk(t), K - 1) - bk(t)) * ksb];
            }
        }
    };
    // chunk c from slot S into LDS buffer buf
    auto sstore = [&](int buf, int c, auto S_) {
        constexpr int S = decltype(S_)::value;
        const int k0 = c * BK;
        if constexpr (VA) {
            if constexpr (OPA == 1)
                va.store(rva[S], sm.ah[buf], sm.al[buf], m0, M, k0, K);
            else
                va.store(rva[S], sm.ah[buf], sm.al[buf], k0, K);
        } else {
            // a chunk inside the operand is stored without the bound selects
            auto put_a = [&](auto MASK_) {
                constexpr bool MASK = decltype(MASK_)::value;
#pragma unroll
                for (int t = 0; t < LA; t++) {
                    const int i = ai(t), k = ak(t);
                    const T v = (!MASK || (m0 + i < M && k0 + k < K)) ? (T)ra[S][t] : (T)0;
                    if constexpr (MODE == CMP_BF16X3) {
                        const __bf16 h = (__bf16)v;
                        sm.ah[buf][i][k] = h;
                        sm.al[buf][i][k] = (__bf16)(v - (float)h);
                    } else {
                        sm.a[buf][k][i] = v;
                    }
                }
            };
            if (m0 + BM <= M && k0 + BK <= K)
                put_a(std::false_type{});
            else
                put_a(std::true_type{});
        }
        if constexpr (VB) {
            if constexpr (OPB == 0)
                vb.store(rvb[S], sm.bh[buf], sm.bl[buf], n0, N, k0, K);
            else
                vb.store(rvb[S], sm.bh[buf], sm.bl[buf], k0, K);
        } else {
            auto put_b = [&](auto MASK_) {
                constexpr bool MASK = decltype(MASK_)::value;
#pragma unroll
                for (int t = 0; t < LB; t++) {
                    const int j = bj(t), k = bk(t);
                    const T v = (!MASK || (n0 + j < N && k0 + k < K)) ? (T)rb[S][t] : (T)0;
                    if constexpr (MODE == CMP_BF16X3) {
                        const __bf16 h = (__bf16)v;
                        sm.bh[buf][j][k] = h;
                        sm.bl[buf][j][k] = (__bf16)(v - (float)h);
                    } else {
                        sm.b[buf][k][j] = v;
                    }
                }
            };
            if (n0 + BN <= N && k0 + BK <= K)
                put_b(std::false_type{});
            else
                put_b(std::true_type{});
        }
    };
    auto compute = [&](int buf) {
        if constexpr (MODE == CMP_BF16X3) {
#pragma unroll
            for (int kq = 0; kq < BK; kq += 32) {
                const int kb = kq + 8 * (lane >> 4);
                v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
                for (int i = 0; i < TM; i++) {
                    const int r = wm * WM + i * 16 + (lane & 15);
                    const int kr = (VA && OPA == 0) ? kb ^ VecA::swz(r) : kb;  // SplitMRows order
                    ah[i] = *(const v8bf *)&sm.ah[buf][r][kr];
                    al[i] = *(const v8bf *)&sm.al[buf][r][kr];
                }
#pragma unroll
                for (int j = 0; j < TN; j++) {
                    const int c = wn * WN + j * 16 + (lane & 15);
                    const int kc = (VB && OPB == 1) ? kb ^ VecB::swz(c) : kb;
                    bh[j] = *(const v8bf *)&sm.bh[buf][c][kc];
                    bl[j] = *(const v8bf *)&sm.bl[buf][c][kc];
                }
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[i][j], 0, 0, 0);
                    }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kr = kk + (lane >> 4);
                T av[TM], bv[TN];
#pragma unroll
                for (int i = 0; i < TM; i++) av[i] = sm.a[buf][kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < TN; j++) bv[j] = sm.b[buf][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++) {
                        if constexpr (MODE == CMP_F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j], av[i], acc[i][j], 0, 0, 0);
                    }
            }
        }
    };

    // K == 0 (C = beta Cin): no chunk, no operand read.  Chunks whose
    // products are all zero by the operands' triangular structure are
    // skipped (p.ktri; with p.cpx, column n of op(B) is its column 2 n).
    const int klo = max((p.ktri & 1) ? (p.cpx ? 2 * n0 : n0) : 0, (p.ktri & 2) ? m0 : 0);
    const int c0 = min(klo / BK, nch);
    typedef std::integral_constant<int, 0> Slot0;
    typedef std::integral_constant<int, PF - 1> SlotL;
    if (c0 < nch) {
        if constexpr (GA) cload(c0);
        gload(c0, Slot0{});
        if constexpr (PF == 2) {
            if (c0 + 1 < nch) gload(c0 + 1, SlotL{});
        }
        sstore(c0 & 1, c0, Slot0{});
    }
    __syncthreads();
    if constexpr (PF == 1) {
        for (int c = c0; c < nch; c++) {
            const int buf = c & 1;
            const bool more = c + 1 < nch;
            if (more) gload(c + 1, Slot0{});
            compute(buf);
            if (more) sstore(buf ^ 1, c + 1, Slot0{});
            __syncthreads();
        }
    } else {
        // chunk c0 + i waits in slot i & 1 from its load until its LDS stage;
        // step c refills the slot of chunk c (staged one step earlier) with
        // chunk c + 2 and stages chunk c + 1 (loaded one step earlier)
        auto step = [&](int c, auto S_) {
            constexpr int S = decltype(S_)::value;
            if (c + 2 < nch) gload(c + 2, S_);
            compute(c & 1);
            if (c + 1 < nch) sstore((c + 1) & 1, c + 1, std::integral_constant<int, 1 - S>{});
            __syncthreads();
        };
        for (int c = c0; c < nch; c += 2) {
            step(c, Slot0{});
            if (c + 1 < nch) step(c + 1, SlotL{});
        }
    }

    SELINV_GLOBAL TC *__restrict__ C = gptr_w((TC *)p.C);
    const SELINV_GLOBAL TC *__restrict__ Cin = gptr((const TC *)p.Cin);
    const int64_t ldc = p.ldc, ldcin = p.ldcin;
    const double alpha = p.alpha, beta = p.beta;
    // rows of the 16x16 result held by this lane: v_mfma_f64_16x16x4
    // interleaves the four row groups (row = lane/16 + 4v); the f32 and bf16
    // forms keep them contiguous (row = 4 (lane/16) + v)
    auto row_n = [&](int j, int v) {
        const int nr = (MODE == CMP_F64) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
        return n0 + wn * WN + j * 16 + nr;
    };
    const bool has_cin = CIN && p.Cin != nullptr;
    // The Cin loads of CR rows of 16x16 tiles in flight together (clamped
    // addresses): every row of the wavefront's tiles up to 16 values per lane
    // (Cin is C itself in step 4, so later loads cannot pass the stores)
    constexpr int CR = TM * TN <= 4 ? TM : 1;
#pragma unroll
    for (int i0 = 0; i0 < TM; i0 += CR) {
        double cin[CR][TN][4];
        if (has_cin) {
#pragma unroll
            for (int ii = 0; ii < CR; ii++)
#pragma unroll
                for (int j = 0; j < TN; j++)
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int64_t gm = min(m0 + wm * WM + (i0 + ii) * 16 + (lane & 15), M - 1);
                        const int64_t gn = min(row_n(j, v), N - 1);
                        cin[ii][j][v] = (double)Cin[gm + gn * ldcin];
                    }
        }
#pragma unroll
        for (int ii = 0; ii < CR; ii++) {
            const int i = i0 + ii;
            const int gm = m0 + wm * WM + i * 16 + (lane & 15);
            if (gm >= M) continue;
            // complex blocks: the entry of the odd column that this one gives
            const double csign = (gm & 1) ? -1.0 : 1.0;
#pragma unroll
            for (int j = 0; j < TN; j++)
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int gn = row_n(j, v);
                    if (gn >= N) continue;
                    double r = alpha * (double)acc[i][j][v];
                    if (has_cin) r += beta * cin[ii][j][v];
                    C[gm + (int64_t)gn * ldc] = (TC)r;
                    if (p.cpx) C[(gm ^ 1) + (int64_t)gn * ldc + ldc / 2] = (TC)(csign * r);
                    if constexpr (PUSH) acc[i][j][v] = (TC)r;  // the stored value, for the push below
                }
        }
    }
    if constexpr (PUSH) {
        if (p.push_sn >= 0) {
            const MatDev &Md = mats[p.push_mat];
            const SELINV_GLOBAL SnRec *sn = gptr(Md.sn);
            const SELINV_GLOBAL int32_t *kp = gptr(Md.kids_ptr);
            const SELINV_GLOBAL int32_t *kids = gptr(Md.kids);
            const int P = p.push_sn, sP = M;  // A^{-T}(P,P) is M x M
            const int q1 = kp[P + 1];
            for (int q = kp[P]; q < q1; q++) {
                const int32_t K = kids[q];
                const SELINV_GLOBAL int32_t *posL = gptr(Md.push_pos) + gptr(Md.push_off)[K];
                const SELINV_GLOBAL int32_t *posU = posL + sP;
                const int64_t clK = sn[K].cl;
                SELINV_GLOBAL TG *G = gptr_w((TG *)Md.G) + sn[K].g_off;
#pragma unroll
                for (int i = 0; i < TM; i++) {
                    const int gm = m0 + wm * WM + i * 16 + (lane & 15);
                    if (gm >= M) continue;
                    const int a = posL[gm];
                    // complex blocks: column gn of the problem is column 2 gn
                    // of A^{-T}(P,P), and it gives entry (gm ^ 1, 2 gn + 1)
                    const int a1 = p.cpx ? posL[gm ^ 1] : -1;
                    const TG csign = (gm & 1) ? (TG)-1 : (TG)1;
#pragma unroll
                    for (int j = 0; j < TN; j++)
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int gn = row_n(j, v);
                            if (gn >= N) continue;
                            const int c = p.cpx ? 2 * gn : gn;
                            const int b = posU[c];
                            if (a >= 0 && b >= 0) G[a + b * clK] = (TG)acc[i][j][v];
                            if (p.cpx) {
                                const int b1 = posU[c + 1];
                                if (a1 >= 0 && b1 >= 0) G[a1 + b1 * clK] = csign * (TG)acc[i][j][v];
                            }
                        }
                }
            }
        }
    }
}

// Dispatch on the operand forms of the problem (uniform across the
// workgroup).
template <int MODE, int BM, int BN, typename TA, typename TC, bool CIN, bool PUSH = false,
          int BK = ChunkK<MODE, BM>::value>
__device__ __forceinline__ void gemm_tile(const GemmProb &p, const int m0, const int n0,
                                          Smem<MODE, BM, BN, BK> &sm, const MatDev *mats = nullptr) {
    typedef typename Mode<MODE>::T TG;
    if (p.opA == 0) {
        if (p.opB == 0)
            gemm_tile_op<MODE, BM, BN, TA, TC, CIN, BK, 0, 0, PUSH, TG>(p, m0, n0, sm, mats);
        else
            gemm_tile_op<MODE, BM, BN, TA, TC, CIN, BK, 0, 1, PUSH, TG>(p, m0, n0, sm, mats);
    } else {
        if (p.opB == 0)
            gemm_tile_op<MODE, BM, BN, TA, TC, CIN, BK, 1, 0, PUSH, TG>(p, m0, n0, sm, mats);
        else
            gemm_tile_op<MODE, BM, BN, TA, TC, CIN, BK, 1, 1, PUSH, TG>(p, m0, n0, sm, mats);
    }
}

// A step-3 (op(A) = G_K^T) or step-5 (op(A) = G_K) product tile with G_K
// taken from its sources through its codes; op(B) = B, results in TA.
template <int MODE, int BM, int BN, typename TA, int BK = ChunkK<MODE, BM>::value>
__device__ __forceinline__ void gemm_tile_g35(const GemmProb &p, const int m0, const int n0,
                                              Smem<MODE, BM, BN, BK> &sm, const MatDev *mats) {
    if (p.opA == 0)
        gemm_tile_op<MODE, BM, BN, TA, TA, false, BK, 0, 0, false, TA, true>(p, m0, n0, sm, mats);
    else
        gemm_tile_op<MODE, BM, BN, TA, TA, false, BK, 1, 0, false, TA, true>(p, m0, n0, sm, mats);
}

// LDS of one gather tile
template <typename T>
struct GatherSmem {
    T tileS[64][65];  // [b][a]
    int32_t rowR[64], rowI[64], colJ[64];
    int64_t rowUp[64], rowUoff[64], colDiag[64], colLow[64], colLoff[64];
    uint32_t sides;  // map path: bit 0 the tile has diagonal-block or L-side entries, bit 1 U-side ones
};

// Gather tile descriptor of supernode K of matrix `mat` from its record.
__device__ __forceinline__ GatherTile gather_desc(const MatDev &M, int mat, int K, int a0, int b0) {
    const SELINV_GLOBAL SnRec *sn = gptr(M.sn);
    GatherTile gt;
    gt.mat = mat;
    gt.K = K;
    gt.a0 = a0;
    gt.b0 = b0;
    gt.skip = -1;
    gt.cl = sn[K].cl;
    gt.cu = sn[K].cu;
    gt.pad = 0;
    gt.g_off = sn[K].g_off;
    gt.c_off = sn[K].c_off;
    gt.skip_lo = gt.skip_hi = 0;
    gt.rl_off = sn[K].rl_off;
    gt.ru_off = sn[K].ru_off;
    return gt;
}

// Tile of G_K from the precomputed source codes: every thread loads the codes
// of its entries (they do not depend on earlier launches), then the values
// they name, in two rounds of 2 x 8 entries (the register budget of the GEMM
// kernels that share this code stays unchanged).  Diagonal-block and L-side
// entries are read with the threads along the rows of G (contiguous in ZL),
// U-side entries with the threads along its columns (contiguous in ZU).
template <typename T, bool STORE>
__device__ __forceinline__ void gather_tile_codes(const MatDev &M, const GatherTile &gt, GatherSmem<T> &sm) {
    T(&tileS)[64][65] = sm.tileS;
    constexpr int CH = 8;
    const int tid = threadIdx.x;
    const int a0 = gt.a0, b0 = gt.b0, cl = gt.cl, cu = gt.cu;
    const int na = min(64, cl - a0), nb = min(64, cu - b0);
    const SELINV_GLOBAL uint32_t *cL = gptr(M.gcL) + gt.c_off;
    const SELINV_GLOBAL uint32_t *cU = gptr(M.gcU) + gt.c_off;
    const SELINV_GLOBAL T *ZL = gptr((const T *)M.ZL);
    const SELINV_GLOBAL T *ZU = gptr((const T *)M.ZU);
    const SELINV_GLOBAL double *Zd = gptr(M.Zd);
    uint32_t keep = 0;  // bit t: entry tid + 256 t of the tile is written to G
#pragma unroll
    for (int h = 0; h < 2; h++) {
        uint32_t kl[CH], ku[CH];
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const int e = tid + 256 * (h * CH + t), ia = e & 63, ib = e >> 6;
            kl[t] = cL[(ia < na && ib < nb) ? (a0 + ia) + (int64_t)(b0 + ib) * cl : 0];
            const int jb = e & 63, ja = e >> 6;
            ku[t] = cU[(ja < na && jb < nb) ? (b0 + jb) + (int64_t)(a0 + ja) * cu : 0];
        }
        T vl[CH], vu[CH];
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const uint32_t k = kl[t] >> GCODE_SHIFT, off = kl[t] & GCODE_MASK;
            if constexpr (sizeof(T) == sizeof(double)) {
                // one load: the diagonal blocks and the L panels hold the same type
                vl[t] = (k == 1 ? (const SELINV_GLOBAL T *)Zd : ZL)[k >= 1 && k <= 2 ? off : 0];
            } else {
                const double vd = Zd[k == 1 ? off : 0];
                const T v = ZL[k == 2 ? off : 0];
                vl[t] = k == 1 ? (T)vd : v;
            }
            const uint32_t k3 = ku[t] >> GCODE_SHIFT, off3 = ku[t] & GCODE_MASK;
            vu[t] = ZU[k3 == 3 ? off3 : 0];
        }
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const int e = tid + 256 * (h * CH + t), ia = e & 63, ib = e >> 6;
            const uint32_t k = kl[t] >> GCODE_SHIFT, off = kl[t] & GCODE_MASK;
            // (a code of an entry outside the tile is that of entry 0, and its
            // value is dropped here; entries of the skipped diagonal block are
            // written by their owner)
            const bool in = ia < na && ib < nb;
            const bool skipped = k == 1 && (int64_t)off >= gt.skip_lo && (int64_t)off < gt.skip_hi;
            if (in && !skipped) keep |= 1u << (h * CH + t);
            if (in && (k == 2 || (k == 1 && !skipped))) tileS[ib][ia] = vl[t];
            const int jb = e & 63, ja = e >> 6;
            if (ja < na && jb < nb && (ku[t] >> GCODE_SHIFT) == 3) tileS[jb][ja] = vu[t];
        }
    }
    __syncthreads();
    if constexpr (!STORE) return;
    SELINV_GLOBAL T *G = gptr_w((T *)M.G + gt.g_off);
#pragma unroll
    for (int t = 0; t < 2 * CH; t++) {
        const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
        if (keep >> t & 1) G[(a0 + ia) + (int64_t)(b0 + ib) * cl] = tileS[ib][ia];
    }
}

// One 64x64 tile (rows a0.., columns b0..) of G_K = A^{-T}(R_L(K), R_U(K)),
// gathered by the 256 threads of the calling workgroup (see kernels.hip).
// Every load goes through a global-memory view and is issued unconditionally
// (clamped to a valid index, the unused value discarded), so that a thread's
// loads of one stage are all in flight together.  With precomputed codes
// (gt.c_off >= 0) the codes name the sources; otherwise the relative-index
// maps do.
// STORE = false leaves the tile in LDS only (sm.tileS[b][a] = G(a0+a, b0+b)).
template <typename T, bool STORE = true>
__device__ __forceinline__ void gather_tile(const MatDev &M, const GatherTile &gt, GatherSmem<T> &sm) {
    if (gt.c_off >= 0) {
        gather_tile_codes<T, STORE>(M, gt, sm);
        return;
    }
    const int a0 = gt.a0, b0 = gt.b0, skip = gt.skip;
    T(&tileS)[64][65] = sm.tileS;
    int32_t *rowR = sm.rowR, *rowI = sm.rowI, *colJ = sm.colJ;
    int64_t *rowUp = sm.rowUp, *rowUoff = sm.rowUoff, *colDiag = sm.colDiag, *colLow = sm.colLow,
            *colLoff = sm.colLoff;
    const int32_t sk_cl = gt.cl, sk_cu = gt.cu;
    const int64_t sk_g_off = gt.g_off;
    const int tid = threadIdx.x;
    const int na = min(64, sk_cl - a0), nb = min(64, sk_cu - b0);  // both >= 1
    // the tile's row and column records: independent loads (one round trip)
    if (tid == 0) sm.sides = 0;
    if (tid < 64) {
        const int t = min(tid, na - 1);
        const int64_t a = gt.rl_off + a0 + t;
        const int32_t r = gptr(M.rl)[a], I = gptr(M.row_I)[a];
        const int64_t uo = gptr(M.u_rowoff)[a], up = gptr(M.row_up)[a];
        if (tid < na) {
            rowR[tid] = r;
            rowI[tid] = I;
            rowUp[tid] = up;
            rowUoff[tid] = uo + b0;
        }
    } else if (tid < 128) {
        const int t = min(tid - 64, nb - 1);
        const int64_t b = gt.ru_off + b0 + t;
        const int32_t J = gptr(M.col_J)[b];
        const int64_t lo = gptr(M.l_coloff)[b], cd = gptr(M.col_diag)[b], cw = gptr(M.col_low)[b];
        if (tid - 64 < nb) {
            colJ[t] = J;
            colDiag[t] = cd;
            colLow[t] = cw;
            colLoff[t] = lo + a0;
        }
    }
    __syncthreads();
    const SELINV_GLOBAL T *ZL = gptr((const T *)M.ZL);
    const SELINV_GLOBAL T *ZU = gptr((const T *)M.ZU);
    const SELINV_GLOBAL double *Zd = gptr(M.Zd);
    const SELINV_GLOBAL int32_t *mapL = gptr(M.mapL);
    const SELINV_GLOBAL int32_t *mapU = gptr(M.mapU);
    // Each thread owns 16 entries of the tile on each side: diagonal-block and
    // L-side sources with the threads along the rows of G (contiguous in
    // ZL), U-side sources with the threads along its columns (contiguous in
    // ZU).  Both sides' relative positions are read together, then both
    // sides' values: two memory round trips.  Entries outside the tile or of
    // another kind read element 0 of the array instead (every device array
    // holds at least one element) and discard it, so that no load sits
    // behind a branch.
    constexpr int PER = 64 * 64 / 256;
    {
        int kind[PER];  // L side (threads along a): 1 diagonal block, 2 L panel, 0 none
        bool up[PER];   // U side (threads along b)
        bool anyL = false, anyU = false;
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t;
            const int ia = e & 63, ib = e >> 6;
            kind[t] = 0;
            if (ia < na && ib < nb) {
                const int32_t I = rowI[ia], J = colJ[ib];
                kind[t] = I == J ? (I == skip ? 0 : 1) : (I > J ? 2 : 0);
            }
            const int ub = e & 63, ua = e >> 6;
            up[t] = ua < na && ub < nb && rowI[ua] < colJ[ub];
            anyL = anyL || kind[t] != 0;
            anyU = anyU || up[t];
        }
        // Most tiles lie on one side of the ancestors' block diagonal: the
        // loads of a side without entries in the tile are not issued at all
        // (uniform over the workgroup, one barrier).
        {
            const uint32_t mine = (__any(anyL) ? 1u : 0u) | (__any(anyU) ? 2u : 0u);
            if ((tid & 63) == 0 && mine) atomicOr(&sm.sides, mine);
        }
        __syncthreads();
        const uint32_t sides = sm.sides;
        T vl[PER], vu[PER];
        // DL / DU: the loads of that side are issued (a separate code path per
        // combination, so that the two-sided one keeps its registers)
        auto side_loads = [&](auto DL_, auto DU_) {
            constexpr bool DL = decltype(DL_)::value, DU = decltype(DU_)::value;
            int32_t ml[PER], mu[PER];
#pragma unroll
            for (int t = 0; t < PER; t++) {
                const int e = tid + 256 * t;
                if constexpr (DL) ml[t] = mapL[kind[t] == 2 ? colLoff[e >> 6] + (e & 63) : 0];
                if constexpr (DU) mu[t] = mapU[up[t] ? rowUoff[e >> 6] + (e & 63) : 0];
            }
#pragma unroll
            for (int t = 0; t < PER; t++) {
                const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
                if constexpr (DL) {
                    if constexpr (sizeof(T) == sizeof(double)) {
                        // one load: the diagonal blocks and the L panels hold the same type
                        const int64_t i =
                            kind[t] == 1 ? colDiag[ib] + rowR[ia] : kind[t] == 2 ? colLow[ib] + ml[t] : 0;
                        vl[t] = (kind[t] == 1 ? (const SELINV_GLOBAL T *)Zd : ZL)[i];
                    } else {
                        const double vd = Zd[kind[t] == 1 ? colDiag[ib] + rowR[ia] : 0];
                        const T v = ZL[kind[t] == 2 ? colLow[ib] + ml[t] : 0];
                        vl[t] = kind[t] == 1 ? (T)vd : v;
                    }
                }
                if constexpr (DU) vu[t] = ZU[up[t] ? rowUp[e >> 6] + mu[t] : 0];
            }
        };
        if (sides == 3)
            side_loads(std::true_type{}, std::true_type{});
        else if (sides == 1)
            side_loads(std::true_type{}, std::false_type{});
        else if (sides == 2)
            side_loads(std::false_type{}, std::true_type{});
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t;
            if (kind[t]) tileS[e >> 6][e & 63] = vl[t];
            if (up[t]) tileS[e & 63][e >> 6] = vu[t];
        }
    }
    __syncthreads();
    if constexpr (!STORE) return;
    SELINV_GLOBAL T *G = gptr_w((T *)M.G + sk_g_off);
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ia = e & 63, ib = e >> 6;
        // entries of the skipped diagonal block are written by its owner
        if (ia < na && ib < nb && !(rowI[ia] == skip && colJ[ib] == skip))
            G[(a0 + ia) + (int64_t)(b0 + ib) * sk_cl] = tileS[ib][ia];
    }
}

}  // namespace selinv

// Pivot blocks of block Gaussian elimination with no pivoting.
//
// Section 3 of the paper factors A = [[B, C], [D, E]] as in eq. eqgenp and
// recurses on the pivot block B and on the Schur complement S = E - D B^{-1} C;
// with pivot blocks of size 1 this is GENP, and by the order-independence
// argument after eq. eqgenpin every choice of block sizes produces the same
// Schur complements.  The host driver (api.hip) walks the matrix in panels of
// `block` columns.  This file holds
//   * k_leaf_genp: one pivot block of at most 128 x 128 factored with no
//     pivoting by one workgroup, the block in LDS, in panels of 16 columns;
//   * k_leaf_lu: the same with partial pivoting inside the block (the block
//     held in registers, pivot by pivot);
//   * k_diag_inv: the inverses of the 32 x 32 diagonal sub-blocks of the two
//     triangular factors of a factored block;
//   * k_trsm_pair: the off-diagonal blocks of eq. eqgenp,
//     L_B^{-1} C and D U_B^{-1} (their product is D B^{-1} C), each done in
//     place by blocked substitution on the matrix cores: the 32 x 32 diagonal
//     sub-blocks are applied through their inverses, the rest as plain
//     updates.  Only small blocks are inverted, so the error grows with the
//     condition of 32 x 32 blocks, not of the whole pivot block.
//
// Breakdown: a pivot that is exactly 0 (Corollary corec: the input is not
// strongly nonsingular) or not finite stops the elimination; its global index
// is recorded in the device status word and every later kernel exits early.
//
// Bound: the leaves are latency bound (b sequential pivot steps); the solves
// are MFMA work of b^2 / 2 multiply-adds per strip column, with b / 32
// dependent sub-block steps per strip.
#include "mfma.h"
#include "rmge_impl.h"

namespace rmge {
namespace {

constexpr int kSub = 32;  // diagonal sub-blocks that are inverted explicitly

template <typename T>
__device__ inline bool is_bad(T p) {
    return p == T(0) || !isfinite(p);
}

// One pivot block (b <= 128) in registers, 512 threads: each wave holds 16
// columns and lane l holds rows l and l + 64 of them (32 elements a thread).
// A column therefore lives inside one wave, and every wave holds every row.
// Pivot step j:
//   * every wave waits only for the flag of column j (no barrier: waves may
//     run steps behind), reads the column and the reciprocal of its pivot, and
//     takes the pivot row's values for its own columns from lane (row mod 64)
//     with readlane;
//   * each thread applies a_ic -= (a_ij / a_pj) a_pc to its elements, the
//     multiplier formed as a_ij times the reciprocal of the pivot;
//   * the owner of column j + 1 publishes that column (with PIV, electing its
//     pivot by a DPP reduction and ballots inside the wave).
// With pivoting the columns are dealt cyclically (wave w holds w, w + 8, ...,
// w + 120), so consecutive columns belong to different waves, and the owner
// of column j + 1 applies step j to that column first and publishes it before
// updating the rest: the chain from one pivot to the next is one column's
// update and one election.  Without pivoting (no election on the chain)
// wave w holds the block 16 w .. 16 w + 15 and publishes after its update.
// Multipliers of retired rows and pivot-row entries of columns <= j are zero,
// so the update is branch-free and an element left of its row's pivot keeps
// the value it had when its column was eliminated; the multipliers
// l_ic = a_ic / a_cc are formed at write-back from the recorded reciprocals.
//
// PIV = false: GENP, the pivot of step j is row j.
// PIV = true: partial pivoting inside this block (the black-box treatment of a
// small pivot block that Section 3 allows once the recursion of eq. eqgenp
// stops): the pivot of step j is the active row with the largest |a_ij|
// (ties: the lower row index).  Rows stay in their registers; row i is written
// back to position pos[i] (the step that retired it), and
// piv[k0 + pos[i]] = k0 + i records the exchange.
constexpr int kLeafThreads = 512;

template <typename T>
__device__ inline T lane_value(T v, int src);
template <>
__device__ inline float lane_value<float>(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
template <>
__device__ inline double lane_value<double>(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), src);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<unsigned int>(lo)));
}

// Maximum of an unsigned value over the 64 lanes of a wave by DPP moves
// (register to register: quad permutations, row mirrors, row broadcasts), the
// result read from lane 63.  Lanes a move does not write read 0, the identity
// of max, which lets each move fold into its max instruction.
__device__ inline unsigned dpp_max_step(unsigned v, unsigned moved) { return max(v, moved); }
#define RMGE_DPP_MAX(v, ctrl, rows)                                                       \
    v = dpp_max_step(v, static_cast<unsigned>(__builtin_amdgcn_update_dpp(               \
                            0, static_cast<int>(v), ctrl, rows, 0xf, false)))
__device__ inline unsigned wave_max_u32(unsigned v) {
    RMGE_DPP_MAX(v, 0xB1, 0xf);   // quad_perm [1,0,3,2]
    RMGE_DPP_MAX(v, 0x4E, 0xf);   // quad_perm [2,3,0,1]
    RMGE_DPP_MAX(v, 0x141, 0xf);  // row_half_mirror
    RMGE_DPP_MAX(v, 0x140, 0xf);  // row_mirror
    RMGE_DPP_MAX(v, 0x142, 0xa);  // row_bcast:15
    RMGE_DPP_MAX(v, 0x143, 0xc);  // row_bcast:31
    return static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}
#undef RMGE_DPP_MAX

// Pivot election inside the owner wave over the two rows each lane holds
// (rows l and l + 64): the winner is the active row of largest |value|, ties
// going to the lower row index; a NaN outranks every number, and every active
// row outranks a retired one.  Keys: |value|'s bit pattern with the top bit
// set for active rows, 0 for retired ones (FP32: one 32-bit word; FP64: the
// high word decides and the low word breaks its ties).
template <typename T>
__device__ inline int elect_pivot(T x0, T x1, unsigned act);
template <>
__device__ inline int elect_pivot<float>(float x0, float x1, unsigned act) {
    const unsigned k0 = (act & 1u) ? ((__float_as_uint(x0) & 0x7fffffffu) | 0x80000000u) : 0u;
    const unsigned k1 = (act & 2u) ? ((__float_as_uint(x1) & 0x7fffffffu) | 0x80000000u) : 0u;
    const unsigned m = wave_max_u32(max(k0, k1));
    const unsigned long long b0 = __ballot(k0 == m), b1 = __ballot(k1 == m);
    return b0 ? __builtin_ffsll(static_cast<long long>(b0)) - 1
              : 64 + __builtin_ffsll(static_cast<long long>(b1)) - 1;
}
template <>
__device__ inline int elect_pivot<double>(double x0, double x1, unsigned act) {
    const unsigned long long mag = 0x7fffffffffffffffull, top = 0x8000000000000000ull;
    const unsigned long long k0 =
        (act & 1u) ? ((static_cast<unsigned long long>(__double_as_longlong(x0)) & mag) | top) : 0ull;
    const unsigned long long k1 =
        (act & 2u) ? ((static_cast<unsigned long long>(__double_as_longlong(x1)) & mag) | top) : 0ull;
    const unsigned long long kb = k0 > k1 ? k0 : k1;
    const unsigned hi = wave_max_u32(static_cast<unsigned>(kb >> 32));
    const unsigned lo = wave_max_u32(static_cast<unsigned>(kb >> 32) == hi ? static_cast<unsigned>(kb) : 0u);
    const unsigned long long m = (static_cast<unsigned long long>(hi) << 32) | lo;
    const unsigned long long b0 = __ballot(k0 == m), b1 = __ballot(k1 == m);
    return b0 ? __builtin_ffsll(static_cast<long long>(b0)) - 1
              : 64 + __builtin_ffsll(static_cast<long long>(b1)) - 1;
}

// Column of register q in wave w, and the wave that owns column c: cyclic
// (c = 8 q + w) with pivoting, blocks of 16 (c = 16 w + q) without.
template <bool CYCLIC>
__device__ inline int leaf_col(int w, int q) { return CYCLIC ? 8 * q + w : 16 * w + q; }
template <bool CYCLIC>
__device__ inline int leaf_owner(int c) { return CYCLIC ? (c & 7) : (c >> 4); }

template <typename T, bool PIV>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_lu(T *a, int64_t lda, int b, int64_t k0,
                                                          DevStatus *st, int *piv) {
    // Column j is published once, into its own slot: no slot is reused, so a
    // wave may run any number of steps behind the owners without a barrier.
    __shared__ T colv[kLeaf][kLeaf];
    __shared__ int flag[kLeaf];  // 0: not yet; 1 + pivot row: published; -(1 + row): breakdown
    __shared__ T rcp[kLeaf];     // reciprocal of step j's pivot
    __shared__ int pos[kLeaf];
    __shared__ int s_fail;
    if (st->code != 0) return;  // an earlier pivot block broke down
    // This kernel is a chain of short dependent steps that may run beside the
    // wide Schur-update GEMM; raise its waves' issue priority on shared SIMDs.
    __builtin_amdgcn_s_setprio(3);
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    if (tid < kLeaf) {
        flag[tid] = 0;
        pos[tid] = -1;
    }
    if (tid == 0) s_fail = 0;
    T v[2][16];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = l + 64 * p, c = leaf_col<PIV>(w, q);
            v[p][q] = (i < b && c < b) ? a[static_cast<int64_t>(i) * lda + c] : T(0);
        }
    unsigned act = 0;  // bit p: row l + 64 p is still active (PIV)
#pragma unroll
    for (int p = 0; p < 2; ++p)
        if (l + 64 * p < b) act |= 1u << p;
    // Let the block's loads land here.  (A wave whose columns the loop never
    // updates reaches the write-back with them still outstanding as far as
    // the compiler can tell, and it would then wait for all memory traffic,
    // its own stores included, before every store of the write-back.)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // The owner of column j publishes it once step j - 1 has reached it: the
    // column, the pivot's reciprocal and position, then (after a release
    // fence) the flag carrying the pivot row, negative if the pivot is zero or
    // not finite (the breakdown is recorded here).  The owner keeps what it
    // published for its own next step.
    T pub0 = T(0), pub1 = T(0), pub_rp = T(0);
    int pub_fv = 0;
    auto publish = [&](int j, T x0, T x1) {
        colv[j][l] = x0;
        colv[j][l + 64] = x1;
        const int sel = PIV ? elect_pivot<T>(x0, x1, act) : j;
        const T pv = lane_value<T>((sel >> 6) ? x1 : x0, sel & 63);
        const bool ok = !is_bad(pv);
        const T rp = ok ? T(1) / pv : T(0);
        if (l == 0) {
            if (ok) {
                rcp[j] = rp;
                if (PIV) pos[sel] = j;
            } else {
                st->info = k0 + j;
                st->code = (pv == T(0)) ? 4 : 5;
            }
        }
        pub0 = x0;
        pub1 = x1;
        pub_rp = rp;
        pub_fv = ok ? 1 + sel : -(1 + sel);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (l == 0) __hip_atomic_store(&flag[j], pub_fv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // Wait for column j (bounded: a wave that gives up records an error) and
    // return its flag, or 0.
    auto await_column = [&](int j) {
        int fv = 0, spins = 0;
        while ((fv = __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                    &flag[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))) == 0) {
            if (++spins > (1 << 24)) break;
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        return fv;
    };

    bool mine = false;  // this wave published column j and holds it in registers
    if (w == 0 && b > 0) {
        publish(0, v[0][0], v[1][0]);
        mine = true;
    }
    int done = b, j = 0;
    // Steps that change this wave's columns: j < its last column.  A failed
    // step still runs its (then empty) update and leaves after it, so the loop
    // has a single exit and the columns are updated in place.
    const int jw = min(b, leaf_col<PIV>(w, 15));
    for (; j < jw; ++j) {
        // with pivoting, the wave that publishes the next column (and elects
        // its pivot) is the chain: let it issue first on its SIMD; the other
        // waves keep a priority above a GEMM's.  (Measured: slower without
        // pivoting, where all waves keep the kernel's raised priority.)
        const bool next = j + 1 < b && leaf_owner<PIV>(j + 1) == w;
        if (PIV) {
            if (next)
                __builtin_amdgcn_s_setprio(3);
            else
                __builtin_amdgcn_s_setprio(1);
        }
        int fv;
        T c0, c1, rp;
        if (mine) {
            fv = pub_fv;
            c0 = pub0;
            c1 = pub1;
            rp = pub_rp;
        } else {
            fv = await_column(j);
            c0 = colv[j][l];
            c1 = colv[j][l + 64];
            rp = rcp[j];
        }
        const bool ok = fv > 0;
        if (!ok) {
            if (fv == 0 && l == 0) s_fail = 1;  // never published (cannot happen unless the schedule is broken)
            done = j;
        }
        const int sel = (fv > 0 ? fv : -fv) - 1, sl = sel & 63, sp = sel >> 6;
        if (PIV && ok && l == sl) act &= ~(1u << sp);
        const bool live0 = PIV ? (act & 1u) != 0 : l > j;
        const bool live1 = PIV ? (act & 2u) != 0 : l + 64 > j;
        const T m0 = (ok && live0) ? c0 * rp : T(0), m1 = (ok && live1) ? c1 * rp : T(0);
        if (PIV && ok && next) {
            // with pivoting, column j + 1 is updated first and published
            // before the rest of the update.  It sits in register (j + 1) / 8,
            // a uniform index: one case runs, with static register numbers
            // (the empty asm keeps each case a plain register read rather
            // than an indexed load)
            T x0 = T(0), x1 = T(0);
            switch ((j + 1) >> 3) {
#define RMGE_COL(Q)                                        \
    case Q: {                                              \
        x0 = v[0][Q];                                      \
        x1 = v[1][Q];                                      \
        asm volatile("" : "+v"(x0), "+v"(x1));             \
        const T uq = lane_value<T>(sp ? x1 : x0, sl);      \
        x0 -= m0 * uq;                                     \
        x1 -= m1 * uq;                                     \
        break;                                             \
    }
                RMGE_COL(0) RMGE_COL(1) RMGE_COL(2) RMGE_COL(3) RMGE_COL(4) RMGE_COL(5)
                RMGE_COL(6) RMGE_COL(7) RMGE_COL(8) RMGE_COL(9) RMGE_COL(10) RMGE_COL(11)
                RMGE_COL(12) RMGE_COL(13) RMGE_COL(14) RMGE_COL(15)
#undef RMGE_COL
            }
            publish(j + 1, x0, x1);
        }
        // the pivot row's entries of this wave's columns (wave-uniform values).
        // Columns <= j are final in their LDS slots, so their registers take
        // the update too and are never read again; column j + 1 gets exactly
        // the values just published.
        T u[16];
        if (sp) {
#pragma unroll
            for (int q = 0; q < 16; ++q) u[q] = lane_value<T>(v[1][q], sl);
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) u[q] = lane_value<T>(v[0][q], sl);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            v[0][q] -= m0 * u[q];
            v[1][q] -= m1 * u[q];
        }
        if (!ok) break;
        if (!PIV && next) {
            // without pivoting, column j + 1 is published after the full
            // update (its owner is mostly the owner of column j as well)
            T x0 = T(0), x1 = T(0);
            switch ((j + 1) & 15) {
#define RMGE_COL(Q)                            \
    case Q:                                    \
        x0 = v[0][Q];                          \
        x1 = v[1][Q];                          \
        asm volatile("" : "+v"(x0), "+v"(x1)); \
        break;
                RMGE_COL(0) RMGE_COL(1) RMGE_COL(2) RMGE_COL(3) RMGE_COL(4) RMGE_COL(5)
                RMGE_COL(6) RMGE_COL(7) RMGE_COL(8) RMGE_COL(9) RMGE_COL(10) RMGE_COL(11)
                RMGE_COL(12) RMGE_COL(13) RMGE_COL(14) RMGE_COL(15)
#undef RMGE_COL
            }
            publish(j + 1, x0, x1);
        }
        mine = next;
    }
    // The remaining steps leave this wave's columns alone: follow the flags
    // and stop where the others stop.
    if (PIV) __builtin_amdgcn_s_setprio(1);
    if (done == b) {
        for (; j < b; ++j) {
            const int fv = await_column(j);
            if (fv <= 0) {
                if (fv == 0 && l == 0) s_fail = 1;
                done = j;
                break;
            }
        }
    }
    __syncthreads();
    if (s_fail && tid == 0) st->code = 3;  // reported as a device error
    if (PIV) {
        if (done < b && tid == 0) {  // breakdown: keep the row order a permutation
            int next = done;
            for (int i = 0; i < b; ++i)
                if (pos[i] < 0) pos[i] = next++;
        }
        __syncthreads();
        if (tid < b) piv[k0 + pos[tid]] = static_cast<int>(k0 + tid);
    }
    // write back (row i to its position), forming the multipliers left of the
    // pivot.  A column eliminated before the stop is taken from its LDS slot,
    // which holds its final values; later columns from the registers.
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int i = l + 64 * p;
        if (i >= b) continue;
        const int dst = PIV ? pos[i] : i;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = leaf_col<PIV>(w, q);
            if (c >= b) continue;
            T val = c < done ? colv[c][i] : v[p][q];
            if (c < dst && c < done) val *= rcp[c];
            a[static_cast<int64_t>(dst) * lda + c] = val;
        }
    }
}

// Reciprocal of a pivot: the hardware estimate refined by Newton steps (two
// for FP64, one for FP32), within an ulp or two of 1 / p.  Its dependent
// chain is about half that of the IEEE division sequence, and it sits on
// the critical path of every pivot step below.
__device__ inline double pivot_recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    double e = __builtin_fma(-p, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-p, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ inline float pivot_recip(float p) {
    const float r = __builtin_amdgcn_rcpf(p);
    return __builtin_fmaf(r, __builtin_fmaf(-p, r, 1.0f), r);
}

// One wave's share of a 16-column panel of the LDS-resident pivot block
// (rows c0 .. b - 1, columns c0 .. c0 + 15; eq. eqgenp with pivot blocks of 1).
// Lanes 0..15 hold the panel's 16 pivot rows, lanes 16..63 the rows
// c0 + 16 + 48 pw + (lane - 16) below them: every panel wave eliminates the
// pivot rows itself, so no pivot row crosses between waves.  Pivot step j
// reads the pivot row's entries from lane j (readlane), updates the next
// pivot column first and starts that pivot's reciprocal before the rest of
// the step's updates.  Multipliers are a_ij * (1 / a_jj).  A zero or
// non-finite pivot is only recorded (bits of `bad`, `zero`); the block is
// abandoned after the panel, and wave 0 (pw == 0), which also writes the
// pivot rows, writes the first such pivot's global index to the status word.
template <typename T>
__device__ __attribute__((always_inline)) inline void leaf_panel(T *S, int b, int c0, int lane,
                                                                 int pw, DevStatus *st, int64_t k0,
                                                                 int *s_fail) {
    constexpr int LD = kLeaf + 1;
    int w = min(16, b - c0);
    // Opaque to the optimiser at each call: the per-step lane masks are then
    // formed inside the panel rather than hoisted out of the panel loop and
    // held across it in scalar registers (which spills them).
    asm volatile("" : "+v"(lane));
    asm volatile("" : "+s"(w));
    const int row = lane < 16 ? c0 + lane : c0 + 16 + 48 * pw + (lane - 16);
    const bool valid = row < b;
    T x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = (valid && k < w) ? S[row * LD + c0 + k] : T(0);
    // steps past the panel's width see zero columns and change nothing
    unsigned bad = 0, zero = 0;
    auto note = [&](int j, T p) {
        bad |= (j < w && is_bad(p)) ? (1u << j) : 0u;
        zero |= (p == T(0)) ? (1u << j) : 0u;
    };
    T p0 = lane_value<T>(x[0], 0);
    note(0, p0);
    T inv = pivot_recip(p0);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const T m = lane > j ? x[j] * inv : T(0);
        x[j] = lane > j ? m : x[j];
        T inv_next = T(0);
        if (j + 1 < 16) {
            x[j + 1] -= m * lane_value<T>(x[j + 1], j);
            const T pn = lane_value<T>(x[j + 1], j + 1);
            note(j + 1, pn);
            inv_next = pivot_recip(pn);
        }
#pragma unroll
        for (int k = j + 2; k < 16; ++k) x[k] -= m * lane_value<T>(x[k], j);
        inv = inv_next;
        // keep each step's pivot-row reads next to their use
        __builtin_amdgcn_sched_barrier(0);
    }
    if (pw == 0 && bad != 0 && lane == 0) {
        const int fj = __builtin_ctz(bad);
        st->info = k0 + c0 + fj;
        st->code = ((zero >> fj) & 1u) ? 4 : 5;
        *s_fail = 1;
    }
    if (valid && (lane >= 16 || pw == 0)) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k < w) S[row * LD + c0 + k] = x[k];
    }
}

// U12 = L11^{-1} A12 for one column of the 16 rows c0 .. c0 + 15 by
// substitution (L11 unit lower, its entries LDS broadcasts): y holds the
// column, sums in ascending k.  Substitution, not a product with an explicit
// inverse of L11: without pivoting L11 may be ill conditioned, and the
// explicit inverse would carry that into U12.
template <typename T>
__device__ inline void panel_row_solve(const T *S, int c0, int col, bool in, T (&y)[16]) {
    constexpr int LD = kLeaf + 1;
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = in ? S[(c0 + i) * LD + col] : T(0);
#pragma unroll
    for (int i = 1; i < 16; ++i)
#pragma unroll
        for (int k = 0; k < i; ++k) y[i] -= S[(c0 + i) * LD + c0 + k] * y[k];
}

// GENP of one pivot block (b <= 128) held in LDS, by eight waves in panels of
// 16 columns (eq. eqgenp with pivot blocks of 16 inside the pivot block).
// Panel p (columns c0 .. c0 + 15), once factored:
//   phase 1 (all waves): U12 = L11^{-1} A12 for the next panel's 16 columns
//     (every wave solves them itself, one column a lane) and the Schur update
//     A22 -= L21 U12 of those columns, row tiles dealt to the waves;
//   phase 2: the panel waves (leaf_panel) factor the next panel, while the
//     other waves solve for U12 in the remaining column blocks and update them.
// The updates run on the matrix cores in 16 x 16 tiles (K = 16).  Two
// barriers a panel; the chain is the panel factorisation.  The block is
// written back in place; after a breakdown the later kernels see the status
// and exit.
template <typename T>
__global__ __launch_bounds__(512) void k_leaf_genp(T *a, int64_t lda, int b, int64_t k0,
                                                   DevStatus *st) {
    using acc_t = typename Mma<T>::acc;
    constexpr int NW = 8, LD = kLeaf + 1;
    __shared__ T S[kLeaf * LD];
    __shared__ T Us[NW][16][17];  // a wave's U12 block, transposed to operand layout
    __shared__ int s_fail;
    if (st->code != 0) return;  // an earlier pivot block broke down
    __builtin_amdgcn_s_setprio(3);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) s_fail = 0;
    // the block into LDS: thread (tid & 127) takes a column, rows lr, lr + 4,
    // ..., all 32 of its loads in flight together (one memory round trip)
    const int lc = tid & 127, lr = tid >> 7;
    {
        T v[kLeaf / 4];
#pragma unroll
        for (int u = 0; u < kLeaf / 4; ++u) {
            const int i = 4 * u + lr;
            v[u] = load_if(a, static_cast<int64_t>(i) * lda + lc, i < b && lc < b);
        }
#pragma unroll
        for (int u = 0; u < kLeaf / 4; ++u) {
            const int i = 4 * u + lr;
            if (i < b && lc < b) S[i * LD + lc] = v[u];
        }
    }
    __syncthreads();
    // waves that factor the panel at column c (48 rows below the pivot rows each)
    auto panel_waves = [&](int c) {
        const int below = b - c - 16;
        return below <= 0 ? 1 : (below + 47) / 48;
    };
    if (wave < panel_waves(0)) leaf_panel<T>(S, b, 0, lane, wave, st, k0, &s_fail);
    __syncthreads();
    const int nbk = (b + 15) / 16;
    const int lr16 = lane & 15, lk = lane >> 4;
    for (int p = 0;; ++p) {
        const int c0 = 16 * p, c1 = c0 + 16;
        if (s_fail || c1 >= b) break;
        // U12 rows of column block q (lane c < 16 holds its column c) into
        // this wave's operand slab: bk[kk] = U12[4 kk + (lane >> 4)][lane & 15]
        auto operands = [&](const T(&y)[16], T(&bk)[4]) {
            if (lane < 16) {
#pragma unroll
                for (int i = 0; i < 16; ++i) Us[wave][i][lane] = y[i];
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) bk[kk] = Us[wave][4 * kk + lk][lr16];
        };
        // C[rt, q] -= L21[rt] U12[q] for one or two row tiles of block q
        auto tiles = [&](int q, int rtA, int rtB, bool two, const T(&bk)[4]) {
            const int col = 16 * q + lr16;
            acc_t ca, cb;
            T aa[4], ab[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rowA = 16 * rtA + Mma<T>::row(lane, r);
                ca[r] = (rowA < b && col < b) ? S[rowA * LD + col] : T(0);
                const int rowB = 16 * rtB + Mma<T>::row(lane, r);
                cb[r] = (two && rowB < b && col < b) ? S[rowB * LD + col] : T(0);
            }
            const int arA = 16 * rtA + lr16, arB = 16 * rtB + lr16;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = c0 + 4 * kk + lk;
                aa[kk] = arA < b ? -S[arA * LD + k] : T(0);
                ab[kk] = (two && arB < b) ? -S[arB * LD + k] : T(0);
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                ca = Mma<T>::step(aa[kk], bk[kk], ca);
                cb = Mma<T>::step(ab[kk], bk[kk], cb);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rowA = 16 * rtA + Mma<T>::row(lane, r);
                if (rowA < b && col < b) S[rowA * LD + col] = ca[r];
                const int rowB = 16 * rtB + Mma<T>::row(lane, r);
                if (two && rowB < b && col < b) S[rowB * LD + col] = cb[r];
            }
        };
        auto store_rows = [&](int col, const T(&y)[16]) {  // U12 column back, below row c0
#pragma unroll
            for (int i = 1; i < 16; ++i) S[(c0 + i) * LD + col] = y[i];
        };
        // phase 1: the next panel's column block (every wave solves for its
        // U12, wave w updates row tile p + 1 + w; at most 7 row tiles remain)
        const int ncol = c1 + lr16;
        T yn[16];
        panel_row_solve<T>(S, c0, ncol, lane < 16 && ncol < b, yn);
        {
            T bk[4];
            operands(yn, bk);
            const int rt = p + 1 + wave;
            if (rt < nbk) tiles(p + 1, rt, rt, false, bk);
        }
        __syncthreads();
        // phase 2 (wave 0 stores the next block's U12 only now: every wave
        // read that block's rows c0 .. c0 + 15 in phase 1)
        const int np = panel_waves(c1);
        if (wave < np) {
            if (wave == 0 && lane < 16 && ncol < b) store_rows(ncol, yn);
            leaf_panel<T>(S, b, c1, lane, wave, st, k0, &s_fail);
        } else {
            // column blocks q >= p + 2 dealt to the update waves (at most 6
            // blocks, at least 5 waves): solve for the block's U12, store it,
            // update its row tiles two at a time
            for (int q = p + 2 + (wave - np); q < nbk; q += NW - np) {
                const int col = 16 * q + lr16;
                T y[16];
                panel_row_solve<T>(S, c0, col, lane < 16 && col < b, y);
                if (lane < 16 && col < b) store_rows(col, y);
                T bk[4];
                operands(y, bk);
                for (int rt = p + 1; rt < nbk; rt += 2) tiles(q, rt, rt + 1, rt + 1 < nbk, bk);
            }
        }
        __syncthreads();
    }
    for (int i = lr; i < b; i += 4)
        if (lc < b) a[static_cast<int64_t>(i) * lda + lc] = S[i * LD + lc];
}

// Inverses of the 32 x 32 diagonal sub-blocks of factored diagonal blocks
// (the off-diagonal coupling is applied by blocked substitution, so only these
// small inverses are formed).  Workgroup g covers rows 128 g .. 128 g + 127 of
// the b x b block at `a`; wave w < nsub inverts U's sub-block w, wave nsub + w
// the unit-lower L's.  A wave stages its sub-block in LDS (the identity past
// the block's edge, so the sweeps need no bounds), and lane c (< 32; lanes
// 32 .. 63 repeat 0 .. 31 and store nothing) forms column c of the inverse by
// substitution, the factor's rows read as LDS broadcasts:
//   U: x_i = (delta_ic - sum_{k > i} u_ik x_k) / u_ii, from the bottom row;
//   L: x_i = delta_ic - sum_{k < i} l_ik x_k.
// (Row-oriented, sums in ascending k: the order whose rounding the blocked
// solves were validated with; a column sweep was measured to leave larger
// errors in the U inverses of strongly growing factors.)  Compact output:
// row 32 q + i of Linv / Uinv holds row i of sub-block q's inverse.
template <typename T>
__global__ __launch_bounds__(512, 1) void k_diag_inv(const T *a, int64_t lda, int b, T *Linv, T *Uinv,
                                                  const DevStatus *st) {
    if (st->code != 0) return;
    __shared__ T Bs[8][kSub][kSub + 1];
    __builtin_amdgcn_s_setprio(3);
    const int64_t g0 = static_cast<int64_t>(blockIdx.x) * 4 * kSub;
    a += g0 * lda + g0;
    Linv += g0 * kSub;
    Uinv += g0 * kSub;
    b = (b - g0) < 4 * kSub ? static_cast<int>(b - g0) : 4 * kSub;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nsub = (b + kSub - 1) / kSub;
    if (wave >= 2 * nsub) return;
    const bool upper = wave < nsub;
    const int q0 = (upper ? wave : wave - nsub) * kSub;
    const int sbq = (b - q0) < kSub ? (b - q0) : kSub;
    const int c = lane & (kSub - 1), h = lane >> 5;
    T(*B)[kSub + 1] = Bs[wave];
#pragma unroll
    for (int k = 0; k < kSub; k += 2) {
        const int r = k + h;
        const T v = load_if(a, static_cast<int64_t>(q0 + r) * lda + q0 + c, r < sbq && c < sbq);
        B[r][c] = (r < sbq && c < sbq) ? v : (r == c ? T(1) : T(0));
    }
    // (the wave reads only what it wrote: no barrier)
    T x[kSub];
    if (upper) {
#pragma unroll
        for (int i = kSub - 1; i >= 0; --i) {
            // each row's reads next to their use (hoisted together, the 496
            // entries would not fit in registers)
            asm volatile("" ::: "memory");
            T sum = T(0);
#pragma unroll
            for (int k = i + 1; k < kSub; ++k) sum += B[i][k] * x[k];
            x[i] = ((c == i ? T(1) : T(0)) - sum) * (T(1) / B[i][i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < kSub; ++i) {
            asm volatile("" ::: "memory");
            T sum = T(0);
#pragma unroll
            for (int k = 0; k < i; ++k) sum += B[i][k] * x[k];
            x[i] = (c == i ? T(1) : T(0)) - sum;
        }
    }
    if (lane < kSub && c < sbq) {
        T *out = upper ? Uinv : Linv;
#pragma unroll
        for (int k = 0; k < kSub; ++k)
            if (k < sbq) out[static_cast<int64_t>(q0 + k) * kSub + c] = x[k];
    }
}

// Blocked substitution on the matrix cores.  The pivot block's factors sit
// packed at `lu` (ld, width b <= 256); Dinv holds the inverses of their
// 32 x 32 diagonal sub-blocks (compact: row 32 q + i, 32 columns).  One workgroup owns a 32-wide
// strip of the panel and keeps it in MFMA accumulators, 16 x 16 tiles dealt
// round-robin to its four waves.  Per diagonal sub-block i the two tiles of
// rows i are published to LDS, multiplied by the sub-block inverse (one
// 16 x 16 tile of X_i a wave, back into LDS), and every wave subtracts
// (factor block) x X_i from its tiles further along; X_i is final then and is
// written out from LDS.  Three barriers a step.
//
// The substitution is a chain of b / 32 short steps, so operands are fetched
// one step ahead (the next sub-block inverse and the next step's factor
// operands), which hides their memory latency behind the current step, and
// each phase reads all its LDS operands before its first product.
//
// LEFT:  C (b x count) <- L^{-1} P C, strips of 32 columns (row tiles dealt).
// With `rowsrc` (pivoted blocks) row t of P C is row rowsrc[t] - rowbase of C:
// the strip is read whole into registers before any of it is written back.

// This thread's four elements (e = tid + 256 m) of sub-block q's inverse:
// fetched raw (clamped address), zeroed past the block when stored to LDS.
__device__ inline bool dinv_in(int b, int q, int e) {
    const int q0 = q * kSub, sb = (b - q0) < kSub ? (b - q0) : kSub;
    return sb > 0 && e / kSub < sb && e % kSub < sb;
}
template <typename T>
__device__ inline void fetch_dinv(const T *Dinv, int b, int q, int tid, T (&d)[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int e = tid + 256 * m;
        d[m] = Dinv[dinv_in(b, q, e) ? q * kSub * static_cast<int64_t>(kSub) + e : 0];
    }
}

// Strip `blk` (columns 32 blk ..) of the left solve, one workgroup of 256
// threads.  Step i's factor panel L[32 i + 32 ..][32 i .. 32 i + 31] is read
// row by row, 16 bytes a load, one step ahead into registers and staged in LDS; the
// four waves each apply the sub-block inverse to one 16 x 16 tile of rows i,
// and X_i goes to memory from LDS at the start of the next step.
template <typename T>
__device__ __attribute__((always_inline)) inline void trsm_left_strip(const T *lu, int64_t ld, int b, T *C, int64_t ldc,
                                       int64_t count, const T *Dinv, const int *rowsrc,
                                       int64_t rowbase, int64_t blk) {
    using acc_t = typename Mma<T>::acc;
    constexpr int BN = 32;
    constexpr int PR = kMaxBlock - kSub;  // rows of a step's factor panel, at most
    constexpr int PV = 16 / sizeof(T);    // elements of one 16-byte load
    constexpr int PG = kSub / PV;         // 16-byte groups of a panel row
    constexpr int PL = PR * PG / 256;     // groups a thread stages
    using vec_t = T __attribute__((ext_vector_type(PV)));
    // row strides: a 16 x 4 operand read (rows by lane & 15, columns by
    // lane >> 4) is bank-conflict free at 34, a 4 x 16 one at 48
    __shared__ T Xa[kSub][48];            // rows of sub-block i of the strip (before)
    __shared__ T Xb[kSub][48];            // X_i (after)
    __shared__ T Ds[kSub][34];
    __shared__ T Ls[PR][34];              // L[i0 + 32 + p][i0 + c]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int64_t c0 = blk * BN;
    const int wcols = static_cast<int>((count - c0) < BN ? (count - c0) : BN);
    const int nrt = (b + 15) / 16;
    int64_t src[4][4];
    if (rowsrc) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = wave + 4 * u, row = 16 * t + Mma<T>::row(lane, r);
                src[u][r] = load_if(rowsrc, row, t < nrt && row < b) - rowbase;
            }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) src[u][r] = 16 * (wave + 4 * u) + Mma<T>::row(lane, r);
    }
    acc_t acc[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = wave + 4 * u;
                const int row = 16 * t + Mma<T>::row(lane, r), col = 16 * j + lo;
                const bool in = t < nrt && row < b && col < wcols;
                acc[u][j][r] = load_if(C, src[u][r] * ldc + c0 + col, in);
            }
    // step i's factor panel, row-major and coalesced, 16 bytes a load: load m
    // of a thread is group tid % PG of panel row tid / PG + (256 / PG) m
    constexpr int PS = 256 / PG;
    const int pc = PV * (tid % PG), pr = tid / PG;
    vec_t pf[PL];
    T d[4];
    auto fetch_panel = [&](int i) {
        const int i0 = i * kSub, rows = b - i0 - kSub;
        if (rows <= 0) return;  // no panel (the staging stores zeros)
        // rows past the panel load its first row instead and are zeroed when staged
        const T *top = lu + (i0 + kSub) * ld + i0 + pc, *base = top + pr * ld;
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            const int p = pr + PS * m;
            __builtin_memcpy(&pf[m], p < rows ? base + PS * m * ld : top, sizeof(vec_t));
        }
    };
    auto store_x = [&](int i) {  // X_i (in Xb) to rows 32 i .. of the strip
        const int i0 = i * kSub;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = tid + 256 * m, row = e >> 5, col = e & 31;
            if (i0 + row < b && col < wcols) C[(i0 + row) * ldc + c0 + col] = Xb[row][col];
        }
    };
    fetch_dinv(Dinv, b, 0, tid, d);
    fetch_panel(0);
    const int nsub = (b + kSub - 1) / kSub;
    for (int i = 0; i < nsub; ++i) {
        const int i0 = i * kSub, rows = b - i0 - kSub;
        // publish: the sub-block inverse, the factor panel, rows i of the strip,
        // and the previous step's result to memory
        #pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = tid + 256 * m;
            Ds[e / kSub][e % kSub] = dinv_in(b, i, e) ? d[m] : T(0);
        }
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            const int p = pr + PS * m;
            const vec_t v = p < rows ? pf[m] : vec_t(0);
            __builtin_memcpy(&Ls[p][pc], &v, sizeof(vec_t));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = wave + 4 * u;
            if (t == 2 * i || t == 2 * i + 1)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Xa[16 * (t - 2 * i) + Mma<T>::row(lane, r)][16 * j + lo] = acc[u][j][r];
        }
        if (i > 0) store_x(i - 1);
        __syncthreads();
        if (i + 1 < nsub) {
            fetch_dinv(Dinv, b, i + 1, tid, d);
            fetch_panel(i + 1);
        }
        {  // X_i = D_i^{-1} (rows i): wave w takes row tile w & 1, column tile w >> 1
            const int q = wave & 1, j = wave >> 1;
            T da[kSub / 4], xa[kSub / 4];
#pragma unroll
            for (int kq = 0; kq < kSub / 4; ++kq) {
                da[kq] = Ds[16 * q + lo][4 * kq + hi];
                xa[kq] = Xa[4 * kq + hi][16 * j + lo];
            }
            acc_t x = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int kq = 0; kq < kSub / 4; ++kq) x = Mma<T>::step(da[kq], xa[kq], x);
#pragma unroll
            for (int r = 0; r < 4; ++r) Xb[16 * q + Mma<T>::row(lane, r)][16 * j + lo] = x[r];
        }
        __syncthreads();
        {
            // every operand of the step is read before the first product: the
            // rows of inactive tiles are clamped into the panel and not used
            T xb[kSub / 4][2], fv[4][kSub / 4];
#pragma unroll
            for (int kq = 0; kq < kSub / 4; ++kq)
#pragma unroll
                for (int j = 0; j < 2; ++j) xb[kq][j] = Xb[4 * kq + hi][16 * j + lo];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = wave + 4 * u, pt = 16 * (t - 2 * i - 2);
                const int p = (pt < 0 ? 0 : (pt > PR - 16 ? PR - 16 : pt)) + lo;
#pragma unroll
                for (int kq = 0; kq < kSub / 4; ++kq) fv[u][kq] = Ls[p][4 * kq + hi];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = wave + 4 * u;
                if (t >= 2 * i + 2 && t < nrt) {
#pragma unroll
                    for (int kq = 0; kq < kSub / 4; ++kq)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            acc[u][j] = Mma<T>::step(-fv[u][kq], xb[kq][j], acc[u][j]);
                }
            }
        }
        __syncthreads();
    }
    store_x(nsub - 1);
}

// RIGHT: C (count x b) <- C U^{-1}, strips of 32 rows (column tiles dealt).
// Strip `blk` (rows 32 blk ..), one workgroup of 256 threads; the factor rows
// of step j are read one step ahead straight into the operand registers (four
// rows of 16 consecutive columns a load), the rest as on the left.
template <typename T>
__device__ __attribute__((always_inline)) inline void trsm_right_strip(const T *lu, int64_t ld, int b, T *C, int64_t ldc,
                                        int64_t count, const T *Dinv, int64_t blk) {
    using acc_t = typename Mma<T>::acc;
    constexpr int BM = 32;
    // row strides: a 16 x 4 operand read (rows by lane & 15, columns by
    // lane >> 4) is bank-conflict free at 34, a 4 x 16 one at 48
    __shared__ T Xa[BM][34];   // columns of sub-block j of the strip (before)
    __shared__ T Xb[BM][34];   // X_j (after)
    __shared__ T Ds[kSub][48];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lo = lane & 15, hi = lane >> 4;
    const int64_t r0 = blk * BM;
    const int wrows = static_cast<int>((count - r0) < BM ? (count - r0) : BM);
    const int nct = (b + 15) / 16;
    acc_t acc[4][2];  // [column tile u][row tile]
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = wave + 4 * u;
                const int row = 16 * q + Mma<T>::row(lane, r), col = 16 * c + lo;
                acc[u][q][r] = load_if(C, (r0 + row) * ldc + col, c < nct && row < wrows && col < b);
            }
    // step j's factor rows U[32 j + k][16 c + lo] for the column tiles right of
    // sub-block j (all 32 of its rows are then inside the block); a column past
    // the block reads the block's last one and is masked where it is used
    auto fetch_f = [&](int j, T (&f)[4][kSub / 4]) {
        const int j0 = j * kSub;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = wave + 4 * u, col = 16 * c + lo;
            if (c >= 2 * j + 2 && c < nct) {
                const T *p = lu + (j0 + hi) * ld + (col < b ? col : b - 1);
#pragma unroll
                for (int kq = 0; kq < kSub / 4; ++kq) f[u][kq] = p[4 * kq * ld];
            }
        }
    };
    auto store_x = [&](int j) {  // X_j (in Xb) to columns 32 j .. of the strip
        const int j0 = j * kSub;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = tid + 256 * m, row = e >> 5, col = e & 31;
            if (row < wrows && j0 + col < b) C[(r0 + row) * ldc + j0 + col] = Xb[row][col];
        }
    };
    auto step = [&](int j, const T (&f)[4][kSub / 4], T (&fn)[4][kSub / 4], const T (&d)[4],
                    T (&dn)[4], bool last) {
        const int j0 = j * kSub, sb = (b - j0) < kSub ? (b - j0) : kSub;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = tid + 256 * m;
            Ds[e / kSub][e % kSub] = dinv_in(b, j, e) ? d[m] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = wave + 4 * u;
            if (c == 2 * j || c == 2 * j + 1)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        Xa[16 * q + Mma<T>::row(lane, r)][16 * (c - 2 * j) + lo] = acc[u][q][r];
        }
        if (j > 0) store_x(j - 1);
        __syncthreads();
        if (!last) {
            fetch_f(j + 1, fn);
            fetch_dinv(Dinv, b, j + 1, tid, dn);
        }
        {  // X_j = (columns j) U_jj^{-1}: wave w takes row tile w & 1, column tile w >> 1
            const int q = wave & 1, cc = wave >> 1;
            T xa[kSub / 4], da[kSub / 4];
#pragma unroll
            for (int kq = 0; kq < kSub / 4; ++kq) {
                xa[kq] = Xa[16 * q + lo][4 * kq + hi];
                da[kq] = Ds[4 * kq + hi][16 * cc + lo];
            }
            acc_t x = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int kq = 0; kq < kSub / 4; ++kq) x = Mma<T>::step(xa[kq], da[kq], x);
#pragma unroll
            for (int r = 0; r < 4; ++r) Xb[16 * q + Mma<T>::row(lane, r)][16 * cc + lo] = x[r];
        }
        __syncthreads();
        {
            T xb[2][kSub / 4];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int kq = 0; kq < kSub / 4; ++kq) xb[q][kq] = Xb[16 * q + lo][4 * kq + hi];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = wave + 4 * u;
                if (c >= 2 * j + 2 && c < nct) {
                    const bool cin = 16 * c + lo < b;
#pragma unroll
                    for (int kq = 0; kq < kSub / 4; ++kq) {
                        const int k = 4 * kq + hi;
                        const T fv = (cin && k < sb) ? -f[u][kq] : T(0);
#pragma unroll
                        for (int q = 0; q < 2; ++q)
                            acc[u][q] = Mma<T>::step(xb[q][kq], fv, acc[u][q]);
                    }
                }
            }
        }
        __syncthreads();
    };
    T fa[4][kSub / 4], fb[4][kSub / 4], da[4], db[4];
    fetch_dinv(Dinv, b, 0, tid, da);
    fetch_f(0, fa);
    const int nsub = (b + kSub - 1) / kSub;
    for (int j = 0; j < nsub; j += 2) {
        step(j, fa, fb, da, db, j + 1 >= nsub);
        if (j + 1 < nsub) step(j + 1, fb, fa, db, da, j + 2 >= nsub);
    }
    store_x(nsub - 1);
}

// Both solves of one pivot block in one launch (they touch disjoint blocks
// and only read the factors): workgroups below `nl` take the strips of
// L_B^{-1} P Cl, the others those of Cr U_B^{-1}.  FP64 keeps a step's
// operands in flight at one workgroup per CU (the left solve's staged panel
// also fills most of the LDS); FP32 fits two.
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 1 : 2) void k_trsm_pair(
    const T *lu, int64_t ld, int b, T *Cl, int64_t ldcl, int64_t countl, const T *Linv,
    const int *rowsrc, int64_t rowbase, T *Cr, int64_t ldcr, int64_t countr, const T *Uinv,
    const int *abort, int64_t nl) {
    if (*abort != 0) return;
    __builtin_amdgcn_s_setprio(2);  // on the panel's critical path, beside the update GEMM
    const int64_t g = blockIdx.x;
    if (g < nl)
        trsm_left_strip<T>(lu, ld, b, Cl, ldcl, countl, Linv, rowsrc, rowbase, g);
    else
        trsm_right_strip<T>(lu, ld, b, Cr, ldcr, countr, Uinv, g - nl);
}

// dst[di] = src[si] with si = gather ? gather[i] : i, di = scatter ? scatter[i] : i.
template <typename T, typename U>
__global__ void k_convert_2d(const T *src, int64_t lds, U *dst, int64_t ldd, int64_t rows,
                             int64_t cols, const int *gather, const int *scatter) {
    const int64_t total = rows * cols;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / cols, j = e % cols;
        const int64_t si = gather ? gather[i] : i, di = scatter ? scatter[i] : i;
        dst[di * ldd + j] = static_cast<U>(src[si * lds + j]);
    }
}

__global__ void k_iota(int *p, int64_t n) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[e] = static_cast<int>(e);
}

// Diagonal block (leaf) number `leaf` of the pivoted elimination: panels of nb
// columns, a panel wider than kLeaf cut into kLeaf + rest.  Returns its width
// (0 if there is no such block), its first row in *s and its panel's first
// column in *p0.
__device__ inline int leaf_span(int64_t n, int nb, int64_t leaf, int64_t *s, int64_t *p0) {
    if (nb <= kLeaf) {
        *s = *p0 = leaf * nb;
        const int64_t w = n - *s;
        return w <= 0 ? 0 : static_cast<int>(w < nb ? w : nb);
    }
    *p0 = (leaf >> 1) * nb;
    const int64_t pb = (n - *p0) < nb ? (n - *p0) : nb;
    if (pb <= 0) return 0;
    if ((leaf & 1) == 0) {
        *s = *p0;
        return static_cast<int>(pb < kLeaf ? pb : kLeaf);
    }
    *s = *p0 + kLeaf;
    return pb > kLeaf ? static_cast<int>(pb - kLeaf) : 0;
}

// Rows s .. s + w - 1 of columns c0 .. c0 + cw - 1 (cw <= 32) take the values of
// rows piv[s + t]: the strip is read whole into LDS, then written back.
template <typename T>
__device__ inline void permute_strip(T *a, int64_t ld, int64_t s, int w, int64_t c0, int cw,
                                     const int *piv, T (*tile)[33]) {
    for (int e = threadIdx.x; e < w * 32; e += blockDim.x) {
        const int t = e >> 5, c = e & 31;
        if (c < cw) tile[t][c] = a[static_cast<int64_t>(piv[s + t]) * ld + c0 + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < w * 32; e += blockDim.x) {
        const int t = e >> 5, c = e & 31;
        if (c < cw) a[(s + t) * ld + c0 + c] = tile[t][c];
    }
}

// Apply each diagonal block's row exchanges to the multipliers left of its
// panel, so that the stored factors satisfy P M = L U row by row (the part
// inside the panel is done when the panel is factored).  Block y of the grid
// covers leaf y; block x a strip of 32 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_left(T *a, int64_t ld, int64_t n, int nb,
                                                      const int *piv, const int *abort) {
    __shared__ T tile[kLeaf][33];
    if (*abort != 0) return;
    int64_t s = 0, p0 = 0;
    const int w = leaf_span(n, nb, blockIdx.y, &s, &p0);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * 32;
    if (w == 0 || c0 >= p0) return;
    permute_strip(a, ld, s, w, c0, static_cast<int>((p0 - c0) < 32 ? (p0 - c0) : 32), piv, tile);
}

// One diagonal block's exchanges applied to columns cb .. ce - 1 of its rows.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_rows(T *a, int64_t ld, int64_t s, int w,
                                                      int64_t cb, int64_t ce, const int *piv,
                                                      const int *abort) {
    __shared__ T tile[kLeaf][33];
    if (*abort != 0) return;
    const int64_t c0 = cb + static_cast<int64_t>(blockIdx.x) * 32;
    if (c0 >= ce) return;
    permute_strip(a, ld, s, w, c0, static_cast<int>((ce - c0) < 32 ? (ce - c0) : 32), piv, tile);
}

__device__ inline void atomic_max_nonneg(double *addr, double v) {
    // Non-negative doubles order like their bit patterns (NaN sorts above Inf).
    atomicMax(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ inline void atomic_min_nonneg(double *addr, double v) {
    atomicMin(reinterpret_cast<unsigned long long *>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

// out[0] = max |U| (upper triangle incl. diagonal), out[1] = min |u_kk|, out[2] = max |A|
// over the full n x n matrix (the latter only when `full` is set).
template <typename T>
__global__ void k_lu_stats(const T *lu, int64_t ld, int64_t n, double *out, int full) {
    double umax = 0.0, dmin = INFINITY, amax = 0.0;
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        const double v = fabs(static_cast<double>(lu[i * ld + j]));
        if (full) amax = fmax(amax, v);
        if (j >= i) umax = fmax(umax, v);
        if (j == i) dmin = fmin(dmin, v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        umax = fmax(umax, __shfl_xor(umax, off));
        dmin = fmin(dmin, __shfl_xor(dmin, off));
        amax = fmax(amax, __shfl_xor(amax, off));
    }
    if ((threadIdx.x & 63) == 0) {
        if (full) {
            atomic_max_nonneg(out + 2, amax);
        } else {
            atomic_max_nonneg(out + 0, umax);
            atomic_min_nonneg(out + 1, dmin);
        }
    }
}

int grid_for(int64_t total, int threads) {
    int64_t g = (total + threads - 1) / threads;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

template <typename T>
hipError_t leaf_lu(T *a, int64_t lda, int b, T *Linv, T *Uinv, int64_t k0, DevStatus *st, int *piv,
                   hipStream_t s) {
    if (b < 1 || b > kLeaf) return hipErrorInvalidValue;
    if (piv)
        hipLaunchKernelGGL((k_leaf_lu<T, true>), dim3(1), dim3(kLeafThreads), 0, s, a, lda, b, k0,
                           st, piv);
    else
        hipLaunchKernelGGL(k_leaf_genp<T>, dim3(1), dim3(512), 0, s, a, lda, b, k0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_inv<T>, dim3(1), dim3(512), 0, s, a, lda, b, Linv, Uinv, st);
    return hipGetLastError();
}

template <typename T>
hipError_t diag_inverses(const T *a, int64_t lda, int64_t n, T *Linv, T *Uinv, const DevStatus *st,
                         hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > (int64_t(1) << 30)) return hipErrorInvalidValue;
    const unsigned grid = static_cast<unsigned>((n + 4 * kSub - 1) / (4 * kSub));
    hipLaunchKernelGGL(k_diag_inv<T>, dim3(grid), dim3(512), 0, s, a, lda, static_cast<int>(n),
                       Linv, Uinv, st);
    return hipGetLastError();
}

template <typename T>
hipError_t trsm_pair(const T *lu, int64_t ld, int b, T *Cl, int64_t ldcl, int64_t countl,
                     const T *Linv, const int *rowsrc, int64_t rowbase, T *Cr, int64_t ldcr,
                     int64_t countr, const T *Uinv, const int *abort, hipStream_t s) {
    if (b < 1 || b > kMaxBlock || countl < 0 || countr < 0 || abort == nullptr)
        return hipErrorInvalidValue;
    const int64_t nl = (countl + 31) / 32, nr = (countr + 31) / 32;
    if (nl + nr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_trsm_pair<T>, dim3(static_cast<unsigned>(nl + nr)), dim3(256), 0, s, lu,
                       ld, b, Cl, ldcl, countl, Linv, rowsrc, rowbase, Cr, ldcr, countr, Uinv,
                       abort, nl);
    return hipGetLastError();
}

template <typename T, typename U>
hipError_t convert_2d(const T *src, int64_t lds, U *dst, int64_t ldd, int64_t rows, int64_t cols,
                      hipStream_t s, const int *gather, const int *scatter) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_convert_2d<T, U>), dim3(grid_for(rows * cols, 256)), dim3(256), 0, s,
                       src, lds, dst, ldd, rows, cols, gather, scatter);
    return hipGetLastError();
}

hipError_t iota(int *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t permute_rows(T *a, int64_t ld, int64_t s0, int w, int64_t cb, int64_t ce,
                        const int *piv, const int *abort, hipStream_t s) {
    if (w < 1 || w > kLeaf) return hipErrorInvalidValue;
    if (ce <= cb) return hipSuccess;
    hipLaunchKernelGGL(k_permute_rows<T>, dim3(static_cast<unsigned>((ce - cb + 31) / 32)),
                       dim3(256), 0, s, a, ld, s0, w, cb, ce, piv, abort);
    return hipGetLastError();
}

template <typename T>
hipError_t permute_left(T *a, int64_t ld, int64_t n, int nb, const int *piv, const int *abort,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (nb < 1 || nb > kMaxBlock) return hipErrorInvalidValue;
    const int64_t panels = (n + nb - 1) / nb;
    const int64_t leaves = nb <= kLeaf ? panels : 2 * panels;
    const int64_t strips = (n + 31) / 32;
    if (leaves > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_permute_left<T>, dim3(static_cast<unsigned>(strips),
                                               static_cast<unsigned>(leaves)),
                       dim3(256), 0, s, a, ld, n, nb, piv, abort);
    return hipGetLastError();
}

// out3 must be preset to {0, +Inf, *} (max |U|, min |u_kk|); `full` variant writes out3[2].
template <typename T>
hipError_t lu_stats(const T *lu, int64_t ld, int64_t n, double *out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_stats<T>, dim3(grid_for(n * n, 256)), dim3(256), 0, s, lu, ld, n, out3,
                       0);
    return hipGetLastError();
}

template <typename T>
hipError_t abs_max(const T *m, int64_t ld, int64_t n, double *out3, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_stats<T>, dim3(grid_for(n * n, 256)), dim3(256), 0, s, m, ld, n, out3,
                       1);
    return hipGetLastError();
}

template hipError_t leaf_lu<double>(double *, int64_t, int, double *, double *, int64_t,
                                    DevStatus *, int *, hipStream_t);
template hipError_t leaf_lu<float>(float *, int64_t, int, float *, float *, int64_t, DevStatus *,
                                   int *, hipStream_t);
template hipError_t diag_inverses<double>(const double *, int64_t, int64_t, double *, double *,
                                          const DevStatus *, hipStream_t);
template hipError_t diag_inverses<float>(const float *, int64_t, int64_t, float *, float *,
                                         const DevStatus *, hipStream_t);
template hipError_t trsm_pair<double>(const double *, int64_t, int, double *, int64_t, int64_t,
                                      const double *, const int *, int64_t, double *, int64_t,
                                      int64_t, const double *, const int *, hipStream_t);
template hipError_t trsm_pair<float>(const float *, int64_t, int, float *, int64_t, int64_t,
                                     const float *, const int *, int64_t, float *, int64_t,
                                     int64_t, const float *, const int *, hipStream_t);
template hipError_t permute_left<double>(double *, int64_t, int64_t, int, const int *, const int *,
                                         hipStream_t);
template hipError_t permute_rows<double>(double *, int64_t, int64_t, int, int64_t, int64_t,
                                         const int *, const int *, hipStream_t);
template hipError_t permute_rows<float>(float *, int64_t, int64_t, int, int64_t, int64_t,
                                        const int *, const int *, hipStream_t);
template hipError_t permute_left<float>(float *, int64_t, int64_t, int, const int *, const int *,
                                        hipStream_t);
template hipError_t convert_2d<double, double>(const double *, int64_t, double *, int64_t, int64_t,
                                               int64_t, hipStream_t, const int *, const int *);
template hipError_t convert_2d<double, float>(const double *, int64_t, float *, int64_t, int64_t,
                                              int64_t, hipStream_t, const int *, const int *);
template hipError_t convert_2d<float, double>(const float *, int64_t, double *, int64_t, int64_t,
                                              int64_t, hipStream_t, const int *, const int *);
template hipError_t convert_2d<float, float>(const float *, int64_t, float *, int64_t, int64_t,
                                             int64_t, hipStream_t, const int *, const int *);
template hipError_t lu_stats<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t lu_stats<float>(const float *, int64_t, int64_t, double *, hipStream_t);
template hipError_t abs_max<double>(const double *, int64_t, int64_t, double *, hipStream_t);
template hipError_t abs_max<float>(const float *, int64_t, int64_t, double *, hipStream_t);

}  // namespace rmge

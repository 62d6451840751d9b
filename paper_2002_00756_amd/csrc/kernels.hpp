// Device kernels of the Helmholtz multigrid path (gfx950, wave64).
//
// Data layout in HBM, per multigrid level with ncol columns and nz levels.
// Columns are grouped into tiles of kTile = 32 consecutive columns, and every
// per-level array stores one tile after the other, each tile holding its nz
// levels as rows of 32 values:
//     element (k, c) sits at tile_base(c) + 32 k,
//     tile_base(c) = (c / 32) * 32 nz + c % 32.
// For storage ncol is rounded up to ncolp, a multiple of 32; the padding
// columns hold zeros (the workspace is cleared at set-up and no kernel writes
// them), so reductions may run over the padded length. nvp = nz * ncolp.
//   vectors        [batch][nvp]        tiled as above
//   kh             [2][nvp]            E-face plane, then N-face plane
//   kv             [nvp]               face k|k+1; row nz-1 is zero (no flux
//                                      through the top), so loads need no guard
//   dl (delta)     [nvp]
//   kv2            [nvp]               9-cell stencil only: coupling of levels
//                                      k and k+2; rows nz-2, nz-1 are zero
//   s              [nvp]               weighted operator only: row weight of
//                                      H = delta + S L (below)
//   cc, mm         [nvp]               factors of the column operator (below)
//   nbr            [4][ncol]           E, W, N, S neighbour column
//   fface          [2][ncol]           offset in kh of the W and S face at
//                                      level 0 (plane * nvp + tile_base(owner));
//                                      the E and N faces are at tile_base(c)
//                                      and nvp + tile_base(c)
//   pofs           [3][ncol]           tiled offsets on the next coarser level
//                                      of the parent of the column and of the
//                                      parents of its outward E/W and N/S
//                                      neighbours (prolongation)
// A workgroup that owns a tile reads one contiguous block of every array and
// a wave reads two adjacent rows of one tile. Vectors passed through the C ABI
// keep the natural [batch][nz][ncol] layout; the kernels that take them in or
// hand them out convert on the fly.
//
// Column factorisation. The smoother solves with the column operator Hz (the
// couplings between neighbouring levels of a column plus the full diagonal of
// H; Section 3.5, Eq. jacobi; with the 9-cell stencil the couplings two
// levels apart are dropped from it but stay in its diagonal, Section 3.6) by
// an LU factorisation computed once per operator (the paper stores the same
// factors; Section 3.8). Pivots are computed in a form free of cancellation:
// with s_k = delta_k + sum of the 4 horizontal couplings (+ kv2_k + kv2_{k-2}),
// the top-down pivot excess is e_0 = s_0, e_k = s_k + kv_{k-1} e_{k-1} /
// (e_{k-1} + kv_{k-1}), pivot p_k = e_k + kv_k. Stored: mm_k = 1/p_k and
// cc_k = kv_k / p_k, so that forward elimination is t_k = r_k + cc_{k-1} t_{k-1}
// and back substitution is z_k = mm_k t_k + cc_k z_{k+1}.
// Weighted operator H = delta + S L (S = diag(s), L the flux terms): its column
// matrix is S Hz' with Hz' = delta/s + (the column part of L) symmetric, so the
// factors are those of Hz' (delta/s in place of delta) and the sweeps scale
// by 1/s: forward, Hz^-1 (b + S sum K x_n) = Hz'^-1 (b/s + sum K x_n); for
// H^T = delta + L S, Hz^-T (b + sum K s_n x_n) = S^-1 Hz'^-1 (b + sum K s_n x_n).
// The smoother uses a "twisted" split at row mid = nz / 2: rows above mid
// are factored top-down as above, rows below mid bottom-up (f_{nz-1} =
// s_{nz-1}, f_k = s_k + kv_k f_{k+1} / (f_{k+1} + kv_k), q_k = f_k + kv_{k-1},
// mm_k = 1/q_k, cc_k = kv_{k-1}/q_k) and row mid with both neighbours
// eliminated, so two lanes per column share the sequential work.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hh {

constexpr int kBlock = 256;

// Workgroups of one launch are handed to the 8 XCDs round-robin (bid -> XCD
// bid % 8). Renumber them so that each XCD works through one contiguous range
// of logical blocks: neighbouring tiles (the N/S neighbour rows, the batch
// members sharing coefficients) then meet in the same L2. rev: each XCD walks
// its range backwards. Consecutive kernels on a level alternate the direction,
// so that each starts on the data the previous one touched last, which the
// last-level cache still holds when a level's streams exceed it.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks, int rev = 0) {
    const int xcd = bid & 7, slot = bid >> 3;
    const int q = nblocks >> 3, r = nblocks & 7;
    const int cnt = q + (xcd < r ? 1 : 0);
    return xcd * q + (xcd < r ? xcd : r) + (rev ? cnt - 1 - slot : slot);
}

// Logical block of a launch without the XCD renumbering, walked backwards
// when rev is set.
__device__ __forceinline__ int logical_block(int rev) {
    return rev ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
}

constexpr int kTile = 32;

// Offset of element (0, c) of a tiled array; element (k, c) is 32 k further.
__device__ __forceinline__ int tile_base(int c, int nz) {
    return (c >> 5) * (kTile * nz) + (c & (kTile - 1));
}

template <typename T>
struct LevelView {
    int ncol, nz, nvp;
    int N;  // columns per panel edge (c = p N^2 + j N + i)
    const int32_t* __restrict__ nbr;
    const uint32_t* __restrict__ fface;
    // [3][ncol] on every level but the coarsest: tiled offsets on the next
    // coarser level of the column's parent and of the parents of its outward
    // E/W and N/S neighbours (the other two neighbours share its parent)
    const int32_t* __restrict__ pofs;
    const T* __restrict__ kh;
    const T* __restrict__ kv;
    const T* __restrict__ dl;
    const T* __restrict__ cc;
    const T* __restrict__ mm;
    const T* __restrict__ kv2;  // null for the 7-point stencil
    const T* __restrict__ s;    // row weight; null for the symmetric operator
};

// Loads and stores of a stream that the cache need not keep (NT: non-temporal).
template <bool NT, typename T>
__device__ __forceinline__ T stream_load(const T* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stream_store(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Operator form a kernel is built for: symmetric, row-weighted H = delta + S L,
// or its transpose H^T = delta + L S.
enum { kSym = 0, kRowW = 1, kRowWT = 2 };

// ---------------------------------------------------------------------------
// Block-Jacobi sweep (Eq. jacobi):
//   x_new = x + omega Hz^-1 (b - H x)
//         = (1 - omega) x + omega Hz^-1 (b + sum_d K_d x_nbr(d))
// since H - Hz keeps only the horizontal off-diagonal couplings. The second
// form needs no delta or kv, only the factors: 7 words per unknown instead of
// 8. Neighbours read the old iterate (Jacobi); x and x_new must differ.
// Modes: kZero x = 0 (first sweep of a level), kPlain, kProlong x += P xc
// (first post-smoothing sweep, Algorithm 1 prolongation fused in),
// kProlongZero x = P xc.
//
// One workgroup (256 threads) owns a tile of TC columns and all nz levels.
// The memory-bound work is split from the sequential column recurrence:
//   1. all threads: for their levels k (k = kg, kg+KG, ...), gather the
//      right-hand side b + sum K x_nbr and the factor cc into LDS (coalesced
//      row loads, many independent loads in flight; own x kept in registers);
//   2. one lane per column eliminates top-down over rows [0, mid) and another
//      bottom-up over rows (mid, nz) (the twisted factorisation), from LDS;
//   3. all threads: scale by the pivot reciprocal mm (row mid combines both
//      eliminations);
//   4. the two lanes back-substitute outwards from row mid;
//   5. all threads: x_new = (1 - omega) x + omega z, coalesced stores.
// TC = 32 columns and KG = 8 level groups per 256-thread workgroup (a wave
// instruction touches two rows of 128 (float) or 256 (double) contiguous
// bytes); the small LDS footprint lets up to 8 workgroups share a CU.
enum SweepMode { kZero = 0, kPlain = 1, kProlong = 2, kProlongZero = 3 };

// Phases 2-4 of the column solve z = Hz^-1 r for ncol columns held in LDS
// with row stride S: on entry R[k*S + col] holds r and Cf[k*S + col] the
// factor cc; the calling thread owns column lc (if lc < ncol) at levels
// kg + j KG, whose pivot reciprocals it holds in mo[j]. On exit R holds z.
// Two lanes per column (tid < ncol: rows above mid, top-down; BOT <= tid <
// BOT + ncol: rows below mid, bottom-up) walk the column, SEQ levels per LDS
// round trip; row mid combines both eliminations. E1, E2 hold ncol values.
//
// Each walk is a run of rows k = first + dir * i, i < count, with a
// first-order recurrence along it. Full batches of SEQ rows carry no range
// tests, so their SEQ reads issue together and the recurrence is a plain
// chain of fused multiply-adds; the last, partial batch reads row indices
// clamped into the run and tests only the arithmetic and the stores.
template <typename T, int SEQ, bool ELIM>
__device__ __forceinline__ T walk(T* R, const T* Cf, int S, int lane, int first, int dir,
                                  int count, T v, T& carry) {
    // ELIM: t_k = r_k + carry * t_prev, carry <- cf_k   (elimination; v = t)
    // else: z_k = r_k + cf_k * z_prev                     (substitution; v = z)
    int i0 = 0;
    for (; i0 + SEQ <= count; i0 += SEQ) {
        T rr[SEQ], cf[SEQ];
#pragma unroll
        for (int i = 0; i < SEQ; ++i) {
            const int k = first + dir * (i0 + i);
            rr[i] = R[k * S + lane];
            cf[i] = Cf[k * S + lane];
        }
#pragma unroll
        for (int i = 0; i < SEQ; ++i) {
            if (ELIM) {
                v = rr[i] + carry * v;
                carry = cf[i];
            } else {
                v = rr[i] + cf[i] * v;
            }
            rr[i] = v;
        }
#pragma unroll
        for (int i = 0; i < SEQ; ++i) R[(first + dir * (i0 + i)) * S + lane] = rr[i];
    }
    if (i0 < count) {
        const int last = count - 1;
        T rr[SEQ], cf[SEQ];
#pragma unroll
        for (int i = 0; i < SEQ; ++i) {
            const int k = first + dir * min(i0 + i, last);
            rr[i] = R[k * S + lane];
            cf[i] = Cf[k * S + lane];
        }
#pragma unroll
        for (int i = 0; i < SEQ; ++i) {
            if (i0 + i < count) {
                if (ELIM) {
                    v = rr[i] + carry * v;
                    carry = cf[i];
                } else {
                    v = rr[i] + cf[i] * v;
                }
                rr[i] = v;
            }
        }
#pragma unroll
        for (int i = 0; i < SEQ; ++i)
            if (i0 + i < count) R[(first + dir * (i0 + i)) * S + lane] = rr[i];
    }
    return v;
}

template <typename T, int JMAX>
__device__ __forceinline__ void column_solve(T* R, T* Cf, T* E1, T* E2, const T (&mo)[JMAX],
                                             int tid, int lc, int kg, int KG, int BOT, int mid,
                                             int nz, int S, int ncol) {
    constexpr int SEQ = 8;
    // ---- phase 2: eliminate towards row mid -------------------------------
    if (tid < ncol) {
        T cp = T(0);
        const T t = walk<T, SEQ, true>(R, Cf, S, tid, 0, 1, mid, T(0), cp);
        E1[tid] = cp * t;
    } else if (tid >= BOT && tid < BOT + ncol) {
        const int l2 = tid - BOT;
        T cn = T(0);
        const T t = walk<T, SEQ, true>(R, Cf, S, l2, nz - 1, -1, nz - 1 - mid, T(0), cn);
        E2[l2] = cn * t;
    }
    __syncthreads();

    // ---- phase 3: pivot reciprocals (row mid takes both eliminations) ------
    if (lc < ncol) {
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
            const int k = kg + j * KG;
            if (k < nz) {
                T v = R[k * S + lc];
                if (k == mid) v += E1[lc] + E2[lc];
                R[k * S + lc] = mo[j] * v;
            }
        }
    }
    __syncthreads();

    // ---- phase 4: back substitution outwards from row mid ----------------
    T unused = T(0);
    if (tid < ncol) {
        walk<T, SEQ, false>(R, Cf, S, tid, mid - 1, -1, mid, R[mid * S + tid], unused);
    } else if (tid >= BOT && tid < BOT + ncol) {
        const int l2 = tid - BOT;
        walk<T, SEQ, false>(R, Cf, S, l2, mid + 1, 1, nz - 1 - mid, R[mid * S + l2], unused);
    }
    __syncthreads();
}

template <typename T, int TC_ = 32, int NT_ = kBlock>
struct SweepTile {
    static constexpr int TC = TC_;  // columns per workgroup
    static constexpr int NT = NT_;  // threads per workgroup
    static constexpr int KG = NT / TC;
    static size_t lds_bytes(int nz) { return size_t(2 * nz + 2) * TC * sizeof(T); }
};

// Waves per SIMD asked of the register allocator: the float32 sweep with
// prolongation would otherwise take 85 registers and run 5 waves per SIMD;
// held to 80 it keeps the 6 of the plain sweep (a few values spill).
template <typename T, int JMAX, int MODE, bool K2, int SC>
struct SweepWaves {
    static constexpr int value =
        (sizeof(T) == 4 && MODE == kProlong && !K2 && SC == kSym && JMAX <= 9) ? 6 : 1;
};

// NTS: b and the column factors, read once, are streamed with non-temporal
// loads (for levels much larger than the last-level cache), so that the cache
// keeps x and the face couplings, which neighbouring tiles read again, and
// x_new, which the next kernel reads.
template <typename T, int JMAX, int MODE, int TC_ = SweepTile<T>::TC, int NT = kBlock,
          int CH_ = 0, bool K2 = false, int SC = kSym, bool NTS = false>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(SweepWaves<T, JMAX, MODE, K2, SC>::value)))
k_sweep(LevelView<T> L, const T* __restrict__ b, const T* __restrict__ x,
        const T* __restrict__ xc, int nvp_c,
        T* __restrict__ y, T omega, int batch, const int* __restrict__ active, int mid,
        int rev) {
    constexpr int TC = TC_, KG = NT / TC;
    constexpr int BOT = (TC + 63) / 64 * 64;  // first lane of the bottom elimination (own wave)
    static_assert(BOT + TC <= NT, "two elimination lane groups must fit the workgroup");
    static_assert(kTile % TC == 0, "a sweep tile lies inside one storage tile");
    static_assert(!(K2 && SC != kSym), "the weighted operator has the 7-point stencil");
    constexpr bool kHasX = MODE == kPlain || MODE == kProlong;
    constexpr bool kHasP = MODE == kProlong || MODE == kProlongZero;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);  // [nz][TC]: rhs, then t, u, z
    const int ncol = L.ncol, nz = L.nz;
    T* Cf = R + nz * TC;                    // [nz][TC]: cc
    T* E1 = Cf + nz * TC;                   // [TC]: cc_{mid-1} t_{mid-1}
    T* E2 = E1 + TC;                        // [TC]: cc_{mid+1} t_{mid+1}

    const int lb = xcd_remap(blockIdx.x, gridDim.x, rev);
    const int rhs = lb % batch, tile = lb / batch;
    if (active && !active[rhs]) return;
    const int tid = threadIdx.x;
    const int lc = tid % TC, kg = tid / TC;
    const int c = tile * TC + lc;
    const bool valid = c < ncol;
    const int64_t nv = L.nvp;
    b += rhs * nv;
    y += rhs * nv;
    if (kHasX) x += rhs * nv;
    if (kHasP) xc += rhs * int64_t(nvp_c);
    const T* khN = L.kh + nv;
    const int ob = tile_base(c, nz);

    // ---- phase 1: right-hand side and factors into LDS --------------------
    // nb: tiled offsets of the neighbours; fW, fS: offsets of the W and S
    // faces in kh. Prolongation: the coarse values of the column's parent (pP)
    // and of the parents of its outward E/W (pX) and N/S (pY) neighbours; the
    // E neighbour is outward for odd i, the N neighbour for odd j, and the
    // other neighbour of each pair shares the column's parent.
    int nb[4] = {0, 0, 0, 0};
    int pP = 0, pX = 0, pY = 0;
    bool eOut = false, nOut = false;
    uint32_t fW = 0, fS = 0;
    if (MODE != kZero && valid) {
#pragma unroll
        for (int d = 0; d < 4; ++d) nb[d] = tile_base(L.nbr[d * ncol + c], nz);
        fW = L.fface[c];
        fS = L.fface[ncol + c];
        if (kHasP) {
            pP = L.pofs[c];
            pX = L.pofs[ncol + c];
            pY = L.pofs[2 * ncol + c];
            eOut = ((c % L.N) & 1) != 0;
            nOut = (((c / L.N) % L.N) & 1) != 0;
        }
    }
    auto ld = [](const T* p) -> T {
        if constexpr (NTS) return __builtin_nontemporal_load(p);
        else return *p;
    };
    // the iterate after the prolongation at level k of the column itself
    auto xown = [&](int k) -> T {
        T v = T(0);
        if (kHasX) v = x[ob + kTile * k];
        if (kHasP) v += xc[pP + kTile * k];
        return v;
    };
    // Loads of CH levels are issued together before any is used, so each
    // thread keeps several rows of independent loads in flight.
    constexpr int CH = CH_ > 0 ? CH_ : (MODE == kZero ? 8 : 2);
    T xo[JMAX], mo[JMAX];
    T so[SC == kRowWT ? JMAX : 1];  // H^T: own weight, for z / s
#pragma unroll
    for (int j0 = 0; j0 < JMAX; j0 += CH) {
        T vb[CH], vc[CH], vm[CH], vx[CH][5], vk[CH][4];
        T v2[CH];  // 9-cell: kv2_k x_{k+2} + kv2_{k-2} x_{k-2}
        T vs[CH], vsn[CH][4];  // weighted: own weight, neighbours' weights (H^T)
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
            const int j = j0 + jj;
            const int k = kg + j * KG;
            vb[jj] = vc[jj] = vm[jj] = T(0);
#pragma unroll
            for (int d = 0; d < 5; ++d) vx[jj][d] = T(0);
#pragma unroll
            for (int d = 0; d < 4; ++d) vk[jj][d] = T(0);
            v2[jj] = T(0);
            vs[jj] = T(1);
#pragma unroll
            for (int d = 0; d < 4; ++d) vsn[jj][d] = T(1);
            if (j < JMAX && k < nz && valid) {
                const int o = ob + kTile * k;
                vb[jj] = ld(b + o);
                if constexpr (SC != kSym) vs[jj] = L.s[o];
                vc[jj] = ld(L.cc + o);
                vm[jj] = ld(L.mm + o);
                if (MODE != kZero) {
                    vk[jj][0] = L.kh[o];
                    vk[jj][1] = L.kh[fW + uint32_t(kTile * k)];
                    vk[jj][2] = khN[o];
                    vk[jj][3] = L.kh[fS + uint32_t(kTile * k)];
                    T cP = T(0), cX = T(0), cY = T(0);
                    if constexpr (kHasP) {
                        cP = xc[pP + kTile * k];
                        cX = xc[pX + kTile * k];
                        cY = xc[pY + kTile * k];
                    }
                    const T pe[4] = {eOut ? cX : cP, eOut ? cP : cX, nOut ? cY : cP,
                                     nOut ? cP : cY};
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        T v = T(0);
                        if (kHasX) v = x[nb[d] + kTile * k];
                        if (kHasP) v += pe[d];
                        vx[jj][d] = v;
                    }
                    {
                        T v = T(0);
                        if (kHasX) v = x[ob + kTile * k];
                        if (kHasP) v += cP;
                        vx[jj][4] = v;
                    }
                    if constexpr (SC == kRowWT) {
#pragma unroll
                        for (int d = 0; d < 4; ++d) vsn[jj][d] = L.s[nb[d] + kTile * k];
                    }
                    if constexpr (K2) {
                        if (k + 2 < nz) v2[jj] = L.kv2[o] * xown(k + 2);
                        if (k >= 2) v2[jj] += L.kv2[o - 2 * kTile] * xown(k - 2);
                    }
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
            const int j = j0 + jj;
            const int k = kg + j * KG;
            if (j < JMAX && k < nz) {
                T r = vb[jj];
                if constexpr (SC == kRowW) r = vb[jj] / vs[jj];
                if constexpr (SC == kRowWT) {
                    so[j] = vs[jj];
                    if (MODE != kZero)
                        r += vk[jj][0] * (vsn[jj][0] * vx[jj][0]) +
                             vk[jj][1] * (vsn[jj][1] * vx[jj][1]) +
                             vk[jj][2] * (vsn[jj][2] * vx[jj][2]) +
                             vk[jj][3] * (vsn[jj][3] * vx[jj][3]);
                } else if (MODE != kZero) {
                    r += vk[jj][0] * vx[jj][0] + vk[jj][1] * vx[jj][1] + vk[jj][2] * vx[jj][2] +
                         vk[jj][3] * vx[jj][3];
                }
                if (K2 && MODE != kZero) r += v2[jj];
                xo[j] = vx[jj][4];
                mo[j] = vm[jj];
                R[k * TC + lc] = r;
                Cf[k * TC + lc] = vc[jj];
            }
        }
    }
    __syncthreads();

    column_solve<T, JMAX>(R, Cf, E1, E2, mo, tid, lc, kg, KG, BOT, mid, nz, TC, TC);

    // ---- phase 5: relaxation and store -------------------------------------
    if (!valid) return;
    const T om = omega, om1 = T(1) - omega;
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
        const int k = kg + j * KG;
        if (k < nz) {
            T z = R[k * TC + lc];
            if constexpr (SC == kRowWT) z = z / so[j];
            const T v = (MODE == kZero) ? om * z : om1 * xo[j] + om * z;
            y[ob + kTile * k] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Operator apply y = H x in flux form (no cancellation of the large vertical
// couplings against the diagonal). One thread per (column, chunk of KC
// levels); all loads of the chunk are issued before any arithmetic.
// DOT additionally writes per-block partial sums of x . y (float64) for the
// Krylov loop.
// Sum over the block; the result is valid in thread 0. Fixed order, so
// repeated runs give identical bits.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();  // earlier readers of sh are done
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < int(blockDim.x >> 6); ++i) s += sh[i];
    }
    return s;
}

// Per right-hand-side scalars sc[rhs*kScal + ...] (kBreak: 1 after a
// BiCGStab breakdown):
enum { kBB = 0, kRho = 1, kPQ = 2, kAlpha = 3, kRR = 4, kBeta = 5, kZQ = 6, kRtol2 = 7,
       kOmega = 8, kBreak = 9, kScal = 12 };
// CG: BB, then per iteration Rho/Alpha/RR/Beta(Flex). BiCGStab: BB, then per
// iteration BiAlpha (rho / (r0, v)), BiOmega ((t, s) / (t, t)) and BiRR
// ((r0, r), ||r||^2, convergence test, beta for the next step).
enum FinalizeMode { kFinBB = 0, kFinRho = 1, kFinAlpha = 2, kFinRR = 3, kFinBeta = 4,
                    kFinBetaFlex = 5, kFinBiAlpha = 6, kFinBiOmega = 7, kFinBiRR = 8 };

// Reduction state shared by the Krylov kernels. hsc/hact/hseq live in pinned,
// host-coherent memory: the finalisation of the norm reductions publishes the
// scalars there and then the sequence number, which the host polls.
struct CgState {
    double* partial;   // [B][pstride]
    double* partial2;  // [B][pstride]
    int pstride;
    double* sc;        // [B][8]
    int* active;       // [B]
    int* upd;          // [B] CG: the last residual update included the rhs
    double* hsc;       // host mirror [B][8]
    int* hact;         // host mirror [B]
    int* hseq;         // host mirror [B]
};

__device__ __forceinline__ void grid_range(int64_t n, int nblk, int blk, int64_t& i0, int64_t& i1) {
    const int64_t per = (n + nblk - 1) / nblk;
    i0 = min(n, int64_t(blk) * per);
    i1 = min(n, i0 + per);
}

// Sum `cnt` partials in a fixed order (result in every thread). Four
// independent accumulators per thread keep several loads in flight.
__device__ __forceinline__ double reduce_partials(const double* part, int cnt, double* sh) {
    const int step = blockDim.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * step < cnt; i += 4 * step) {
        a0 += part[i];
        a1 += part[i + step];
        a2 += part[i + 2 * step];
        a3 += part[i + 3 * step];
    }
    for (; i < cnt; i += step) a0 += part[i];
    const double s = block_sum((a0 + a1) + (a2 + a3), sh);
    __syncthreads();
    if (threadIdx.x == 0) sh[0] = s;
    __syncthreads();
    return sh[0];
}

// Store this block's partial sum(s) of a reduction.
__device__ __forceinline__ void store_partial(const CgState& st, int rhs, int blk, double s1,
                                              double s2, bool two) {
    if (threadIdx.x == 0) {
        st.partial[int64_t(rhs) * st.pstride + blk] = s1;
        if (two) st.partial2[int64_t(rhs) * st.pstride + blk] = s2;
    }
}

// One block per right-hand side: add the `cnt` partials in a fixed order and
// derive the Krylov scalar. The norm reductions (kFinBB, kFinRR, kFinBiRR)
// also publish the scalars and flags to the host mirror, then the sequence
// number `seq`; they publish even for a right-hand side that is no longer
// active (its values unchanged), so the host never waits in vain.
constexpr int kFinBlock = 1024;  // threads of the finalisation block

__global__ void __launch_bounds__(kFinBlock)
k_finalize(CgState st, int mode, int cnt, int seq) {
    __shared__ double sh[kFinBlock / 64];
    const int rhs = blockIdx.x;
    const bool publish = mode == kFinBB || mode == kFinRR || mode == kFinBiRR;
    const bool live = mode == kFinBB || st.active[rhs] != 0;
    if (!live && !publish) return;
    const bool two = mode == kFinBetaFlex || mode == kFinBiOmega || mode == kFinBiRR;
    double t1 = 0.0, t2 = 0.0;
    if (live) {
        t1 = reduce_partials(st.partial + int64_t(rhs) * st.pstride, cnt, sh);
        if (two) t2 = reduce_partials(st.partial2 + int64_t(rhs) * st.pstride, cnt, sh);
    }
    if (threadIdx.x != 0) return;
    double* v = st.sc + rhs * kScal;
    // CG: an x update is owed exactly where r was updated
    if (mode == kFinRR) st.upd[rhs] = live ? 1 : 0;
    switch (live ? mode : -1) {
        case kFinBB:
            v[kBB] = t1;
            v[kRR] = t1;
            v[kRho] = t1;  // BiCGStab: (r0, r) with r0 = r = b
            st.active[rhs] = (t1 > 0.0) ? 1 : 0;
            break;
        case kFinRho:
            v[kRho] = t1;
            break;
        case kFinAlpha:
            v[kPQ] = t1;
            v[kAlpha] = v[kRho] / t1;
            break;
        case kFinRR:
            v[kRR] = t1;
            if (t1 <= v[kRtol2] * v[kBB]) st.active[rhs] = 0;
            break;
        case kFinBeta:
            v[kBeta] = t1 / v[kRho];
            v[kRho] = t1;
            break;
        case kFinBetaFlex:
            // Polak-Ribiere: z.(r_new - r_old) / rho with r_new - r_old = -alpha q
            v[kBeta] = -v[kAlpha] * t2 / v[kRho];
            v[kZQ] = t2;
            v[kRho] = t1;
            break;
        case kFinBiAlpha:  // t1 = (r0, v)
            if (t1 == 0.0) {
                v[kBreak] = 1.0;
                st.active[rhs] = 0;
            } else {
                v[kAlpha] = v[kRho] / t1;
            }
            break;
        case kFinBiOmega:  // t1 = (t, s), t2 = (t, t); t = 0 only if s = 0
            v[kOmega] = t2 > 0.0 ? t1 / t2 : 0.0;
            break;
        case kFinBiRR:  // t1 = (r0, r), t2 = ||r||^2
            v[kRR] = t2;
            if (t2 <= v[kRtol2] * v[kBB]) {
                st.active[rhs] = 0;
            } else if (t1 == 0.0 || v[kOmega] == 0.0) {
                v[kBreak] = 1.0;
                st.active[rhs] = 0;
            } else {
                v[kBeta] = (t1 / v[kRho]) * (v[kAlpha] / v[kOmega]);
                v[kRho] = t1;
            }
            break;
        default:
            break;
    }
    if (publish) {
        for (int i = 0; i < kScal; ++i) st.hsc[rhs * kScal + i] = v[i];
        st.hact[rhs] = st.active[rhs];
        __threadfence_system();
        __hip_atomic_store(&st.hseq[rhs], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// DOT: 0 none; kDotXY x . y (CG: p . q); kDotWY w . y (BiCGStab: (r0, v));
// kDotWYYY w . y and y . y (BiCGStab: (t, s), (t, t)). Partial sums per block.
enum { kDotNone = 0, kDotXY = 1, kDotWY = 2, kDotWYYY = 3 };

// NTS: delta (read once) and y bypass the last-level cache (for levels far
// larger than it; see k_sweep).
template <typename T, int DOT, int KC, bool K2 = false, int SC = kSym, bool NTS = false>
__global__ void __launch_bounds__(kBlock)
k_apply(LevelView<T> L, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ w,
        int batch, int nkc, CgState st, const int* __restrict__ active, int rev) {
    __shared__ double sh[kBlock / 64];
    const int lb = xcd_remap(blockIdx.x, gridDim.x, rev);
    const int rhs = lb % batch, rest = lb / batch;
    const int kc = rest % nkc, tile = rest / nkc;
    if (active && !active[rhs]) return;
    const int ncol = L.ncol, nz = L.nz;
    const int c = tile * kBlock + threadIdx.x;
    const bool valid = c < ncol;
    const int64_t nv = L.nvp;
    x += rhs * nv;
    y += rhs * nv;
    if (DOT >= kDotWY) w += rhs * nv;
    const T* khN = L.kh + nv;
    double acc = 0.0, acc2 = 0.0;
    if (valid) {
        int nb[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) nb[d] = tile_base(L.nbr[d * ncol + c], nz);
        const uint32_t fW = L.fface[c], fS = L.fface[ncol + c];
        const int ob = tile_base(c, nz);
        const int k0 = kc * KC;
        // all loads of the chunk are issued before any is used
        T xc[KC + 2], kvv[KC + 1], dl[KC], xn[KC][4], kh[KC][4];
        // weighted operator: own weights at k0-1 .. k0+KC (as xc) and, for
        // H^T, the neighbours' weights
        T sc[KC + 2], sn[KC][4];
#pragma unroll
        for (int j = 0; j < KC + 2; ++j) {
            const int k = k0 - 1 + j;
            xc[j] = (k >= 0 && k < nz) ? x[ob + kTile * k] : T(0);
            sc[j] = T(1);
            if (SC != kSym && k >= 0 && k < nz) sc[j] = L.s[ob + kTile * k];
        }
#pragma unroll
        for (int j = 0; j < KC + 1; ++j) {
            const int k = k0 - 1 + j;
            kvv[j] = (k >= 0 && k < nz) ? L.kv[ob + kTile * k] : T(0);
        }
        // 9-cell: x at k0-2 and k0+KC+1 (xc holds k0-1 .. k0+KC), kv2 at
        // k0-2 .. k0+KC-1
        T xlo = T(0), xhi = T(0), k2v[KC + 2];
        if constexpr (K2) {
            if (k0 >= 2) xlo = x[ob + kTile * (k0 - 2)];
            if (k0 + KC + 1 < nz) xhi = x[ob + kTile * (k0 + KC + 1)];
#pragma unroll
            for (int j = 0; j < KC + 2; ++j) {
                const int k = k0 - 2 + j;
                k2v[j] = (k >= 0 && k < nz) ? L.kv2[ob + kTile * k] : T(0);
            }
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = k0 + j;
            dl[j] = T(0);
#pragma unroll
            for (int d = 0; d < 4; ++d) xn[j][d] = kh[j][d] = T(0);
            if (k < nz) {
                const int o = ob + kTile * k;
                if constexpr (NTS) dl[j] = __builtin_nontemporal_load(L.dl + o);
                else dl[j] = L.dl[o];
#pragma unroll
                for (int d = 0; d < 4; ++d) xn[j][d] = x[nb[d] + kTile * k];
#pragma unroll
                for (int d = 0; d < 4; ++d) sn[j][d] = SC == kRowWT ? L.s[nb[d] + kTile * k] : T(1);
                kh[j][0] = L.kh[o];
                kh[j][1] = L.kh[fW + uint32_t(kTile * k)];
                kh[j][2] = khN[o];
                kh[j][3] = L.kh[fS + uint32_t(kTile * k)];
            }
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int k = k0 + j;
            if (k < nz) {
                const T xo = xc[j + 1];
                T v = dl[j] * xo;
                if constexpr (SC == kRowWT) {
                    // H^T x = delta x + L (s x)
                    const T uo = sc[j + 1] * xo;
#pragma unroll
                    for (int d = 0; d < 4; ++d) v += kh[j][d] * (uo - sn[j][d] * xn[j][d]);
                    v += kvv[j + 1] * (uo - sc[j + 2] * xc[j + 2]);
                    v += kvv[j] * (uo - sc[j] * xc[j]);
                } else if constexpr (SC == kRowW) {
                    // H x = delta x + s (L x)
                    T f = T(0);
#pragma unroll
                    for (int d = 0; d < 4; ++d) f += kh[j][d] * (xo - xn[j][d]);
                    f += kvv[j + 1] * (xo - xc[j + 2]);
                    f += kvv[j] * (xo - xc[j]);
                    v += sc[j + 1] * f;
                } else {
#pragma unroll
                    for (int d = 0; d < 4; ++d) v += kh[j][d] * (xo - xn[j][d]);
                    v += kvv[j + 1] * (xo - xc[j + 2]);
                    v += kvv[j] * (xo - xc[j]);
                }
                if constexpr (K2) {
                    // x[k-2] and x[k+2] (xc[i] holds x[k0-1+i])
                    const T xm2 = j >= 1 ? xc[j - 1] : xlo;
                    const T xp2 = j + 3 <= KC + 1 ? xc[j + 3] : xhi;
                    v += k2v[j + 2] * (xo - xp2);
                    v += k2v[j] * (xo - xm2);
                }
                if constexpr (NTS) __builtin_nontemporal_store(v, y + ob + kTile * k);
                else y[ob + kTile * k] = v;
                if (DOT == kDotXY) acc += double(xo) * double(v);
                if (DOT >= kDotWY) acc += double(w[ob + kTile * k]) * double(v);
                if (DOT == kDotWYYY) acc2 += double(v) * double(v);
            }
        }
    }
    if (DOT != kDotNone) {
        const double s = block_sum(acc, sh);
        double s2 = 0.0;
        if (DOT == kDotWYYY) {
            __syncthreads();
            s2 = block_sum(acc2, sh);
        }
        store_partial(st, rhs, rest, s, s2, DOT == kDotWYYY);
    }
}

// The operator apply of the symmetric 7-point operator with the neighbours'
// values exchanged in LDS (panels whose width is a multiple of PX, 32 or 64).
// One workgroup owns a PX x PY patch of columns of one panel
// (PX PY = kBlock, each patch row one storage tile) and a chunk of KC levels;
// thread t = pi + PX pj owns column (i, j), whose W, E, S, N neighbours are
// threads t - 1, t + 1, t - PX, t + PX. All loads of the chunk are issued
// first; then each thread publishes its x and its E and N faces (the W face
// of a column is the E face of its W neighbour, the S face the N face of its S
// neighbour) and, after one barrier, takes its neighbours' values from LDS;
// only the patch's edge columns gather from global memory. In k_apply those
// gathers cost 31 of 172 us at C192 x 70 (measured by skipping them): the N
// and S ones often miss L2, and the E and W ones, shifted by one element,
// touch an extra line per wave. Here: 162 us with 64 x 4 patches, 163 with
// 32 x 8 (patches walked column by column: 168 us). y is computed by the same
// expression as in k_apply and is identical; the partial sums of the dot
// products follow the patches.
template <typename T, int DOT, int KC, bool NTS, int PX, bool K2 = false>
__global__ void __launch_bounds__(kBlock)
k_apply_lds(LevelView<T> L, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ w,
            int batch, int nkc, CgState st, const int* __restrict__ active, int rev) {
    constexpr int PY = kBlock / PX;
    static_assert(PX * PY == kBlock && PX % kTile == 0, "patch rows are whole storage tiles");
    __shared__ T lx[KC][kBlock];   // x at k0 .. k0 + KC - 1
    __shared__ T lfe[KC][kBlock];  // E faces
    __shared__ T lfn[KC][kBlock];  // N faces
    __shared__ double sh[kBlock / 64];
    const int lb = xcd_remap(blockIdx.x, gridDim.x, rev);
    const int rhs = lb % batch, rest = lb / batch;
    const int kc = rest % nkc, tile = rest / nkc;
    if (active && !active[rhs]) return;  // the whole workgroup
    const int t = threadIdx.x, pi = t % PX, pj = t / PX;
    const int N = L.N, pwx = N / PX, npp = pwx * (N / PY);
    const int pan = tile / npp, q = tile % npp;
    // every column of a patch exists, so no thread leaves before the barrier
    const int c = (pan * N + (q / pwx) * PY + pj) * N + (q % pwx) * PX + pi;
    const bool eW = pi == 0, eE = pi == PX - 1, eS = pj == 0, eN = pj == PY - 1;
    const int ncol = L.ncol, nz = L.nz;
    const int64_t nv = L.nvp;
    x += rhs * nv;
    y += rhs * nv;
    if (DOT >= kDotWY) w += rhs * nv;
    const T* khN = L.kh + nv;
    const int ob = tile_base(c, nz);
    // neighbours in the order of the nbr table (E, W, N, S); only the edge
    // columns look theirs up
    int nb[4] = {0, 0, 0, 0};
    uint32_t fW = 0, fS = 0;
    if (eE) nb[0] = tile_base(L.nbr[0 * ncol + c], nz);
    if (eW) {
        nb[1] = tile_base(L.nbr[1 * ncol + c], nz);
        fW = L.fface[c];
    }
    if (eN) nb[2] = tile_base(L.nbr[2 * ncol + c], nz);
    if (eS) {
        nb[3] = tile_base(L.nbr[3 * ncol + c], nz);
        fS = L.fface[ncol + c];
    }
    const bool edge[4] = {eE, eW, eN, eS};
    const int k0 = kc * KC;
    T xc[KC + 2], kvv[KC + 1], dl[KC], xn[KC][4], kh[KC][4];
#pragma unroll
    for (int j = 0; j < KC + 2; ++j) {
        const int k = k0 - 1 + j;
        xc[j] = (k >= 0 && k < nz) ? x[ob + kTile * k] : T(0);
    }
#pragma unroll
    for (int j = 0; j < KC + 1; ++j) {
        const int k = k0 - 1 + j;
        kvv[j] = (k >= 0 && k < nz) ? L.kv[ob + kTile * k] : T(0);
    }
    // 9-cell: x at k0-2 and k0+KC+1 (xc holds k0-1 .. k0+KC), kv2 at
    // k0-2 .. k0+KC-1
    T xlo = T(0), xhi = T(0), k2v[KC + 2];
    if constexpr (K2) {
        if (k0 >= 2) xlo = x[ob + kTile * (k0 - 2)];
        if (k0 + KC + 1 < nz) xhi = x[ob + kTile * (k0 + KC + 1)];
#pragma unroll
        for (int j = 0; j < KC + 2; ++j) {
            const int k = k0 - 2 + j;
            k2v[j] = (k >= 0 && k < nz) ? L.kv2[ob + kTile * k] : T(0);
        }
    }
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        const int k = k0 + j;
        dl[j] = T(0);
#pragma unroll
        for (int d = 0; d < 4; ++d) xn[j][d] = kh[j][d] = T(0);
        if (k < nz) {
            const int o = ob + kTile * k;
            if constexpr (NTS) dl[j] = __builtin_nontemporal_load(L.dl + o);
            else dl[j] = L.dl[o];
            kh[j][0] = L.kh[o];
            kh[j][2] = khN[o];
#pragma unroll
            for (int d = 0; d < 4; ++d)
                if (edge[d]) xn[j][d] = x[nb[d] + kTile * k];
            if (eW) kh[j][1] = L.kh[fW + uint32_t(kTile * k)];
            if (eS) kh[j][3] = L.kh[fS + uint32_t(kTile * k)];
        }
    }
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        lx[j][t] = xc[j + 1];
        lfe[j][t] = kh[j][0];
        lfn[j][t] = kh[j][2];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        if (!eE) xn[j][0] = lx[j][t + 1];
        if (!eW) {
            xn[j][1] = lx[j][t - 1];
            kh[j][1] = lfe[j][t - 1];
        }
        if (!eN) xn[j][2] = lx[j][t + PX];
        if (!eS) {
            xn[j][3] = lx[j][t - PX];
            kh[j][3] = lfn[j][t - PX];
        }
    }
    double acc = 0.0, acc2 = 0.0;
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        const int k = k0 + j;
        if (k < nz) {
            const T xo = xc[j + 1];
            T v = dl[j] * xo;
#pragma unroll
            for (int d = 0; d < 4; ++d) v += kh[j][d] * (xo - xn[j][d]);
            v += kvv[j + 1] * (xo - xc[j + 2]);
            v += kvv[j] * (xo - xc[j]);
            if constexpr (K2) {
                const T xm2 = j >= 1 ? xc[j - 1] : xlo;
                const T xp2 = j + 3 <= KC + 1 ? xc[j + 3] : xhi;
                v += k2v[j + 2] * (xo - xp2);
                v += k2v[j] * (xo - xm2);
            }
            if constexpr (NTS) __builtin_nontemporal_store(v, y + ob + kTile * k);
            else y[ob + kTile * k] = v;
            if (DOT == kDotXY) acc += double(xo) * double(v);
            if (DOT >= kDotWY) acc += double(w[ob + kTile * k]) * double(v);
            if (DOT == kDotWYYY) acc2 += double(v) * double(v);
        }
    }
    if (DOT != kDotNone) {
        const double s = block_sum(acc, sh);
        double s2 = 0.0;
        if (DOT == kDotWYYY) {
            __syncthreads();
            s2 = block_sum(acc2, sh);
        }
        store_partial(st, rhs, rest, s, s2, DOT == kDotWYYY);
    }
}

// ---------------------------------------------------------------------------
// Residual and restriction fused (Algorithm 1): bc[k][C] = sum over the four
// children ch of C of (b - H x)[k][ch]. The sum has no averaging factor:
// restriction is the dual of injection (Section 3.6). In that sum the flux
// through each of the four faces between siblings enters twice with opposite
// signs, so only the eight faces on the boundary of the coarse cell are
// evaluated:
//   bc = sum b - sum delta x - sum_{8 outer faces} K (x_in - x_out)
//        - sum over children of the vertical fluxes.
// One thread per (coarse column, chunk of KC levels); ZEROX: x = 0, bc = R b.
// Children (0,0),(1,0) and (0,1),(1,1) are adjacent pairs in memory (same
// panel row, even first index, so the same tile); PAIR loads each pair with
// one vector load (the host uses it when b and x are aligned to two elements).
template <typename T>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float2;
};
template <>
struct Vec2<double> {
    using type = double2;
};

template <typename T, bool PAIR>
__device__ __forceinline__ void load_pair(const T* __restrict__ p, int64_t i, T& a, T& c) {
    if (PAIR) {
        const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type*>(p + i);
        a = v.x;
        c = v.y;
    } else {
        a = p[i];
        c = p[i + 1];
    }
}

// The same with non-temporal loads, for a stream that is read exactly once.
template <typename T, bool PAIR>
__device__ __forceinline__ void load_pair_nt(const T* __restrict__ p, int64_t i, T& a, T& c) {
    if (PAIR) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p + i));
        a = v.x;
        c = v.y;
    } else {
        a = __builtin_nontemporal_load(p + i);
        c = __builtin_nontemporal_load(p + i + 1);
    }
}

// NTS: b and delta, each read exactly once, bypass the last-level cache (for
// levels far larger than it; see k_sweep).
template <typename T, bool ZEROX, bool PAIR, bool K2 = false, int SC = kSym, bool NTS = false>
__global__ void __launch_bounds__(kBlock)
k_resid_restrict(LevelView<T> F, const int32_t* __restrict__ child, int ncol_c, int nvp_c,
                 const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ bc,
                 int batch, int kchunk, int nkc, const int* __restrict__ active, int rev) {
    const int lb = xcd_remap(blockIdx.x, gridDim.x, rev);
    const int rhs = lb % batch, rest = lb / batch;
    const int kc = rest % nkc, tile = rest / nkc;
    if (active && !active[rhs]) return;
    const int C = tile * kBlock + threadIdx.x;
    if (C >= ncol_c) return;
    const int ncol = F.ncol, nz = F.nz;
    const int64_t nv = F.nvp;
    b += rhs * nv;
    if (!ZEROX) x += rhs * nv;
    bc += rhs * int64_t(nvp_c) + tile_base(C, nz);
    auto load_once = [](const T* p, int64_t i, T& a, T& c) {
        if constexpr (NTS) load_pair_nt<T, PAIR>(p, i, a, c);
        else load_pair<T, PAIR>(p, i, a, c);
    };
    // children (0,0), (1,0) share a tile and are adjacent, as are (0,1), (1,1)
    int ch[4], cb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ch[s] = child[s * ncol_c + C];
        cb[s] = tile_base(ch[s], nz);
    }
    const int k0 = kc * kchunk, k1 = min(nz, k0 + kchunk);
    if (ZEROX) {
        for (int k = k0; k < k1; ++k) {
            const int r = kTile * k;
            T v0, v1, v2, v3;
            load_once(b, r + cb[0], v0, v1);
            load_once(b, r + cb[2], v2, v3);
            bc[r] = ((v0 + v1) + v2) + v3;
        }
        return;
    }
    // outer faces: tiled offset of the outside column and offset of the face
    // in kh, two per child in child order:
    //   child (0,0): W, S   child (1,0): E, S   child (0,1): W, N   child (1,1): E, N
    int out[8];
    uint32_t fc[8];
    {
        const int c00 = ch[0], c10 = ch[1], c01 = ch[2], c11 = ch[3];
        const uint32_t nvu = uint32_t(nv);
        out[0] = F.nbr[1 * ncol + c00]; fc[0] = F.fface[c00];
        out[1] = F.nbr[3 * ncol + c00]; fc[1] = F.fface[ncol + c00];
        out[2] = F.nbr[0 * ncol + c10]; fc[2] = uint32_t(cb[1]);
        out[3] = F.nbr[3 * ncol + c10]; fc[3] = F.fface[ncol + c10];
        out[4] = F.nbr[1 * ncol + c01]; fc[4] = F.fface[c01];
        out[5] = F.nbr[2 * ncol + c01]; fc[5] = nvu + uint32_t(cb[2]);
        out[6] = F.nbr[0 * ncol + c11]; fc[6] = uint32_t(cb[3]);
        out[7] = F.nbr[2 * ncol + c11]; fc[7] = nvu + uint32_t(cb[3]);
#pragma unroll
        for (int f = 0; f < 8; ++f) out[f] = tile_base(out[f], nz);
    }
    static_assert(!(K2 && SC != kSym), "the weighted operator has the 7-point stencil");
    // H^T: the flux terms act on u = s x, so every x below is multiplied by its
    // weight; H: each child's flux terms are weighted by its own s, so the
    // fluxes between siblings no longer cancel and are evaluated too.
    auto su = [&](T& v0, T& v1, int off) {
        if constexpr (SC == kRowWT) {
            T w0, w1;
            load_pair<T, PAIR>(F.s, off, w0, w1);
            v0 *= w0;
            v1 *= w1;
        }
    };
    T xdn[4] = {T(0), T(0), T(0), T(0)}, xo[4], kvdn[4] = {T(0), T(0), T(0), T(0)};
    if (k0 > 0) {
        const int rdn = kTile * (k0 - 1);
        load_pair<T, PAIR>(x, rdn + cb[0], xdn[0], xdn[1]);
        load_pair<T, PAIR>(x, rdn + cb[2], xdn[2], xdn[3]);
        su(xdn[0], xdn[1], rdn + cb[0]);
        su(xdn[2], xdn[3], rdn + cb[2]);
        load_pair<T, PAIR>(F.kv, rdn + cb[0], kvdn[0], kvdn[1]);
        load_pair<T, PAIR>(F.kv, rdn + cb[2], kvdn[2], kvdn[3]);
    }
    load_pair<T, PAIR>(x, kTile * k0 + cb[0], xo[0], xo[1]);
    load_pair<T, PAIR>(x, kTile * k0 + cb[2], xo[2], xo[3]);
    // (H^T: xo holds u = s x; the delta term needs x itself, kept in xr)
    T xr[4] = {xo[0], xo[1], xo[2], xo[3]};
    su(xo[0], xo[1], kTile * k0 + cb[0]);
    su(xo[2], xo[3], kTile * k0 + cb[2]);
    // 9-cell: window x[k-2], kv2[k-2], kv2[k-1] of the four children
    T xm2[4] = {T(0), T(0), T(0), T(0)}, k2m2[4] = {T(0), T(0), T(0), T(0)};
    T k2m1[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (K2) {
        if (k0 >= 2) {
            const int r2 = kTile * (k0 - 2);
            load_pair<T, PAIR>(x, r2 + cb[0], xm2[0], xm2[1]);
            load_pair<T, PAIR>(x, r2 + cb[2], xm2[2], xm2[3]);
            load_pair<T, PAIR>(F.kv2, r2 + cb[0], k2m2[0], k2m2[1]);
            load_pair<T, PAIR>(F.kv2, r2 + cb[2], k2m2[2], k2m2[3]);
        }
        if (k0 >= 1) {
            const int r1 = kTile * (k0 - 1);
            load_pair<T, PAIR>(F.kv2, r1 + cb[0], k2m1[0], k2m1[1]);
            load_pair<T, PAIR>(F.kv2, r1 + cb[2], k2m1[2], k2m1[3]);
        }
    }
    // two levels per step: the loads of the second are issued with the first's
#pragma unroll 2
    for (int k = k0; k < k1; ++k) {
        const int r = kTile * k;
        T xup[4] = {T(0), T(0), T(0), T(0)}, vb[4], vd[4], vkv[4], vxo[8], vk[8];
        T xupr[4] = {T(0), T(0), T(0), T(0)};  // H^T: raw x at k+1
        if (k + 1 < nz) {
            load_pair<T, PAIR>(x, r + kTile + cb[0], xup[0], xup[1]);
            load_pair<T, PAIR>(x, r + kTile + cb[2], xup[2], xup[3]);
            if constexpr (SC == kRowWT) {
#pragma unroll
                for (int q = 0; q < 4; ++q) xupr[q] = xup[q];
                su(xup[0], xup[1], r + kTile + cb[0]);
                su(xup[2], xup[3], r + kTile + cb[2]);
            }
        }
        load_once(b, r + cb[0], vb[0], vb[1]);
        load_once(b, r + cb[2], vb[2], vb[3]);
        load_once(F.dl, r + cb[0], vd[0], vd[1]);
        load_once(F.dl, r + cb[2], vd[2], vd[3]);
        load_pair<T, PAIR>(F.kv, r + cb[0], vkv[0], vkv[1]);
        load_pair<T, PAIR>(F.kv, r + cb[2], vkv[2], vkv[3]);
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            vxo[f] = x[out[f] + r];
            if constexpr (SC == kRowWT) vxo[f] *= F.s[out[f] + r];
            vk[f] = F.kh[fc[f] + uint32_t(r)];
        }
        T acc = ((vb[0] + vb[1]) + vb[2]) + vb[3];
        if constexpr (SC == kRowW) {
            // each child's flux row, with the four faces between siblings:
            // c00|c10 and c01|c11 (E faces of c00, c01), c00|c01 and c10|c11
            // (N faces of c00, c10)
            T sw[4], iE0, iE1, iN0, iN1, unused;
            load_pair<T, PAIR>(F.s, r + cb[0], sw[0], sw[1]);
            load_pair<T, PAIR>(F.s, r + cb[2], sw[2], sw[3]);
            load_pair<T, PAIR>(F.kh, r + cb[0], iE0, unused);
            load_pair<T, PAIR>(F.kh, r + cb[2], iE1, unused);
            load_pair<T, PAIR>(F.kh + nv, r + cb[0], iN0, iN1);
            T Lr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Lr[q] = vkv[q] * (xo[q] - xup[q]) + kvdn[q] * (xo[q] - xdn[q]);
#pragma unroll
            for (int f = 0; f < 8; ++f) Lr[f >> 1] += vk[f] * (xo[f >> 1] - vxo[f]);
            Lr[0] += iE0 * (xo[0] - xo[1]) + iN0 * (xo[0] - xo[2]);
            Lr[1] += iE0 * (xo[1] - xo[0]) + iN1 * (xo[1] - xo[3]);
            Lr[2] += iE1 * (xo[2] - xo[3]) + iN0 * (xo[2] - xo[0]);
            Lr[3] += iE1 * (xo[3] - xo[2]) + iN1 * (xo[3] - xo[1]);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc -= vd[q] * xo[q] + sw[q] * Lr[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc -= vd[q] * (SC == kRowWT ? xr[q] : xo[q]);
                acc -= vkv[q] * (xo[q] - xup[q]) + kvdn[q] * (xo[q] - xdn[q]);
            }
#pragma unroll
            for (int f = 0; f < 8; ++f) acc -= vk[f] * (xo[f >> 1] - vxo[f]);
        }
        T k2[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (K2) {
            T xp2[4] = {T(0), T(0), T(0), T(0)};
            if (k + 2 < nz) {
                load_pair<T, PAIR>(x, r + 2 * kTile + cb[0], xp2[0], xp2[1]);
                load_pair<T, PAIR>(x, r + 2 * kTile + cb[2], xp2[2], xp2[3]);
            }
            load_pair<T, PAIR>(F.kv2, r + cb[0], k2[0], k2[1]);
            load_pair<T, PAIR>(F.kv2, r + cb[2], k2[2], k2[3]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc -= k2[s] * (xo[s] - xp2[s]) + k2m2[s] * (xo[s] - xm2[s]);
        }
        bc[r] = acc;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if constexpr (K2) {
                xm2[s] = xdn[s];
                k2m2[s] = k2m1[s];
                k2m1[s] = k2[s];
            }
            xdn[s] = xo[s];
            xo[s] = xup[s];
            if constexpr (SC == kRowWT) xr[s] = xupr[s];
            kvdn[s] = vkv[s];
        }
    }
}

// Residual and restriction with the children's values exchanged in LDS (the
// symmetric 7-point operator on coarse panels whose width is a multiple of
// PX). One workgroup owns a PX x PY patch of coarse cells of one panel
// (PX PY = kBlock) and a chunk of levels; thread t = pi + PX pj owns cell
// (I, J) of the patch, whose W, E, S, N neighbours are threads t - 1, t + 1,
// t - PX, t + PX (inside a panel the E, N neighbour of column (i, j) is
// (i + 1, j), (i, j + 1), and cell (I, J) has children (2I + di, 2J + dj)).
// At every level each thread publishes the x of its four children and the
// faces it owns (E faces of its east children, N faces of its north
// children); the eight outer x and four outer faces a cell needs then come
// from its neighbours, and only the cells on the patch's edges read theirs
// from global memory. In k_resid_restrict those reads are gathers from rows
// that other waves or workgroups load at other times, and a third of them
// found the line gone from L2 (1.28x the kernel's words at C192 x 70). A
// patch twice as wide as high (32 x 8) has half the W and E edge cells of a
// square one, each of which reads a whole line for one value: at C192 x 70,
// float32, 88.7 us (k_resid_restrict) -> 76.6 (16 x 16) -> 71.8 us (32 x 8).
// Same arithmetic, in the same order, as k_resid_restrict: the results are
// identical.
template <typename T, bool NTS, int PX, bool K2 = false, int SC = kSym>
__global__ void __launch_bounds__(kBlock)
k_resid_restrict_lds(LevelView<T> F, const int32_t* __restrict__ child, int ncol_c, int nvp_c,
                     const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ bc,
                     int batch, int kchunk, int nkc, const int* __restrict__ active, int rev) {
    // [level parity][value][thread]: x of children 00, 10, 01, 11 (H^T:
    // u = s x, the values its fluxes act on); then the E faces of 10, 11 and
    // the N faces of 01, 11
    static_assert(!(K2 && SC != kSym), "the weighted operator has the 7-point stencil");
    __shared__ T lx[2][4][kBlock];
    __shared__ T lf[2][4][kBlock];
    constexpr int PY = kBlock / PX;
    static_assert(PX * PY == kBlock, "a patch is one workgroup");
    const int lb = xcd_remap(blockIdx.x, gridDim.x, rev);
    const int rhs = lb % batch, rest = lb / batch;
    const int kc = rest % nkc, tile = rest / nkc;
    if (active && !active[rhs]) return;  // the whole workgroup
    const int t = threadIdx.x, pi = t % PX, pj = t / PX;
    const int Nc = F.N >> 1, pwx = Nc / PX, npp = pwx * (Nc / PY);
    const int pan = tile / npp, q = tile % npp;
    // every cell of a patch exists (ncol_c = 6 Nc^2 is a multiple of kBlock),
    // so no thread leaves before the barriers
    const int C = (pan * Nc + (q / pwx) * PY + pj) * Nc + (q % pwx) * PX + pi;
    const bool eW = pi == 0, eE = pi == PX - 1, eS = pj == 0, eN = pj == PY - 1;
    const int ncol = F.ncol, nz = F.nz;
    const int64_t nv = F.nvp;
    b += rhs * nv;
    x += rhs * nv;
    bc += rhs * int64_t(nvp_c) + tile_base(C, nz);
    auto load_once = [](const T* p, int64_t i, T& a, T& c) {
        if constexpr (NTS) load_pair_nt<T, true>(p, i, a, c);
        else load_pair<T, true>(p, i, a, c);
    };
    int ch[4], cb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ch[s] = child[s * ncol_c + C];
        cb[s] = tile_base(ch[s], nz);
    }
    // outer x and faces from global memory, for the patch's edge cells only
    // (the numbering of k_resid_restrict: f = 2 child + {0: W or E, 1: S or N})
    int out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t fc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (eW) {
        out[0] = tile_base(F.nbr[1 * ncol + ch[0]], nz); fc[0] = F.fface[ch[0]];
        out[4] = tile_base(F.nbr[1 * ncol + ch[2]], nz); fc[4] = F.fface[ch[2]];
    }
    if (eE) {
        out[2] = tile_base(F.nbr[0 * ncol + ch[1]], nz);
        out[6] = tile_base(F.nbr[0 * ncol + ch[3]], nz);
    }
    if (eS) {
        out[1] = tile_base(F.nbr[3 * ncol + ch[0]], nz); fc[1] = F.fface[ncol + ch[0]];
        out[3] = tile_base(F.nbr[3 * ncol + ch[1]], nz); fc[3] = F.fface[ncol + ch[1]];
    }
    if (eN) {
        out[5] = tile_base(F.nbr[2 * ncol + ch[2]], nz);
        out[7] = tile_base(F.nbr[2 * ncol + ch[3]], nz);
    }
    const int k0 = kc * kchunk, k1 = min(nz, k0 + kchunk);
    // H^T: the flux terms act on u = s x, so every x below but the one of
    // the delta term (xr) is multiplied by its weight
    auto su = [&](T& v0, T& v1, int off) {
        if constexpr (SC == kRowWT) {
            T w0, w1;
            load_pair<T, true>(F.s, off, w0, w1);
            v0 *= w0;
            v1 *= w1;
        }
    };
    T xdn[4] = {T(0), T(0), T(0), T(0)}, xo[4], kvdn[4] = {T(0), T(0), T(0), T(0)};
    if (k0 > 0) {
        const int rdn = kTile * (k0 - 1);
        load_pair<T, true>(x, rdn + cb[0], xdn[0], xdn[1]);
        load_pair<T, true>(x, rdn + cb[2], xdn[2], xdn[3]);
        su(xdn[0], xdn[1], rdn + cb[0]);
        su(xdn[2], xdn[3], rdn + cb[2]);
        load_pair<T, true>(F.kv, rdn + cb[0], kvdn[0], kvdn[1]);
        load_pair<T, true>(F.kv, rdn + cb[2], kvdn[2], kvdn[3]);
    }
    load_pair<T, true>(x, kTile * k0 + cb[0], xo[0], xo[1]);
    load_pair<T, true>(x, kTile * k0 + cb[2], xo[2], xo[3]);
    T xr[4] = {xo[0], xo[1], xo[2], xo[3]};
    su(xo[0], xo[1], kTile * k0 + cb[0]);
    su(xo[2], xo[3], kTile * k0 + cb[2]);
    // 9-cell: window x[k-2], kv2[k-2], kv2[k-1] of the four children
    T xm2[4] = {T(0), T(0), T(0), T(0)}, k2m2[4] = {T(0), T(0), T(0), T(0)};
    T k2m1[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (K2) {
        if (k0 >= 2) {
            const int r2 = kTile * (k0 - 2);
            load_pair<T, true>(x, r2 + cb[0], xm2[0], xm2[1]);
            load_pair<T, true>(x, r2 + cb[2], xm2[2], xm2[3]);
            load_pair<T, true>(F.kv2, r2 + cb[0], k2m2[0], k2m2[1]);
            load_pair<T, true>(F.kv2, r2 + cb[2], k2m2[2], k2m2[3]);
        }
        if (k0 >= 1) {
            const int r1 = kTile * (k0 - 1);
            load_pair<T, true>(F.kv2, r1 + cb[0], k2m1[0], k2m1[1]);
            load_pair<T, true>(F.kv2, r1 + cb[2], k2m1[2], k2m1[3]);
        }
    }
    for (int k = k0; k < k1; ++k) {
        const int r = kTile * k, buf = k & 1;
        T xup[4] = {T(0), T(0), T(0), T(0)}, vb[4], vd[4], vkv[4], vxo[8], vk[8], iE[2];
        T xupr[4] = {T(0), T(0), T(0), T(0)};  // H^T: raw x at k+1
        if (k + 1 < nz) {
            load_pair<T, true>(x, r + kTile + cb[0], xup[0], xup[1]);
            load_pair<T, true>(x, r + kTile + cb[2], xup[2], xup[3]);
            if constexpr (SC == kRowWT) {
#pragma unroll
                for (int s = 0; s < 4; ++s) xupr[s] = xup[s];
                su(xup[0], xup[1], r + kTile + cb[0]);
                su(xup[2], xup[3], r + kTile + cb[2]);
            }
        }
        load_once(b, r + cb[0], vb[0], vb[1]);
        load_once(b, r + cb[2], vb[2], vb[3]);
        load_once(F.dl, r + cb[0], vd[0], vd[1]);
        load_once(F.dl, r + cb[2], vd[2], vd[3]);
        load_pair<T, true>(F.kv, r + cb[0], vkv[0], vkv[1]);
        load_pair<T, true>(F.kv, r + cb[2], vkv[2], vkv[3]);
        // own faces: E of 10 and 11 (the E of 00, 01 is between siblings:
        // iE, used by H only), N of 01, 11
        load_pair<T, true>(F.kh, r + cb[0], iE[0], vk[2]);
        load_pair<T, true>(F.kh, r + cb[2], iE[1], vk[6]);
        load_pair<T, true>(F.kh + nv, r + cb[2], vk[5], vk[7]);
        auto outer = [&](int f) {
            vxo[f] = x[out[f] + r];
            if constexpr (SC == kRowWT) vxo[f] *= F.s[out[f] + r];
        };
        if (eW) {
            outer(0); vk[0] = F.kh[fc[0] + uint32_t(r)];
            outer(4); vk[4] = F.kh[fc[4] + uint32_t(r)];
        }
        if (eE) {
            outer(2);
            outer(6);
        }
        if (eS) {
            outer(1); vk[1] = F.kh[fc[1] + uint32_t(r)];
            outer(3); vk[3] = F.kh[fc[3] + uint32_t(r)];
        }
        if (eN) {
            outer(5);
            outer(7);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) lx[buf][s][t] = xo[s];
        lf[buf][0][t] = vk[2];
        lf[buf][1][t] = vk[6];
        lf[buf][2][t] = vk[5];
        lf[buf][3][t] = vk[7];
        // the writes of level k - 1's buffer were read before the last barrier
        __syncthreads();
        if (!eW) {
            vxo[0] = lx[buf][1][t - 1]; vk[0] = lf[buf][0][t - 1];
            vxo[4] = lx[buf][3][t - 1]; vk[4] = lf[buf][1][t - 1];
        }
        if (!eE) {
            vxo[2] = lx[buf][0][t + 1];
            vxo[6] = lx[buf][2][t + 1];
        }
        if (!eS) {
            vxo[1] = lx[buf][2][t - PX]; vk[1] = lf[buf][2][t - PX];
            vxo[3] = lx[buf][3][t - PX]; vk[3] = lf[buf][3][t - PX];
        }
        if (!eN) {
            vxo[5] = lx[buf][0][t + PX];
            vxo[7] = lx[buf][1][t + PX];
        }
        T acc = ((vb[0] + vb[1]) + vb[2]) + vb[3];
        if constexpr (SC == kRowW) {
            // each child's flux row, with the four faces between siblings:
            // c00|c10 and c01|c11 (E faces of c00, c01), c00|c01 and c10|c11
            // (N faces of c00, c10)
            T sw[4], iN0, iN1;
            load_pair<T, true>(F.s, r + cb[0], sw[0], sw[1]);
            load_pair<T, true>(F.s, r + cb[2], sw[2], sw[3]);
            load_pair<T, true>(F.kh + nv, r + cb[0], iN0, iN1);
            T Lr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Lr[q] = vkv[q] * (xo[q] - xup[q]) + kvdn[q] * (xo[q] - xdn[q]);
#pragma unroll
            for (int f = 0; f < 8; ++f) Lr[f >> 1] += vk[f] * (xo[f >> 1] - vxo[f]);
            Lr[0] += iE[0] * (xo[0] - xo[1]) + iN0 * (xo[0] - xo[2]);
            Lr[1] += iE[0] * (xo[1] - xo[0]) + iN1 * (xo[1] - xo[3]);
            Lr[2] += iE[1] * (xo[2] - xo[3]) + iN0 * (xo[2] - xo[0]);
            Lr[3] += iE[1] * (xo[3] - xo[2]) + iN1 * (xo[3] - xo[1]);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc -= vd[q] * xo[q] + sw[q] * Lr[q];
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                acc -= vd[s] * (SC == kRowWT ? xr[s] : xo[s]);
                acc -= vkv[s] * (xo[s] - xup[s]) + kvdn[s] * (xo[s] - xdn[s]);
            }
#pragma unroll
            for (int f = 0; f < 8; ++f) acc -= vk[f] * (xo[f >> 1] - vxo[f]);
        }
        T k2[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (K2) {
            T xp2[4] = {T(0), T(0), T(0), T(0)};
            if (k + 2 < nz) {
                load_pair<T, true>(x, r + 2 * kTile + cb[0], xp2[0], xp2[1]);
                load_pair<T, true>(x, r + 2 * kTile + cb[2], xp2[2], xp2[3]);
            }
            load_pair<T, true>(F.kv2, r + cb[0], k2[0], k2[1]);
            load_pair<T, true>(F.kv2, r + cb[2], k2[2], k2[3]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
                acc -= k2[s] * (xo[s] - xp2[s]) + k2m2[s] * (xo[s] - xm2[s]);
        }
        bc[r] = acc;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if constexpr (K2) {
                xm2[s] = xdn[s];
                k2m2[s] = k2m1[s];
                k2m1[s] = k2[s];
            }
            xdn[s] = xo[s];
            xo[s] = xup[s];
            if constexpr (SC == kRowWT) xr[s] = xupr[s];
            kvdn[s] = vkv[s];
        }
    }
}

// Prolongation by natural injection on its own (only when there is no
// post-smoothing sweep to fuse it into): y = x + xc[parent] (x may be null).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_prolong(int ncol, int nz, int nvp, int nvp_c, const int32_t* __restrict__ parent,
          const T* __restrict__ x, const T* __restrict__ xc, T* __restrict__ y, int64_t total) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * kBlock) {
        const int64_t per = int64_t(nz) * ncol;
        const int64_t rhs = i / per, rem = i % per;
        const int k = int(rem / ncol);
        const int c = int(rem % ncol);
        const T v = xc[rhs * nvp_c + tile_base(parent[c], nz) + kTile * k];
        const int64_t o = rhs * nvp + tile_base(c, nz) + kTile * k;
        y[o] = x ? x[o] + v : v;
    }
}

// ---------------------------------------------------------------------------
// Setup kernels (float64): coefficient layout, coarsening, factors, casts.

// ABI layout -> internal layout on the finest level.
__global__ void __launch_bounds__(kBlock)
k_setup_fine(int ncol, int nz, int nvp, const double* __restrict__ kh_in,
             const double* __restrict__ kv_in, const double* __restrict__ dl_in,
             const double* __restrict__ kv2_in, const double* __restrict__ s_in,
             double* __restrict__ kh, double* __restrict__ kv, double* __restrict__ dl,
             double* __restrict__ kv2, double* __restrict__ sw, int* __restrict__ flags) {
    const int64_t total = int64_t(nz) * ncol;
    int bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * kBlock) {
        const int k = int(i / ncol), c = int(i % ncol);
        const double e = kh_in[i], n = kh_in[total + i];
        const double v = (k + 1 < nz) ? kv_in[i] : 0.0;
        const double d = dl_in[i];
        const int o = tile_base(c, nz) + kTile * k;
        kh[o] = e;
        kh[int64_t(nvp) + o] = n;
        kv[o] = v;
        dl[o] = d;
        if (!isfinite(e) || !isfinite(n) || !isfinite(v) || !isfinite(d)) bad |= 1;
        if (!(e >= 0.0) || !(n >= 0.0) || !(v >= 0.0) || !(d > 0.0)) bad |= 2;
        if (kv2) {
            const double v2 = (k + 2 < nz) ? kv2_in[i] : 0.0;
            kv2[o] = v2;
            if (!isfinite(v2)) bad |= 1;
            if (!(v2 >= 0.0)) bad |= 2;
        }
        if (sw) {
            const double w = s_in[i];
            sw[o] = w;
            if (!isfinite(w)) bad |= 1;
            if (!(w > 0.0)) bad |= 2;
        }
    }
    if (bad) atomicOr(flags, bad);
}

// Coarse coefficients by re-discretisation (Section 3.6 with the scalings of
// Eq. DH_ratios): coarse E face = mean of the E faces of children (1,0),(1,1);
// N face = mean of the N faces of (0,1),(1,1); kv and delta summed over all four.
__global__ void __launch_bounds__(kBlock)
k_coarsen(int ncol_c, int nz, int nvp_f, int nvp_c, const int32_t* __restrict__ child,
          const double* __restrict__ khf, const double* __restrict__ kvf,
          const double* __restrict__ dlf, const double* __restrict__ kv2f,
          const double* __restrict__ sf, double* __restrict__ khc, double* __restrict__ kvc,
          double* __restrict__ dlc, double* __restrict__ kv2c, double* __restrict__ sc) {
    const int64_t total = int64_t(nz) * ncol_c;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * kBlock) {
        const int k = int(i / ncol_c);
        const int C = int(i % ncol_c);
        const int r = kTile * k;
        const int c00 = tile_base(child[C], nz) + r, c10 = tile_base(child[ncol_c + C], nz) + r,
                  c01 = tile_base(child[2 * ncol_c + C], nz) + r,
                  c11 = tile_base(child[3 * ncol_c + C], nz) + r;
        const int o = tile_base(C, nz) + r;
        const double* khfN = khf + nvp_f;
        khc[o] = 0.5 * (khf[c10] + khf[c11]);
        khc[int64_t(nvp_c) + o] = 0.5 * (khfN[c01] + khfN[c11]);
        kvc[o] = ((kvf[c00] + kvf[c10]) + kvf[c01]) + kvf[c11];
        dlc[o] = ((dlf[c00] + dlf[c10]) + dlf[c01]) + dlf[c11];
        if (kv2c) kv2c[o] = ((kv2f[c00] + kv2f[c10]) + kv2f[c01]) + kv2f[c11];
        // row weight (a pointwise field): mean of the four children
        if (sc) sc[o] = 0.25 * (((sf[c00] + sf[c10]) + sf[c01]) + sf[c11]);
    }
}

// Column factors (see the header comment), one thread per column.
__global__ void __launch_bounds__(kBlock)
k_factor(LevelView<double> L, int mid, double* __restrict__ cc, double* __restrict__ mm) {
    const int ncol = L.ncol, nz = L.nz;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncol) return;
    const uint32_t fW = L.fface[c], fS = L.fface[ncol + c];
    const int ob = tile_base(c, nz);
    const double* khN = L.kh + L.nvp;
    auto s_of = [&](int k) {
        const int o = ob + kTile * k;
        // weighted operator: the factors are those of Hz' (delta / s)
        double v = (L.s ? L.dl[o] / L.s[o] : L.dl[o]) + L.kh[o] + L.kh[fW + uint32_t(kTile * k)] +
                   khN[o] + L.kh[fS + uint32_t(kTile * k)];
        // 9-cell: the dropped couplings two levels apart stay in the diagonal
        if (L.kv2) v += L.kv2[o] + (k >= 2 ? L.kv2[o - 2 * kTile] : 0.0);
        return v;
    };
    auto kv_of = [&](int k) { return L.kv[ob + kTile * k]; };
    auto put = [&](int k, double m, double cv) {
        mm[ob + kTile * k] = m;
        cc[ob + kTile * k] = cv;
    };
    const int top_end = mid < nz ? mid : nz;  // rows [0, top_end) top-down
    double e = 0.0;
    for (int k = 0; k < top_end; ++k) {
        const double s = s_of(k);
        if (k == 0) {
            e = s;
        } else {
            const double a = kv_of(k - 1);
            e = s + a * e / (e + a);
        }
        const double kvk = kv_of(k);
        const double m = 1.0 / (e + kvk);
        put(k, m, kvk * m);
    }
    if (mid >= nz) return;
    double f = 0.0;
    for (int k = nz - 1; k > mid; --k) {
        const double s = s_of(k);
        if (k == nz - 1) {
            f = s;
        } else {
            const double a = kv_of(k);
            f = s + a * f / (f + a);
        }
        const double up = kv_of(k - 1);
        const double m = 1.0 / (f + up);
        put(k, m, up * m);
    }
    double tau = s_of(mid);
    if (mid > 0) {
        const double a = kv_of(mid - 1);
        tau += a * e / (e + a);
    }
    if (mid < nz - 1) {
        const double a = kv_of(mid);
        tau += a * f / (f + a);
    }
    put(mid, 1.0 / tau, 0.0);
}

template <typename S, typename D>
__global__ void __launch_bounds__(kBlock)
k_convert(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * kBlock)
        dst[i] = D(src[i]);
}

// ---------------------------------------------------------------------------
// Krylov (float64) kernels. Reductions are deterministic: a fixed grid of
// blocks per right-hand side writes one partial sum each, and one block per
// right-hand side adds the partials in a fixed order and derives the CG
// scalar, so repeated runs give identical bits.
//
// Kernels that meet a vector in the ABI layout run one workgroup per
// (right-hand side, tile): thread (lc, g) visits levels g, g + 8, ... of
// column tile * 32 + lc, so the tiled side is read as contiguous rows and the
// ABI side as 32-column row pieces.
struct TileGrid {
    int rhs, tile, lc, g, c;
    bool valid;
};
__device__ __forceinline__ TileGrid tile_grid(int ncol, int rev = 0) {
    const int ntile = (ncol + kTile - 1) / kTile;
    const int lb = logical_block(rev);
    TileGrid t;
    t.rhs = lb / ntile;
    t.tile = lb % ntile;
    t.lc = threadIdx.x & (kTile - 1);
    t.g = threadIdx.x / kTile;
    t.c = t.tile * kTile + t.lc;
    t.valid = t.c < ncol;
    return t;
}
constexpr int kTileGroups = kBlock / kTile;

// x = 0, r = b, r32 = float(b), r0 = b (b and x in the ABI layout; x, r32
// and r0 may be null: CG writes x in its first update, see k_cg_update);
// partial ||b||^2 per tile.
__global__ void __launch_bounds__(kBlock)
k_cg_init(const double* __restrict__ b, double* __restrict__ x, double* __restrict__ r,
          float* __restrict__ r32, double* __restrict__ r0, int ncol, int nz, int nvp,
          CgState st) {
    __shared__ double sh[kBlock / 64];
    const TileGrid t = tile_grid(ncol);
    const int64_t n = int64_t(nz) * ncol;
    double acc = 0.0;
    if (t.valid) {
        const int64_t ia = t.rhs * n + t.c, it = t.rhs * int64_t(nvp) + tile_base(t.c, nz);
        for (int k = t.g; k < nz; k += kTileGroups) {
            const double v = b[ia + int64_t(k) * ncol];
            if (x) x[ia + int64_t(k) * ncol] = 0.0;
            r[it + kTile * k] = v;
            if (r32) r32[it + kTile * k] = float(v);
            if (r0) r0[it + kTile * k] = v;
            acc += v * v;
        }
    }
    const double s = block_sum(acc, sh);
    store_partial(st, t.rhs, t.tile, s, 0.0, false);
}

// x = 0 for the right-hand sides that do not start (b = 0 or not finite);
// the others get x in the first CG update.
__global__ void __launch_bounds__(kBlock)
k_cg_zero_idle(double* __restrict__ x, int ncol, int nz, CgState st) {
    const TileGrid t = tile_grid(ncol);
    if (st.active[t.rhs] || !t.valid) return;
    const int64_t ia = t.rhs * int64_t(nz) * ncol + t.c;
    for (int k = t.g; k < nz; k += kTileGroups) x[ia + int64_t(k) * ncol] = 0.0;
}

// r -= alpha q; r32 = float(r); partial ||r||^2 per tile. The matching
// x += alpha p is owed: k_p_update applies it as it replaces p (one read of
// p for both), k_cg_x where the iteration stops. NT (vectors far larger than
// the last-level cache): q and r, whose next reader comes after a whole
// V-cycle, bypass the cache, so that it keeps r32 for the first smoothing
// sweep.
template <bool NT>
__global__ void __launch_bounds__(kBlock)
k_cg_update(double* __restrict__ r, float* __restrict__ r32, const double* __restrict__ q,
            int ncol, int nz, int nvp, CgState st, int rev) {
    __shared__ double sh[kBlock / 64];
    const TileGrid t = tile_grid(ncol, rev);
    if (!st.active[t.rhs]) return;
    const double alpha = st.sc[t.rhs * kScal + kAlpha];
    double acc = 0.0;
    if (t.valid) {
        const int64_t it = t.rhs * int64_t(nvp) + tile_base(t.c, nz);
        for (int k = t.g; k < nz; k += kTileGroups) {
            const int64_t o = it + kTile * k;
            const double v = stream_load<NT>(r + o) - alpha * stream_load<NT>(q + o);
            stream_store<NT>(r + o, v);
            if (r32) r32[o] = float(v);
            acc += v * v;
        }
    }
    const double s = block_sum(acc, sh);
    store_partial(st, t.rhs, t.tile, s, 0.0, false);
}

// The x update of CG (x in the ABI layout): kXSet x = alpha p (the first
// iteration: x is not read), kXAdd x += alpha p.
enum { kXNone = 0, kXSet = 1, kXAdd = 2 };

// The owed x update where the iteration stops: for the right-hand sides that
// the last residual update included (upd) and that `sel` names: kXAll all of
// them, kXDone those that have converged in it, kXLive the others. NT: x
// bypasses the cache.
enum { kXAll = 0, kXDone = 1, kXLive = 2 };

template <bool NT>
__global__ void __launch_bounds__(kBlock)
k_cg_x(double* __restrict__ x, const double* __restrict__ p, int ncol, int nz, int nvp,
       CgState st, int xmode, int sel, int rev) {
    const TileGrid t = tile_grid(ncol, rev);
    if (!t.valid || !st.upd[t.rhs]) return;
    if ((sel == kXDone && st.active[t.rhs]) || (sel == kXLive && !st.active[t.rhs])) return;
    const double alpha = st.sc[t.rhs * kScal + kAlpha];
    const int64_t ia = t.rhs * int64_t(nz) * ncol + t.c;
    const int64_t it = t.rhs * int64_t(nvp) + tile_base(t.c, nz);
    for (int k = t.g; k < nz; k += kTileGroups) {
        double* xk = x + ia + int64_t(k) * ncol;
        const double ap = alpha * p[it + kTile * k];
        stream_store<NT>(xk, xmode == kXSet ? ap : stream_load<NT>(xk) + ap);
    }
}

// Layout conversion between the ABI layout and the tiled one, with a cast.
template <typename S, typename D, bool TO_TILED>
__global__ void __launch_bounds__(kBlock)
k_retile(const S* __restrict__ src, D* __restrict__ dst, int ncol, int nz, int nvp) {
    const TileGrid t = tile_grid(ncol);
    if (!t.valid) return;
    const int64_t n = int64_t(nz) * ncol;
    const int64_t ia = t.rhs * n + t.c, it = t.rhs * int64_t(nvp) + tile_base(t.c, nz);
    for (int k = t.g; k < nz; k += kTileGroups) {
        if (TO_TILED)
            dst[it + kTile * k] = D(src[ia + int64_t(k) * ncol]);
        else
            dst[ia + int64_t(k) * ncol] = D(src[it + kTile * k]);
    }
}

// partial r . z (and z . q for the flexible beta). NT: r bypasses the cache,
// which keeps z for the direction update that follows.
template <typename Z, bool NT>
__global__ void __launch_bounds__(kBlock)
k_dot_rz(const double* __restrict__ r, const Z* __restrict__ z, const double* __restrict__ q,
         int64_t n, int nblk, CgState st, int rev) {
    __shared__ double sh[kBlock / 64];
    const int lbk = logical_block(rev);
    const int rhs = lbk / nblk, blk = lbk % nblk;
    if (!st.active[rhs]) return;
    int64_t i0, i1;
    grid_range(n, nblk, blk, i0, i1);
    const int64_t off = int64_t(rhs) * n;
    double a1 = 0.0, a2 = 0.0;
#pragma unroll 4
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double zv = double(z[off + i]);
        a1 += stream_load<NT>(r + off + i) * zv;
        if (q) a2 += zv * q[off + i];
    }
    const double s1 = block_sum(a1, sh);
    double s2 = 0.0;
    if (q) {
        __syncthreads();
        s2 = block_sum(a2, sh);
    }
    store_partial(st, rhs, blk, s1, s2, q != nullptr);
}

// p = z + beta p (init: p = z) for the right-hand sides still iterating and,
// first, the x update owed from the last iteration (xmode), with the p about
// to be replaced: one read of p for both. One workgroup per (right-hand side,
// tile); x in the ABI layout. NT: z (read for the last time) and x bypass
// the cache, which keeps p for the apply that follows.
template <typename Z, bool NT>
__global__ void __launch_bounds__(kBlock)
k_p_update(const Z* __restrict__ z, double* __restrict__ p, double* __restrict__ x, int ncol,
           int nz, int nvp, CgState st, int init, int xmode, int rev) {
    const TileGrid t = tile_grid(ncol, rev);
    if (!t.valid || !st.active[t.rhs]) return;
    const double beta = init ? 0.0 : st.sc[t.rhs * kScal + kBeta];
    const double alpha = xmode != kXNone ? st.sc[t.rhs * kScal + kAlpha] : 0.0;
    const int64_t ia = t.rhs * int64_t(nz) * ncol + t.c;
    const int64_t it = t.rhs * int64_t(nvp) + tile_base(t.c, nz);
    for (int k = t.g; k < nz; k += kTileGroups) {
        const int64_t o = it + kTile * k;
        const double zv = double(stream_load<NT>(z + o));
        if (init) {
            p[o] = zv;
            continue;
        }
        const double pv = p[o];
        if (xmode != kXNone) {
            double* xk = x + ia + int64_t(k) * ncol;
            stream_store<NT>(xk, xmode == kXSet ? alpha * pv : stream_load<NT>(xk) + alpha * pv);
        }
        p[o] = zv + beta * pv;
    }
}

// ---------------------------------------------------------------------------
// Gradients for the weighted operator H = delta + S L given lam = H^-T g (ABI
// layout, summed over the batch): dH/dK = S a a^T for a face vector a, so
//   g_kh = -(s_c lam_c - s_n lam_n)(x_c - x_n) (E, N faces), g_kv likewise
//   along k, g_delta = -lam x, g_s = -lam (L x).
// Reads the finest level's float64 coefficients and weights (tiled).
__global__ void __launch_bounds__(kBlock)
k_face_grad_w(LevelView<double> L, const double* __restrict__ lam, const double* __restrict__ x,
              int batch, double* __restrict__ gkh, double* __restrict__ gkv,
              double* __restrict__ gdl, double* __restrict__ gs) {
    const int ncol = L.ncol, nz = L.nz;
    const int64_t total = int64_t(nz) * ncol;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = int64_t(lb) * kBlock + threadIdx.x;
    if (i >= total) return;
    const int k = int(i / ncol);
    const int c = int(i % ncol);
    int nbc[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) nbc[d] = L.nbr[d * ncol + c];
    const int o = tile_base(c, nz) + kTile * k;
    const double* khN = L.kh + L.nvp;
    // couplings of the four faces of c (E, W, N, S) and the vertical ones
    const double K[4] = {L.kh[o], L.kh[L.fface[c] + uint32_t(kTile * k)], khN[o],
                         L.kh[L.fface[ncol + c] + uint32_t(kTile * k)]};
    const double kup = L.kv[o], kdn = k > 0 ? L.kv[o - kTile] : 0.0;
    const double sc = L.s[o];
    const double se = L.s[tile_base(nbc[0], nz) + kTile * k];
    const double sn = L.s[tile_base(nbc[2], nz) + kTile * k];
    const double su = k + 1 < nz ? L.s[o + kTile] : 0.0;
    const int64_t row = int64_t(k) * ncol;
    double ge = 0.0, gn = 0.0, gv = 0.0, gd = 0.0, gw = 0.0;
    for (int bi = 0; bi < batch; ++bi) {
        const double* l = lam + int64_t(bi) * total;
        const double* xx = x + int64_t(bi) * total;
        const double lc = l[row + c], xc = xx[row + c];
        ge -= (sc * lc - se * l[row + nbc[0]]) * (xc - xx[row + nbc[0]]);
        gn -= (sc * lc - sn * l[row + nbc[2]]) * (xc - xx[row + nbc[2]]);
        double lx = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) lx += K[d] * (xc - xx[row + nbc[d]]);
        if (k + 1 < nz) {
            gv -= (sc * lc - su * l[row + ncol + c]) * (xc - xx[row + ncol + c]);
            lx += kup * (xc - xx[row + ncol + c]);
        }
        if (k > 0) lx += kdn * (xc - xx[row - ncol + c]);
        gd -= lc * xc;
        gw -= lc * lx;
    }
    gkh[i] = ge;
    gkh[total + i] = gn;
    if (k + 1 < nz) gkv[i] = gv;
    gdl[i] = gd;
    gs[i] = gw;
}

// ---------------------------------------------------------------------------
// BiCGStab vector steps (tiled vectors; x in the ABI layout).

// p = r + beta (p - omega v)   (init: p = r)
__global__ void __launch_bounds__(kBlock)
k_bicg_p(const double* __restrict__ r, const double* __restrict__ v, double* __restrict__ p,
         int64_t n, int nblk, const double* __restrict__ sc, const int* __restrict__ active,
         int init) {
    const int rhs = blockIdx.x / nblk, blk = blockIdx.x % nblk;
    if (!active[rhs]) return;
    const double beta = init ? 0.0 : sc[rhs * kScal + kBeta];
    const double omega = init ? 0.0 : sc[rhs * kScal + kOmega];
    int64_t i0, i1;
    grid_range(n, nblk, blk, i0, i1);
    const int64_t off = int64_t(rhs) * n;
#pragma unroll 4
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock)
        p[off + i] = init ? r[off + i] : r[off + i] + beta * (p[off + i] - omega * v[off + i]);
}

// s = r - alpha v
__global__ void __launch_bounds__(kBlock)
k_bicg_s(const double* __restrict__ r, const double* __restrict__ v, double* __restrict__ s,
         int64_t n, int nblk, const double* __restrict__ sc, const int* __restrict__ active) {
    const int rhs = blockIdx.x / nblk, blk = blockIdx.x % nblk;
    if (!active[rhs]) return;
    const double alpha = sc[rhs * kScal + kAlpha];
    int64_t i0, i1;
    grid_range(n, nblk, blk, i0, i1);
    const int64_t off = int64_t(rhs) * n;
#pragma unroll 4
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock)
        s[off + i] = r[off + i] - alpha * v[off + i];
}

// x += alpha p_hat + omega s_hat (x in the ABI layout); r = s - omega t;
// partials (r0, r) and ||r||^2 per tile.
__global__ void __launch_bounds__(kBlock)
k_bicg_xr(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ ph,
          const double* __restrict__ shat, const double* __restrict__ s,
          const double* __restrict__ t, const double* __restrict__ r0, int ncol, int nz, int nvp,
          CgState st) {
    __shared__ double sh[kBlock / 64];
    const TileGrid g = tile_grid(ncol);
    if (!st.active[g.rhs]) return;
    const double alpha = st.sc[g.rhs * kScal + kAlpha];
    const double omega = st.sc[g.rhs * kScal + kOmega];
    const int64_t n = int64_t(nz) * ncol;
    double a1 = 0.0, a2 = 0.0;
    if (g.valid) {
        const int64_t ia = g.rhs * n + g.c, it = g.rhs * int64_t(nvp) + tile_base(g.c, nz);
        for (int k = g.g; k < nz; k += kTileGroups) {
            const int64_t o = it + kTile * k;
            x[ia + int64_t(k) * ncol] += alpha * ph[o] + omega * shat[o];
            const double v = s[o] - omega * t[o];
            r[o] = v;
            a1 += r0[o] * v;
            a2 += v * v;
        }
    }
    const double s1 = block_sum(a1, sh);
    __syncthreads();
    const double s2 = block_sum(a2, sh);
    store_partial(st, g.rhs, g.tile, s1, s2, true);
}

// ---------------------------------------------------------------------------
// Face-coefficient gradients of L = g . x (summed over the batch), written in
// the ABI layout: g_kh[2][nz][ncol], g_kv[nz-1][ncol], g_delta[nz][ncol] and,
// for the 9-cell stencil, g_kv2[nz-2][ncol] (gkv2 non-null).
__global__ void __launch_bounds__(kBlock)
k_face_grad(int ncol, int nz, const int32_t* __restrict__ nbr, const double* __restrict__ lam,
            const double* __restrict__ x, int batch, double* __restrict__ gkh,
            double* __restrict__ gkv, double* __restrict__ gdl, double* __restrict__ gkv2) {
    const int64_t total = int64_t(nz) * ncol;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t i = int64_t(lb) * kBlock + threadIdx.x;
    if (i >= total) return;
    const int64_t k = i / ncol;
    const int c = int(i % ncol);
    const int e = nbr[c], nn = nbr[2 * ncol + c];
    const int64_t row = k * ncol;
    double ge = 0.0, gn = 0.0, gv = 0.0, gd = 0.0, gv2 = 0.0;
    for (int bi = 0; bi < batch; ++bi) {
        const double* l = lam + int64_t(bi) * total;
        const double* xx = x + int64_t(bi) * total;
        const double lc = l[row + c], xc = xx[row + c];
        ge -= (lc - l[row + e]) * (xc - xx[row + e]);
        gn -= (lc - l[row + nn]) * (xc - xx[row + nn]);
        if (k + 1 < nz) gv -= (lc - l[row + ncol + c]) * (xc - xx[row + ncol + c]);
        if (gkv2 && k + 2 < nz)
            gv2 -= (lc - l[row + 2 * ncol + c]) * (xc - xx[row + 2 * ncol + c]);
        gd -= lc * xc;
    }
    gkh[i] = ge;
    gkh[total + i] = gn;
    if (k + 1 < nz) gkv[i] = gv;
    if (gkv2 && k + 2 < nz) gkv2[i] = gv2;
    gdl[i] = gd;
}

// ---------------------------------------------------------------------------
// Achievable-bandwidth yardstick: one pass of a plain streaming kernel,
// 16-byte accesses, each thread four vectors 256 apart (all loads of a thread
// issued before its stores). Not part of the method.
enum { kStreamRead = 0, kStreamWrite = 1, kStreamCopy = 2, kStreamTriad = 3 };
constexpr int kStreamUnroll = 4;
constexpr int64_t kStreamPerBlock = int64_t(kBlock) * kStreamUnroll * 4;  // floats per block

template <int KIND>
__global__ void __launch_bounds__(kBlock)
k_stream(const float4* __restrict__ a, const float4* __restrict__ b, float4* __restrict__ c,
         int64_t n4, float s, float* __restrict__ partial) {
    __shared__ double sh[kBlock / 64];
    const int64_t i0 = int64_t(blockIdx.x) * (kBlock * kStreamUnroll) + threadIdx.x;
    float4 va[kStreamUnroll], vb[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t i = i0 + int64_t(u) * kBlock;
        if (i < n4) {
            if (KIND != kStreamWrite) va[u] = a[i];
            if (KIND == kStreamTriad) vb[u] = b[i];
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const int64_t i = i0 + int64_t(u) * kBlock;
        if (i < n4) {
            if (KIND == kStreamRead) acc += (va[u].x + va[u].y) + (va[u].z + va[u].w);
            if (KIND == kStreamWrite) c[i] = make_float4(s, s, s, s);
            if (KIND == kStreamCopy) c[i] = va[u];
            if (KIND == kStreamTriad)
                c[i] = make_float4(va[u].x + s * vb[u].x, va[u].y + s * vb[u].y,
                                   va[u].z + s * vb[u].z, va[u].w + s * vb[u].w);
        }
    }
    if (KIND == kStreamRead) {
        const double t = block_sum(double(acc), sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = float(t);
    }
}

}  // namespace hh

// Host side of the C ABI declared in include/helmholtz.h: workspace layout,
// operator set-up, the V-cycle of Algorithm 1 and the conjugate-gradient
// loop, all as stream-ordered launches of the kernels in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "helmholtz.h"
#include "kernels.hpp"
#include "mesh.hpp"

using namespace hh;

namespace {

constexpr int kRedBlocks = 2048;  // partial sums per right-hand side for vector reductions
constexpr int kMaxLevels = 20;    // deepest hierarchy a configuration may ask for
constexpr int kApplyChunk = 4;   // vertical levels per thread in apply / residual kernels
constexpr int kSmallSweepCols = 5000;  // levels below this use narrow sweep tiles

// Per-level arrays use the column-tile layout of the kernels (element (k, c)
// at tile_base(c) + 32 k, columns padded to ncolp, nvp = nz * ncolp).
template <typename T>
struct LevelData {
    T* kh = nullptr;  // [2][nvp]  E faces, N faces
    T* kv = nullptr;  // [nvp]
    T* dl = nullptr;  // [nvp]
    T* cc = nullptr;  // [nvp]
    T* mm = nullptr;  // [nvp]
    T* kv2 = nullptr; // [nvp]     9-cell stencil only
    T* s = nullptr;   // [nvp]     weighted operator only: row weight
    T* b = nullptr;   // [B][nvp]   level >= 1 (and level 0 for float32)
    T* x = nullptr;   // [B][nvp]   level >= 1 (and level 0 for float32)
    T* t = nullptr;   // [B][nvp]   ping-pong partner of x
};

// The vectors one V-cycle works in, per level: right-hand side b, iterate x
// and its Jacobi ping-pong partner t. They come from the handle's workspace
// or, for the allocation-free entry point, from the static scratch array.
template <typename T>
struct VBufs {
    T* b[kMaxLevels] = {};
    T* x[kMaxLevels] = {};
    T* t[kMaxLevels] = {};
};

struct Level {
    int N = 0;
    int ncol = 0;
    int ncolp = 0;              // ncol rounded up to whole tiles
    int nvp = 0;                // nz * ncolp
    int32_t* nbr = nullptr;     // [4][ncol]
    uint32_t* fface = nullptr;  // [2][ncol] offsets of the W and S faces in kh
    int32_t* parent = nullptr;  // [ncol] into level + 1 (not on the coarsest)
    int32_t* pofs = nullptr;    // [3][ncol] prolongation offsets (not on the coarsest)
    int32_t* child = nullptr;   // [4][ncol] into level - 1 (not on the finest)
    LevelData<double> d;
    LevelData<float> f;
};

// Bump allocator over the caller's workspace; run with base 0 to size it.
struct Carver {
    uintptr_t base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + HELMHOLTZ_WORKSPACE_ALIGN - 1) / HELMHOLTZ_WORKSPACE_ALIGN *
              HELMHOLTZ_WORKSPACE_ALIGN;
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

bool config_ok(const helmholtz_config* c) {
    if (!c) return false;
    if (c->N < 1 || c->nz < 1 || c->nz > HELMHOLTZ_NZ_MAX || c->nlevels < 1 ||
        c->nlevels > kMaxLevels)
        return false;
    if (c->n_pre < 0 || c->n_post < 0 || c->n_coarse < 1) return false;
    if (!(c->omega > 0.0 && c->omega <= 1.5)) return false;
    if (c->mg_precision != HELMHOLTZ_FP64 && c->mg_precision != HELMHOLTZ_FP32) return false;
    if (c->cg_variant != HELMHOLTZ_CG_STANDARD && c->cg_variant != HELMHOLTZ_CG_FLEXIBLE &&
        c->cg_variant != HELMHOLTZ_BICGSTAB)
        return false;
    if (c->max_batch < 1) return false;
    if (c->stencil != 0 && c->stencil != 7 && c->stencil != 9) return false;
    if (c->weighted != 0 && c->weighted != 1) return false;
    // the weighted operator is not symmetric: BiCGStab, 7-point stencil
    if (c->weighted && (c->cg_variant != HELMHOLTZ_BICGSTAB || c->stencil == 9)) return false;
    return true;
}

int shape_error(const helmholtz_config* c) {
    if (c->N % (1 << (c->nlevels - 1)) != 0) return HELMHOLTZ_ESHAPE;
    const int64_t ncol = 6 * int64_t(c->N) * c->N;
    const int64_t ncolp = (ncol + kTile - 1) / kTile * kTile;
    // tables and offsets inside one vector are 32-bit (face offsets into the
    // two kh planes unsigned); batch offsets are 64-bit
    if (2 * ncol >= (int64_t(1) << 31)) return HELMHOLTZ_ESHAPE;
    if (int64_t(c->nz) * ncolp >= (int64_t(1) << 31)) return HELMHOLTZ_ESHAPE;
    return HELMHOLTZ_OK;
}

}  // namespace

// ---- allocation-free V-cycle: static scratch -------------------------------
// helmholtz_vcycle_noalloc keeps its level vectors in this file-scope device
// array instead of the workspace. Each GPU holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the device that is current (the array's
// name is a host-side stand-in, not a device address).
constexpr size_t kScratchBytes = HELMHOLTZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Address of the scratch array on the current device, looked up once per
// device; `dev` receives the device index.
int scratch_of_current_device(unsigned char** out, int* dev) {
    *out = nullptr;
    if (hipGetDevice(dev) != hipSuccess) return HELMHOLTZ_EHIP;
    if (*dev < 0 || *dev >= kMaxDevices) return HELMHOLTZ_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[*dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return HELMHOLTZ_EHIP;
        g_scratch_ptr[*dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_ptr[*dev];
    return HELMHOLTZ_OK;
}

}  // namespace

struct helmholtz_s {
    helmholtz_config cfg{};
    int L = 0, nz = 0, B = 0;
    bool nine = false;  // 9-cell stencil (next-to-nearest vertical couplings)
    bool weighted = false;  // row-weighted operator H = delta + S L
    bool adj = false;       // the current call works with H^T (weighted handles)
    int64_t n = 0;    // unknowns per right-hand side on the finest level
    int64_t nvp = 0;  // tiled length of a finest-level vector (n plus padding)
    std::vector<Level> lev;
    // Krylov vectors [B][n]
    double* r = nullptr;
    double* p = nullptr;
    double* q = nullptr;
    double* z = nullptr;  // float64 preconditioned residual (float64 V-cycle)
    // BiCGStab only: shadow residual r0, s, t, s_hat (p_hat is z, v is q)
    double* r0 = nullptr;
    double* s = nullptr;
    double* t = nullptr;
    double* sh = nullptr;
    // r, p, q, z are tiled [B][nvp]; x and b of the ABI are [B][n]
    double* partial = nullptr;
    double* partial2 = nullptr;
    int pstride = 0;
    double* sc = nullptr;     // [B][8] scalars
    int* active = nullptr;    // [B]
    int* upd = nullptr;       // [B] CG: the last residual update included the rhs
    int* flags = nullptr;     // set-up validation bits
    // pinned, host-coherent mirror written by the device: scalars, flags,
    // per-RHS sequence numbers; plus the set-up flags
    double* hsc = nullptr;
    int* hact = nullptr;
    int* hseq = nullptr;
    int* hflags = nullptr;
    size_t ws_bytes = 0;
    // kernel timing hook: event pairs recorded around profiled launches
    struct Prof {
        double ms = 0.0, bytes = 0.0;
        int64_t launches = 0;
        std::vector<hipEvent_t> start, stop;
        std::vector<double> pend_bytes;
    };
    bool prof_on = false;
    mutable Prof prof[HELMHOLTZ_PROF_COUNT];
    // V-cycle vectors in the workspace (float64: level 0 comes from the caller)
    VBufs<double> vb64;
    VBufs<float> vb32;
    // this device's copy of the static scratch array (allocation-free entry
    // point) and the device the handle was created on
    unsigned char* scratch = nullptr;
    int device = -1;
    // traversal direction of the next kernel on each level (alternates, see
    // xcd_remap)
    mutable int dir[kMaxLevels] = {};
    int flip(int l) const {
        const int d = dir[l];
        dir[l] ^= 1;
        return d;
    }
};

namespace {

void layout(helmholtz_s* h, Carver& cv) {
    const int nz = h->nz, B = h->B;
    for (int l = 0; l < h->L; ++l) {
        Level& v = h->lev[l];
        const size_t nc = size_t(v.ncol);
        const size_t nv = size_t(v.nvp);
        v.nbr = cv.take<int32_t>(4 * nc);
        v.fface = cv.take<uint32_t>(2 * nc);
        v.parent = (l + 1 < h->L) ? cv.take<int32_t>(nc) : nullptr;
        v.pofs = (l + 1 < h->L) ? cv.take<int32_t>(3 * nc) : nullptr;
        v.child = (l > 0) ? cv.take<int32_t>(4 * nc) : nullptr;
        v.d.kh = cv.take<double>(2 * nv);
        v.d.kv = cv.take<double>(nv);
        v.d.dl = cv.take<double>(nv);
        v.d.cc = cv.take<double>(nv);
        v.d.mm = cv.take<double>(nv);
        // float32 copies: contiguous in the same order, so one conversion per level
        v.f.kh = cv.take<float>(6 * nv);
        v.f.kv = v.f.kh + 2 * nv;
        v.f.dl = v.f.kh + 3 * nv;
        v.f.cc = v.f.kh + 4 * nv;
        v.f.mm = v.f.kh + 5 * nv;
        if (h->nine) {
            v.d.kv2 = cv.take<double>(nv);
            v.f.kv2 = cv.take<float>(nv);
        }
        if (h->weighted) {
            v.d.s = cv.take<double>(nv);
            v.f.s = cv.take<float>(nv);
        }
        if (l > 0) {
            v.d.b = cv.take<double>(size_t(B) * nv);
            v.d.x = cv.take<double>(size_t(B) * nv);
        }
        v.d.t = cv.take<double>(size_t(B) * nv);
        v.f.b = cv.take<float>(size_t(B) * nv);
        v.f.x = cv.take<float>(size_t(B) * nv);
        v.f.t = cv.take<float>(size_t(B) * nv);
        h->vb64.b[l] = v.d.b;
        h->vb64.x[l] = v.d.x;
        h->vb64.t[l] = v.d.t;
        h->vb32.b[l] = v.f.b;
        h->vb32.x[l] = v.f.x;
        h->vb32.t[l] = v.f.t;
    }
    const size_t nb = size_t(B) * size_t(h->nvp);
    h->r = cv.take<double>(nb);
    h->p = cv.take<double>(nb);
    h->q = cv.take<double>(nb);
    h->z = cv.take<double>(nb);
    if (h->cfg.cg_variant == HELMHOLTZ_BICGSTAB) {
        h->r0 = cv.take<double>(nb);
        h->s = cv.take<double>(nb);
        h->t = cv.take<double>(nb);
        h->sh = cv.take<double>(nb);
    }
    const int ntile0 = (h->lev[0].ncol + kBlock - 1) / kBlock;
    const int nkc0 = (nz + kApplyChunk - 1) / kApplyChunk;
    const int ntile32 = h->lev[0].ncolp / kTile;
    h->pstride = std::max(std::max(kRedBlocks, ntile0 * nkc0), ntile32);
    h->partial = cv.take<double>(size_t(B) * h->pstride);
    h->partial2 = cv.take<double>(size_t(B) * h->pstride);
    h->sc = cv.take<double>(size_t(B) * kScal);
    h->active = cv.take<int>(size_t(B));
    h->upd = cv.take<int>(size_t(B));
    h->flags = cv.take<int>(4);
}

void init_shape(helmholtz_s* h, const helmholtz_config* cfg) {
    h->cfg = *cfg;
    h->L = cfg->nlevels;
    h->nz = cfg->nz;
    h->B = cfg->max_batch;
    h->nine = cfg->stencil == 9;
    h->weighted = cfg->weighted == 1;
    h->lev.assign(h->L, Level{});
    for (int l = 0; l < h->L; ++l) {
        Level& v = h->lev[l];
        v.N = cfg->N >> l;
        v.ncol = 6 * v.N * v.N;
        v.ncolp = (v.ncol + kTile - 1) / kTile * kTile;
        v.nvp = cfg->nz * v.ncolp;
    }
    h->n = int64_t(cfg->nz) * h->lev[0].ncol;
    h->nvp = h->lev[0].nvp;
}

inline int grid_for(int64_t n) {
    return int(std::min<int64_t>((n + kBlock - 1) / kBlock, 65536));
}

#define HH_CHECK(expr)                                   \
    do {                                                 \
        if ((expr) != hipSuccess) return HELMHOLTZ_EHIP; \
    } while (0)

inline int last_error() { return hipGetLastError() == hipSuccess ? HELMHOLTZ_OK : HELMHOLTZ_EHIP; }

// Fold the finished event pairs of one profiled kernel into its totals.
int prof_flush(const helmholtz_s* h, int kernel) {
    helmholtz_s::Prof& P = h->prof[kernel];
    for (size_t i = 0; i < P.start.size(); ++i) {
        float ms = 0.f;
        if (hipEventSynchronize(P.stop[i]) != hipSuccess) return HELMHOLTZ_EHIP;
        if (hipEventElapsedTime(&ms, P.start[i], P.stop[i]) != hipSuccess) return HELMHOLTZ_EHIP;
        P.ms += ms;
        P.bytes += P.pend_bytes[i];
        P.launches += 1;
        (void)hipEventDestroy(P.start[i]);
        (void)hipEventDestroy(P.stop[i]);
    }
    P.start.clear();
    P.stop.clear();
    P.pend_bytes.clear();
    return HELMHOLTZ_OK;
}

// Record an event before a profiled launch; returns false when profiling is off.
bool prof_begin(const helmholtz_s* h, int kernel, hipStream_t s) {
    if (!h->prof_on) return false;
    helmholtz_s::Prof& P = h->prof[kernel];
    if (P.start.size() >= 256 && prof_flush(h, kernel) != HELMHOLTZ_OK) return false;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return false;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return false;
    }
    P.start.push_back(a);
    P.stop.push_back(b);
    P.pend_bytes.push_back(0.0);
    (void)hipEventRecord(a, s);
    return true;
}

void prof_end(const helmholtz_s* h, int kernel, double bytes, hipStream_t s) {
    helmholtz_s::Prof& P = h->prof[kernel];
    P.pend_bytes.back() = bytes;
    (void)hipEventRecord(P.stop.back(), s);
}

CgState cg_state(const helmholtz_s* h) {
    return CgState{h->partial, h->partial2, h->pstride, h->sc, h->active, h->upd,
                   h->hsc,     h->hact,     h->hseq};
}

template <typename T>
LevelView<T> view(const helmholtz_s* h, int l) {
    const Level& v = h->lev[l];
    const LevelData<T>& d = [&]() -> const LevelData<T>& {
        if constexpr (std::is_same<T, double>::value) return v.d;
        else return v.f;
    }();
    return LevelView<T>{v.ncol, h->nz, v.nvp, v.N,  v.nbr, v.fface, v.pofs,
                        d.kh,   d.kv,  d.dl,  d.cc, d.mm,  d.kv2,  d.s};
}

// ---- sweep launch: compile-time bound on levels per thread ---------------
inline int sweep_mid(int nz) { return nz / 2; }

// Whether one sweep over level l streams far more data than the last-level
// cache (256 MiB Infinity Cache) holds: then its read-once streams bypass the
// cache (k_sweep with NTS). On smaller levels the next kernel finds the
// previous one's output there, and plain accesses are faster.
bool streams_past_cache(const helmholtz_s* h, int l, int batch, size_t word) {
    constexpr int64_t kLastLevelCache = int64_t(256) << 20;
    // kh[2], cc, mm and the neighbour couplings; b, x, x_new per right-hand side
    return int64_t(h->lev[l].nvp) * int64_t(word) * (5 + 3 * int64_t(batch)) > kLastLevelCache;
}

// The sweep and the residual restriction stream past the cache only for one
// right-hand side: the members of a batch share each tile's coefficients
// through L2, so there the coefficients stay cached (float32 V-cycle at
// C384 x 70 with four right-hand sides: 7.19 -> 7.09 ms).
bool sweep_streams_past_cache(const helmholtz_s* h, int l, int batch, size_t word) {
    return batch == 1 && streams_past_cache(h, l, batch, word);
}

template <typename T, int JMAX, int MODE, int TC, bool VARIANTS>
void launch_sweep_b(const helmholtz_s* h, int l, const T* b, const T* x, const T* xc, T* y,
                    int batch, const int* active, hipStream_t s) {
    const Level& v = h->lev[l];
    using Tile = SweepTile<T, TC, kBlock>;
    const int ntile = (v.ncol + TC - 1) / TC;
    const int nvp_c = (l + 1 < h->L) ? h->lev[l + 1].nvp : 0;
    const bool prof = (l == 0 && MODE == kPlain) && prof_begin(h, HELMHOLTZ_PROF_SWEEP_FINE, s);
    const int rev = h->flip(l);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(ntile * batch), dim3(kBlock), Tile::lds_bytes(h->nz), s,
                           view<T>(h, l), b, x, xc, nvp_c, y, T(h->cfg.omega), batch, active,
                           sweep_mid(h->nz), rev);
    };
    // only the large levels use 32-column tiles and can stream past the cache
    constexpr bool kCanStream = TC == kTile;
    const bool nts = kCanStream && sweep_streams_past_cache(h, l, batch, sizeof(T));
    auto pick = [&](auto plain, auto streamed) {
        if constexpr (kCanStream) {
            if (nts) {
                go(streamed);
                return;
            }
        }
        go(plain);
    };
    if constexpr (VARIANTS) {
        if (h->weighted && h->adj)
            pick(k_sweep<T, JMAX, MODE, TC, kBlock, 0, false, kRowWT>,
                 k_sweep<T, JMAX, MODE, TC, kBlock, 0, false, kRowWT, kCanStream>);
        else if (h->weighted)
            pick(k_sweep<T, JMAX, MODE, TC, kBlock, 0, false, kRowW>,
                 k_sweep<T, JMAX, MODE, TC, kBlock, 0, false, kRowW, kCanStream>);
        else
            pick(k_sweep<T, JMAX, MODE, TC, kBlock, 0, true>,
                 k_sweep<T, JMAX, MODE, TC, kBlock, 0, true, kSym, kCanStream>);
    } else {
        pick(k_sweep<T, JMAX, MODE, TC, kBlock, 0, false>,
             k_sweep<T, JMAX, MODE, TC, kBlock, 0, false, kSym, kCanStream>);
    }
    if (prof)  // b, x, kh[2], cc, mm (, kv2) read; x_new written
        prof_end(h, HELMHOLTZ_PROF_SWEEP_FINE,
                 (h->nine ? 8.0 : 7.0) * sizeof(T) * double(batch) * h->nz * v.ncol, s);
}

// Large levels: 32-column tiles (8 level groups, several workgroups per CU).
// Small levels cannot fill the GPU and are bound by the latency of a few
// dependent steps per thread: 8-column tiles with 32 level groups let each
// thread load its few levels in one batch.
template <typename T, int MODE, int TC>
void launch_sweep_tc(const helmholtz_s* h, int l, const T* b, const T* x, const T* xc, T* y,
                     int batch, const int* active, hipStream_t s) {
    constexpr int KG = kBlock / TC;
    const int jn = (h->nz + KG - 1) / KG;
#define HH_SWEEP_BUCKET(J, V)                                                    \
    if (jn <= J) {                                                               \
        launch_sweep_b<T, J, MODE, TC, V>(h, l, b, x, xc, y, batch, active, s);  \
        return;                                                                  \
    }
    if (h->nine || h->weighted) {
        // the 9-cell and weighted operators: fewer compiled bucket sizes
        HH_SWEEP_BUCKET(4, true)
        if (TC == 32) {
            HH_SWEEP_BUCKET(9, true)
            HH_SWEEP_BUCKET(15, true)
        }
        return;
    }
    HH_SWEEP_BUCKET(1, false)
    HH_SWEEP_BUCKET(2, false)
    HH_SWEEP_BUCKET(4, false)
    if (TC == 32) {
        HH_SWEEP_BUCKET(9, false)
        HH_SWEEP_BUCKET(15, false)
    }
#undef HH_SWEEP_BUCKET
}

template <typename T, int MODE>
void launch_sweep_m(const helmholtz_s* h, int l, const T* b, const T* x, const T* xc, T* y,
                    int batch, const int* active, hipStream_t s) {
    if (h->lev[l].ncol < kSmallSweepCols)
        launch_sweep_tc<T, MODE, 8>(h, l, b, x, xc, y, batch, active, s);
    else
        launch_sweep_tc<T, MODE, 32>(h, l, b, x, xc, y, batch, active, s);
}

// Levels too small to fill the GPU are bound by the latency of a few dependent
// steps per thread; their kernels give each thread less work.
inline bool small_level(const helmholtz_s* h, int l) { return h->lev[l].ncol < 4096; }

template <typename T>
void launch_sweep(const helmholtz_s* h, int l, int mode, const T* b, const T* x, const T* xc,
                  T* y, int batch, const int* active, hipStream_t s) {
    switch (mode) {
        case kZero: launch_sweep_m<T, kZero>(h, l, b, x, xc, y, batch, active, s); break;
        case kPlain: launch_sweep_m<T, kPlain>(h, l, b, x, xc, y, batch, active, s); break;
        case kProlong: launch_sweep_m<T, kProlong>(h, l, b, x, xc, y, batch, active, s); break;
        default: launch_sweep_m<T, kProlongZero>(h, l, b, x, xc, y, batch, active, s); break;
    }
}

template <typename T>
void launch_resid_restrict(const helmholtz_s* h, int l, const T* b, const T* x, T* bc, int batch,
                           const int* active, hipStream_t s) {
    const Level& c = h->lev[l + 1];
    const int ntile = (c.ncol + kBlock - 1) / kBlock;
    // one level per thread on small levels (one dependent step), four otherwise
    const int kchunk = small_level(h, l) ? 1 : kApplyChunk;
    const int nkc = (h->nz + kchunk - 1) / kchunk;
    const dim3 grid(ntile * nkc * batch);
    // child pairs load as one vector when b and x are aligned to two elements
    // (the level's own arrays always are: tiles hold an even number of values)
    const uintptr_t al = 2 * sizeof(T);
    const bool pair = reinterpret_cast<uintptr_t>(b) % al == 0 &&
                      reinterpret_cast<uintptr_t>(x) % al == 0;
    const int rev = h->flip(l);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, view<T>(h, l), c.child, c.ncol, c.nvp,
                           b, x, bc, batch, kchunk, nkc, active, rev);
    };
    // paired loads (the library's own buffers): streamed past the cache on
    // levels far larger than it
    const bool nts = sweep_streams_past_cache(h, l, batch, sizeof(T));
    auto pick = [&](auto plain, auto streamed) {
        if (nts) go(streamed);
        else go(plain);
    };
    // each operator form: where the coarse panels tile into patches (32 x 8,
    // else 16 x 16 coarse cells), the children's values go through LDS
    // (k_resid_restrict_lds); otherwise the gathering kernel
    auto form = [&](auto k2, auto sc) {
        constexpr bool K2 = decltype(k2)::value;
        constexpr int SC = decltype(sc)::value;
        if (pair && c.N % 32 == 0)
            pick(k_resid_restrict_lds<T, false, 32, K2, SC>,
                 k_resid_restrict_lds<T, true, 32, K2, SC>);
        else if (pair && c.N % 16 == 0)
            pick(k_resid_restrict_lds<T, false, 16, K2, SC>,
                 k_resid_restrict_lds<T, true, 16, K2, SC>);
        else if (pair)
            pick(k_resid_restrict<T, false, true, K2, SC>,
                 k_resid_restrict<T, false, true, K2, SC, true>);
        else
            go(k_resid_restrict<T, false, false, K2, SC>);
    };
    using Sym = std::integral_constant<int, kSym>;
    if (!x) {
        if (pair)
            pick(k_resid_restrict<T, true, true>,
                 k_resid_restrict<T, true, true, false, kSym, true>);
        else go(k_resid_restrict<T, true, false>);
    } else if (h->nine) {
        form(std::true_type{}, Sym{});
    } else if (h->weighted && h->adj) {
        form(std::false_type{}, std::integral_constant<int, kRowWT>{});
    } else if (h->weighted) {
        form(std::false_type{}, std::integral_constant<int, kRowW>{});
    } else {
        form(std::false_type{}, Sym{});
    }
}

template <typename T>
void launch_apply(const helmholtz_s* h, int l, const T* x, T* y, int batch, int dot,
                  const int* active, hipStream_t s, const T* w = nullptr) {
    const Level& v = h->lev[l];
    const int ntile = (v.ncol + kBlock - 1) / kBlock;
    const int nkc = (h->nz + kApplyChunk - 1) / kApplyChunk;
    const dim3 grid(ntile * nkc * batch);
    const bool prof = (l == 0 && sizeof(T) == 8) && prof_begin(h, HELMHOLTZ_PROF_APPLY_FINE, s);
    const int rev = h->flip(l);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, view<T>(h, l), x, y, w, batch, nkc,
                           cg_state(h), active, rev);
    };
    if (v.N % kTile == 0 && !h->weighted) {
        // the panels tile into patches of 64 x 4 (else 32 x 8) columns:
        // neighbours' values through LDS (7-point and 9-cell stencils; with
        // the row-weighted operator it was no faster: each thread's weights
        // must arrive before it publishes s x, H 227 -> 229, H^T 263 -> 278 us)
        auto patch = [&](auto nts, auto px, auto k2) {
            constexpr bool NT = decltype(nts)::value;
            constexpr int PX = decltype(px)::value;
            constexpr bool K2 = decltype(k2)::value;
            switch (dot) {
                case kDotXY: go(k_apply_lds<T, kDotXY, kApplyChunk, NT, PX, K2>); break;
                case kDotWY: go(k_apply_lds<T, kDotWY, kApplyChunk, NT, PX, K2>); break;
                case kDotWYYY: go(k_apply_lds<T, kDotWYYY, kApplyChunk, NT, PX, K2>); break;
                default: go(k_apply_lds<T, kDotNone, kApplyChunk, NT, PX, K2>); break;
            }
        };
        auto by_width = [&](auto nts, auto k2) {
            if (v.N % 64 == 0) patch(nts, std::integral_constant<int, 64>{}, k2);
            else patch(nts, std::integral_constant<int, 32>{}, k2);
        };
        if (streams_past_cache(h, l, batch, sizeof(T)))
            h->nine ? by_width(std::true_type{}, std::true_type{})
                    : by_width(std::true_type{}, std::false_type{});
        else
            h->nine ? by_width(std::false_type{}, std::true_type{})
                    : by_width(std::false_type{}, std::false_type{});
    } else if (h->weighted) {
        if (h->adj) {
            switch (dot) {
                case kDotXY: go(k_apply<T, kDotXY, kApplyChunk, false, kRowWT>); break;
                case kDotWY: go(k_apply<T, kDotWY, kApplyChunk, false, kRowWT>); break;
                case kDotWYYY: go(k_apply<T, kDotWYYY, kApplyChunk, false, kRowWT>); break;
                default: go(k_apply<T, kDotNone, kApplyChunk, false, kRowWT>); break;
            }
        } else {
            switch (dot) {
                case kDotXY: go(k_apply<T, kDotXY, kApplyChunk, false, kRowW>); break;
                case kDotWY: go(k_apply<T, kDotWY, kApplyChunk, false, kRowW>); break;
                case kDotWYYY: go(k_apply<T, kDotWYYY, kApplyChunk, false, kRowW>); break;
                default: go(k_apply<T, kDotNone, kApplyChunk, false, kRowW>); break;
            }
        }
    } else if (h->nine) {
        switch (dot) {
            case kDotXY: go(k_apply<T, kDotXY, kApplyChunk, true>); break;
            case kDotWY: go(k_apply<T, kDotWY, kApplyChunk, true>); break;
            case kDotWYYY: go(k_apply<T, kDotWYYY, kApplyChunk, true>); break;
            default: go(k_apply<T, kDotNone, kApplyChunk, true>); break;
        }
    } else if (streams_past_cache(h, l, batch, sizeof(T))) {
        switch (dot) {
            case kDotXY: go(k_apply<T, kDotXY, kApplyChunk, false, kSym, true>); break;
            case kDotWY: go(k_apply<T, kDotWY, kApplyChunk, false, kSym, true>); break;
            case kDotWYYY: go(k_apply<T, kDotWYYY, kApplyChunk, false, kSym, true>); break;
            default: go(k_apply<T, kDotNone, kApplyChunk, false, kSym, true>); break;
        }
    } else {
        switch (dot) {
            case kDotXY: go(k_apply<T, kDotXY, kApplyChunk>); break;
            case kDotWY: go(k_apply<T, kDotWY, kApplyChunk>); break;
            case kDotWYYY: go(k_apply<T, kDotWYYY, kApplyChunk>); break;
            default: go(k_apply<T, kDotNone, kApplyChunk>); break;
        }
    }
    if (prof)  // x, kh[2], kv, delta (, kv2) read; y written
        prof_end(h, HELMHOLTZ_PROF_APPLY_FINE,
                 (h->nine ? 7.0 : 6.0) * sizeof(T) * double(batch) * h->nz * v.ncol, s);
}

// ---- V-cycle (Algorithm 1) ------------------------------------------------
// Number of x writes on level l and the buffer that write j goes to: the
// writes alternate between out_l and tmp_l, assigned from the last one
// backwards so that the last lands in out_l.
inline int level_writes(const helmholtz_s* h, int l) {
    const helmholtz_config& cfg = h->cfg;
    return l == h->L - 1 ? cfg.n_coarse : cfg.n_pre + std::max(cfg.n_post, 1);
}

template <typename T>
T* write_dst(const helmholtz_s* h, int l, int j, T* out, T* tmp) {
    return ((level_writes(h, l) - 1 - j) % 2 == 0) ? out : tmp;
}

// Level l smooths b_l into out_l (Algorithm 1), using V.t[l] as the Jacobi
// ping-pong partner and V.b, V.x of the coarser levels.
template <typename T>
void vcycle_level(helmholtz_s* h, const VBufs<T>& V, int l, const T* b, T* out, int batch,
                  const int* active, hipStream_t s) {
    const helmholtz_config& cfg = h->cfg;
    T* tmp = V.t[l];
    const int W = level_writes(h, l);
    if (l == h->L - 1) {
        const T* prev = nullptr;
        for (int j = 0; j < W; ++j) {
            T* dst = write_dst<T>(h, l, j, out, tmp);
            launch_sweep<T>(h, l, j == 0 ? kZero : kPlain, b, prev, nullptr, dst, batch, active, s);
            prev = dst;
        }
        return;
    }
    int j = 0;
    const T* prev = nullptr;
    for (int i = 0; i < cfg.n_pre; ++i, ++j) {
        T* dst = write_dst<T>(h, l, j, out, tmp);
        launch_sweep<T>(h, l, j == 0 ? kZero : kPlain, b, prev, nullptr, dst, batch, active, s);
        prev = dst;
    }
    T* cb = V.b[l + 1];
    T* cx = V.x[l + 1];
    launch_resid_restrict<T>(h, l, b, prev, cb, batch, active, s);
    vcycle_level<T>(h, V, l + 1, cb, cx, batch, active, s);
    if (cfg.n_post == 0) {
        T* dst = write_dst<T>(h, l, j, out, tmp);
        const Level& v = h->lev[l];
        const int64_t total = int64_t(batch) * h->nz * v.ncol;
        hipLaunchKernelGGL((k_prolong<T>), dim3(grid_for(total)), dim3(kBlock), 0, s, v.ncol,
                           h->nz, v.nvp, h->lev[l + 1].nvp, v.parent, prev, cx, dst, total);
        return;
    }
    for (int i = 0; i < cfg.n_post; ++i, ++j) {
        T* dst = write_dst<T>(h, l, j, out, tmp);
        int mode = kPlain;
        if (i == 0) mode = prev ? kProlong : kProlongZero;
        launch_sweep<T>(h, l, mode, b, prev, cx, dst, batch, active, s);
        prev = dst;
    }
}

int check_batch(const helmholtz_s* h, int32_t batch) {
    if (!h) return HELMHOLTZ_EINVAL;
    if (batch < 1 || batch > h->B) return HELMHOLTZ_ESHAPE;
    return HELMHOLTZ_OK;
}

template <typename S, typename D>
void convert(const S* src, D* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<S, D>), dim3(grid_for(n)), dim3(kBlock), 0, s, src, dst, n);
}

// Finest-level vector between the ABI layout and the tiled layout, with a cast.
template <typename S, typename D, bool TO_TILED>
void retile(const helmholtz_s* h, const S* src, D* dst, int batch, hipStream_t s) {
    const Level& v = h->lev[0];
    hipLaunchKernelGGL((k_retile<S, D, TO_TILED>), dim3(v.ncolp / kTile * batch), dim3(kBlock), 0,
                       s, src, dst, v.ncol, h->nz, v.nvp);
}

// Algorithmic bytes of one V-cycle with these kernels (the words each kernel
// must move per unknown of its level, times the unknowns and the batch):
// first sweep from zero 4 words (b, two factors, x_new), further sweeps 7
// (b, x, two face couplings, two factors, x_new), residual + restriction 6.25
// (b, x, kh[2], kv, delta; a quarter-size coarse b), sweep with prolongation
// 7.25 (the coarse x), a lone prolongation 2.25; the 9-cell and the weighted
// operators add one word (kv2 or s) to every sweep and residual.
double vcycle_bytes(const helmholtz_s* h, int batch, size_t word) {
    const helmholtz_config& c = h->cfg;
    const double extra = (h->nine || h->weighted) ? 1.0 : 0.0;
    const double sw = 7.0 + extra;
    auto smooth = [&](int n) { return n > 0 ? 4.0 + sw * (n - 1) : 0.0; };
    double total = 0.0;
    for (int l = 0; l < h->L; ++l) {
        double w;
        if (l == h->L - 1) {
            w = smooth(c.n_coarse);
        } else {
            w = smooth(c.n_pre) + (c.n_pre > 0 ? 6.25 + extra : 1.25);
            w += c.n_post > 0 ? sw + 0.25 + sw * (c.n_post - 1) : 2.25;
        }
        total += w * double(h->nz) * h->lev[l].ncol;
    }
    return total * double(batch) * double(word);
}

// z = M r on the finest level in the handle's precision (tiled vectors). The
// float32 V-cycle reads r32 (the level-0 float32 right-hand side, which the
// Krylov kernels keep equal to float(r)) and leaves z32 in the level-0 float32
// solution buffer; r and z are then not touched. `prof`: time the V-cycle
// with the kernel timing hook (the solves).
int precondition(helmholtz_s* h, const double* r, double* z, int batch, const int* active,
                 hipStream_t s, bool prof = false) {
    const bool mixed = h->cfg.mg_precision == HELMHOLTZ_FP32;
    prof = prof && prof_begin(h, HELMHOLTZ_PROF_VCYCLE, s);
    if (!mixed) {
        vcycle_level<double>(h, h->vb64, 0, r, z, batch, active, s);
    } else {
        vcycle_level<float>(h, h->vb32, 0, h->vb32.b[0], h->vb32.x[0], batch, active, s);
    }
    if (prof) prof_end(h, HELMHOLTZ_PROF_VCYCLE, vcycle_bytes(h, batch, mixed ? 4 : 8), s);
    return last_error();
}

// Wait until the device has published sequence number `seq` for every
// right-hand side with need[i] != 0 (written by the last block of a norm
// reduction into host-coherent memory). Polls the flags; falls back on the
// stream state so that a failed launch cannot leave the host spinning.
int wait_published(helmholtz_s* h, hipStream_t s, const std::vector<int>& need, int seq) {
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    for (unsigned spin = 1;; ++spin) {
        bool done = true;
        for (size_t i = 0; i < need.size(); ++i)
            if (need[i] && __atomic_load_n(&h->hseq[i], __ATOMIC_ACQUIRE) != seq) {
                done = false;
                break;
            }
        if (done) return HELMHOLTZ_OK;
        if (spin % 256 == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                // the stream is idle: the values must be there now
                for (size_t i = 0; i < need.size(); ++i)
                    if (need[i] && __atomic_load_n(&h->hseq[i], __ATOMIC_ACQUIRE) != seq)
                        return HELMHOLTZ_EHIP;
                return HELMHOLTZ_OK;
            }
            if (q != hipErrorNotReady) return HELMHOLTZ_EHIP;
            if (clock::now() - t0 > std::chrono::seconds(120)) return HELMHOLTZ_EHIP;
        }
    }
}

// out = M u for float64 tiled vectors (float32 V-cycles convert on the way in
// and out through the level-0 float32 buffers).
int precondition_into(helmholtz_s* h, const double* u, double* out, int batch, const int* active,
                      hipStream_t s) {
    const bool mixed = h->cfg.mg_precision == HELMHOLTZ_FP32;
    if (!mixed) {
        const bool prof = prof_begin(h, HELMHOLTZ_PROF_VCYCLE, s);
        vcycle_level<double>(h, h->vb64, 0, u, out, batch, active, s);
        if (prof) prof_end(h, HELMHOLTZ_PROF_VCYCLE, vcycle_bytes(h, batch, 8), s);
    } else {
        const VBufs<float>& V = h->vb32;
        const int64_t n = int64_t(batch) * h->nvp;
        convert<double, float>(u, V.b[0], n, s);
        const bool prof = prof_begin(h, HELMHOLTZ_PROF_VCYCLE, s);
        vcycle_level<float>(h, V, 0, V.b[0], V.x[0], batch, active, s);
        if (prof) prof_end(h, HELMHOLTZ_PROF_VCYCLE, vcycle_bytes(h, batch, 4), s);
        convert<float, double>(V.x[0], out, n, s);
    }
    return last_error();
}

// Right-preconditioned BiCGStab (Section 4.1) after the shared start
// (x = 0, r = r0 = b, rho = ||b||^2 published). Per iteration two products
// with H and two V-cycles; the inner products (r0, v), (t, s) with (t, t),
// and (r0, r) with ||r||^2 are the four global sums of Section 3.7. it/rel
// are updated for every right-hand side that was active in an iteration.
int bicgstab_loop(helmholtz_s* h, double* x, int batch, double rtol, int maxiter,
                  const std::vector<double>& bnorm2, std::vector<int32_t>& it,
                  std::vector<double>& rel, hipStream_t s) {
    const Level& v0 = h->lev[0];
    const int64_t n = h->nvp;
    const int ntile32 = v0.ncolp / kTile;
    const int ntile0 = (v0.ncol + kBlock - 1) / kBlock;
    const int nkc0 = (h->nz + kApplyChunk - 1) / kApplyChunk;
    const dim3 red(kRedBlocks * batch), blk(kBlock), fin(kFinBlock), tgrid(ntile32 * batch);
    const CgState st = cg_state(h);
    std::vector<int> was_active(batch);
    bool broke = false;
    // Everything of an iteration up to its x and r update skips the
    // right-hand sides whose device flag the last norm cleared, so, as in CG,
    // it is queued before the host reads that norm when the norm is predicted
    // to stay above 4x the tolerance (the update and the published norm are
    // queued after the read: the host mirror holds one iteration's values).
    const bool ahead = !h->prof_on;
    auto first_half = [&](int iter) -> int {
        // p = r + beta (p - omega v); p_hat = M p; v = H p_hat; alpha = rho / (r0, v)
        hipLaunchKernelGGL(k_bicg_p, red, blk, 0, s, h->r, h->q, h->p, n, kRedBlocks, h->sc,
                           h->active, iter == 1 ? 1 : 0);
        if (int e = precondition_into(h, h->p, h->z, batch, h->active, s)) return e;
        launch_apply<double>(h, 0, h->z, h->q, batch, kDotWY, h->active, s, h->r0);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinBiAlpha),
                           ntile0 * nkc0, 0);
        // s = r - alpha v; s_hat = M s; t = H s_hat; omega = (t, s) / (t, t)
        hipLaunchKernelGGL(k_bicg_s, red, blk, 0, s, h->r, h->q, h->s, n, kRedBlocks, h->sc,
                           h->active);
        if (int e = precondition_into(h, h->s, h->sh, batch, h->active, s)) return e;
        launch_apply<double>(h, 0, h->sh, h->t, batch, kDotWYYY, h->active, s, h->s);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinBiOmega),
                           ntile0 * nkc0, 0);
        return last_error();
    };
    std::vector<double> fac(batch, 0.05), rel_prev(batch, 1.0);
    auto expect_more = [&]() {
        for (int i = 0; i < batch; ++i)
            if (h->hact[i] && rel_prev[i] * fac[i] > 4.0 * rtol) return true;
        return false;
    };
    if (int e = first_half(1)) return e;
    for (int iter = 1;; ++iter) {
        for (int i = 0; i < batch; ++i) was_active[i] = h->hact[i];
        // x += alpha p_hat + omega s_hat; r = s - omega t; (r0, r), ||r||^2, published
        hipLaunchKernelGGL(k_bicg_xr, tgrid, blk, 0, s, x, h->r, h->z, h->sh, h->s, h->t, h->r0,
                           v0.ncol, h->nz, v0.nvp, st);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinBiRR), ntile32, iter);
        const bool queued = ahead && iter < maxiter && expect_more();
        if (queued)
            if (int e = first_half(iter + 1)) return e;
        if (last_error() != HELMHOLTZ_OK) return HELMHOLTZ_EHIP;
        if (int e = wait_published(h, s, was_active, iter)) return e;
        bool still = false;
        for (int i = 0; i < batch; ++i) {
            if (!was_active[i]) continue;
            it[i] = iter;
            const double rr = h->hsc[i * kScal + kRR];
            if (!std::isfinite(rr)) {
                HH_CHECK(hipStreamSynchronize(s));
                return HELMHOLTZ_ENONFINITE;
            }
            rel[i] = std::sqrt(rr / bnorm2[i]);
            fac[i] = rel[i] / rel_prev[i];
            rel_prev[i] = rel[i];
            broke = broke || h->hsc[i * kScal + kBreak] != 0.0;
            still = still || h->hact[i];
        }
        if (!still) break;
        if (iter >= maxiter) {
            broke = true;
            break;
        }
        if (!queued)
            if (int e = first_half(iter + 1)) return e;
    }
    // the caller may read x as soon as this returns on the host
    HH_CHECK(hipStreamSynchronize(s));
    return broke ? HELMHOLTZ_NOT_CONVERGED : HELMHOLTZ_OK;
}

int create_impl(const helmholtz_config* cfg, const double* kh, const double* kv,
                const double* kv2, const double* delta, const double* sw, void* workspace,
                size_t workspace_bytes, helmholtz_stream_t stream_, helmholtz_t* out);
int set_coefficients(helmholtz_s* h, const double* kh, const double* kv, const double* kv2,
                     const double* delta, const double* sw, hipStream_t s);

// Level vectors b, x, t of every level for `batch` right-hand sides, carved
// from `base`; returns the bytes they take.
template <typename T>
size_t carve_levels(const helmholtz_s* h, uintptr_t base, int batch, VBufs<T>& V) {
    Carver cv{base};
    for (int l = 0; l < h->L; ++l) {
        const size_t nv = size_t(batch) * size_t(h->lev[l].nvp);
        V.b[l] = cv.take<T>(nv);
        V.x[l] = cv.take<T>(nv);
        V.t[l] = cv.take<T>(nv);
    }
    return cv.off;
}

// One V-cycle from the ABI layout to the ABI layout with the level vectors in
// the static scratch array (helmholtz_vcycle_noalloc).
template <typename T>
int vcycle_in_scratch(helmholtz_s* h, const double* b, double* x, int batch, hipStream_t s) {
    VBufs<T> V;
    if (carve_levels<T>(h, reinterpret_cast<uintptr_t>(h->scratch), batch, V) > kScratchBytes)
        return HELMHOLTZ_ESCRATCH;
    retile<double, T, true>(h, b, V.b[0], batch, s);
    vcycle_level<T>(h, V, 0, V.b[0], V.x[0], batch, nullptr, s);
    retile<T, double, false>(h, V.x[0], x, batch, s);
    return last_error();
}

// Weighted handles run the calls that take H^T with the transposed kernels.
struct AdjointScope {
    helmholtz_s* h;
    bool old;
    explicit AdjointScope(helmholtz_s* h_) : h(h_), old(h_->adj) { h->adj = h->weighted; }
    ~AdjointScope() { h->adj = old; }
};

}  // namespace

// ===========================================================================
extern "C" {

size_t helmholtz_workspace_bytes(const helmholtz_config* cfg) {
    if (!config_ok(cfg) || shape_error(cfg) != HELMHOLTZ_OK) return 0;
    helmholtz_s tmp;
    init_shape(&tmp, cfg);
    Carver cv{0};
    layout(&tmp, cv);
    return cv.off;
}

const char* helmholtz_strerror(int code) {
    switch (code) {
        case HELMHOLTZ_OK: return "ok";
        case HELMHOLTZ_NOT_CONVERGED: return "solve reached maxiter before rtol";
        case HELMHOLTZ_EINVAL: return "invalid argument, configuration or coefficient";
        case HELMHOLTZ_ESHAPE: return "invalid shape (N, nz, levels or batch)";
        case HELMHOLTZ_EWORKSPACE: return "workspace missing, too small or misaligned";
        case HELMHOLTZ_ENONFINITE: return "non-finite value (NaN or Inf)";
        case HELMHOLTZ_EHIP: return "HIP runtime error";
        case HELMHOLTZ_ESCRATCH:
            return "level vectors exceed the static scratch of the allocation-free entry point";
        default: return "unknown error code";
    }
}

int helmholtz_mesh_tables(int32_t N, int32_t* nbr, int32_t* ftab, int32_t* parent) {
    if (N < 1 || !nbr || !ftab) return HELMHOLTZ_EINVAL;
    if (2 * 6 * int64_t(N) * N >= (int64_t(1) << 31)) return HELMHOLTZ_ESHAPE;
    build_neighbours(N, nbr);
    build_face_table(N, nbr, ftab);
    if (parent && N % 2 == 0) build_parent(N, parent);
    return HELMHOLTZ_OK;
}

int helmholtz_create(const helmholtz_config* cfg, const double* kh, const double* kv,
                     const double* delta, void* workspace, size_t workspace_bytes,
                     helmholtz_stream_t stream_, helmholtz_t* out) {
    if (!out) return HELMHOLTZ_EINVAL;
    *out = nullptr;
    if (config_ok(cfg) && (cfg->stencil == 9 || cfg->weighted)) return HELMHOLTZ_EINVAL;
    return create_impl(cfg, kh, kv, nullptr, delta, nullptr, workspace, workspace_bytes, stream_,
                       out);
}

int helmholtz_create9(const helmholtz_config* cfg, const double* kh, const double* kv,
                      const double* kv2, const double* delta, void* workspace,
                      size_t workspace_bytes, helmholtz_stream_t stream_, helmholtz_t* out) {
    if (!out) return HELMHOLTZ_EINVAL;
    *out = nullptr;
    if (config_ok(cfg) && cfg->weighted) return HELMHOLTZ_EINVAL;
    return create_impl(cfg, kh, kv, kv2, delta, nullptr, workspace, workspace_bytes, stream_, out);
}

int helmholtz_create_weighted(const helmholtz_config* cfg, const double* kh, const double* kv,
                              const double* delta, const double* s, void* workspace,
                              size_t workspace_bytes, helmholtz_stream_t stream_,
                              helmholtz_t* out) {
    if (!out) return HELMHOLTZ_EINVAL;
    *out = nullptr;
    if (config_ok(cfg) && (!cfg->weighted || !s)) return HELMHOLTZ_EINVAL;
    return create_impl(cfg, kh, kv, nullptr, delta, s, workspace, workspace_bytes, stream_, out);
}

}  // extern "C"

namespace {

int create_impl(const helmholtz_config* cfg, const double* kh, const double* kv,
                const double* kv2, const double* delta, const double* sw, void* workspace,
                size_t workspace_bytes, helmholtz_stream_t stream_, helmholtz_t* out) {
    if (!out) return HELMHOLTZ_EINVAL;
    *out = nullptr;
    if (!config_ok(cfg)) return HELMHOLTZ_EINVAL;
    if (int e = shape_error(cfg)) return e;
    if (!kh || !delta || (cfg->nz > 1 && !kv)) return HELMHOLTZ_EINVAL;
    const bool nine = cfg->stencil == 9;
    if (nine != (kv2 != nullptr) && !(nine && cfg->nz <= 2)) return HELMHOLTZ_EINVAL;
    if ((cfg->weighted == 1) != (sw != nullptr)) return HELMHOLTZ_EINVAL;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % HELMHOLTZ_WORKSPACE_ALIGN))
        return HELMHOLTZ_EWORKSPACE;
    const size_t need = helmholtz_workspace_bytes(cfg);
    if (workspace_bytes < need) return HELMHOLTZ_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream_);
    // padding columns of the tiled arrays must read as zero
    if (hipMemsetAsync(workspace, 0, need, s) != hipSuccess) return HELMHOLTZ_EHIP;

    helmholtz_s* h = new (std::nothrow) helmholtz_s;
    if (!h) return HELMHOLTZ_EINVAL;
    init_shape(h, cfg);
    Carver cv{reinterpret_cast<uintptr_t>(workspace)};
    layout(h, cv);
    h->ws_bytes = need;
    auto fail = [&](int code) {
        helmholtz_destroy(h);
        return code;
    };
    if (int e = scratch_of_current_device(&h->scratch, &h->device)) return fail(e);
    // host-coherent pinned memory: the device publishes the CG scalars here
    if (hipHostMalloc(reinterpret_cast<void**>(&h->hsc),
                      size_t(h->B) * kScal * sizeof(double) + size_t(h->B) * 2 * sizeof(int) + 16,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        h->hsc = nullptr;
        return fail(HELMHOLTZ_EHIP);
    }
    h->hact = reinterpret_cast<int*>(h->hsc + size_t(h->B) * kScal);
    h->hseq = h->hact + h->B;
    h->hflags = h->hseq + h->B;
    for (int i = 0; i < h->B; ++i) h->hseq[i] = -1;

    // mesh tables of every level, built on the host and copied once
    const int nz = h->nz;
    std::vector<int32_t> tab;
    for (int l = 0; l < h->L; ++l) {
        Level& v = h->lev[l];
        const size_t nc = size_t(v.ncol);
        tab.assign(4 * nc, 0);
        build_neighbours(v.N, tab.data());
        std::vector<int32_t> ft(4 * nc);
        build_face_table(v.N, tab.data(), ft.data());
        if (hipMemcpyAsync(v.nbr, tab.data(), 4 * nc * sizeof(int32_t), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(HELMHOLTZ_EHIP);
        // W and S faces: stored face slot * ncol + owner -> offset in the tiled kh
        std::vector<uint32_t> ff(2 * nc);
        for (size_t c = 0; c < nc; ++c) {
            for (int w = 0; w < 2; ++w) {
                const int32_t f = ft[(w == 0 ? 1 : 3) * nc + c];
                const int slot = f >= v.ncol ? 1 : 0, owner = f - slot * v.ncol;
                ff[w * nc + c] = uint32_t(slot) * uint32_t(v.nvp) +
                                 uint32_t((owner / kTile) * kTile * nz + owner % kTile);
            }
        }
        if (hipMemcpyAsync(v.fface, ff.data(), 2 * nc * sizeof(uint32_t), hipMemcpyHostToDevice,
                           s) != hipSuccess)
            return fail(HELMHOLTZ_EHIP);
        std::vector<int32_t> par, po;
        if (v.parent) {
            par.resize(nc);
            build_parent(v.N, par.data());
            if (hipMemcpyAsync(v.parent, par.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice,
                               s) != hipSuccess)
                return fail(HELMHOLTZ_EHIP);
            // prolongation offsets: the parent and the parents of the outward
            // E/W (W for even i, E for odd i) and N/S (S for even j, N for
            // odd j) neighbours, as tiled offsets on the coarse level
            auto tb = [&](int32_t cc) { return (cc / kTile) * kTile * nz + cc % kTile; };
            po.resize(3 * nc);
            for (size_t c = 0; c < nc; ++c) {
                const int i = int(c % v.N), j = int((c / v.N) % v.N);
                const int32_t ew = tab[((i & 1) ? 0 : 1) * nc + c];
                const int32_t ns = tab[((j & 1) ? 2 : 3) * nc + c];
                po[c] = tb(par[c]);
                po[nc + c] = tb(par[ew]);
                po[2 * nc + c] = tb(par[ns]);
            }
            if (hipMemcpyAsync(v.pofs, po.data(), 3 * nc * sizeof(int32_t), hipMemcpyHostToDevice,
                               s) != hipSuccess)
                return fail(HELMHOLTZ_EHIP);
        }
        if (v.child) {
            std::vector<int32_t> ch(4 * nc);
            build_children(v.N, ch.data());
            if (hipMemcpyAsync(v.child, ch.data(), 4 * nc * sizeof(int32_t), hipMemcpyHostToDevice,
                               s) != hipSuccess)
                return fail(HELMHOLTZ_EHIP);
        }
        // the host vectors must stay alive until the copies have run
        if (hipStreamSynchronize(s) != hipSuccess) return fail(HELMHOLTZ_EHIP);
    }

    if (int e = set_coefficients(h, kh, kv, kv2, delta, sw, s)) return fail(e);
    *out = h;
    return HELMHOLTZ_OK;
}

// Coefficients of every level: finest from the caller (validated), coarser by
// re-discretisation, then the column factors and the float32 copies.
// Synchronises `s` once.
int set_coefficients(helmholtz_s* h, const double* kh, const double* kv, const double* kv2,
                     const double* delta, const double* sw, hipStream_t s) {
    const int nz = h->nz;
    if (hipMemsetAsync(h->flags, 0, 4 * sizeof(int), s) != hipSuccess) return HELMHOLTZ_EHIP;
    {
        Level& v = h->lev[0];
        const int64_t nv = int64_t(nz) * v.ncol;
        hipLaunchKernelGGL(k_setup_fine, dim3(grid_for(nv)), dim3(kBlock), 0, s, v.ncol, nz,
                           v.nvp, kh, kv, delta, kv2, sw, v.d.kh, v.d.kv, v.d.dl,
                           kv2 ? v.d.kv2 : nullptr, sw ? v.d.s : nullptr, h->flags);
    }
    for (int l = 1; l < h->L; ++l) {
        Level& f = h->lev[l - 1];
        Level& c = h->lev[l];
        const int64_t nv = int64_t(nz) * c.ncol;
        hipLaunchKernelGGL(k_coarsen, dim3(grid_for(nv)), dim3(kBlock), 0, s, c.ncol, nz, f.nvp,
                           c.nvp, c.child, f.d.kh, f.d.kv, f.d.dl, f.d.kv2, f.d.s, c.d.kh,
                           c.d.kv, c.d.dl, c.d.kv2, c.d.s);
    }
    for (int l = 0; l < h->L; ++l) {
        Level& v = h->lev[l];
        hipLaunchKernelGGL(k_factor, dim3((v.ncol + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                           view<double>(h, l), sweep_mid(nz), v.d.cc, v.d.mm);
        // float32 copies, rounded once from float64 (padding included)
        const int64_t nv = v.nvp;
        convert<double, float>(v.d.kh, v.f.kh, 2 * nv, s);
        convert<double, float>(v.d.kv, v.f.kv, nv, s);
        convert<double, float>(v.d.dl, v.f.dl, nv, s);
        convert<double, float>(v.d.cc, v.f.cc, nv, s);
        convert<double, float>(v.d.mm, v.f.mm, nv, s);
        if (h->nine) convert<double, float>(v.d.kv2, v.f.kv2, nv, s);
        if (h->weighted) convert<double, float>(v.d.s, v.f.s, nv, s);
    }
    if (last_error() != HELMHOLTZ_OK) return HELMHOLTZ_EHIP;
    if (hipMemcpyAsync(h->hflags, h->flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return HELMHOLTZ_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return HELMHOLTZ_EHIP;
    if (h->hflags[0] & 1) return HELMHOLTZ_ENONFINITE;
    if (h->hflags[0] & 2) return HELMHOLTZ_EINVAL;
    return HELMHOLTZ_OK;
}

}  // namespace

extern "C" {

int helmholtz_update(helmholtz_t h, const double* kh, const double* kv, const double* kv2,
                     const double* delta, const double* s, helmholtz_stream_t stream) {
    if (!h || !kh || !delta || (h->nz > 1 && !kv)) return HELMHOLTZ_EINVAL;
    if ((kv2 != nullptr) != (h->nine && h->nz > 2)) return HELMHOLTZ_EINVAL;
    if ((s != nullptr) != h->weighted) return HELMHOLTZ_EINVAL;
    return set_coefficients(h, kh, kv, kv2, delta, s, reinterpret_cast<hipStream_t>(stream));
}

int helmholtz_profile_enable(helmholtz_t h, int enable) {
    if (!h) return HELMHOLTZ_EINVAL;
    for (int k = 0; k < HELMHOLTZ_PROF_COUNT; ++k) {
        if (int e = prof_flush(h, k)) return e;
        h->prof[k].ms = h->prof[k].bytes = 0.0;
        h->prof[k].launches = 0;
    }
    h->prof_on = enable != 0;
    return HELMHOLTZ_OK;
}

int helmholtz_profile_read(helmholtz_t h, int32_t kernel, double* ms, int64_t* launches,
                           double* bytes) {
    if (!h || kernel < 0 || kernel >= HELMHOLTZ_PROF_COUNT) return HELMHOLTZ_EINVAL;
    if (int e = prof_flush(h, kernel)) return e;
    if (ms) *ms = h->prof[kernel].ms;
    if (launches) *launches = h->prof[kernel].launches;
    if (bytes) *bytes = h->prof[kernel].bytes;
    return HELMHOLTZ_OK;
}

int helmholtz_destroy(helmholtz_t h) {
    if (!h) return HELMHOLTZ_EINVAL;
    for (int k = 0; k < HELMHOLTZ_PROF_COUNT; ++k) (void)prof_flush(h, k);
    if (h->hsc) (void)hipHostFree(h->hsc);
    delete h;
    return HELMHOLTZ_OK;
}

int helmholtz_apply(helmholtz_t h, const double* x, double* y, int32_t batch,
                    helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!x || !y) return HELMHOLTZ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    retile<double, double, true>(h, x, h->p, batch, s);
    launch_apply<double>(h, 0, h->p, h->q, batch, kDotNone, nullptr, s);
    retile<double, double, false>(h, h->q, y, batch, s);
    return last_error();
}

int helmholtz_vcycle(helmholtz_t h, const double* b, double* x, int32_t batch,
                     helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!b || !x) return HELMHOLTZ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (h->cfg.mg_precision == HELMHOLTZ_FP64) {
        retile<double, double, true>(h, b, h->r, batch, s);
        if (int e = precondition(h, h->r, h->z, batch, nullptr, s)) return e;
        retile<double, double, false>(h, h->z, x, batch, s);
    } else {
        const VBufs<float>& V = h->vb32;
        retile<double, float, true>(h, b, V.b[0], batch, s);
        if (int e = precondition(h, nullptr, nullptr, batch, nullptr, s)) return e;
        retile<float, double, false>(h, V.x[0], x, batch, s);
    }
    return last_error();
}

int helmholtz_vcycle_noalloc(helmholtz_t h, const double* b, double* x, int32_t batch,
                             helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!b || !x) return HELMHOLTZ_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HELMHOLTZ_EHIP;
    if (dev != h->device || !h->scratch) return HELMHOLTZ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (h->cfg.mg_precision == HELMHOLTZ_FP64) return vcycle_in_scratch<double>(h, b, x, batch, s);
    return vcycle_in_scratch<float>(h, b, x, batch, s);
}

int helmholtz_vcycle_f32(helmholtz_t h, const float* b, float* x, int32_t batch,
                         helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!b || !x) return HELMHOLTZ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const VBufs<float>& V = h->vb32;
    retile<float, float, true>(h, b, V.b[0], batch, s);
    vcycle_level<float>(h, V, 0, V.b[0], V.x[0], batch, nullptr, s);
    retile<float, float, false>(h, V.x[0], x, batch, s);
    return last_error();
}

int helmholtz_solve(helmholtz_t h, const double* b, double* x, int32_t batch, double rtol,
                    int32_t maxiter, int32_t* iters, double* relres, helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!b || !x || maxiter < 1 || !(rtol >= 0.0)) return HELMHOLTZ_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = h->nvp;  // tiled vector length (elementwise kernels)
    const Level& v0 = h->lev[0];
    const int ntile32 = v0.ncolp / kTile;
    const dim3 tgrid(ntile32 * batch);
    const bool mixed = h->cfg.mg_precision == HELMHOLTZ_FP32;
    const bool flex = h->cfg.cg_variant == HELMHOLTZ_CG_FLEXIBLE;
    const bool bicg = h->cfg.cg_variant == HELMHOLTZ_BICGSTAB;
    float* r32 = mixed && !bicg ? h->vb32.b[0] : nullptr;
    float* z32 = mixed ? h->vb32.x[0] : nullptr;
    const dim3 red(kRedBlocks * batch), blk(kBlock), fin(kFinBlock);
    const CgState st = cg_state(h);

    // the host mirror doubles as staging for the initial scalars
    for (int i = 0; i < batch; ++i) {
        for (int j = 0; j < kScal; ++j) h->hsc[i * kScal + j] = 0.0;
        h->hsc[i * kScal + kRtol2] = rtol * rtol;
        __atomic_store_n(&h->hseq[i], -1, __ATOMIC_RELEASE);
    }
    HH_CHECK(hipMemcpyAsync(h->sc, h->hsc, size_t(batch) * kScal * sizeof(double),
                            hipMemcpyHostToDevice, s));
    // x = 0, r = b, ||b||^2
    // (CG writes x in its first update; the right-hand sides that do not
    // start are zeroed after the norms)
    hipLaunchKernelGGL(k_cg_init, tgrid, blk, 0, s, b, bicg ? x : nullptr, h->r, r32,
                       bicg ? h->r0 : nullptr, v0.ncol, h->nz, v0.nvp, st);
    hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinBB), ntile32, 0);
    if (!bicg) hipLaunchKernelGGL(k_cg_zero_idle, tgrid, blk, 0, s, x, v0.ncol, h->nz, st);
    if (last_error() != HELMHOLTZ_OK) return HELMHOLTZ_EHIP;

    // vectors far larger than the last-level cache: the streams that are not
    // read again soon bypass it (see the kernels)
    const bool vnt = streams_past_cache(h, 0, batch, sizeof(double));
    auto dot_rz = [&](const double* q) {
        const int rev = h->flip(0);
        auto go = [&](auto kern, auto z) {
            hipLaunchKernelGGL(kern, red, blk, 0, s, h->r, z, q, n, kRedBlocks, st, rev);
        };
        if (mixed) vnt ? go(k_dot_rz<float, true>, z32) : go(k_dot_rz<float, false>, z32);
        else vnt ? go(k_dot_rz<double, true>, h->z) : go(k_dot_rz<double, false>, h->z);
    };
    // p = z + beta p, with the x update owed from the last iteration (xmode)
    auto p_update = [&](int init, int xmode) {
        const int rev = h->flip(0);
        auto go = [&](auto kern, auto z) {
            hipLaunchKernelGGL(kern, tgrid, blk, 0, s, z, h->p, x, v0.ncol, h->nz, v0.nvp, st,
                               init, xmode, rev);
        };
        if (mixed) vnt ? go(k_p_update<float, true>, z32) : go(k_p_update<float, false>, z32);
        else vnt ? go(k_p_update<double, true>, h->z) : go(k_p_update<double, false>, h->z);
    };
    // the owed x update where the iteration stops, for the right-hand sides
    // that `sel` names (see k_cg_x)
    auto x_update = [&](int xmode, int sel) {
        const int rev = h->flip(0);
        if (vnt)
            hipLaunchKernelGGL(k_cg_x<true>, tgrid, blk, 0, s, x, h->p, v0.ncol, h->nz, v0.nvp,
                               st, xmode, sel, rev);
        else
            hipLaunchKernelGGL(k_cg_x<false>, tgrid, blk, 0, s, x, h->p, v0.ncol, h->nz, v0.nvp,
                               st, xmode, sel, rev);
    };
    // z = M r, rho = r.z, p = z
    auto cg_start = [&]() -> int {
        if (int e = precondition(h, h->r, h->z, batch, h->active, s, true)) return e;
        dot_rz(nullptr);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinRho), kRedBlocks, 0);
        p_update(1, kXNone);
        return last_error();
    };
    // z = M r and beta of the next iteration
    auto cg_next_m = [&]() -> int {
        if (int e = precondition(h, h->r, h->z, batch, h->active, s, true)) return e;
        dot_rz(flex ? h->q : nullptr);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st,
                           int(flex ? kFinBetaFlex : kFinBeta), kRedBlocks, 0);
        return last_error();
    };

    // Work queued ahead of the host's decisions. The host reads each published
    // norm before it decides how to go on, and the GPU would sit idle through
    // that round trip and the next launch (~25 us; about 2.5 % of a float32
    // solve at C192 x 70). Every kernel of M r, r.z and beta skips the
    // right-hand sides whose device flag the norm reduction cleared, so the
    // host may queue them before it knows the norm: the results are the same
    // either way, and a wrong guess costs only launches that return at once.
    // Off while the timing hooks are on, so that each timed V-cycle is a whole
    // one.
    const bool ahead = !bicg && !h->prof_on;
    if (ahead)
        if (int e = cg_start()) return e;  // b = 0 or not finite: flag cleared

    std::vector<int> need(batch, 1);
    if (int e = wait_published(h, s, need, 0)) return e;
    std::vector<double> bnorm2(batch);
    std::vector<int32_t> it(batch, 0);
    std::vector<double> rel(batch, 0.0);
    bool any = false, finite = true;
    for (int i = 0; i < batch; ++i) {
        bnorm2[i] = h->hsc[i * kScal + kBB];
        finite = finite && std::isfinite(bnorm2[i]);
        any = any || h->hact[i];
        rel[i] = h->hact[i] ? 1.0 : 0.0;
    }
    auto finish = [&](int status) {
        for (int i = 0; i < batch; ++i) {
            if (iters) iters[i] = it[i];
            if (relres) relres[i] = rel[i];
        }
        return status;
    };
    // x of the idle right-hand sides is cleared after the norms: let it land
    if (!finite || !any) HH_CHECK(hipStreamSynchronize(s));
    if (!finite) return HELMHOLTZ_ENONFINITE;
    if (!any) return finish(HELMHOLTZ_OK);
    if (bicg) return finish(bicgstab_loop(h, x, batch, rtol, maxiter, bnorm2, it, rel, s));
    if (!ahead)
        if (int e = cg_start()) return e;

    // The next norm predicted from the last one and the last contraction
    // (1/20 before there is one): if some right-hand side is expected to stay
    // above 4x the tolerance, M r of the next iteration is queued ahead;
    // otherwise the x update of those that stop is.
    std::vector<double> fac(batch, 0.05), rel_prev(batch, 1.0);
    auto expect_more = [&]() {
        for (int i = 0; i < batch; ++i)
            if (h->hact[i] && rel_prev[i] * fac[i] > 4.0 * rtol) return true;
        return false;
    };

    const int ntile0 = (h->lev[0].ncol + kBlock - 1) / kBlock;
    const int nkc0 = (h->nz + kApplyChunk - 1) / kApplyChunk;
    std::vector<int> was_active(batch);
    int status = HELMHOLTZ_OK;
    for (int iter = 1;; ++iter) {
        for (int i = 0; i < batch; ++i) was_active[i] = h->hact[i];
        const bool more = ahead && iter < maxiter && expect_more();
        // q = H p, alpha = rho / p.q
        launch_apply<double>(h, 0, h->p, h->q, batch, kDotXY, h->active, s);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinAlpha), ntile0 * nkc0,
                           0);
        // r -= alpha q, ||r||^2 and the convergence flags, published; the
        // matching x += alpha p is owed (applied with the next p update, or
        // by x_update where the iteration stops)
        const int rev = h->flip(0);
        if (vnt)
            hipLaunchKernelGGL(k_cg_update<true>, tgrid, blk, 0, s, h->r, r32, h->q, v0.ncol,
                               h->nz, v0.nvp, st, rev);
        else
            hipLaunchKernelGGL(k_cg_update<false>, tgrid, blk, 0, s, h->r, r32, h->q, v0.ncol,
                               h->nz, v0.nvp, st, rev);
        hipLaunchKernelGGL(k_finalize, dim3(batch), fin, 0, s, st, int(kFinRR), ntile32, iter);
        const int xmode = iter == 1 ? kXSet : kXAdd;  // x is first written here
        // queued ahead of the norm: M r of the next iteration, or the x update
        // of the right-hand sides that stop here (no-op for the others)
        const bool queued_m = more, queued_x = ahead && !more;
        if (queued_m)
            if (int e = cg_next_m()) return e;
        if (queued_x) x_update(xmode, kXDone);
        if (last_error() != HELMHOLTZ_OK) return HELMHOLTZ_EHIP;
        if (int e = wait_published(h, s, was_active, iter)) return e;
        bool still = false, some_done = false;
        for (int i = 0; i < batch; ++i) {
            if (!was_active[i]) continue;
            it[i] = iter;
            const double rr = h->hsc[i * kScal + kRR];
            if (!std::isfinite(rr)) {
                HH_CHECK(hipStreamSynchronize(s));
                return finish(HELMHOLTZ_ENONFINITE);
            }
            rel[i] = std::sqrt(rr / bnorm2[i]);
            fac[i] = rel[i] / rel_prev[i];
            rel_prev[i] = rel[i];
            still = still || h->hact[i];
            some_done = some_done || !h->hact[i];
        }
        if (!still || iter >= maxiter) {
            if (!queued_x) x_update(xmode, kXAll);
            else if (still) x_update(xmode, kXLive);
            if (still) status = HELMHOLTZ_NOT_CONVERGED;
            break;
        }
        if (some_done && !queued_x) x_update(xmode, kXDone);
        // z = M r, beta (unless queued ahead), p = z + beta p (with the owed
        // x update)
        if (!queued_m)
            if (int e = cg_next_m()) return e;
        p_update(0, xmode);
    }
    // the caller may read x as soon as this returns on the host
    HH_CHECK(hipStreamSynchronize(s));
    return finish(status);
}

int helmholtz_bandwidth_kernel(int32_t kind, const float* a, const float* b, float* c, int64_t n,
                               float sv, helmholtz_stream_t stream) {
    if (n <= 0 || n % 4 != 0) return HELMHOLTZ_EINVAL;
    const int64_t nblk = (n + kStreamPerBlock - 1) / kStreamPerBlock;
    if (nblk >= (int64_t(1) << 31)) return HELMHOLTZ_ESHAPE;
    auto aligned = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const float4* b4 = reinterpret_cast<const float4*>(b);
    float4* c4 = reinterpret_cast<float4*>(c);
    const int64_t n4 = n / 4;
    const dim3 grid(static_cast<unsigned>(nblk)), blk(kBlock);
    switch (kind) {
        case HELMHOLTZ_BW_READ:
            if (!a || !c || !aligned(a)) return HELMHOLTZ_EINVAL;
            hipLaunchKernelGGL(k_stream<kStreamRead>, grid, blk, 0, s, a4, b4, c4, n4, sv, c);
            break;
        case HELMHOLTZ_BW_WRITE:
            if (!c || !aligned(c)) return HELMHOLTZ_EINVAL;
            hipLaunchKernelGGL(k_stream<kStreamWrite>, grid, blk, 0, s, a4, b4, c4, n4, sv, c);
            break;
        case HELMHOLTZ_BW_COPY:
            if (!a || !c || !aligned(a) || !aligned(c)) return HELMHOLTZ_EINVAL;
            hipLaunchKernelGGL(k_stream<kStreamCopy>, grid, blk, 0, s, a4, b4, c4, n4, sv, c);
            break;
        case HELMHOLTZ_BW_TRIAD:
            if (!a || !b || !c || !aligned(a) || !aligned(b) || !aligned(c)) return HELMHOLTZ_EINVAL;
            hipLaunchKernelGGL(k_stream<kStreamTriad>, grid, blk, 0, s, a4, b4, c4, n4, sv, c);
            break;
        default:
            return HELMHOLTZ_EINVAL;
    }
    return last_error();
}

int helmholtz_face_grad(helmholtz_t h, const double* lam, const double* x, int32_t batch,
                        double* g_kh, double* g_kv, double* g_delta, helmholtz_stream_t stream) {
    return helmholtz_face_grad9(h, lam, x, batch, g_kh, g_kv, nullptr, g_delta, stream);
}

int helmholtz_face_grad9(helmholtz_t h, const double* lam, const double* x, int32_t batch,
                         double* g_kh, double* g_kv, double* g_kv2, double* g_delta,
                         helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!lam || !x || !g_kh || !g_delta || (h->nz > 1 && !g_kv)) return HELMHOLTZ_EINVAL;
    if (g_kv2 && !h->nine) return HELMHOLTZ_EINVAL;
    if (h->weighted) return HELMHOLTZ_EINVAL;  // helmholtz_face_grad_weighted
    const Level& v = h->lev[0];
    const int64_t total = int64_t(h->nz) * v.ncol;
    const int grid = int((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_face_grad, dim3(grid), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), v.ncol, h->nz, v.nbr, lam, x, batch,
                       g_kh, g_kv, g_delta, h->nz > 2 ? g_kv2 : nullptr);
    return last_error();
}

int helmholtz_apply_adjoint(helmholtz_t h, const double* x, double* y, int32_t batch,
                            helmholtz_stream_t stream) {
    if (!h) return HELMHOLTZ_EINVAL;
    AdjointScope scope(h);
    return helmholtz_apply(h, x, y, batch, stream);
}

int helmholtz_vcycle_adjoint(helmholtz_t h, const double* b, double* x, int32_t batch,
                             helmholtz_stream_t stream) {
    if (!h) return HELMHOLTZ_EINVAL;
    AdjointScope scope(h);
    return helmholtz_vcycle(h, b, x, batch, stream);
}

int helmholtz_solve_adjoint(helmholtz_t h, const double* g, double* lam, int32_t batch,
                            double rtol, int32_t maxiter, int32_t* iters, double* relres,
                            helmholtz_stream_t stream) {
    if (!h) return HELMHOLTZ_EINVAL;
    AdjointScope scope(h);
    return helmholtz_solve(h, g, lam, batch, rtol, maxiter, iters, relres, stream);
}

int helmholtz_face_grad_weighted(helmholtz_t h, const double* lam, const double* x,
                                 int32_t batch, double* g_kh, double* g_kv, double* g_delta,
                                 double* g_s, helmholtz_stream_t stream) {
    if (int e = check_batch(h, batch)) return e;
    if (!h->weighted) return HELMHOLTZ_EINVAL;
    if (!lam || !x || !g_kh || !g_delta || !g_s || (h->nz > 1 && !g_kv)) return HELMHOLTZ_EINVAL;
    const Level& v = h->lev[0];
    const int64_t total = int64_t(h->nz) * v.ncol;
    const int grid = int((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_face_grad_w, dim3(grid), dim3(kBlock), 0,
                       reinterpret_cast<hipStream_t>(stream), view<double>(h, 0), lam, x, batch,
                       g_kh, g_kv, g_delta, g_s);
    return last_error();
}

}  // extern "C"

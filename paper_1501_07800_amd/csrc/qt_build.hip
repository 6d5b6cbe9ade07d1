// Building a quadtree matrix from a block list, copying it back out, and the
// derived operand forms (fp32 copy, bf16 hi/lo split) and count histograms.
//
// Representation (Sec. 3.1 and 4.1 of the paper): blocks sorted by Morton
// key, so every quadtree node covers a contiguous run; leaves are lb x lb
// block grids stored as three 64-bit occupancy masks plus the index of their
// first block; every level above holds a 4-entry child table per node, -1
// marking a NIL child. Nodes carry no global offsets, only their Morton key.
#include "qt_internal.h"
#include "qt_morton.h"

#include <algorithm>
#include <atomic>
#include <set>

namespace qt {

// ------------------------------------------------------------ allocation

static std::mutex g_pool_mu;
static std::set<int> g_pool_ready;

static void ensure_pool() {
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_ready.count(dev)) return;
    hipMemPool_t pool;
    QT_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
    uint64_t thr = ~0ull;
    QT_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
    g_pool_ready.insert(dev);
}

static std::atomic<const Allocator*> g_allocator{nullptr};

const Allocator* current_allocator() { return g_allocator.load(std::memory_order_acquire); }

void set_allocator(const Allocator* a) { g_allocator.store(a, std::memory_order_release); }

void* dev_alloc(size_t bytes, hipStream_t s, const Allocator** who) {
    const Allocator* a = current_allocator();
    *who = a;
    void* p = nullptr;
    if (a) {
        p = a->alloc(bytes, (void*)s, a->ctx);
        if (!p) fail(QT_ERR_OOM, "the installed allocator returned no memory");
        if (reinterpret_cast<uintptr_t>(p) & 255) {
            a->free_(p, (void*)s, a->ctx);
            fail(QT_ERR_DEVICE, "the installed allocator returned memory not aligned to 256 bytes");
        }
        return p;
    }
    ensure_pool();
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        hip_check(e, "hipMallocAsync");
    }
    return p;
}

void dev_free(void* p, hipStream_t s, const Allocator* who) {
    if (!p) return;
    if (who)
        who->free_(p, (void*)s, who->ctx);
    else
        (void)hipFreeAsync(p, s);
}

// --------------------------------------------------------------- kernels

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_build_keys(const int32_t* __restrict__ I, const int32_t* __restrict__ J, int64_t n,
                             int64_t nbr, int64_t nbc, uint64_t* __restrict__ keys,
                             int32_t* __restrict__ perm, int32_t* __restrict__ err) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int32_t i = I[t], j = J[t];
    if (i < 0 || j < 0 || i >= nbr || j >= nbc) {
        atomicOr(err, 1);
        keys[t] = (uint64_t)t;
    } else {
        keys[t] = morton_key((uint32_t)i, (uint32_t)j);
    }
    perm[t] = (int32_t)t;
}

__global__ void k_build_dups(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ err) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 1 && t < n && keys[t] == keys[t - 1]) atomicOr(err, 2);
}

// dst block t = src block perm[t]; one workgroup copies one block.
template <class T>
__global__ void k_gather_blocks(const T* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                                int bb, T* __restrict__ dst) {
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        const T* s = src + (size_t)perm[t] * bb;
        T* d = dst + (size_t)t * bb;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = s[e];
    }
}

// Node counts of every level at once from the sorted block keys: node
// boundaries at level l are where the key prefix above shift(l) changes.
// cnt[l] for l = 0 .. L (L: the leaves); one ballot per wave and level.
__global__ void k_level_counts(const uint64_t* __restrict__ keys, int64_t n, int L, int leaf_shift,
                               int32_t* __restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = t < n;
    const uint64_t k = in ? keys[t] : 0, kp = (in && t > 0) ? keys[t - 1] : 0;
    for (int l = 0; l <= L; ++l) {
        const int sh = leaf_shift + 2 * (L - l);
        const bool first = in && (t == 0 || (sh < 64 ? (k >> sh) != (kp >> sh) : false));
        const uint64_t m = __ballot(first);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(cnt + l, (int32_t)__popcll(m));
    }
}

// Every level's tables in one pass. flags[l*n + t] = 1 when block t starts a
// node of level l (l = 0 .. L, L the leaves); with ex the exclusive scan of
// the concatenated flags, block t lies in node rank(l, t) = ex[l*n + t + 1] -
// ex[l*n] - 1 of level l. The flags and their scan are int32 while (L+1) n
// fits, int64 beyond.
constexpr int MAX_FUSED_LEVELS = 32;
struct LevelTables {
    int32_t* child[MAX_FUSED_LEVELS];     // levels 0 .. L-1: 4 per node, -1 for NIL (cleared first)
    uint64_t* key[MAX_FUSED_LEVELS];
    int32_t* base;                         // leaves
    uint64_t* lkey;
    uint64_t* mo;
    uint64_t* rm;
    uint64_t* cm;
};

__device__ __forceinline__ int level_shift(int l, int L, int leaf_shift) { return leaf_shift + 2 * (L - l); }

template <class I>
__global__ void k_level_flags(const uint64_t* __restrict__ keys, int64_t n, int L, int leaf_shift,
                              I* __restrict__ flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint64_t k = keys[t], kp = t > 0 ? keys[t - 1] : 0;
    for (int l = 0; l <= L; ++l) {
        const int sh = level_shift(l, L, leaf_shift);
        flags[(int64_t)l * n + t] = (t == 0 || (sh < 64 && (k >> sh) != (kp >> sh))) ? 1 : 0;
    }
}

template <class I>
__global__ void k_level_fill(const uint64_t* __restrict__ keys, int64_t n, int L, int lb_log,
                             const I* __restrict__ flags, const I* __restrict__ ex, LevelTables tb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int leaf_shift = 2 * lb_log;
    const uint64_t k = keys[t];
    auto rank = [&](int l) { return (int32_t)(ex[(int64_t)l * n + t + 1] - ex[(int64_t)l * n] - 1); };
    for (int l = 0; l < L; ++l) {
        const int sh = level_shift(l, L, leaf_shift);
        if (flags[(int64_t)l * n + t]) tb.key[l][rank(l)] = sh < 64 ? (k >> sh) : 0;
        if (flags[(int64_t)(l + 1) * n + t]) {   // t starts a child node: link it to its parent
            const int shc = sh - 2;                 // the child level's shift
            const int q = shc < 64 ? (int)((k >> shc) & 3) : 0;
            tb.child[l][4 * (int64_t)rank(l) + q] = rank(l + 1);
        }
    }
    if (!flags[(int64_t)L * n + t]) return;
    // t starts a leaf: its base, key and masks
    const int lb = 1 << lb_log;
    const uint64_t lk = k >> leaf_shift;
    const int32_t li = rank(L);
    uint64_t m0 = 0, m1 = 0, m2 = 0;
    for (int64_t u = t; u < n && (keys[u] >> leaf_shift) == lk; ++u) {
        const uint32_t q = (uint32_t)(keys[u] & ((1ull << leaf_shift) - 1));
        const uint32_t r = morton_row(q), c = morton_col(q);
        m0 |= 1ull << q;
        m1 |= 1ull << (r * lb + c);
        m2 |= 1ull << (c * lb + r);
    }
    tb.base[li] = (int32_t)t;
    tb.lkey[li] = lk;
    tb.mo[li] = m0;
    tb.rm[li] = m1;
    tb.cm[li] = m2;
}

__global__ void k_hist(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ rowcnt,
                       int32_t* __restrict__ colcnt) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint64_t k = keys[t];
    atomicAdd(rowcnt + morton_row(k), 1);
    atomicAdd(colcnt + morton_col(k), 1);
}

__global__ void k_f64_to_f32(const double* __restrict__ s, int64_t n, float* __restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = __double2float_rn(s[i]);
}

__global__ void k_f32_to_f64(const float* __restrict__ s, int64_t n, double* __restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (double)s[i];
}

// Round a binary32 value to bfloat16, nearest even, on the bit pattern.
__device__ inline uint16_t bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// hi = bf16(a32), lo = bf16(a32 - hi) per entry, row-major and transposed.
template <class T>
__global__ void k_bf16_split(const T* __restrict__ src, int64_t nblk, int b, uint16_t* __restrict__ hi,
                             uint16_t* __restrict__ lo, uint16_t* __restrict__ hi_t, uint16_t* __restrict__ lo_t) {
    const int64_t bb = (int64_t)b * b;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nblk * bb) return;
    float a = (float)src[i];   // fp64 -> fp32 rounds to nearest even
    uint16_t h = bf16_round(a);
    uint16_t l = bf16_round(a - bf16_to_f32(h));
    int64_t t = i / bb;
    int e = (int)(i - t * bb);
    int r = e / b, c = e - r * b;
    hi[i] = h;
    lo[i] = l;
    hi_t[t * bb + (int64_t)c * b + r] = h;
    lo_t[t * bb + (int64_t)c * b + r] = l;
}

__global__ void k_rowmajor_keys(const uint64_t* __restrict__ bkey, int64_t n, int64_t nbc,
                                uint64_t* __restrict__ rk, int32_t* __restrict__ perm) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    rk[t] = (uint64_t)morton_row(bkey[t]) * (uint64_t)nbc + morton_col(bkey[t]);
    perm[t] = (int32_t)t;
}

__global__ void k_coords(const uint64_t* __restrict__ bkey, const int32_t* __restrict__ perm, int64_t n,
                         int32_t* __restrict__ I, int32_t* __restrict__ J) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    uint64_t k = bkey[perm[t]];
    I[t] = (int32_t)morton_row(k);
    J[t] = (int32_t)morton_col(k);
}

template <class S, class D>
__global__ void k_gather_convert(const S* __restrict__ src, const int32_t* __restrict__ perm, int64_t n, int bb,
                                 D* __restrict__ dst) {
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        const S* s = src + (size_t)perm[t] * bb;
        D* d = dst + (size_t)t * bb;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = (D)s[e];
    }
}

template <>
__global__ void k_gather_convert<double, float>(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                                int64_t n, int bb, float* __restrict__ dst) {
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        const double* s = src + (size_t)perm[t] * bb;
        float* d = dst + (size_t)t * bb;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = __double2float_rn(s[e]);
    }
}

// One workgroup per requested block: binary search of its Morton key, then
// a copy (or zeros when the block is not stored).
template <class S, class D>
__global__ void k_get_blocks(const uint64_t* __restrict__ bkey, int64_t nblocks, int64_t nbr, int64_t nbc,
                             const S* __restrict__ vals, const int32_t* __restrict__ I,
                             const int32_t* __restrict__ J, int64_t count, int bb, D* __restrict__ out,
                             int32_t* __restrict__ found) {
    __shared__ int64_t pos;
    for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
        if (threadIdx.x == 0) {
            int64_t at = -1;
            const int32_t i = I[t], j = J[t];
            if (i >= 0 && j >= 0 && i < nbr && j < nbc) {
                const uint64_t k = morton_key((uint32_t)i, (uint32_t)j);
                int64_t lo = 0, hi = nblocks;           // first index with bkey >= k
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (bkey[mid] < k) lo = mid + 1; else hi = mid;
                }
                if (lo < nblocks && bkey[lo] == k) at = lo;
            }
            pos = at;
            found[t] = at >= 0 ? 1 : 0;
        }
        __syncthreads();
        const int64_t at = pos;
        D* d = out + (size_t)t * bb;
        if (at >= 0) {
            const S* src = vals + (size_t)at * bb;
            for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = (D)src[e];
        } else {
            for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = (D)0;
        }
        __syncthreads();
    }
}

template <>
__global__ void k_get_blocks<double, float>(const uint64_t* __restrict__ bkey, int64_t nblocks, int64_t nbr,
                                            int64_t nbc, const double* __restrict__ vals,
                                            const int32_t* __restrict__ I, const int32_t* __restrict__ J,
                                            int64_t count, int bb, float* __restrict__ out,
                                            int32_t* __restrict__ found) {
    __shared__ int64_t pos;
    for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
        if (threadIdx.x == 0) {
            int64_t at = -1;
            const int32_t i = I[t], j = J[t];
            if (i >= 0 && j >= 0 && i < nbr && j < nbc) {
                const uint64_t k = morton_key((uint32_t)i, (uint32_t)j);
                int64_t lo = 0, hi = nblocks;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (bkey[mid] < k) lo = mid + 1; else hi = mid;
                }
                if (lo < nblocks && bkey[lo] == k) at = lo;
            }
            pos = at;
            found[t] = at >= 0 ? 1 : 0;
        }
        __syncthreads();
        const int64_t at = pos;
        float* d = out + (size_t)t * bb;
        if (at >= 0) {
            const double* src = vals + (size_t)at * bb;
            for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = __double2float_rn(src[e]);
        } else {
            for (int e = threadIdx.x; e < bb; e += blockDim.x) d[e] = 0.f;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- helpers

static inline unsigned grid_for(int64_t n, int T = 256) {
    int64_t g = (n + T - 1) / T;
    return (unsigned)std::max<int64_t>(g, 1);
}

static inline unsigned block_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 1 << 20));
}

template <class T>
static T read_scalar(const T* dptr, hipStream_t s) {
    T v{};
    QT_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, s));
    QT_HIP(hipStreamSynchronize(s));
    return v;
}

uint64_t morton2(uint32_t r, uint32_t c) { return morton_key(r, c); }

static int ilog2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

// ------------------------------------------------------------ histograms

void build_histograms(qt_matrix* M, hipStream_t s) {
    std::lock_guard<std::mutex> lk(M->mu);
    if (M->hist.ready) return;
    Histograms h;
    h.rowcnt.resize(M->L + 1);
    h.colcnt.resize(M->L + 1);
    const int64_t nb_pad = (int64_t)M->lb << M->L;
    int64_t total = 2 * nb_pad;
    for (int l = 0; l <= M->L; ++l) total += 2 * (int64_t(1) << l);
    DBuf<int32_t> d(total, s);
    QT_HIP(hipMemsetAsync(d.p, 0, total * sizeof(int32_t), s));
    int64_t off = 0;
    std::vector<int64_t> offs;
    for (int l = 0; l <= M->L; ++l) {
        const int64_t side = int64_t(1) << l;
        const uint64_t* keys = (l < M->L) ? M->levels[l].key.p : M->leaves.key.p;
        const int64_t n = (l < M->L) ? M->levels[l].n : M->leaves.n;
        offs.push_back(off);
        if (n > 0) {
            k_hist<<<grid_for(n), 256, 0, s>>>(keys, n, d.p + off, d.p + off + side);
            QT_LAUNCH("k_hist");
        }
        off += 2 * side;
    }
    if (M->nblocks > 0) {
        k_hist<<<grid_for(M->nblocks), 256, 0, s>>>(M->bkey.p, M->nblocks, d.p + off, d.p + off + nb_pad);
        QT_LAUNCH("k_hist");
    }
    std::vector<int32_t> host(total);
    QT_HIP(hipMemcpyAsync(host.data(), d.p, total * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QT_HIP(hipStreamSynchronize(s));
    for (int l = 0; l <= M->L; ++l) {
        const int64_t side = int64_t(1) << l;
        h.rowcnt[l].assign(host.begin() + offs[l], host.begin() + offs[l] + side);
        h.colcnt[l].assign(host.begin() + offs[l] + side, host.begin() + offs[l] + 2 * side);
    }
    h.blk_row.assign(host.begin() + off, host.begin() + off + nb_pad);
    h.blk_col.assign(host.begin() + off + nb_pad, host.begin() + off + 2 * nb_pad);
    h.ready = true;
    M->hist = std::move(h);
}

// ----------------------------------------------------- operand forms

// A derived form was just queued on s: record its event there.
static void form_mark(hipEvent_t& ev, hipStream_t s) {
    if (!ev) QT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    QT_HIP(hipEventRecord(ev, s));
}

// Work queued on s from here on must see the form: wait for its event unless
// it has completed already (then the event is dropped, so later calls skip
// even the query). Called with M->mu held.
static void form_ready(hipEvent_t& ev, hipStream_t s) {
    if (!ev) return;
    const hipError_t q = hipEventQuery(ev);
    if (q == hipSuccess) {
        (void)hipEventDestroy(ev);
        ev = nullptr;
        return;
    }
    if (q != hipErrorNotReady) hip_check(q, "hipEventQuery");
    QT_HIP(hipStreamWaitEvent(s, ev, 0));
}

const double* operand_f64(qt_matrix* M, hipStream_t s) {
    if (M->vtype == QT_F64) return M->v64.p;
    std::lock_guard<std::mutex> lk(M->mu);
    if (!M->v64_cache.p && M->nblocks > 0) {
        const int64_t n = M->nblocks * (int64_t)M->b * M->b;
        M->v64_cache.alloc(n, s);
        k_f32_to_f64<<<grid_for(n), 256, 0, s>>>(M->v32.p, n, M->v64_cache.p);
        QT_LAUNCH("k_f32_to_f64");
        form_mark(M->ev_v64, s);
    }
    form_ready(M->ev_v64, s);
    return M->v64_cache.p;
}

const float* operand_f32(qt_matrix* M, hipStream_t s) {
    std::lock_guard<std::mutex> lk(M->mu);
    if (!M->v32.p && M->nblocks > 0) {
        const int64_t n = M->nblocks * (int64_t)M->b * M->b;
        M->v32.alloc(n, s);
        k_f64_to_f32<<<grid_for(n), 256, 0, s>>>(M->v64.p, n, M->v32.p);
        QT_LAUNCH("k_f64_to_f32");
        form_mark(M->ev_v32, s);
    }
    form_ready(M->ev_v32, s);
    return M->v32.p;
}

void operand_bf16(qt_matrix* M, hipStream_t s) {
    std::lock_guard<std::mutex> lk(M->mu);
    if (!M->bf_hi.p && M->nblocks > 0) {
        // all four parts are obtained before any is attached to the handle,
        // so a failed allocation leaves no partial form behind
        const int64_t n = M->nblocks * (int64_t)M->b * M->b;
        DBuf<uint16_t> hi(n, s), lo(n, s), hi_t(n, s), lo_t(n, s);
        if (M->vtype == QT_F64)
            k_bf16_split<double><<<grid_for(n), 256, 0, s>>>(M->v64.p, M->nblocks, M->b, hi.p, lo.p, hi_t.p, lo_t.p);
        else
            k_bf16_split<float><<<grid_for(n), 256, 0, s>>>(M->v32.p, M->nblocks, M->b, hi.p, lo.p, hi_t.p, lo_t.p);
        QT_LAUNCH("k_bf16_split");
        form_mark(M->ev_bf16, s);
        M->bf_hi = std::move(hi);
        M->bf_lo = std::move(lo);
        M->bf_hi_t = std::move(hi_t);
        M->bf_lo_t = std::move(lo_t);
    }
    form_ready(M->ev_bf16, s);
}

// ----------------------------------------------------------------- build

void build_tree_levels(qt_matrix* M, hipStream_t s);

// Block keys in Morton order and the quadtree levels of M (shape fields set,
// nblocks > 0) from a device block list; perm[t] receives the list position
// of the block at sorted position t. Rejects out-of-range and repeated (I, J).
static void build_structure(qt_matrix* M, const int32_t* pI, const int32_t* pJ, int64_t nblocks, int64_t nbr,
                            int64_t nbc, DBuf<int32_t>& perm, hipStream_t s) {
    int64_t npow2 = 1;
    while (npow2 < nblocks) npow2 <<= 1;
    DBuf<uint64_t> keys(npow2, s);
    perm.alloc(npow2, s);
    DBuf<int32_t> derr(1, s);
    QT_HIP(hipMemsetAsync(derr.p, 0, sizeof(int32_t), s));
    k_build_keys<<<grid_for(nblocks), 256, 0, s>>>(pI, pJ, nblocks, nbr, nbc, keys.p, perm.p, derr.p);
    QT_LAUNCH("k_build_keys");
    bitonic_sort(keys.p, perm.p, nblocks, s);
    k_build_dups<<<grid_for(nblocks), 256, 0, s>>>(keys.p, nblocks, derr.p);
    QT_LAUNCH("k_build_dups");
    const int32_t err = read_scalar(derr.p, s);
    if (err & 1) fail(QT_ERR_ARG, "block index out of range");
    if (err & 2) fail(QT_ERR_DUPLICATE, "the same (I, J) block is listed twice");
    M->bkey = std::move(keys);   // first nblocks entries are the sorted keys
    build_tree_levels(M, s);
}

qt_matrix* build(int64_t n_rows, int64_t n_cols, int32_t b, int32_t leaf, int64_t nblocks, const int32_t* I,
                 const int32_t* J, const double* values, qt_mem where, hipStream_t s) {
    if (n_rows < 0 || n_cols < 0 || nblocks < 0) fail(QT_ERR_ARG, "negative size");
    if (where != QT_MEM_HOST && where != QT_MEM_DEVICE) fail(QT_ERR_ARG, "bad memory kind");
    if (nblocks > 0 && (!I || !J || !values)) fail(QT_ERR_ARG, "NULL block list");
    if (b != 16 && b != 32 && b != 64) fail(QT_ERR_SHAPE, "block size must be 16, 32 or 64");
    if (leaf <= 0 || leaf % b) fail(QT_ERR_SHAPE, "leaf size must be a positive multiple of the block size");
    const int lb = leaf / b;
    if (lb & (lb - 1)) fail(QT_ERR_SHAPE, "leaf size / block size must be a power of two");
    if (lb > 8) fail(QT_ERR_SHAPE, "leaf size / block size must be at most 8");
    if (n_rows % b || n_cols % b) fail(QT_ERR_SHAPE, "dimensions must be multiples of the block size");
    const int64_t nbr = n_rows / b, nbc = n_cols / b;
    if (nbr > (int64_t(1) << 30) || nbc > (int64_t(1) << 30)) fail(QT_ERR_UNSUPPORTED, "too many blocks per side");
    if (nblocks > (int64_t(1) << 31) - 2) fail(QT_ERR_UNSUPPORTED, "too many blocks");

    std::unique_ptr<qt_matrix> M(new qt_matrix);
    M->n_rows = n_rows;
    M->n_cols = n_cols;
    M->b = b;
    M->leaf = leaf;
    M->lb = lb;
    M->lb_log = ilog2(lb);
    int64_t side = lb;
    int L = 0;
    while (side < std::max<int64_t>(std::max<int64_t>(nbr, nbc), 1)) {
        side *= 2;
        ++L;
    }
    M->L = L;
    M->vtype = QT_F64;
    M->nblocks = nblocks;
    M->stream = s;
    QT_HIP(hipGetDevice(&M->device));
    M->levels.resize(L);
    const int bb = b * b;

    if (nblocks == 0) {
        build_histograms(M.get(), s);
        return M.release();
    }

    // operands on the device
    DBuf<int32_t> dI, dJ;
    DBuf<double> dV;
    const int32_t* pI = I;
    const int32_t* pJ = J;
    const double* pV = values;
    if (where == QT_MEM_HOST) {
        dI.alloc(nblocks, s);
        dJ.alloc(nblocks, s);
        dV.alloc((size_t)nblocks * bb, s);
        QT_HIP(hipMemcpyAsync(dI.p, I, nblocks * sizeof(int32_t), hipMemcpyHostToDevice, s));
        QT_HIP(hipMemcpyAsync(dJ.p, J, nblocks * sizeof(int32_t), hipMemcpyHostToDevice, s));
        QT_HIP(hipMemcpyAsync(dV.p, values, (size_t)nblocks * bb * sizeof(double), hipMemcpyHostToDevice, s));
        pI = dI.p;
        pJ = dJ.p;
        pV = dV.p;
    }

    DBuf<int32_t> perm;
    build_structure(M.get(), pI, pJ, nblocks, nbr, nbc, perm, s);
    M->v64.alloc((size_t)nblocks * bb, s);
    k_gather_blocks<double><<<block_grid(nblocks), 256, 0, s>>>(pV, perm.p, nblocks, bb, M->v64.p);
    QT_LAUNCH("k_gather_blocks");
    build_histograms(M.get(), s);
    QT_HIP(hipStreamSynchronize(s));
    return M.release();
}

// Leaves and levels above, from the sorted block keys of M.
// The node-start flags of every level, their scan, and the tables from them.
template <class I>
static void fill_levels(qt_matrix* M, int64_t nflags, int shift, const LevelTables& tb, hipStream_t s) {
    const int64_t n = M->nblocks;
    DBuf<I> flags(nflags, s), ex(nflags + 1, s), tmp(scan_tmp_elems(nflags) + 1, s);
    k_level_flags<I><<<grid_for(n), 256, 0, s>>>(M->bkey.p, n, M->L, shift, flags.p);
    QT_LAUNCH("k_level_flags");
    exclusive_scan(flags.p, ex.p, nflags, tmp.p, s);
    k_level_fill<I><<<grid_for(n), 256, 0, s>>>(M->bkey.p, n, M->L, M->lb_log, flags.p, ex.p, tb);
    QT_LAUNCH("k_level_fill");
}

void build_tree_levels(qt_matrix* M, hipStream_t s) {
    const int64_t n = M->nblocks;
    const int shift = 2 * M->lb_log;
    // all node counts in one pass and one read-back, so the levels below
    // are built without further synchronization
    std::vector<int32_t> counts(M->L + 1);
    {
        DBuf<int32_t> dcnt(M->L + 1, s);
        k_fill_i32<<<1, 64, 0, s>>>(dcnt.p, M->L + 1, 0);
        QT_LAUNCH("k_fill_i32");
        k_level_counts<<<grid_for(n), 256, 0, s>>>(M->bkey.p, n, M->L, shift, dcnt.p);
        QT_LAUNCH("k_level_counts");
        QT_HIP(hipMemcpyAsync(counts.data(), dcnt.p, counts.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QT_HIP(hipStreamSynchronize(s));
    }
    const int32_t nleaves = counts[M->L];
    const int64_t nflags = (int64_t)(M->L + 1) * n;
    if (M->L >= MAX_FUSED_LEVELS) fail(QT_ERR_UNSUPPORTED, "quadtree too deep");
    ArenaPlan plan;
    std::vector<size_t> o_child(M->L), o_key(M->L);
    for (int l = 0; l < M->L; ++l) {
        o_child[l] = plan.take(4 * (size_t)counts[l] * sizeof(int32_t));
        o_key[l] = plan.take((size_t)counts[l] * sizeof(uint64_t));
    }
    const size_t child_end = plan.bytes;   // the child tables come first: one clear covers them
    const size_t o_base = plan.take((size_t)nleaves * sizeof(int32_t));
    const size_t o_lkey = plan.take((size_t)nleaves * sizeof(uint64_t));
    const size_t o_mo = plan.take((size_t)nleaves * sizeof(uint64_t));
    const size_t o_rm = plan.take((size_t)nleaves * sizeof(uint64_t));
    const size_t o_cm = plan.take((size_t)nleaves * sizeof(uint64_t));
    M->arena.alloc(plan.bytes, s);
    char* base = M->arena.p;
    LevelTables tb{};
    for (int l = 0; l < M->L; ++l) {
        TreeLevel& tl = M->levels[l];
        tl.n = counts[l];
        tl.child.view(base + o_child[l], 4 * (size_t)counts[l]);
        tl.key.view(base + o_key[l], counts[l]);
        tb.child[l] = tl.child.p;
        tb.key[l] = tl.key.p;
    }
    LeafLevel& lv = M->leaves;
    lv.n = nleaves;
    lv.base.view(base + o_base, nleaves);
    lv.key.view(base + o_lkey, nleaves);
    lv.mask_mo.view(base + o_mo, nleaves);
    lv.mask_rm.view(base + o_rm, nleaves);
    lv.mask_cm.view(base + o_cm, nleaves);
    tb.base = lv.base.p;
    tb.lkey = lv.key.p;
    tb.mo = lv.mask_mo.p;
    tb.rm = lv.mask_rm.p;
    tb.cm = lv.mask_cm.p;
    if (child_end > 0) {
        const int64_t words = (int64_t)(child_end / sizeof(int32_t));
        k_fill_i32<<<grid_for(words), 256, 0, s>>>((int32_t*)base, words, -1);
        QT_LAUNCH("k_fill_i32");
    }
    if (nflags < (int64_t(1) << 31) - 2)
        fill_levels<int32_t>(M, nflags, shift, tb, s);
    else
        fill_levels<int64_t>(M, nflags, shift, tb, s);
}

// ------------------------------------------------------------ copy out

// Copy-out into device arrays I, J, values (values may be NULL): row-major
// sort keys and the permutation go to rk / perm, which hold npow2 entries
// each (npow2 = the next power of two >= M->nblocks, as the sort needs).
static void rowmajor_copy(const qt_matrix* M, uint64_t* rk, int32_t* perm, int32_t* I, int32_t* J, void* values,
                          qt_prec out_type, hipStream_t s) {
    const int64_t n = M->nblocks;
    const int bb = M->b * M->b;
    const int64_t nbc = M->n_cols / M->b;
    k_rowmajor_keys<<<grid_for(n), 256, 0, s>>>(M->bkey.p, n, nbc, rk, perm);
    QT_LAUNCH("k_rowmajor_keys");
    bitonic_sort(rk, perm, n, s);
    k_coords<<<grid_for(n), 256, 0, s>>>(M->bkey.p, perm, n, I, J);
    QT_LAUNCH("k_coords");
    if (!values) return;   // pattern only
    const unsigned g = block_grid(n);
    if (M->vtype == QT_F64 && out_type == QT_F64)
        k_gather_convert<double, double><<<g, 256, 0, s>>>(M->v64.p, perm, n, bb, (double*)values);
    else if (M->vtype == QT_F64)
        k_gather_convert<double, float><<<g, 256, 0, s>>>(M->v64.p, perm, n, bb, (float*)values);
    else if (out_type == QT_F64)
        k_gather_convert<float, double><<<g, 256, 0, s>>>(M->v32.p, perm, n, bb, (double*)values);
    else
        k_gather_convert<float, float><<<g, 256, 0, s>>>(M->v32.p, perm, n, bb, (float*)values);
    QT_LAUNCH("k_gather_convert");
}

static int64_t pow2_at_least(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

void to_blocks(const qt_matrix* M, int32_t* I, int32_t* J, void* values, qt_prec out_type, qt_mem where,
               hipStream_t s) {
    if (out_type != QT_F64 && out_type != QT_F32) fail(QT_ERR_UNSUPPORTED, "output type must be F64 or F32");
    if (where != QT_MEM_HOST && where != QT_MEM_DEVICE) fail(QT_ERR_ARG, "bad memory kind");
    const int64_t n = M->nblocks;
    if (n == 0) return;
    if (!I || !J) fail(QT_ERR_ARG, "NULL output array");
    const int bb = M->b * M->b;
    const int64_t npow2 = pow2_at_least(n);
    DBuf<uint64_t> rk(npow2, s);
    DBuf<int32_t> perm(npow2, s);
    const size_t vbytes = values ? (size_t)n * bb * (out_type == QT_F64 ? sizeof(double) : sizeof(float)) : 0;
    DBuf<int32_t> tI, tJ;
    DBuf<char> tV;
    int32_t* oI = I;
    int32_t* oJ = J;
    void* oV = values;
    if (where == QT_MEM_HOST) {
        tI.alloc(n, s);
        tJ.alloc(n, s);
        if (values) tV.alloc(vbytes, s);
        oI = tI.p;
        oJ = tJ.p;
        oV = values ? (void*)tV.p : nullptr;
    }
    rowmajor_copy(M, rk.p, perm.p, oI, oJ, oV, out_type, s);
    if (where == QT_MEM_HOST) {
        QT_HIP(hipMemcpyAsync(I, oI, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QT_HIP(hipMemcpyAsync(J, oJ, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (values) QT_HIP(hipMemcpyAsync(values, oV, vbytes, hipMemcpyDeviceToHost, s));
        QT_HIP(hipStreamSynchronize(s));
    }
}

// -------------------------------------------- copy-out without allocation

// Scratch of the allocation-free copy-out: the row-major sort keys (8 bytes
// per entry) followed by the permutation (4 bytes per entry) of up to
// QT_NOALLOC_MAX_BLOCKS blocks, 12 MiB, one copy per device for the life of
// the process. Host code never passes `scratch` itself (on the host it names
// a stand-in, not device memory): it takes the array's device address once
// per device with hipGetSymbolAddress and uses that address only.
constexpr int64_t kNoAllocEntries = QT_NOALLOC_MAX_BLOCKS;
static __device__ __align__(256) uint64_t scratch[kNoAllocEntries + kNoAllocEntries / 2];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken on the first call
// made with that device current).
static void* scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(QT_ERR_UNSUPPORTED, "device ordinal beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(QT_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_addr[dev] = p;
    }
    return g_scratch_addr[dev];
}

void to_blocks_noalloc(const qt_matrix* M, int32_t* I, int32_t* J, void* values, qt_prec out_type, hipStream_t s) {
    if (out_type != QT_F64 && out_type != QT_F32) fail(QT_ERR_UNSUPPORTED, "output type must be F64 or F32");
    const int64_t n = M->nblocks;
    if (n > QT_NOALLOC_MAX_BLOCKS)
        fail(QT_ERR_UNSUPPORTED, "matrix has " + std::to_string(n) + " blocks; the allocation-free copy-out takes at most " +
                                     std::to_string((long long)QT_NOALLOC_MAX_BLOCKS));
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    if (dev != M->device) fail(QT_ERR_ARG, "the matrix lives on another device than the current one");
    uint64_t* rk = static_cast<uint64_t*>(scratch_address(dev));
    if (n == 0) return;
    if (!I || !J) fail(QT_ERR_ARG, "NULL output array");
    int32_t* perm = reinterpret_cast<int32_t*>(rk + kNoAllocEntries);
    // rk and perm are written in full (entries < n by the key kernel, the
    // rest up to the power of two by the sort's padding) before any read, so
    // nothing left by an earlier call is seen and nothing needs clearing.
    rowmajor_copy(M, rk, perm, I, J, values, out_type, s);
}

// ------------------------------------------------------------ norms
//
// Squared Frobenius norms of a matrix and of every submatrix in its
// quadtree (the paper's conclusions name such per-submatrix norms as an
// addition to the library, after Bock and Challacombe): of every block, one
// wave per block; of every leaf, the sum over its blocks; of every node
// above, the sum over its present children. A node's squared norm is at
// least each block's below it, whatever the order of the sums (every term is
// non-negative and rounding is monotone), which is what lets a product be
// dropped by its norm at any level.

template <class T>
__global__ __launch_bounds__(64) void k_block_norm2(const T* __restrict__ v, int64_t n, int bb,
                                                   double* __restrict__ out) {
    const int64_t t = blockIdx.x;
    if (t >= n) return;
    const T* x = v + (size_t)t * bb;
    double s = 0.0;
    for (int e = threadIdx.x; e < bb; e += 64) {
        const double d = (double)x[e];
        s += d * d;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if (threadIdx.x == 0) out[t] = s;
}

__global__ void k_leaf_norm2(const int32_t* __restrict__ base, const uint64_t* __restrict__ mo, int64_t n,
                             const double* __restrict__ bn2, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b0 = base[i], cnt = __popcll(mo[i]);
    double s = 0.0;
    for (int32_t k = 0; k < cnt; ++k) s += bn2[b0 + k];
    out[i] = s;
}

__global__ void k_node_norm2(const int32_t* __restrict__ child, int64_t n, const double* __restrict__ below,
                             double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t c = child[4 * i + q];
        if (c >= 0) s += below[c];
    }
    out[i] = s;
}

void build_norms(qt_matrix* M, hipStream_t s) {
    std::lock_guard<std::mutex> lk(M->mu);
    if (M->vsrc) fail(QT_ERR_UNSUPPORTED, "norms of a structure-only matrix");
    if (!M->bn2) {
        const int L = M->L;
        int64_t total = std::max<int64_t>(M->nblocks, 1) + M->leaves.n;
        for (int l = 0; l < L; ++l) total += M->levels[l].n;
        M->norms.alloc(total, s);
        double* p = M->norms.p;
        double* bn2 = p;
        p += std::max<int64_t>(M->nblocks, 1);
        const int bb = M->b * M->b;
        if (M->nblocks > 0) {
            if (M->vtype == QT_F64)
                k_block_norm2<double><<<(unsigned)M->nblocks, 64, 0, s>>>(M->v64.p, M->nblocks, bb, bn2);
            else
                k_block_norm2<float><<<(unsigned)M->nblocks, 64, 0, s>>>(M->v32.p, M->nblocks, bb, bn2);
            QT_LAUNCH("k_block_norm2");
        }
        std::vector<const double*> nn2(L + 1, nullptr);
        double* below = p;
        p += M->leaves.n;
        if (M->leaves.n > 0) {
            k_leaf_norm2<<<grid_for(M->leaves.n), 256, 0, s>>>(M->leaves.base.p, M->leaves.mask_mo.p, M->leaves.n,
                                                              bn2, below);
            QT_LAUNCH("k_leaf_norm2");
        }
        nn2[L] = below;
        for (int l = L - 1; l >= 0; --l) {
            double* here = p;
            p += M->levels[l].n;
            if (M->levels[l].n > 0) {
                k_node_norm2<<<grid_for(M->levels[l].n), 256, 0, s>>>(M->levels[l].child.p, M->levels[l].n, below,
                                                                     here);
                QT_LAUNCH("k_node_norm2");
            }
            nn2[l] = here;
            below = here;
        }
        M->nn2 = nn2;
        M->bn2 = bn2;
        form_mark(M->ev_norms, s);
    }
    form_ready(M->ev_norms, s);
}

__global__ void k_gather_f64(const double* __restrict__ src, const int32_t* __restrict__ idx, int64_t n,
                             double* __restrict__ dst);   // dst[i] = src[idx[i]] (below)

// The squared norms of M's blocks in (I, J) row-major order, and of M.
void norms_out(qt_matrix* M, double* block_norm2, double* total_norm2, qt_mem where, hipStream_t s) {
    build_norms(M, s);
    const int64_t n = M->nblocks;
    if (block_norm2 && n > 0) {
        const int64_t npow2 = pow2_at_least(n);
        DBuf<uint64_t> rk(npow2, s);
        DBuf<int32_t> perm(npow2, s);
        k_rowmajor_keys<<<grid_for(n), 256, 0, s>>>(M->bkey.p, n, M->n_cols / M->b, rk.p, perm.p);
        QT_LAUNCH("k_rowmajor_keys");
        bitonic_sort(rk.p, perm.p, n, s);
        DBuf<double> tmp;
        double* out = block_norm2;
        if (where == QT_MEM_HOST) {
            tmp.alloc(n, s);
            out = tmp.p;
        }
        k_gather_f64<<<grid_for(n), 256, 0, s>>>(M->bn2, perm.p, n, out);
        QT_LAUNCH("k_gather_f64");
        if (where == QT_MEM_HOST) QT_HIP(hipMemcpyAsync(block_norm2, tmp.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (total_norm2) {
        // the root's squared norm (0 for an all-NIL matrix)
        const bool any = M->L == 0 ? M->leaves.n > 0 : M->levels[0].n > 0;
        if (!any) {
            if (where == QT_MEM_HOST)
                *total_norm2 = 0.0;
            else
                QT_HIP(hipMemsetAsync(total_norm2, 0, sizeof(double), s));
        } else {
            QT_HIP(hipMemcpyAsync(total_norm2, M->nn2[0], sizeof(double),
                                  where == QT_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
        }
    }
    if (where == QT_MEM_HOST) QT_HIP(hipStreamSynchronize(s));
}

// The full symmetric matrix S from its upper block triangle A, as structure
// only: block (I, J), I <= J, of A is block (I, J) of S, and for I < J also
// block (J, I) of S, read transposed. S holds no values; its block map points
// every block of S at the block of A that holds it (top bit: transposed).
__global__ void k_mirror_flags(const uint64_t* __restrict__ bkey, int64_t n, int32_t* __restrict__ upper,
                               int32_t* __restrict__ err) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t i = morton_row(bkey[t]), j = morton_col(bkey[t]);
    upper[t] = i < j ? 1 : 0;
    if (i > j) atomicOr(err, 1);
}

// entries t < n: A's blocks; entry n + rank[t]: the mirror of strictly upper block t
__global__ void k_mirror_list(const uint64_t* __restrict__ bkey, int64_t n, const int32_t* __restrict__ upper,
                              const int32_t* __restrict__ rank, int32_t* __restrict__ I, int32_t* __restrict__ J,
                              int32_t* __restrict__ src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = (int32_t)morton_row(bkey[t]), j = (int32_t)morton_col(bkey[t]);
    I[t] = i;
    J[t] = j;
    src[t] = (int32_t)t;
    if (upper[t]) {
        const int64_t m = n + rank[t];
        I[m] = j;
        J[m] = i;
        src[m] = (int32_t)((uint32_t)t | PROD_TRANS);
    }
}

__global__ void k_gather_i32(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                             int32_t* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[perm[t]];
}

qt_matrix* symmetric_full(qt_matrix* A, hipStream_t s) {
    std::lock_guard<std::mutex> lk(A->mu);
    if (A->sym_full) return A->sym_full.get();
    if (A->n_rows != A->n_cols) fail(QT_ERR_SHAPE, "a symmetric matrix must be square");
    const int64_t n = A->nblocks;
    std::unique_ptr<qt_matrix> S(new qt_matrix);
    S->n_rows = A->n_rows;
    S->n_cols = A->n_cols;
    S->b = A->b;
    S->leaf = A->leaf;
    S->lb = A->lb;
    S->lb_log = A->lb_log;
    S->L = A->L;
    S->vtype = A->vtype;
    S->stream = s;
    S->device = A->device;
    S->levels.resize(S->L);
    S->vsrc = A;
    if (n > 0) {
        DBuf<int32_t> up(n, s), rank(n + 1, s), tmp(scan_tmp_elems(n) + 1, s), err(1, s);
        QT_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
        k_mirror_flags<<<grid_for(n), 256, 0, s>>>(A->bkey.p, n, up.p, err.p);
        QT_LAUNCH("k_mirror_flags");
        exclusive_scan(up.p, rank.p, n, tmp.p, s);
        int32_t h[2] = {0, 0};
        QT_HIP(hipMemcpyAsync(&h[0], rank.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QT_HIP(hipMemcpyAsync(&h[1], err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QT_HIP(hipStreamSynchronize(s));
        if (h[1]) fail(QT_ERR_ARG, "upper-triangular storage holds a block below the diagonal");
        const int64_t total = n + h[0];
        if (total > (int64_t(1) << 31) - 2) fail(QT_ERR_UNSUPPORTED, "too many blocks");
        DBuf<int32_t> I(total, s), J(total, s), src(total, s);
        k_mirror_list<<<grid_for(n), 256, 0, s>>>(A->bkey.p, n, up.p, rank.p, I.p, J.p, src.p);
        QT_LAUNCH("k_mirror_list");
        S->nblocks = total;
        DBuf<int32_t> perm;
        build_structure(S.get(), I.p, J.p, total, A->n_rows / A->b, A->n_cols / A->b, perm, s);
        S->bmap.alloc(total, s);
        k_gather_i32<<<grid_for(total), 256, 0, s>>>(src.p, perm.p, total, S->bmap.p);
        QT_LAUNCH("k_gather_i32");
    }
    build_histograms(S.get(), s);
    QT_HIP(hipStreamSynchronize(s));
    A->sym_full = std::move(S);
    return A->sym_full.get();
}

// ------------------------------------------------------------- C = A + B

// A matrix shaped like `like` from nb blocks whose keys are already in
// ascending Morton order (adopts keys and values).
static qt_matrix* assemble_sorted(const qt_matrix* like, int L, int64_t nb, DBuf<uint64_t>&& keys,
                                  DBuf<double>&& values, hipStream_t s) {
    std::unique_ptr<qt_matrix> C(new qt_matrix);
    C->n_rows = like->n_rows;
    C->n_cols = like->n_cols;
    C->b = like->b;
    C->leaf = like->leaf;
    C->lb = like->lb;
    C->lb_log = like->lb_log;
    C->L = L;
    C->vtype = QT_F64;
    C->nblocks = nb;
    C->stream = s;
    QT_HIP(hipGetDevice(&C->device));
    C->levels.resize(L);
    C->bkey = std::move(keys);
    C->v64 = std::move(values);
    if (nb > 0) build_tree_levels(C.get(), s);
    build_histograms(C.get(), s);
    QT_HIP(hipStreamSynchronize(s));
    return C.release();
}

// Merge of two ascending key lists without a sort: A's key i lands at
// i + #{B keys < it}, B's key j at j + #{A keys <= it}, so a key present in
// both comes out as A's entry followed by B's. src: s < na for A block s,
// na + j for B block j.
__device__ __forceinline__ int64_t count_below(const uint64_t* __restrict__ k, int64_t n, uint64_t x, bool le) {
    int64_t lo = 0, hi = n;   // first position whose key is >= x (le: > x)
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const bool left = le ? (k[mid] <= x) : (k[mid] < x);
        if (left)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_merge_keys(const uint64_t* __restrict__ ka, int64_t na, const uint64_t* __restrict__ kb,
                             int64_t nb, uint64_t* __restrict__ keys, int32_t* __restrict__ src) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < na) {
        const int64_t pos = t + count_below(kb, nb, ka[t], false);
        keys[pos] = ka[t];
        src[pos] = (int32_t)t;
    } else if (t < na + nb) {
        const int64_t j = t - na;
        const int64_t pos = j + count_below(ka, na, kb[j], true);
        keys[pos] = kb[j];
        src[pos] = (int32_t)t;
    }
}

__global__ void k_key_flags(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) flags[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

// Sorted keys of A's and B's blocks (source s < na: A block s, else B block
// s - na): the first entry of every key writes the output block, adding the
// second entry when both matrices hold the block.
__global__ void k_add_blocks(const uint64_t* __restrict__ keys, const int32_t* __restrict__ src, int64_t n,
                             const int32_t* __restrict__ flags, const int32_t* __restrict__ ex, int64_t na,
                             const double* __restrict__ va, const double* __restrict__ vb, int bb,
                             uint64_t* __restrict__ ckey, double* __restrict__ vc) {
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        if (!flags[t]) continue;
        const int64_t o = ex[t];
        const int32_t s0 = src[t];
        const double* x = (s0 < na) ? va + (size_t)s0 * bb : vb + (size_t)(s0 - na) * bb;
        const bool two = (t + 1 < n) && keys[t + 1] == keys[t];
        const double* y = nullptr;
        if (two) {
            const int32_t s1 = src[t + 1];
            y = (s1 < na) ? va + (size_t)s1 * bb : vb + (size_t)(s1 - na) * bb;
        }
        if (threadIdx.x == 0) ckey[o] = keys[t];
        for (int e = threadIdx.x; e < bb; e += blockDim.x) vc[(size_t)o * bb + e] = two ? x[e] + y[e] : x[e];
    }
}

qt_matrix* add(qt_matrix* A, qt_matrix* B, hipStream_t s) {
    if (A->b != B->b || A->leaf != B->leaf) fail(QT_ERR_SHAPE, "operands differ in block or leaf size");
    if (A->n_rows != B->n_rows || A->n_cols != B->n_cols) fail(QT_ERR_SHAPE, "operands differ in dimensions");
    const double* va = operand_f64(A, s);
    const double* vb = operand_f64(B, s);
    const int64_t na = A->nblocks, nb = B->nblocks, n = na + nb;
    if (n > (int64_t(1) << 31) - 2) fail(QT_ERR_UNSUPPORTED, "too many blocks");
    if (n == 0) return build(A->n_rows, A->n_cols, A->b, A->leaf, 0, nullptr, nullptr, nullptr, QT_MEM_DEVICE, s);
    const int bb = A->b * A->b;
    // both key lists are ascending (Morton order): merge them
    DBuf<uint64_t> keys(n, s);
    DBuf<int32_t> src(n, s);
    k_merge_keys<<<grid_for(n), 256, 0, s>>>(A->bkey.p, na, B->bkey.p, nb, keys.p, src.p);
    QT_LAUNCH("k_merge_keys");
    DBuf<int32_t> flags(n, s), ex(n + 1, s), tmp(scan_tmp_elems(n) + 1, s);
    k_key_flags<<<grid_for(n), 256, 0, s>>>(keys.p, n, flags.p);
    QT_LAUNCH("k_key_flags");
    exclusive_scan(flags.p, ex.p, n, tmp.p, s);
    const int32_t nc = read_scalar(ex.p + n, s);

    DBuf<uint64_t> ck(nc, s);
    DBuf<double> cv((size_t)nc * bb, s);
    k_add_blocks<<<block_grid(n), 256, 0, s>>>(keys.p, src.p, n, flags.p, ex.p, na, va, vb, bb, ck.p, cv.p);
    QT_LAUNCH("k_add_blocks");
    return assemble_sorted(A, std::max(A->L, B->L), nc, std::move(ck), std::move(cv), s);
}

// --------------------------------------------------- value truncation

// Squared Frobenius norm of every block, and its bit pattern as a sort key
// (non-negative doubles order like their bit patterns).
__global__ void k_block_norm2(const double* __restrict__ v, int64_t n, int bb, double* __restrict__ norm2,
                              uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
    __shared__ double part[256];
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        double s = 0.0;
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            const double x = v[(size_t)t * bb + e];
            s += x * x;
        }
        part[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            norm2[t] = part[0];
            key[t] = (uint64_t)__double_as_longlong(part[0]);
            idx[t] = (int32_t)t;
        }
        __syncthreads();
    }
}

__global__ void k_gather_f64(const double* __restrict__ src, const int32_t* __restrict__ idx, int64_t n,
                             double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// Sorted position p is removed while the running sum of squared norms up to
// and including p stays below eps^2; the survivors are flagged by block.
__global__ void k_trunc_flags(const double* __restrict__ excl, const double* __restrict__ sorted, int64_t n,
                              double eps2, const int32_t* __restrict__ idx, int32_t* __restrict__ keep) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) keep[idx[p]] = (excl[p] + sorted[p] < eps2) ? 0 : 1;
}

// Kept blocks, in their (Morton) order: keys and values of the result.
__global__ void k_compact_blocks(const uint64_t* __restrict__ bkey, const double* __restrict__ v, int64_t n, int bb,
                                 const int32_t* __restrict__ keep, const int32_t* __restrict__ pos,
                                 uint64_t* __restrict__ okey, double* __restrict__ out) {
    for (int64_t t = blockIdx.x; t < n; t += gridDim.x) {
        if (!keep[t]) continue;
        const int64_t o = pos[t];
        if (threadIdx.x == 0) okey[o] = bkey[t];
        for (int e = threadIdx.x; e < bb; e += blockDim.x) out[(size_t)o * bb + e] = v[(size_t)t * bb + e];
    }
}



qt_matrix* truncate(qt_matrix* M, double eps, hipStream_t s, int64_t* removed, double* removed_norm2) {
    if (!(eps >= 0.0)) fail(QT_ERR_ARG, "eps must be a non-negative number");
    const double* v = operand_f64(M, s);
    const int64_t n = M->nblocks;
    const int bb = M->b * M->b;
    if (removed) *removed = 0;
    if (removed_norm2) *removed_norm2 = 0.0;
    if (n == 0) return build(M->n_rows, M->n_cols, M->b, M->leaf, 0, nullptr, nullptr, nullptr, QT_MEM_DEVICE, s);
    int64_t npow2 = 1;
    while (npow2 < n) npow2 <<= 1;
    DBuf<double> norm2(n, s), sorted(n, s), excl(n + 1, s), dtmp(scan_tmp_elems(n) + 1, s);
    DBuf<uint64_t> key(npow2, s);
    DBuf<int32_t> idx(npow2, s), keep(n, s), pos(n + 1, s), itmp(scan_tmp_elems(n) + 1, s);
    k_block_norm2<<<block_grid(n), 256, 0, s>>>(v, n, bb, norm2.p, key.p, idx.p);
    QT_LAUNCH("k_block_norm2");
    bitonic_sort(key.p, idx.p, n, s);
    k_gather_f64<<<grid_for(n), 256, 0, s>>>(norm2.p, idx.p, n, sorted.p);
    QT_LAUNCH("k_gather_f64");
    exclusive_scan(sorted.p, excl.p, n, dtmp.p, s);
    k_trunc_flags<<<grid_for(n), 256, 0, s>>>(excl.p, sorted.p, n, eps * eps, idx.p, keep.p);
    QT_LAUNCH("k_trunc_flags");
    exclusive_scan(keep.p, pos.p, n, itmp.p, s);
    const int32_t nk = read_scalar(pos.p + n, s);
    DBuf<uint64_t> K(nk, s);
    DBuf<double> V((size_t)nk * bb, s);
    if (nk > 0) {
        k_compact_blocks<<<block_grid(n), 256, 0, s>>>(M->bkey.p, v, n, bb, keep.p, pos.p, K.p, V.p);
        QT_LAUNCH("k_compact_blocks");
    }
    if (removed || removed_norm2) {
        const int64_t k = n - nk;   // the k smallest blocks were removed
        if (removed) *removed = k;
        if (removed_norm2 && k > 0) {
            double e = 0.0, last = 0.0;
            QT_HIP(hipMemcpyAsync(&e, excl.p + (k - 1), sizeof(double), hipMemcpyDeviceToHost, s));
            QT_HIP(hipMemcpyAsync(&last, sorted.p + (k - 1), sizeof(double), hipMemcpyDeviceToHost, s));
            QT_HIP(hipStreamSynchronize(s));
            *removed_norm2 = e + last;
        }
    }
    return assemble_sorted(M, M->L, nk, std::move(K), std::move(V), s);
}

void get_blocks(const qt_matrix* M, int64_t count, const int32_t* I, const int32_t* J, void* values,
                int32_t* found, qt_prec out_type, qt_mem where, hipStream_t s) {
    if (out_type != QT_F64 && out_type != QT_F32) fail(QT_ERR_UNSUPPORTED, "output type must be F64 or F32");
    if (where != QT_MEM_HOST && where != QT_MEM_DEVICE) fail(QT_ERR_ARG, "bad memory kind");
    if (count < 0) fail(QT_ERR_ARG, "negative count");
    if (count == 0) return;
    if (!I || !J || !values || !found) fail(QT_ERR_ARG, "NULL array");
    const int bb = M->b * M->b;
    const size_t esz = out_type == QT_F64 ? sizeof(double) : sizeof(float);
    DBuf<int32_t> dI, dJ, dF;
    DBuf<char> dV;
    const int32_t* pI = I;
    const int32_t* pJ = J;
    int32_t* pF = found;
    void* pV = values;
    if (where == QT_MEM_HOST) {
        dI.alloc(count, s);
        dJ.alloc(count, s);
        dF.alloc(count, s);
        dV.alloc((size_t)count * bb * esz, s);
        QT_HIP(hipMemcpyAsync(dI.p, I, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
        QT_HIP(hipMemcpyAsync(dJ.p, J, count * sizeof(int32_t), hipMemcpyHostToDevice, s));
        pI = dI.p;
        pJ = dJ.p;
        pF = dF.p;
        pV = dV.p;
    }
    const int64_t nbr = M->n_rows / M->b, nbc = M->n_cols / M->b;
    const unsigned g = block_grid(count);
    const bool src64 = M->vtype == QT_F64;
    if (src64 && out_type == QT_F64)
        k_get_blocks<double, double><<<g, 256, 0, s>>>(M->bkey.p, M->nblocks, nbr, nbc, M->v64.p, pI, pJ, count, bb,
                                                      (double*)pV, pF);
    else if (src64)
        k_get_blocks<double, float><<<g, 256, 0, s>>>(M->bkey.p, M->nblocks, nbr, nbc, M->v64.p, pI, pJ, count, bb,
                                                     (float*)pV, pF);
    else if (out_type == QT_F64)
        k_get_blocks<float, double><<<g, 256, 0, s>>>(M->bkey.p, M->nblocks, nbr, nbc, M->v32.p, pI, pJ, count, bb,
                                                     (double*)pV, pF);
    else
        k_get_blocks<float, float><<<g, 256, 0, s>>>(M->bkey.p, M->nblocks, nbr, nbc, M->v32.p, pI, pJ, count, bb,
                                                    (float*)pV, pF);
    QT_LAUNCH("k_get_blocks");
    if (where == QT_MEM_HOST) {
        QT_HIP(hipMemcpyAsync(found, pF, count * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        QT_HIP(hipMemcpyAsync(values, pV, (size_t)count * bb * esz, hipMemcpyDeviceToHost, s));
        QT_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace qt

// Internal declarations of libqt: handle layout, device buffers, error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "qt.h"

namespace qt {

// ---------------------------------------------------------------- errors

struct Error : std::runtime_error {
    qt_status status;
    Error(qt_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(qt_status s, const std::string& m) { throw Error(s, m); }

inline void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(QT_ERR_OOM, std::string(what) + ": out of device memory");
    fail(QT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define QT_HIP(call) ::qt::hip_check((call), #call)
#define QT_LAUNCH(what) ::qt::hip_check(hipGetLastError(), what)

void set_last_error(const std::string& m);

// ------------------------------------------------------- device buffers

// A caller-installed device allocator (qt_set_allocator). Records are never
// freed, so a buffer can always be returned to the allocator that made it.
struct Allocator {
    void* (*alloc)(size_t bytes, void* stream, void* ctx);
    void (*free_)(void* p, void* stream, void* ctx);
    void* ctx;
};
// The allocator new buffers come from (nullptr: HIP's stream-ordered pool).
const Allocator* current_allocator();
void set_allocator(const Allocator* a);   // nullptr: back to HIP's pool

// Stream-ordered device allocation: from the installed allocator, else
// hipMallocAsync from the device's default pool (whose release threshold is
// raised so freed memory is reused). *who receives the allocator used.
// Throws QT_ERR_OOM when the allocation fails.
void* dev_alloc(size_t bytes, hipStream_t s, const Allocator** who);
void dev_free(void* p, hipStream_t s, const Allocator* who);

// Owning device buffer; released stream-ordered on the stream it was made on
// (or on the stream assigned to `s` later), through the allocator that made
// it. A DBuf may also be a non-owning view into memory owned elsewhere (an
// arena).
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    bool own = true;
    const Allocator* al = nullptr;
    DBuf() = default;
    DBuf(size_t count, hipStream_t st) { alloc(count, st); }
    void alloc(size_t count, hipStream_t st) {
        release();
        s = st;
        n = count;
        p = count ? static_cast<T*>(dev_alloc(count * sizeof(T), st, &al)) : nullptr;
    }
    void view(void* ptr, size_t count) {
        release();
        p = static_cast<T*>(ptr);
        n = count;
        own = false;
    }
    void release() {
        if (p && own) dev_free(p, s, al);
        p = nullptr;
        n = 0;
        own = true;
        al = nullptr;
    }
    ~DBuf() { release(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), own(o.own), al(o.al) {
        o.p = nullptr; o.n = 0; o.own = true; o.al = nullptr;
    }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; s = o.s; own = o.own; al = o.al;
            o.p = nullptr; o.n = 0; o.own = true; o.al = nullptr;
        }
        return *this;
    }
};

// ------------------------------------------------------------ the handle

// An entry of a product list is a block index into the operand's values; its
// top bit marks a block read transposed (every block of an operand used as
// X^T, or a mirrored block of a symmetric matrix stored as its upper
// triangle). Block counts stay below 2^31 - 1, so the index fits below it.
constexpr int32_t PROD_INDEX = 0x7fffffff;
constexpr uint32_t PROD_TRANS = 0x80000000u;

// One quadtree level above the leaves: n nodes, child[4*i + q] is the index
// of child q = 2*m + n of node i in the next level, or -1 for NIL.
// key[i] is the node's Morton index at this level (row bits interleaved above
// column bits, so q is the lowest two bits of the child's key).
struct TreeLevel {
    int32_t n = 0;
    DBuf<int32_t> child;
    DBuf<uint64_t> key;
};

// Leaves (the lowest level): n leaves; for leaf i the stored blocks are
// base[i] .. base[i] + popcount(mask_mo[i]) - 1 in Morton order.
//   mask_mo: bit q set iff the block at local Morton index q is present
//   mask_rm: bit (r*lb + c) set iff local block (r, c) is present (row-major)
//   mask_cm: bit (c*lb + r) set iff local block (r, c) is present (column-major)
struct LeafLevel {
    int32_t n = 0;
    DBuf<int32_t> base;
    DBuf<uint64_t> mask_mo, mask_rm, mask_cm;
    DBuf<uint64_t> key;
};

// Host copies of per-level node counts by row and by column, used to count
// multiply pairs exactly before any device work: the pairs at level l of
// A*B are sum_k colcnt_A[l][k] * rowcnt_B[l][k] (every pair of present nodes
// A(i,k), B(k,j) is reached, since all their ancestors are present).
struct Histograms {
    bool ready = false;
    std::vector<std::vector<int32_t>> rowcnt, colcnt;   // levels 0..L (leaf level)
    std::vector<int32_t> blk_row, blk_col;              // block level
};

}  // namespace qt

struct qt_matrix {
    int64_t n_rows = 0, n_cols = 0;
    int32_t b = 0, leaf = 0, lb = 0, lb_log = 0;
    int32_t L = 0;            // leaf level index (root = 0); padded side = leaf * 2^L
    qt_prec vtype = QT_F64;   // stored value type (QT_F64 or QT_F32)
    int64_t nblocks = 0;
    int device = 0;
    hipStream_t stream = nullptr;

    qt::DBuf<uint64_t> bkey;  // Morton key of each block, ascending
    qt::DBuf<double> v64;     // values (fp64), Morton order, when vtype == QT_F64
    qt::DBuf<float> v32;      // values (fp32), when vtype == QT_F32 or prepared

    std::vector<qt::TreeLevel> levels;   // levels 0 .. L-1
    qt::LeafLevel leaves;                // level L
    qt::DBuf<char> arena;                // owns the tree arrays (of a multiply result, and of
                                         // a built matrix unless it is very large); the DBufs
                                         // below then view into it

    // derived operand forms (built on demand, guarded by mu). Each is queued
    // on the stream of the call that first needs it; the matching event is
    // recorded there, and every later user on any stream waits for it (see
    // form_ready) before reading the form.
    std::mutex mu;
    qt::DBuf<uint16_t> bf_hi, bf_lo;     // bf16 split, row-major per block
    qt::DBuf<uint16_t> bf_hi_t, bf_lo_t; // same, each block transposed
    qt::DBuf<double> v64_cache;          // fp64 copy when vtype == QT_F32
    std::unique_ptr<qt_matrix> sym_full; // structure of the full symmetric matrix from this upper triangle
    hipEvent_t ev_v32 = nullptr, ev_v64 = nullptr, ev_bf16 = nullptr, ev_norms = nullptr;
    // squared Frobenius norms (built on demand, like the forms above): of every
    // block (Morton order), and of every node of every level (level L: leaves)
    qt::DBuf<double> norms;
    const double* bn2 = nullptr;
    std::vector<const double*> nn2;
    qt::Histograms hist;                 // built once, under mu (build_histograms)

    // counters of the multiply that produced this matrix
    std::vector<int64_t> pairs;
    int64_t products = 0;
    bool plan_owned = false;  // a batch plan's result: released with the plan

    // A structure-only matrix (the full symmetric form of an upper block
    // triangle) holds no values: its block t is block bmap[t] & PROD_INDEX of
    // vsrc, read transposed when the top bit of bmap[t] is set.
    qt_matrix* vsrc = nullptr;
    qt::DBuf<int32_t> bmap;

    qt_matrix() = default;
    qt_matrix(const qt_matrix&) = delete;
    qt_matrix& operator=(const qt_matrix&) = delete;
    ~qt_matrix() {
        for (hipEvent_t e : {ev_v32, ev_v64, ev_bf16, ev_norms})
            if (e) (void)hipEventDestroy(e);
    }
};

namespace qt {

// scan.hip -----------------------------------------------------------------
// Exclusive prefix sum of n int32 counts into out[0..n], out[n] = total.
// tmp must come from scan_tmp_elems(n).
size_t scan_tmp_elems(int64_t n);
void exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s);
void exclusive_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
void exclusive_scan(const double* in, double* out, int64_t n, double* tmp, hipStream_t s);

// Sub-allocation of one device allocation: offsets are planned on the host
// (256-byte aligned) before the single allocation is made.
struct ArenaPlan {
    size_t bytes = 0;
    size_t take(size_t n) {
        size_t off = bytes;
        bytes += (n + 255) & ~size_t(255);
        return off;
    }
};

// sort.hip -----------------------------------------------------------------
// Sort n (key, value) pairs by key, ascending (keys assumed distinct for a
// unique order; equal keys are kept adjacent). Buffers of length npow2 >= n.
void bitonic_sort(uint64_t* keys, int32_t* vals, int64_t n, hipStream_t s);

// build.hip ----------------------------------------------------------------
void build_histograms(qt_matrix* M, hipStream_t s);   // fills M->hist (synchronizes)
const double* operand_f64(qt_matrix* M, hipStream_t s);
const float* operand_f32(qt_matrix* M, hipStream_t s);
void operand_bf16(qt_matrix* M, hipStream_t s);
// the squared Frobenius norms of M's blocks and nodes (M->bn2, M->nn2), made
// on s the first time and waited for on s afterwards
void build_norms(qt_matrix* M, hipStream_t s);
uint64_t morton2(uint32_t r, uint32_t c);

// numeric.hip --------------------------------------------------------------
struct NumericArgs {
    int b;
    qt_prec prec;
    const void* A;            // fp64 or fp32 blocks of A
    const void* B;
    const uint16_t* Ahi; const uint16_t* Alo;    // bf16 split of A (row-major blocks)
    const uint16_t* Ahi_t; const uint16_t* Alo_t; // bf16 split of A (transposed blocks)
    const uint16_t* Bhi; const uint16_t* Blo;    // bf16 split of B (row-major blocks)
    const uint16_t* Bhi_t; const uint16_t* Blo_t; // bf16 split of B (transposed blocks)
    const int32_t* prodA;     // per product: block index into A (top bit: read transposed, if dyn)
    const int32_t* prodB;     // per product: block index into B
    int dyn;                  // products may read operand blocks transposed (PROD_TRANS)
    const int32_t* seg;       // nseg + 1 offsets into the product lists
    int32_t nseg;
    const int32_t* order;     // launch slot q computes C block order[q] (a permutation
                              // of 0 .. nseg-1); nullptr: block q, i.e. Morton order
    int by_k;                 // order groups C blocks by inner index (their first product's)
    void* C;                  // fp64 or fp32 C blocks, one per segment
};
void launch_numeric(const NumericArgs& a, hipStream_t s);
double probe_mfma(qt_prec prec, hipStream_t s);   // TFLOP/s of a register-only MFMA loop
double probe_batched(qt_prec prec, int b, int64_t count, hipStream_t s);   // TFLOP/s of count block products

// One problem of a batch, as the batch kernels read it (device memory): the
// problem's arrays as byte offsets from the launch's base pointer (a kernel
// argument, so the compiler addresses them as device memory; -1: none).
struct BatchProblem {
    int64_t A, B;             // fp64 / fp32 operands
    int64_t Ahi, Alo;         // split-bf16 operands
    int64_t Bhi_t, Blo_t;
    int64_t prodA, prodB, seg;
    int64_t order;            // launch order of C's blocks (-1: Morton order)
    int64_t C;
};
// schedules of the batch kernel: 0 flat grid, 1 persistent with work-balanced
// contiguous runs, 2 persistent taking 4 items per grab from a counter per
// XCD, 3 persistent taking 16 items per grab from one counter
constexpr int kBatchSchedules = 4;
struct BatchLaunch {
    int b = 0;
    qt_prec prec = QT_F64;
    int schedule = 0;
    bool lds = false;         // b = 64: one four-wave workgroup per C block, operands shared through LDS
    const BatchProblem* probs = nullptr;
    const char* base = nullptr;           // the problems' offsets are from here
    const int64_t* item_base = nullptr;   // nprob + 1 prefix offsets of work items
    int32_t nprob = 0;
    int64_t total_items = 0;
    unsigned long long* counter = nullptr;   // 64 words: the work counters
    const int64_t* cum = nullptr;         // balanced schedules: exclusive scan of the items' work
};
void launch_batch(const BatchLaunch& L, hipStream_t s);
// work of every item of L (block products + 1) into cost[0 .. total_items)
void batch_item_costs(const BatchLaunch& L, int64_t* cost, hipStream_t s);

// profiling ----------------------------------------------------------------
bool profiling_on();
// An event used only to time work on a stream: created without the
// system-scope fence an event record otherwise implies (on this GPU an L2
// write-back and invalidate that delays the next launch by ~15 us).
inline void timing_event(hipEvent_t* e) {
    QT_HIP(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
}

// e0 .. e1: symbolic kernels; e3 .. e2: the numeric launch (recorded after
// the host has read C's size, so host latency falls in neither interval).
struct PhaseEvents { hipEvent_t e0, e1, e2, e3; int64_t products, cblocks; };
void profile_push(const PhaseEvents& ev);

// multiply.hip -------------------------------------------------------------
struct SymbolicOut {
    std::unique_ptr<qt_matrix> C;
    DBuf<char> scratch;       // product lists and other symbolic buffers
    NumericArgs na{};         // ready for launch_numeric (na.nseg C blocks)
    PhaseEvents ev{};
    bool prof = false;
};
// Which product: op(A) op(B), op(X) = X or X^T, optionally only the blocks
// of C on or above the block diagonal.
struct MulOp {
    int ta = 0, tb = 0, upper = 0;
    double tau2 = 0;          // > 0: drop pairs and block products with ||A||^2 ||B||^2 < tau2
};
// launch_order: also build the launch order of C's blocks that suits the
// product, for a numeric kernel launched from out.na (a batch plan does not)
void symbolic(qt_matrix* A, qt_matrix* B, qt_prec prec, hipStream_t s, SymbolicOut& out,
              bool allow_profile = true, const MulOp& op = MulOp{}, bool launch_order = true);
qt_matrix* multiply(qt_matrix* A, qt_matrix* B, qt_prec prec, hipStream_t s, const MulOp& op = MulOp{});
qt_matrix* build(int64_t n_rows, int64_t n_cols, int32_t b, int32_t leaf, int64_t nblocks, const int32_t* I,
                 const int32_t* J, const double* values, qt_mem where, hipStream_t s);
qt_matrix* add(qt_matrix* A, qt_matrix* B, hipStream_t s);
qt_matrix* truncate(qt_matrix* M, double eps, hipStream_t s, int64_t* removed, double* removed_norm2);
// The structure of the full symmetric matrix whose upper block triangle is A
// (cached in A; its values are A's, through its block map).
qt_matrix* symmetric_full(qt_matrix* A, hipStream_t s);

}  // namespace qt

// Exported C entry points: argument checks, exception-to-status mapping,
// per-phase event timing.
#include "qt_internal.h"

#include <cstdio>

namespace qt {

static thread_local std::string t_last_error;

void set_last_error(const std::string& m) { t_last_error = m; }

void to_blocks(const qt_matrix*, int32_t*, int32_t*, void*, qt_prec, qt_mem, hipStream_t);
void to_blocks_noalloc(const qt_matrix*, int32_t*, int32_t*, void*, qt_prec, hipStream_t);
void norms_out(qt_matrix*, double*, double*, qt_mem, hipStream_t);
void get_blocks(const qt_matrix*, int64_t, const int32_t*, const int32_t*, void*, int32_t*, qt_prec, qt_mem,
                hipStream_t);
qt_plan* plan_create(int32_t, const qt_matrix* const*, const qt_matrix* const*, qt_prec, hipStream_t);
void plan_execute(qt_plan*, hipStream_t, int);
int plan_tune(qt_plan*, hipStream_t, int, float*);
void tune_cache_set(const char*);
int32_t tune_leaf_cached(const qt_matrix*, const qt_matrix*, qt_prec, hipStream_t, int, const char*, int*);
int32_t plan_tune_cached(qt_plan*, hipStream_t, int, const char*, int*);
int32_t tune_leaf(const qt_matrix*, const qt_matrix*, qt_prec, hipStream_t, int, int32_t*, float*, int32_t,
                  int32_t*);
int32_t plan_count(const qt_plan*);
qt_matrix* plan_result(const qt_plan*, int32_t);
void plan_info(const qt_plan*, int64_t*, int64_t*, int32_t*);
void plan_destroy(qt_plan*);
void plan_set_schedule(qt_plan*, int32_t);

// ------------------------------------------------------------ profiling

static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<PhaseEvents> g_prof_events;
static double g_prof_sym = 0, g_prof_num = 0;
static int64_t g_prof_calls = 0, g_prof_products = 0, g_prof_cblocks = 0;

bool profiling_on() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}

void profile_push(const PhaseEvents& ev) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_events.push_back(ev);
}

static void profile_drain() {
    for (auto& ev : g_prof_events) {
        QT_HIP(hipEventSynchronize(ev.e2));
        float a = 0, b = 0;
        QT_HIP(hipEventElapsedTime(&a, ev.e0, ev.e1));
        QT_HIP(hipEventElapsedTime(&b, ev.e3, ev.e2));
        g_prof_sym += a;
        g_prof_num += b;
        g_prof_calls += 1;
        g_prof_products += ev.products;
        g_prof_cblocks += ev.cblocks;
        (void)hipEventDestroy(ev.e0);
        (void)hipEventDestroy(ev.e1);
        (void)hipEventDestroy(ev.e2);
        (void)hipEventDestroy(ev.e3);
    }
    g_prof_events.clear();
}

}  // namespace qt

using namespace qt;

#define QT_GUARD_BEGIN \
    try {              \
        set_last_error("");
#define QT_GUARD_END                                         \
    }                                                        \
    catch (const qt::Error& e) {                             \
        set_last_error(e.what());                            \
        return e.status;                                     \
    }                                                        \
    catch (const std::bad_alloc&) {                          \
        set_last_error("host allocation failed");            \
        return QT_ERR_OOM;                                   \
    }                                                        \
    catch (const std::exception& e) {                        \
        set_last_error(e.what());                            \
        return QT_ERR_DEVICE;                                \
    }                                                        \
    catch (...) {                                            \
        set_last_error("unknown error");                     \
        return QT_ERR_DEVICE;                                \
    }

namespace qt {
static std::mutex g_alloc_mu;
static std::vector<std::unique_ptr<Allocator>> g_alloc_records;   // kept until the process ends
}  // namespace qt

extern "C" {

qt_status qt_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*, void*), void* ctx) {
    if ((alloc == nullptr) != (free_ == nullptr)) {
        set_last_error("alloc and free_ must both be set or both be NULL");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    if (!alloc) {
        set_allocator(nullptr);
        return QT_OK;
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc_records.push_back(std::unique_ptr<Allocator>(new Allocator{alloc, free_, ctx}));
    set_allocator(g_alloc_records.back().get());
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_build(int64_t n_rows, int64_t n_cols, int32_t block_size, int32_t leaf_size, int64_t nblocks,
                   const int32_t* I, const int32_t* J, const double* values, qt_mem where, void* stream,
                   qt_matrix** out) {
    if (!out) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *out = nullptr;
    QT_GUARD_BEGIN
    *out = build(n_rows, n_cols, block_size, leaf_size, nblocks, I, J, values, where, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_multiply(const qt_matrix* A, const qt_matrix* B, qt_prec prec, void* stream, qt_matrix** C) {
    if (!C) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *C = nullptr;
    if (!A || !B) {
        set_last_error("NULL operand");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    *C = multiply(const_cast<qt_matrix*>(A), const_cast<qt_matrix*>(B), prec, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_multiply_ex(const qt_matrix* A, const qt_matrix* B, int32_t op_flags, qt_prec prec, void* stream,
                         qt_matrix** C) {
    if (!C) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *C = nullptr;
    if (!A || !B || (op_flags & ~(QT_OP_TRANS_A | QT_OP_TRANS_B | QT_OP_UPPER))) {
        set_last_error("NULL operand or unknown flag");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    MulOp op;
    op.ta = (op_flags & QT_OP_TRANS_A) ? 1 : 0;
    op.tb = (op_flags & QT_OP_TRANS_B) ? 1 : 0;
    op.upper = (op_flags & QT_OP_UPPER) ? 1 : 0;
    *C = multiply(const_cast<qt_matrix*>(A), const_cast<qt_matrix*>(B), prec, (hipStream_t)stream, op);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_multiply_tau(const qt_matrix* A, const qt_matrix* B, double tau, qt_prec prec, void* stream,
                          qt_matrix** C) {
    if (!C) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *C = nullptr;
    if (!A || !B || !(tau >= 0.0) || tau > 1e150) {
        set_last_error("NULL operand, or tau negative, NaN or beyond 1e150");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    MulOp op;
    op.tau2 = tau * tau;
    *C = multiply(const_cast<qt_matrix*>(A), const_cast<qt_matrix*>(B), prec, (hipStream_t)stream, op);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_norms(const qt_matrix* M, double* block_norm2, double* total_norm2, qt_mem where, void* stream) {
    if (!M || (where != QT_MEM_HOST && where != QT_MEM_DEVICE)) {
        set_last_error("NULL matrix or bad memory kind");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    norms_out(const_cast<qt_matrix*>(M), block_norm2, total_norm2, where, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_add(const qt_matrix* A, const qt_matrix* B, void* stream, qt_matrix** C) {
    if (!C) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *C = nullptr;
    if (!A || !B) {
        set_last_error("NULL operand");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    *C = add(const_cast<qt_matrix*>(A), const_cast<qt_matrix*>(B), (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_truncate(const qt_matrix* M, double eps, void* stream, qt_matrix** T, int64_t* removed,
                      double* removed_norm2) {
    if (!T) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *T = nullptr;
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    *T = truncate(const_cast<qt_matrix*>(M), eps, (hipStream_t)stream, removed, removed_norm2);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_sysq(const qt_matrix* A, qt_prec prec, void* stream, qt_matrix** C) {
    if (!C) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *C = nullptr;
    if (!A) {
        set_last_error("NULL operand");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    qt_matrix* S = symmetric_full(const_cast<qt_matrix*>(A), (hipStream_t)stream);
    MulOp op;
    op.upper = 1;
    *C = multiply(S, S, prec, (hipStream_t)stream, op);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_info(const qt_matrix* M, int64_t* n_rows, int64_t* n_cols, int32_t* block_size, int32_t* leaf_size,
                  qt_prec* value_type) {
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    if (n_rows) *n_rows = M->n_rows;
    if (n_cols) *n_cols = M->n_cols;
    if (block_size) *block_size = M->b;
    if (leaf_size) *leaf_size = M->leaf;
    if (value_type) *value_type = M->vtype;
    return QT_OK;
}

qt_status qt_nblocks(const qt_matrix* M, int64_t* nblocks) {
    if (!M || !nblocks) {
        set_last_error("NULL matrix or output");
        return QT_ERR_ARG;
    }
    *nblocks = M->nblocks;
    return QT_OK;
}

qt_status qt_to_blocks(const qt_matrix* M, int32_t* I, int32_t* J, void* values, qt_prec out_type, qt_mem where,
                       void* stream) {
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    to_blocks(M, I, J, values, out_type, where, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_to_blocks_noalloc(const qt_matrix* M, int32_t* I, int32_t* J, void* values, qt_prec out_type,
                               void* stream) {
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    to_blocks_noalloc(M, I, J, values, out_type, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_get_blocks(const qt_matrix* M, int64_t count, const int32_t* I, const int32_t* J, void* values,
                        int32_t* found, qt_prec out_type, qt_mem where, void* stream) {
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    get_blocks(M, count, I, J, values, found, out_type, where, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_stats(const qt_matrix* C, int64_t* pairs, int32_t max_levels, int64_t* products) {
    if (!C || max_levels < 0 || (max_levels > 0 && !pairs)) {
        set_last_error("bad argument");
        return QT_ERR_ARG;
    }
    const int32_t nl = C->L + 1;
    for (int32_t l = 0; l < nl && l < max_levels; ++l) pairs[l] = (l < (int32_t)C->pairs.size()) ? C->pairs[l] : 0;
    if (products) *products = C->products;
    return QT_OK;
}

qt_status qt_levels(const qt_matrix* M, int64_t* nodes, int32_t max_levels, int32_t* n_levels) {
    if (!M || max_levels < 0 || (max_levels > 0 && !nodes)) {
        set_last_error("bad argument");
        return QT_ERR_ARG;
    }
    const int32_t nl = M->L + 1;
    if (n_levels) *n_levels = nl;
    for (int32_t l = 0; l < nl && l < max_levels; ++l) nodes[l] = (l < M->L) ? M->levels[l].n : M->leaves.n;
    return QT_OK;
}

qt_status qt_prepare(const qt_matrix* M, qt_prec prec, void* stream) {
    if (!M) {
        set_last_error("NULL matrix");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    qt_matrix* m = const_cast<qt_matrix*>(M);
    hipStream_t s = (hipStream_t)stream;
    if (prec == QT_F64)
        operand_f64(m, s);
    else if (prec == QT_F32)
        operand_f32(m, s);
    else if (prec == QT_BF16X3)
        operand_bf16(m, s);
    else
        fail(QT_ERR_ARG, "unknown precision");
    build_histograms(m, s);
    return QT_OK;
    QT_GUARD_END
}

void qt_free(qt_matrix* M) {
    if (M && M->plan_owned) return;   // released by qt_plan_destroy
    try {
        delete M;
    } catch (...) {
    }
}

qt_status qt_profile(int enable) {
    QT_GUARD_BEGIN
    std::lock_guard<std::mutex> lk(g_prof_mu);
    profile_drain();
    g_prof_on = enable != 0;
    g_prof_sym = g_prof_num = 0;
    g_prof_calls = g_prof_products = g_prof_cblocks = 0;
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_profile_read(double* symbolic_ms, double* numeric_ms, int64_t* calls, int64_t* products,
                          int64_t* c_blocks) {
    QT_GUARD_BEGIN
    std::lock_guard<std::mutex> lk(g_prof_mu);
    profile_drain();
    if (symbolic_ms) *symbolic_ms = g_prof_sym;
    if (numeric_ms) *numeric_ms = g_prof_num;
    if (calls) *calls = g_prof_calls;
    if (products) *products = g_prof_products;
    if (c_blocks) *c_blocks = g_prof_cblocks;
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_probe_batched(qt_prec prec, int32_t block_size, int64_t count, void* stream, double* tflops) {
    if (!tflops) {
        set_last_error("NULL output");
        return QT_ERR_ARG;
    }
    *tflops = 0;
    QT_GUARD_BEGIN
    *tflops = probe_batched(prec, block_size, count, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_probe_mfma(qt_prec prec, void* stream, double* tflops) {
    if (!tflops) {
        set_last_error("NULL output");
        return QT_ERR_ARG;
    }
    *tflops = 0;
    QT_GUARD_BEGIN
    *tflops = probe_mfma(prec, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_create(int32_t count, const qt_matrix* const* A, const qt_matrix* const* B, qt_prec prec,
                         void* stream, qt_plan** plan) {
    if (!plan) {
        set_last_error("NULL output handle");
        return QT_ERR_ARG;
    }
    *plan = nullptr;
    QT_GUARD_BEGIN
    *plan = plan_create(count, A, B, prec, (hipStream_t)stream);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_execute(qt_plan* plan, void* stream) {
    if (!plan) {
        set_last_error("NULL plan");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    plan_execute(plan, (hipStream_t)stream, 0);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_replay(qt_plan* plan, void* stream) {
    if (!plan) {
        set_last_error("NULL plan");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    plan_execute(plan, (hipStream_t)stream, 1);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_tune(qt_plan* plan, void* stream, int reps, int32_t* schedule, float* ms) {
    if (!plan) {
        set_last_error("NULL plan");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    const int v = plan_tune(plan, (hipStream_t)stream, reps, ms);
    if (schedule) *schedule = v;
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_set_schedule(qt_plan* plan, int32_t schedule) {
    if (!plan || schedule < 0 || schedule >= QT_PLAN_CONFIGS) {
        set_last_error("bad plan or schedule");
        return QT_ERR_ARG;
    }
    plan_set_schedule(plan, schedule);
    return QT_OK;
}

qt_status qt_plan_result(const qt_plan* plan, int32_t i, qt_matrix** C) {
    if (!plan || !C || i < 0 || i >= plan_count(plan)) {
        set_last_error("bad plan, index or output");
        if (C) *C = nullptr;
        return QT_ERR_ARG;
    }
    *C = plan_result(plan, i);
    return QT_OK;
}

qt_status qt_plan_info(const qt_plan* plan, int64_t* work_items, int64_t* products, int32_t* schedule) {
    if (!plan) {
        set_last_error("NULL plan");
        return QT_ERR_ARG;
    }
    plan_info(plan, work_items, products, schedule);
    return QT_OK;
}

void qt_plan_destroy(qt_plan* plan) {
    try {
        plan_destroy(plan);
    } catch (...) {
    }
}

qt_status qt_tune_leaf(const qt_matrix* A, const qt_matrix* B, qt_prec prec, void* stream, int reps,
                       int32_t* best_leaf, int32_t* leaves, float* ms, int32_t max_out, int32_t* n_tried) {
    if (!A || !B || !best_leaf || max_out < 0) {
        set_last_error("bad argument");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    *best_leaf = tune_leaf(A, B, prec, (hipStream_t)stream, reps, leaves, ms, max_out, n_tried);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_tune_cache(const char* path) {
    QT_GUARD_BEGIN
    tune_cache_set(path);
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_tune_leaf_cached(const qt_matrix* A, const qt_matrix* B, qt_prec prec, void* stream, int reps,
                              const char* pattern_class, int32_t* best_leaf, int32_t* cached) {
    if (!A || !B || !best_leaf || !pattern_class) {
        set_last_error("bad argument");
        return QT_ERR_ARG;
    }
    if (prec != QT_F64 && prec != QT_F32 && prec != QT_BF16X3) {
        set_last_error("unknown precision");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    int c = 0;
    *best_leaf = tune_leaf_cached(A, B, prec, (hipStream_t)stream, reps, pattern_class, &c);
    if (cached) *cached = c;
    return QT_OK;
    QT_GUARD_END
}

qt_status qt_plan_tune_cached(qt_plan* plan, void* stream, int reps, const char* batch_class, int32_t* schedule,
                              int32_t* cached) {
    if (!plan || !batch_class) {
        set_last_error("bad argument");
        return QT_ERR_ARG;
    }
    QT_GUARD_BEGIN
    int c = 0;
    const int32_t v = plan_tune_cached(plan, (hipStream_t)stream, reps, batch_class, &c);
    if (schedule) *schedule = v;
    if (cached) *cached = c;
    return QT_OK;
    QT_GUARD_END
}

const char* qt_last_error(void) { return t_last_error.c_str(); }

const char* qt_version(void) { return "qt 0.1 (gfx950)"; }

}  // extern "C"

// Batched multiplies: many independent C_i = A_i * B_i in one launch.
//
// qt_plan_create runs the symbolic phase of every problem (it synchronizes
// and allocates every C_i), then lays the numeric work of all problems out as
// one list of work items: problems ordered by decreasing block products (the
// longest first, so the tail of the launch is made of small ones), the C
// blocks of a problem in Morton order (neighbouring blocks share operand
// blocks in cache). qt_plan_execute runs the numeric phase of the whole batch
// as one kernel launch that allocates nothing and never synchronizes; the
// first graph execution captures it (counter reset kernel + batch kernel)
// into a HIP graph that later executions replay. qt_plan_tune times each
// schedule of the batch kernel on the plan itself and keeps the fastest.
//
// The leaf-size tuner (qt_tune_leaf) rebuilds the operands at every allowed
// leaf size and times the whole multiply, since the leaf size changes only
// the symbolic phase: the products, their order and the result do not depend
// on it.
#include "qt_internal.h"

#include <algorithm>
#include <numeric>

struct qt_plan {
    int32_t count = 0;
    qt_prec prec = QT_F64;
    int b = 0;
    hipStream_t stream = nullptr;
    std::vector<std::unique_ptr<qt_matrix>> results;   // input order
    std::vector<qt::DBuf<char>> scratch;               // product lists per problem
    qt::DBuf<char> dev;                                // problems, item offsets, counter
    qt::BatchLaunch launch;
    int64_t products = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t last_stream = nullptr;

    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
    ~qt_plan() {
        (void)hipStreamSynchronize(last_stream ? last_stream : stream);   // NULL: the default stream
        drop_graph();
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        for (auto& r : results)
            if (r) r->plan_owned = false;
    }
};

namespace qt {

qt_plan* plan_create(int32_t count, const qt_matrix* const* A, const qt_matrix* const* B, qt_prec prec,
                     hipStream_t s) {
    if (count <= 0 || !A || !B) fail(QT_ERR_ARG, "empty batch");
    if (prec != QT_F64 && prec != QT_F32 && prec != QT_BF16X3) fail(QT_ERR_ARG, "unknown precision");
    const int b = A[0] ? A[0]->b : 0;
    for (int32_t i = 0; i < count; ++i) {
        if (!A[i] || !B[i]) fail(QT_ERR_ARG, "NULL operand in batch");
        if (A[i]->b != b || B[i]->b != b) fail(QT_ERR_SHAPE, "a batch needs one block size");
    }
    std::unique_ptr<qt_plan> plan(new qt_plan);
    plan->count = count;
    plan->prec = prec;
    plan->b = b;
    plan->stream = s;
    plan->results.resize(count);
    plan->scratch.resize(count);
    std::vector<NumericArgs> na(count);
    std::vector<int64_t> prods(count, 0);
    for (int32_t i = 0; i < count; ++i) {
        SymbolicOut sym;
        symbolic(const_cast<qt_matrix*>(A[i]), const_cast<qt_matrix*>(B[i]), prec, s, sym, false, MulOp{}, false);
        na[i] = sym.na;
        prods[i] = sym.C->products;
        plan->results[i] = std::move(sym.C);
        plan->results[i]->plan_owned = true;
        plan->scratch[i] = std::move(sym.scratch);
    }
    // problems with work, largest first
    std::vector<int32_t> order;
    for (int32_t i = 0; i < count; ++i)
        if (na[i].nseg > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return prods[x] > prods[y]; });
    const int wpb = (b == 64) ? 4 : 1;
    std::vector<BatchProblem> hp(order.size());
    std::vector<int64_t> base(order.size() + 1, 0);
    for (size_t j = 0; j < order.size(); ++j) {
        const NumericArgs& a = na[order[j]];
        BatchProblem& P = hp[j];
        P.A = a.A;
        P.B = a.B;
        P.Ahi = a.Ahi;
        P.Alo = a.Alo;
        P.Bhi_t = a.Bhi_t;
        P.Blo_t = a.Blo_t;
        P.prodA = a.prodA;
        P.prodB = a.prodB;
        P.seg = a.seg;
        P.C = a.C;
        base[j + 1] = base[j] + (int64_t)a.nseg * wpb;
        plan->products += prods[order[j]];
    }
    ArenaPlan ap;
    const size_t o_probs = ap.take(std::max<size_t>(hp.size(), 1) * sizeof(BatchProblem));
    const size_t o_base = ap.take(base.size() * sizeof(int64_t));
    const size_t o_counter = ap.take(sizeof(unsigned long long));
    plan->dev.alloc(ap.bytes, s);
    char* D = plan->dev.p;
    if (!hp.empty())
        QT_HIP(hipMemcpyAsync(D + o_probs, hp.data(), hp.size() * sizeof(BatchProblem), hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(D + o_base, base.data(), base.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    QT_HIP(hipStreamSynchronize(s));

    BatchLaunch& L = plan->launch;
    L.b = b;
    L.prec = prec;
    L.variant = 0;
    L.probs = (const BatchProblem*)(D + o_probs);
    L.item_base = (const int64_t*)(D + o_base);
    L.nprob = (int32_t)hp.size();
    L.total_items = base.back();
    L.counter = (unsigned long long*)(D + o_counter);
    L.persistent_grid = batch_persistent_grid(b, prec);
    return plan.release();
}

void plan_execute(qt_plan* plan, hipStream_t s, int use_graph) {
    plan->last_stream = s;
    if (plan->launch.total_items <= 0) return;
    if (!use_graph) {
        launch_batch(plan->launch, s);
        return;
    }
    if (!plan->gexec) {
        if (!plan->capture_stream) QT_HIP(hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
        QT_HIP(hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal));
        try {
            launch_batch(plan->launch, plan->capture_stream);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(plan->capture_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        QT_HIP(hipStreamEndCapture(plan->capture_stream, &plan->graph));
        QT_HIP(hipGraphInstantiate(&plan->gexec, plan->graph, nullptr, nullptr, 0));
    }
    QT_HIP(hipGraphLaunch(plan->gexec, s));
}

int plan_tune(qt_plan* plan, hipStream_t s, int reps, float* ms_out) {
    if (reps <= 0) reps = 3;
    hipEvent_t e0, e1;
    timing_event(&e0);
    timing_event(&e1);
    int best = plan->launch.variant;
    float best_ms = -1.f;
    try {
        for (int v = 0; v < kBatchVariants; ++v) {
            plan->launch.variant = v;
            launch_batch(plan->launch, s);   // warm
            QT_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) launch_batch(plan->launch, s);
            QT_HIP(hipEventRecord(e1, s));
            QT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            QT_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (ms_out) ms_out[v] = ms;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->launch.variant = best;
    plan->drop_graph();
    plan->last_stream = s;
    return best;
}

// ------------------------------------------------------------ leaf tuner

void to_blocks(const qt_matrix*, int32_t*, int32_t*, void*, qt_prec, qt_mem, hipStream_t);

static qt_matrix* rebuild(const qt_matrix* M, int32_t leaf, hipStream_t s) {
    const int64_t n = M->nblocks;
    const size_t bb = (size_t)M->b * M->b;
    DBuf<int32_t> I(std::max<int64_t>(n, 1), s), J(std::max<int64_t>(n, 1), s);
    DBuf<double> V(std::max<size_t>(n * bb, 1), s);
    if (n > 0) to_blocks(M, I.p, J.p, V.p, QT_F64, QT_MEM_DEVICE, s);
    return build(M->n_rows, M->n_cols, M->b, leaf, n, I.p, J.p, V.p, QT_MEM_DEVICE, s);
}

int32_t tune_leaf(const qt_matrix* A, const qt_matrix* B, qt_prec prec, hipStream_t s, int reps, int32_t* leaves,
                  float* ms_out, int32_t max_out, int32_t* n_out) {
    if (reps <= 0) reps = 3;
    if (A->b != B->b) fail(QT_ERR_SHAPE, "operands differ in block size");
    hipEvent_t e0, e1;
    timing_event(&e0);
    timing_event(&e1);
    int32_t best = A->leaf;
    float best_ms = -1.f;
    int32_t k = 0;
    try {
        for (int32_t lb = 1; lb <= 8; lb *= 2) {
            const int32_t leaf = lb * A->b;
            std::unique_ptr<qt_matrix> a(rebuild(A, leaf, s));
            std::unique_ptr<qt_matrix> bm;
            qt_matrix* bp = a.get();
            if (B != A) {
                bm.reset(rebuild(B, leaf, s));
                bp = bm.get();
            }
            delete multiply(a.get(), bp, prec, s);   // warm: operand forms, pools
            QT_HIP(hipStreamSynchronize(s));
            QT_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) delete multiply(a.get(), bp, prec, s);
            QT_HIP(hipEventRecord(e1, s));
            QT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            QT_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (k < max_out) {
                if (leaves) leaves[k] = leaf;
                if (ms_out) ms_out[k] = ms;
            }
            ++k;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = leaf;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_out) *n_out = k;
    return best;
}

int32_t plan_count(const qt_plan* p) { return p->count; }

qt_matrix* plan_result(const qt_plan* p, int32_t i) { return p->results[i].get(); }

void plan_info(const qt_plan* p, int64_t* items, int64_t* products, int32_t* schedule) {
    if (items) *items = p->launch.total_items;
    if (products) *products = p->products;
    if (schedule) *schedule = p->launch.variant;
}

void plan_destroy(qt_plan* p) { delete p; }

void plan_set_schedule(qt_plan* p, int32_t v) {
    if (p->launch.variant != v) p->drop_graph();
    p->launch.variant = v;
}

}  // namespace qt

// Batched multiplies: many independent C_i = A_i * B_i in one launch.
//
// qt_plan_create runs the symbolic phase of every problem (it synchronizes
// and allocates every C_i), then lays the numeric work of all problems out as
// one list of work items: problems ordered by decreasing block products (the
// longest first, so the tail of the launch is made of small ones), the C
// blocks of a problem in the launch order a single multiply would use
// (Morton order, whose neighbouring blocks share operand blocks in cache, or
// grouped by inner index where C blocks average under two block products).
// qt_plan_execute runs the numeric phase of the whole batch as one kernel
// launch that allocates nothing and never synchronizes (a caller may capture
// it); the first qt_plan_replay captures it (counter reset kernel + batch
// kernel) into a HIP graph that later replays launch. qt_plan_tune times each configuration
// of the batch kernel (schedule, launch order, b = 64 tile shape) on the plan
// itself and keeps the fastest.
//
// The leaf-size tuner (qt_tune_leaf) rebuilds the operands at every allowed
// leaf size and times the whole multiply, since the leaf size changes only
// the symbolic phase: the products, their order and the result do not depend
// on it.
#include "qt_internal.h"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>

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
    // both layouts of the work list: the problems with their own launch orders
    // or all in Morton order; items as per-wave tiles or as C blocks
    const qt::BatchProblem* probs_own = nullptr;
    const qt::BatchProblem* probs_morton = nullptr;
    const int64_t* base_tiles = nullptr;
    const int64_t* base_blocks = nullptr;
    int64_t items_tiles = 0, items_blocks = 0;
    bool has_order = false;   // some problem has a launch order of its own
    qt::DBuf<char> cum;       // work prefix sums of the balanced schedules
    const int64_t* cum_of[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [Morton][C blocks]
    int32_t config = 0;       // schedule | QT_PLAN_ORDER_MORTON | QT_PLAN_TILE_WAVE
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
    // Configuration c: schedule c & 3; Morton order for every problem when
    // QT_PLAN_ORDER_MORTON is set; at b = 64 one wave per 32 x 32 tile when
    // QT_PLAN_TILE_WAVE is set, else one four-wave workgroup per C block
    // sharing its operands through LDS (the bit is ignored below b = 64).
    void configure(int32_t c) {
        if (c != config) drop_graph();
        config = c;
        launch.schedule = c & 3;
        launch.probs = (c & QT_PLAN_ORDER_MORTON) ? probs_morton : probs_own;
        launch.lds = b == 64 && !(c & QT_PLAN_TILE_WAVE);
        launch.item_base = launch.lds ? base_blocks : base_tiles;
        launch.total_items = launch.lds ? items_blocks : items_tiles;
        launch.cum = cum_of[(c & QT_PLAN_ORDER_MORTON) ? 1 : 0][launch.lds ? 1 : 0];
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
        // with the launch order the single multiply would use (by inner index
        // where C blocks average under two block products)
        symbolic(const_cast<qt_matrix*>(A[i]), const_cast<qt_matrix*>(B[i]), prec, s, sym, false, MulOp{}, true);
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
    const int wpb = (b == 64) ? 4 : 1;   // per-wave tiles of a C block
    const size_t np = order.size();
    std::vector<BatchProblem> hp(2 * std::max<size_t>(np, 1));   // [0, np): own launch orders; [np, 2 np): Morton
    std::vector<int64_t> base_t(np + 1, 0), base_b(np + 1, 0);    // items: per-wave tiles, C blocks
    // the problems' arrays as offsets from the lowest address among them
    const char* lowest = nullptr;
    auto note = [&](const void* p) {
        if (p && (!lowest || (const char*)p < lowest)) lowest = (const char*)p;
    };
    for (size_t j = 0; j < np; ++j) {
        const NumericArgs& a = na[order[j]];
        for (const void* p : {a.A, a.B, (const void*)a.Ahi, (const void*)a.Alo, (const void*)a.Bhi_t,
                              (const void*)a.Blo_t, (const void*)a.prodA, (const void*)a.prodB, (const void*)a.seg,
                              (const void*)a.order, (const void*)a.C})
            note(p);
    }
    auto off = [&](const void* p) -> int64_t { return p ? (int64_t)((const char*)p - lowest) : -1; };
    for (size_t j = 0; j < np; ++j) {
        const NumericArgs& a = na[order[j]];
        BatchProblem& P = hp[j];
        P.A = off(a.A);
        P.B = off(a.B);
        P.Ahi = off(a.Ahi);
        P.Alo = off(a.Alo);
        P.Bhi_t = off(a.Bhi_t);
        P.Blo_t = off(a.Blo_t);
        P.prodA = off(a.prodA);
        P.prodB = off(a.prodB);
        P.seg = off(a.seg);
        P.order = off(a.order);
        P.C = off(a.C);
        hp[np + j] = P;
        hp[np + j].order = -1;
        if (a.order) plan->has_order = true;
        base_t[j + 1] = base_t[j] + (int64_t)a.nseg * wpb;
        base_b[j + 1] = base_b[j] + (int64_t)a.nseg;
        plan->products += prods[order[j]];
    }
    ArenaPlan ap;
    const size_t o_probs = ap.take(hp.size() * sizeof(BatchProblem));
    const size_t o_base_t = ap.take(base_t.size() * sizeof(int64_t));
    const size_t o_base_b = ap.take(base_b.size() * sizeof(int64_t));
    const size_t o_counter = ap.take(64 * sizeof(unsigned long long));
    plan->dev.alloc(ap.bytes, s);
    char* D = plan->dev.p;
    QT_HIP(hipMemcpyAsync(D + o_probs, hp.data(), hp.size() * sizeof(BatchProblem), hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(D + o_base_t, base_t.data(), base_t.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(D + o_base_b, base_b.data(), base_b.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    QT_HIP(hipStreamSynchronize(s));

    plan->probs_own = (const BatchProblem*)(D + o_probs);
    plan->probs_morton = plan->probs_own + np;
    plan->base_tiles = (const int64_t*)(D + o_base_t);
    plan->base_blocks = (const int64_t*)(D + o_base_b);
    plan->items_tiles = base_t.back();
    plan->items_blocks = base_b.back();
    BatchLaunch& L = plan->launch;
    L.b = b;
    L.prec = prec;
    L.nprob = (int32_t)np;
    L.counter = (unsigned long long*)(D + o_counter);
    L.base = lowest;

    // the balanced schedules' work prefix sums, one per layout of the work
    // list (own launch orders or Morton; per-wave tiles or C blocks at b = 64)
    {
        ArenaPlan cp;
        size_t o_cum[2][2];
        const int64_t nmax = std::max(plan->items_tiles, plan->items_blocks);
        for (int o = 0; o < 2; ++o)
            for (int t = 0; t < 2; ++t)
                o_cum[o][t] = cp.take(((t ? plan->items_blocks : plan->items_tiles) + 1) * sizeof(int64_t));
        DBuf<int64_t> cost(std::max<int64_t>(nmax, 1), s), stmp(scan_tmp_elems(nmax) + 1, s);
        plan->cum.alloc(cp.bytes, s);
        for (int o = 0; o < 2; ++o)
            for (int t = 0; t < 2; ++t) {
                plan->configure((o ? QT_PLAN_ORDER_MORTON : 0) | (t ? 0 : QT_PLAN_TILE_WAVE));
                int64_t* cum = (int64_t*)(plan->cum.p + o_cum[o][t]);
                plan->cum_of[o][t] = cum;
                if (L.total_items > 0) {
                    batch_item_costs(L, cost.p, s);
                    exclusive_scan(cost.p, cum, L.total_items, stmp.p, s);
                }
            }
        QT_HIP(hipStreamSynchronize(s));
    }
    plan->config = -1;
    plan->configure(0);
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

// Times every configuration that differs for this plan (the order bit only
// if some problem has a launch order of its own, the tile bit only at
// b = 64), keeps the fastest; ms_out[c] gets each time, -1 for the others.
int plan_tune(qt_plan* plan, hipStream_t s, int reps, float* ms_out) {
    if (reps <= 0) reps = 3;
    hipEvent_t e0, e1;
    timing_event(&e0);
    timing_event(&e1);
    const int32_t start = plan->config;
    int32_t best = start;
    float best_ms = -1.f;
    try {
        for (int32_t c = 0; c < QT_PLAN_CONFIGS; ++c) {
            const bool same = ((c & QT_PLAN_ORDER_MORTON) && !plan->has_order) ||
                              ((c & QT_PLAN_TILE_WAVE) && plan->b != 64);
            if (ms_out) ms_out[c] = -1.f;
            if (same) continue;
            plan->configure(c);
            launch_batch(plan->launch, s);   // warm
            QT_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) launch_batch(plan->launch, s);
            QT_HIP(hipEventRecord(e1, s));
            QT_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            QT_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (ms_out) ms_out[c] = ms;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        plan->configure(start);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->configure(best);
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

// ------------------------------------------------------------ tuning cache
//
// The tuners' choices, kept in a text file so that a later process (or call)
// reuses them instead of timing again: one line per choice, "key<TAB>value",
// the key made of the GPU's architecture, the block size, the precision, the
// tuner ("leaf" or "plan") and a class the caller names (for the leaf tuner a
// pattern class such as the pattern kind, size and fill bucket; for the plan
// tuner the batch it describes). The file is read when it is set and written
// whole (to a temporary file, then renamed over it) after every new entry;
// lines that do not parse are ignored. All of it is under one mutex.

static std::mutex g_tc_mu;
static std::string g_tc_path;
static std::map<std::string, int32_t> g_tc;

void tune_cache_set(const char* path) {
    std::lock_guard<std::mutex> lk(g_tc_mu);
    g_tc.clear();
    g_tc_path = path ? path : "";
    if (g_tc_path.empty()) return;
    FILE* f = std::fopen(g_tc_path.c_str(), "r");
    if (!f) return;   // no file yet: made on the first entry
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char* tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        char* end = nullptr;
        const long v = std::strtol(tab + 1, &end, 10);
        if (end == tab + 1 || v < INT32_MIN || v > INT32_MAX) continue;
        g_tc[line] = (int32_t)v;
    }
    std::fclose(f);
}

static std::string tune_key(const char* tuner, int b, qt_prec prec, const char* cls) {
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QT_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    static const char* pn[] = {"f64", "f32", "bf16x3"};
    std::string c = cls ? cls : "";
    for (char& ch : c)
        if (ch == '\t' || ch == '\n' || ch == '\r') ch = ' ';
    return arch + " b" + std::to_string(b) + " " + pn[prec] + " " + tuner + " " + c;
}

static bool tune_lookup(const std::string& key, int32_t* v) {
    std::lock_guard<std::mutex> lk(g_tc_mu);
    if (g_tc_path.empty()) return false;
    auto it = g_tc.find(key);
    if (it == g_tc.end()) return false;
    *v = it->second;
    return true;
}

static void tune_store(const std::string& key, int32_t v) {
    std::lock_guard<std::mutex> lk(g_tc_mu);
    if (g_tc_path.empty()) return;
    g_tc[key] = v;
    const std::string tmp = g_tc_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) fail(QT_ERR_ARG, "cannot write the tuning cache " + tmp);
    bool ok = true;
    for (const auto& kv : g_tc) ok = ok && std::fprintf(f, "%s\t%d\n", kv.first.c_str(), kv.second) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), g_tc_path.c_str()) != 0) {
        std::remove(tmp.c_str());
        fail(QT_ERR_ARG, "cannot write the tuning cache " + g_tc_path);
    }
}

int32_t tune_leaf_cached(const qt_matrix* A, const qt_matrix* B, qt_prec prec, hipStream_t s, int reps,
                         const char* cls, int* cached) {
    const std::string key = tune_key("leaf", A->b, prec, cls);
    int32_t v = 0;
    if (tune_lookup(key, &v)) {
        *cached = 1;
        return v;
    }
    *cached = 0;
    v = tune_leaf(A, B, prec, s, reps, nullptr, nullptr, 0, nullptr);
    tune_store(key, v);
    return v;
}

int32_t plan_tune_cached(qt_plan* plan, hipStream_t s, int reps, const char* cls, int* cached) {
    const std::string key = tune_key("plan", plan->b, plan->prec, cls);
    int32_t v = 0;
    if (tune_lookup(key, &v) && v >= 0 && v < QT_PLAN_CONFIGS) {
        *cached = 1;
        plan->configure(v);
        return v;
    }
    *cached = 0;
    v = plan_tune(plan, s, reps, nullptr);
    tune_store(key, v);
    return v;
}

int32_t plan_count(const qt_plan* p) { return p->count; }

qt_matrix* plan_result(const qt_plan* p, int32_t i) { return p->results[i].get(); }

void plan_info(const qt_plan* p, int64_t* items, int64_t* products, int32_t* config) {
    if (items) *items = p->launch.total_items;
    if (products) *products = p->products;
    if (config) *config = p->config;
}

void plan_destroy(qt_plan* p) { delete p; }

void plan_set_schedule(qt_plan* p, int32_t c) { p->configure(c); }

}  // namespace qt

// C = A*B: symbolic traversal of both quadtrees, then the numeric kernel.
//
// Algorithm 1 of the paper recurses from the roots: a pair of present nodes
// (A_mk, B_kn) spawns the eight child pairs (A_m'k', B_k'n'), pairs with a
// NIL operand are dropped, and at the leaves the block-sparse leaf multiply
// runs; Algorithm 2 then sums the products landing on the same C node.
//
// On the GPU the recursion runs breadth-first, one level per step, with the
// frontier of pairs grouped by the C node they contribute to and, inside a
// group, in ascending inner index k. One wavefront owns one C node:
//   count: it counts, for each of the four child quadrants (m, n), the child
//          pairs present(A_m0) & present(B_0n) + present(A_m1) & present(B_1n)
//          over its pairs, giving (child pairs, child C nodes) packed in an
//          int64;
//   offsets: an exclusive prefix sum of those packed counts gives every C
//          node the place of its child pairs and child C nodes in the next
//          level (from per-workgroup aggregates, or a scan for large levels);
//   fill:  it writes its child pairs, quadrant by quadrant, pairs in order and
//          k' = 0 before k' = 1 (child k = 2k + k'), so the new frontier is
//          again grouped by C node with k ascending; quadrants without pairs
//          are NIL children and get no node.
// Each level takes two launches (count, fill), plus a scan on large levels.
//
// The leaf step gives a C leaf one wavefront whose lanes are the lb x lb
// blocks of the leaf: lane (i, j) counts popcount(rowmask_A(i) & colmask_B(j))
// over the leaf pairs of the C leaf, then lists its products, pair by pair,
// k ascending. The result is the product list of every C block with C blocks
// in Morton order -- which is also C's block order, so no sort is needed, and
// since the order of products inside a C block does not depend on the leaf
// size, neither does the result.
//
// The number of pairs at every level and the number of block products are
// known on the host before any launch (from per-level row/column counts of
// both operands), so all buffers are sized up front in two allocations (the
// result's tree, and scratch); the single synchronization reads back how many
// C blocks there are before C's values are allocated. A level's per-node
// arrays and its grids are sized by a bound on its C nodes: the smaller of its
// pair count and the number of node positions C's shape has at that level.
// A launch order of C's blocks may also be built: leaf-row strips with the
// traversal, or, once the C block count is known, a grouping by inner index
// (see "launch order" below).
// The whole phase runs on a stream of the library, beside the caller's (see
// side_stream below).
#include "qt_internal.h"
#include "qt_morton.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <string>

namespace qt {

constexpr int kPublishMax = 128;  // counts read back per multiply: 3 * (depth + 1) + 1

// ------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t pack2(int32_t lo, int32_t hi) {
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int32_t lo32(int64_t v) { return (int32_t)(uint32_t)((uint64_t)v & 0xffffffffu); }
__device__ __forceinline__ int32_t hi32(int64_t v) { return (int32_t)((uint64_t)v >> 32); }

__device__ __forceinline__ uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x |= __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ int wave_excl_scan(int x, int lane) {
    int v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v - x;
}

__device__ __forceinline__ int4 load_children(const int32_t* tab, int32_t node) {
    return *reinterpret_cast<const int4*>(tab + 4 * (int64_t)node);
}

// bits k of row r of an lb x lb occupancy mask stored row-major
__device__ __forceinline__ uint32_t mask_row(uint64_t m, int r, int lb) {
    return (uint32_t)((m >> (r * lb)) & ((1ull << lb) - 1));
}

// the OR of all lb rows of such a mask: bit k set iff column k holds a block
// (for a column-major mask: bit k set iff row k does)
__device__ __forceinline__ uint32_t mask_fold(uint64_t m, int lb) {
    for (int sh = lb * lb / 2; sh >= lb; sh >>= 1) m |= m >> sh;
    return (uint32_t)(m & ((1ull << lb) - 1));
}

// ------------------------------------------------- one level of the tree

struct TreeStep {
    // this level
    const int32_t* fa;        // A node of each pair
    const int32_t* fb;        // B node of each pair
    const int32_t* cseg;      // pairs of C node c: cseg[c] .. cseg[c+1]-1
    const uint64_t* ckey;     // Morton key of C node c
    const int32_t* ncount;    // number of C nodes (device)
    const int32_t* Ach;       // child tables of A and B at this level
    const int32_t* Bch;
    int64_t* cnt;             // per C node: (child pairs, child C nodes)
    int4* tot4;               // per C node: child pairs per quadrant
    int64_t* off;             // exclusive scan of cnt; off[ncap] = totals (scan path)
                              // or each node's offset inside its workgroup (aggregate path)
    int64_t* wagg;            // aggregate path: per count workgroup, the sum of its nodes' cnt
    int64_t* gsum;            // aggregate path: per group of 64 count workgroups, their sum (zeroed first)
    int use_agg;              // offsets from workgroup aggregates instead of a scan
    int32_t ncap;             // bound on C nodes at this level
    // next level
    int32_t* nfa;
    int32_t* nfb;
    int32_t* ncseg;
    uint64_t* nckey;
    int32_t* cchild;          // C's child table at this level (4 per node), before NIL normalisation
    int32_t* nparent;         // parent (C node at this level) of every C node of the next level
    int32_t* ncount_next;
    int32_t np_next;          // bound on pairs at the next level (exact unless `upper`)
    int32_t nc_next;          // bound on C nodes at the next level
    int32_t* check;           // device total of child pairs, for the host check
    int ta, tb;               // operand used transposed: child (m, k) of op(A) is child (k, m) of A
    int upper;                // keep only C nodes on or above the block diagonal
    const double* An2;        // squared norms of the operands' next-level nodes (nullptr: no
    const double* Bn2;        // norm threshold): a child pair is dropped when An2 Bn2 < tau2
    double tau2;
    // The next level's counts, made by this level's fill when ncnt is set (a
    // single-wave next level): the fill holds every pair of each child node it
    // creates, so it counts their child pairs too, and the next level needs no
    // count kernel of its own.
    const int32_t* nAch;      // child tables of A and B at the next level
    const int32_t* nBch;
    const double* nAn2;       // norms of the nodes two levels down (norm threshold)
    const double* nBn2;
    int64_t* ncnt;            // the next level's cnt, tot4, off, wagg, gsum
    int4* ntot4;
    int64_t* noff;
    int64_t* nwagg;
    int64_t* ngsum;
};

// Child a of op(A) and child b of op(B) form a pair: both present and, with
// a norm threshold, the product of their norms not below it.
__device__ __forceinline__ bool pair_kept(const TreeStep& st, int32_t a, int32_t b) {
    return a >= 0 && b >= 0 && (!st.An2 || st.An2[a] * st.Bn2[b] >= st.tau2);
}

// Children of an operand node in the orientation of op(X): for a transposed
// operand the off-diagonal children swap (quadrant (m, k) of X^T is (k, m) of X).
__device__ __forceinline__ int4 op_swap(int4 c, int transposed) {
    if (transposed) {
        const int t = c.y;
        c.y = c.z;
        c.z = t;
    }
    return c;
}

__device__ __forceinline__ int4 op_children(const int32_t* tab, int32_t node, int transposed) {
    return op_swap(*reinterpret_cast<const int4*>(tab + 4 * (int64_t)node), transposed);
}

// The child tables of A node a and B node b, both loads issued before either
// is used (left alone, the compiler waits for the first before it issues
// the second).
__device__ __forceinline__ void op_children2(const int32_t* atab, int32_t a, int ta, const int32_t* btab, int32_t b,
                                             int tb, int4& x, int4& y) {
    const int4 ra = *reinterpret_cast<const int4*>(atab + 4 * (int64_t)a);
    const int4 rb = *reinterpret_cast<const int4*>(btab + 4 * (int64_t)b);
    __builtin_amdgcn_sched_barrier(0);
    x = op_swap(ra, ta);
    y = op_swap(rb, tb);
}

// Quadrant mn of C node `key` is dropped when only the upper triangle is
// wanted and the node lies on the diagonal (its lower-left child is strictly
// below it); nodes off the diagonal are entirely above it.
__device__ __forceinline__ bool quadrant_dropped(int upper, uint64_t key, int mn) {
    return upper && mn == 2 && morton_row(key) == morton_col(key);
}

__device__ int64_t tree_count_node(const TreeStep& st, int32_t c, int lane) {
    if (c >= *st.ncount) {
        if (lane == 0) st.cnt[c] = 0;
        return 0;
    }
    const int32_t s0 = st.cseg[c], len = st.cseg[c + 1] - s0;
    int t0 = 0, t1 = 0, t2 = 0, t3 = 0;
    for (int32_t base = 0; base < len; base += 64) {
        if (base + lane < len) {
            const int32_t p = s0 + base + lane;
            int4 a, b;   // A child (m, k) at 2m + k, B child (k, n) at 2k + n
            op_children2(st.Ach, st.fa[p], st.ta, st.Bch, st.fb[p], st.tb, a, b);
            t0 += pair_kept(st, a.x, b.x) + pair_kept(st, a.y, b.z);
            t1 += pair_kept(st, a.x, b.y) + pair_kept(st, a.y, b.w);
            t2 += pair_kept(st, a.z, b.x) + pair_kept(st, a.w, b.z);
            t3 += pair_kept(st, a.z, b.y) + pair_kept(st, a.w, b.w);
        }
    }
    if (quadrant_dropped(st.upper, st.ckey[c], 2)) t2 = 0;
    t0 = wave_sum(t0);
    t1 = wave_sum(t1);
    t2 = wave_sum(t2);
    t3 = wave_sum(t3);
    const int64_t v = pack2(t0 + t1 + t2 + t3, (t0 > 0) + (t1 > 0) + (t2 > 0) + (t3 > 0));
    if (lane == 0) {
        st.cnt[c] = v;
        st.tot4[c] = make_int4(t0, t1, t2, t3);
    }
    return v;
}

// Totals T = (child pairs, child C nodes) of a whole level.
__device__ void tree_level_totals(const TreeStep& st, int64_t T) {
    const int32_t nc_next = hi32(T);
    *st.ncount_next = nc_next;
    if (nc_next <= st.nc_next) st.ncseg[nc_next] = lo32(T);
    *st.check = lo32(T);
}

// Workgroup aggregates of a level are summed in groups of 64 (aggregate path, below).
constexpr int AGG_GROUP_LOG = 6;

// Child pairs of the next level's pairs, per quadrant q, summed over the
// wave (the rule of tree_count_node one level down), into u: each lane
// holds at most two pairs (a0, b0) and (a1, b1) (valid: has0, has1), whose
// child tables x0, y0, x1, y1 were loaded by next_level_tables; the totals
// are wave-uniform, kept in scalar registers (popcounts of ballots).
__device__ __forceinline__ void next_level_tables(const TreeStep& st, bool has0, int32_t a0, int32_t b0, bool has1,
                                                  int32_t a1, int32_t b1, int4& x0, int4& y0, int4& x1,
                                                  int4& y1) {
    // a lane without a pair reads node 0 (every level of a non-empty operand
    // has one) and drops the value, so the loads need no branch
    const int4 rx0 = *reinterpret_cast<const int4*>(st.nAch + 4 * (int64_t)(has0 ? a0 : 0));
    const int4 ry0 = *reinterpret_cast<const int4*>(st.nBch + 4 * (int64_t)(has0 ? b0 : 0));
    const int4 rx1 = *reinterpret_cast<const int4*>(st.nAch + 4 * (int64_t)(has1 ? a1 : 0));
    const int4 ry1 = *reinterpret_cast<const int4*>(st.nBch + 4 * (int64_t)(has1 ? b1 : 0));
    const int4 none = make_int4(-1, -1, -1, -1);
    x0 = has0 ? rx0 : none;
    y0 = has0 ? ry0 : none;
    x1 = has1 ? rx1 : none;
    y1 = has1 ? ry1 : none;
}

__device__ __forceinline__ void next_level_count(const TreeStep& st, int4 x, int4 y, uint32_t (&u)[4]) {
    x = op_swap(x, st.ta);
    y = op_swap(y, st.tb);
    auto kept = [&](int32_t p, int32_t q) {
        return p >= 0 && q >= 0 && (!st.nAn2 || st.nAn2[p] * st.nBn2[q] >= st.tau2);
    };
    u[0] += __popcll(__ballot(kept(x.x, y.x))) + __popcll(__ballot(kept(x.y, y.z)));
    u[1] += __popcll(__ballot(kept(x.x, y.y))) + __popcll(__ballot(kept(x.y, y.w)));
    u[2] += __popcll(__ballot(kept(x.z, y.x))) + __popcll(__ballot(kept(x.w, y.z)));
    u[3] += __popcll(__ballot(kept(x.z, y.y))) + __popcll(__ballot(kept(x.w, y.w)));
}

// The counts of c's children, as the next level's count kernel would write
// them for single-wave workgroups (node c2 is workgroup c2, its offset inside
// the workgroup 0); lane mn writes those of child quadrant mn.
__device__ void next_level_write(const TreeStep& st, int32_t c, int lane, const int (&cid)[4],
                                 const uint32_t (&u)[4][4]) {
    if (lane >= 4) return;
    int c2 = -1;
    int mine[4] = {0, 0, 0, 0};
#pragma unroll
    for (int mn = 0; mn < 4; ++mn)
        if (mn == lane) {
            c2 = cid[mn];
#pragma unroll
            for (int q = 0; q < 4; ++q) mine[q] = (int)u[mn][q];
        }
    if (c2 < 0 || c2 >= st.nc_next) return;
    if (quadrant_dropped(st.upper, st.ckey[c] * 4 + (uint64_t)lane, 2)) mine[2] = 0;
    const int64_t v = pack2(mine[0] + mine[1] + mine[2] + mine[3],
                            (mine[0] > 0) + (mine[1] > 0) + (mine[2] > 0) + (mine[3] > 0));
    st.ncnt[c2] = v;
    st.ntot4[c2] = make_int4(mine[0], mine[1], mine[2], mine[3]);
    st.noff[c2] = 0;
    st.nwagg[c2] = v;
    if (v) atomicAdd((unsigned long long*)(st.ngsum + (c2 >> AGG_GROUP_LOG)), (unsigned long long)v);
}

// o: (first child pair, first child C node) of node c in the next level.
__device__ void tree_fill_node(const TreeStep& st, int32_t c, int lane, int64_t o) {
    if (c >= *st.ncount) return;
    const int4 t4 = st.tot4[c];
    const int t[4] = {t4.x, t4.y, t4.z, t4.w};
    int run[4], cid[4];
    int pr = lo32(o), ci = hi32(o);
#pragma unroll
    for (int mn = 0; mn < 4; ++mn) {
        run[mn] = pr;
        pr += t[mn];
        cid[mn] = t[mn] > 0 ? ci++ : -1;
    }
    if (lane < 4) {
        int my_c = -1, my_run = 0;
#pragma unroll
        for (int mn = 0; mn < 4; ++mn)
            if (mn == lane) {
                my_c = cid[mn];
                my_run = run[mn];
            }
        st.cchild[4 * (int64_t)c + lane] = my_c;
        if (my_c >= 0 && my_c < st.nc_next) {
            st.nckey[my_c] = st.ckey[c] * 4 + (uint64_t)lane;
            st.ncseg[my_c] = my_run;
            st.nparent[my_c] = c;
        }
    }
    const int32_t s0 = st.cseg[c], len = st.cseg[c + 1] - s0;
    const uint64_t below = lanes_below(lane);
    const bool drop_lower = quadrant_dropped(st.upper, st.ckey[c], 2);
    const bool counts = st.ncnt != nullptr;
    uint32_t u[4][4] = {};   // per child quadrant mn of c: that child's child pairs, per quadrant
    for (int32_t base = 0; base < len; base += 64) {
        const bool act = base + lane < len;
        int4 a = make_int4(-1, -1, -1, -1), b = make_int4(-1, -1, -1, -1);
        if (act) {
            const int32_t p = s0 + base + lane;
            op_children2(st.Ach, st.fa[p], st.ta, st.Bch, st.fb[p], st.tb, a, b);
        }
        const int av[4] = {a.x, a.y, a.z, a.w};
        const int bv[4] = {b.x, b.y, b.z, b.w};
        // per child quadrant mn: this lane's pairs (k' = 0 and 1) and where they go
        bool e[4][2];
        int out[4];
#pragma unroll
        for (int mn = 0; mn < 4; ++mn) {
            const int m = mn >> 1, n = mn & 1;
            const bool keep = !(mn == 2 && drop_lower);
            e[mn][0] = keep && pair_kept(st, av[2 * m], bv[n]);           // k' = 0
            e[mn][1] = keep && pair_kept(st, av[2 * m + 1], bv[2 + n]);   // k' = 1
            const uint64_t m0 = __ballot(e[mn][0]), m1 = __ballot(e[mn][1]);
            out[mn] = run[mn] + __popcll(m0 & below) + __popcll(m1 & below);
            run[mn] += __popcll(m0) + __popcll(m1);
        }
        // the next level's counts first, the chunk's pair stores after them: a
        // wait for loads issued after stores would wait for the stores too
        if (counts) {
#pragma unroll
            for (int mn = 0; mn < 4; ++mn) {
                const int m = mn >> 1, n = mn & 1;
                int4 x0, y0, x1, y1;
                next_level_tables(st, e[mn][0], av[2 * m], bv[n], e[mn][1], av[2 * m + 1], bv[2 + n], x0, y0, x1,
                                  y1);
                next_level_count(st, x0, y0, u[mn]);
                next_level_count(st, x1, y1, u[mn]);
            }
        }
#pragma unroll
        for (int mn = 0; mn < 4; ++mn) {
            const int m = mn >> 1, n = mn & 1;
            int w = out[mn];
            if (e[mn][0]) {
                if (w < st.np_next) {
                    st.nfa[w] = av[2 * m];
                    st.nfb[w] = bv[n];
                }
                ++w;
            }
            if (e[mn][1] && w < st.np_next) {
                st.nfa[w] = av[2 * m + 1];
                st.nfb[w] = bv[2 + n];
            }
        }
    }
    if (counts) next_level_write(st, c, lane, cid, u);
}

// The per-level kernels run W waves (one C node each) per workgroup: W = 1
// for levels of up to WIDE_LEVEL nodes, so that while a previous numeric
// kernel still fills the GPU with single-wave workgroups the traversal's
// workgroups find room as soon as any wave ends (a wider workgroup waits for
// several free slots on one CU); W = 4 above that, where the number of
// workgroups itself costs.
constexpr int64_t WIDE_LEVEL = 65536;
static inline int level_waves(int64_t n) { return n <= WIDE_LEVEL ? 1 : 4; }

constexpr int32_t AGG_MAX = 65536;   // workgroups per level on the aggregate path

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// Aggregate path, count side: node offsets inside the workgroup and the
// workgroup's aggregate, from each wave's packed count v.
template <int W>
__device__ __forceinline__ void level_local_offsets(int64_t v, int32_t c, int32_t ncap, int64_t* off,
                                                    int64_t* wagg, int64_t* gsum, int64_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (lane == 0 && c < ncap) {
        int64_t pre = 0;
        for (int w = 0; w < wave; ++w) pre += lds[w];
        off[c] = pre;
    }
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < W; ++w) tot += lds[w];
        wagg[blockIdx.x] = tot;
        if (tot) atomicAdd((unsigned long long*)(gsum + (blockIdx.x >> AGG_GROUP_LOG)), (unsigned long long)tot);
    }
}

// Aggregate path, fill side: the sum of the aggregates of all earlier
// workgroups (every thread gets it).
template <int W>
__device__ __forceinline__ int64_t level_base(const int64_t* wagg, const int64_t* gsum, int64_t* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t b = (int32_t)blockIdx.x, g = b >> AGG_GROUP_LOG, first = g << AGG_GROUP_LOG;
    int64_t part = 0;
    for (int32_t i = threadIdx.x; i < g; i += 64 * W) part += gsum[i];
    for (int32_t i = first + threadIdx.x; i < b; i += 64 * W) part += wagg[i];
    part = wave_sum64(part);
    if (lane == 0) lds[wave] = part;
    __syncthreads();
    int64_t base = 0;
    for (int w = 0; w < W; ++w) base += lds[w];
    return base;
}

// Only the first ncount of the ncap node slots hold C nodes: on the aggregate
// path a workgroup whose slots are all past ncount has a zero aggregate and
// nothing to fill, and only the last workgroup (which writes the level's
// totals) still runs.
template <int W>
__device__ __forceinline__ bool level_wg_empty(const int32_t* ncount) {
    return (int64_t)blockIdx.x * W >= *ncount;
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_tree_count(TreeStep st) {
    __shared__ int64_t lds[W];
    if (st.use_agg && level_wg_empty<W>(st.ncount)) {
        if (threadIdx.x == 0) st.wagg[blockIdx.x] = 0;
        return;
    }
    const int32_t c = (int32_t)(blockIdx.x * W + (threadIdx.x >> 6));
    int64_t v = 0;
    if (c < st.ncap) v = tree_count_node(st, c, threadIdx.x & 63);
    if (st.use_agg) level_local_offsets<W>(v, c, st.ncap, st.off, st.wagg, st.gsum, lds);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_tree_fill(TreeStep st) {
    __shared__ int64_t lds[W];
    const int32_t c = (int32_t)(blockIdx.x * W + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (st.use_agg) {
        if (level_wg_empty<W>(st.ncount) && blockIdx.x != gridDim.x - 1) return;
        const int64_t base = level_base<W>(st.wagg, st.gsum, lds);
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) tree_level_totals(st, base + st.wagg[blockIdx.x]);
        if (c < st.ncap) tree_fill_node(st, c, lane, base + st.off[c]);
    } else {
        if (c == 0 && lane == 0) tree_level_totals(st, st.off[st.ncap]);
        if (c < st.ncap) tree_fill_node(st, c, lane, st.off[c]);
    }
}

// Level-0 frontier: the pair of roots, one C node.
struct RootInit {
    int32_t* fa;
    int32_t* fb;
    int32_t* cseg;
    uint64_t* ckey;
    int32_t* ncount;
    int32_t* clear;           // NIL flags and tile counts, group sums, workgroup aggregates (as words)
    int64_t nclear;
};

// The first kernel of the traversal: every workgroup clears its part of the
// scratch that later kernels accumulate into; the first writes the roots.
__device__ void root_init(const RootInit& r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < r.nclear) r.clear[i] = 0;
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        r.fa[0] = 0;
        r.fb[0] = 0;
        r.cseg[0] = 0;
        r.cseg[1] = 1;
        r.ckey[0] = 0;
        r.ncount[0] = 1;
    }
}

__global__ __launch_bounds__(64) void k_root_init(RootInit r) { root_init(r); }

// ------------------------------------------------------ the leaf step

// NIL normalisation of C (see below): the leaf step flags every C leaf that
// receives a block, and its ancestors, as it fills the leaf.
constexpr int NIL_MAX_LEVELS = 32;

struct NilMark {
    int L;
    int64_t foff[NIL_MAX_LEVELS + 2];              // flags of level l at foff[l] .. foff[l+1]-1
    const int32_t* uparent[NIL_MAX_LEVELS + 1];    // parent of every C node, levels 1 .. L
    int32_t* flags;                                // foff[L+1] entries, cleared before the traversal
    int32_t* tcnt;                                 // flags set per tile of 64, cleared with them
};

// Flags C node p of level l; true when this call set it. Each flag is set
// once (an atomic exchange), and each first setting is counted in its tile.
__device__ __forceinline__ bool nil_flag(const NilMark& m, int l, int32_t p) {
    const int64_t f = m.foff[l] + p;
    if (atomicExch(m.flags + f, 1) != 0) return false;
    atomicAdd(m.tcnt + (f >> 6), 1);
    return true;
}

// C leaf c holds a block: it and its ancestors are kept. A walk stops at the
// first node flagged already: whoever flagged it walks on from there.
__device__ void nil_mark_up(const NilMark& m, int32_t c) {
    if (!nil_flag(m, m.L, c)) return;
    int32_t p = c;
    for (int l = m.L; l > 0; --l) {
        p = m.uparent[l][p];
        if (!nil_flag(m, l - 1, p)) return;
    }
}

struct LeafStep {
    const int32_t* fa;        // A leaf of each leaf pair
    const int32_t* fb;        // B leaf of each leaf pair
    const int32_t* cseg;
    const uint64_t* ckey;
    const int32_t* ncount;
    int32_t ncap;
    int lb_log;
    const uint64_t* Arm;      // A leaves: row-major masks
    const uint64_t* Bcm;      // B leaves: column-major masks
    const uint64_t* Amo;      // Morton-order masks (rank of a block in its leaf)
    const uint64_t* Bmo;
    const int32_t* Abase;
    const int32_t* Bbase;
    int64_t* cnt;             // per C leaf: (products, C blocks)
    int32_t* lane_cnt;        // per C leaf, 64 entries: the block products of each block position
    int64_t* off;             // scan path: exclusive scan of cnt; aggregate path: offset inside the workgroup
    int64_t* wagg;            // aggregate path: per count workgroup, the sum of its leaves' cnt
    int64_t* gsum;            // aggregate path: per group of 64 count workgroups, their sum (zeroed first)
    int use_agg;
    int32_t* prodA;
    int32_t* prodB;
    int32_t P;
    uint64_t* cbkey;          // C block keys, Morton order
    int32_t* cbseg;           // first product of each C block
    int32_t cap;              // bound on C blocks
    int32_t* lbase;           // C leaves: first block, masks
    uint64_t* lmo;
    uint64_t* lrm;
    uint64_t* lcm;
    int32_t* nblocks_out;
    int32_t* check;
    int ta, tb;               // op(A) = A^T / op(B) = B^T (masks already swapped by the host)
    int upper;                // keep only blocks on or above the diagonal
    const int32_t* amap;      // structure-only A: its block t is held by its value source as amap[t]
    const int32_t* bmap;
    const double* Abn2;       // squared block norms (nullptr: no norm threshold): a block product
    const double* Bbn2;       // is dropped when Abn2 Bbn2 < tau2
    double tau2;
    NilMark nil;              // the fill flags the kept C leaves and their ancestors
};

// Lane t's value in every lane, for a t that is the same in every lane: a
// read of one lane into a scalar register, with no LDS round trip (a general
// shuffle goes through the LDS crossbar).
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int t) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, t);
}
__device__ __forceinline__ uint64_t lane_value(uint64_t v, int t) {
    return (uint64_t)lane_value((uint32_t)v, t) | ((uint64_t)lane_value((uint32_t)(v >> 32), t) << 32);
}

// Block q of a C leaf is kept unless only the upper triangle is wanted and
// it lies below the diagonal of a diagonal leaf.
__device__ __forceinline__ bool leaf_block_kept(const LeafStep& st, uint64_t leafkey, int i, int j) {
    return !(st.upper && i > j && morton_row(leafkey) == morton_col(leafkey));
}

// Lane q (a block of the C leaf, local Morton index) counts its products.
// The leaf pairs are taken 64 at a time, one per lane, and only those that
// can add a block product at all are walked: some inner index k with column
// k of the op(A) leaf and row k of the op(B) leaf both occupied. In an
// unstructured product most leaf pairs have none (random65536: four in five).
__device__ int leaf_lane_count_norms(const LeafStep& st, int32_t s0, int32_t len, int lane, int i, int j, int lb,
                                     bool on);

__device__ int leaf_lane_count(const LeafStep& st, int32_t s0, int32_t len, int lane, int i, int j, int lb,
                               bool on) {
    if (st.Abn2) return leaf_lane_count_norms(st, s0, len, lane, i, j, lb, on);
    int cnt = 0;
    for (int32_t base = 0; base < len; base += 64) {
        const int32_t nb = min(64, len - base);
        uint64_t ra = 0, cb = 0;
        if (lane < nb) {
            ra = st.Arm[st.fa[s0 + base + lane]];
            cb = st.Bcm[st.fb[s0 + base + lane]];
        }
        for (uint64_t live = __ballot((mask_fold(ra, lb) & mask_fold(cb, lb)) != 0); live; live &= live - 1) {
            const int t = __ffsll((unsigned long long)live) - 1;
            const uint64_t rat = lane_value(ra, t);
            const uint64_t cbt = lane_value(cb, t);
            if (on) cnt += __popc(mask_row(rat, i, lb) & mask_row(cbt, j, lb));
        }
    }
    return cnt;
}

// Local Morton positions of A(i,k) and B(k,j) in the stored (untransposed) leaves.
__device__ __forceinline__ void leaf_positions(const LeafStep& st, int i, int k, int j, uint32_t& qa, uint32_t& qb) {
    qa = st.ta ? (uint32_t)morton_key((uint32_t)k, (uint32_t)i) : (uint32_t)morton_key((uint32_t)i, (uint32_t)k);
    qb = st.tb ? (uint32_t)morton_key((uint32_t)j, (uint32_t)k) : (uint32_t)morton_key((uint32_t)k, (uint32_t)j);
}

// leaf_lane_count with a norm threshold: every candidate product A(i,k)
// B(k,j) is looked at on its own, kept when its blocks' squared norms
// multiply to at least tau2.
__device__ int leaf_lane_count_norms(const LeafStep& st, int32_t s0, int32_t len, int lane, int i, int j, int lb,
                                     bool on) {
    int cnt = 0;
    for (int32_t base = 0; base < len; base += 64) {
        const int32_t nb = min(64, len - base);
        uint64_t ra = 0, cb = 0, amo = 0, bmo = 0;
        int32_t ab = 0, bb = 0;
        if (lane < nb) {
            const int32_t a = st.fa[s0 + base + lane], b = st.fb[s0 + base + lane];
            ra = st.Arm[a];
            cb = st.Bcm[b];
            amo = st.Amo[a];
            bmo = st.Bmo[b];
            ab = st.Abase[a];
            bb = st.Bbase[b];
        }
        for (uint64_t live = __ballot((mask_fold(ra, lb) & mask_fold(cb, lb)) != 0); live; live &= live - 1) {
            const int t = __ffsll((unsigned long long)live) - 1;
            uint32_t m = on ? (mask_row(lane_value(ra, t), i, lb) & mask_row(lane_value(cb, t), j, lb)) : 0u;
            if (__ballot(m != 0) == 0) continue;
            const uint64_t amot = lane_value(amo, t), bmot = lane_value(bmo, t);
            const int32_t abt = (int32_t)lane_value((uint32_t)ab, t), bbt = (int32_t)lane_value((uint32_t)bb, t);
            while (m) {
                const int k = __ffs(m) - 1;
                m &= m - 1;
                uint32_t qa, qb;
                leaf_positions(st, i, k, j, qa, qb);
                const int32_t ia = abt + __popcll(amot & ((1ull << qa) - 1));
                const int32_t ib = bbt + __popcll(bmot & ((1ull << qb) - 1));
                cnt += st.Abn2[ia] * st.Bbn2[ib] >= st.tau2;
            }
        }
    }
    return cnt;
}

__device__ int64_t leaf_count_node(const LeafStep& st, int32_t c, int lane) {
    if (c >= *st.ncount) {
        if (lane == 0) st.cnt[c] = 0;
        return 0;
    }
    const int lb = 1 << st.lb_log;
    const int i = (int)morton_row((uint64_t)lane), j = (int)morton_col((uint64_t)lane);
    const bool on = lane < lb * lb && leaf_block_kept(st, st.ckey[c], i, j);
    const int32_t s0 = st.cseg[c], len = st.cseg[c + 1] - s0;
    const int cnt = leaf_lane_count(st, s0, len, lane, i, j, lb, on);
    st.lane_cnt[(int64_t)c * 64 + lane] = cnt;   // the fill reads it instead of walking the pairs twice
    const uint64_t em = __ballot(cnt > 0);
    const int tot = wave_sum(cnt);
    const int64_t v = pack2(tot, __popcll(em));
    if (lane == 0) st.cnt[c] = v;
    return v;
}

// Totals T = (block products, C blocks) of the leaf level.
__device__ void leaf_level_totals(const LeafStep& st, int64_t T) {
    const int32_t nb = hi32(T);
    *st.nblocks_out = nb;
    if (nb <= st.cap) st.cbseg[nb] = lo32(T);
    *st.check = lo32(T);
}

// o: (first product, first C block) of leaf c.
__device__ void leaf_fill_node(const LeafStep& st, int32_t c, int lane, int64_t o) {
    if (c >= *st.ncount) return;
    const int lb = 1 << st.lb_log;
    const int i = (int)morton_row((uint64_t)lane), j = (int)morton_col((uint64_t)lane);
    const bool on = lane < lb * lb && leaf_block_kept(st, st.ckey[c], i, j);
    const int32_t s0 = st.cseg[c], len = st.cseg[c + 1] - s0;
    const int cnt = st.lane_cnt[(int64_t)c * 64 + lane];   // from the count kernel
    const bool exists = cnt > 0;
    const uint64_t em = __ballot(exists);
    const int32_t bidx = hi32(o) + __popcll(em & lanes_below(lane));
    int32_t out = lo32(o) + wave_excl_scan(cnt, lane);
    if (exists && bidx < st.cap) {
        st.cbkey[bidx] = (st.ckey[c] << (2 * st.lb_log)) | (uint64_t)lane;
        st.cbseg[bidx] = out;
    }
    const bool plain = !st.amap && !st.bmap && !st.Abn2;
    for (int32_t base = 0; base < len; base += 64) {
        const int32_t nb = min(64, len - base);
        uint64_t ra = 0, cb = 0, amo = 0, bmo = 0;
        int32_t ab = 0, bb = 0;
        if (lane < nb) {
            const int32_t a = st.fa[s0 + base + lane], b = st.fb[s0 + base + lane];
            ra = st.Arm[a];
            cb = st.Bcm[b];
            amo = st.Amo[a];
            bmo = st.Bmo[b];
            ab = st.Abase[a];
            bb = st.Bbase[b];
        }
        for (uint64_t live = __ballot((mask_fold(ra, lb) & mask_fold(cb, lb)) != 0); live; live &= live - 1) {
            const int t = __ffsll((unsigned long long)live) - 1;
            const uint64_t rat = lane_value(ra, t);
            const uint64_t cbt = lane_value(cb, t);
            uint32_t m = on ? (mask_row(rat, i, lb) & mask_row(cbt, j, lb)) : 0u;
            // most leaf pairs of an unstructured product add no block product
            // to any block of this C leaf: skip their block positions
            if (__ballot(m != 0) == 0) continue;
            const uint64_t amot = lane_value(amo, t);
            const uint64_t bmot = lane_value(bmo, t);
            const int32_t abt = (int32_t)lane_value((uint32_t)ab, t);
            const int32_t bbt = (int32_t)lane_value((uint32_t)bb, t);
            if (plain) {
                // stored operands, no norm threshold: no loads in this loop, so
                // no wait on memory (a wait here would also wait for the stores
                // of the products before)
                const uint32_t tra = st.ta ? PROD_TRANS : 0u, trb = st.tb ? PROD_TRANS : 0u;
                while (m) {
                    const int k = __ffs(m) - 1;
                    m &= m - 1;
                    uint32_t qa, qb;   // local Morton positions of A(i,k) / B(k,j) in the stored leaves
                    leaf_positions(st, i, k, j, qa, qb);
                    const int32_t ia = abt + __popcll(amot & ((1ull << qa) - 1));
                    const int32_t ib = bbt + __popcll(bmot & ((1ull << qb) - 1));
                    if (out < st.P) {
                        st.prodA[out] = (int32_t)((uint32_t)ia | tra);
                        st.prodB[out] = (int32_t)((uint32_t)ib | trb);
                    }
                    ++out;
                }
                continue;
            }
            while (m) {
                const int k = __ffs(m) - 1;
                m &= m - 1;
                uint32_t qa, qb;   // local Morton positions of A(i,k) / B(k,j) in the stored leaves
                leaf_positions(st, i, k, j, qa, qb);
                const int32_t ia = abt + __popcll(amot & ((1ull << qa) - 1));
                const int32_t ib = bbt + __popcll(bmot & ((1ull << qb) - 1));
                if (st.Abn2 && st.Abn2[ia] * st.Bbn2[ib] < st.tau2) continue;   // dropped by its norm
                if (out < st.P) {
                    // the block of the value source, with the transposition bit
                    st.prodA[out] = st.amap ? st.amap[ia] : (int32_t)((uint32_t)ia | (st.ta ? PROD_TRANS : 0u));
                    st.prodB[out] = st.bmap ? st.bmap[ib] : (int32_t)((uint32_t)ib | (st.tb ? PROD_TRANS : 0u));
                }
                ++out;
            }
        }
    }
    const uint64_t rm = wave_or(exists ? (1ull << (i * lb + j)) : 0ull);
    const uint64_t cm = wave_or(exists ? (1ull << (j * lb + i)) : 0ull);
    if (lane == 0) {
        st.lbase[c] = hi32(o);
        st.lmo[c] = em;
        st.lrm[c] = rm;
        st.lcm[c] = cm;
        if (em) nil_mark_up(st.nil, c);
    }
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_leaf_count(LeafStep st) {
    __shared__ int64_t lds[W];
    if (st.use_agg && level_wg_empty<W>(st.ncount)) {
        if (threadIdx.x == 0) st.wagg[blockIdx.x] = 0;
        return;
    }
    const int32_t c = (int32_t)(blockIdx.x * W + (threadIdx.x >> 6));
    int64_t v = 0;
    if (c < st.ncap) v = leaf_count_node(st, c, threadIdx.x & 63);
    if (st.use_agg) level_local_offsets<W>(v, c, st.ncap, st.off, st.wagg, st.gsum, lds);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_leaf_fill(LeafStep st) {
    __shared__ int64_t lds[W];
    const int32_t c = (int32_t)(blockIdx.x * W + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (st.use_agg) {
        if (level_wg_empty<W>(st.ncount) && blockIdx.x != gridDim.x - 1) return;
        const int64_t base = level_base<W>(st.wagg, st.gsum, lds);
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) leaf_level_totals(st, base + st.wagg[blockIdx.x]);
        if (c < st.ncap) leaf_fill_node(st, c, lane, base + st.off[c]);
    } else {
        if (c == 0 && lane == 0) leaf_level_totals(st, st.off[st.ncap]);
        if (c < st.ncap) leaf_fill_node(st, c, lane, st.off[c]);
    }
}

// ---------------------------------------------- NIL normalisation of C
//
// The traversal creates a C node for every quadrant that receives a pair, and
// a C leaf for every leaf pair group, before it knows whether any block
// product lands there: a leaf whose pairs all miss (no k with A(i,k) and
// B(k,j) both present) holds no block, and so does a node above only such
// leaves. Zero submatrices are NIL at every level of the quadtree (Sec. 3.1),
// so C's tree keeps exactly the nodes with a stored block below them:
//   mark:    the leaf fill flags every leaf that receives a block, and its
//            ancestors (parents were recorded by the traversal), counting
//            the flags set per tile of 64 (nil_mark_up);
//   offsets: one wave per tile adds up the counts of the tiles before it and
//            ranks its own flags with a ballot: the exclusive scan of the
//            flags of all levels, concatenated, which gives every kept node
//            its index among the kept nodes of its level (one launch, where
//            a general scan takes three);
//   compact: kept nodes are copied into C's tree, child tables remapped
//            (a child that is not kept becomes NIL), and the kept counts of
//            every level are written for the read-back.
// C's blocks, their order and the product lists do not change: an empty leaf
// owns none of them. The traversal runs beside the previous multiply's
// numeric kernel, where each launch waits tens of microseconds for wave
// slots; folding the marks into the leaf fill and the scan into one launch
// leaves two launches of the five a separate pass would take.

struct NilTree {
    int L;
    int64_t foff[NIL_MAX_LEVELS + 2];        // flags of level l at foff[l] .. foff[l+1]-1
    const int32_t* uchild[NIL_MAX_LEVELS];   // levels 0 .. L-1 (4 per node)
    const uint64_t* ukey[NIL_MAX_LEVELS + 1];
    const int32_t* ubase;                    // leaves
    const uint64_t* umo;
    const uint64_t* urm;
    const uint64_t* ucm;
    const int32_t* flags;                    // foff[L+1] entries, set by the leaf fill
    const int32_t* ex;                       // exclusive scan of flags (foff[L+1] + 1 entries)
    int32_t* child[NIL_MAX_LEVELS];          // the kept tree
    uint64_t* key[NIL_MAX_LEVELS + 1];
    int32_t* base;
    uint64_t* mo;
    uint64_t* rm;
    uint64_t* cm;
    int32_t* kept;                           // kept nodes per level, levels 0 .. L
};

// ex[i] = number of flags set before i, for i <= n: one wave per tile of 64
// indices, n / 64 + 1 tiles (the lane of index n writes the total); tcnt
// holds the flags set in each tile.
__global__ __launch_bounds__(64) void k_nil_offsets(const int32_t* __restrict__ flags,
                                                    const int32_t* __restrict__ tcnt, int64_t n,
                                                    int32_t* __restrict__ ex) {
    const int lane = threadIdx.x;
    const int64_t t = blockIdx.x;
    int before = 0;
    for (int64_t u = lane; u < t; u += 64) before += tcnt[u];
    before = wave_sum(before);
    const int64_t i = t * 64 + lane;
    const uint64_t set = __ballot(i < n && flags[i] != 0);
    if (i < n) ex[i] = before + __popcll(set & lanes_below(lane));
    if (i == n) ex[n] = before + __popcll(set);
}

__device__ __forceinline__ int32_t nil_rank(const NilTree& t, int l, int64_t c) {
    return t.ex[t.foff[l] + c] - t.ex[t.foff[l]];
}

__global__ void k_nil_compact(NilTree t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int L = t.L;
    if (i == 0)
        for (int l = 0; l <= L; ++l) t.kept[l] = t.ex[t.foff[l + 1]] - t.ex[t.foff[l]];
    if (i >= t.foff[L + 1] || !t.flags[i]) return;
    int l = 0;
    while (i >= t.foff[l + 1]) ++l;
    const int64_t c = i - t.foff[l];
    const int32_t n = nil_rank(t, l, c);
    t.key[l][n] = t.ukey[l][c];
    if (l < L) {
        const int4 u = *reinterpret_cast<const int4*>(t.uchild[l] + 4 * c);
        const int32_t uc[4] = {u.x, u.y, u.z, u.w};
        int32_t out[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            out[q] = (uc[q] >= 0 && t.flags[t.foff[l + 1] + uc[q]]) ? nil_rank(t, l + 1, uc[q]) : -1;
        *reinterpret_cast<int4*>(t.child[l] + 4 * (int64_t)n) = make_int4(out[0], out[1], out[2], out[3]);
    } else {
        t.base[n] = t.ubase[c];
        t.mo[n] = t.umo[c];
        t.rm[n] = t.urm[c];
        t.cm[n] = t.ucm[c];
    }
}

// ------------------------------------------------ launch order of C's blocks
//
// The numeric kernels give each XCD runs of consecutive launch slots. With
// the blocks taken leaf row by leaf row (leaves left to right, the blocks of
// a leaf in Morton order), a run of about a thousand blocks is a strip a leaf
// high across many leaf columns: the strip's A block rows stay in the XCD's
// L2 while B streams past, instead of the square patch of C that a run in
// Morton order covers. Measured on gfx950 this helps only the split kernel at
// b = 64 when a C block has several block products (decay131072: 2.4%
// faster); where C blocks average about one product a kernel is bound by
// writing C, which Morton order keeps contiguous (random65536 fp64: 10%
// slower in strips), and the other kernels gain nothing or lose (the b = 32
// fp64 kernel gained 2.3% before its loads were issued ahead of the MFMAs,
// and is 1% slower in strips since). So the order is built for the split
// kernel at b = 64 and used when the products are at least twice the C
// blocks. It comes from a table of leaf positions,
// row-major: position p holds the C leaf there (or -1), and a scan over the
// positions' block counts gives each leaf its first slot.
__global__ void k_order_clear(int32_t* __restrict__ table, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) table[i] = -1;
}

__global__ void k_order_place(const uint64_t* __restrict__ lkey, const int32_t* __restrict__ ncount, int32_t ncap,
                              int64_t rows, int64_t cols, int32_t* __restrict__ table) {
    const int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= ncap || c >= *ncount) return;
    const uint64_t k = lkey[c];
    const int64_t r = morton_row(k), q = morton_col(k);
    if (r < rows && q < cols) table[r * cols + q] = c;   // always true for a leaf of C
}

__global__ void k_order_counts(const int32_t* __restrict__ table, int64_t n, const uint64_t* __restrict__ lmo,
                               int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = table[i];
    cnt[i] = c >= 0 ? __popcll(lmo[c]) : 0;
}

__global__ void k_order_fill(const int32_t* __restrict__ table, int64_t n, const int32_t* __restrict__ lbase,
                             const int32_t* __restrict__ cnt, const int32_t* __restrict__ off, int32_t cap,
                             int32_t* __restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t c = table[i];
    if (c < 0) return;
    const int32_t o = off[i], b0 = lbase[c], m = cnt[i];
    for (int32_t j = 0; j < m; ++j)
        if (o + j < cap) order[o + j] = b0 + j;
}

// leaf positions up to which the launch order is built (a 16 MiB table)
constexpr int64_t ORDER_MAX_POSITIONS = int64_t(1) << 22;

// Where C blocks average fewer than two block products (an unstructured
// pattern such as random65536), neighbouring C blocks in Morton order share
// no operand, and nearly every block product fetches its A and B blocks from
// beyond L2. Taking the C blocks grouped by the inner index k of their first
// product instead puts C(i,j) = A(i,k) B(k,j) for all i and j of one k into
// consecutive launch slots: the run an XCD receives reads block column k of
// A and block row k of B, both small enough to stay in its L2, and the
// blocks of each are fetched about once (random65536 fp64: 2.3 GB fetched
// instead of 11.8 GB). A counting sort over k without global atomics: each
// workgroup counts its KORDER_WG C blocks per k in LDS, an exclusive scan of
// the counts taken k-major over (k, workgroup) gives each workgroup its first
// slot for every k, and a second pass places the blocks. Inside one
// workgroup and one k the slots are claimed by LDS atomics, so that order
// varies from call to call; each C block is still computed by one wave with
// its products in ascending k, so no result depends on it.
constexpr int KORDER_THREADS = 64, KORDER_ITEMS = 32;   // single waves (see the scan)
constexpr int64_t KORDER_WG = KORDER_THREADS * KORDER_ITEMS;   // C blocks per workgroup
constexpr int64_t KORDER_MAX_K = 16384;                        // LDS table of 64 KiB
constexpr int64_t KORDER_MAX_CELLS = int64_t(1) << 24;         // (k, workgroup) counts

__device__ __forceinline__ int32_t first_k(const uint64_t* __restrict__ akey, const int32_t* __restrict__ prodA,
                                           const int32_t* __restrict__ seg, int64_t s, bool ta, int32_t kdim) {
    // a product whose A block is read transposed (top bit set) has its inner
    // index in the stored block's row
    const int32_t pa = prodA[seg[s]];
    const uint64_t key = akey[pa & PROD_INDEX];
    const int64_t k = (pa < 0) ? (int64_t)morton_row(key) : (int64_t)morton_col(key);   // column of op(A)
    (void)ta;
    return (int32_t)(k < 0 ? 0 : (k >= kdim ? kdim - 1 : k));
}

// k of the workgroup's C blocks (-1 past the end), loaded before any use
__device__ __forceinline__ void korder_keys(const uint64_t* __restrict__ akey, const int32_t* __restrict__ prodA,
                                            const int32_t* __restrict__ seg, int32_t nseg, bool ta, int32_t kdim,
                                            int32_t (&kk)[KORDER_ITEMS]) {
    const int64_t base = (int64_t)blockIdx.x * KORDER_WG + threadIdx.x;
#pragma unroll
    for (int j = 0; j < KORDER_ITEMS; ++j) {
        const int64_t s = base + j * KORDER_THREADS;
        kk[j] = s < nseg ? first_k(akey, prodA, seg, s, ta, kdim) : -1;
    }
}

// cnt[k * nwg + w]: C blocks of workgroup w whose first product has inner index k
__global__ __launch_bounds__(KORDER_THREADS) void k_korder_counts(const uint64_t* __restrict__ akey,
                                                                  const int32_t* __restrict__ prodA,
                                                                  const int32_t* __restrict__ seg, int32_t nseg,
                                                                  bool ta, int32_t kdim, int32_t nwg,
                                                                  int32_t* __restrict__ cnt) {
    extern __shared__ int32_t ktab[];
    int32_t kk[KORDER_ITEMS];
    korder_keys(akey, prodA, seg, nseg, ta, kdim, kk);
    for (int32_t k = threadIdx.x; k < kdim; k += KORDER_THREADS) ktab[k] = 0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KORDER_ITEMS; ++j)
        if (kk[j] >= 0) atomicAdd(&ktab[kk[j]], 1);
    __syncthreads();
    for (int32_t k = threadIdx.x; k < kdim; k += KORDER_THREADS) cnt[(int64_t)k * nwg + blockIdx.x] = ktab[k];
}

// off: the exclusive scan of cnt; order[slot] = C block
__global__ __launch_bounds__(KORDER_THREADS) void k_korder_place(const uint64_t* __restrict__ akey,
                                                                 const int32_t* __restrict__ prodA,
                                                                 const int32_t* __restrict__ seg, int32_t nseg,
                                                                 bool ta, int32_t kdim, int32_t nwg,
                                                                 const int32_t* __restrict__ off,
                                                                 int32_t* __restrict__ order) {
    extern __shared__ int32_t ktab[];
    int32_t kk[KORDER_ITEMS];
    korder_keys(akey, prodA, seg, nseg, ta, kdim, kk);
    for (int32_t k = threadIdx.x; k < kdim; k += KORDER_THREADS) ktab[k] = off[(int64_t)k * nwg + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * KORDER_WG + threadIdx.x;
#pragma unroll
    for (int j = 0; j < KORDER_ITEMS; ++j)
        if (kk[j] >= 0) {
            const int32_t o = atomicAdd(&ktab[kk[j]], 1);
            if (o >= 0 && o < nseg) order[o] = (int32_t)(base + j * KORDER_THREADS);
        }
}

// ----------------------------------------------------------- host side

// Reading C's counts back. Instead of a device-to-host copy followed by a
// stream synchronization (whose wake-up latency is tens of microseconds), a
// one-wave kernel writes the counts into pinned, host-coherent memory and
// then releases a sequence number there at system scope; the host spins on
// that word. The spin checks the stream every so often, so a failed launch
// ends it with the stream's error instead of a hang.
struct alignas(64) HostSlot {
    int32_t counts[kPublishMax];
    uint32_t flag;
};

__global__ void k_publish(const int32_t* __restrict__ counts, int n, HostSlot* slot, uint32_t seq) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) slot->counts[t] = counts[t];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(&slot->flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Events that order one stream after another (record on one, wait on the
// other), kept for reuse per device: a wait already queued keeps the
// recording it was queued after, so an event can be recorded again as soon as
// the wait is queued.
static std::mutex g_order_ev_mu;
static std::map<int, std::vector<hipEvent_t>> g_order_ev;

static void stream_after(hipStream_t waiter, hipStream_t first) {
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    hipEvent_t e = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_order_ev_mu);
        auto& pool = g_order_ev[dev];
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        }
    }
    if (!e) QT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const hipError_t r1 = hipEventRecord(e, first);
    const hipError_t r2 = r1 == hipSuccess ? hipStreamWaitEvent(waiter, e, 0) : r1;
    {
        std::lock_guard<std::mutex> lk(g_order_ev_mu);
        g_order_ev[dev].push_back(e);
    }
    QT_HIP(r1);
    QT_HIP(r2);
}

static std::mutex g_slot_mu;
static std::vector<std::pair<HostSlot*, HostSlot*>> g_slot_free;   // (host address, device address)
static uint32_t g_slot_seq = 0;

// A pinned slot for one read-back, returned to the free list on scope exit.
struct SlotLease {
    HostSlot* slot = nullptr;
    HostSlot* dslot = nullptr;
    uint32_t seq = 0;
    SlotLease() {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        if (g_slot_free.empty()) {
            constexpr int kChunk = 16;
            HostSlot* chunk = nullptr;
            QT_HIP(hipHostMalloc((void**)&chunk, kChunk * sizeof(HostSlot),
                                 hipHostMallocCoherent | hipHostMallocPortable | hipHostMallocMapped));
            HostSlot* dchunk = nullptr;
            QT_HIP(hipHostGetDevicePointer((void**)&dchunk, chunk, 0));
            for (int i = 0; i < kChunk; ++i) {
                chunk[i].flag = 0;
                g_slot_free.emplace_back(chunk + i, dchunk + i);
            }
        }
        slot = g_slot_free.back().first;
        dslot = g_slot_free.back().second;
        g_slot_free.pop_back();
        if (++g_slot_seq == 0) ++g_slot_seq;   // 0 never marks a publication
        seq = g_slot_seq;
    }
    ~SlotLease() {
        std::lock_guard<std::mutex> lk(g_slot_mu);
        g_slot_free.emplace_back(slot, dslot);
    }
    SlotLease(const SlotLease&) = delete;
    SlotLease& operator=(const SlotLease&) = delete;
};

// Reads n counts from the device after the work queued on s; when `waiter`
// is given, work queued on it afterwards follows that work too (ordered while
// the counts are still on their way).
static void read_back_counts(const int32_t* dcount, int n, hipStream_t s, int32_t* out, hipStream_t waiter) {
    if (n > kPublishMax) fail(QT_ERR_UNSUPPORTED, "tree too deep for the count read-back");
    SlotLease lease;
    __atomic_store_n(&lease.slot->flag, 0u, __ATOMIC_RELAXED);
    k_publish<<<1, 64, 0, s>>>(dcount, n, lease.dslot, lease.seq);
    QT_LAUNCH("k_publish");
    if (waiter) stream_after(waiter, s);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(&lease.slot->flag, __ATOMIC_ACQUIRE) == lease.seq) break;
        if ((it & 4095) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (__atomic_load_n(&lease.slot->flag, __ATOMIC_ACQUIRE) == lease.seq) break;
                fail(QT_ERR_DEVICE, "symbolic phase: counts were not published");
            }
            if (e != hipErrorNotReady) fail(QT_ERR_DEVICE, std::string("symbolic phase: ") + hipGetErrorString(e));
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(600))
                fail(QT_ERR_DEVICE, "symbolic phase: no progress for 600 s");
        }
    }
    std::memcpy(out, (const void*)lease.slot->counts, n * sizeof(int32_t));
}

// Workgroups of the per-level kernels for n C nodes (one wave each).
static inline int64_t level_wgs(int64_t n) {
    const int w = level_waves(n);
    return std::max<int64_t>((n + w - 1) / w, 1);
}

// Launch kernel template K (count or fill) with the level's workgroup width.
#define QT_LEVEL_LAUNCH(K, n, wgs, stream, arg)                                  \
    do {                                                                          \
        if (level_waves(n) == 1)                                                  \
            K<1><<<(unsigned)(wgs), 64, 0, (stream)>>>(arg);                      \
        else                                                                      \
            K<4><<<(unsigned)(wgs), 256, 0, (stream)>>>(arg);                     \
        QT_LAUNCH(#K);                                                            \
    } while (0)

// The symbolic phase reads only the operands' structure (child tables, keys,
// masks), which every handle has complete when the call that made it returns
// (build and multiply both wait for it). So it runs on a library stream of its
// own and overlaps whatever is still queued on the caller's stream -- in a
// loop of multiplies, the previous numeric kernel. The numeric launch on the
// caller's stream then waits for the symbolic phase through an event. The
// stream has the default priority.
static std::mutex g_side_mu;
static std::map<int, hipStream_t> g_side;

static hipStream_t side_stream() {
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto it = g_side.find(dev);
    if (it != g_side.end()) return it->second;
    hipStream_t st = nullptr;
    QT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    g_side[dev] = st;
    return st;
}

// A device-resident child table {0, -1, -1, -1}: the single node of a level
// added above a shallower operand so both trees have the same depth (the
// shallower matrix sits in the top-left quadrant at every added level).
static std::mutex g_lift_mu;
static std::map<int, int32_t*> g_lift;

static const int32_t* lift_table() {
    int dev = 0;
    QT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_lift_mu);
    auto it = g_lift.find(dev);
    if (it != g_lift.end()) return it->second;
    int32_t* p = nullptr;
    QT_HIP(hipMalloc(&p, 4 * sizeof(int32_t)));
    const int32_t h[4] = {0, -1, -1, -1};
    QT_HIP(hipMemcpy(p, h, sizeof(h), hipMemcpyHostToDevice));
    g_lift[dev] = p;
    return p;
}

static const std::vector<int32_t>& unit_hist() {
    static const std::vector<int32_t> one(1, 1);
    return one;
}

static int64_t dot_counts(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
    const size_t n = std::min(a.size(), b.size());
    int64_t s = 0;
    for (size_t k = 0; k < n; ++k) s += (int64_t)a[k] * b[k];
    return s;
}

static const int64_t kMaxI32 = (int64_t(1) << 31) - 2;

static qt_matrix* new_result(const qt_matrix* A, const qt_matrix* B, int L, qt_prec prec, hipStream_t s,
                             const MulOp& op) {
    std::unique_ptr<qt_matrix> C(new qt_matrix);
    C->n_rows = op.ta ? A->n_cols : A->n_rows;
    C->n_cols = op.tb ? B->n_rows : B->n_cols;
    C->b = A->b;
    C->leaf = A->leaf;
    C->lb = A->lb;
    C->lb_log = A->lb_log;
    C->L = L;
    C->vtype = (prec == QT_F32) ? QT_F32 : QT_F64;
    C->nblocks = 0;
    C->stream = s;
    QT_HIP(hipGetDevice(&C->device));
    C->levels.resize(L);
    return C.release();
}

static qt_matrix* empty_result(const qt_matrix* A, const qt_matrix* B, int L, qt_prec prec, hipStream_t s,
                               const MulOp& op) {
    qt_matrix* C = new_result(A, B, L, prec, s, op);
    C->pairs.assign(L + 1, 0);
    C->hist.ready = true;
    C->hist.rowcnt.resize(L + 1);
    C->hist.colcnt.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        C->hist.rowcnt[l].assign(size_t(1) << l, 0);
        C->hist.colcnt[l].assign(size_t(1) << l, 0);
    }
    C->hist.blk_row.assign((size_t)C->lb << L, 0);
    C->hist.blk_col.assign((size_t)C->lb << L, 0);
    return C;
}

// Symbolic phase of C = A*B: C's tree, block keys and (uninitialised) value
// array, plus the product lists the numeric phase reads (kept in
// out.scratch). Synchronizes once. out.na.nseg == 0 means C has no blocks.
void symbolic(qt_matrix* A, qt_matrix* B, qt_prec prec, hipStream_t s, SymbolicOut& out, bool allow_profile,
              const MulOp& op, bool launch_order) {
    if (prec != QT_F64 && prec != QT_F32 && prec != QT_BF16X3) fail(QT_ERR_ARG, "unknown precision");
    if (A->b != B->b || A->leaf != B->leaf) fail(QT_ERR_SHAPE, "operands differ in block or leaf size");
    const int64_t a_cols = op.ta ? A->n_rows : A->n_cols;   // op(A) = A or A^T
    const int64_t b_rows = op.tb ? B->n_cols : B->n_rows;
    if (a_cols != b_rows) fail(QT_ERR_SHAPE, "inner dimensions differ");
    if (op.upper && (op.ta ? A->n_cols : A->n_rows) != (op.tb ? B->n_rows : B->n_cols))
        fail(QT_ERR_SHAPE, "an upper-triangular product must be square");
    if (prec == QT_BF16X3 && A->b == 16) fail(QT_ERR_UNSUPPORTED, "split-bf16 path needs b = 32 or 64");
    const bool prune = op.tau2 > 0;   // a norm threshold
    if (prune && (op.ta || op.tb || op.upper || A->vsrc || B->vsrc))
        fail(QT_ERR_UNSUPPORTED, "a norm threshold needs C = A * B of stored operands");
    // with a norm threshold (or only the upper triangle) the counts known
    // beforehand are bounds, not exact
    const bool bounds = op.upper || prune;
    const int L = std::max(A->L, B->L);
    const int liftA = L - A->L, liftB = L - B->L;
    out.na = NumericArgs{};
    out.prof = false;
    if (A->nblocks == 0 || B->nblocks == 0) {
        out.C.reset(empty_result(A, B, L, prec, s, op));
        return;
    }

    const hipStream_t ss = side_stream();   // the traversal's stream
    build_histograms(A, ss);
    build_histograms(B, ss);
    if (prune) {
        // the norms read the operands' values, ready in order on the caller's
        // stream: made there, and the traversal waits for them
        build_norms(A, s);
        build_norms(B, s);
        stream_after(ss, s);
    }

    // pair counts per level and block products: exact, or upper bounds when
    // only the upper triangle of C is formed. Columns of op(A) are rows of A
    // when A is used transposed, and likewise for B.
    const auto& a_col = op.ta ? A->hist.rowcnt : A->hist.colcnt;
    const auto& b_row = op.tb ? B->hist.colcnt : B->hist.rowcnt;
    std::vector<int64_t> pairs(L + 1);
    for (int l = 0; l <= L; ++l) {
        const auto& ca = (l < liftA) ? unit_hist() : a_col[l - liftA];
        const auto& rb = (l < liftB) ? unit_hist() : b_row[l - liftB];
        pairs[l] = dot_counts(ca, rb);
    }
    const int64_t P = dot_counts(op.ta ? A->hist.blk_row : A->hist.blk_col,
                                 op.tb ? B->hist.blk_col : B->hist.blk_row);
    const int lb_log = A->lb_log;
    const int64_t lb2 = int64_t(1) << (2 * lb_log);
    for (int l = 0; l <= L; ++l)
        if (4 * pairs[l] > kMaxI32) fail(QT_ERR_UNSUPPORTED, "too many node pairs at one level");
    // bound on C nodes per level: every C node has at least one pair, and
    // there are only so many node positions in C's shape at that level (the
    // per-node arrays and the level kernels' grids are sized by this; at the
    // deep levels of an unstructured product it is far below the pair count)
    std::vector<int64_t> ncap(L + 1);
    {
        const int64_t c_rows = op.ta ? A->n_cols : A->n_rows, c_cols = op.tb ? B->n_rows : B->n_cols;
        for (int l = 0; l <= L; ++l) {
            const int64_t side = (int64_t)A->leaf << (L - l);
            const int64_t pos = ((c_rows + side - 1) / side) * ((c_cols + side - 1) / side);
            ncap[l] = std::max<int64_t>(std::min(pairs[l], pos), 1);
        }
    }
    if (P > kMaxI32) fail(QT_ERR_UNSUPPORTED, "too many block products");
    if (P == 0) {
        out.C.reset(empty_result(A, B, L, prec, s, op));
        out.C->pairs = pairs;
        return;
    }

    // operand forms for this precision, from the matrices that hold the values
    // (a structure-only operand reads its value source's blocks). A block read
    // transposed is marked in the product lists and transposed as it is
    // loaded: no transposed copy of any operand is made.
    qt_matrix* Av = A->vsrc ? A->vsrc : A;
    qt_matrix* Bv = B->vsrc ? B->vsrc : B;
    NumericArgs na{};
    na.b = A->b;
    na.prec = prec;
    na.dyn = (op.ta || op.tb || A->vsrc || B->vsrc) ? 1 : 0;
    if (prec == QT_F64) {
        na.A = operand_f64(Av, s);
        na.B = operand_f64(Bv, s);
    } else if (prec == QT_F32) {
        na.A = operand_f32(Av, s);
        na.B = operand_f32(Bv, s);
    } else {
        operand_bf16(Av, s);
        operand_bf16(Bv, s);
        na.Ahi = Av->bf_hi.p;
        na.Alo = Av->bf_lo.p;
        na.Ahi_t = Av->bf_hi_t.p;
        na.Alo_t = Av->bf_lo_t.p;
        na.Bhi = Bv->bf_hi.p;
        na.Blo = Bv->bf_lo.p;
        na.Bhi_t = Bv->bf_hi_t.p;
        na.Blo_t = Bv->bf_lo_t.p;
    }

    // ---- plan the two allocations
    const int64_t cap = std::min<int64_t>(P, lb2 * ncap[L]);   // bound on C blocks
    // leaf grid of C (row-major positions) for the launch order in leaf-row strips
    const int64_t c_rows_all = op.ta ? A->n_cols : A->n_rows, c_cols_all = op.tb ? B->n_rows : B->n_cols;
    const int64_t lrows = (c_rows_all + A->leaf - 1) / A->leaf, lcols = (c_cols_all + A->leaf - 1) / A->leaf;
    const int64_t lpos = lrows * lcols;
    const bool make_order = launch_order && prec == QT_BF16X3 && A->b == 64 && lpos <= ORDER_MAX_POSITIONS;
    // the order by inner index is built once C's block count is known, if
    // the products are then fewer than twice the C blocks (cap bounds those)
    const int64_t kdim = ((op.ta ? A->n_rows : A->n_cols) + A->b - 1) / A->b;
    const int64_t kwg_cap = (cap + KORDER_WG - 1) / KORDER_WG;   // workgroups of the counting sort
    const bool may_korder =
        launch_order && P < 2 * cap && kdim >= 1 && kdim <= KORDER_MAX_K && kdim * kwg_cap <= KORDER_MAX_CELLS;
    ArenaPlan keep, tmp;   // keep: C's tree; tmp: scratch freed after the call
    std::vector<size_t> o_child(L), o_key(L + 1);
    for (int l = 0; l < L; ++l) o_child[l] = keep.take(4 * ncap[l] * sizeof(int32_t));
    for (int l = 0; l <= L; ++l) o_key[l] = keep.take(ncap[l] * sizeof(uint64_t));
    const size_t o_lbase = keep.take(ncap[L] * sizeof(int32_t));
    const size_t o_lmo = keep.take(ncap[L] * sizeof(uint64_t));
    const size_t o_lrm = keep.take(ncap[L] * sizeof(uint64_t));
    const size_t o_lcm = keep.take(ncap[L] * sizeof(uint64_t));
    const size_t o_bkey = keep.take(cap * sizeof(uint64_t));
    // the tree as the traversal forms it, before NIL normalisation (scratch)
    std::vector<size_t> u_child(L), u_key(L + 1), u_parent(L + 1);
    for (int l = 0; l < L; ++l) u_child[l] = tmp.take(4 * ncap[l] * sizeof(int32_t));
    for (int l = 0; l <= L; ++l) u_key[l] = tmp.take(ncap[l] * sizeof(uint64_t));
    for (int l = 1; l <= L; ++l) u_parent[l] = tmp.take(ncap[l] * sizeof(int32_t));
    const size_t u_lbase = tmp.take(ncap[L] * sizeof(int32_t));
    const size_t u_lmo = tmp.take(ncap[L] * sizeof(uint64_t));
    const size_t u_lrm = tmp.take(ncap[L] * sizeof(uint64_t));
    const size_t u_lcm = tmp.take(ncap[L] * sizeof(uint64_t));
    if (L + 1 > NIL_MAX_LEVELS) fail(QT_ERR_UNSUPPORTED, "quadtree too deep");
    std::vector<int64_t> foff(L + 2, 0);
    for (int l = 0; l <= L; ++l) foff[l + 1] = foff[l] + ncap[l];
    if (foff[L + 1] > kMaxI32) fail(QT_ERR_UNSUPPORTED, "too many C nodes");
    // Cleared by the traversal's first kernel, in one run: the NIL flags of all
    // levels and their counts per tile of 64, the group sums of every level's
    // workgroup aggregates, and the aggregates themselves (the levels whose
    // counts the previous level's fill makes have no count kernel to write
    // the aggregates of workgroups without a node).
    const int64_t nil_tiles = foff[L + 1] / 64 + 1;
    const int64_t nil_flags = foff[L + 1] + nil_tiles;
    const size_t o_nflags = tmp.take(nil_flags * sizeof(int32_t));
    std::vector<int64_t> gsum_at(L + 1);
    int64_t gsum_total = 0;
    for (int l = 0; l <= L; ++l) {
        gsum_at[l] = gsum_total;
        gsum_total += (level_wgs(ncap[l]) + (1 << AGG_GROUP_LOG) - 1) >> AGG_GROUP_LOG;
    }
    const size_t o_gsum = tmp.take(std::max<int64_t>(gsum_total, 1) * sizeof(int64_t));
    std::vector<size_t> o_fa(L + 1), o_fb(L + 1), o_cseg(L + 1), o_cnt(L + 1), o_off(L + 1), o_tot(L + 1),
        o_wagg(L + 1);
    for (int l = 0; l <= L; ++l) o_wagg[l] = tmp.take(level_wgs(ncap[l]) * sizeof(int64_t));
    const int64_t nclear = (int64_t)(tmp.bytes - o_nflags) / (int64_t)sizeof(int32_t);
    const size_t o_nex = tmp.take((foff[L + 1] + 1) * sizeof(int32_t));
    size_t scan_elems = 0;
    for (int l = 0; l <= L; ++l) {
        o_fa[l] = tmp.take(pairs[l] * sizeof(int32_t));
        o_fb[l] = tmp.take(pairs[l] * sizeof(int32_t));
        o_cseg[l] = tmp.take((ncap[l] + 1) * sizeof(int32_t));
        o_cnt[l] = tmp.take(ncap[l] * sizeof(int64_t));
        o_off[l] = tmp.take((ncap[l] + 1) * sizeof(int64_t));
        o_tot[l] = tmp.take(ncap[l] * sizeof(int4));
        scan_elems = std::max(scan_elems, scan_tmp_elems(ncap[l]));
    }
    const size_t o_scan = tmp.take((scan_elems + 1) * sizeof(int64_t));
    const size_t o_lcnt = tmp.take(ncap[L] * 64 * sizeof(int32_t));   // leaf step: products per block position
    const size_t o_prodA = tmp.take(P * sizeof(int32_t));
    const size_t o_prodB = tmp.take(P * sizeof(int32_t));
    const size_t o_cbseg = tmp.take((cap + 1) * sizeof(int32_t));
    size_t o_otab = 0, o_ocnt = 0, o_ooff = 0, o_oscan = 0, o_order = 0;
    if (make_order) {
        o_otab = tmp.take(lpos * sizeof(int32_t));
        o_ocnt = tmp.take(lpos * sizeof(int32_t));
        o_ooff = tmp.take((lpos + 1) * sizeof(int32_t));
        o_oscan = tmp.take((scan_tmp_elems(lpos) + 1) * sizeof(int32_t));
    }
    size_t o_kcnt = 0, o_knext = 0, o_kscan = 0;
    if (may_korder) {
        o_kcnt = tmp.take(kdim * kwg_cap * sizeof(int32_t));
        o_knext = tmp.take((kdim * kwg_cap + 1) * sizeof(int32_t));
        o_kscan = tmp.take((scan_tmp_elems(kdim * kwg_cap) + 1) * sizeof(int32_t));
    }
    if (make_order || may_korder) o_order = tmp.take(cap * sizeof(int32_t));   // one order is used at most
    const size_t o_count = tmp.take((3 * L + 4) * sizeof(int32_t));

    out.C.reset(new_result(A, B, L, prec, s, op));
    qt_matrix* C = out.C.get();
    C->pairs = pairs;
    C->products = P;
    // both live on past this call and are released on the caller's stream,
    // after the numeric kernel that reads them
    C->arena.alloc(keep.bytes, ss);
    C->arena.s = s;
    out.scratch.alloc(tmp.bytes, ss);
    out.scratch.s = s;
    char* K = C->arena.p;
    char* W = out.scratch.p;
    auto at = [](char* base, size_t off) { return (void*)(base + off); };
    // [0..L] C nodes per level as traversed, [L+1] C blocks, [L+2..2L+2] checks,
    // [2L+3..3L+3] C nodes per level after NIL normalisation
    int32_t* dcount = (int32_t*)at(W, o_count);
    int32_t* nflags = (int32_t*)at(W, o_nflags);

    const bool prof = out.prof = allow_profile && profiling_on();
    PhaseEvents& ev = out.ev;
    if (prof) {
        timing_event(&ev.e0);
        timing_event(&ev.e1);
        timing_event(&ev.e2);
        timing_event(&ev.e3);
        QT_HIP(hipEventRecord(ev.e0, ss));
    }

    const int32_t* lift = (liftA > 0 || liftB > 0) ? lift_table() : nullptr;
    auto tree_step = [&](int l) {
        TreeStep st{};
        st.fa = (const int32_t*)at(W, o_fa[l]);
        st.fb = (const int32_t*)at(W, o_fb[l]);
        st.cseg = (const int32_t*)at(W, o_cseg[l]);
        st.ckey = (const uint64_t*)at(W, u_key[l]);
        st.ncount = dcount + l;
        st.Ach = (l < liftA) ? lift : A->levels[l - liftA].child.p;
        st.Bch = (l < liftB) ? lift : B->levels[l - liftB].child.p;
        st.cnt = (int64_t*)at(W, o_cnt[l]);
        st.tot4 = (int4*)at(W, o_tot[l]);
        st.wagg = (int64_t*)at(W, o_wagg[l]);
        st.gsum = (int64_t*)at(W, o_gsum) + gsum_at[l];
        st.off = (int64_t*)at(W, o_off[l]);
        st.ncap = (int32_t)ncap[l];
        st.nfa = (int32_t*)at(W, o_fa[l + 1]);
        st.nfb = (int32_t*)at(W, o_fb[l + 1]);
        st.ncseg = (int32_t*)at(W, o_cseg[l + 1]);
        st.nckey = (uint64_t*)at(W, u_key[l + 1]);
        st.cchild = (int32_t*)at(W, u_child[l]);
        st.nparent = (int32_t*)at(W, u_parent[l + 1]);
        st.ncount_next = dcount + l + 1;
        st.np_next = (int32_t)pairs[l + 1];
        st.nc_next = (int32_t)ncap[l + 1];
        st.check = dcount + L + 2 + l;
        st.ta = op.ta;
        st.tb = op.tb;
        st.upper = op.upper;
        if (prune) {
            // norms of the next level's nodes; above a shallower operand's root
            // (the lifted levels) every child is its root
            st.An2 = (l + 1 <= liftA) ? A->nn2[0] : A->nn2[l + 1 - liftA];
            st.Bn2 = (l + 1 <= liftB) ? B->nn2[0] : B->nn2[l + 1 - liftB];
            st.tau2 = op.tau2;
        }
        return st;
    };
    RootInit root{(int32_t*)at(W, o_fa[0]), (int32_t*)at(W, o_fb[0]), (int32_t*)at(W, o_cseg[0]),
                  (uint64_t*)at(W, u_key[0]), dcount, nflags, nclear};

    k_root_init<<<(unsigned)((nclear + 63) / 64), 64, 0, ss>>>(root);
    QT_LAUNCH("k_root_init");
    int64_t* scan_tmp = (int64_t*)at(W, o_scan);
    bool counted = false;   // this level's counts were made by the previous level's fill
    for (int l = 0; l < L; ++l) {
        TreeStep sl = tree_step(l);
        const int64_t wgs = level_wgs(ncap[l]);
        sl.use_agg = wgs <= AGG_MAX;
        if (!counted) {
            QT_LEVEL_LAUNCH(k_tree_count, ncap[l], wgs, ss, sl);
            if (!sl.use_agg) exclusive_scan(sl.cnt, sl.off, ncap[l], scan_tmp, ss);
        }
        // a single-wave next tree level gets its counts from this fill
        counted = l + 1 < L && level_waves(ncap[l + 1]) == 1;
        if (counted) {
            const TreeStep nx = tree_step(l + 1);
            sl.nAch = nx.Ach;
            sl.nBch = nx.Bch;
            sl.nAn2 = nx.An2;
            sl.nBn2 = nx.Bn2;
            sl.ncnt = nx.cnt;
            sl.ntot4 = nx.tot4;
            sl.noff = nx.off;
            sl.nwagg = nx.wagg;
            sl.ngsum = nx.gsum;
        }
        QT_LEVEL_LAUNCH(k_tree_fill, ncap[l], wgs, ss, sl);
    }

    // leaf step
    LeafStep ls{};
    ls.fa = (const int32_t*)at(W, o_fa[L]);
    ls.fb = (const int32_t*)at(W, o_fb[L]);
    ls.cseg = (const int32_t*)at(W, o_cseg[L]);
    ls.ckey = (const uint64_t*)at(W, u_key[L]);
    ls.ncount = dcount + L;
    ls.ncap = (int32_t)ncap[L];
    ls.lb_log = lb_log;
    // rows of op(A) are columns of A when transposed; columns of op(B) rows of B
    ls.Arm = op.ta ? A->leaves.mask_cm.p : A->leaves.mask_rm.p;
    ls.Bcm = op.tb ? B->leaves.mask_rm.p : B->leaves.mask_cm.p;
    ls.ta = op.ta;
    ls.tb = op.tb;
    ls.upper = op.upper;
    ls.amap = A->vsrc ? A->bmap.p : nullptr;
    ls.bmap = B->vsrc ? B->bmap.p : nullptr;
    if (prune) {
        ls.Abn2 = A->bn2;
        ls.Bbn2 = B->bn2;
        ls.tau2 = op.tau2;
    }
    ls.Amo = A->leaves.mask_mo.p;
    ls.Bmo = B->leaves.mask_mo.p;
    ls.Abase = A->leaves.base.p;
    ls.Bbase = B->leaves.base.p;
    ls.cnt = (int64_t*)at(W, o_cnt[L]);
    ls.lane_cnt = (int32_t*)at(W, o_lcnt);
    ls.off = (int64_t*)at(W, o_off[L]);
    ls.wagg = (int64_t*)at(W, o_wagg[L]);
    ls.gsum = (int64_t*)at(W, o_gsum) + gsum_at[L];
    const int64_t leaf_wgs = level_wgs(ncap[L]);
    ls.use_agg = leaf_wgs <= AGG_MAX;
    ls.prodA = (int32_t*)at(W, o_prodA);
    ls.prodB = (int32_t*)at(W, o_prodB);
    ls.P = (int32_t)P;
    ls.cbkey = (uint64_t*)at(K, o_bkey);
    ls.cbseg = (int32_t*)at(W, o_cbseg);
    ls.cap = (int32_t)cap;
    ls.lbase = (int32_t*)at(W, u_lbase);
    ls.lmo = (uint64_t*)at(W, u_lmo);
    ls.lrm = (uint64_t*)at(W, u_lrm);
    ls.lcm = (uint64_t*)at(W, u_lcm);
    ls.nblocks_out = dcount + L + 1;
    ls.check = dcount + 2 * L + 2;
    ls.nil.L = L;
    for (int l = 0; l <= L + 1; ++l) ls.nil.foff[l] = foff[l];
    for (int l = 1; l <= L; ++l) ls.nil.uparent[l] = (const int32_t*)at(W, u_parent[l]);
    ls.nil.flags = nflags;
    ls.nil.tcnt = nflags + foff[L + 1];
    QT_LEVEL_LAUNCH(k_leaf_count, ncap[L], leaf_wgs, ss, ls);
    if (!ls.use_agg) exclusive_scan(ls.cnt, ls.off, ncap[L], scan_tmp, ss);
    QT_LEVEL_LAUNCH(k_leaf_fill, ncap[L], leaf_wgs, ss, ls);
    int32_t* order = (make_order || may_korder) ? (int32_t*)at(W, o_order) : nullptr;
    if (make_order) {
        int32_t* otab = (int32_t*)at(W, o_otab);
        int32_t* ocnt = (int32_t*)at(W, o_ocnt);
        int32_t* ooff = (int32_t*)at(W, o_ooff);
        const unsigned gp = (unsigned)((lpos + 63) / 64);
        k_order_clear<<<gp, 64, 0, ss>>>(otab, lpos);
        QT_LAUNCH("k_order_clear");
        k_order_place<<<(unsigned)((ncap[L] + 63) / 64), 64, 0, ss>>>(ls.ckey, ls.ncount, ls.ncap, lrows, lcols,
                                                                          otab);
        QT_LAUNCH("k_order_place");
        k_order_counts<<<gp, 64, 0, ss>>>(otab, lpos, ls.lmo, ocnt);
        QT_LAUNCH("k_order_counts");
        exclusive_scan(ocnt, ooff, lpos, (int32_t*)at(W, o_oscan), ss);
        k_order_fill<<<gp, 64, 0, ss>>>(otab, lpos, ls.lbase, ocnt, ooff, ls.cap, order);
        QT_LAUNCH("k_order_fill");
    }
    {
        // NIL normalisation: C keeps only the nodes with a block below them
        NilTree nt{};
        nt.L = L;
        for (int l = 0; l <= L + 1; ++l) nt.foff[l] = foff[l];
        for (int l = 0; l < L; ++l) {
            nt.uchild[l] = (const int32_t*)at(W, u_child[l]);
            nt.child[l] = (int32_t*)at(K, o_child[l]);
        }
        for (int l = 0; l <= L; ++l) {
            nt.ukey[l] = (const uint64_t*)at(W, u_key[l]);
            nt.key[l] = (uint64_t*)at(K, o_key[l]);
        }
        nt.ubase = ls.lbase;
        nt.umo = ls.lmo;
        nt.urm = ls.lrm;
        nt.ucm = ls.lcm;
        nt.flags = nflags;
        nt.ex = (const int32_t*)at(W, o_nex);
        nt.base = (int32_t*)at(K, o_lbase);
        nt.mo = (uint64_t*)at(K, o_lmo);
        nt.rm = (uint64_t*)at(K, o_lrm);
        nt.cm = (uint64_t*)at(K, o_lcm);
        nt.kept = dcount + 2 * L + 3;
        k_nil_offsets<<<(unsigned)nil_tiles, 64, 0, ss>>>(nflags, ls.nil.tcnt, foff[L + 1],
                                                            (int32_t*)at(W, o_nex));
        QT_LAUNCH("k_nil_offsets");
        k_nil_compact<<<(unsigned)((foff[L + 1] + 63) / 64), 64, 0, ss>>>(nt);
        QT_LAUNCH("k_nil_compact");
    }
    if (prof) QT_HIP(hipEventRecord(ev.e1, ss));

    // the one synchronization: node and block counts of C
    std::vector<int32_t> hc(3 * L + 4);
    // the caller's stream follows the traversal from here on (the numeric
    // kernel first); a launch order built below adds a second wait
    read_back_counts(dcount, (int)hc.size(), ss, hc.data(), s);
    for (int l = 0; l <= L; ++l) {
        if (hc[l] < 0 || hc[l] > ncap[l]) fail(QT_ERR_DEVICE, "symbolic phase: C node count out of range");
        if (hc[2 * L + 3 + l] < 0 || hc[2 * L + 3 + l] > hc[l])
            fail(QT_ERR_DEVICE, "symbolic phase: kept C node count out of range");
        const int64_t expect = (l < L) ? pairs[l + 1] : P;
        const bool bad = bounds ? (hc[L + 2 + l] < 0 || hc[L + 2 + l] > expect) : (hc[L + 2 + l] != expect);
        if (bad) fail(QT_ERR_DEVICE, "symbolic phase: pair count mismatch");
        if (l < L) C->pairs[l + 1] = hc[L + 2 + l];   // pairs actually formed
    }
    C->products = hc[2 * L + 2];
    const int32_t nnzC = hc[L + 1];
    if (nnzC < 0 || nnzC > cap || (nnzC == 0 && !bounds)) fail(QT_ERR_DEVICE, "symbolic phase: C block count out of range");

    const bool leafrow = make_order && C->products >= 2 * (int64_t)nnzC;
    const bool korder = may_korder && nnzC > 0 && C->products < 2 * (int64_t)nnzC;
    if (korder) {
        int32_t* kcnt = (int32_t*)at(W, o_kcnt);
        int32_t* knext = (int32_t*)at(W, o_knext);
        const uint64_t* akey = Av->bkey.p;   // keys of the blocks the products name
        const int64_t nwg = (nnzC + KORDER_WG - 1) / KORDER_WG;   // <= kwg_cap, as nnzC <= cap
        const size_t lds = (size_t)kdim * sizeof(int32_t);
        k_korder_counts<<<(unsigned)nwg, KORDER_THREADS, lds, ss>>>(akey, ls.prodA, ls.cbseg, nnzC, op.ta,
                                                                     (int32_t)kdim, (int32_t)nwg, kcnt);
        QT_LAUNCH("k_korder_counts");
        exclusive_scan(kcnt, knext, kdim * nwg, (int32_t*)at(W, o_kscan), ss);
        k_korder_place<<<(unsigned)nwg, KORDER_THREADS, lds, ss>>>(akey, ls.prodA, ls.cbseg, nnzC, op.ta,
                                                                    (int32_t)kdim, (int32_t)nwg, knext, order);
        QT_LAUNCH("k_korder_place");
        if (prof) QT_HIP(hipEventRecord(ev.e1, ss));   // the symbolic phase ends here then
        stream_after(s, ss);
    }

    // C's tree (NIL-normalised): views into its arena
    const int32_t* kept = hc.data() + 2 * L + 3;
    for (int l = 0; l < L; ++l) {
        C->levels[l].n = kept[l];
        C->levels[l].child.view(at(K, o_child[l]), 4 * (size_t)kept[l]);
        C->levels[l].key.view(at(K, o_key[l]), kept[l]);
    }
    LeafLevel& CL = C->leaves;
    CL.n = kept[L];
    CL.key.view(at(K, o_key[L]), kept[L]);
    CL.base.view(at(K, o_lbase), kept[L]);
    CL.mask_mo.view(at(K, o_lmo), kept[L]);
    CL.mask_rm.view(at(K, o_lrm), kept[L]);
    CL.mask_cm.view(at(K, o_lcm), kept[L]);
    if ((nnzC > 0) != (kept[L] > 0)) fail(QT_ERR_DEVICE, "symbolic phase: C leaves and blocks disagree");
    C->bkey.view(at(K, o_bkey), nnzC);
    C->nblocks = nnzC;

    const size_t bb = (size_t)C->b * C->b;
    if (prec == QT_F32)
        C->v32.alloc(nnzC * bb, s);
    else
        C->v64.alloc(nnzC * bb, s);
    na.prodA = ls.prodA;
    na.prodB = ls.prodB;
    na.seg = ls.cbseg;
    na.order = (leafrow || korder) ? order : nullptr;
    na.by_k = korder ? 1 : 0;
    na.nseg = nnzC;
    na.C = (prec == QT_F32) ? (void*)C->v32.p : (void*)C->v64.p;
    out.na = na;
    ev.products = C->products;
    ev.cblocks = nnzC;
}

qt_matrix* multiply(qt_matrix* A, qt_matrix* B, qt_prec prec, hipStream_t s, const MulOp& op) {
    SymbolicOut sym;
    symbolic(A, B, prec, s, sym, true, op);
    if (sym.prof) QT_HIP(hipEventRecord(sym.ev.e3, s));
    if (sym.na.nseg > 0) launch_numeric(sym.na, s);
    if (sym.prof) {
        QT_HIP(hipEventRecord(sym.ev.e2, s));
        profile_push(sym.ev);
    }
    return sym.C.release();   // sym.scratch is released in stream order
}

}  // namespace qt

// bat_host.cpp -- the C ABI declared in include/bat.h.
//
// Per call: validate -> plan (which arcs can matter, sweep order, launch
// shape) -> queue on one stream: probability tables from p (on the device),
// the enumeration kernel over the counter range, a fixed-order reduction of
// the per-work-item partials, and either a copy back (synchronous entry
// points) or a finalize kernel into the caller's device buffers (_async).
//
// The enumeration kernel is the template in bat_device.hpp, instantiated
// either ahead of time with the graph read at run time (k_fwd_dyn /
// k_grad_dyn) or at run time through hiprtc with the graph's arcs as
// compile-time constants, so that every node's reach word lives in a fixed
// register (bat_fwd_jit / bat_grad_jit).  Compiled modules are cached per
// (device, graph structure, kernel kind).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include <dlfcn.h>
#include <spawn.h>
#include <sys/stat.h>
#include <sys/wait.h>
#include <unistd.h>

#include "bat.h"
#include "bat_launch.hpp"

using bat::u32;
using bat::u64;


namespace {

const char *kVersion = "bat-mi355x 0.1.0";

#include "bat_device_embed.inc"  // kDeviceSource: bat_device.hpp as text

// ------------------------------------------------------------ errors
thread_local std::string t_err;

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? BAT_ENOMEM : BAT_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

// ------------------------------------------------------------ options
struct Options {
    std::atomic<int64_t> jit{2}, chunk_log2{0}, seg_log2{6}, check_every{1}, autotune{1}, perm{-1}, chain_log2{-1}, item_order{-1},
        window_test{1}, block_waves{-1}, super_restart{-1}, simd_waves{-1}, keep_bottom{-1}, series{1},
        grad_keep_bottom{2}, ms_run{0}, jit_procs{16}, batch_jit_arcs{-1}, batch_streams{-1}, ms_bits{1}, batch_acc{1}, jit_flush_req{0};
    Options()
    {
        auto rd = [](const char *k, std::atomic<int64_t> &v) {
            const char *e = getenv(k);
            if (e && *e) v = strtoll(e, nullptr, 10);
        };
        rd("BAT_JIT", jit);
        rd("BAT_CHUNK_LOG2", chunk_log2);
        rd("BAT_SEG_LOG2", seg_log2);
        rd("BAT_CHECK_EVERY", check_every);
        rd("BAT_AUTOTUNE", autotune);
        rd("BAT_PERM", perm);
        rd("BAT_CHAIN_LOG2", chain_log2);
        rd("BAT_ITEM_ORDER", item_order);
        rd("BAT_WINDOW_TEST", window_test);
        rd("BAT_BLOCK_WAVES", block_waves);
        rd("BAT_SUPER_RESTART", super_restart);
        rd("BAT_SIMD_WAVES", simd_waves);
        rd("BAT_KEEP_BOTTOM", keep_bottom);
        rd("BAT_SERIES", series);
        rd("BAT_GRAD_KEEP_BOTTOM", grad_keep_bottom);
        rd("BAT_MS_RUN", ms_run);
        rd("BAT_JIT_PROCS", jit_procs);
        rd("BAT_BATCH_JIT_ARCS", batch_jit_arcs);
        rd("BAT_BATCH_STREAMS", batch_streams);
        rd("BAT_MS_BITS", ms_bits);
        rd("BAT_BATCH_ACC", batch_acc);
    }
    std::atomic<int64_t> *find(const char *k)
    {
        if (!k) return nullptr;
        if (!strcmp(k, "BAT_JIT")) return &jit;
        if (!strcmp(k, "BAT_CHUNK_LOG2")) return &chunk_log2;
        if (!strcmp(k, "BAT_SEG_LOG2")) return &seg_log2;
        if (!strcmp(k, "BAT_CHECK_EVERY")) return &check_every;
        if (!strcmp(k, "BAT_AUTOTUNE")) return &autotune;
        if (!strcmp(k, "BAT_PERM")) return &perm;
        if (!strcmp(k, "BAT_CHAIN_LOG2")) return &chain_log2;
        if (!strcmp(k, "BAT_ITEM_ORDER")) return &item_order;
        if (!strcmp(k, "BAT_WINDOW_TEST")) return &window_test;
        if (!strcmp(k, "BAT_BLOCK_WAVES")) return &block_waves;
        if (!strcmp(k, "BAT_SUPER_RESTART")) return &super_restart;
        if (!strcmp(k, "BAT_SIMD_WAVES")) return &simd_waves;
        if (!strcmp(k, "BAT_KEEP_BOTTOM")) return &keep_bottom;
        if (!strcmp(k, "BAT_SERIES")) return &series;
        if (!strcmp(k, "BAT_GRAD_KEEP_BOTTOM")) return &grad_keep_bottom;
        if (!strcmp(k, "BAT_MS_RUN")) return &ms_run;
        if (!strcmp(k, "BAT_JIT_PROCS")) return &jit_procs;
        if (!strcmp(k, "BAT_BATCH_JIT_ARCS")) return &batch_jit_arcs;
        if (!strcmp(k, "BAT_BATCH_STREAMS")) return &batch_streams;
        if (!strcmp(k, "BAT_MS_BITS")) return &ms_bits;
        if (!strcmp(k, "BAT_BATCH_ACC")) return &batch_acc;
        if (!strcmp(k, "BAT_JIT_FLUSH")) return &jit_flush_req;
        return nullptr;
    }
};
Options &opts()
{
    static Options o;
    return o;
}

// ------------------------------------------------------------ validation
int validate(int32_t n, int32_t m, const bat_arc *arcs, const double *p_host, int32_t s, int32_t t)
{
    if (n < 2) return fail(BAT_EINVAL, "n_nodes must be >= 2 (got %d)", n);
    if (m < 0) return fail(BAT_EINVAL, "n_arcs must be >= 0 (got %d)", m);
    if (n > BAT_MAX_NODES) return fail(BAT_ETOOBIG, "n_nodes %d exceeds %d", n, BAT_MAX_NODES);
    if (m > BAT_MAX_ARCS) return fail(BAT_ETOOBIG, "n_arcs %d exceeds %d", m, BAT_MAX_ARCS);
    if (s < 0 || s >= n || t < 0 || t >= n) return fail(BAT_EINVAL, "s=%d or t=%d outside [0,%d)", s, t, n);
    if (s == t) return fail(BAT_EINVAL, "s and t must differ (both %d)", s);
    if (m > 0 && !arcs) return fail(BAT_EINVAL, "arcs is NULL");
    for (int32_t i = 0; i < m; ++i)
        if (arcs[i].u < 0 || arcs[i].u >= n || arcs[i].v < 0 || arcs[i].v >= n)
            return fail(BAT_EINVAL, "arc %d = (%d,%d) has a node outside [0,%d)", i, arcs[i].u, arcs[i].v, n);
    if (p_host)
        for (int32_t i = 0; i < m; ++i)
            if (!(p_host[i] >= 0.0 && p_host[i] <= 1.0))
                return fail(BAT_EINVAL, "p[%d] = %g is not a probability", i, p_host[i]);
    return BAT_OK;
}

// ------------------------------------------------------------ planning
// Arcs that lie on some simple s-t path: exactly those in the biconnected
// component of the graph plus a virtual arc (s, t) that contains the
// virtual arc (two edges share a biconnected component iff a simple cycle
// passes through both).  Every other arc never changes whether s reaches t,
// so the sweeps skip it; its state is still enumerated and weighted.
struct Bcc {
    int n, m;
    std::vector<std::vector<std::pair<int, int>>> adj;
    std::vector<int> disc, low, stk;
    std::vector<char> rel;
    int timer = 0;
    void dfs(int u, int pe)
    {
        disc[u] = low[u] = ++timer;
        for (auto [v, e] : adj[u]) {
            if (e == pe) continue;
            if (!disc[v]) {
                stk.push_back(e);
                dfs(v, e);
                low[u] = std::min(low[u], low[v]);
                if (low[v] >= disc[u]) {
                    std::vector<int> comp;
                    for (;;) {
                        int x = stk.back();
                        stk.pop_back();
                        comp.push_back(x);
                        if (x == e) break;
                    }
                    bool has_virtual = false;
                    for (int x : comp) has_virtual |= (x == m);
                    if (has_virtual)
                        for (int x : comp)
                            if (x < m) rel[x] = 1;
                }
            } else if (disc[v] < disc[u]) {
                stk.push_back(e);
                low[u] = std::min(low[u], disc[v]);
            }
        }
    }
};

struct Plan {
    int n = 0, m = 0, s = 0, t = 0;
    int perm = 0;                         // arc -> counter bit assignment kind (0 = the paper's order)
    bool directed = false;                // arcs are u -> v
    bool identity = true;                 // cb_of_arc is the paper's backward order
    std::vector<int> cb_of_arc;           // counter bit of each arc
    std::vector<unsigned char> row;       // row[j] = arc at counter bit m-1-j
    int N = 0, S = 0, T = 0;              // relevant nodes, renumbered
    std::vector<int> ru, rv, rb, rd;      // relaxations (forward order): nodes, counter bit, discovers rv
    std::vector<u32> code, wconst;        // the same for the generic kernel
    // The graph-specialised kernel's relaxations: as above, after series
    // contraction (undirected graphs), so a relaxation may stand for two
    // arcs in series; rb2 is the second arc's counter bit, -1 for one arc.
    int jN = 0, jS = 0, jT = 0;
    std::vector<int> jru, jrv, jrb, jrb2, jrd;
    std::vector<u32> prog;                // code/wconst pairs, groups of 4, forward then backward
    std::string structure;                // JIT key (graph structure only)
};

// Which arc sits at which counter bit.  Kind 0 is the paper's backward
// order (arc i at bit m-1-i) and kind kPermForward its forward BAT order
// (arc i at bit i): the range entry points use one of these two, since
// their indices are the paper's.  The others only reorder a full sweep (R
// and the count are sums over all vectors):
//   1: the 11 in-wavefront bits (word + lane) on the relevant arcs latest in
//      BFS order (nearest t), the 3 chained iteration bits on pruned arcs
//      first (their warm steps are free), then on the next-latest arcs;
//   2: in-wavefront bits as in kind 0, chained bits on pruned arcs, then on
//      arcs from the middle of the BFS order;
//   3: in-wavefront bits as in kind 1, chained bits as in kind 2.
// Every other arc keeps the relative order of kind 0.
constexpr int kPermKinds = 4;
constexpr int kDefaultPerm = 3;  // untuned whole sweeps
constexpr int kPermForward = 4;  // the forward BAT order (ranges only; never tuned)
constexpr int kGradThreeWaveNodes = 28;  // gradient sweeps of graphs up to this size run 3 waves/SIMD
constexpr int kSuperMaxNodes = 28;       // forward sweeps keep super-block bottoms in LDS up to this size

void assign_bits(int m, const std::vector<int> &rel_bfs, const std::vector<char> &rel, int kind,
                 std::vector<int> &cb_of_arc)
{
    cb_of_arc.assign(m, -1);
    if (kind == kPermForward) {  // forward BAT (Section 4.2): arc i on counter bit i
        for (int i = 0; i < m; ++i) cb_of_arc[i] = i;
        return;
    }
    if (kind == 0 || m <= bat::kWordBits) {
        for (int i = 0; i < m; ++i) cb_of_arc[i] = m - 1 - i;
        return;
    }
    std::vector<int> by_cb;
    std::vector<char> used(m, 0);
    auto take = [&](int a) {
        if (a >= 0 && a < m && !used[a]) {
            used[a] = 1;
            by_cb.push_back(a);
        }
    };
    const int nr = (int)rel_bfs.size();
    // in-wavefront bits
    if (kind == 2) {
        for (int c = 0; c < bat::kWordBits; ++c) take(m - 1 - c);
    } else {
        for (int k = nr - 1; k >= 0 && (int)by_cb.size() < bat::kWordBits; --k) take(rel_bfs[k]);
        for (int i = m - 1; i >= 0 && (int)by_cb.size() < bat::kWordBits; --i) take(i);
    }
    // chained iteration bits
    const size_t want = bat::kWordBits + 3;
    for (int i = m - 1; i >= 0 && by_cb.size() < want; --i)
        if (!rel[i]) take(i);
    if (kind == 1) {
        for (int k = nr - 1; k >= 0 && by_cb.size() < want; --k) take(rel_bfs[k]);
    } else {
        for (int d = 0; d < nr && by_cb.size() < want; ++d) {
            int k = nr / 2 + ((d & 1) ? -(d + 1) / 2 : d / 2);
            if (k >= 0 && k < nr) take(rel_bfs[k]);
        }
    }
    for (int i = m - 1; i >= 0; --i) take(i);
    for (int c = 0; c < m; ++c) cb_of_arc[by_cb[c]] = c;
}

// The specialised kernel's relaxation list.  In an undirected graph a
// node other than s and t with exactly two relevant arcs, to two different
// neighbours u and w, only ever passes reach between them: it is reached
// from u through its first arc or from w through its second, and it passes
// on nothing else.  Removing it and joining u and w by one relaxation whose
// working mask is the AND of the two arcs' masks leaves every other node's
// reach, t's in particular, exactly as it was.  Only pairs of real arcs are
// joined (a relaxation stands for at most two arcs).  Digraphs keep the
// plain list.
void contract_series(int32_t n, int32_t m, const bat_arc *arcs, int32_t s, int32_t t, const std::vector<char> &rel,
                     Plan &P)
{
    struct VArc {
        int u, v, b1, b2;
    };
    std::vector<VArc> va;
    std::vector<std::vector<int>> inc(n);  // relevant arcs at each node
    for (int i = 0; i < m; ++i)
        if (rel[i] && arcs[i].u != arcs[i].v) {
            inc[arcs[i].u].push_back(i);
            inc[arcs[i].v].push_back(i);
        }
    std::vector<char> used(m, 0), gone(n, 0);
    if (!P.directed && opts().series.load() != 0) {
        for (int v = 0; v < n; ++v) {
            if (v == s || v == t || inc[v].size() != 2) continue;
            const int a = inc[v][0], b = inc[v][1];
            if (used[a] || used[b]) continue;
            const int u = arcs[a].u == v ? arcs[a].v : arcs[a].u;
            const int w = arcs[b].u == v ? arcs[b].v : arcs[b].u;
            if (u == w || gone[u] || gone[w]) continue;
            used[a] = used[b] = 1;
            gone[v] = 1;
            va.push_back({u, w, P.cb_of_arc[a], P.cb_of_arc[b]});
        }
    }
    for (int i = 0; i < m; ++i)
        if (rel[i] && !used[i] && arcs[i].u != arcs[i].v) va.push_back({arcs[i].u, arcs[i].v, P.cb_of_arc[i], -1});
    // BFS from s in arc-list order, as for the plain list
    std::vector<int> id(n, -1), order{s};
    std::vector<char> listed(va.size(), 0);
    id[s] = 0;
    P.jru.clear(); P.jrv.clear(); P.jrb.clear(); P.jrb2.clear(); P.jrd.clear();
    for (size_t h = 0; h < order.size(); ++h) {
        const int x = order[h];
        for (size_t k = 0; k < va.size(); ++k) {
            if (listed[k]) continue;
            const VArc &e = va[k];
            if (P.directed ? e.u != x : (e.u != x && e.v != x)) continue;
            const int y = e.u == x ? e.v : e.u;
            int disc = 0;
            if (id[y] < 0) {
                id[y] = (int)order.size();
                order.push_back(y);
                disc = 1;
            }
            listed[k] = 1;
            P.jru.push_back(id[x]);
            P.jrv.push_back(id[y]);
            P.jrb.push_back(e.b1);
            P.jrb2.push_back(e.b2);
            P.jrd.push_back(disc);
        }
    }
    if (id[t] < 0) {
        id[t] = (int)order.size();
        order.push_back(t);
    }
    P.jN = (int)order.size();
    P.jS = 0;
    P.jT = id[t];
}

void make_plan(int32_t n, int32_t m, const bat_arc *arcs, int32_t s, int32_t t, Plan &P, int perm_kind = 0,
               bool directed = false)
{
    P.n = n;
    P.m = m;
    P.s = s;
    P.t = t;
    P.perm = perm_kind;
    P.directed = directed;
    Bcc B;
    B.n = n;
    B.m = m;
    B.rel.assign(m + 1, 0);
    if (!directed) {
        B.adj.assign(n, {});
        for (int i = 0; i < m; ++i) {
            int u = arcs[i].u, v = arcs[i].v;
            if (u == v) continue;  // a self-loop never joins two nodes
            B.adj[u].push_back({v, i});
            B.adj[v].push_back({u, i});
        }
        B.adj[s].push_back({t, m});
        B.adj[t].push_back({s, m});
        B.disc.assign(n, 0);
        B.low.assign(n, 0);
        B.dfs(s, -1);
    } else {
        // arc u -> v can only matter when s reaches u and v reaches t, and
        // it neither enters s nor leaves t (a superset of the arcs on simple
        // s -> t paths, which is hard to decide exactly for digraphs)
        std::vector<char> from_s(n, 0), to_t(n, 0);
        std::vector<int> q{s};
        from_s[s] = 1;
        for (size_t h = 0; h < q.size(); ++h)
            for (int i = 0; i < m; ++i)
                if (arcs[i].u == q[h] && !from_s[arcs[i].v]) {
                    from_s[arcs[i].v] = 1;
                    q.push_back(arcs[i].v);
                }
        q.assign(1, t);
        to_t[t] = 1;
        for (size_t h = 0; h < q.size(); ++h)
            for (int i = 0; i < m; ++i)
                if (arcs[i].v == q[h] && !to_t[arcs[i].u]) {
                    to_t[arcs[i].u] = 1;
                    q.push_back(arcs[i].u);
                }
        for (int i = 0; i < m; ++i) {
            const int u = arcs[i].u, v = arcs[i].v;
            B.rel[i] = u != v && v != s && u != t && from_s[u] && to_t[v];
        }
    }

    // BFS from s over relevant arcs: node numbering and sweep order
    std::vector<int> id(n, -1), order, rel_bfs, disc_flag;
    std::vector<char> listed(m, 0);
    std::vector<std::pair<int, int>> ends;
    id[s] = 0;
    order.push_back(s);
    for (size_t h = 0; h < order.size(); ++h) {
        int u = order[h];
        for (int i = 0; i < m; ++i) {
            if (!B.rel[i] || listed[i]) continue;
            int a = arcs[i].u, b = arcs[i].v;
            if (directed ? a != u : (a != u && b != u)) continue;  // directed: leave by the tail
            int w = (a == u) ? b : a;
            int discovers = 0;
            if (id[w] < 0) {
                id[w] = (int)order.size();
                order.push_back(w);
                discovers = 1;
            }
            listed[i] = 1;
            rel_bfs.push_back(i);
            ends.push_back({id[u], id[w]});
            disc_flag.push_back(discovers);
        }
    }
    if (id[t] < 0) {  // s and t never connected: keep both as nodes, no arcs
        id[t] = (int)order.size();
        order.push_back(t);
    }
    // relevant = swept: an arc the search from s never lists cannot matter
    std::vector<char> rel(m, 0);
    for (int i = 0; i < m; ++i) rel[i] = listed[i];
    assign_bits(m, rel_bfs, rel, perm_kind, P.cb_of_arc);
    {  // must be a bijection onto [0, m); otherwise use the paper's order
        std::vector<char> hit(std::max(m, 1), 0);
        bool ok = true;
        for (int i = 0; i < m; ++i) {
            int c = P.cb_of_arc[i];
            if (c < 0 || c >= m || hit[c]) ok = false;
            else hit[c] = 1;
        }
        if (!ok) {
            P.perm = 0;
            for (int i = 0; i < m; ++i) P.cb_of_arc[i] = m - 1 - i;
        }
    }
    P.identity = true;  // the paper's backward order: arc i on counter bit m - 1 - i
    for (int i = 0; i < m; ++i)
        if (P.cb_of_arc[i] != m - 1 - i) P.identity = false;
    P.row.assign(std::max(m, 1), 0);
    for (int i = 0; i < m; ++i) P.row[m - 1 - P.cb_of_arc[i]] = (unsigned char)i;
    P.ru.clear(); P.rv.clear(); P.rb.clear(); P.rd.clear();
    for (size_t k = 0; k < rel_bfs.size(); ++k) {
        P.ru.push_back(ends[k].first);
        P.rv.push_back(ends[k].second);
        P.rb.push_back(P.cb_of_arc[rel_bfs[k]]);
        P.rd.push_back(disc_flag[k]);
    }
    P.N = (int)order.size();
    P.S = 0;
    P.T = id[t];
    P.code.resize(P.ru.size());
    P.wconst.resize(P.ru.size());
    for (size_t k = 0; k < P.ru.size(); ++k) {
        P.code[k] = (u32)P.ru[k] | ((u32)P.rv[k] << 6) | ((u32)P.rb[k] << 12);
        P.wconst[k] = P.rb[k] < bat::kSliceBits ? bat::slice_pattern(P.rb[k]) : 0u;
    }
    // the generic kernel's program: (code, pattern) pairs in sweep order,
    // each direction padded to whole groups of 4 with (0, 0), which relaxes
    // node 0 against itself with an empty mask (a no-op)
    {
        const size_t nr = P.code.size(), ng = (nr + 3) / 4;
        P.prog.assign(2 * ng * 8 + 8, 0u);  // + the spare group read ahead of the last
        for (size_t k = 0; k < nr; ++k) {
            P.prog[2 * k] = P.code[k];
            P.prog[2 * k + 1] = P.wconst[k];
            const size_t kb = nr - 1 - k;  // backward sweep position of relaxation k
            P.prog[ng * 8 + 2 * kb] = P.code[k];
            P.prog[ng * 8 + 2 * kb + 1] = P.wconst[k];
        }
    }
    contract_series(n, m, arcs, s, t, rel, P);
    std::string sdesc = std::string(directed ? "D " : "") + "N" + std::to_string(P.jN) + " S" + std::to_string(P.jS) +
                        " T" + std::to_string(P.jT) + " m" + std::to_string(m) + " :";
    for (size_t k = 0; k < P.jru.size(); ++k)
        sdesc += " " + std::to_string(P.jru[k]) + "," + std::to_string(P.jrv[k]) + "," + std::to_string(P.jrb[k]) +
                 (P.jrb2[k] >= 0 ? "&" + std::to_string(P.jrb2[k]) : std::string()) + (P.jrd[k] ? "d" : "");
    P.structure = sdesc;
}

// Relaxation code of each chained counter bit 11 + b (b = 0..5), ~0 where
// that arc is pruned (no relaxation) or absent.
void chain_codes(const Plan &P, u32 out[6])
{
    for (int b = 0; b < 6; ++b) out[b] = ~0u;
    for (size_t k = 0; k < P.code.size(); ++k)
        if (P.rb[k] >= bat::kWordBits && P.rb[k] < bat::kWordBits + 6) out[P.rb[k] - bat::kWordBits] = P.code[k];
}

// ------------------------------------------------------------ device state
struct DeviceInfo {
    int id = -1;
    int cus = 0;
    std::string arch;
};

int current_device(DeviceInfo &D)
{
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        DeviceInfo d;
        d.id = dev;
        d.cus = prop.multiProcessorCount;
        d.arch = prop.gcnArchName;
        it = cache.emplace(dev, d).first;
    }
    D = it->second;
    return BAT_OK;
}

// Per thread and device: a device workspace and a pinned host staging
// buffer the synchronous calls reuse (grown, never shrunk), so a small call
// makes one host-to-device and one device-to-host copy and no allocation.
struct Scratch {
    char *dev = nullptr;
    size_t dev_cap = 0;
    char *host = nullptr;
    size_t host_cap = 0;
};

// What exiting threads leave behind, for later threads to take over. A
// thread's destructor makes no HIP call (the runtime may already be torn
// down at process exit), so its streams, events and scratch come here
// instead of being freed; the pool itself lives until the process ends.
// Side streams of a thread on one device, for launches that may overlap
// (the batched sweep's graph-specialised kernels), with the events that
// fork them from and join them to the thread's stream.
constexpr int kSideStreams = 4;
struct SideStreams {
    hipStream_t s[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

struct ResourcePool {
    std::mutex mu;
    std::multimap<int, hipStream_t> streams;
    std::multimap<int, Scratch> scratch;
    std::vector<std::vector<hipEvent_t>> events;
    std::multimap<int, SideStreams> side;
};
ResourcePool &pool()
{
    static ResourcePool *P = new ResourcePool;  // never destroyed
    return *P;
}

struct ThreadState {
    std::map<int, hipStream_t> streams;
    std::map<int, SideStreams> side;
    std::map<int, Scratch> scratch;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool have_launch = false;
    bat_launch_info info{};
    ~ThreadState()
    {
        ResourcePool &P = pool();
        std::lock_guard<std::mutex> g(P.mu);
        for (auto &kv : streams) P.streams.emplace(kv.first, kv.second);
        for (auto &kv : side) P.side.emplace(kv.first, kv.second);
        for (auto &kv : scratch)
            if (kv.second.dev || kv.second.host) P.scratch.emplace(kv.first, kv.second);
        if (ev[0]) P.events.emplace_back(ev, ev + 4);
    }
};
thread_local ThreadState t_state;

int thread_stream(int dev, hipStream_t &s)
{
    auto it = t_state.streams.find(dev);
    if (it == t_state.streams.end()) {
        hipStream_t st = nullptr;
        {
            ResourcePool &P = pool();
            std::lock_guard<std::mutex> g(P.mu);
            auto pit = P.streams.find(dev);
            if (pit != P.streams.end()) {
                st = pit->second;
                P.streams.erase(pit);
            }
        }
        if (!st) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        it = t_state.streams.emplace(dev, st).first;
    }
    s = it->second;
    return BAT_OK;
}

int side_streams(int dev, SideStreams *&out)
{
    auto it = t_state.side.find(dev);
    if (it == t_state.side.end()) {
        SideStreams S;
        bool have = false;
        {
            ResourcePool &P = pool();
            std::lock_guard<std::mutex> g(P.mu);
            auto pit = P.side.find(dev);
            if (pit != P.side.end()) {
                S = pit->second;
                P.side.erase(pit);
                have = true;
            }
        }
        if (!have) {
            // default priority, like every stream of the library
            for (int k = 0; k < kSideStreams; ++k) HIPCHK(hipStreamCreateWithFlags(&S.s[k], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&S.fork, hipEventDisableTiming));
            for (int k = 0; k < kSideStreams; ++k) HIPCHK(hipEventCreateWithFlags(&S.join[k], hipEventDisableTiming));
        }
        it = t_state.side.emplace(dev, S).first;
    }
    out = &it->second;
    return BAT_OK;
}

// Make the thread's scratch on device `dev` at least this large; growing
// waits for the stream first (the old buffers may still be in use).
int scratch_reserve(int dev, hipStream_t st, size_t dev_bytes, size_t host_bytes, Scratch *&S)
{
    auto sit = t_state.scratch.find(dev);
    if (sit == t_state.scratch.end()) {
        Scratch taken;
        {
            ResourcePool &P = pool();
            std::lock_guard<std::mutex> g(P.mu);
            auto pit = P.scratch.find(dev);
            if (pit != P.scratch.end()) {
                taken = pit->second;
                P.scratch.erase(pit);
            }
        }
        sit = t_state.scratch.emplace(dev, taken).first;
    }
    S = &sit->second;
    if (S->dev_cap < dev_bytes) {
        HIPCHK(hipStreamSynchronize(st));
        if (S->dev) HIPCHK(hipFree(S->dev));
        S->dev = nullptr;
        S->dev_cap = 0;
        const size_t cap = std::max<size_t>(dev_bytes, 1 << 20);
        HIPCHK(hipMalloc((void **)&S->dev, cap));
        S->dev_cap = cap;
    }
    if (S->host_cap < host_bytes) {
        HIPCHK(hipStreamSynchronize(st));
        if (S->host) HIPCHK(hipHostFree(S->host));
        S->host = nullptr;
        S->host_cap = 0;
        const size_t cap = std::max<size_t>(host_bytes, 64 << 10);
        HIPCHK(hipHostMalloc((void **)&S->host, cap, hipHostMallocDefault));
        S->host_cap = cap;
    }
    return BAT_OK;
}

int events_ready()
{
    if (!t_state.ev[0]) {
        {
            ResourcePool &P = pool();
            std::lock_guard<std::mutex> g(P.mu);
            if (!P.events.empty()) {
                for (int i = 0; i < 4; ++i) t_state.ev[i] = P.events.back()[i];
                P.events.pop_back();
            }
        }
        if (!t_state.ev[0])
            for (auto &e : t_state.ev) HIPCHK(hipEventCreate(&e));
    }
    return BAT_OK;
}

// ------------------------------------------------- fixed device scratch
// The workspace of bat_reliability_noalloc: a fixed array in device memory,
// one copy per GPU the library runs on, held until the process ends.  In
// host code `scratch` names the symbol, not a device address: the address
// of a GPU's copy comes from hipGetSymbolAddress with that GPU current, once
// per device, and only that address is passed to kernels and copies.
constexpr size_t kNoAllocScratchBytes = BAT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

int noalloc_scratch(int dev, char *&ptr)
{
    static std::mutex mu;
    static std::map<int, char *> addr;  // device -> its copy of `scratch`
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void *a = nullptr;
        HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a) return fail(BAT_EDEVICE, "no device address for the fixed scratch on device %d", dev);
        it = addr.emplace(dev, (char *)a).first;
    }
    ptr = it->second;
    return BAT_OK;
}

// ------------------------------------------------------------ JIT cache
struct JitEntry {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    uint64_t id = 0;  // hash of the compiled code object
};
std::mutex g_jit_mu;
std::map<std::string, JitEntry> g_jit;

// Drop every compiled kernel of this process (modules unloaded) after the
// current device has finished its work.
// Code objects compiled before their first launch (the autotuner compiles
// its candidates' kernels side by side), by the key of their source text.
std::mutex g_pre_mu;
std::map<std::pair<uint64_t, uint64_t>, std::vector<char>> g_precompiled;

void jit_flush()
{
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(g_pre_mu);
        g_precompiled.clear();
    }
    std::lock_guard<std::mutex> lk(g_jit_mu);
    for (auto &kv : g_jit)
        if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
    g_jit.clear();
}

// ---------------------------------------------------- on-disk code cache
// Compiled code objects are kept across processes, keyed by two
// independent 64-bit hashes of the whole source text, the target and the
// compile options, so a changed kernel is never served stale.  Directory:
// BAT_JIT_CACHE_DIR, else $XDG_CACHE_HOME/bat-mi355x, else
// $HOME/.cache/bat-mi355x; BAT_JIT_CACHE=0 turns it off.  Anything that
// fails to read, write or load falls back to compiling.
struct CacheKey {
    uint64_t h1, h2, len;
};
CacheKey cache_key(const std::string &text)
{
    uint64_t a = 1469598103934665603ull, b = 0x9E3779B97F4A7C15ull;
    for (unsigned char c : text) {
        a = (a ^ c) * 1099511628211ull;           // FNV-1a
        b = (b + c) * 0xBF58476D1CE4E5B9ull;       // multiply-add, then mix
        b ^= b >> 31;
    }
    return {a, b, (uint64_t)text.size()};
}
// Identity of a code object's machine code: a hash of its .text and
// .rodata sections. The rest of the object varies between compilations of
// the same source (the compilation-unit id symbol), the code does not. A
// blob that does not parse as a 64-bit ELF is hashed whole.
uint64_t machine_code_id(const std::vector<char> &co)
{
    const size_t n = co.size();
    auto rd = [&](size_t off, size_t len, uint64_t &v) {
        if (off + len > n) return false;
        v = 0;
        for (size_t i = 0; i < len; ++i) v |= (uint64_t)(unsigned char)co[off + i] << (8 * i);
        return true;
    };
    uint64_t shoff = 0, shentsize = 0, shnum = 0, shstrndx = 0;
    const bool elf = n > 64 && co[0] == 0x7f && co[1] == 'E' && co[2] == 'L' && co[3] == 'F' && co[4] == 2 &&
                     rd(0x28, 8, shoff) && rd(0x3A, 2, shentsize) && rd(0x3C, 2, shnum) && rd(0x3E, 2, shstrndx) &&
                     shentsize >= 64 && shstrndx < shnum && shoff + shnum * shentsize <= n;
    if (!elf) return cache_key(std::string(co.begin(), co.end())).h1;
    uint64_t stroff = 0;
    if (!rd(shoff + shstrndx * shentsize + 0x18, 8, stroff)) return cache_key(std::string(co.begin(), co.end())).h1;
    std::string text;
    for (uint64_t i = 0; i < shnum; ++i) {
        const size_t h = shoff + i * shentsize;
        uint64_t name = 0, type = 0, off = 0, size = 0;
        if (!rd(h, 4, name) || !rd(h + 4, 4, type) || !rd(h + 0x18, 8, off) || !rd(h + 0x20, 8, size)) continue;
        if (type == 8 || off + size > n || stroff + name >= n) continue;  // no bits in the file
        const char *nm = co.data() + stroff + name;
        const size_t room = n - (stroff + name);
        if (strnlen(nm, room) == room) continue;
        if (!strcmp(nm, ".text") || !strcmp(nm, ".rodata")) text.append(co.data() + off, size);
    }
    if (text.empty()) return cache_key(std::string(co.begin(), co.end())).h1;
    return cache_key(text).h1;
}

// Identity of an ahead-of-time kernel instance: the digest of the sources
// it was compiled from, the kernel and its node-count class.
uint64_t aot_kernel_id(const char *kernel, int nodes, bool directed)
{
    const int nmax = nodes <= 16 ? 16 : nodes <= 32 ? 32 : 64;
    return cache_key(std::string(kAotKernelDigest) + " " + kernel + " " + std::to_string(nmax) +
                     (directed ? " directed" : ""))
        .h1;
}

std::string cache_dir()
{
    const char *on = getenv("BAT_JIT_CACHE");
    if (on && !strcmp(on, "0")) return "";
    std::string d;
    if (const char *e = getenv("BAT_JIT_CACHE_DIR"); e && *e) {
        d = e;
    } else if (const char *x = getenv("XDG_CACHE_HOME"); x && *x) {
        d = std::string(x) + "/bat-mi355x";
    } else if (const char *h = getenv("HOME"); h && *h) {
        d = std::string(h) + "/.cache";
        mkdir(d.c_str(), 0755);
        d += "/bat-mi355x";
    } else {
        return "";
    }
    mkdir(d.c_str(), 0755);  // may exist already
    struct stat st;
    if (stat(d.c_str(), &st) != 0 || !S_ISDIR(st.st_mode)) return "";
    return d;
}
std::string cache_path(const std::string &dir, const CacheKey &k)
{
    char name[64];
    snprintf(name, sizeof name, "/%016llx.co", (unsigned long long)k.h1);
    return dir + name;
}
constexpr char kCacheMagic[8] = {'B', 'A', 'T', 'J', 'I', 'T', '1', '\n'};
bool cache_read(const std::string &path, const CacheKey &k, std::vector<char> &code)
{
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return false;
    char magic[8];
    uint64_t hdr[3], n = 0;
    bool ok = fread(magic, 1, 8, f) == 8 && !memcmp(magic, kCacheMagic, 8) && fread(hdr, 8, 3, f) == 3 &&
              hdr[0] == k.h1 && hdr[1] == k.h2 && hdr[2] == k.len && fread(&n, 8, 1, f) == 1 && n > 0 &&
              n < (1ull << 30);
    if (ok) {
        code.resize(n);
        ok = fread(code.data(), 1, n, f) == n;
    }
    fclose(f);
    return ok;
}
void cache_write(const std::string &path, const CacheKey &k, const std::vector<char> &code)
{
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    const uint64_t hdr[4] = {k.h1, k.h2, k.len, (uint64_t)code.size()};
    bool ok = fwrite(kCacheMagic, 1, 8, f) == 8 && fwrite(hdr, 8, 4, f) == 4 &&
              fwrite(code.data(), 1, code.size(), f) == code.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path.c_str()) != 0) unlink(tmp.c_str());
}

// Launch shape of a specialised kernel: wavefronts per block and whether
// forward sweeps keep super-block bottoms in LDS.  The gradient sweep
// always runs 4 wavefronts per block and no super-block store.
struct JitShape {
    int waves = bat::kWavesPerBlock;
    bool super_restart = false;
    int simd_waves = 0;  // > 0: ask the compiler to fit this many wavefronts per SIMD
    bool keep_bottom = true;  // chain starts resume from the kept block bottom
    bool bottom_lds = false;  // ... kept in LDS instead of registers
};

// Default shape of the forward sweep: 4 wavefronts per block, kept block
// bottoms, no super-block store, compiled to fit 6 wavefronts per SIMD.
// The kernel is latency-bound: on the 5x5 grid, fitting 6 wavefronts (80
// registers, spills outside the innermost loops) instead of the compiler's
// 4 (109 registers) takes the sweep from 161 to 141 ms.  Bigger plans
// spill inside the sweeps at that budget but still gained (a 29-word
// plan: 11.6 ms against 13.5 ms with the compiler's budget).
constexpr int kDefaultSimdWaves = 6;

// waves: 1, 2 or 4 (anything else: 4); super_restart: 1 on, else off;
// simd_waves: 5 to 8, 0 = the compiler's own register budget, else the
// default; keep_bottom: 0 off, else on
JitShape jit_shape(bool grad, int waves, int super_restart, int simd_waves, int keep_bottom)
{
    JitShape sh;
    if (grad) {
        // the gradient sweep of a graph of up to kGradThreeWaveNodes nodes
        // fits 3 wavefronts per SIMD without spilling; on the 36-arc random
        // graph 4 (128 registers, spilling) took 32 ms against 20 ms
        sh.simd_waves = 3;
        // the gradient's registers are full: a kept bottom lives in LDS
        sh.keep_bottom = opts().grad_keep_bottom.load() == 2;
        sh.bottom_lds = sh.keep_bottom;
    } else {
        sh.keep_bottom = keep_bottom != 0;
        sh.bottom_lds = keep_bottom == 2;
        sh.waves = waves == 1 ? 1 : waves == 2 ? 2 : 4;
        sh.super_restart = super_restart == 1;
        sh.simd_waves = (simd_waves >= 5 && simd_waves <= 8) ? simd_waves : simd_waves == 0 ? 0 : kDefaultSimdWaves;
    }
    return sh;
}

// batch_np > 0: instead of the forward or gradient sweep, the batched
// sweep of batch_np probability vectors, in blocks of batch_jit_waves
// wavefronts: 3 per SIMD (168 registers) keep the sweep loops free of
// spills up to 16 p-vectors, beyond that 2 per SIMD (256 registers); at 3
// per SIMD 32 accumulators spill inside the sweeps
constexpr int batch_jit_waves(int np) { return np > 16 ? 8 : 12; }
// the transposed accumulation (option BAT_BATCH_ACC 1, 9..32 p-vectors:
// two lanes per p-vector above 16, else four): one accumulator per lane,
// blocks of kBatchTWaves wavefronts
constexpr int kBatchTWaves = 16;
static_assert(kBatchTWaves <= bat::kBatchTMaxWaves, "one LDS row per wavefront");
bool batch_transposed(int np) { return np > 8 && np <= bat::kBatchCols && opts().batch_acc.load() == 1; }
int batch_waves(int np) { return batch_transposed(np) ? kBatchTWaves : batch_jit_waves(np); }
// p-vectors per specialised entry: 32 (blocks of 8 wavefronts) measured
// faster than two entries of 16 (blocks of 12) on 256 graphs x 32
// p-vectors, 18.7 against 19.4 ms: the closure then runs once
constexpr int kBatchSpecP = 32;

std::string jit_source(const Plan &P, bool grad, const JitShape &sh, int batch_np = 0)
{
    std::string s;
    s.reserve(strlen(kDeviceSource) + 4096);
    s += kDeviceSource;
    s += "\nstruct JitGraph {\n";
    s += "  static constexpr int N = " + std::to_string(P.jN) + ";\n";
    s += "  static constexpr int S = " + std::to_string(P.jS) + ";\n";
    s += "  static constexpr int T = " + std::to_string(P.jT) + ";\n";
    size_t nr = P.jru.size();
    s += "  static constexpr int NR = " + std::to_string(nr) + ";\n";
    auto arr = [&](const char *name, const std::vector<int> &v) {
        s += std::string("  static constexpr unsigned char ") + name + "[" + std::to_string(nr ? nr : 1) + "] = {";
        if (nr == 0) s += "0";
        for (size_t k = 0; k < nr; ++k) s += (k ? "," : "") + std::to_string(v[k]);
        s += "};\n";
    };
    arr("RU", P.jru);
    arr("RV", P.jrv);
    arr("RB", P.jrb);
    arr("RD", P.jrd);
    // second counter bit of a relaxation that joins two arcs in series
    // (255: one arc)
    {
        std::vector<int> b2(nr);
        for (size_t k = 0; k < nr; ++k) b2[k] = P.jrb2[k] < 0 ? 255 : P.jrb2[k];
        arr("RB2", b2);
    }
    s += std::string("  static constexpr bool DIR = ") + (P.directed ? "true" : "false") + ";\n";
    // forward sweeps of graphs small enough for the LDS store (4 blocks of
    // 4 wavefronts per CU keep (N + 2) words per lane each) also resume
    // block bottoms from the kept bottom of their 2^6-aligned super-block
    s += std::string("  static constexpr bool SUPER = ") +
         (!grad && sh.super_restart && P.jN <= kSuperMaxNodes ? "true" : "false") + ";\n";
    // wavefronts per block (the launch uses the same)
    s += "  static constexpr int WAVES = " + std::to_string(sh.waves) + ";\n";
    s += std::string("  static constexpr bool KEEPB = ") + (sh.keep_bottom ? "true" : "false") + ";\n";
    s += std::string("  static constexpr bool BOTTOM_LDS = ") + (sh.bottom_lds ? "true" : "false") + ";\n";
    // relaxations of counter bits 11..16 (the chained iteration arcs)
    int ck[6] = {-1, -1, -1, -1, -1, -1};
    for (size_t k = 0; k < nr; ++k)
        for (int b : {P.jrb[k], P.jrb2[k]})
            if (b >= bat::kWordBits && b < bat::kWordBits + 6) ck[b - bat::kWordBits] = (int)k;
    s += "  static constexpr int CK[6] = {";
    for (int b = 0; b < 6; ++b) s += (b ? "," : "") + std::to_string(ck[b]);
    s += "};\n";
    s += "};\n";
    // the gradient sweep of a small graph fits three wavefronts per SIMD
    // with spills confined to once-per-segment code; larger graphs keep the
    // compiler's register budget
    if (grad && P.jN <= kGradThreeWaveNodes && sh.simd_waves)
        s += "extern \"C\" __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(" +
             std::to_string(sh.simd_waves) + ", " + std::to_string(sh.simd_waves) + ")))\n"
             "bat_grad_jit(bat::KParams P) {\n"
             "  __shared__ bat::LdsTables L; __shared__ bat::LdsGrad LG;\n"
             "  bat::sweep_kernel<bat::StaticClosure<JitGraph>, true>(P, L, &LG);\n}\n";
    else if (batch_np > 0 && batch_transposed(batch_np))
        s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(bat::kWave * kBatchTWaves) +
             ") bat_batch_jit(bat::KParams P) {\n"
             "  __shared__ bat::LdsBatchT<" + std::to_string(batch_np) + "> L;\n"
             "  bat::batch_kernel_t<bat::StaticClosure<JitGraph>, " + std::to_string(batch_np) + ">(P, L);\n}\n";
    else if (batch_np > 0)
        s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(bat::kWave * batch_jit_waves(batch_np)) +
             ") bat_batch_jit(bat::KParams P) {\n"
             "  __shared__ bat::LdsBatch<" + std::to_string(batch_np) + "> L;\n"
             "  bat::batch_kernel<bat::StaticClosure<JitGraph>, " + std::to_string(batch_np) + ">(P, L);\n}\n";
    else if (grad)
        s += "extern \"C\" __global__ void __launch_bounds__(256) bat_grad_jit(bat::KParams P) {\n"
             "  __shared__ bat::LdsTables L; __shared__ bat::LdsGrad LG;\n"
             "  bat::sweep_kernel<bat::StaticClosure<JitGraph>, true>(P, L, &LG);\n}\n";
    else
        s += "extern \"C\" __global__ void __launch_bounds__(" + std::to_string(bat::kWave * sh.waves) + ")" +
             (sh.simd_waves ? " __attribute__((amdgpu_waves_per_eu(" + std::to_string(sh.simd_waves) + ", " +
                                  std::to_string(sh.simd_waves) + ")))"
                            : std::string()) +
             " bat_fwd_jit(bat::KParams P) {\n"
             "  __shared__ bat::LdsTables L;\n"
             "  bat::sweep_kernel<bat::StaticClosure<JitGraph>, false>(P, L, nullptr);\n}\n";
    return s;
}

// One hiprtc compilation of a specialised kernel's source (no shared state:
// several may run at once on host threads).
const char *const kJitOpts[] = {"-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

std::string jit_key_text(const std::string &src, const std::string &arch)
{
    std::string keytext = src;
    keytext += "\n//--offload-arch=" + arch;
    for (const char *opt : kJitOpts) keytext += std::string("\n//") + opt;
    return keytext;
}

bool jit_compile(const std::string &src, const std::string &arch, std::vector<char> &code, std::string &err)
{
    const std::string a = "--offload-arch=" + arch;
    std::vector<const char *> o{a.c_str()};
    for (const char *opt : kJitOpts) o.push_back(opt);
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "bat_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)o.size(), o.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        err = std::string(hiprtcGetErrorString(rc)) + ": " + log.substr(0, 800);
        return false;
    }
    size_t sz = 0;
    hiprtcGetCodeSize(prog, &sz);
    code.assign(sz, 0);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

// The compile helper (bat_jitc) installed beside this library, or "".
std::string jitc_path()
{
    Dl_info di;
    if (!dladdr((const void *)&jitc_path, &di) || !di.dli_fname) return "";
    std::string p = di.dli_fname;
    const size_t slash = p.rfind('/');
    p = (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/bat_jitc";
    return access(p.c_str(), X_OK) == 0 ? p : "";
}

// The file of the hiprtc library this process compiles with, or "".
std::string hiprtc_path()
{
    Dl_info di;
    if (!dladdr((const void *)&hiprtcCompileProgram, &di) || !di.dli_fname) return "";
    return di.dli_fname;
}

// Compile the kernels of these sources that are neither precompiled nor
// on disk.  hiprtc runs one compilation at a time per process, so they run
// in child processes of the compile helper, up to option BAT_JIT_PROCS at
// once; their first launch then only loads the code.  Whatever does not
// come back (no helper, a failed child) is compiled in-process by that
// launch as usual.
void jit_precompile_sources(const DeviceInfo &D, const std::vector<std::string> &sources);

// The same for the kernels of these (plan, gradient?, shape) launches.
void jit_precompile(const DeviceInfo &D, const std::vector<std::tuple<const Plan *, bool, JitShape>> &want)
{
    std::vector<std::string> sources;
    for (const auto &w : want) sources.push_back(jit_source(*std::get<0>(w), std::get<1>(w), std::get<2>(w)));
    jit_precompile_sources(D, sources);
}

void jit_precompile_sources(const DeviceInfo &D, const std::vector<std::string> &sources)
{
    const int64_t procs = std::min<int64_t>(opts().jit_procs.load(), 64);
    if (procs < 1) return;
    const std::string helper = jitc_path(), rtc = hiprtc_path();
    if (helper.empty() || rtc.empty()) return;
    struct Job {
        std::string src;
        CacheKey ck;
        std::string src_path, out_path;
        pid_t pid = -1;
    };
    std::vector<Job> jobs;
    const std::string cdir = cache_dir();
    for (const std::string &src : sources) {
        Job j;
        j.src = src;
        j.ck = cache_key(jit_key_text(j.src, D.arch));
        {
            std::lock_guard<std::mutex> lk(g_pre_mu);
            if (g_precompiled.count({j.ck.h1, j.ck.h2})) continue;
        }
        if (!cdir.empty()) {
            struct stat st;
            if (stat(cache_path(cdir, j.ck).c_str(), &st) == 0) continue;  // on disk already
        }
        bool dup = false;
        for (const Job &o : jobs) dup = dup || (o.ck.h1 == j.ck.h1 && o.ck.h2 == j.ck.h2);
        if (!dup) jobs.push_back(std::move(j));
    }
    if (jobs.empty()) return;
    const char *tenv = getenv("TMPDIR");
    std::string dir = std::string(tenv && *tenv ? tenv : "/tmp") + "/bat_jitc.XXXXXX";
    if (!mkdtemp(&dir[0])) return;
    const std::string arch = "--offload-arch=" + D.arch;
    for (size_t i0 = 0; i0 < jobs.size(); i0 += (size_t)procs) {
        const size_t i1 = std::min(jobs.size(), i0 + (size_t)procs);
        for (size_t i = i0; i < i1; ++i) {
            Job &j = jobs[i];
            j.src_path = dir + "/" + std::to_string(i) + ".hip";
            j.out_path = dir + "/" + std::to_string(i) + ".co";
            FILE *f = fopen(j.src_path.c_str(), "wb");
            if (!f) continue;
            const bool ok = fwrite(j.src.data(), 1, j.src.size(), f) == j.src.size();
            if (fclose(f) != 0 || !ok) continue;
            std::vector<char *> argv{(char *)helper.c_str(), (char *)rtc.c_str(), (char *)j.src_path.c_str(),
                                     (char *)j.out_path.c_str(), (char *)arch.c_str()};
            for (const char *opt : kJitOpts) argv.push_back((char *)opt);
            argv.push_back(nullptr);
            pid_t pid;
            if (posix_spawn(&pid, helper.c_str(), nullptr, nullptr, argv.data(), environ) == 0) j.pid = pid;
        }
        for (size_t i = i0; i < i1; ++i) {
            Job &j = jobs[i];
            if (j.pid > 0) {
                int st = 0;
                pid_t r;
                while ((r = waitpid(j.pid, &st, 0)) < 0 && errno == EINTR) {
                }
                std::vector<char> code;
                if (r == j.pid && WIFEXITED(st) && WEXITSTATUS(st) == 0) {
                    if (FILE *f = fopen(j.out_path.c_str(), "rb")) {
                        char buf[1 << 16];
                        size_t k;
                        while ((k = fread(buf, 1, sizeof buf, f)) > 0) code.insert(code.end(), buf, buf + k);
                        fclose(f);
                    }
                }
                if (!code.empty()) {
                    if (!cdir.empty()) cache_write(cache_path(cdir, j.ck), j.ck, code);
                    std::lock_guard<std::mutex> lk(g_pre_mu);
                    g_precompiled[{j.ck.h1, j.ck.h2}] = std::move(code);
                }
            }
            unlink(j.src_path.c_str());
            unlink(j.out_path.c_str());
        }
    }
    rmdir(dir.c_str());
}

// The kernel `kname` of source `src`, loaded once per process under `key`:
// from the precompiled table, else the disk cache, else compiled here.
int jit_load(const DeviceInfo &D, const std::string &key, const std::string &src, const char *kname,
             hipFunction_t &fn, double &compile_ms, uint64_t &id)
{
    compile_ms = 0.0;
    std::lock_guard<std::mutex> lk(g_jit_mu);
    auto it = g_jit.find(key);
    if (it != g_jit.end()) {
        fn = it->second.fn;
        id = it->second.id;
        return BAT_OK;
    }
    auto t0 = std::chrono::steady_clock::now();
    const CacheKey ck = cache_key(jit_key_text(src, D.arch));
    const std::string cdir = cache_dir();
    std::vector<char> code;
    // the kernel's identity: its machine code, so that edits which leave
    // the code alone (comments) keep it
    auto code_id = [&]() { return machine_code_id(code); };
    bool pre = false;
    {
        std::lock_guard<std::mutex> lk2(g_pre_mu);
        auto pit = g_precompiled.find({ck.h1, ck.h2});
        if (pit != g_precompiled.end()) {
            code = std::move(pit->second);
            g_precompiled.erase(pit);
            pre = true;
        }
    }
    if (!pre && !cdir.empty() && cache_read(cache_path(cdir, ck), ck, code)) {
        JitEntry e;
        e.id = id = code_id();
        if (hipModuleLoadData(&e.mod, code.data()) == hipSuccess && hipModuleGetFunction(&e.fn, e.mod, kname) == hipSuccess) {
            g_jit.emplace(key, e);
            fn = e.fn;
            compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            return BAT_OK;
        }
        if (e.mod) (void)hipModuleUnload(e.mod);
        (void)hipGetLastError();  // a stale or damaged entry: compile afresh
    }
    if (!pre) {
        std::string err;
        if (!jit_compile(src, D.arch, code, err)) return fail(BAT_EDEVICE, "hiprtc compile failed (%s)", err.c_str());
        if (!cdir.empty()) cache_write(cache_path(cdir, ck), ck, code);
    }
    JitEntry e;
    e.id = id = code_id();
    HIPCHK(hipModuleLoadData(&e.mod, code.data()));
    HIPCHK(hipModuleGetFunction(&e.fn, e.mod, kname));
    g_jit.emplace(key, e);
    fn = e.fn;
    compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return BAT_OK;
}

int jit_get(const DeviceInfo &D, const Plan &P, bool grad, const JitShape &sh, hipFunction_t &fn, double &compile_ms,
            uint64_t &id)
{
    compile_ms = 0.0;
    const std::string key = std::to_string(D.id) + (grad ? " grad " : " fwd ") + std::to_string(sh.waves) +
                            (sh.super_restart ? "s" : "") + (sh.keep_bottom ? (sh.bottom_lds ? "K" : "k") : "") + "/" +
                            std::to_string(sh.simd_waves) + " " + P.structure;
    {
        std::lock_guard<std::mutex> lk(g_jit_mu);
        auto it = g_jit.find(key);
        if (it != g_jit.end()) {
            fn = it->second.fn;
            id = it->second.id;
            return BAT_OK;
        }
    }
    return jit_load(D, key, jit_source(P, grad, sh), grad ? "bat_grad_jit" : "bat_fwd_jit", fn, compile_ms, id);
}

// ------------------------------------------------------------ autotune cache
struct TuneChoice {
    int chunk_log2, check_every, jit, perm, chain = -1, order = -1;
    // specialised forward launch shape (-1: default)
    int waves = -1, super_restart = -1, simd_waves = -1, keep_bottom = -1;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;

// The graph itself (node count, arcs, terminals): what tuned choices are
// remembered under.
std::string graph_key(int32_t n, int32_t m, const bat_arc *arcs, int32_t s, int32_t t, bool directed = false)
{
    std::string k = std::string(directed ? "D" : "") + std::to_string(n) + "/" + std::to_string(s) + "/" +
                    std::to_string(t) + ":";
    for (int32_t i = 0; i < m; ++i) k += std::to_string(arcs[i].u) + "-" + std::to_string(arcs[i].v) + ",";
    return k;
}

// ------------------------------------------------------------ the sweep
struct Request {
    int32_t n, m, s, t;
    const bat_arc *arcs;
    const double *p_dev;    // device probabilities
    u64 c_lo, c_hi;
    bool grad;
    // forced knobs (autotuner); -1 = from options / the tuned choice
    int force_chunk_log2 = -1, force_check = -1, force_jit = -1, force_perm = -1, force_chain = -1,
        force_order = -1, force_waves = -1, force_super = -1, force_simd = -1, force_keep = -1;
    // timing sample (autotuner): sweep only this many work items, spread
    // over the whole counter by an odd multiplier (0 = everything)
    u64 sample_items = 0;
    // a part of the counter, or the first part of a split sweep: work items
    // no larger than fill_item_log2's size
    bool fill = false;
    // one part of a whole sweep split into split_parts (a power of two):
    // part split_index (0 = no split)
    u64 split_parts = 0, split_index = 0;
};

// Options, then the tuned choice for this graph (if any and enabled), then
// what the request forces.
TuneChoice choose(const DeviceInfo &D, const std::string &gkey, bool grad, const Request *rq)
{
    Options &O = opts();
    TuneChoice tc{(int)O.chunk_log2.load(), (int)O.check_every.load(), (int)O.jit.load(), -1};
    if (O.autotune.load()) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(std::to_string(D.id) + (grad ? " grad " : " fwd ") + gkey);
        if (it != g_tune.end()) tc = it->second;
    }
    if (O.perm.load() >= 0) tc.perm = (int)O.perm.load();
    if (O.chain_log2.load() >= 0) tc.chain = (int)O.chain_log2.load();
    if (O.item_order.load() >= 0) tc.order = (int)O.item_order.load();
    if (O.block_waves.load() >= 0) tc.waves = (int)O.block_waves.load();
    if (O.super_restart.load() >= 0) tc.super_restart = (int)O.super_restart.load();
    if (O.simd_waves.load() >= 0) tc.simd_waves = (int)O.simd_waves.load();
    if (O.keep_bottom.load() >= 0) tc.keep_bottom = (int)O.keep_bottom.load();
    if (rq) {
        if (rq->force_chunk_log2 >= 0) tc.chunk_log2 = rq->force_chunk_log2;
        if (rq->force_check >= 0) tc.check_every = rq->force_check;
        if (rq->force_jit >= 0) tc.jit = rq->force_jit;
        if (rq->force_perm >= 0) tc.perm = rq->force_perm;
        if (rq->force_chain >= 0) tc.chain = rq->force_chain;
        if (rq->force_order >= 0) tc.order = rq->force_order;
        if (rq->force_waves >= 0) tc.waves = rq->force_waves;
        if (rq->force_super >= 0) tc.super_restart = rq->force_super;
        if (rq->force_simd >= 0) tc.simd_waves = rq->force_simd;
        if (rq->force_keep >= 0) tc.keep_bottom = rq->force_keep;
    }
    return tc;
}

struct Launch {
    void *ws = nullptr;     // workspace (stream-ordered; null when the thread's scratch is used)
    double *res = nullptr;  // [ncol][2]
    u64 *count = nullptr;
    int *status = nullptr;
    const unsigned char *cb_of_arc = nullptr;
    u32 ncol = 1;
    // the output block res | count | status, contiguous in the workspace,
    // and where its host copy goes in the thread's staging buffer
    const char *out_dev = nullptr;
    size_t out_bytes = 0, out_host_off = 0;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Work-item size (log2 iterations) for `iters` iterations in `parts` launches
// (0 or 1: one): ~256 work items per CU per launch, so that the last,
// partly idle round of items is a small share of a launch, but at most 4096
// and, for one launch where the sweep has that many, at least 32 iterations
// per item (a split sweep needs the items to deal out into its parts).
// Measured: the 36-arc graph (2^25 iterations) 6.3 ms at 512 iterations
// per item against 8.4 ms at 2048 (64 items per CU); the 40-arc grid in 16
// parts 127 ms against 154 ms (one launch: 118 ms); items of 8 iterations
// slowed the 30-arc graph's gradient sweep (2.3 against 1.9 ms at 32).
// min_log2: the smallest item for one launch where the sweep has that many
// iterations (32 for the graph-specialised kernels and for gradients; the
// generic forward kernel on small graphs is faster with items of one
// chained block: on 256 graphs of 16 to 28 arcs, 20.9 ms in all at 8
// iterations per item against 42.3 ms at 32)
int fill_item_log2(u64 iters, int cus, u64 parts, int min_log2 = 5)
{
    const u64 target = iters / ((u64)std::max(cus, 1) * 256ull * std::max<u64>(parts, 1));
    int c = 0;
    while (c < 12 && (2ull << c) <= target) ++c;
    if (parts <= 1)
        while (c < min_log2 && (2ull << c) <= iters) ++c;
    return c;
}

// Queue tables + sweep + reduce on `stream`.  Allocates the workspace with
// hipMallocAsync; the caller frees it on the same stream.
// p_host (synchronous calls) is uploaded with the plan through the thread's
// pinned staging buffer into its reused workspace; otherwise rq.p_dev is
// already on the device and the workspace is allocated on the stream.
// fixed_ws (fixed_cap bytes): a caller-provided device workspace instead of
// an allocation.  The ahead-of-time kernels then run (loading a compiled
// kernel module would take device memory), and work items grow until the
// partials fit; BAT_ETOOBIG when even items of 2^kFixedMaxItemLog2
// iterations do not fit.  Every byte the sweep reads is written first by
// this call's own kernels and copy, so the workspace needs no clearing.
constexpr int kFixedMaxItemLog2 = 24;

int queue_sweep(const Request &rq, const Plan &P, const DeviceInfo &D, const TuneChoice &tc, hipStream_t stream,
                Launch &L, const double *p_host = nullptr, char *fixed_ws = nullptr, size_t fixed_cap = 0)
{
    const u32 m = (u32)rq.m;
    const u32 ubits = m > (u32)bat::kWordBits ? m - bat::kWordBits : 0u;
    const u64 g_first = rq.c_lo >> bat::kWordBits;
    const u64 g_last = (rq.c_hi - 1) >> bat::kWordBits;
    Options &O = opts();
    // pick the kernel
    bool use_jit = false;
    if (tc.jit == 1) use_jit = true;
    else if (tc.jit == 2) use_jit = (rq.c_hi - rq.c_lo) >= (1ull << 32) || (P.N > 32 && (rq.c_hi - rq.c_lo) >= (1ull << 22));
    if (fixed_ws) use_jit = false;
    // warm-started chains need >= k iteration bits; k = 3..6 (the gradient
    // sweep keeps at most 4 fast bits: k <= 4)
    u32 ck = tc.chain < 0 ? 3u : (tc.chain >= 6 ? 6u : (tc.chain >= 3 ? (u32)tc.chain : 0u));
    if (rq.grad && ck > (u32)bat::kGradFastMax) ck = bat::kGradFastMax;
    if (ubits < ck) ck = ubits >= 3 ? 3u : 0u;
    const bool chain = ck > 0 && !P.ru.empty();
    const u64 bmask = chain ? (1ull << ck) - 1ull : 0ull;
    const u64 g_base = g_first & ~bmask;
    const u64 g_end = g_last | bmask;
    const u64 iters = g_end - g_base + 1;

    const int clog_fill = fill_item_log2(iters, D.cus, rq.split_parts, use_jit || rq.grad ? 5 : 0);
    int clog = tc.chunk_log2;
    // a size tuned for the whole counter would leave a short range's last
    // round of work items mostly idle
    if (clog <= 0 || (rq.fill && clog > clog_fill)) clog = clog_fill;
    clog = std::min(clog, 20);
    if (chain) clog = std::max(clog, (int)ck);
    u32 f = (u32)std::max<int64_t>(0, std::min<int64_t>(O.seg_log2.load(), bat::kMaxSegLog));
    if (rq.grad) f = std::min<u32>(f, bat::kGradFastMax);
    if (chain) f = std::max<u32>(f, ck);
    if (f > ubits) f = ubits;
    const u32 ncol = rq.grad ? 1u + 2u * m : 1u;
    // workspace: input block (p | row, cb_of_arc maps | relaxation program),
    // then tables | partials | counts | output block (res | count | status)
    auto in_size = [&]() {
        size_t o = 0;
        if (p_host) o = align_up(o + sizeof(double) * (m + 1), 256);
        o = align_up(o + 128, 256);
        return align_up(o + sizeof(u32) * (P.prog.size() + 1), 256);
    };
    auto ws_size = [&](u64 n_chunks) {
        size_t o = in_size();
        o = align_up(o + sizeof(double) * bat::kTables, 256);
        o = align_up(o + sizeof(double) * 2 * ncol * n_chunks, 256);
        o = align_up(o + sizeof(u64) * n_chunks, 256);
        return align_up(o + sizeof(double) * 2 * ncol + sizeof(u64) + 64, 256);
    };
    if (fixed_ws) {
        if (rq.split_parts || rq.sample_items) return fail(BAT_EINVAL, "a fixed workspace sweeps whole ranges only");
        while (ws_size((iters + (1ull << clog) - 1) >> clog) > fixed_cap) {
            if (clog >= kFixedMaxItemLog2)
                return fail(BAT_ETOOBIG,
                            "%llu iterations need %zu bytes of fixed scratch even in work items of 2^%d "
                            "iterations; it holds %zu",
                            (unsigned long long)iters, ws_size((iters + (1ull << clog) - 1) >> clog), clog,
                            fixed_cap);
            ++clog;
        }
    }

    bat::KParams K;
    memset(&K, 0, sizeof K);
    K.c_lo = rq.c_lo;
    K.c_hi = rq.c_hi;
    K.g_first = g_first;
    K.g_last = g_last;
    K.g_base = g_base;
    K.g_end = g_end;
    K.chunk_iters = 1ull << clog;
    K.n_chunks = (iters + K.chunk_iters - 1) >> clog;
    K.chunk_mul = 1;
    K.chunk_mask = ~0ull;
    const bool pow2 = (K.n_chunks & (K.n_chunks - 1)) == 0;
    const bool sample = rq.sample_items && rq.sample_items < K.n_chunks && pow2;
    if (pow2 && (sample || tc.order != 0)) {
        // work item -> chunk through an odd multiplier: a bijection modulo
        // n_chunks that spreads consecutive items over the whole counter
        K.chunk_mul = 0x9E3779B97F4A7C15ull;
        K.chunk_mask = K.n_chunks - 1;
        if (sample) K.n_chunks = rq.sample_items;
    }
    if (rq.split_parts) {
        // Part j of J: the work items whose blocks are j modulo J, visited
        // in spread order (item i sweeps block j + J ((i M) mod S), S = N / J
        // items per part), so every part samples the whole counter the way
        // a whole sweep does.  min(J, N) parts.
        const u64 N = K.n_chunks;
        if (!pow2 || sample || (rq.split_parts & (rq.split_parts - 1)))
            return fail(BAT_EINVAL, "cannot split %llu work items into %llu parts", (unsigned long long)N,
                        (unsigned long long)rq.split_parts);
        const u64 parts = std::min<u64>(rq.split_parts, N);
        if (rq.split_index >= parts)
            return fail(BAT_EINVAL, "part %llu of %llu", (unsigned long long)rq.split_index, (unsigned long long)parts);
        K.g_base = g_base + rq.split_index * K.chunk_iters;
        K.chunk_mul = 0x9E3779B97F4A7C15ull * parts;
        K.chunk_mask = N - 1;
        K.n_chunks = N / parts;
    }
    K.m = m;
    K.ubits = ubits;
    K.seg_log = f;
    K.check_every = tc.check_every >= 2 ? 2u : 1u;
    K.chain = chain ? ck : 0u;
    K.ncol = ncol;
    K.window_test = (chain && O.window_test.load() != 0) ? 1u : 0u;
    K.n_nodes = (u32)P.N;
    K.s = (u32)P.S;
    K.t = (u32)P.T;
    K.n_relax = (u32)P.code.size();
    K.n_groups = (u32)((P.prog.size() - 8) / 16);
    chain_codes(P, K.ck_code);
    L.ncol = K.ncol;

    size_t off = 0;
    const size_t o_p = off;
    if (p_host) off = align_up(off + sizeof(double) * (m + 1), 256);
    const size_t o_map = off;  // row[64] | cb_of_arc[64]
    off = align_up(off + 128, 256);
    const size_t o_rl = off;
    off = align_up(off + sizeof(u32) * (P.prog.size() + 1), 256);
    const size_t in_bytes = off;
    const size_t o_tab = off;
    off = align_up(off + sizeof(double) * bat::kTables, 256);
    const size_t o_part = off;
    off = align_up(off + sizeof(double) * 2 * K.ncol * K.n_chunks, 256);
    const size_t o_pc = off;
    off = align_up(off + sizeof(u64) * K.n_chunks, 256);
    const size_t o_res = off;
    const size_t o_cnt = o_res + sizeof(double) * 2 * K.ncol;
    const size_t o_st = o_cnt + sizeof(u64);
    const size_t out_bytes = o_st + sizeof(int) - o_res;
    off = align_up(o_st + 64, 256);
    char *ws = nullptr;
    Scratch *S = nullptr;
    const size_t out_host_off = align_up(in_bytes, 256);
    if (in_bytes != in_size() || off != ws_size(K.n_chunks))
        return fail(BAT_EDEVICE, "workspace layout mismatch (%zu/%zu, %zu/%zu)", in_bytes, in_size(), off,
                    ws_size(K.n_chunks));
    if (fixed_ws) {
        if (off > fixed_cap) return fail(BAT_ETOOBIG, "needs %zu bytes of fixed scratch; it holds %zu", off, fixed_cap);
        ws = fixed_ws;
    } else if (p_host) {
        int rc = scratch_reserve(D.id, stream, off, out_host_off + out_bytes, S);
        if (rc) return rc;
        ws = S->dev;
    } else {
        HIPCHK(hipMallocAsync((void **)&ws, off, stream));
        L.ws = ws;
    }
    K.tables = (const double *)(ws + o_tab);
    K.status = (const int *)(ws + o_st);
    K.prog = (const u32 *)(ws + o_rl);
    K.part = (double *)(ws + o_part);
    K.pcount = (u64 *)(ws + o_pc);
    L.res = (double *)(ws + o_res);
    L.count = (u64 *)(ws + o_cnt);
    L.status = (int *)(ws + o_st);
    L.out_dev = ws + o_res;
    L.out_bytes = out_bytes;
    L.out_host_off = out_host_off;
    // the input block, built once on the host and copied in one piece
    std::vector<char> local;
    char *in = nullptr;
    if (S) {
        in = S->host;
    } else {
        local.assign(in_bytes, 0);
        in = local.data();
    }
    if (p_host && m > 0) memcpy(in + o_p, p_host, sizeof(double) * m);
    unsigned char *maps = (unsigned char *)(in + o_map);
    memset(maps, 0, 128);
    for (int i = 0; i < P.m; ++i) {
        maps[i] = P.row[i];
        maps[64 + i] = (unsigned char)P.cb_of_arc[i];
    }
    if (!P.prog.empty()) memcpy(in + o_rl, P.prog.data(), sizeof(u32) * P.prog.size());
    HIPCHK(hipMemcpyAsync(ws, in, in_bytes, hipMemcpyHostToDevice, stream));
    // (a copy from pageable memory has read its source when the call returns)
    const double *p_dev = p_host ? (const double *)(ws + o_p) : rq.p_dev;
    const bool identity = P.identity;
    const unsigned char *d_row = identity ? nullptr : (const unsigned char *)(ws + o_map);
    L.cb_of_arc = identity ? nullptr : (const unsigned char *)(ws + o_map + 64);

    hipFunction_t jfn = nullptr;
    double jit_ms = 0.0;
    uint64_t kernel_id = 0;
    const JitShape shape = jit_shape(rq.grad, tc.waves, tc.super_restart, tc.simd_waves, tc.keep_bottom);
    if (use_jit) {
        int rc = jit_get(D, P, rq.grad, shape, jfn, jit_ms, kernel_id);
        if (rc) return rc;
    } else {
        kernel_id = aot_kernel_id(rq.grad ? "k_grad_dyn" : "k_fwd_dyn", (int)P.N, P.directed);
    }

    int rc = events_ready();
    if (rc) return rc;
    HIPCHK(hipEventRecord(t_state.ev[0], stream));
    HIPCHK(batk::build_tables(stream, p_dev, d_row, m, f, (double *)K.tables, (int *)K.status));
    HIPCHK(hipEventRecord(t_state.ev[1], stream));
    // one work item per wavefront
    const u64 wpb = use_jit ? (u64)shape.waves : (u64)bat::kWavesPerBlock;
    const u64 blocks = (K.n_chunks + wpb - 1) / wpb;
    if (blocks > 0x7fffffffull) return fail(BAT_ETOOBIG, "too many work items (%llu)", (unsigned long long)blocks);
    if (use_jit) {
        void *args[] = {&K};
        HIPCHK(hipModuleLaunchKernel(jfn, (unsigned)blocks, 1, 1, (unsigned)(bat::kWave * wpb), 1, 1, 0, stream, args,
                                     nullptr));
    } else {
        HIPCHK(batk::sweep_dyn(stream, (unsigned)blocks, rq.grad, P.N, P.directed, K));
    }
    HIPCHK(hipEventRecord(t_state.ev[2], stream));
    HIPCHK(batk::reduce(stream, (const double *)K.part, (const u64 *)K.pcount, K.n_chunks, K.ncol, L.res, L.count));
    HIPCHK(hipEventRecord(t_state.ev[3], stream));

    bat_launch_info &I = t_state.info;
    memset(&I, 0, sizeof I);
    I.jit_ms = jit_ms;
    I.vectors = std::min<u64>(rq.c_hi - rq.c_lo, K.n_chunks * K.chunk_iters << bat::kWordBits);
    I.specialised = use_jit ? 1 : 0;
    I.chunk_log2 = clog;
    I.n_chunks = (int32_t)std::min<u64>(K.n_chunks, 0x7fffffff);
    I.relaxations = (int32_t)(use_jit ? P.jru.size() : P.code.size());
    I.kernel_id = kernel_id;
    I.perm = P.perm;
    I.chain_log2 = (int32_t)K.chain;
    I.check_every = (int32_t)K.check_every;
    I.item_order = K.chunk_mul != 1 ? 1 : 0;
    I.block_waves = (int32_t)wpb;
    I.keep_bottom =
        (use_jit && shape.keep_bottom && P.jN <= bat::kKeepBottomMaxNodes) ? (shape.bottom_lds ? 2 : 1) : 0;
    I.super_restart = (I.keep_bottom && shape.super_restart && P.jN <= kSuperMaxNodes) ? 1 : 0;
    I.window_test = use_jit ? (int32_t)K.window_test : 0;
    I.simd_waves = (use_jit && !(rq.grad && P.jN > kGradThreeWaveNodes)) ? shape.simd_waves : 0;
    t_state.have_launch = true;
    return BAT_OK;
}

struct Prepared {
    DeviceInfo D;
    Plan P;
    hipStream_t stream = nullptr;
};

// Validate, pick the launch choices and plan.  full_range: the whole
// counter, where any arc order may be used; otherwise the paper's order.
int prepare(int32_t n, int32_t m, const bat_arc *arcs, const double *p_host, int32_t s, int32_t t, bool grad,
            bool full_range, const Request *forced, Prepared &X, TuneChoice &tc, uint32_t flags = 0)
{
    int rc = validate(n, m, arcs, p_host, s, t);
    if (rc) return rc;
    rc = current_device(X.D);
    if (rc) return rc;
    const bool directed = (flags & BAT_DIRECTED) != 0;
    tc = choose(X.D, graph_key(n, m, arcs, s, t, directed), grad, forced);
    const bool forward = forced && forced->force_perm == kPermForward;
    if (!forward && (tc.perm < 0 || tc.perm >= kPermKinds)) tc.perm = kDefaultPerm;
    if (!full_range && !forward) tc.perm = 0;
    make_plan(n, m, arcs, s, t, X.P, tc.perm, directed);
    return BAT_OK;
}

// Synchronous driver over host p; fills res (ncol double-double pairs),
// count and the plan's arc -> counter bit map (for the gradient columns).
int run_sync(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t, u64 c_lo,
             u64 c_hi, bool grad, std::vector<double> &res, u64 &count, Request *tmpl = nullptr,
             std::vector<int> *cb_of_arc = nullptr, uint32_t flags = 0)
{
    Prepared X;
    TuneChoice tc;
    const bool full = c_lo == 0 && c_hi == (1ull << m);
    if (!p && m > 0) return fail(BAT_EINVAL, "p is NULL");
    // any arc order for a whole sweep; a partial range is in the paper's
    // order unless the caller (the autotuner timing a sample) forces one
    const bool allow_perm = full || (tmpl && tmpl->force_perm >= 0);
    int rc = prepare(n, m, arcs, p, s, t, grad, allow_perm, tmpl, X, tc, flags);
    if (rc) return rc;
    rc = thread_stream(X.D.id, X.stream);
    if (rc) return rc;
    Request rq = tmpl ? *tmpl : Request{};
    rq.n = n; rq.m = m; rq.s = s; rq.t = t; rq.arcs = arcs; rq.p_dev = nullptr;
    rq.c_lo = c_lo; rq.c_hi = c_hi; rq.grad = grad;
    Launch L;
    static const double kNoArcs = 0.0;
    rc = queue_sweep(rq, X.P, X.D, tc, X.stream, L, m > 0 ? p : &kNoArcs);
    if (rc) {
        (void)hipStreamSynchronize(X.stream);
        return rc;
    }
    // one copy back: res | count | status, into the pinned staging buffer
    Scratch &S = t_state.scratch[X.D.id];
    char *out = S.host + L.out_host_off;
    HIPCHK(hipMemcpyAsync(out, L.out_dev, L.out_bytes, hipMemcpyDeviceToHost, X.stream));
    HIPCHK(hipStreamSynchronize(X.stream));
    res.assign(2 * L.ncol, 0.0);
    memcpy(res.data(), out, sizeof(double) * 2 * L.ncol);
    memcpy(&count, out + sizeof(double) * 2 * L.ncol, sizeof(u64));
    int st = 0;
    memcpy(&st, out + sizeof(double) * 2 * L.ncol + sizeof(u64), sizeof(int));
    if (st) return fail(BAT_EINVAL, "a probability is outside [0,1]");
    if (cb_of_arc) *cb_of_arc = X.P.cb_of_arc;
    return BAT_OK;
}

void split_grad(const std::vector<double> &res, const std::vector<int> &cb_of_arc, int32_t m, double *dRdp,
                double *T1, double *T0)
{
    for (int32_t a = 0; a < m; ++a) {
        int cb = cb_of_arc[a];
        const double *t0 = &res[2 * (1 + 2 * cb)], *t1 = &res[2 * (1 + 2 * cb + 1)];
        if (dRdp) dRdp[a] = (t1[0] - t0[0]) + (t1[1] - t0[1]);
        if (T1) T1[a] = t1[0] + t1[1];
        if (T0) T0[a] = t0[0] + t0[1];
    }
}

// Partial sums over [c_lo, c_hi) of the counter whose bits follow arc-to-bit
// order kind `perm` (0: the paper's backward BAT indices, kPermForward: its
// forward ones); arguments already validated except the probabilities.
int range_in_order(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                   uint32_t flags, int perm, u64 c_lo, u64 c_hi, double *R_hi, double *R_lo, uint64_t *count_out,
                   double *T1_out, double *T0_out)
{
    const bool grad = T1_out != nullptr;
    if (c_lo == c_hi) {
        int rc = validate(n, m, arcs, p, s, t);
        if (rc) return rc;
        *R_hi = *R_lo = 0.0;
        *count_out = 0;
        if (grad)
            for (int32_t a = 0; a < m; ++a) T1_out[a] = T0_out[a] = 0.0;
        return BAT_OK;
    }
    std::vector<double> res;
    std::vector<int> cba;
    u64 cnt = 0;
    Request order{};
    order.force_perm = perm;
    order.fill = true;
    int rc = run_sync(n, m, arcs, p, s, t, c_lo, c_hi, grad, res, cnt, &order, &cba, flags);
    if (rc) return rc;
    *R_hi = res[0];
    *R_lo = res[1];
    *count_out = cnt;
    if (grad) split_grad(res, cba, m, nullptr, T1_out, T0_out);
    return BAT_OK;
}

// The arc-to-bit order a whole sweep of this graph would take (tuned or
// default); the forward BAT order when the flags ask for it.
int whole_sweep_order(int32_t n, int32_t m, const bat_arc *arcs, int32_t s, int32_t t, uint32_t flags, bool grad,
                      int &perm)
{
    if (flags & BAT_FORWARD_ORDER) {
        perm = kPermForward;
        return BAT_OK;
    }
    DeviceInfo D;
    int rc = current_device(D);
    if (rc) return rc;
    const TuneChoice tc = choose(D, graph_key(n, m, arcs, s, t, (flags & BAT_DIRECTED) != 0), grad, nullptr);
    perm = tc.perm >= 0 && tc.perm < kPermKinds ? tc.perm : kDefaultPerm;
    return BAT_OK;
}

// ------------------------------------------------------------ checkpoints
// A chunked sweep's running sums: R and the per-arc T1 / T0 as unevaluated
// double-doubles (hi, lo), the count exactly.
struct RunningSums {
    // the launch every chunk repeats (-1: no chunk run yet): arc-to-bit
    // order kind, work-item size (log2 iterations), chain length
    int order = -1, items = -1, chain = -1;
    u64 parts = 0;  // chunks: parts of the whole sweep's work items
    u64 done = 0;
    u64 count = 0;
    double R[2] = {0.0, 0.0};
    std::vector<double> T1, T0;  // 2 m each (hi, lo per arc) when kept
};

// hi + lo += x_hi + x_lo (Knuth's two-sum on the high parts)
void dd_acc(double *d, double x_hi, double x_lo)
{
    const double s = d[0] + x_hi;
    const double bb = s - d[0];
    const double e = (d[0] - (s - bb)) + (x_hi - bb);
    const double lo = e + d[1] + x_lo;
    d[0] = s + lo;
    d[1] = lo - (d[0] - s);
}

uint64_t fnv_bytes(uint64_t h, const void *data, size_t len)
{
    const unsigned char *b = (const unsigned char *)data;
    for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;  // FNV-1a
    return h;
}

// The line that names the problem a checkpoint file belongs to.
std::string checkpoint_problem(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                               uint32_t flags, int32_t clog, bool grad)
{
    uint64_t ha = fnv_bytes(1469598103934665603ull, arcs, sizeof(bat_arc) * (size_t)m);
    uint64_t hp = fnv_bytes(1469598103934665603ull, p, sizeof(double) * (size_t)m);
    char buf[256];
    snprintf(buf, sizeof buf, "problem n=%d m=%d s=%d t=%d flags=%u chunk_log2=%d grad=%d arcs=%016llx p=%016llx",
             n, m, s, t, flags, clog, grad ? 1 : 0, (unsigned long long)ha, (unsigned long long)hp);
    return buf;
}

const char *kCheckpointMagic = "bat-checkpoint 1";

// Reads `path` into S.  1: no such file (a fresh start), 0: read, < 0: error.
int checkpoint_read(const char *path, const std::string &problem, bool grad, int32_t m, uint32_t flags,
                    RunningSums &S)
{
    FILE *f = fopen(path, "r");
    if (!f) {
        if (errno == ENOENT) return 1;
        return fail(BAT_EIO, "checkpoint %s: cannot open (%s)", path, strerror(errno));
    }
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    const bool bad_read = ferror(f) != 0;
    fclose(f);
    if (bad_read) return fail(BAT_EIO, "checkpoint %s: read error", path);
    std::vector<std::string> lines;
    for (size_t a = 0, b; a < text.size(); a = b + 1) {
        b = text.find('\n', a);
        if (b == std::string::npos) b = text.size();
        lines.push_back(text.substr(a, b - a));
    }
    if (lines.size() < 2 || lines[0] != kCheckpointMagic)
        return fail(BAT_EIO, "checkpoint %s: not a checkpoint file", path);
    if (lines[1] != problem)
        return fail(BAT_EINVAL, "checkpoint %s belongs to another problem (%s; this call: %s)", path,
                    lines[1].c_str(), problem.c_str());
    if (lines.size() < (grad ? 9u : 7u)) return fail(BAT_EIO, "checkpoint %s: truncated", path);
    unsigned long long parts = 0, done = 0, cnt = 0;
    int order = -1, items = -1, chain = -1;
    char tail;
    if (sscanf(lines[2].c_str(), "parts %llu %c", &parts, &tail) != 1 ||
        sscanf(lines[3].c_str(), "launch order=%d items=%d chain=%d %c", &order, &items, &chain, &tail) != 3 ||
        sscanf(lines[4].c_str(), "done %llu %c", &done, &tail) != 1 ||
        sscanf(lines[5].c_str(), "count %llu %c", &cnt, &tail) != 1)
        return fail(BAT_EIO, "checkpoint %s: malformed header", path);
    const int ubits = m > bat::kWordBits ? m - bat::kWordBits : 0;
    const bool fwd = (flags & BAT_FORWARD_ORDER) != 0;
    if (fwd ? order != kPermForward : (order < 0 || order >= kPermKinds))
        return fail(BAT_EIO, "checkpoint %s: bad arc order %d", path, order);
    if (items < 0 || items > 20 || (chain != 0 && (chain < 3 || chain > 6)) || parts == 0 ||
        (parts & (parts - 1)) != 0 || parts > (1ull << std::max(ubits - items, 0)) || done > parts)
        return fail(BAT_EIO, "checkpoint %s: bad launch or part counts", path);
    // "<tag> hi lo [hi lo ...]" with hexadecimal floats (exact round trip)
    auto doubles = [&](const std::string &ln, const char *tag, size_t want, double *out) {
        const size_t tl = strlen(tag);
        if (ln.compare(0, tl, tag) != 0) return false;
        const char *q = ln.c_str() + tl;
        for (size_t i = 0; i < want; ++i) {
            char *e = nullptr;
            out[i] = strtod(q, &e);
            if (e == q || !std::isfinite(out[i])) return false;
            q = e;
        }
        while (*q == ' ') ++q;
        return *q == '\0';
    };
    RunningSums R;
    R.order = order;
    R.items = items;
    R.chain = chain;
    R.parts = parts;
    R.done = done;
    R.count = cnt;
    if (!doubles(lines[6], "R", 2, R.R)) return fail(BAT_EIO, "checkpoint %s: malformed R line", path);
    if (grad) {
        R.T1.assign(2 * (size_t)m, 0.0);
        R.T0.assign(2 * (size_t)m, 0.0);
        if (!doubles(lines[7], "T1", 2 * (size_t)m, R.T1.data()) || !doubles(lines[8], "T0", 2 * (size_t)m, R.T0.data()))
            return fail(BAT_EIO, "checkpoint %s: malformed T1/T0 lines", path);
    }
    S = std::move(R);
    return 0;
}

// Writes S to path + ".tmp", then renames it over `path`, so a reader sees
// either the old file or the new one whole.
int checkpoint_write(const char *path, const std::string &problem, bool grad, const RunningSums &S)
{
    std::string text = std::string(kCheckpointMagic) + "\n" + problem + "\n";
    char buf[128];
    snprintf(buf, sizeof buf, "parts %llu\nlaunch order=%d items=%d chain=%d\ndone %llu\ncount %llu\nR %a %a\n",
             (unsigned long long)S.parts, S.order, S.items, S.chain, (unsigned long long)S.done,
             (unsigned long long)S.count, S.R[0], S.R[1]);
    text += buf;
    if (grad) {
        for (int w = 0; w < 2; ++w) {
            const std::vector<double> &v = w ? S.T0 : S.T1;
            text += w ? "T0" : "T1";
            for (double x : v) {
                snprintf(buf, sizeof buf, " %a", x);
                text += buf;
            }
            text += "\n";
        }
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(BAT_EIO, "checkpoint %s: cannot create (%s)", tmp.c_str(), strerror(errno));
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size() && fflush(f) == 0 && fsync(fileno(f)) == 0;
    if (fclose(f) != 0 || !ok) {
        unlink(tmp.c_str());
        return fail(BAT_EIO, "checkpoint %s: write failed", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        unlink(tmp.c_str());
        return fail(BAT_EIO, "checkpoint %s: rename failed (%s)", path, strerror(errno));
    }
    return BAT_OK;
}

// Chunk S.done of a checkpointed sweep: one part of the whole sweep's work
// items (queue_sweep's split), under the launch the first chunk took: its
// arc order, work-item size and chain length fix which blocks each part
// holds and how its sums are rounded.
int run_part(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t, uint32_t flags,
             bool grad, u64 parts_wanted, RunningSums &S, double *R_hl, uint64_t *count, double *T1, double *T0)
{
    Request rq{};
    const bool first = S.order < 0;
    if (first) {
        int rc = whole_sweep_order(n, m, arcs, s, t, flags, grad, rq.force_perm);
        if (rc) return rc;
        rq.split_parts = parts_wanted;
        rq.fill = true;
    } else {
        rq.force_perm = S.order;
        rq.force_chunk_log2 = S.items;
        rq.force_chain = S.chain;
        rq.split_parts = S.parts;
    }
    rq.split_index = S.done;
    std::vector<double> res;
    std::vector<int> cba;
    u64 cnt = 0;
    int rc = run_sync(n, m, arcs, p, s, t, 0, 1ull << m, grad, res, cnt, &rq, &cba, flags);
    if (rc) return rc;
    if (first) {
        const bat_launch_info &I = t_state.info;
        const int ubits = m > bat::kWordBits ? m - bat::kWordBits : 0;
        S.order = I.perm;
        S.items = I.chunk_log2;
        S.chain = I.chain_log2;
        S.parts = std::min<u64>(parts_wanted, 1ull << std::max(ubits - S.items, 0));
    }
    R_hl[0] = res[0];
    R_hl[1] = res[1];
    *count = cnt;
    if (grad) split_grad(res, cba, m, nullptr, T1, T0);
    return BAT_OK;
}

}  // namespace

namespace {

// ------------------------------------------------------------ multi-state
// Arcs with sigma_i states (bat_ms.hip): validate, order the arcs for the
// flow searches, and sweep [c_lo, c_hi) of the mixed-radix counter.
int ms_validate(int32_t n, int32_t m, const bat_arc *arcs, const int32_t *sigma, const int32_t *cap, const double *w,
                int32_t s, int32_t t, int32_t d, uint32_t flags, u64 &N, int32_t &n_table)
{
    if (flags & ~(uint32_t)BAT_DIRECTED) return fail(BAT_EINVAL, "unknown flags 0x%x", flags);
    if (n < 2 || m < 0) return fail(BAT_EINVAL, "need n_nodes >= 2 and n_arcs >= 0 (got %d, %d)", n, m);
    if (n > batk::kMsMaxNodes || m > batk::kMsMaxArcs)
        return fail(BAT_ETOOBIG, "multi-state arcs: at most %d nodes and %d arcs (got %d, %d)", batk::kMsMaxNodes,
                    batk::kMsMaxArcs, n, m);
    if (s < 0 || s >= n || t < 0 || t >= n || s == t) return fail(BAT_EINVAL, "bad terminals s=%d t=%d", s, t);
    if (d < 1 || d > batk::kMsMaxDemand) return fail(BAT_EINVAL, "demand %d outside [1, %d]", d, batk::kMsMaxDemand);
    if (m > 0 && (!arcs || !sigma || !w)) return fail(BAT_EINVAL, "NULL arcs, n_states or probabilities");
    N = 1;
    n_table = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (arcs[i].u < 0 || arcs[i].u >= n || arcs[i].v < 0 || arcs[i].v >= n)
            return fail(BAT_EINVAL, "arc %d has a node outside [0, %d)", i, n);
        if (sigma[i] < 1 || sigma[i] > batk::kMsMaxStates)
            return fail(BAT_EINVAL, "arc %d has %d states, outside [1, %d]", i, sigma[i], batk::kMsMaxStates);
        for (int32_t k = 0; k < sigma[i]; ++k) {
            const double x = w[n_table + k];
            if (!(x >= 0.0 && x <= 1.0)) return fail(BAT_EINVAL, "probability of arc %d state %d is %g", i, k, x);
            if (cap && (cap[n_table + k] < 0 || cap[n_table + k] > batk::kMsMaxCapacity))
                return fail(BAT_EINVAL, "capacity of arc %d state %d outside [0, %d]", i, k, batk::kMsMaxCapacity);
        }
        n_table += sigma[i];
        if (n_table > batk::kMsMaxTable)
            return fail(BAT_ETOOBIG, "more than %d (arc, state) pairs", batk::kMsMaxTable);
        if ((u64)sigma[i] > (1ull << 62) / N) return fail(BAT_ETOOBIG, "more than 2^62 state vectors");
        N *= (u64)sigma[i];
    }
    return BAT_OK;
}

// Demand <= 3: the bit-sliced kernel (ms_bits_kernel in bat_device.hpp)
// compiled for the graph and its states, over the vector indices
// [c_lo, c_hi) (slot 0 least significant).  Slots in sweep order: slot j
// joins su[j] and sv[j] and has sig[j] states whose capacities and
// probabilities are capt / wt at off[j].
int ms_bits_run(int32_t n, int32_t m, const int *su, const int *sv, const bat::u32 *sig, const bat::u32 *off,
                const std::vector<int32_t> &capt, const std::vector<double> &wt, int32_t s, int32_t t, int32_t d,
                bool directed, u64 c_lo, u64 c_hi, double &R_hi, double &R_lo, u64 &count, std::string *src_only)
{
    // word slots: the longest prefix whose states fit the 32 bits of a word
    int kw = 0;
    u64 B = 1;
    while (kw < m && B * sig[kw] <= 32) B *= sig[kw++];
    // the words the range touches
    const u64 w_lo = c_lo / B, w_hi = c_hi > c_lo ? (c_hi + B - 1) / B : w_lo;
    // run slots: as many as keep about 2^19 lane runs (32 wavefronts per
    // CU: the kernel is latency-bound; on the 3^18 workload runs of 27
    // steps took 0.94 ms, of 81 steps 1.15 ms, of 9 steps 1.09 ms) and a
    // run within 2^31 steps (option BAT_MS_RUN > 0: runs of at most that
    // many steps)
    const u64 want_run =
        opts().ms_run.load() > 0 ? (u64)opts().ms_run.load() : std::max<u64>(1, (w_hi - w_lo) >> 19);
    int kr = 0;
    u64 run = 1;
    while (kw + kr < m && run * sig[kw + kr] <= std::min<u64>(want_run, 1ull << 31)) run *= sig[kw + kr++];
    const u64 rl_lo = w_lo / run, rl_hi = (w_hi + run - 1) / run;
    const u64 n_lane = rl_hi - rl_lo;
    const u64 n_items = (n_lane + bat::kWave - 1) / bat::kWave;
    const u64 blocks = (n_items + bat::kWavesPerBlock - 1) / bat::kWavesPerBlock;
    if (blocks > 0x7fffffffull) return fail(BAT_ETOOBIG, "too many work items (%llu)", (unsigned long long)n_items);
    auto capof = [&](int j, u32 x) { return capt[off[j] + x]; };
    // the kernel's constants
    std::vector<u32> c1(m, 0u), ce1(m, 0u), ce12(m, 0u), ww1(m, 0u), wu1(m, 0u), wu12(m, 0u);
    u32 upair = 0u;
    for (int j = 0; j < m; ++j)
        for (u32 x = 0; x < sig[j]; ++x) {
            if (capof(j, x) >= 1) c1[j] |= 1u << x;
            if (capof(j, x) == 1) ce1[j] |= 1u << x;
            if (capof(j, x) == 1 || capof(j, x) == 2) ce12[j] |= 1u << x;
        }
    for (int j = 0; j < m; ++j)
        if (ce1[j]) upair |= 1u << j;
    u64 stride = 1;
    for (int j = 0; j < kw; ++j) {
        for (u64 b = 0; b < B; ++b) {
            const u32 x = (u32)((b / stride) % sig[j]);
            if (capof(j, x) >= 1) ww1[j] |= 1u << b;
            if (capof(j, x) == 1) wu1[j] |= 1u << b;
            if (capof(j, x) == 1 || capof(j, x) == 2) wu12[j] |= 1u << b;
        }
        stride *= sig[j];
    }
    const u32 full = B == 32 ? ~0u : (u32)((1ull << B) - 1ull);
    std::string g = "\nstruct JitMs {\n";
    auto num = [&](const char *k, u64 v) { g += std::string("  static constexpr unsigned ") + k + " = " + std::to_string(v) + "u;\n"; };
    num("N", (u64)n);
    num("S", (u64)s);
    num("T", (u64)t);
    num("M", (u64)m);
    num("KW", (u64)kw);
    num("KR", (u64)kr);
    num("D", (u64)d);
    num("B", B);
    num("FULL", full);
    num("RUN", run);
    num("UPAIR", upair);
    g += std::string("  static constexpr bool DIR = ") + (directed ? "true" : "false") + ";\n";
    auto arr = [&](const char *k, auto get) {
        g += std::string("  static constexpr unsigned ") + k + "[" + std::to_string(m) + "] = {";
        for (int j = 0; j < m; ++j) g += (j ? "," : "") + std::to_string((u64)get(j)) + "u";
        g += "};\n";
    };
    arr("NU", [&](int j) { return su[j]; });
    arr("NV", [&](int j) { return sv[j]; });
    arr("SIG", [&](int j) { return sig[j]; });
    arr("OFF", [&](int j) { return off[j]; });
    arr("C1", [&](int j) { return c1[j]; });
    arr("CE1", [&](int j) { return ce1[j]; });
    arr("CE12", [&](int j) { return ce12[j]; });
    arr("WW1", [&](int j) { return ww1[j]; });
    arr("WU1", [&](int j) { return wu1[j]; });
    arr("WU12", [&](int j) { return wu12[j]; });
    g += "};\n";
    g += "extern \"C\" __global__ void __launch_bounds__(256) bat_ms_bits(bat::MsBitsParams P) {\n"
         "  __shared__ double tb[4][256];\n"
         "  bat::ms_bits_kernel<JitMs>(P, tb);\n}\n";
    if (src_only) {
        *src_only = std::string(kDeviceSource) + g;
        return BAT_OK;
    }
    DeviceInfo D;
    int rc = current_device(D);
    if (rc) return rc;
    hipFunction_t fn;
    double jit_ms = 0.0;
    uint64_t kid = 0;
    rc = jit_load(D, std::to_string(D.id) + " ms" + g, std::string(kDeviceSource) + g, "bat_ms_bits", fn, jit_ms, kid);
    if (rc) return rc;
    hipStream_t st;
    rc = thread_stream(D.id, st);
    if (rc) return rc;
    // F tables of the word slots: Q_in(b) is the product of the word
    // slots' probabilities in vector b, TB_h[x] the sum of Q_in(8h + i)
    // over the bits i of x
    std::vector<double> qin(32, 0.0), tb(1024, 0.0);
    for (u64 b = 0; b < B; ++b) {
        double q = 1.0;
        u64 r = b;
        for (int j = 0; j < kw; ++j) {
            q *= wt[off[j] + (u32)(r % sig[j])];
            r /= sig[j];
        }
        qin[b] = q;
    }
    for (int h = 0; h < 4; ++h)
        for (int x = 0; x < 256; ++x) {
            double a = 0.0;
            for (int i = 0; i < 8; ++i)
                if ((x >> i) & 1) a += qin[8 * h + i];
            tb[256 * h + x] = a;
        }
    // workspace: input (tb | w) | partials | counts | output (res | count)
    const size_t o_tb = 0;
    const size_t o_w = align_up(o_tb + sizeof(double) * tb.size(), 256);
    const size_t in_bytes = align_up(o_w + sizeof(double) * (wt.size() + 1), 256);
    const u64 items = std::max<u64>(n_items, 1);
    const size_t o_part = in_bytes;
    const size_t o_pc = align_up(o_part + sizeof(double) * 2 * items, 256);
    const size_t o_res = align_up(o_pc + sizeof(u64) * items, 256);
    const size_t o_cnt = o_res + 2 * sizeof(double);
    const size_t out_bytes = o_cnt + sizeof(u64) - o_res;
    const size_t total = align_up(o_cnt + sizeof(u64) + 64, 256);
    Scratch *S = nullptr;
    const size_t out_host_off = in_bytes;
    rc = scratch_reserve(D.id, st, total, out_host_off + out_bytes, S);
    if (rc) return rc;
    char *ws = S->dev;
    memcpy(S->host + o_tb, tb.data(), sizeof(double) * tb.size());
    memcpy(S->host + o_w, wt.data(), sizeof(double) * wt.size());
    HIPCHK(hipMemcpyAsync(ws, S->host, in_bytes, hipMemcpyHostToDevice, st));
    bat::MsBitsParams K;
    memset(&K, 0, sizeof K);
    K.n_lane = n_lane;
    K.rl_base = rl_lo;
    K.c_lo = c_lo;
    K.c_hi = c_hi;
    K.n_items = n_items;
    K.tb = (const double *)(ws + o_tb);
    K.w = (const double *)(ws + o_w);
    K.part = (double *)(ws + o_part);
    K.pcount = (u64 *)(ws + o_pc);
    double *res = (double *)(ws + o_res);
    u64 *cnt = (u64 *)(ws + o_cnt);
    rc = events_ready();
    if (rc) return rc;
    HIPCHK(hipEventRecord(t_state.ev[0], st));
    HIPCHK(hipEventRecord(t_state.ev[1], st));
    void *args[] = {&K};
    if (blocks)
        HIPCHK(hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, (unsigned)(bat::kWave * bat::kWavesPerBlock), 1, 1, 0,
                                     st, args, nullptr));
    HIPCHK(hipEventRecord(t_state.ev[2], st));
    HIPCHK(batk::reduce(st, (const double *)K.part, (const u64 *)K.pcount, n_items, 1, res, cnt));
    HIPCHK(hipEventRecord(t_state.ev[3], st));
    char *out = S->host + out_host_off;
    HIPCHK(hipMemcpyAsync(out, ws + o_res, out_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bat_launch_info &I = t_state.info;
    memset(&I, 0, sizeof I);
    I.vectors = c_hi - c_lo;
    I.n_chunks = (int32_t)std::min<u64>(n_items, 0x7fffffff);
    I.chunk_log2 = -1;
    I.relaxations = m;
    I.specialised = 1;
    I.jit_ms = jit_ms;
    I.kernel_id = kid;
    I.block_waves = bat::kWavesPerBlock;
    t_state.have_launch = true;
    memcpy(&R_hi, out, sizeof(double));
    memcpy(&R_lo, out + sizeof(double), sizeof(double));
    memcpy(&count, out + 2 * sizeof(double), sizeof(u64));
    return BAT_OK;
}

int ms_run(int32_t n, int32_t m, const bat_arc *arcs, const int32_t *sigma, const int32_t *cap, const double *w,
           int32_t s, int32_t t, int32_t d, uint32_t flags, bool whole, u64 c_lo, u64 c_hi, double &R_hi,
           double &R_lo, u64 &count, std::string *src_only = nullptr)
{
    u64 N = 0;
    int32_t n_table = 0;
    int rc = ms_validate(n, m, arcs, sigma, cap, w, s, t, d, flags, N, n_table);
    if (rc) return rc;
    if (whole) {
        c_lo = 0;
        c_hi = N;
    }
    if (c_lo > c_hi || c_hi > N)
        return fail(BAT_EINVAL, "range [%llu, %llu) outside [0, %llu)", (unsigned long long)c_lo,
                    (unsigned long long)c_hi, (unsigned long long)N);
    // Slots: the kernel sweeps arcs in slot order, and slot 0 is the
    // fastest-changing coordinate of its index.  A whole space may take any
    // arc order (R and the count are sums over every vector): arcs near s
    // first, by breadth-first distance of their nearer end, so one search
    // sweep reaches far.  A range reads its indices in the caller's order,
    // arc 0 most significant: slot j is arc m - 1 - j.
    std::vector<int> ord(m);
    for (int i = 0; i < m; ++i) ord[i] = whole ? i : m - 1 - i;
    if (whole && m > 1) {
        std::vector<int> dist(n, 1 << 30);
        std::vector<int> q{s};
        dist[s] = 0;
        for (size_t h = 0; h < q.size(); ++h)
            for (int i = 0; i < m; ++i) {
                const int a = arcs[i].u, b = arcs[i].v, x = q[h];
                const int y = a == x ? b : (b == x ? a : -1);
                if (y >= 0 && dist[y] > dist[x] + 1) {
                    dist[y] = dist[x] + 1;
                    q.push_back(y);
                }
            }
        auto key = [&](int i) {
            const int a = dist[arcs[i].u], b = dist[arcs[i].v];
            return std::make_pair(std::min(a, b), std::max(a, b));
        };
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key(x) < key(y); });
    }
    batk::MsParams K;
    memset(&K, 0, sizeof K);
    K.m = (u32)m;
    K.n = (u32)n;
    K.s = (u32)s;
    K.t = (u32)t;
    K.d = (u32)d;
    K.directed = (flags & BAT_DIRECTED) ? 1u : 0u;
    K.n_table = (u32)n_table + (u32)(batk::ms_slots(m) - m);
    std::vector<int> first(m + 1, 0);
    for (int i = 0; i < m; ++i) first[i + 1] = first[i] + sigma[i];
    // the kernel instance's slot count; the slots past the last arc are
    // one-state self-loops at s (capacity 0, probability 1): no-ops
    const int slots = batk::ms_slots(m);
    std::vector<int32_t> capt(n_table + (slots - m));
    std::vector<double> wt(n_table + (slots - m));
    u32 o = 0;
    for (int j = m; j < slots; ++j) {
        K.sig[j] = 1u;
        K.off[j] = (u32)(n_table + (j - m));
        K.u[j] = K.v[j] = (unsigned char)s;
        capt[n_table + (j - m)] = 0;
        wt[n_table + (j - m)] = 1.0;
    }
    for (int j = 0; j < m; ++j) {
        const int i = ord[j];
        K.sig[j] = (u32)sigma[i];
        K.off[j] = o;
        K.u[j] = (unsigned char)arcs[i].u;
        K.v[j] = (unsigned char)arcs[i].v;
        for (int k = 0; k < sigma[i]; ++k) {
            capt[o + k] = cap ? cap[first[i] + k] : k;
            wt[o + k] = w[first[i] + k];
        }
        o += (u32)sigma[i];
    }
    // demand 1 to 3: the bit-sliced kernel
    if (d <= 3 && m > 0 && c_hi > c_lo && opts().ms_bits.load() != 0) {
        std::vector<int> su(m), sv(m);
        for (int j = 0; j < m; ++j) {
            su[j] = K.u[j];
            sv[j] = K.v[j];
        }
        return ms_bits_run(n, m, su.data(), sv.data(), K.sig, K.off, capt, wt, s, t, d, K.directed != 0, c_lo, c_hi,
                           R_hi, R_lo, count, src_only);
    }
    if (src_only) return fail(BAT_EINVAL, "no bit-sliced kernel for this sweep (it needs demand 1 to 3 and arcs)");
    // slot 0's capacity nondecreasing in its state: the kernel's shortcuts
    // along slot 0 are exact
    K.warm = m > 0 ? 1u : 0u;
    for (int k = 1; m > 0 && k < sigma[ord[0]]; ++k)
        if (capt[k] < capt[k - 1]) K.warm = 0u;
    // launch shape: ~32K wavefront work items, each 64 runs of `run` indices
    const u64 span = c_hi - c_lo;
    const u64 target = 32768;
    K.run = std::max<u64>(1, (span + 64 * target - 1) / (64 * target));
    if (opts().ms_run.load() > 0) K.run = (u64)opts().ms_run.load();
    K.n_items = span ? (span + 64 * K.run - 1) / (64 * K.run) : 0;
    K.c_lo = c_lo;
    K.c_hi = c_hi;
    DeviceInfo D;
    rc = current_device(D);
    if (rc) return rc;
    hipStream_t st;
    rc = thread_stream(D.id, st);
    if (rc) return rc;
    // workspace: input (cap | w tables) | partials | counts | output (res | count)
    const size_t n_tab = capt.size();
    const size_t o_cap = 0;
    const size_t o_w = align_up(o_cap + sizeof(int32_t) * (n_tab + 1), 256);
    const size_t in_bytes = align_up(o_w + sizeof(double) * (n_tab + 1), 256);
    const u64 items = std::max<u64>(K.n_items, 1);
    const size_t o_part = in_bytes;
    const size_t o_pc = align_up(o_part + sizeof(double) * 2 * items, 256);
    const size_t o_res = align_up(o_pc + sizeof(u64) * items, 256);
    const size_t o_cnt = o_res + 2 * sizeof(double);
    const size_t out_bytes = o_cnt + sizeof(u64) - o_res;
    const size_t total = align_up(o_cnt + sizeof(u64) + 64, 256);
    Scratch *S = nullptr;
    const size_t out_host_off = in_bytes;
    rc = scratch_reserve(D.id, st, total, out_host_off + out_bytes, S);
    if (rc) return rc;
    char *ws = S->dev;
    memcpy(S->host + o_cap, capt.data(), sizeof(int32_t) * n_tab);
    memcpy(S->host + o_w, wt.data(), sizeof(double) * n_tab);
    HIPCHK(hipMemcpyAsync(ws, S->host, in_bytes, hipMemcpyHostToDevice, st));
    K.cap = (const int *)(ws + o_cap);
    K.w = (const double *)(ws + o_w);
    K.part = (double *)(ws + o_part);
    K.pcount = (u64 *)(ws + o_pc);
    double *res = (double *)(ws + o_res);
    u64 *cnt = (u64 *)(ws + o_cnt);
    rc = events_ready();
    if (rc) return rc;
    const u64 blocks = (K.n_items + bat::kWavesPerBlock - 1) / bat::kWavesPerBlock;
    if (blocks > 0x7fffffffull) return fail(BAT_ETOOBIG, "too many work items (%llu)", (unsigned long long)blocks);
    HIPCHK(hipEventRecord(t_state.ev[0], st));
    HIPCHK(hipEventRecord(t_state.ev[1], st));
    if (blocks) HIPCHK(batk::ms_sweep(st, (unsigned)blocks, K));
    HIPCHK(hipEventRecord(t_state.ev[2], st));
    HIPCHK(batk::reduce(st, (const double *)K.part, (const u64 *)K.pcount, K.n_items, 1, res, cnt));
    HIPCHK(hipEventRecord(t_state.ev[3], st));
    char *out = S->host + out_host_off;
    HIPCHK(hipMemcpyAsync(out, ws + o_res, out_bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bat_launch_info &I = t_state.info;
    memset(&I, 0, sizeof I);
    I.vectors = span;
    I.n_chunks = (int32_t)std::min<u64>(K.n_items, 0x7fffffff);
    I.chunk_log2 = -1;
    I.relaxations = m;
    I.kernel_id = aot_kernel_id("k_ms_flow", batk::ms_slots(m), K.directed != 0);
    I.block_waves = bat::kWavesPerBlock;
    t_state.have_launch = true;
    memcpy(&R_hi, out, sizeof(double));
    memcpy(&R_lo, out + sizeof(double), sizeof(double));
    memcpy(&count, out + 2 * sizeof(double), sizeof(u64));
    return BAT_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *bat_version(void) { return kVersion; }

const char *bat_last_error(void) { return t_err.c_str(); }

int bat_set_option(const char *key, int64_t value)
{
    auto *o = opts().find(key);
    if (!o) return fail(BAT_EINVAL, "unknown option '%s'", key ? key : "(null)");
    if (!strcmp(key, "BAT_JIT_FLUSH")) {  // an action, not a setting
        if (value) jit_flush();
        return BAT_OK;
    }
    *o = value;
    return BAT_OK;
}

int bat_get_option(const char *key, int64_t *value)
{
    auto *o = opts().find(key);
    if (!o || !value) return fail(BAT_EINVAL, "unknown option '%s'", key ? key : "(null)");
    *value = o->load();
    return BAT_OK;
}

int bat_reliability_ex(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                       uint32_t flags, double *R_out, uint64_t *count_out, double *dRdp_out, double *T1_out,
                       double *T0_out)
{
    t_err.clear();
    if (!R_out || !count_out) return fail(BAT_EINVAL, "NULL output pointer");
    if (flags & ~(uint32_t)(BAT_DIRECTED | BAT_FORWARD_ORDER)) return fail(BAT_EINVAL, "unknown flags 0x%x", flags);
    if (m < 0 || m > BAT_MAX_ARCS) return validate(n, m, arcs, p, s, t);
    const bool grad = dRdp_out || T1_out || T0_out;
    std::vector<double> res;
    std::vector<int> cba;
    u64 cnt = 0;
    // a whole sweep: the index order does not matter, any arc order is used
    int rc = run_sync(n, m, arcs, p, s, t, 0, 1ull << m, grad, res, cnt, nullptr, &cba, flags);
    if (rc) return rc;
    *R_out = res[0] + res[1];
    *count_out = cnt;
    if (grad) split_grad(res, cba, m, dRdp_out, T1_out, T0_out);
    return BAT_OK;
}

int bat_reliability(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                    double *R_out, uint64_t *count_out)
{
    return bat_reliability_ex(n, m, arcs, p, s, t, 0u, R_out, count_out, nullptr, nullptr, nullptr);
}

int bat_reliability_grad(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                         double *R_out, uint64_t *count_out, double *dRdp_out, double *T1_out, double *T0_out)
{
    t_err.clear();
    if (!dRdp_out && m > 0) return fail(BAT_EINVAL, "NULL output pointer");
    if (m == 0) {  // no arcs: no gradient to write, R = 0 from the forward sweep
        return bat_reliability_ex(n, m, arcs, p, s, t, 0u, R_out, count_out, nullptr, nullptr, nullptr);
    }
    return bat_reliability_ex(n, m, arcs, p, s, t, 0u, R_out, count_out, dRdp_out, T1_out, T0_out);
}

int bat_reliability_range_ex(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                             uint32_t flags, uint64_t c_lo, uint64_t c_hi, double *R_hi, double *R_lo,
                             uint64_t *count_out, double *T1_out, double *T0_out)
{
    t_err.clear();
    if (!R_hi || !R_lo || !count_out) return fail(BAT_EINVAL, "NULL output pointer");
    if ((T1_out == nullptr) != (T0_out == nullptr)) return fail(BAT_EINVAL, "T1_out and T0_out must both be set or both NULL");
    if (flags & ~(uint32_t)(BAT_DIRECTED | BAT_FORWARD_ORDER)) return fail(BAT_EINVAL, "unknown flags 0x%x", flags);
    if (m < 0 || m > BAT_MAX_ARCS) return validate(n, m, arcs, p, s, t);
    if (c_lo > c_hi || c_hi > (1ull << m)) return fail(BAT_EINVAL, "bad range [%llu, %llu) for m = %d",
                                                     (unsigned long long)c_lo, (unsigned long long)c_hi, m);
    // the indices are the paper's: backward BAT (Eq. 2-3) or forward (Eq. 4-5)
    return range_in_order(n, m, arcs, p, s, t, flags, (flags & BAT_FORWARD_ORDER) ? kPermForward : 0, c_lo, c_hi,
                          R_hi, R_lo, count_out, T1_out, T0_out);
}

int bat_reliability_range(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                          uint64_t c_lo, uint64_t c_hi, double *R_hi, double *R_lo, uint64_t *count_out,
                          double *T1_out, double *T0_out)
{
    return bat_reliability_range_ex(n, m, arcs, p, s, t, 0u, c_lo, c_hi, R_hi, R_lo, count_out, T1_out, T0_out);
}

int bat_reliability_checkpointed(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                                 uint32_t flags, int32_t chunk_log2, const char *path, int64_t max_chunks,
                                 double *R_out, uint64_t *count_out, double *dRdp_out, double *T1_out,
                                 double *T0_out)
{
    t_err.clear();
    if (!R_out || !count_out) return fail(BAT_EINVAL, "NULL output pointer");
    if (flags & ~(uint32_t)(BAT_DIRECTED | BAT_FORWARD_ORDER)) return fail(BAT_EINVAL, "unknown flags 0x%x", flags);
    if (chunk_log2 < 0 || chunk_log2 > BAT_MAX_ARCS)
        return fail(BAT_EINVAL, "chunk_log2 %d outside [0, %d]", chunk_log2, BAT_MAX_ARCS);
    if (!p && m > 0) return fail(BAT_EINVAL, "p is NULL");
    int rc = validate(n, m, arcs, p, s, t);
    if (rc) return rc;
    const bool grad = dRdp_out || T1_out || T0_out;
    const int32_t clog = chunk_log2 < m ? chunk_log2 : m;
    const u64 parts_wanted = 1ull << (m - clog);
    const std::string problem = checkpoint_problem(n, m, arcs, p, s, t, flags, chunk_log2, grad);
    RunningSums S;
    if (grad) {
        S.T1.assign(2 * (size_t)m, 0.0);
        S.T0.assign(2 * (size_t)m, 0.0);
    }
    if (path) {
        rc = checkpoint_read(path, problem, grad, m, flags, S);
        if (rc < 0) return rc;
    }
    std::vector<double> t1(m > 0 ? m : 1), t0(m > 0 ? m : 1);
    for (int64_t ran = 0; (S.parts == 0 || S.done < S.parts) && (max_chunks < 0 || ran < max_chunks); ++ran) {
        double hl[2] = {0.0, 0.0};
        uint64_t c = 0;
        rc = run_part(n, m, arcs, p, s, t, flags, grad, parts_wanted, S, hl, &c, grad ? t1.data() : nullptr,
                      grad ? t0.data() : nullptr);
        if (rc) return rc;
        dd_acc(S.R, hl[0], hl[1]);
        S.count += c;
        for (int32_t a = 0; grad && a < m; ++a) {
            dd_acc(&S.T1[2 * a], t1[a], 0.0);
            dd_acc(&S.T0[2 * a], t0[a], 0.0);
        }
        ++S.done;
        if (path) {
            rc = checkpoint_write(path, problem, grad, S);
            if (rc) return rc;
        }
    }
    if (S.parts == 0 || S.done < S.parts) return BAT_PENDING;
    *R_out = S.R[0] + S.R[1];
    *count_out = S.count;
    for (int32_t a = 0; grad && a < m; ++a) {
        const double *a1 = &S.T1[2 * a], *a0 = &S.T0[2 * a];
        if (dRdp_out) dRdp_out[a] = (a1[0] - a0[0]) + (a1[1] - a0[1]);
        if (T1_out) T1_out[a] = a1[0] + a1[1];
        if (T0_out) T0_out[a] = a0[0] + a0[1];
    }
    return BAT_OK;
}

static int async_common(int32_t n, int32_t m, const bat_arc *arcs, const double *p_dev, int32_t s, int32_t t,
                        double *R_dev, uint64_t *count_dev, bool grad, double *dRdp_dev, double *T1_dev,
                        double *T0_dev, int32_t *status_dev, void *stream)
{
    t_err.clear();
    if (!R_dev || !count_dev || (grad && !dRdp_dev && m > 0)) return fail(BAT_EINVAL, "NULL output pointer");
    if (m > 0 && !p_dev) return fail(BAT_EINVAL, "p_dev is NULL");
    Prepared X;
    TuneChoice tc;
    int rc = prepare(n, m, arcs, nullptr, s, t, grad, true, nullptr, X, tc);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Request rq{};
    rq.n = n; rq.m = m; rq.s = s; rq.t = t; rq.arcs = arcs; rq.p_dev = p_dev;
    rq.c_lo = 0; rq.c_hi = 1ull << m; rq.grad = grad;
    Launch L;
    rc = queue_sweep(rq, X.P, X.D, tc, st, L);
    if (rc) {
        if (L.ws) (void)hipFreeAsync(L.ws, st);
        return rc;
    }
    HIPCHK(batk::finalize(st, (const double *)L.res, (const u64 *)L.count, (const int *)L.status, L.cb_of_arc,
                          (u32)m, grad, R_dev, (u64 *)count_dev, dRdp_dev, T1_dev, T0_dev, (int *)status_dev));
    HIPCHK(hipFreeAsync(L.ws, st));
    return BAT_OK;
}

int bat_reliability_async(int32_t n, int32_t m, const bat_arc *arcs, const double *p_dev, int32_t s, int32_t t,
                          double *R_dev, uint64_t *count_dev, int32_t *status_dev, void *stream)
{
    return async_common(n, m, arcs, p_dev, s, t, R_dev, count_dev, false, nullptr, nullptr, nullptr, status_dev,
                        stream);
}

int bat_reliability_grad_async(int32_t n, int32_t m, const bat_arc *arcs, const double *p_dev, int32_t s,
                               int32_t t, double *R_dev, uint64_t *count_dev, double *dRdp_dev, double *T1_dev,
                               double *T0_dev, int32_t *status_dev, void *stream)
{
    return async_common(n, m, arcs, p_dev, s, t, R_dev, count_dev, true, dRdp_dev, T1_dev, T0_dev, status_dev,
                        stream);
}

int bat_reliability_noalloc(int32_t n, int32_t m, const bat_arc *arcs, const double *p_dev, int32_t s, int32_t t,
                            double *R_dev, uint64_t *count_dev, int32_t *status_dev, void *stream)
{
    t_err.clear();
    if (!R_dev || !count_dev) return fail(BAT_EINVAL, "NULL output pointer");
    if (m > 0 && !p_dev) return fail(BAT_EINVAL, "p_dev is NULL");
    Prepared X;
    TuneChoice tc;
    int rc = prepare(n, m, arcs, nullptr, s, t, false, true, nullptr, X, tc);
    if (rc) return rc;
    // set-up on this device's first call: the address of its scratch copy
    char *ws = nullptr;
    rc = noalloc_scratch(X.D.id, ws);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Request rq{};
    rq.n = n; rq.m = m; rq.s = s; rq.t = t; rq.arcs = arcs; rq.p_dev = p_dev;
    rq.c_lo = 0; rq.c_hi = 1ull << m; rq.grad = false;
    Launch L;
    rc = queue_sweep(rq, X.P, X.D, tc, st, L, nullptr, ws, kNoAllocScratchBytes);
    if (rc) return rc;
    HIPCHK(batk::finalize(st, (const double *)L.res, (const u64 *)L.count, (const int *)L.status, L.cb_of_arc,
                          (u32)m, false, R_dev, (u64 *)count_dev, nullptr, nullptr, nullptr, (int *)status_dev));
    return BAT_OK;
}

int bat_ms_reliability(int32_t n, int32_t m, const bat_arc *arcs, const int32_t *n_states, const int32_t *capacity,
                       const double *w, int32_t s, int32_t t, int32_t demand, uint32_t flags, double *R_out,
                       uint64_t *count_out)
{
    t_err.clear();
    if (!R_out || !count_out) return fail(BAT_EINVAL, "NULL output pointer");
    double hi = 0.0, lo = 0.0;
    u64 c = 0;
    int rc = ms_run(n, m, arcs, n_states, capacity, w, s, t, demand, flags, true, 0, 0, hi, lo, c);
    if (rc) return rc;
    *R_out = hi + lo;
    *count_out = c;
    return BAT_OK;
}

int bat_ms_reliability_range(int32_t n, int32_t m, const bat_arc *arcs, const int32_t *n_states,
                             const int32_t *capacity, const double *w, int32_t s, int32_t t, int32_t demand,
                             uint32_t flags, uint64_t c_lo, uint64_t c_hi, double *R_hi, double *R_lo,
                             uint64_t *count_out)
{
    t_err.clear();
    if (!R_hi || !R_lo || !count_out) return fail(BAT_EINVAL, "NULL output pointer");
    double hi = 0.0, lo = 0.0;
    u64 c = 0;
    int rc = ms_run(n, m, arcs, n_states, capacity, w, s, t, demand, flags, false, c_lo, c_hi, hi, lo, c);
    if (rc) return rc;
    *R_hi = hi;
    *R_lo = lo;
    *count_out = c;
    return BAT_OK;
}

int bat_valu_peak(double *lane_ops_per_s)
{
    t_err.clear();
    if (!lane_ops_per_s) return fail(BAT_EINVAL, "NULL output pointer");
    DeviceInfo D;
    int rc = current_device(D);
    if (rc) return rc;
    hipStream_t st;
    rc = thread_stream(D.id, st);
    if (rc) return rc;
    rc = events_ready();
    if (rc) return rc;
    void *sink = nullptr;
    HIPCHK(hipMallocAsync(&sink, 64 * sizeof(u32), st));
    // 64 blocks of 256 threads per CU; 2048 trips of 16 instructions each
    const unsigned blocks = (unsigned)std::max(D.cus, 1) * 64u;
    const u32 iters = 2048;
    const double ops = (double)blocks * 256.0 * iters * batk::kValuPeakOpsPerTrip;
    double best = 0.0;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // the first is a warm-up
        float ms = 0.0f;
        e = hipEventRecord(t_state.ev[0], st);
        if (e == hipSuccess) e = batk::valu_peak(st, blocks, iters, (u32 *)sink);
        if (e == hipSuccess) e = hipEventRecord(t_state.ev[1], st);
        if (e == hipSuccess) e = hipEventSynchronize(t_state.ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t_state.ev[0], t_state.ev[1]);
        if (e == hipSuccess && rep > 0 && ms > 0.0f) best = std::max(best, ops / (ms * 1e-3));
    }
    const hipError_t ef = hipFreeAsync(sink, st);
    if (e == hipSuccess) e = ef;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(BAT_EDEVICE, "bat_valu_peak: %s", hipGetErrorString(e));
    *lane_ops_per_s = best;
    return BAT_OK;
}

int bat_last_launch(bat_launch_info *info)
{
    if (!info) return fail(BAT_EINVAL, "NULL info");
    if (!t_state.have_launch) return fail(BAT_EINVAL, "no launch on this thread yet");
    HIPCHK(hipEventSynchronize(t_state.ev[3]));
    float k = 0.f, tot = 0.f;
    HIPCHK(hipEventElapsedTime(&k, t_state.ev[1], t_state.ev[2]));
    HIPCHK(hipEventElapsedTime(&tot, t_state.ev[0], t_state.ev[3]));
    t_state.info.kernel_ms = k;
    t_state.info.total_ms = tot;
    *info = t_state.info;
    return BAT_OK;
}

int bat_jit_source(int32_t n, int32_t m, const bat_arc *arcs, int32_t s, int32_t t, uint32_t flags, int32_t grad,
                   int32_t perm, char *buf, uint64_t *len)
{
    t_err.clear();
    if (!len) return fail(BAT_EINVAL, "len is NULL");
    if (flags & ~(uint32_t)BAT_DIRECTED) return fail(BAT_EINVAL, "unknown flags 0x%x", flags);
    int rc = validate(n, m, arcs, nullptr, s, t);
    if (rc) return rc;
    if (perm < 0 || perm >= kPermKinds) return fail(BAT_EINVAL, "perm %d outside [0, %d)", perm, kPermKinds);
    if (grad < -batk::kBatchMaxP || grad > 1) return fail(BAT_EINVAL, "grad %d outside [-%d, 1]", grad, batk::kBatchMaxP);
    if (grad < 0 && (flags & BAT_DIRECTED)) return fail(BAT_EINVAL, "the batched sweep is undirected");
    Plan P;
    make_plan(n, m, arcs, s, t, P, perm, (flags & BAT_DIRECTED) != 0);
    Options &O = opts();
    const std::string src =
        grad < 0 ? jit_source(P, false, jit_shape(false, 4, 0, 0, 1), -grad)
                 : jit_source(P, grad != 0,
                              jit_shape(grad != 0, (int)O.block_waves.load(), (int)O.super_restart.load(),
                                        (int)O.simd_waves.load(), (int)O.keep_bottom.load()));
    const uint64_t need = (uint64_t)src.size() + 1;
    const uint64_t have = *len;
    *len = need;
    if (!buf) return BAT_OK;
    if (have < need) return fail(BAT_ETOOBIG, "buffer of %llu bytes, need %llu", (unsigned long long)have,
                                 (unsigned long long)need);
    memcpy(buf, src.c_str(), need);
    return BAT_OK;
}

int bat_ms_jit_source(int32_t n, int32_t m, const bat_arc *arcs, const int32_t *n_states, const int32_t *capacity,
                      int32_t s, int32_t t, int32_t demand, uint32_t flags, uint64_t c_lo, uint64_t c_hi, char *buf,
                      uint64_t *len)
{
    t_err.clear();
    if (!len) return fail(BAT_EINVAL, "len is NULL");
    if (m > 0 && !n_states) return fail(BAT_EINVAL, "NULL n_states");
    // the source does not depend on the probabilities: any valid ones
    int64_t pairs = 0;
    for (int32_t i = 0; i < m; ++i) pairs += n_states[i] > 0 ? n_states[i] : 0;
    if (pairs > batk::kMsMaxTable) return fail(BAT_ETOOBIG, "more than %d (arc, state) pairs", batk::kMsMaxTable);
    std::vector<double> w((size_t)pairs + 1, 1.0);
    std::string src;
    double hi = 0.0, lo = 0.0;
    u64 c = 0;
    const bool whole = c_lo == 0 && c_hi == 0;
    int rc = ms_run(n, m, arcs, n_states, capacity, w.data(), s, t, demand, flags, whole, c_lo, c_hi, hi, lo, c, &src);
    if (rc) return rc;
    const uint64_t need = (uint64_t)src.size() + 1;
    const uint64_t have = *len;
    *len = need;
    if (!buf) return BAT_OK;
    if (have < need) return fail(BAT_ETOOBIG, "buffer of %llu bytes, need %llu", (unsigned long long)have,
                                 (unsigned long long)need);
    memcpy(buf, src.c_str(), need);
    return BAT_OK;
}

int bat_autotune(int32_t n, int32_t m, const bat_arc *arcs, const double *p, int32_t s, int32_t t,
                 double *best_ns_per_vector)
{
    t_err.clear();
    int rc = validate(n, m, arcs, p, s, t);
    if (rc) return rc;
    if (!p && m > 0) return fail(BAT_EINVAL, "p is NULL");
    DeviceInfo D;
    rc = current_device(D);
    if (rc) return rc;
    // Each candidate sweeps a sample of its work items spread over the whole
    // counter (an odd-multiplier hash of the item index, so every arc's
    // state varies across the sample), about 2^38 vectors or everything if
    // that is less; candidates are compared by their best time per vector
    // over two timed passes.
    const u64 total = 1ull << m;
    const u32 ubits = m > bat::kWordBits ? (u32)m - bat::kWordBits : 0u;
    // the automatic work-item size (as queue_sweep picks it)
    const int clog_auto = fill_item_log2(1ull << ubits, D.cus, 1);
    struct Cand {
        int clog, check, jit, perm, chain, waves = -1, super_restart = -1, simd_waves = -1, keep_bottom = -1;
    };
    constexpr double kTuneMargin = 0.01;
    auto measure = [&](const Cand &c, double &ns, bool grad = false) -> bool {
        ns = 1e300;
        // the best of at least two timed passes, more for short samples (up
        // to ~40 ms of timed kernel, at most 6 passes), whose times scatter
        // more; a pass whose kernel was compiled or loaded first is not
        // timed (the kernels were compiled ahead, so that is one pass)
        double timed_ms = 0.0;
        int timed = 0;
        for (int rep = 0; rep < 8 && (timed < 2 || (timed < 6 && timed_ms < 40.0)); ++rep) {
            Request tmpl{};
            tmpl.force_chunk_log2 = c.clog;
            tmpl.force_check = c.check;
            tmpl.force_jit = c.jit;
            tmpl.force_perm = c.perm;
            tmpl.force_chain = c.chain;
            tmpl.force_waves = c.waves;
            tmpl.force_super = c.super_restart;
            tmpl.force_simd = c.simd_waves;
            tmpl.force_keep = c.keep_bottom;
            const int cl = c.clog > 0 ? c.clog : std::max(clog_auto, 3);
            const u64 per_item = 1ull << (cl + bat::kWordBits);
            tmpl.sample_items = std::max<u64>(1024, (1ull << 38) / per_item);
            std::vector<double> res;
            u64 cnt = 0;
            bat_launch_info li;
            if (run_sync(n, m, arcs, p, s, t, 0, total, grad, res, cnt, &tmpl) || bat_last_launch(&li)) return false;
            if (li.jit_ms == 0.0) {
                ns = std::min(ns, li.kernel_ms * 1e6 / (double)li.vectors);
                timed_ms += li.kernel_ms;
                ++timed;
            }
        }
        return true;
    };
    double best = 1e300;
    Cand bc{0, 1, 2, kDefaultPerm, 3};
    const char *vb = getenv("BAT_AUTOTUNE_VERBOSE");
    const bool verbose = vb && *vb && *vb != '0';
    auto consider = [&](const Cand &c) {
        double ns;
        const bool ok = measure(c, ns);
        if (verbose)
            fprintf(stderr,
                    "bat_autotune: chunk_log2=%d check=%d jit=%d perm=%d chain=%d waves=%d super=%d simd=%d "
                    "keep=%d -> %s %.6f ns/vector\n",
                    c.clog, c.check, c.jit, c.perm, c.chain, c.waves, c.super_restart, c.simd_waves, c.keep_bottom,
                    ok ? "ok" : "failed", ok ? ns : 0.0);
        // a later candidate must win by a margin: near ties keep the
        // earlier (default-first) choice, so repeated tuning agrees
        if (ok && ns < best * (1.0 - kTuneMargin)) {
            best = ns;
            bc = c;
        }
    };
    // compile the specialised kernels of candidates ahead of their runs, in
    // parallel (their knobs resolved as a launch resolves them)
    const std::string gkey = graph_key(n, m, arcs, s, t);
    auto precompile = [&](const std::vector<std::pair<Cand, bool>> &cands) {
        std::vector<Plan> plans(cands.size());
        std::vector<std::tuple<const Plan *, bool, JitShape>> want;
        for (size_t i = 0; i < cands.size(); ++i) {
            const Cand &c = cands[i].first;
            const bool grad = cands[i].second;
            Request r{};
            r.force_chunk_log2 = c.clog;
            r.force_check = c.check;
            r.force_jit = c.jit;
            r.force_perm = c.perm;
            r.force_chain = c.chain;
            r.force_waves = c.waves;
            r.force_super = c.super_restart;
            r.force_simd = c.simd_waves;
            r.force_keep = c.keep_bottom;
            TuneChoice tc = choose(D, gkey, grad, &r);
            if (tc.jit != 1) continue;
            if (tc.perm < 0 || tc.perm >= kPermKinds) tc.perm = kDefaultPerm;
            make_plan(n, m, arcs, s, t, plans[i], tc.perm);
            want.emplace_back(&plans[i], grad, jit_shape(grad, tc.waves, tc.super_restart, tc.simd_waves, tc.keep_bottom));
        }
        jit_precompile(D, want);
    };
    {
        std::vector<std::pair<Cand, bool>> first;
        for (int i = 0; i < kPermKinds; ++i) first.push_back({{0, 1, 1, i, 3}, false});
        for (int perm : {kDefaultPerm, 0}) first.push_back({{0, 1, 1, perm, 3}, true});
        precompile(first);
    }
    // stage 1: arc-to-bit order x chain length, specialised kernel,
    // automatic work-item size (the two interact); the default order first
    for (int i = 0; i < kPermKinds; ++i) {
        const int perm = (kDefaultPerm + i) % kPermKinds;
        for (int k : {3, 5}) consider({0, 1, 1, perm, k});
    }
    {
        const Cand w1 = bc;
        for (int k : {4, 6})
            if (k != w1.chain) consider({0, 1, 1, w1.perm, k});
    }
    // stage 2: work-item size, convergence-test cadence, generic kernel
    const Cand w = bc;
    for (int d : {-2, 2}) {
        int cl = clog_auto + d;
        if (cl >= 5 && cl <= 14) consider({cl, w.check, w.jit, w.perm, w.chain});
    }
    consider({bc.clog, 2, bc.jit, bc.perm, bc.chain});
    // launch shape of the specialised forward sweep: the register budget
    // (5 wavefronts per SIMD, or the compiler's own), then blocks of 2
    // wavefronts and the super-block store (which takes LDS, so whole
    // 4-wavefront blocks wait for it)
    if (bc.jit != 0) {
        {
            std::vector<std::pair<Cand, bool>> shapes;
            for (int sw : {5, 6, 0}) shapes.push_back({{bc.clog, bc.check, bc.jit, bc.perm, bc.chain, -1, -1, sw}, false});
            shapes.push_back({{bc.clog, bc.check, bc.jit, bc.perm, bc.chain, -1, -1, -1, 2}, false});
            shapes.push_back({{bc.clog, bc.check, bc.jit, bc.perm, bc.chain, 2, 0}, false});
            shapes.push_back({{bc.clog, bc.check, bc.jit, bc.perm, bc.chain, 4, 1}, false});
            shapes.push_back({{bc.clog, bc.check, bc.jit, bc.perm, 3}, true});
            precompile(shapes);
        }
        const Cand w2 = bc;
        // (-1 is the default: 6, or the compiler's budget for big plans)
        for (int sw : {5, 6, 0})
            consider({w2.clog, w2.check, w2.jit, w2.perm, w2.chain, -1, -1, sw});
        const Cand w3 = bc;
        // the kept block bottom in LDS: no spills for it, but fewer blocks fit
        consider({w3.clog, w3.check, w3.jit, w3.perm, w3.chain, -1, -1, w3.simd_waves, 2});
        const Cand w4 = bc;
        consider({w4.clog, w4.check, w4.jit, w4.perm, w4.chain, 2, 0, w4.simd_waves, w4.keep_bottom});
        consider({w4.clog, w4.check, w4.jit, w4.perm, w4.chain, 4, 1, w4.simd_waves, w4.keep_bottom});
    }
    if (total <= (1ull << 32)) consider({bc.clog, 1, 0, 0, 0});
    if (best >= 1e300) return fail(BAT_EDEVICE, "autotune: no candidate ran (%s)", t_err.c_str());
    if (best_ns_per_vector) *best_ns_per_vector = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        TuneChoice tc{bc.clog, bc.check, bc.jit, bc.perm, bc.chain};
        tc.waves = bc.waves;
        tc.super_restart = bc.super_restart;
        tc.simd_waves = bc.simd_waves;
        tc.keep_bottom = bc.keep_bottom;
        const std::string gk = graph_key(n, m, arcs, s, t);
        g_tune[std::to_string(D.id) + " fwd " + gk] = tc;
    }
    // the gradient sweep: its own arc order and chain length (it keeps at
    // most 4 chained bits, and its cost is spread differently), starting
    // from the forward's choice; the launch shape is its own and fixed
    {
        Cand gb{bc.clog, bc.check, bc.jit, bc.perm, std::min(bc.chain, 4)};
        double gbest = 1e300;
        auto gconsider = [&](const Cand &c) {
            double ns;
            const bool ok = measure(c, ns, true);
            if (verbose)
                fprintf(stderr, "bat_autotune (gradient): chunk_log2=%d check=%d jit=%d perm=%d chain=%d -> %s %.6f ns/vector\n",
                        c.clog, c.check, c.jit, c.perm, c.chain, ok ? "ok" : "failed", ok ? ns : 0.0);
            if (ok && ns < gbest * (1.0 - kTuneMargin)) {
                gbest = ns;
                gb = c;
            }
        };
        gconsider(gb);
        if (bc.jit != 0) {
            for (int perm : {kDefaultPerm, 0})
                for (int k : {3, 4})
                    if (perm != gb.perm || k != gb.chain) gconsider({bc.clog, bc.check, bc.jit, perm, k});
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        TuneChoice tc{gb.clog, gb.check, gb.jit, gb.perm, gb.chain};
        g_tune[std::to_string(D.id) + " grad " + graph_key(n, m, arcs, s, t)] = tc;
    }
    t_err.clear();
    return BAT_OK;
}

}  // extern "C"

// Tuned knobs of the batched launch: chained iteration bits and the
// per-wavefront segment size, cached under the batch's structure.
struct BatchTune {
    int chain = -1;  // -1: option BAT_CHAIN_LOG2 (-1 = 3)
    int seg = -1;    // -1: batk::kBatchSegLog
    int jit_arcs = -1;  // graphs with at least this many arcs run graph-specialised (0: none; -1: option)
    int streams = -1;   // side streams of the specialised kernels (0: the thread's stream; -1: option, else 3)
};
std::mutex g_btune_mu;
std::map<std::string, BatchTune> g_btune;

// The batch's structure (graphs, terminals, p-vector count) as a key.
std::string batch_key(int device, int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets,
                      const bat_arc *arcs, const int32_t *s, const int32_t *t, int32_t n_pvec)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the structure
    auto mix = [&](const void *d, size_t n) {
        const unsigned char *c = (const unsigned char *)d;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    };
    mix(n_nodes, sizeof(int32_t) * n_graphs);
    mix(arc_offsets, sizeof(int32_t) * (n_graphs + 1));
    mix(arcs, sizeof(bat_arc) * arc_offsets[n_graphs]);
    mix(s, sizeof(int32_t) * n_graphs);
    mix(t, sizeof(int32_t) * n_graphs);
    return std::to_string(device) + " batch " + std::to_string(n_graphs) + " " + std::to_string(n_pvec) + " " +
           std::to_string(h);
}

int batched_impl(int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets, const bat_arc *arcs,
                 const int32_t *s, const int32_t *t, int32_t n_pvec, const double *p, double *R_out,
                 uint64_t *counts_out, const BatchTune *force)
{
    t_err.clear();
    if (n_graphs <= 0) return fail(BAT_EINVAL, "n_graphs must be >= 1");
    if (!n_nodes || !arc_offsets || !s || !t || !R_out || !counts_out) return fail(BAT_EINVAL, "NULL argument");
    if (n_pvec < 1 || n_pvec > BAT_MAX_PVEC) return fail(BAT_EINVAL, "n_pvec %d outside [1, %d]", n_pvec, BAT_MAX_PVEC);
    if (arc_offsets[0] != 0) return fail(BAT_EINVAL, "arc_offsets[0] must be 0");
    for (int32_t g = 0; g < n_graphs; ++g) {
        int32_t m = arc_offsets[g + 1] - arc_offsets[g];
        if (m < 0) return fail(BAT_EINVAL, "arc_offsets not ascending at graph %d", g);
        int rc = validate(n_nodes[g], m, m ? arcs + arc_offsets[g] : nullptr, nullptr, s[g], t[g]);
        if (rc) return fail(rc, "graph %d: %s", g, t_err.c_str());
        if (m > 0 && !p) return fail(BAT_EINVAL, "p is NULL");
        const double *pg = p + (int64_t)n_pvec * arc_offsets[g];
        for (int64_t i = 0; i < (int64_t)n_pvec * m; ++i)
            if (!(pg[i] >= 0.0 && pg[i] <= 1.0))
                return fail(BAT_EINVAL, "graph %d: p[%lld] = %g is not a probability", g, (long long)i, pg[i]);
    }
    DeviceInfo D;
    int rc = current_device(D);
    if (rc) return rc;
    hipStream_t st;
    rc = thread_stream(D.id, st);
    if (rc) return rc;

    // plans, entries (graph x group of <= 32 p-vectors), longest first
    std::vector<Plan> plans(n_graphs);
    std::vector<u32> progs;
    std::vector<u32> prog_off(n_graphs);
    int nmax = 2;
    for (int32_t g = 0; g < n_graphs; ++g) {
        int32_t m = arc_offsets[g + 1] - arc_offsets[g];
        make_plan(n_nodes[g], m, arcs + arc_offsets[g], s[g], t[g], plans[g]);
        prog_off[g] = (u32)progs.size();
        progs.insert(progs.end(), plans[g].prog.begin(), plans[g].prog.end());
        nmax = std::max(nmax, plans[g].N);
    }
    // knobs: forced (autotuner), else the tuned choice, else the options
    BatchTune bt;
    if (force) {
        bt = *force;
    } else if (opts().autotune.load()) {
        std::lock_guard<std::mutex> lk(g_btune_mu);
        auto it = g_btune.find(batch_key(D.id, n_graphs, n_nodes, arc_offsets, arcs, s, t, n_pvec));
        if (it != g_btune.end()) bt = it->second;
    }
    if (!force && opts().chain_log2.load() >= 0) bt.chain = (int)opts().chain_log2.load();
    if (!force && opts().batch_jit_arcs.load() >= 0) bt.jit_arcs = (int)opts().batch_jit_arcs.load();
    const int jit_arcs = bt.jit_arcs > 0 ? bt.jit_arcs : 0;
    // chained iteration bits (-1 = 3, 0 = none, 3..6)
    const int bchain = bt.chain < 0 ? 3 : (bt.chain >= 3 ? std::min(bt.chain, 6) : 0);
    const u32 bseg = bt.seg > 0 ? (u32)std::min(bt.seg, batk::kBatchSegLog) : (u32)batk::kBatchSegLog;
    // graphs of at least jit_arcs arcs (and a full work item) get their own
    // graph-specialised kernel, for at most kBatchSpecP p-vectors per entry;
    // the rest share the generic persistent one
    auto specialised = [&](const batk::BatchEntry &e) {
        return jit_arcs > 0 && (int)e.m >= jit_arcs && e.ubits >= e.f && e.f >= 3;
    };
    std::vector<batk::BatchEntry> ents;
    for (int32_t g = 0; g < n_graphs; ++g) {
        const Plan &P = plans[g];
        u32 m = (u32)P.m;
        u32 ubits = m > (u32)bat::kWordBits ? m - bat::kWordBits : 0u;
        batk::BatchEntry probe;
        memset(&probe, 0, sizeof probe);
        probe.m = m;
        probe.ubits = ubits;
        probe.f = std::min<u32>(ubits, bseg);
        const int32_t per = specialised(probe) ? kBatchSpecP : batk::kBatchMaxP;
        for (int32_t b = 0; b < n_pvec; b += per) {
            batk::BatchEntry e;
            memset(&e, 0, sizeof e);
            e.m = m;
            e.ubits = ubits;
            e.f = std::min<u32>(ubits, bseg);
            e.P = (u32)std::min<int32_t>(per, n_pvec - b);
            e.n_nodes = (u32)P.N;
            e.s = (u32)P.S;
            e.t = (u32)P.T;
            e.n_relax = (u32)P.code.size();
            e.prog_off = prog_off[g];
            e.n_groups = (u32)((P.prog.size() - 8) / 16);
            // warm-started chains over k <= f iteration bits
            e.chain = (bchain >= 3 && e.f >= (u32)bchain) ? (u32)bchain : (e.f >= 3 && bchain >= 3 ? e.f : 0u);
            chain_codes(P, e.ck_code);
            e.graph = (u32)g;
            e.pv_base = (u32)b;
            ents.push_back(e);
        }
    }
    // generic entries first (one queue), then the specialised ones; each
    // part longest first
    std::stable_sort(ents.begin(), ents.end(), [&](const batk::BatchEntry &a, const batk::BatchEntry &b) {
        const bool sa = specialised(a), sb = specialised(b);
        return sa != sb ? sb : a.m > b.m;
    });
    size_t n_gen = 0;
    while (n_gen < ents.size() && !specialised(ents[n_gen])) ++n_gen;
    nmax = 2;
    for (size_t i = 0; i < n_gen; ++i) nmax = std::max(nmax, (int)ents[i].n_nodes);
    // wavefronts per block of the generic kernel: an item is that many
    // segments
    const bool gen_t = opts().batch_acc.load() == 1;
    const int gen_waves = gen_t ? batk::batch_waves_t(nmax) : batk::batch_waves(nmax);
    u64 n_items = 0, n_gen_items = 0, tab = 0;
    std::vector<u64> item_start;
    std::vector<u32> pair_entry, pair_pv;
    std::vector<u64> entry_p_off;
    u64 vectors = 0;
    for (size_t i = 0; i < ents.size(); ++i) {
        batk::BatchEntry &e = ents[i];
        u64 iters = 1ull << e.ubits;
        // a generic item is a block's worth of segments, a specialised one a
        // single segment (one wavefront)
        u64 per_item = i < n_gen ? (u64)gen_waves << e.f : 1ull << e.f;
        e.item_begin = n_items;
        e.n_items = (iters + per_item - 1) / per_item;
        e.tab_off = tab;
        item_start.push_back(n_items);
        n_items += e.n_items;
        if (i < n_gen) n_gen_items = n_items;
        tab += (u64)e.P * bat::kTablesFwd;
        for (u32 q = 0; q < e.P; ++q) {
            pair_entry.push_back((u32)i);
            pair_pv.push_back(q);
        }
        entry_p_off.push_back((u64)n_pvec * (u64)arc_offsets[e.graph]);
        vectors += 1ull << e.m;
    }
    item_start.push_back(n_items);
    const int64_t p_total = (int64_t)n_pvec * arc_offsets[n_graphs];

    // the specialised kernels: one per (graph, p-vectors in the entry),
    // compiled side by side before the first is loaded
    std::vector<hipFunction_t> spec_fn(ents.size(), nullptr);
    uint64_t spec_id = 0;
    double spec_jit_ms = 0.0;
    if (n_gen < ents.size()) {
        const JitShape sh = jit_shape(false, 4, 0, 0, 1);
        auto t0 = std::chrono::steady_clock::now();
        std::vector<std::string> srcs(ents.size()), keys(ents.size()), todo;
        for (size_t i = n_gen; i < ents.size(); ++i) {
            keys[i] = std::to_string(D.id) + " batch" + std::to_string(ents[i].P) +
                      (batch_transposed((int)ents[i].P) ? "t " : " ") + plans[ents[i].graph].structure;
            srcs[i] = jit_source(plans[ents[i].graph], false, sh, (int)ents[i].P);
            std::lock_guard<std::mutex> lk(g_jit_mu);
            if (!g_jit.count(keys[i])) todo.push_back(srcs[i]);
        }
        if (!todo.empty()) jit_precompile_sources(D, todo);
        for (size_t i = n_gen; i < ents.size(); ++i) {
            const std::string &key = keys[i];
            double ms = 0.0;
            uint64_t id = 0;
            rc = jit_load(D, key, srcs[i], "bat_batch_jit", spec_fn[i], ms, id);
            if (rc) return rc;
            spec_id = spec_id * 0x100000001b3ull + id;
        }
        spec_jit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }

    // device buffers (one stream-ordered allocation)
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_ent = take(sizeof(batk::BatchEntry) * ents.size());
    const size_t o_ist = take(sizeof(u64) * item_start.size());
    const size_t o_prog = take(sizeof(u32) * (progs.size() + 1));
    const size_t o_pe = take(sizeof(u32) * pair_entry.size());
    const size_t o_pp = take(sizeof(u32) * pair_pv.size());
    const size_t o_epo = take(sizeof(u64) * entry_p_off.size());
    const size_t o_p = take(sizeof(double) * (size_t)(p_total + 1));
    const size_t o_tab = take(sizeof(double) * tab);
    const size_t o_part = take(sizeof(double) * 2 * batk::kBatchMaxP * n_items);
    const size_t o_pc = take(sizeof(u64) * n_items);
    const size_t o_ctr = take(sizeof(unsigned long long));
    const size_t o_R = take(sizeof(double) * (size_t)n_graphs * n_pvec);
    const size_t o_cnt = take(sizeof(u64) * (size_t)n_graphs);
    char *ws = nullptr;
    // side streams for the specialised kernels (before anything is queued)
    const size_t n_spec = ents.size() - n_gen;
    SideStreams *SS = nullptr;
    // how many side streams: forced by the option, else tuned, else 3 (with
    // the thread's stream, the 4 hardware queues HIP gives a process by
    // default; which queue a stream shares depends on the streams the
    // process made before it, so the autotuner measures 1 to 3)
    int want_side = bt.streams >= 0 ? bt.streams : 3;
    if (opts().batch_streams.load() >= 0 && (!force || bt.streams < 0)) want_side = (int)opts().batch_streams.load();
    const int n_side = (int)std::min<int64_t>(std::min<int64_t>(want_side, kSideStreams), (int64_t)n_spec);
    if (n_side > 0) {
        rc = side_streams(D.id, SS);
        if (rc) return rc;
    }
    // lanes for the specialised kernels: the thread's stream (lane 0, which
    // runs its share first and the generic persistent kernel after it) and
    // the side streams; each kernel goes to the least-loaded lane, largest
    // first, lane 0 starting with the generic kernel's work (weighted by
    // its slower closure)
    double lane_load[kSideStreams + 1] = {};
    for (size_t i = 0; i < n_gen; ++i) lane_load[0] += 1.5 * (double)ents[i].P * (double)(1ull << ents[i].m);
    HIPCHK(hipMallocAsync((void **)&ws, off, st));
    auto h2d = [&](size_t o, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(ws + o, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
    };
    HIPCHK(h2d(o_ent, ents.data(), sizeof(batk::BatchEntry) * ents.size()));
    HIPCHK(h2d(o_ist, item_start.data(), sizeof(u64) * item_start.size()));
    HIPCHK(h2d(o_prog, progs.data(), sizeof(u32) * progs.size()));
    HIPCHK(h2d(o_pe, pair_entry.data(), sizeof(u32) * pair_entry.size()));
    HIPCHK(h2d(o_pp, pair_pv.data(), sizeof(u32) * pair_pv.size()));
    HIPCHK(h2d(o_epo, entry_p_off.data(), sizeof(u64) * entry_p_off.size()));
    HIPCHK(h2d(o_p, p, sizeof(double) * (size_t)p_total));
    HIPCHK(hipMemsetAsync(ws + o_ctr, 0, sizeof(unsigned long long), st));

    const batk::BatchEntry *d_ent = (const batk::BatchEntry *)(ws + o_ent);
    rc = events_ready();
    if (rc) return rc;
    HIPCHK(hipEventRecord(t_state.ev[0], st));
    HIPCHK(batk::batched_tables(st, d_ent, (const u32 *)(ws + o_pe), (const u32 *)(ws + o_pp),
                                (const u64 *)(ws + o_epo), (const double *)(ws + o_p), (unsigned)pair_entry.size(),
                                (double *)(ws + o_tab)));
    HIPCHK(hipEventRecord(t_state.ev[1], st));
    batk::BatchParams BP;
    memset(&BP, 0, sizeof BP);
    BP.entries = d_ent;
    BP.item_start = (const u64 *)(ws + o_ist);
    BP.n_entries = (u32)n_gen;
    BP.check_every = opts().check_every.load() >= 2 ? 2u : 1u;
    BP.n_items = n_gen_items;
    BP.prog = (const u32 *)(ws + o_prog);
    BP.tables = (const double *)(ws + o_tab);
    BP.part = (double *)(ws + o_part);
    BP.pcount = (u64 *)(ws + o_pc);
    BP.ctr = (unsigned long long *)(ws + o_ctr);
    // the specialised kernels run on side streams forked from the thread's
    // stream after the tables, so that small ones overlap; joined before
    // the reduction
    if (n_side > 0) {
        HIPCHK(hipEventRecord(SS->fork, st));
        for (int k = 0; k < n_side; ++k) HIPCHK(hipStreamWaitEvent(SS->s[k], SS->fork, 0));
    }
    const int window = opts().window_test.load() != 0 ? 1 : 0;
    for (size_t i = n_gen; i < ents.size(); ++i) {
        const batk::BatchEntry &e = ents[i];
        bat::KParams K;
        memset(&K, 0, sizeof K);
        const u64 iters = 1ull << e.ubits;
        K.c_lo = 0;
        K.c_hi = 1ull << e.m;
        K.g_first = 0;
        K.g_last = iters - 1;
        K.g_base = 0;
        K.g_end = iters - 1;
        K.chunk_iters = 1ull << e.f;  // one segment per work item
        K.n_chunks = e.n_items;
        K.chunk_mul = 1;
        K.chunk_mask = ~0ull;
        K.m = e.m;
        K.ubits = e.ubits;
        K.seg_log = e.f;
        K.check_every = BP.check_every;
        K.chain = e.chain;
        K.ncol = 1;
        K.window_test = (e.chain && window) ? 1u : 0u;
        K.n_nodes = e.n_nodes;
        K.s = e.s;
        K.t = e.t;
        K.tables = (const double *)(ws + o_tab) + e.tab_off;
        K.part = (double *)(ws + o_part) + e.item_begin * batk::kBatchMaxP * 2;
        K.pcount = (u64 *)(ws + o_pc) + e.item_begin;
        const u64 wpb = (u64)batch_waves((int)e.P);
        const u64 blocks = std::min<u64>((u64)D.cus, (e.n_items + wpb - 1) / wpb);
        void *args[] = {&K};
        int k_min = 0;
        for (int k = 1; k <= n_side; ++k)
            if (lane_load[k] < lane_load[k_min]) k_min = k;
        lane_load[k_min] += (double)e.P * (double)(1ull << e.m);
        hipStream_t ls = k_min > 0 ? SS->s[k_min - 1] : st;
        HIPCHK(hipModuleLaunchKernel(spec_fn[i], (unsigned)blocks, 1, 1, (unsigned)(bat::kWave * wpb), 1, 1, 0, ls, args,
                                     nullptr));
    }
    // the generic queue after the specialised kernels (the largest graphs)
    // are queued, behind lane 0's: its persistent blocks then fill the CUs
    // the others leave
    if (n_gen_items > 0) {
        unsigned blocks = (unsigned)std::max<u64>(1, std::min<u64>((u64)D.cus, n_gen_items));
        HIPCHK(batk::batched_sweep(st, blocks, nmax, gen_t, BP));
    }
    for (int k = 0; k < n_side; ++k) {
        HIPCHK(hipEventRecord(SS->join[k], SS->s[k]));
        HIPCHK(hipStreamWaitEvent(st, SS->join[k], 0));
    }
    HIPCHK(hipEventRecord(t_state.ev[2], st));
    HIPCHK(batk::batched_reduce(st, d_ent, (unsigned)ents.size(), (const double *)(ws + o_part),
                                (const u64 *)(ws + o_pc), (u32)n_pvec, (double *)(ws + o_R), (u64 *)(ws + o_cnt)));
    HIPCHK(hipEventRecord(t_state.ev[3], st));
    HIPCHK(hipMemcpyAsync(R_out, ws + o_R, sizeof(double) * (size_t)n_graphs * n_pvec, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(counts_out, ws + o_cnt, sizeof(u64) * (size_t)n_graphs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipFreeAsync(ws, st));
    HIPCHK(hipStreamSynchronize(st));
    bat_launch_info &I = t_state.info;
    memset(&I, 0, sizeof I);
    I.vectors = vectors;
    I.specialised = n_gen < ents.size() ? 1 : 0;
    I.jit_ms = spec_jit_ms;
    I.chunk_log2 = (int32_t)bseg;
    I.n_chunks = (int32_t)std::min<u64>(n_items, 0x7fffffff);
    {
        size_t nrel = 0;
        for (const Plan &pl : plans) nrel += pl.code.size();
        I.relaxations = (int32_t)nrel;
    }
    I.kernel_id = aot_kernel_id(gen_t ? "k_batched_dyn_t" : "k_batched_dyn", (int)nmax, false) ^
                  spec_id;
    I.perm = -1;
    I.chain_log2 = (int32_t)bchain;
    I.check_every = 1;
    I.item_order = 0;
    I.block_waves = (int32_t)gen_waves;
    I.super_restart = 0;
    I.window_test = 0;
    t_state.have_launch = true;
    return BAT_OK;
}

extern "C" int bat_reliability_batched(int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets,
                                       const bat_arc *arcs, const int32_t *s, const int32_t *t, int32_t n_pvec,
                                       const double *p, double *R_out, uint64_t *counts_out)
{
    return batched_impl(n_graphs, n_nodes, arc_offsets, arcs, s, t, n_pvec, p, R_out, counts_out, nullptr);
}

extern "C" int bat_autotune_batched(int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets,
                                    const bat_arc *arcs, const int32_t *s, const int32_t *t, int32_t n_pvec,
                                    const double *p, double *best_kernel_ms)
{
    t_err.clear();
    if (n_graphs <= 0 || !n_nodes || !arc_offsets || !arcs || !s || !t)
        return fail(BAT_EINVAL, "invalid batch description");
    if (n_pvec < 1 || n_pvec > BAT_MAX_PVEC) return fail(BAT_EINVAL, "n_pvec %d outside [1, %d]", n_pvec, BAT_MAX_PVEC);
    DeviceInfo D;
    int rc = current_device(D);
    if (rc) return rc;
    std::vector<double> R((size_t)n_graphs * n_pvec);
    std::vector<uint64_t> cnt((size_t)n_graphs);
    const char *vb = getenv("BAT_AUTOTUNE_VERBOSE");
    const bool verbose = vb && *vb && *vb != '0';
    // the whole batch, each candidate once untimed and then the best of two
    // (a batch is one launch: sampling it would change its load balance)
    double best = 1e300;
    BatchTune bb;
    for (int seg : {6, 5, 4})
        for (int chain : {0, 3, 4, 5, 6}) {
            if (chain > seg) continue;
            const BatchTune c{chain, seg};
            double ms = 1e300;
            for (int rep = 0; rep < 3; ++rep) {
                rc = batched_impl(n_graphs, n_nodes, arc_offsets, arcs, s, t, n_pvec, p, R.data(), cnt.data(), &c);
                if (rc) return rc;
                bat_launch_info li;
                rc = bat_last_launch(&li);
                if (rc) return rc;
                if (rep > 0) ms = std::min(ms, li.kernel_ms);
            }
            if (verbose) fprintf(stderr, "bat_autotune_batched: seg_log2=%d chain=%d -> %.3f ms\n", seg, chain, ms);
            if (ms < best) {
                best = ms;
                bb = c;
            }
        }
    // then graph-specialised kernels for the largest graphs (thresholds on
    // the arc count: the largest, 2 and 4 below it), with the winning
    // segment size and chain length; a threshold must win by 2% over none.
    // (Smaller segments for the specialised graphs, which spread a graph
    // over more wavefronts, measured slower on 256 graphs x 32 p-vectors.)
    if (bb.chain != 0) {
        int32_t m_max = 0;
        for (int32_t g = 0; g < n_graphs; ++g) m_max = std::max(m_max, arc_offsets[g + 1] - arc_offsets[g]);
        const double base = best;
        const BatchTune gen = bb;
        // each threshold with 3, 2 and 1 side streams: which hardware queue
        // a stream lands on depends on the streams the process made before
        // it (torch's default stream, once used, holds one of HIP's 4), and
        // a threshold measured on shared queues loses to a worse one
        for (int arcs_min : {m_max - 4, m_max - 2, m_max}) {
            if (arcs_min < bat::kWordBits + 3) continue;
            for (int ns : {3, 2, 1}) {
                BatchTune c = gen;
                c.jit_arcs = arcs_min;
                c.streams = ns;
                double ms = 1e300;
                for (int rep = 0; rep < 3; ++rep) {
                    rc = batched_impl(n_graphs, n_nodes, arc_offsets, arcs, s, t, n_pvec, p, R.data(), cnt.data(), &c);
                    if (rc) return rc;
                    bat_launch_info li;
                    rc = bat_last_launch(&li);
                    if (rc) return rc;
                    if (rep > 0) ms = std::min(ms, li.kernel_ms);
                }
                if (verbose)
                    fprintf(stderr,
                            "bat_autotune_batched: seg_log2=%d chain=%d specialised from %d arcs on %d side streams "
                            "-> %.3f ms\n",
                            c.seg, c.chain, arcs_min, ns, ms);
                if (ms < best && ms < base * 0.98) {
                    best = ms;
                    bb = c;
                }
            }
        }
        if (bb.jit_arcs < 0) bb.jit_arcs = 0;  // tuned: none
    }
    {
        std::lock_guard<std::mutex> lk(g_btune_mu);
        g_btune[batch_key(D.id, n_graphs, n_nodes, arc_offsets, arcs, s, t, n_pvec)] = bb;
    }
    if (best_kernel_ms) *best_kernel_ms = best;
    t_err.clear();
    return BAT_OK;
}

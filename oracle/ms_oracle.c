/*
 * ms_oracle.c -- CPU reference for multi-state arcs: the BAT over a
 * mixed-radix solution space and a demand-level flow test.
 *
 * TEST INFRASTRUCTURE ONLY, like bat_oracle.c: only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant with the HIP path (nor with
 * bat_oracle.c).
 *
 * The paper treats binary arcs only.  It sizes the solution space of arcs
 * with sigma_i states each as the product of the sigma_i (Section 4.1) and
 * names multi-state network reliability as the problem to extend to next
 * (Section 6), without defining it.  The reading taken here is the usual
 * multi-state flow network one:
 *   - arc i is in one of sigma_i states k = 0..sigma_i-1 with probability
 *     w_i(k) (independent arcs, as the paper's assumption 2 for binary
 *     arcs), and state k gives it the integer capacity cap_i(k);
 *   - a state vector X = (x_1, ..., x_m) meets demand d when the maximum
 *     flow from s to t, with arc i carrying at most cap_i(x_i) units (in
 *     either direction for an undirected arc), is at least d;
 *   - R_d = sum over X meeting d of prod_i w_i(x_i)  (Eq. 1 with the
 *     connectivity test replaced by the flow test).
 * With two states of capacity 0 and 1 and d = 1 this is the binary problem
 * of Eq. 1 exactly: the flow test is then s-t connectivity.
 *
 * Plain, slow and obviously correct:
 *   - enumeration: the backward BAT generalised to sigma_i states.  X starts
 *     at the vector of the range's first index, read as a mixed-radix number
 *     with x_1 most significant (for sigma_i = 2: Eq. 3); every later vector
 *     comes from the generalised Rule 1: the last coordinate below its top
 *     state goes up by one and every coordinate after it returns to state 0.
 *     No coordinate below its top state left ends the space (Rule 2);
 *   - flow test: Edmonds-Karp (breadth-first shortest augmenting paths on
 *     the residual graph), stopping once d units flow or no augmenting path
 *     is left;
 *   - probability: the product of the w_i(x_i), left to right, in IEEE
 *     binary64; sums with Neumaier compensation.
 *
 * Compile with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MS_OK 0
#define MS_EINVAL (-1)
#define MS_ETOOBIG (-2)
#define MS_ENOMEM (-4)

#define MS_MAX_ARCS 62
#define MS_MAX_NODES 4096
#define MS_MAX_STATES 256

/* Number of state vectors, or 0 when it exceeds 2^62. */
static uint64_t ms_space(int32_t m, const int32_t *sigma)
{
    uint64_t N = 1;
    for (int32_t i = 0; i < m; ++i) {
        if ((uint64_t)sigma[i] > (((uint64_t)1 << 62) / N)) return 0;
        N *= (uint64_t)sigma[i];
    }
    return N;
}

int orc_ms_validate(int32_t n, int32_t m, const int32_t *uv, const int32_t *sigma, const int32_t *cap,
                    const double *w, int32_t s, int32_t t, int32_t d)
{
    if (n < 2 || m < 0 || d < 1) return MS_EINVAL;
    if (n > MS_MAX_NODES || m > MS_MAX_ARCS) return MS_ETOOBIG;
    if (s < 0 || s >= n || t < 0 || t >= n || s == t) return MS_EINVAL;
    if (m > 0 && (uv == NULL || sigma == NULL || w == NULL)) return MS_EINVAL;
    int32_t off = 0;
    for (int32_t i = 0; i < m; ++i) {
        if (uv[2 * i] < 0 || uv[2 * i] >= n || uv[2 * i + 1] < 0 || uv[2 * i + 1] >= n) return MS_EINVAL;
        if (sigma[i] < 1 || sigma[i] > MS_MAX_STATES) return MS_EINVAL;
        for (int32_t k = 0; k < sigma[i]; ++k) {
            if (!(w[off + k] >= 0.0 && w[off + k] <= 1.0)) return MS_EINVAL;
            if (cap && cap[off + k] < 0) return MS_EINVAL;
        }
        off += sigma[i];
    }
    if (m > 0 && ms_space(m, sigma) == 0) return MS_ETOOBIG;
    return MS_OK;
}

/* The vector with 0-based index c: mixed radix, x_1 most significant. */
void orc_ms_decode(int32_t m, const int32_t *sigma, uint64_t c, int32_t *x)
{
    for (int32_t k = m - 1; k >= 0; --k) {
        x[k] = (int32_t)(c % (uint64_t)sigma[k]);
        c /= (uint64_t)sigma[k];
    }
}

/* Generalised Rule 1: returns 0 when X was the last vector (Rule 2). */
int orc_ms_next(int32_t m, const int32_t *sigma, int32_t *x)
{
    for (int32_t k = m - 1; k >= 0; --k) {
        if (x[k] + 1 < sigma[k]) {
            x[k] += 1;
            return 1;
        }
        x[k] = 0;
    }
    return 0;
}

/* Residual network of G(X): every arc i becomes a pair of residual edges
 * 2i (u -> v) and 2i+1 (v -> u), each the other's reverse.  An undirected
 * arc of capacity c gives both edges capacity c; a directed one gives the
 * reverse edge capacity 0. */
typedef struct {
    int32_t n, m;
    int32_t *start, *edge;  /* edges leaving each node: edge[start[u] .. start[u+1]) */
    int32_t *head;          /* 2m: head of each residual edge */
    int64_t *res;           /* 2m: residual capacity */
    int32_t *pred, *queue;  /* n: BFS bookkeeping */
} ms_net;

static int ms_net_init(ms_net *g, int32_t n, int32_t m, const int32_t *uv)
{
    memset(g, 0, sizeof *g);
    g->n = n;
    g->m = m;
    g->start = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->edge = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->head = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->res = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
    g->pred = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    g->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!g->start || !g->edge || !g->head || !g->res || !g->pred || !g->queue) return MS_ENOMEM;
    for (int32_t i = 0; i < m; ++i) {
        g->head[2 * i] = uv[2 * i + 1];
        g->head[2 * i + 1] = uv[2 * i];
        g->start[uv[2 * i] + 1]++;
        g->start[uv[2 * i + 1] + 1]++;
    }
    for (int32_t u = 0; u < n; ++u) g->start[u + 1] += g->start[u];
    int32_t *fill = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!fill) return MS_ENOMEM;
    for (int32_t i = 0; i < m; ++i) {
        int32_t u = uv[2 * i], v = uv[2 * i + 1];
        g->edge[g->start[u] + fill[u]++] = 2 * i;
        g->edge[g->start[v] + fill[v]++] = 2 * i + 1;
    }
    free(fill);
    return MS_OK;
}

static void ms_net_free(ms_net *g)
{
    free(g->start); free(g->edge); free(g->head); free(g->res); free(g->pred); free(g->queue);
}

/* Edmonds-Karp from s to t on the residual capacities already set, until
 * `want` units flow or no augmenting path is left; returns the flow found
 * (at most want plus the last path's excess).  *looks counts the residual
 * edges examined by the searches. */
static int64_t ms_maxflow(ms_net *g, int32_t s, int32_t t, int64_t want, int64_t *looks)
{
    int64_t flow = 0;
    while (flow < want) {
        for (int32_t v = 0; v < g->n; ++v) g->pred[v] = -1;
        int32_t qh = 0, qt = 0;
        g->queue[qt++] = s;
        g->pred[s] = 2 * g->m; /* marks s as reached */
        while (qh < qt && g->pred[t] < 0) {
            int32_t u = g->queue[qh++];
            for (int32_t q = g->start[u]; q < g->start[u + 1]; ++q) {
                int32_t e = g->edge[q];
                ++*looks;
                int32_t v = g->head[e];
                if (g->res[e] > 0 && g->pred[v] < 0) {
                    g->pred[v] = e;
                    g->queue[qt++] = v;
                }
            }
        }
        if (g->pred[t] < 0) break; /* no augmenting path: the flow is maximal */
        int64_t b = INT64_MAX;
        for (int32_t v = t; v != s; v = g->head[g->pred[v] ^ 1]) {
            int32_t e = g->pred[v];
            if (g->res[e] < b) b = g->res[e];
        }
        for (int32_t v = t; v != s; v = g->head[g->pred[v] ^ 1]) {
            int32_t e = g->pred[v];
            g->res[e] -= b;
            g->res[e ^ 1] += b;
        }
        flow += b;
    }
    return flow;
}

static void ms_neumaier(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/*
 * The multi-state BAT over 0-based indices [c_lo, c_hi) of the mixed-radix
 * order.  sigma[m]: states per arc; cap and w: sum(sigma) entries, arc 0's
 * states first (cap NULL: state k has capacity k).  Outputs: sum2[2]
 * (sum, compensation) of Pr(X) over X meeting demand d, *count of them,
 * usum2[2] (nullable) over the others, stats[1] (nullable): residual edges
 * examined by the flow searches.
 */
int orc_ms_range(int32_t n, int32_t m, const int32_t *uv, const int32_t *sigma, const int32_t *cap,
                 const double *w, int32_t s, int32_t t, int32_t d, int32_t directed, uint64_t c_lo,
                 uint64_t c_hi, double *sum2, uint64_t *count, double *usum2, int64_t *stats)
{
    int rc = orc_ms_validate(n, m, uv, sigma, cap, w, s, t, d);
    if (rc != MS_OK) return rc;
    const uint64_t N = m > 0 ? ms_space(m, sigma) : 1;
    if (c_lo > c_hi || c_hi > N || sum2 == NULL || count == NULL) return MS_EINVAL;
    int32_t off[MS_MAX_ARCS + 1];
    off[0] = 0;
    for (int32_t i = 0; i < m; ++i) off[i + 1] = off[i] + sigma[i];
    ms_net g;
    if (ms_net_init(&g, n, m, uv) != MS_OK) {
        ms_net_free(&g);
        return MS_ENOMEM;
    }
    int32_t x[MS_MAX_ARCS + 1];
    double s_sum = 0.0, s_cmp = 0.0, u_sum = 0.0, u_cmp = 0.0;
    uint64_t cnt = 0;
    int64_t looks = 0;
    if (c_lo < c_hi) {
        orc_ms_decode(m, sigma, c_lo, x);
        for (uint64_t c = c_lo;;) {
            for (int32_t i = 0; i < m; ++i) {
                int64_t ci = cap ? cap[off[i] + x[i]] : x[i];
                g.res[2 * i] = ci;
                g.res[2 * i + 1] = directed ? 0 : ci;
            }
            int ok = ms_maxflow(&g, s, t, d, &looks) >= d;
            double pr = 1.0;
            for (int32_t i = 0; i < m; ++i) pr = pr * w[off[i] + x[i]];
            if (ok) {
                ++cnt;
                ms_neumaier(&s_sum, &s_cmp, pr);
            } else if (usum2) {
                ms_neumaier(&u_sum, &u_cmp, pr);
            }
            if (++c == c_hi) break;
            orc_ms_next(m, sigma, x);
        }
    }
    sum2[0] = s_sum;
    sum2[1] = s_cmp;
    *count = cnt;
    if (usum2) {
        usum2[0] = u_sum;
        usum2[1] = u_cmp;
    }
    if (stats) stats[0] = looks;
    ms_net_free(&g);
    return MS_OK;
}

/* Maximum flow of one state vector (test helper): the flow is pushed to
 * completion (demand = the sum of all capacities). */
int64_t orc_ms_maxflow(int32_t n, int32_t m, const int32_t *uv, const int64_t *capx, int32_t s, int32_t t,
                       int32_t directed)
{
    ms_net g;
    if (ms_net_init(&g, n, m, uv) != MS_OK) {
        ms_net_free(&g);
        return MS_ENOMEM;
    }
    int64_t total = 0;
    for (int32_t i = 0; i < m; ++i) {
        g.res[2 * i] = capx[i];
        g.res[2 * i + 1] = directed ? 0 : capx[i];
        total += capx[i];
    }
    int64_t looks = 0;
    int64_t f = ms_maxflow(&g, s, t, total + 1, &looks);
    ms_net_free(&g);
    return f;
}

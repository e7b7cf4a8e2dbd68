/*
 * bat_oracle.c -- CPU reference for exact two-terminal reliability by the
 * binary-addition-tree algorithm (BAT) with the PLSA connectivity test.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent oracle that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code, header, table or constant with the HIP path.
 *
 * Plain, slow and obviously correct by construction:
 *   - enumeration: the backward BAT of Section 3.1 -- X starts at the vector
 *     Dec^-1 of the first index of the range (Eq. 3, backward order, x_1 the
 *     most significant coordinate, X_1 = 0) and every later vector comes from
 *     Rule 1 (the last zero coordinate becomes one, all later coordinates
 *     become zero); Rule 2 ends the whole space;
 *   - connectivity: PLSA of Section 3.2 (layers L_1 = {s}, L_l = nodes first
 *     reached from L_{l-1} over working arcs; disconnected when a layer is
 *     empty, connected when the sink enters a layer);
 *   - probability: Pr(X) = prod_i q_i(x_i) with q_i(1) = p_i and
 *     q_i(0) = 1 - p_i, multiplied left to right in IEEE binary64 (Eq. 1;
 *     the per-arc definition printed just before Eq. 1 is garbled into a sum
 *     and is read as this product);
 *   - accumulation: R = sum over connected X of Pr(X) (Eq. 1, STEP B4) with
 *     Neumaier compensated summation;
 *   - gradient (not in the paper; follows from Eq. 1 being multilinear in
 *     p): T1_i = sum_{X conn, x_i = 1} prod_{j != i} q_j(x_j) = R|p_i<-1 and
 *     T0_i likewise with x_i = 0, so dR/dp_i = T1_i - T0_i.  The products
 *     that skip q_i come from prefix and suffix products, so p_i in {0, 1} is
 *     allowed (no division).
 *
 * Readings of the paper (its garbled or silent passages):
 *   - arcs are undirected (Table 6 row (1), the bridge, prints the
 *     undirected value); a directed variant is available by flag;
 *   - PLSA layers exclude nodes already placed in an earlier layer, else a
 *     layer never empties in an undirected graph;
 *   - self-loops and parallel arcs are accepted: Eq. 1 is defined for them;
 *   - m = 0 gives one empty vector, which is disconnected since s != t.
 *
 * Compile with -ffp-contract=off so that no product or sum is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ETOOBIG (-2)
#define ORC_ENOMEM (-4)

#define ORC_MAX_ARCS 62
#define ORC_MAX_NODES 4096

int orc_validate(int32_t n, int32_t m, const int32_t *uv, const double *p,
                 int32_t s, int32_t t)
{
    if (n < 2 || m < 0) return ORC_EINVAL;
    if (n > ORC_MAX_NODES || m > ORC_MAX_ARCS) return ORC_ETOOBIG;
    if (s < 0 || s >= n || t < 0 || t >= n || s == t) return ORC_EINVAL;
    if (m > 0 && (uv == NULL || p == NULL)) return ORC_EINVAL;
    for (int32_t i = 0; i < m; ++i) {
        if (uv[2 * i] < 0 || uv[2 * i] >= n) return ORC_EINVAL;
        if (uv[2 * i + 1] < 0 || uv[2 * i + 1] >= n) return ORC_EINVAL;
        if (!(p[i] >= 0.0 && p[i] <= 1.0)) return ORC_EINVAL; /* rejects NaN too */
    }
    return ORC_OK;
}

/* Eq. 3 (backward BAT, X_1 = 0): the vector with 0-based index c, i.e.
 * x_k = bit (m - k) of c for k = 1..m.  x[k-1] holds x_k. */
void orc_dec_inv(int32_t m, uint64_t c, uint8_t *x)
{
    for (int32_t k = 1; k <= m; ++k) x[k - 1] = (uint8_t)((c >> (m - k)) & 1u);
}

/* Eq. 2 (backward BAT): Dec(X) = sum_k x_k 2^(m-k); the paper's 1-based
 * index of X is Dec(X) + 1. */
uint64_t orc_dec(int32_t m, const uint8_t *x)
{
    uint64_t c = 0;
    for (int32_t k = 1; k <= m; ++k) c = (c << 1) | (uint64_t)(x[k - 1] & 1u);
    return c;
}

/* Forward BAT (Section 4.2, Eq. 4-5 with the worked examples there:
 * X_3 = (0,1,0,0,0,0) and X_31 = (0,1,1,1,1,0) when X_1 = 0): coordinate
 * x_1 is the least significant, x_k = bit (k - 1) of the 0-based index. */
void orc_dec_inv_fwd(int32_t m, uint64_t c, uint8_t *x)
{
    for (int32_t k = 1; k <= m; ++k) x[k - 1] = (uint8_t)((c >> (k - 1)) & 1u);
}

/* The forward update: Rule 1 applied from the first coordinate, i.e. the
 * first zero-valued coordinate becomes one and every coordinate before it
 * becomes zero.  Returns 0 when no zero coordinate is left. */
int orc_bat_next_fwd(int32_t m, uint8_t *x)
{
    for (int32_t k = 1; k <= m; ++k) {
        if (x[k - 1] == 0) {
            x[k - 1] = 1;
            return 1;
        }
        x[k - 1] = 0;
    }
    return 0;
}

/* One BAT update (Section 3.1, STEPs B1-B3): Rule 1 turns the last
 * zero-valued coordinate into one and every coordinate after it into zero.
 * Returns 1 if X was updated, 0 if no zero coordinate exists (Rule 2: all
 * vectors have been generated). */
int orc_bat_next(int32_t m, uint8_t *x)
{
    if (m <= 0) return 0;
    int32_t k = m; /* k restarts at m after every update (STEPs B0, B1) */
    for (;;) {
        if (x[k - 1] == 0) { /* STEP B1: X(a_k) = 1, X is updated */
            x[k - 1] = 1;
            return 1;
        }
        if (k == 1) return 0; /* STEP B2: halt */
        x[k - 1] = 0;         /* STEP B3: X(a_k) = 0, k = k - 1 */
        --k;
    }
}

/* Incidence lists of G(V, E): for node u, the arcs that can be traversed
 * out of u (both endpoints for undirected arcs, the tail only when
 * directed). */
typedef struct {
    int32_t n;
    int32_t *start; /* n + 1 */
    int32_t *arc;   /* arc index */
    int32_t *other; /* the node reached over that arc */
} orc_incidence;

static int orc_incidence_build(orc_incidence *g, int32_t n, int32_t m, const int32_t *uv,
                               int32_t directed)
{
    g->n = n;
    g->start = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g->arc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    g->other = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    if (!g->start || !g->arc || !g->other) return ORC_ENOMEM;
    for (int32_t i = 0; i < m; ++i) {
        int32_t u = uv[2 * i], v = uv[2 * i + 1];
        g->start[u + 1]++;
        if (!directed && v != u) g->start[v + 1]++;
    }
    for (int32_t u = 0; u < n; ++u) g->start[u + 1] += g->start[u];
    int32_t *fill = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!fill) return ORC_ENOMEM;
    for (int32_t i = 0; i < m; ++i) {
        int32_t u = uv[2 * i], v = uv[2 * i + 1];
        int32_t pos = g->start[u] + fill[u]++;
        g->arc[pos] = i;
        g->other[pos] = v;
        if (!directed && v != u) {
            pos = g->start[v] + fill[v]++;
            g->arc[pos] = i;
            g->other[pos] = u;
        }
    }
    free(fill);
    return ORC_OK;
}

static void orc_incidence_free(orc_incidence *g)
{
    free(g->start);
    free(g->arc);
    free(g->other);
}

/* PLSA (Section 3.2, STEPs P0-P4) on G(X).  Returns 1 if s and t are
 * connected, 0 if not.  *layers receives the number of layers built,
 * *inspections the number of (node, incident arc) pairs examined.
 * layer_of (nullable, n entries) receives each node's 1-based layer, 0 if
 * never reached. */
static int orc_plsa_core(const orc_incidence *g, const uint8_t *x, int32_t s, int32_t t,
                         int32_t *layer_of, int32_t *cur, int32_t *nxt,
                         int32_t *layers, int64_t *inspections)
{
    for (int32_t v = 0; v < g->n; ++v) layer_of[v] = 0;
    int32_t ncur = 1, l = 1;
    cur[0] = s; /* STEP P0: L_1 = {s}, l = 2 */
    layer_of[s] = 1;
    int64_t insp = 0;
    for (;;) {
        ++l;
        int32_t nnext = 0;
        /* STEP P1: L_l = nodes not yet in a layer, joined by a working arc
         * to a node of L_{l-1} */
        for (int32_t a = 0; a < ncur; ++a) {
            int32_t u = cur[a];
            for (int32_t q = g->start[u]; q < g->start[u + 1]; ++q) {
                ++insp;
                if (!x[g->arc[q]]) continue;
                int32_t v = g->other[q];
                if (layer_of[v]) continue;
                layer_of[v] = l;
                nxt[nnext++] = v;
            }
        }
        if (nnext == 0) { /* STEP P2 */
            *layers = l - 1;
            *inspections = insp;
            return 0;
        }
        if (layer_of[t]) { /* STEP P3 */
            *layers = l;
            *inspections = insp;
            return 1;
        }
        memcpy(cur, nxt, sizeof(int32_t) * (size_t)nnext); /* STEP P4 */
        ncur = nnext;
    }
}

int orc_plsa(int32_t n, int32_t m, const int32_t *uv, const uint8_t *x, int32_t s, int32_t t,
             int32_t directed, int32_t *layers, int64_t *inspections, int32_t *layer_of_out)
{
    if (n < 2 || m < 0 || s < 0 || s >= n || t < 0 || t >= n || s == t) return ORC_EINVAL;
    orc_incidence g;
    int rc = orc_incidence_build(&g, n, m, uv, directed);
    int32_t *lay = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (rc != ORC_OK || !lay || !cur || !nxt) {
        orc_incidence_free(&g);
        free(lay); free(cur); free(nxt);
        return ORC_ENOMEM;
    }
    int32_t L = 0;
    int64_t I = 0;
    int conn = orc_plsa_core(&g, x, s, t, lay, cur, nxt, &L, &I);
    if (layers) *layers = L;
    if (inspections) *inspections = I;
    if (layer_of_out) memcpy(layer_of_out, lay, sizeof(int32_t) * (size_t)n);
    orc_incidence_free(&g);
    free(lay); free(cur); free(nxt);
    return conn;
}

/* Pr(X) = prod_{i=1..m} q_i(x_i), left to right. */
double orc_pr(int32_t m, const double *p, const uint8_t *x)
{
    double w = 1.0;
    for (int32_t i = 0; i < m; ++i) w = w * (x[i] ? p[i] : (1.0 - p[i]));
    return w;
}

/* Neumaier's improvement of Kahan summation: (*s + *c) carries the sum. */
static void orc_neumaier(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

/*
 * BAT over the 0-based index range [c_lo, c_hi) of the backward order.
 * Outputs (all may be NULL except where stated):
 *   sum2[2]      : (sum, compensation) of Pr(X) over connected X  (required)
 *   count        : number of connected X                           (required)
 *   usum2[2]     : (sum, compensation) over disconnected X
 *   T1[2m], T0[2m]: per arc i, (sum, compensation) pairs at [2i], [2i+1]
 *                  of prod_{j != i} q_j over connected X with x_i = 1 / 0
 *   stats[2]     : total PLSA layers and arc inspections over the range
 */
int orc_range_order(int32_t n, int32_t m, const int32_t *uv, const double *p, int32_t s, int32_t t,
                    int32_t directed, int32_t forward, uint64_t c_lo, uint64_t c_hi, double *sum2,
                    uint64_t *count, double *usum2, double *T1, double *T0, int64_t *stats);

int orc_range(int32_t n, int32_t m, const int32_t *uv, const double *p, int32_t s, int32_t t,
              int32_t directed, uint64_t c_lo, uint64_t c_hi, double *sum2, uint64_t *count,
              double *usum2, double *T1, double *T0, int64_t *stats)
{
    return orc_range_order(n, m, uv, p, s, t, directed, 0, c_lo, c_hi, sum2, count, usum2, T1, T0, stats);
}

/* orc_range with a choice of index order: forward = 0 is the backward BAT
 * of Section 3.1 (Eq. 2-3), forward = 1 the forward BAT of Section 4.2
 * (Eq. 4-5). */
int orc_range_order(int32_t n, int32_t m, const int32_t *uv, const double *p, int32_t s, int32_t t,
                    int32_t directed, int32_t forward, uint64_t c_lo, uint64_t c_hi, double *sum2,
                    uint64_t *count, double *usum2, double *T1, double *T0, int64_t *stats)
{
    int rc = orc_validate(n, m, uv, p, s, t);
    if (rc != ORC_OK) return rc;
    uint64_t total = (uint64_t)1 << m;
    if (c_lo > c_hi || c_hi > total || sum2 == NULL || count == NULL) return ORC_EINVAL;

    orc_incidence g;
    if (orc_incidence_build(&g, n, m, uv, directed) != ORC_OK) {
        orc_incidence_free(&g);
        return ORC_ENOMEM;
    }
    uint8_t x[ORC_MAX_ARCS + 1];
    double pre[ORC_MAX_ARCS + 2], suf[ORC_MAX_ARCS + 2];
    int32_t *lay = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!lay || !cur || !nxt) {
        orc_incidence_free(&g);
        free(lay); free(cur); free(nxt);
        return ORC_ENOMEM;
    }
    int grad = (T1 != NULL && T0 != NULL);
    double s_sum = 0.0, s_cmp = 0.0, u_sum = 0.0, u_cmp = 0.0;
    uint64_t cnt = 0;
    int64_t tot_layers = 0, tot_insp = 0;
    if (grad)
        for (int32_t i = 0; i < 2 * m; ++i) T1[i] = T0[i] = 0.0;

    if (c_lo < c_hi) {
        if (forward)
            orc_dec_inv_fwd(m, c_lo, x); /* the first vector of the range, Eq. 5 */
        else
            orc_dec_inv(m, c_lo, x); /* the first vector of the range, Eq. 3 */
        for (uint64_t c = c_lo;;) {
            int32_t L = 0;
            int64_t I = 0;
            int conn = orc_plsa_core(&g, x, s, t, lay, cur, nxt, &L, &I);
            tot_layers += L;
            tot_insp += I;
            if (conn) { /* STEP B4 */
                ++cnt;
                orc_neumaier(&s_sum, &s_cmp, orc_pr(m, p, x));
                if (grad) {
                    pre[0] = 1.0;
                    for (int32_t i = 0; i < m; ++i) pre[i + 1] = pre[i] * (x[i] ? p[i] : (1.0 - p[i]));
                    suf[m] = 1.0;
                    for (int32_t i = m - 1; i >= 0; --i) suf[i] = (x[i] ? p[i] : (1.0 - p[i])) * suf[i + 1];
                    for (int32_t i = 0; i < m; ++i) {
                        double w = pre[i] * suf[i + 1];
                        if (x[i])
                            orc_neumaier(&T1[2 * i], &T1[2 * i + 1], w);
                        else
                            orc_neumaier(&T0[2 * i], &T0[2 * i + 1], w);
                    }
                }
            } else if (usum2) {
                orc_neumaier(&u_sum, &u_cmp, orc_pr(m, p, x));
            }
            if (++c == c_hi) break;
            if (forward)
                orc_bat_next_fwd(m, x);
            else
                orc_bat_next(m, x); /* Rule 1 */
        }
    }
    sum2[0] = s_sum;
    sum2[1] = s_cmp;
    *count = cnt;
    if (usum2) {
        usum2[0] = u_sum;
        usum2[1] = u_cmp;
    }
    if (stats) {
        stats[0] = tot_layers;
        stats[1] = tot_insp;
    }
    orc_incidence_free(&g);
    free(lay); free(cur); free(nxt);
    return ORC_OK;
}

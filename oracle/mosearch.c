/*
 * Oracle: sequential multiobjective label-setting search.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links or calls this
 * file; it exists to state, in plain sequential code, the result the
 * wavefront search of Sec. 3 (Alg. 3, Explore) is after, so that the GPU path
 * can be compared with it.
 *
 * What is computed.  A plan is a walk from the root; its label is folded along
 * the walk in float32 (Alg. 3, the child line: cost plus edge cost, heuristic
 * PH of the parent plan extended by the edge):
 *     c'     = c + c_e
 *     d_pre  = d + delta_e          the perception-heuristic drift (Sec. 4.1)
 *     keep only if d_pre <= beta    the heuristic cutoff of Alg. 3 / eq. (2)
 *     d'     = reset(v) ? 0 : d_pre relocalisation at a feature-rich node
 *     m'     = max(m, d_pre)        third objective, max drift so far (n_obj 3)
 * Every operation is a separately rounded float32 operation.  RemoveDominated
 * (Sec. 3) is read as weak Pareto dominance: a label a removes b at the same
 * head when every component of a is <= the one of b; of equal vectors one is
 * kept.  The result is the set of Pareto-minimal label vectors at every node
 * (which Alg. 3 builds up in P(x)) and, from it, the goal front.
 *
 * How.  Martins' multicriteria label-setting method: labels are taken from a
 * binary heap in lexicographic order of (c, d, m); a taken label that some
 * permanent label at its node weakly dominates is discarded, otherwise it is
 * made permanent and its children along every out-edge are generated; a child
 * that fails the cutoff or is weakly dominated by a permanent label at its
 * target is dropped.  Because every child has strictly larger cost than its
 * parent (edge costs are positive and large enough not to vanish in the
 * float32 sum), a label's dominators are always taken before it.  A guard
 * counts any violation of that order (it must stay zero).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no fused multiply-add,
 * IEEE float32 round-to-nearest).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float c, d, m;
    int32_t node;
    int32_t parent; /* arena index of the parent label, -1 for the root */
    int64_t seq;    /* insertion order, last tie-breaker */
} tlab;

typedef struct {
    int32_t n;
    int32_t nobj;
    /* arena of permanent labels */
    float *c, *d, *m;
    int32_t *node, *parent;
    int64_t len, cap;
    /* per-node lists of permanent labels (arena indices) */
    int32_t **perm;
    int32_t *pn, *pcap;
    /* heap */
    tlab *heap;
    int64_t hn, hcap;
    int64_t seq;
    /* counters */
    int64_t violations, pushes, pops;
    int status;
} mo_state;

static int lex_less(const tlab *a, const tlab *b) {
    if (a->c != b->c) return a->c < b->c;
    if (a->d != b->d) return a->d < b->d;
    if (a->m != b->m) return a->m < b->m;
    if (a->node != b->node) return a->node < b->node;
    return a->seq < b->seq;
}

static int heap_push(mo_state *s, tlab x) {
    if (s->hn == s->hcap) {
        int64_t nc = s->hcap ? 2 * s->hcap : 1024;
        tlab *h = (tlab *)realloc(s->heap, (size_t)nc * sizeof(tlab));
        if (!h) return -1;
        s->heap = h;
        s->hcap = nc;
    }
    int64_t i = s->hn++;
    s->heap[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!lex_less(&s->heap[i], &s->heap[p])) break;
        tlab t = s->heap[i];
        s->heap[i] = s->heap[p];
        s->heap[p] = t;
        i = p;
    }
    s->pushes++;
    return 0;
}

static tlab heap_pop(mo_state *s) {
    tlab top = s->heap[0];
    s->hn--;
    if (s->hn > 0) {
        s->heap[0] = s->heap[s->hn];
        int64_t i = 0;
        for (;;) {
            int64_t l = 2 * i + 1, r = l + 1, b = i;
            if (l < s->hn && lex_less(&s->heap[l], &s->heap[b])) b = l;
            if (r < s->hn && lex_less(&s->heap[r], &s->heap[b])) b = r;
            if (b == i) break;
            tlab t = s->heap[i];
            s->heap[i] = s->heap[b];
            s->heap[b] = t;
            i = b;
        }
    }
    s->pops++;
    return top;
}

/* a weakly dominates (c, d, m): every component <= */
static int weakly_dominates(const mo_state *s, int32_t a, float c, float d, float m) {
    if (s->c[a] > c) return 0;
    if (s->d[a] > d) return 0;
    if (s->nobj >= 3 && s->m[a] > m) return 0;
    return 1;
}

static int dominated_at(const mo_state *s, int32_t v, float c, float d, float m) {
    const int32_t *p = s->perm[v];
    for (int32_t k = 0; k < s->pn[v]; ++k)
        if (weakly_dominates(s, p[k], c, d, m)) return 1;
    return 0;
}

static int arena_push(mo_state *s, const tlab *x) {
    if (s->len == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 4096;
        float *c = (float *)realloc(s->c, (size_t)nc * sizeof(float));
        if (!c) return -1;
        s->c = c;
        float *d = (float *)realloc(s->d, (size_t)nc * sizeof(float));
        if (!d) return -1;
        s->d = d;
        float *m = (float *)realloc(s->m, (size_t)nc * sizeof(float));
        if (!m) return -1;
        s->m = m;
        int32_t *nd = (int32_t *)realloc(s->node, (size_t)nc * sizeof(int32_t));
        if (!nd) return -1;
        s->node = nd;
        int32_t *pa = (int32_t *)realloc(s->parent, (size_t)nc * sizeof(int32_t));
        if (!pa) return -1;
        s->parent = pa;
        s->cap = nc;
    }
    s->c[s->len] = x->c;
    s->d[s->len] = x->d;
    s->m[s->len] = x->m;
    s->node[s->len] = x->node;
    s->parent[s->len] = x->parent;
    s->len++;
    return 0;
}

static int perm_push(mo_state *s, int32_t v, int32_t a) {
    if (s->pn[v] == s->pcap[v]) {
        int32_t nc = s->pcap[v] ? 2 * s->pcap[v] : 4;
        int32_t *p = (int32_t *)realloc(s->perm[v], (size_t)nc * sizeof(int32_t));
        if (!p) return -1;
        s->perm[v] = p;
        s->pcap[v] = nc;
    }
    s->perm[v][s->pn[v]++] = a;
    return 0;
}

void mo_free(void *h) {
    mo_state *s = (mo_state *)h;
    if (!s) return;
    free(s->c);
    free(s->d);
    free(s->m);
    free(s->node);
    free(s->parent);
    if (s->perm)
        for (int32_t v = 0; v < s->n; ++v) free(s->perm[v]);
    free(s->perm);
    free(s->pn);
    free(s->pcap);
    free(s->heap);
    free(s);
}

/*
 * Run the search.  status: 0 ok, 1 label limit exceeded, 2 out of memory,
 * 3 invalid arguments.  Returns a handle (free with mo_free) or NULL.
 */
void *mo_run(int32_t n, const int32_t *row_ptr, const int32_t *col, const float *cost,
             const float *drift, const uint8_t *reset, float beta, int32_t nobj, int32_t root,
             int64_t max_labels, int32_t *status) {
    *status = 3;
    if (n <= 0 || root < 0 || root >= n || (nobj != 2 && nobj != 3)) return NULL;
    mo_state *s = (mo_state *)calloc(1, sizeof(mo_state));
    if (!s) {
        *status = 2;
        return NULL;
    }
    s->n = n;
    s->nobj = nobj;
    s->perm = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
    s->pn = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    s->pcap = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!s->perm || !s->pn || !s->pcap) goto oom;

    tlab root_lab = {0.0f, 0.0f, 0.0f, root, -1, s->seq++};
    if (heap_push(s, root_lab)) goto oom;

    while (s->hn > 0) {
        tlab l = heap_pop(s);
        if (dominated_at(s, l.node, l.c, l.d, l.m)) continue;
        /* guard: a new permanent label must not strictly dominate an older one */
        for (int32_t k = 0; k < s->pn[l.node];) {
            int32_t a = s->perm[l.node][k];
            int le = (l.c <= s->c[a]) && (l.d <= s->d[a]) && (nobj < 3 || l.m <= s->m[a]);
            if (le) {
                s->violations++;
                s->perm[l.node][k] = s->perm[l.node][--s->pn[l.node]];
            } else {
                ++k;
            }
        }
        int32_t id = (int32_t)s->len;
        if (arena_push(s, &l)) goto oom;
        if (perm_push(s, l.node, id)) goto oom;
        if (max_labels > 0 && s->len > max_labels) {
            *status = 1;
            return s;
        }
        for (int32_t e = row_ptr[l.node]; e < row_ptr[l.node + 1]; ++e) {
            int32_t v = col[e];
            float c2 = l.c + cost[e];
            float dpre = l.d + drift[e];
            if (!(dpre <= beta)) continue;
            float d2 = reset[v] ? 0.0f : dpre;
            float m2 = 0.0f;
            if (nobj >= 3) m2 = (l.m > dpre) ? l.m : dpre;
            if (dominated_at(s, v, c2, d2, m2)) continue;
            tlab ch = {c2, d2, m2, v, id, s->seq++};
            if (heap_push(s, ch)) goto oom;
        }
    }
    *status = 0;
    return s;
oom:
    *status = 2;
    mo_free(s);
    return NULL;
}

int64_t mo_num_labels(void *h) { return ((mo_state *)h)->len; }

void mo_copy_arena(void *h, float *c, float *d, float *m, int32_t *node, int32_t *parent) {
    mo_state *s = (mo_state *)h;
    memcpy(c, s->c, (size_t)s->len * sizeof(float));
    memcpy(d, s->d, (size_t)s->len * sizeof(float));
    memcpy(m, s->m, (size_t)s->len * sizeof(float));
    memcpy(node, s->node, (size_t)s->len * sizeof(int32_t));
    memcpy(parent, s->parent, (size_t)s->len * sizeof(int32_t));
}

/* Per-node fronts: off[n+1] prefix offsets, lab[] arena indices in the order
 * the labels became permanent (which is lexicographic order). */
void mo_copy_fronts(void *h, int64_t *off, int32_t *lab) {
    mo_state *s = (mo_state *)h;
    off[0] = 0;
    for (int32_t v = 0; v < s->n; ++v) {
        memcpy(lab + off[v], s->perm[v], (size_t)s->pn[v] * sizeof(int32_t));
        off[v + 1] = off[v] + s->pn[v];
    }
}

/* out: [0] permanent labels in fronts, [1] arena labels, [2] violations,
 *      [3] heap pushes, [4] heap pops */
void mo_counters(void *h, int64_t *out) {
    mo_state *s = (mo_state *)h;
    int64_t x = 0;
    for (int32_t v = 0; v < s->n; ++v) x += s->pn[v];
    out[0] = x;
    out[1] = s->len;
    out[2] = s->violations;
    out[3] = s->pushes;
    out[4] = s->pops;
}

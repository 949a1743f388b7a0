/*
 * ac_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded, deliberately unoptimised CPU reference for
 * multi-pattern exact string matching. Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it. The GPU library shares no
 * code, header or table with this file and never calls it.
 *
 * What it computes: for patterns P_0..P_{n-1} (pattern id = input index) and a
 * text T[0..N-1], every pair (e, k) such that P_k ends at position e of T,
 * i.e. T[e-|P_k|+1 .. e] == P_k (abstract and Sec. I of the paper: find all
 * occurrences of a set of patterns in a string). Each pair is reported as the
 * 64-bit key (e << 32) | k; sorting the keys numerically orders the pairs by
 * (e, k).
 *
 * Two matchers are provided, both following the paper's Sec. II:
 *
 *  1. ac_scan: the Aho-Corasick machine with failure links (Sec. II.A, Fig. 1).
 *     Step 1 builds the machine: a goto function (the trie of the patterns,
 *     states numbered in the order the patterns insert them, root = 0), a
 *     failure function and an output function. Step 2 reads the text once; on
 *     a byte with no goto edge it follows failure links and re-reads the same
 *     byte until an edge exists (or the root is reached), then emits the
 *     output set of the state it lands in.
 *
 *  2. pfac_scan: the failure-less machine of Sec. II.B / Sec. IV.A (Figs. 2-6).
 *     The machine is the goto function alone. A walk is started at every text
 *     position; each walk follows goto edges from the root, emits the
 *     patterns that end exactly at each state it enters, and stops at the
 *     first byte with no edge.
 *
 * Representation: the goto function is a dense table go[s*256 + a] over all
 * 256 byte values (-1 = no edge). Output sets are small growable arrays.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NO_EDGE (-1)

typedef struct {
    int32_t *v;
    int32_t n, cap;
} ivec;

static int ivec_push(ivec *a, int32_t x) {
    if (a->n == a->cap) {
        int32_t nc = a->cap ? 2 * a->cap : 2;
        int32_t *nv = (int32_t *)realloc(a->v, (size_t)nc * sizeof(int32_t));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

typedef struct oracle_ac {
    int32_t *go;      /* goto function: go[s*256 + a], NO_EDGE if undefined */
    int32_t *fail;    /* failure function */
    int32_t *depth;   /* length of the string spelled from the root to s */
    ivec *own;        /* ids of the patterns that end exactly at s */
    ivec *out;        /* output function: own(s) plus out(fail(s)), ascending */
    int32_t n_states, cap_states;
    uint32_t n_patterns;
    int32_t m_max;
} oracle_ac;

static int new_state(oracle_ac *m) {
    if (m->n_states == m->cap_states) {
        int32_t nc = m->cap_states ? 2 * m->cap_states : 64;
        int32_t *go = (int32_t *)realloc(m->go, (size_t)nc * 256 * sizeof(int32_t));
        if (!go) return -1;
        m->go = go;
        int32_t *dp = (int32_t *)realloc(m->depth, (size_t)nc * sizeof(int32_t));
        if (!dp) return -1;
        m->depth = dp;
        ivec *own = (ivec *)realloc(m->own, (size_t)nc * sizeof(ivec));
        if (!own) return -1;
        m->own = own;
        m->cap_states = nc;
    }
    int32_t s = m->n_states++;
    for (int a = 0; a < 256; a++) m->go[(size_t)s * 256 + a] = NO_EDGE;
    m->depth[s] = 0;
    m->own[s].v = NULL;
    m->own[s].n = m->own[s].cap = 0;
    return s;
}

void oracle_ac_free(oracle_ac *m) {
    if (!m) return;
    if (m->own)
        for (int32_t s = 0; s < m->n_states; s++) free(m->own[s].v);
    if (m->out)
        for (int32_t s = 0; s < m->n_states; s++) free(m->out[s].v);
    free(m->own);
    free(m->out);
    free(m->go);
    free(m->fail);
    free(m->depth);
    free(m);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Step 1 of the algorithm (Sec. II): construct the machine.
 * pat: concatenated pattern bytes; off: n+1 offsets; pattern k is
 * pat[off[k] .. off[k+1]). Returns NULL if n == 0, a pattern is empty, the
 * offsets are not non-decreasing, or memory runs out. */
oracle_ac *oracle_ac_build(const uint8_t *pat, const uint64_t *off, uint32_t n) {
    if (n == 0 || !pat || !off) return NULL;
    for (uint32_t k = 0; k < n; k++)
        if (off[k + 1] <= off[k]) return NULL; /* empty pattern or bad offsets */

    oracle_ac *m = (oracle_ac *)calloc(1, sizeof(oracle_ac));
    if (!m) return NULL;
    m->n_patterns = n;
    if (new_state(m) != 0) goto fail_out; /* the root, state 0 */

    /* goto function: insert the patterns in id order; a byte with no edge
     * gets a new state numbered one past the last (the numbering the paper's
     * Fig. 1 and Fig. 6 walk-throughs use). */
    for (uint32_t k = 0; k < n; k++) {
        int32_t s = 0;
        int32_t len = (int32_t)(off[k + 1] - off[k]);
        if (len > m->m_max) m->m_max = len;
        for (uint64_t i = off[k]; i < off[k + 1]; i++) {
            uint8_t a = pat[i];
            int32_t t = m->go[(size_t)s * 256 + a];
            if (t == NO_EDGE) {
                t = new_state(m);
                if (t < 0) goto fail_out;
                m->go[(size_t)s * 256 + a] = t;
                m->depth[t] = m->depth[s] + 1;
            }
            s = t;
        }
        if (ivec_push(&m->own[s], (int32_t)k)) goto fail_out;
    }

    /* failure and output functions, computed breadth first so that the
     * failure state of every state is finished before the state itself. */
    int32_t S = m->n_states;
    m->fail = (int32_t *)calloc((size_t)S, sizeof(int32_t));
    m->out = (ivec *)calloc((size_t)S, sizeof(ivec));
    int32_t *queue = (int32_t *)malloc((size_t)S * sizeof(int32_t));
    if (!m->fail || !m->out || !queue) { free(queue); goto fail_out; }
    int32_t head = 0, tail = 0;
    queue[tail++] = 0;
    m->fail[0] = 0;
    while (head < tail) {
        int32_t s = queue[head++];
        /* out(s) = own(s) U out(fail(s)); fail(s) is shallower, so done. */
        for (int32_t i = 0; i < m->own[s].n; i++)
            if (ivec_push(&m->out[s], m->own[s].v[i])) { free(queue); goto fail_out; }
        if (s != 0) {
            ivec *f = &m->out[m->fail[s]];
            for (int32_t i = 0; i < f->n; i++)
                if (ivec_push(&m->out[s], f->v[i])) { free(queue); goto fail_out; }
        }
        if (m->out[s].n > 1) qsort(m->out[s].v, (size_t)m->out[s].n, sizeof(int32_t), cmp_i32);

        for (int a = 0; a < 256; a++) {
            int32_t t = m->go[(size_t)s * 256 + a];
            if (t == NO_EDGE) continue;
            queue[tail++] = t;
            if (s == 0) {
                m->fail[t] = 0; /* states one byte deep fail to the root */
                continue;
            }
            /* follow failure links from fail(s) until a state with an edge
             * on a, or the root; fail(t) is that edge's target (or the root). */
            int32_t r = m->fail[s];
            while (r != 0 && m->go[(size_t)r * 256 + a] == NO_EDGE) r = m->fail[r];
            int32_t g = m->go[(size_t)r * 256 + a];
            m->fail[t] = (g != NO_EDGE && g != t) ? g : 0;
        }
    }
    free(queue);
    return m;

fail_out:
    oracle_ac_free(m);
    return NULL;
}

int32_t oracle_ac_states(const oracle_ac *m) { return m->n_states; }
int32_t oracle_ac_m_max(const oracle_ac *m) { return m->m_max; }
int32_t oracle_ac_fail(const oracle_ac *m, int32_t s) { return m->fail[s]; }
int32_t oracle_ac_goto(const oracle_ac *m, int32_t s, int32_t a) {
    return m->go[(size_t)s * 256 + (a & 255)];
}

typedef struct {
    uint64_t *v;
    uint64_t n, cap;
} kvec;

static int kvec_push(kvec *a, uint64_t x) {
    if (a->n == a->cap) {
        uint64_t nc = a->cap ? 2 * a->cap : 1024;
        uint64_t *nv = (uint64_t *)realloc(a->v, nc * sizeof(uint64_t));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

void oracle_buf_free(uint64_t *p) { free(p); }

/* Step 2 (Sec. II.A): one pass over the text with failure links.
 * Writes a malloc'd array of (e << 32) | k keys to *res (free with
 * oracle_buf_free) and returns how many; -1 on allocation failure.
 * If trace is non-NULL, trace[i] receives the state after byte i. */
int64_t oracle_ac_scan(const oracle_ac *m, const uint8_t *text, uint64_t n,
                       uint64_t **res, int32_t *trace) {
    kvec out = {0, 0, 0};
    int32_t s = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint8_t a = text[i];
        /* no valid transition: take failure links, re-reading the same byte */
        while (s != 0 && m->go[(size_t)s * 256 + a] == NO_EDGE) s = m->fail[s];
        int32_t g = m->go[(size_t)s * 256 + a];
        s = (g == NO_EDGE) ? 0 : g;
        if (trace) trace[i] = s;
        for (int32_t j = 0; j < m->out[s].n; j++)
            if (kvec_push(&out, (i << 32) | (uint32_t)m->out[s].v[j])) {
                free(out.v);
                return -1;
            }
    }
    *res = out.v;
    return (int64_t)out.n;
}

/* The failure-less walk of Sec. II.B / IV.A started at text position p:
 * follows goto edges from the root and stops at the first byte with no edge.
 * Appends each entered state to states[] (up to cap) and each pattern that
 * ends exactly at an entered state to *out. Returns the number of states
 * entered. */
static int64_t pfac_walk(const oracle_ac *m, const uint8_t *text, uint64_t n, uint64_t p,
                         kvec *out, int32_t *states, int64_t cap) {
    int32_t s = 0;
    int64_t steps = 0;
    for (uint64_t j = p; j < n; j++) {
        int32_t t = m->go[(size_t)s * 256 + text[j]];
        if (t == NO_EDGE) break;
        s = t;
        if (states && steps < cap) states[steps] = s;
        steps++;
        if (out)
            for (int32_t i = 0; i < m->own[s].n; i++)
                if (kvec_push(out, (j << 32) | (uint32_t)m->own[s].v[i])) return -1;
    }
    return steps;
}

int64_t oracle_pfac_walk(const oracle_ac *m, const uint8_t *text, uint64_t n, uint64_t p,
                         int32_t *states, int64_t cap) {
    if (p >= n) return 0;
    return pfac_walk(m, text, n, p, NULL, states, cap);
}

/* Failure-less matching over every start position 0..n-1 (in start order, so
 * the keys come out unsorted). Same result contract as oracle_ac_scan. */
int64_t oracle_pfac_scan(const oracle_ac *m, const uint8_t *text, uint64_t n, uint64_t **res) {
    kvec out = {0, 0, 0};
    for (uint64_t p = 0; p < n; p++)
        if (pfac_walk(m, text, n, p, &out, NULL, 0) < 0) {
            free(out.v);
            return -1;
        }
    *res = out.v;
    return (int64_t)out.n;
}

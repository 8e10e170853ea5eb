/*
 * cos_oracle.c -- TEST INFRASTRUCTURE ONLY (never part of the product path).
 *
 * Plain, slow CPU reference for the per-configuration sum of connected
 * bare-U diagrams of the SU(N) Hubbard model computed by CoS / SB-CoS
 * (arXiv 2507.12349).  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it.  It shares no code, header or
 * table with the HIP library under paper_2507_12349_amd/.
 *
 * Conventions (Methods, Alg. 1-3 input: n interaction pairs, N = 2n points,
 * interaction lines I = {(i, i+n)}; matrices indexed by (point-1) mod n):
 *   n vertices, points p in [0, 2n), vertex(p) = p mod n,
 *   partner(p) = (p + n) mod 2n.
 *   variant 0 ("U"): one matrix G[n][n]; every closed cycle carries w * nf
 *                    (uniform SU(N): the close factor of Alg. 2 is -N_f).
 *   variant 1 ("F"): nf matrices G[l][n][n]; every cycle carries a flavour l
 *                    and the factor w (Alg. 3, "close cycle" rule).
 *   stubs (SB-CoS shift heads, Results / Alg. 3): a point may instead be a
 *   one-point "shift" cycle of weight -sigma[l], l = flavour of the cycle
 *   through its partner; at most one stub per vertex.  Variant U uses the
 *   single weight sigma[0].
 *   Only connected diagrams count: the graph on vertices whose edges join
 *   the vertices of each cycle must be connected (Results, CoS-2).
 *
 * Every routine is compiled twice: REAL = long double (reference, suffix
 * _ld) and REAL = double (timed CPU baseline, suffix _d).
 *
 * Routines
 *   O1  brute_*  : the definition, by enumerating stub sets, permutations
 *                  cycle by cycle and one flavour per cycle, with an explicit
 *                  connectivity test (Results, "Theoretical Constructions").
 *   O3  dp_*     : vertex-level dynamic programme with merged contact states
 *                  and shift heads folded into the partner's first visit
 *                  (Results, CoS-2 with visited sets, state merging for
 *                  contact interactions, SB-CoS typed heads; Alg. 3), plus
 *                  its reverse (adjoint) sweep over stored layers.
 *   O3L alg3_*   : Alg. 3 taken step by step at point level, states keyed by
 *                  ((head, type, flavour), current, R, U) without any
 *                  canonicalisation.
 */
#ifndef REAL
#define REAL long double
#define SFX(name) name##_ld
#define ORACLE_SECOND_PASS 1
#endif

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_COMMON_DEFINED
#define ORACLE_COMMON_DEFINED
#define MAXN 12
#define MAXF 16

static int ipow3(int k) { int r = 1; while (k-- > 0) r *= 3; return r; }

/* union-find over vertices */
static int uf_find(int *p, int x) { while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; } return x; }
static void uf_join(int *p, int a, int b) { a = uf_find(p, a); b = uf_find(p, b); if (a != b) p[a] = b; }

/* ---- simple open-addressing hash map: uint64 key -> index into a value array ---- */
typedef struct {
    uint64_t *keys;   /* key+1, 0 = empty */
    int64_t *slot;    /* index into vals */
    int64_t cap, count;
} hmap_t;

static void hm_init(hmap_t *h, int64_t cap0) {
    int64_t cap = 16; while (cap < 2 * cap0) cap <<= 1;
    h->cap = cap; h->count = 0;
    h->keys = (uint64_t *)calloc((size_t)cap, sizeof(uint64_t));
    h->slot = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
}
static void hm_free(hmap_t *h) { free(h->keys); free(h->slot); h->keys = NULL; h->slot = NULL; h->cap = h->count = 0; }
static uint64_t hm_hash(uint64_t k) { k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ULL; k ^= k >> 33; return k; }
/* returns slot index; *isnew set when inserted with index newidx */
static int64_t hm_get_or_insert(hmap_t *h, uint64_t key, int64_t newidx, int *isnew) {
    if (2 * (h->count + 1) > h->cap) {
        hmap_t g; hm_init(&g, h->cap);
        for (int64_t i = 0; i < h->cap; i++) if (h->keys[i]) {
            uint64_t k = h->keys[i] - 1; int64_t j = (int64_t)(hm_hash(k) & (uint64_t)(g.cap - 1));
            while (g.keys[j]) j = (j + 1) & (g.cap - 1);
            g.keys[j] = k + 1; g.slot[j] = h->slot[i]; g.count++;
        }
        hm_free(h); *h = g;
    }
    int64_t j = (int64_t)(hm_hash(key) & (uint64_t)(h->cap - 1));
    while (h->keys[j]) {
        if (h->keys[j] == key + 1) { *isnew = 0; return h->slot[j]; }
        j = (j + 1) & (h->cap - 1);
    }
    h->keys[j] = key + 1; h->slot[j] = newidx; h->count++; *isnew = 1; return newidx;
}
static int64_t hm_find(const hmap_t *h, uint64_t key) {
    if (!h->cap) return -1;
    int64_t j = (int64_t)(hm_hash(key) & (uint64_t)(h->cap - 1));
    while (h->keys[j]) { if (h->keys[j] == key + 1) return h->slot[j]; j = (j + 1) & (h->cap - 1); }
    return -1;
}
typedef struct {
    int64_t states, ext, closes, stub_edges, masks;
} oracle_counts_t;
#endif /* ORACLE_COMMON_DEFINED */

/* matrix element G_l[a][b] (U: l ignored) */
#define GEL(G, variant, n, l, a, b) ((REAL)(G)[((variant) ? (size_t)(l) * (n) * (n) : 0) + (size_t)(a) * (n) + (b)])

/* ======================================================================
 * O1: brute force over the definition.
 * ====================================================================== */
typedef struct {
    int n, npts, nf, variant, use_stubs, connected_only;
    const double *G, *stub;
    REAL w;
    int is_stub[2 * MAXN];
    int nxt[2 * MAXN];        /* permutation of the non-stub points */
    int cyc_of[2 * MAXN];     /* cycle id of each non-stub point */
    int flav_of_cyc[2 * MAXN];
    int ncyc;
    REAL acc;
} SFX(bf_t);

static void SFX(bf_leaf)(SFX(bf_t) *s, REAL prod) {
    int n = s->n, par[MAXN];
    for (int k = 0; k < n; k++) par[k] = k;
    for (int p = 0; p < s->npts; p++) if (!s->is_stub[p]) uf_join(par, p % n, s->nxt[p] % n);
    if (s->connected_only) {
        int r = uf_find(par, 0);
        for (int k = 1; k < n; k++) if (uf_find(par, k) != r) return;
    }
    for (int p = 0; p < s->npts; p++) if (s->is_stub[p]) {
        int q = (p + n) % s->npts;             /* partner is a cycle point */
        int l = s->variant ? s->flav_of_cyc[s->cyc_of[q]] : 0;
        prod *= -(REAL)s->stub[l];
    }
    s->acc += prod;
}

static void SFX(bf_cycles)(SFX(bf_t) *s, uint32_t used, REAL prod);

/* extend the open cycle (head, cur, flavour l) or close it */
static void SFX(bf_extend)(SFX(bf_t) *s, uint32_t used, int head, int cur, int l, REAL prod) {
    int n = s->n;
    /* close: cur -> head */
    s->nxt[cur] = head;
    SFX(bf_cycles)(s, used, prod * GEL(s->G, s->variant, n, l, cur % n, head % n));
    /* continue to any unused non-stub point */
    for (int q = 0; q < s->npts; q++) {
        if ((used >> q) & 1u || s->is_stub[q]) continue;
        s->nxt[cur] = q;
        s->cyc_of[q] = s->cyc_of[head];
        SFX(bf_extend)(s, used | (1u << q), head, q, l, prod * GEL(s->G, s->variant, n, l, cur % n, q % n));
    }
}

/* open a new cycle at the lowest unused non-stub point, one flavour at a time */
static void SFX(bf_cycles)(SFX(bf_t) *s, uint32_t used, REAL prod) {
    int start = -1;
    for (int q = 0; q < s->npts; q++) if (!((used >> q) & 1u) && !s->is_stub[q]) { start = q; break; }
    if (start < 0) { SFX(bf_leaf)(s, prod); return; }
    int c = s->ncyc++;
    s->cyc_of[start] = c;
    if (s->variant == 0) {
        s->flav_of_cyc[c] = 0;
        SFX(bf_extend)(s, used | (1u << start), start, start, 0, prod * s->w * (REAL)s->nf);
    } else {
        for (int l = 0; l < s->nf; l++) {
            s->flav_of_cyc[c] = l;
            SFX(bf_extend)(s, used | (1u << start), start, start, l, prod * s->w);
        }
    }
    s->ncyc--;
}

/* O1: returns the connected sum (connected_only=1) or the full sum a(V) (=0). */
REAL SFX(cos_oracle_brute)(int n, int nf, int variant, int use_stubs, const double *G,
                           const double *stub, double w, int connected_only) {
    SFX(bf_t) s;
    memset(&s, 0, sizeof(s));
    s.n = n; s.npts = 2 * n; s.nf = nf; s.variant = variant; s.use_stubs = use_stubs;
    s.connected_only = connected_only; s.G = G; s.stub = stub; s.w = (REAL)w;
    int nchoice = use_stubs ? ipow3(n) : 1;
    REAL total = 0;
    for (int code = 0; code < nchoice; code++) {
        int c = code;
        for (int k = 0; k < n; k++) {
            int d = c % 3; c /= 3;
            s.is_stub[k] = (d == 1);
            s.is_stub[k + n] = (d == 2);
        }
        s.acc = 0; s.ncyc = 0;
        SFX(bf_cycles)(&s, 0u, (REAL)1);
        total += s.acc;
    }
    return total;
}

/* ======================================================================
 * O3: vertex-level DP.  State (u, l, v, m): u = head vertex of the open
 * cycle, l = its flavour (variant U: 0), v = current vertex, m in {0,1,2}^n
 * = number of visited points per vertex (base-3 code).  Level = sum(m).
 * Rules (one per paragraph of the Results section and Alg. 3):
 *   start  : F(0,l,0,e_0) = 1 for every l; with stubs also
 *            F(0,l,0,2e_0) = -2 sigma_l (either point of vertex 0 is a
 *            shift head whose colour is that of the cycle through the other).
 *   extend : for w with m_w < 2: F(u,l,w,m+e_w) += c_w G_l[v][w] F,
 *            c_w = 2 if m_w = 0 (either point of w), 1 if m_w = 1.
 *   stub   : for w with m_w = 0: F(u,l,w,m+2e_w) += 2 G_l[v][w] (-sigma_l) F
 *            (the other point of w becomes a shift head of colour l).
 *   close  : t = W G_l[v][u] F with W = w*nf (U) or w (F).  If m is full,
 *            S += t.  Else h = min{k : m_k = 1}; if it exists,
 *            F(h,l',h,m+e_h) += t for every flavour l' (U: one slot);
 *            otherwise the visited set is closed and the path is dropped
 *            (it would be disconnected).
 * ====================================================================== */
typedef struct {
    int64_t n_states;      /* stored states */
    uint64_t *key;         /* packed key per state */
    REAL *val;             /* forward value */
    hmap_t map;
} SFX(layer_t);

static uint64_t SFX(pack)(int u, int l, int v, int code) {
    return ((uint64_t)(uint32_t)code << 16) | ((uint64_t)u << 10) | ((uint64_t)l << 5) | (uint64_t)v;
}
static void SFX(unpack)(uint64_t k, int *u, int *l, int *v, int *code) {
    *v = (int)(k & 31u); *l = (int)((k >> 5) & 31u); *u = (int)((k >> 10) & 63u); *code = (int)(k >> 16);
}

static void SFX(layer_add)(SFX(layer_t) *L, uint64_t key, REAL x) {
    int isnew;
    int64_t idx = hm_get_or_insert(&L->map, key, L->n_states, &isnew);
    if (isnew) {
        if ((L->n_states & (L->n_states - 1)) == 0) {   /* grow at powers of two */
            int64_t cap = L->n_states ? 2 * L->n_states : 1;
            L->key = (uint64_t *)realloc(L->key, (size_t)cap * sizeof(uint64_t));
            L->val = (REAL *)realloc(L->val, (size_t)cap * sizeof(REAL));
        }
        L->key[idx] = key; L->val[idx] = 0; L->n_states++;
    }
    L->val[idx] += x;
}

/* Runs the forward DP; optionally keeps all layers (for the reverse sweep).
 * Returns S.  counts may be NULL.  Layers are indexed by level 1..2n. */
static REAL SFX(dp_forward)(int n, int nf, int variant, int use_stubs, const double *G,
                            const double *stub, double w, SFX(layer_t) *layers,
                            oracle_counts_t *counts) {
    int p3[MAXN + 1];
    for (int k = 0; k <= n; k++) p3[k] = ipow3(k);
    int full = 0; for (int k = 0; k < n; k++) full += 2 * p3[k];
    int nfs = variant ? nf : 1;                     /* flavour slots */
    REAL W = (REAL)w * (variant ? (REAL)1 : (REAL)nf);
    for (int lv = 0; lv <= 2 * n + 1; lv++) { memset(&layers[lv], 0, sizeof(layers[lv])); hm_init(&layers[lv].map, 64); }
    for (int l = 0; l < nfs; l++) {
        SFX(layer_add)(&layers[1], SFX(pack)(0, l, 0, 1), (REAL)1);
        if (use_stubs) SFX(layer_add)(&layers[2], SFX(pack)(0, l, 0, 2), -(REAL)2 * (REAL)stub[variant ? l : 0]);
    }
    REAL S = 0;
    oracle_counts_t cnt = {0, 0, 0, 0, 0};
    for (int lv = 1; lv <= 2 * n; lv++) {
        SFX(layer_t) *L = &layers[lv];
        for (int64_t i = 0; i < L->n_states; i++) {
            int u, l, v, code; SFX(unpack)(L->key[i], &u, &l, &v, &code);
            REAL f = L->val[i];
            int m[MAXN]; { int c = code; for (int k = 0; k < n; k++) { m[k] = c % 3; c /= 3; } }
            if (l == 0 || !variant) cnt.states++;
            /* extend and stub */
            for (int x = 0; x < n; x++) {
                if (m[x] >= 2) continue;
                REAL g = GEL(G, variant, n, l, v, x);
                REAL cw = (m[x] == 0) ? (REAL)2 : (REAL)1;
                SFX(layer_add)(&layers[lv + 1], SFX(pack)(u, l, x, code + p3[x]), cw * g * f);
                if (l == 0 || !variant) cnt.ext++;
                if (use_stubs && m[x] == 0) {
                    REAL sg = (REAL)stub[variant ? l : 0];
                    SFX(layer_add)(&layers[lv + 2], SFX(pack)(u, l, x, code + 2 * p3[x]), (REAL)2 * g * (-sg) * f);
                    if (l == 0 || !variant) cnt.stub_edges++;
                }
            }
            /* close */
            REAL t = W * GEL(G, variant, n, l, v, u) * f;
            if (l == 0 || !variant) cnt.closes++;
            if (code == full) { S += t; continue; }
            int h = -1; for (int k = 0; k < n; k++) if (m[k] == 1) { h = k; break; }
            if (h < 0) continue;
            for (int l2 = 0; l2 < nfs; l2++)
                SFX(layer_add)(&layers[lv + 1], SFX(pack)(h, l2, h, code + p3[h]), t);
        }
    }
    if (counts) {
        /* distinct masks over all levels */
        int64_t nm = 0;
        char *seen = (char *)calloc((size_t)p3[n], 1);
        for (int lv = 1; lv <= 2 * n; lv++)
            for (int64_t i = 0; i < layers[lv].n_states; i++) {
                int u, l, v, code; SFX(unpack)(layers[lv].key[i], &u, &l, &v, &code);
                if (!seen[code]) { seen[code] = 1; nm++; }
            }
        free(seen);
        cnt.masks = nm;
        *counts = cnt;
    }
    return S;
}

static void SFX(free_layers)(SFX(layer_t) *layers, int n) {
    for (int lv = 0; lv <= 2 * n + 1; lv++) { free(layers[lv].key); free(layers[lv].val); hm_free(&layers[lv].map); }
}

/* O3 forward.  out_counts (5 int64: states, extensions, closes, stub edges,
 * masks; per flavour slot) may be NULL. */
REAL SFX(cos_oracle_dp)(int n, int nf, int variant, int use_stubs, const double *G,
                        const double *stub, double w, int64_t *out_counts) {
    SFX(layer_t) *layers = (SFX(layer_t) *)calloc((size_t)(2 * n + 2), sizeof(SFX(layer_t)));
    oracle_counts_t c;
    REAL S = SFX(dp_forward)(n, nf, variant, use_stubs, G, stub, w, layers, out_counts ? &c : NULL);
    if (out_counts) { out_counts[0] = c.states; out_counts[1] = c.ext; out_counts[2] = c.closes; out_counts[3] = c.stub_edges; out_counts[4] = c.masks; }
    SFX(free_layers)(layers, n);
    free(layers);
    return S;
}

/* O3 reverse sweep: dS/dG (same layout as G) and dS/dsigma ([nf] for F,
 * [1] for U).  B(s) = dS/dF(s), taken over all layers in reverse level
 * order; each transition s -> s' with coefficient a(G, sigma) adds
 * a * B(s') to B(s) and F(s) * B(s') * da/dG to Gbar. */
REAL SFX(cos_oracle_dp_adjoint)(int n, int nf, int variant, int use_stubs, const double *G,
                                const double *stub, double w, REAL *Gbar, REAL *stubbar) {
    int p3[MAXN + 1];
    for (int k = 0; k <= n; k++) p3[k] = ipow3(k);
    int full = 0; for (int k = 0; k < n; k++) full += 2 * p3[k];
    int nfs = variant ? nf : 1;
    int nG = variant ? nf : 1;
    REAL W = (REAL)w * (variant ? (REAL)1 : (REAL)nf);
    SFX(layer_t) *layers = (SFX(layer_t) *)calloc((size_t)(2 * n + 2), sizeof(SFX(layer_t)));
    REAL S = SFX(dp_forward)(n, nf, variant, use_stubs, G, stub, w, layers, NULL);
    for (int i = 0; i < nG * n * n; i++) Gbar[i] = 0;
    for (int i = 0; i < nfs; i++) stubbar[i] = 0;
    REAL **B = (REAL **)calloc((size_t)(2 * n + 2), sizeof(REAL *));
    for (int lv = 0; lv <= 2 * n + 1; lv++) B[lv] = (REAL *)calloc((size_t)(layers[lv].n_states + 1), sizeof(REAL));
#define GB(l, a, b) Gbar[((variant) ? (size_t)(l) * n * n : 0) + (size_t)(a) * n + (b)]
    for (int lv = 2 * n; lv >= 1; lv--) {
        SFX(layer_t) *L = &layers[lv];
        for (int64_t i = 0; i < L->n_states; i++) {
            int u, l, v, code; SFX(unpack)(L->key[i], &u, &l, &v, &code);
            REAL f = L->val[i], b = 0;
            int m[MAXN]; { int c = code; for (int k = 0; k < n; k++) { m[k] = c % 3; c /= 3; } }
            for (int x = 0; x < n; x++) {
                if (m[x] >= 2) continue;
                REAL g = GEL(G, variant, n, l, v, x);
                REAL cw = (m[x] == 0) ? (REAL)2 : (REAL)1;
                int64_t j = hm_find(&layers[lv + 1].map, SFX(pack)(u, l, x, code + p3[x]));
                if (j >= 0) { REAL bt = B[lv + 1][j]; b += cw * g * bt; GB(l, v, x) += cw * f * bt; }
                if (use_stubs && m[x] == 0) {
                    REAL sg = (REAL)stub[variant ? l : 0];
                    int64_t j2 = hm_find(&layers[lv + 2].map, SFX(pack)(u, l, x, code + 2 * p3[x]));
                    if (j2 >= 0) {
                        REAL bt = B[lv + 2][j2];
                        b += (REAL)2 * g * (-sg) * bt;
                        GB(l, v, x) += (REAL)2 * (-sg) * f * bt;
                        stubbar[variant ? l : 0] += -(REAL)2 * g * f * bt;
                    }
                }
            }
            /* close */
            REAL tbar = 0;
            if (code == full) tbar = 1;
            else {
                int h = -1; for (int k = 0; k < n; k++) if (m[k] == 1) { h = k; break; }
                if (h >= 0)
                    for (int l2 = 0; l2 < nfs; l2++) {
                        int64_t j = hm_find(&layers[lv + 1].map, SFX(pack)(h, l2, h, code + p3[h]));
                        if (j >= 0) tbar += B[lv + 1][j];
                    }
            }
            b += W * GEL(G, variant, n, l, v, u) * tbar;
            GB(l, v, u) += W * f * tbar;
            B[lv][i] = b;
        }
    }
    /* start term F(0,l,0,2e_0) = -2 sigma_l */
    if (use_stubs)
        for (int l = 0; l < nfs; l++) {
            int64_t j = hm_find(&layers[2].map, SFX(pack)(0, l, 0, 2));
            if (j >= 0) stubbar[variant ? l : 0] += -(REAL)2 * B[2][j];
        }
#undef GB
    for (int lv = 0; lv <= 2 * n + 1; lv++) free(B[lv]);
    free(B);
    SFX(free_layers)(layers, n);
    free(layers);
    return S;
}

/* Connected sums of every vertex subset that contains vertex 0, read off the
 * same DP: a close at a mask with no half-visited vertex ends a connected
 * component made of the vertices with m_k = 2 (Results, CoS-2: a new head
 * must hang on an interaction line of the visited part).  out[bits] for
 * bits = subset bitmask (bit 0 set); entries for other bitmasks are 0. */
void SFX(cos_oracle_dp_subsets)(int n, int nf, int variant, int use_stubs, const double *G,
                                const double *stub, double w, REAL *out) {
    int p3[MAXN + 1];
    for (int k = 0; k <= n; k++) p3[k] = ipow3(k);
    int nfs = variant ? nf : 1;
    REAL W = (REAL)w * (variant ? (REAL)1 : (REAL)nf);
    for (int b = 0; b < (1 << n); b++) out[b] = 0;
    SFX(layer_t) *layers = (SFX(layer_t) *)calloc((size_t)(2 * n + 2), sizeof(SFX(layer_t)));
    (void)SFX(dp_forward)(n, nf, variant, use_stubs, G, stub, w, layers, NULL);
    for (int lv = 1; lv <= 2 * n; lv++)
        for (int64_t i = 0; i < layers[lv].n_states; i++) {
            int u, l, v, code; SFX(unpack)(layers[lv].key[i], &u, &l, &v, &code);
            int m[MAXN], c = code, ones = 0, bits = 0;
            for (int k = 0; k < n; k++) { m[k] = c % 3; c /= 3; if (m[k] == 1) ones++; if (m[k] == 2) bits |= 1 << k; }
            if (ones) continue;
            out[bits] += W * GEL(G, variant, n, l, v, u) * layers[lv].val[i];
        }
    (void)nfs;
    SFX(free_layers)(layers, n);
    free(layers);
}

/* ======================================================================
 * O3L: Alg. 3 at point level, no canonicalisation.  Key fields:
 *   head point u, head type tu (0 normal, 1 shift), head flavour lu,
 *   current point v, visited set R (bitmask over 2n points),
 *   unpaired set U: per point a code 0 = absent, else 1 + type*MAXF + flavour.
 * Reading of the printed rules (listed in the design notes):
 *   - a new normal head is keyed with its flavour for each l in Lambda and
 *     the shift head with the partner's flavour (the printed key omits them);
 *   - a shift head is offered only when its partner is a normal point.
 * ====================================================================== */
typedef struct { int u, tu, lu, v; uint32_t R; uint8_t U[2 * MAXN]; } SFX(a3state_t);

typedef struct {
    SFX(a3state_t) *st; REAL *val; int64_t n, cap;
    int64_t *tab; int64_t tcap;           /* open-addressing index: -1 = empty */
} SFX(a3layer_t);

static uint64_t SFX(a3_hash)(const SFX(a3state_t) *s, int npts) {
    uint64_t h = 1469598103934665603ULL;
    int f[4] = {s->u, s->tu, s->lu, s->v};
    for (int i = 0; i < 4; i++) { h ^= (uint64_t)(f[i] + 7); h *= 1099511628211ULL; }
    h ^= s->R; h *= 1099511628211ULL;
    for (int i = 0; i < npts; i++) { h ^= s->U[i]; h *= 1099511628211ULL; }
    return hm_hash(h);
}
static int SFX(a3_eq)(const SFX(a3state_t) *t, const SFX(a3state_t) *s, int npts) {
    return t->u == s->u && t->tu == s->tu && t->lu == s->lu && t->v == s->v && t->R == s->R &&
           memcmp(t->U, s->U, (size_t)npts) == 0;
}
static void SFX(a3_add)(SFX(a3layer_t) *L, const SFX(a3state_t) *s, int npts, REAL x) {
    if (2 * (L->n + 1) > L->tcap) {                 /* rebuild the index */
        int64_t cap = L->tcap ? 2 * L->tcap : 128;
        free(L->tab);
        L->tab = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
        for (int64_t i = 0; i < cap; i++) L->tab[i] = -1;
        L->tcap = cap;
        for (int64_t i = 0; i < L->n; i++) {
            int64_t j = (int64_t)(SFX(a3_hash)(&L->st[i], npts) & (uint64_t)(cap - 1));
            while (L->tab[j] >= 0) j = (j + 1) & (cap - 1);
            L->tab[j] = i;
        }
    }
    int64_t j = (int64_t)(SFX(a3_hash)(s, npts) & (uint64_t)(L->tcap - 1));
    while (L->tab[j] >= 0) {
        if (SFX(a3_eq)(&L->st[L->tab[j]], s, npts)) { L->val[L->tab[j]] += x; return; }
        j = (j + 1) & (L->tcap - 1);
    }
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->st = (SFX(a3state_t) *)realloc(L->st, (size_t)L->cap * sizeof(SFX(a3state_t)));
        L->val = (REAL *)realloc(L->val, (size_t)L->cap * sizeof(REAL));
    }
    L->st[L->n] = *s; L->val[L->n] = x; L->tab[j] = L->n; L->n++;
}

REAL SFX(cos_oracle_alg3)(int n, int nf, int variant, int use_stubs, const double *G,
                          const double *stub, double w) {
    int N = 2 * n;
    /* Alg. 3 carries explicit flavours; variant U is the same algorithm with
     * G_l = G for every l and the cycle factor w applied per cycle. */
    SFX(a3layer_t) *V = (SFX(a3layer_t) *)calloc((size_t)N, sizeof(SFX(a3layer_t)));
    int ntypes = use_stubs ? 2 : 1;
#define A3G(l, a, b) GEL(G, variant, n, l, (a) % n, (b) % n)
#define SIG(l) ((REAL)stub[variant ? (l) : 0])
    for (int l = 0; l < nf; l++)
        for (int tp = 0; tp < ntypes; tp++) {
            SFX(a3state_t) s; memset(&s, 0, sizeof(s));
            s.u = 0; s.tu = tp; s.lu = l; s.v = 0; s.R = 1u;
            s.U[0] = (uint8_t)(1 + tp * MAXF + l);
            SFX(a3_add)(&V[0], &s, N, (REAL)1);
        }
    for (int i = 0; i <= N - 2; i++) {
        for (int64_t k = 0; k < V[i].n; k++) {
            SFX(a3state_t) s = V[i].st[k];
            REAL om = V[i].val[k];
            /* Rule 1: continue the cycle (normal heads only) */
            if (s.tu == 0) {
                for (int x = 0; x < N; x++) {
                    if ((s.R >> x) & 1u) continue;
                    SFX(a3state_t) t = s;
                    t.R = s.R | (1u << x);
                    int px = (x + n) % N;
                    if (s.U[px]) t.U[px] = 0;
                    else t.U[x] = (uint8_t)(1 + 0 * MAXF + s.lu);
                    t.v = x;
                    SFX(a3_add)(&V[i + 1], &t, N, om * A3G(s.lu, s.v, x));
                }
            }
            /* Rule 2: close the cycle, open the next head */
            /* the printed close factor is -1 per cycle; w generalises it for
             * normal cycles, a shift head always closes with -sigma */
            REAL omc = (s.tu == 0) ? om * A3G(s.lu, s.v, s.u) * (REAL)w : -om * SIG(s.lu);
            int h = -1;
            for (int p = 0; p < N; p++) if (s.U[p]) { int q = (p + n) % N; if (h < 0 || q < h) h = q; }
            if (h >= 0) {
                int ph = (h + n) % N;
                int code = s.U[ph] - 1, tph = code / MAXF, lph = code % MAXF;
                SFX(a3state_t) t = s;
                t.R = s.R | (1u << h);
                t.U[ph] = 0;
                t.u = h; t.v = h;
                if (tph == 1) {                       /* partner is a shift head: inherit its colour */
                    t.tu = 0; t.lu = lph; SFX(a3_add)(&V[i + 1], &t, N, omc);
                } else {
                    for (int l = 0; l < nf; l++) { t.tu = 0; t.lu = l; SFX(a3_add)(&V[i + 1], &t, N, omc); }
                    if (use_stubs) { t.tu = 1; t.lu = lph; SFX(a3_add)(&V[i + 1], &t, N, omc); }
                }
            }
        }
    }
    REAL S = 0;
    for (int64_t k = 0; k < V[N - 1].n; k++) {
        SFX(a3state_t) s = V[N - 1].st[k];
        S += V[N - 1].val[k] * ((s.tu == 0) ? A3G(s.lu, s.v, s.u) * (REAL)w : -SIG(s.lu));
    }
#undef A3G
#undef SIG
    for (int i = 0; i < N; i++) { free(V[i].st); free(V[i].val); free(V[i].tab); }
    free(V);
    return S;
}

/* ---- second pass: the same routines in double precision ---- */
#ifdef ORACLE_SECOND_PASS
#undef ORACLE_SECOND_PASS
#undef REAL
#undef SFX
#undef GEL
#define REAL double
#define SFX(name) name##_d
#include "cos_oracle.c"
#endif

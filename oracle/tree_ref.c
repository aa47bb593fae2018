/*
 * tree_ref.c -- reference adaptive quadtree over targets plus image sources,
 * and its U/V/W/X interaction lists.  CPU ORACLE: test infrastructure only;
 * nothing in the GPU library links, includes or calls this file.
 *
 * Algorithm 1 (Section 2.2) builds one adaptive tree over the target points
 * and the image source points, and the FMM uses the interaction lists of the
 * classic adaptive FMM.  The paper leaves the details
 * open; this file fixes them (the "tree spec") so that a second, independent
 * build can be compared with it bit for bit:
 *
 *  Root      x_lo = min x, S = max(max x - x_lo, 2 max y) (1 if that is 0).  The
 *            root square is [x_lo, x_lo + S] x [-S/2, S/2]: symmetric about y = 0,
 *            so every box below the root lies wholly in one half plane, and the
 *            lower half is the exact mirror image of the upper half.
 *  Cells     L = 30 bits per axis (27 for an instance of a forest), scale = 2^L / S (one
 *            IEEE division).
 *            ix = clamp(floor((x - x_lo) * scale), 0, 2^L - 1)
 *            iy_up = clamp(floor(y * scale), 0, 2^(L-1) - 1)
 *            iy = 2^(L-1) + iy_up for a point, 2^(L-1) - 1 - iy_up for its image.
 *  Keys      Morton key: bit 2b = bit b of ix, bit 2b+1 = bit b of iy.  Points are
 *            sorted by (key, input index).
 *  Boxes     a box is (level l, bx, by) = cells >> (L - l).  The root always
 *            splits; a box at level l >= 1 splits iff it holds more than
 *            leaf_size points and l < max_level.  Only nonempty boxes exist.
 *            Image boxes mirror upper boxes: (l, bx, 2^l - 1 - by).
 *  Order     upper boxes are numbered by (level, key prefix); the image of box
 *            k is referred to as (k, image).
 *  Adjacent  the closed integer spans [b 2^(L-l), (b+1) 2^(L-l)] of two boxes
 *            intersect in x and in y (touching at a corner counts).
 *  Lists     for an upper target box b (c ranges over upper AND image boxes):
 *            V(b) = { c : level c = level b, c not adjacent to b,
 *                         parent(c) adjacent to parent(b) }
 *            U(b) = { leaf c : c adjacent to b }                  (b a leaf)
 *            W(b) = { c : level c > level b, c not adjacent to b,
 *                         parent(c) adjacent to b }               (b a leaf)
 *            X(b) = { leaf c : level c < level b, c not adjacent to b,
 *                         c adjacent to parent(b) }
 *            Entries are stored as 2*k + image and sorted ascending.
 *
 * The lists are found by testing these predicates literally on every box that
 * meets the square of side 3 * size(parent(b)) centred on parent(b), which
 * contains every box any of the four predicates can accept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Cell bits per axis of the build in progress (set by tree_ref_build; one build at a time). */
static int LBITS = 30;

typedef struct Node {
    int level;
    int64_t bx, by;          /* full-tree integer box coordinates */
    int64_t first, count;    /* range in sorted point order */
    int64_t prefix;          /* Morton key >> 2(L - level) */
    struct Node *child[4];
    int nchild;
    struct Node *parent;     /* NULL for the root */
    int leaf;
    int index;               /* canonical index (-1 for the root) */
} Node;

typedef struct {
    int64_t key;
    int64_t idx;
} KeyIdx;

typedef struct {
    int64_t n;
    int leaf_size, max_level;
    double x_lo, S, scale;
    KeyIdx *sorted;
    Node *root;
    Node **boxes;            /* all non-root nodes; canonical order after sorting */
    int nbox;
    int cap;
    /* CSR lists: 0=U 1=V 2=W 3=X */
    int64_t *off[4];
    int32_t *ent[4];
    int64_t len[4];
} TreeRef;

static int64_t interleave(int64_t ix, int64_t iy) {
    int64_t k = 0;
    for (int b = 0; b < LBITS; ++b) {
        k |= ((ix >> b) & 1LL) << (2 * b);
        k |= ((iy >> b) & 1LL) << (2 * b + 1);
    }
    return k;
}

static int cmp_keyidx(const void *a, const void *b) {
    const KeyIdx *u = (const KeyIdx *)a, *v = (const KeyIdx *)b;
    if (u->key != v->key) return u->key < v->key ? -1 : 1;
    if (u->idx != v->idx) return u->idx < v->idx ? -1 : 1;
    return 0;
}

static Node *new_node(TreeRef *t) {
    if (t->nbox == t->cap) {
        int nc = t->cap ? 2 * t->cap : 1024;
        Node **p = (Node **)realloc(t->boxes, (size_t)nc * sizeof(Node *));
        if (!p) return NULL;
        t->boxes = p;
        t->cap = nc;
    }
    Node *n = (Node *)calloc(1, sizeof(Node));
    if (!n) return NULL;
    t->boxes[t->nbox++] = n;
    return n;
}

static int build_rec(TreeRef *t, Node *nd) {
    int split = (nd->level == 0) ||
                (nd->count > t->leaf_size && nd->level < t->max_level);
    if (!split) {
        nd->leaf = 1;
        return 0;
    }
    nd->leaf = 0;
    int shift = 2 * (LBITS - (nd->level + 1));
    int64_t i = nd->first, end = nd->first + nd->count;
    while (i < end) {
        int64_t digit = (t->sorted[i].key >> shift) & 3;
        int64_t j = i;
        while (j < end && ((t->sorted[j].key >> shift) & 3) == digit) ++j;
        Node *c = new_node(t);
        if (!c) return -1;
        c->level = nd->level + 1;
        c->bx = 2 * nd->bx + (digit & 1);
        c->by = 2 * nd->by + (digit >> 1);
        c->first = i;
        c->count = j - i;
        c->prefix = t->sorted[i].key >> shift;
        c->parent = nd;
        c->index = -1;
        nd->child[nd->nchild++] = c;
        if (build_rec(t, c)) return -1;
        i = j;
    }
    return 0;
}

static int cmp_node(const void *a, const void *b) {
    const Node *u = *(Node *const *)a, *v = *(Node *const *)b;
    if (u->level != v->level) return u->level < v->level ? -1 : 1;
    if (u->prefix != v->prefix) return u->prefix < v->prefix ? -1 : 1;
    return 0;
}

/* A box reference: node plus half flag.  The image of node k is (k, 1). */
typedef struct {
    const Node *nd;
    int img;
} Ref;

static void span(const Ref *r, int64_t *x0, int64_t *x1, int64_t *y0, int64_t *y1) {
    int64_t w = (int64_t)1 << (LBITS - r->nd->level);
    int64_t by = r->img ? (((int64_t)1 << r->nd->level) - 1 - r->nd->by) : r->nd->by;
    if (r->nd->level == 0) by = 0;
    *x0 = r->nd->bx * w;
    *x1 = *x0 + w;
    *y0 = by * w;
    *y1 = *y0 + w;
}

static int adjacent(const Ref *a, const Ref *b) {
    int64_t ax0, ax1, ay0, ay1, bx0, bx1, by0, by1;
    span(a, &ax0, &ax1, &ay0, &ay1);
    span(b, &bx0, &bx1, &by0, &by1);
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

static Ref parent_of(const Ref *r) {
    Ref p;
    p.nd = r->nd->parent;
    p.img = (p.nd && p.nd->level > 0) ? r->img : 0;
    return p;
}

typedef struct {
    int32_t *v;
    int64_t n, cap;
} Vec;

static int vec_push(Vec *v, int32_t x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 64;
        int32_t *p = (int32_t *)realloc(v->v, (size_t)nc * sizeof(int32_t));
        if (!p) return -1;
        v->v = p;
        v->cap = nc;
    }
    v->v[v->n++] = x;
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

typedef struct {
    const Ref *b;
    Ref pb;
    int64_t rx0, rx1, ry0, ry1;   /* search region */
    Vec *out[4];
} Query;

static int visit(Query *q, const Ref *c) {
    int64_t x0, x1, y0, y1;
    span(c, &x0, &x1, &y0, &y1);
    if (x1 < q->rx0 || x0 > q->rx1 || y1 < q->ry0 || y0 > q->ry1) return 0;
    const Ref *b = q->b;
    int lb = b->nd->level, lc = c->nd->level;
    int32_t code = 2 * c->nd->index + c->img;
    int adj_cb = adjacent(c, b);
    Ref pc = parent_of(c);
    /* V */
    if (lc == lb && !adj_cb && adjacent(&pc, &q->pb))
        if (vec_push(q->out[1], code)) return -1;
    if (b->nd->leaf) {
        /* U */
        if (c->nd->leaf && adj_cb)
            if (vec_push(q->out[0], code)) return -1;
        /* W */
        if (lc > lb && !adj_cb && adjacent(&pc, b))
            if (vec_push(q->out[2], code)) return -1;
    }
    /* X */
    if (c->nd->leaf && lc < lb && !adj_cb && adjacent(c, &q->pb))
        if (vec_push(q->out[3], code)) return -1;
    for (int k = 0; k < c->nd->nchild; ++k) {
        Ref ch = {c->nd->child[k], c->img};
        if (visit(q, &ch)) return -1;
    }
    return 0;
}

void tree_ref_free(TreeRef *t) {
    if (!t) return;
    free(t->sorted);
    for (int k = 0; k < t->nbox; ++k) free(t->boxes[k]);
    free(t->boxes);
    free(t->root);
    for (int k = 0; k < 4; ++k) {
        free(t->off[k]);
        free(t->ent[k]);
    }
    free(t);
}

/* Build the tree and lists.  Returns NULL on allocation failure or bad input. */
TreeRef *tree_ref_build(int64_t n, const double *x, const double *y, int leaf_size,
                        int max_level, int lbits) {
    if (lbits < 2 || lbits > 30) return NULL;
    LBITS = lbits;
    if (n <= 0 || leaf_size < 1 || max_level < 1 || max_level > LBITS) return NULL;
    TreeRef *t = (TreeRef *)calloc(1, sizeof(TreeRef));
    if (!t) return NULL;
    t->n = n;
    t->leaf_size = leaf_size;
    t->max_level = max_level;
    double xlo = x[0], xhi = x[0], ymax = y[0];
    for (int64_t i = 1; i < n; ++i) {
        if (x[i] < xlo) xlo = x[i];
        if (x[i] > xhi) xhi = x[i];
        if (y[i] > ymax) ymax = y[i];
    }
    double S = xhi - xlo;
    if (2.0 * ymax > S) S = 2.0 * ymax;
    if (!(S > 0.0)) S = 1.0;
    t->x_lo = xlo;
    t->S = S;
    t->scale = ldexp(1.0, LBITS) / S;
    const int64_t full = (int64_t)1 << LBITS, half = (int64_t)1 << (LBITS - 1);
    t->sorted = (KeyIdx *)malloc((size_t)n * sizeof(KeyIdx));
    if (!t->sorted) goto fail;
    for (int64_t i = 0; i < n; ++i) {
        double fx = floor((x[i] - xlo) * t->scale);
        double fy = floor(y[i] * t->scale);
        int64_t ix = fx < 0.0 ? 0 : (fx > (double)(full - 1) ? full - 1 : (int64_t)fx);
        int64_t iu = fy < 0.0 ? 0 : (fy > (double)(half - 1) ? half - 1 : (int64_t)fy);
        t->sorted[i].key = interleave(ix, half + iu);
        t->sorted[i].idx = i;
    }
    qsort(t->sorted, (size_t)n, sizeof(KeyIdx), cmp_keyidx);

    Node *root = (Node *)calloc(1, sizeof(Node));
    if (!root) goto fail;
    root->level = 0;
    root->first = 0;
    root->count = n;
    root->index = -1;
    t->root = root;
    t->nbox = 0;
    if (build_rec(t, root)) goto fail;

    qsort(t->boxes, (size_t)t->nbox, sizeof(Node *), cmp_node);
    for (int k = 0; k < t->nbox; ++k) t->boxes[k]->index = k;

    Vec lists[4];
    memset(lists, 0, sizeof(lists));
    for (int k = 0; k < 4; ++k) {
        t->off[k] = (int64_t *)calloc((size_t)t->nbox + 1, sizeof(int64_t));
        if (!t->off[k]) goto fail;
    }
    for (int k = 0; k < t->nbox; ++k) {
        Ref b = {t->boxes[k], 0};
        Query q;
        q.b = &b;
        q.pb = parent_of(&b);
        int64_t px0, px1, py0, py1;
        if (q.pb.nd->level == 0) {
            px0 = 0; px1 = full; py0 = 0; py1 = full;
        } else {
            span(&q.pb, &px0, &px1, &py0, &py1);
        }
        int64_t w = px1 - px0;
        q.rx0 = px0 - w; q.rx1 = px1 + w; q.ry0 = py0 - w; q.ry1 = py1 + w;
        int64_t before[4];
        for (int j = 0; j < 4; ++j) {
            q.out[j] = &lists[j];
            before[j] = lists[j].n;
        }
        for (int c = 0; c < root->nchild; ++c) {
            Ref up = {root->child[c], 0}, dn = {root->child[c], 1};
            if (visit(&q, &up) || visit(&q, &dn)) goto fail_lists;
        }
        for (int j = 0; j < 4; ++j) {
            if (lists[j].n > before[j]) /* a list may still be empty (NULL storage) */
                qsort(lists[j].v + before[j], (size_t)(lists[j].n - before[j]), sizeof(int32_t),
                      cmp_i32);
            t->off[j][k + 1] = lists[j].n;
        }
    }
    for (int j = 0; j < 4; ++j) {
        t->ent[j] = lists[j].v;
        t->len[j] = lists[j].n;
    }
    return t;
fail_lists:
    for (int j = 0; j < 4; ++j) free(lists[j].v);
fail:
    tree_ref_free(t);
    return NULL;
}

void tree_ref_info(const TreeRef *t, int64_t *nbox, double *x_lo, double *S, double *scale,
                   int64_t *list_len /* [4]: U V W X */) {
    *nbox = t->nbox;
    *x_lo = t->x_lo;
    *S = t->S;
    *scale = t->scale;
    for (int j = 0; j < 4; ++j) list_len[j] = t->len[j];
}

/* Copy out.  Box arrays have nbox entries; list offsets nbox + 1; perm n. */
void tree_ref_export(const TreeRef *t, int32_t *level, int32_t *bx, int32_t *by,
                     int32_t *first, int32_t *count, int32_t *parent, int32_t *leaf,
                     int32_t *child_first, int32_t *nchild, int64_t *perm,
                     int64_t *u_off, int32_t *u_ent, int64_t *v_off, int32_t *v_ent,
                     int64_t *w_off, int32_t *w_ent, int64_t *x_off, int32_t *x_ent) {
    for (int k = 0; k < t->nbox; ++k) {
        const Node *b = t->boxes[k];
        level[k] = b->level;
        bx[k] = (int32_t)b->bx;
        by[k] = (int32_t)b->by;
        first[k] = (int32_t)b->first;
        count[k] = (int32_t)b->count;
        parent[k] = b->parent && b->parent->level > 0 ? b->parent->index : -1;
        leaf[k] = b->leaf;
        nchild[k] = b->nchild;
        child_first[k] = b->nchild ? b->child[0]->index : -1;
    }
    for (int64_t i = 0; i < t->n; ++i) perm[i] = t->sorted[i].idx;
    int64_t *offs[4] = {u_off, v_off, w_off, x_off};
    int32_t *ents[4] = {u_ent, v_ent, w_ent, x_ent};
    for (int j = 0; j < 4; ++j) {
        memcpy(offs[j], t->off[j], (size_t)(t->nbox + 1) * sizeof(int64_t));
        if (t->len[j]) memcpy(ents[j], t->ent[j], (size_t)t->len[j] * sizeof(int32_t));
    }
}

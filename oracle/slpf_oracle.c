/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, serial CPU implementation of what the SLPF parser computes,
 * written from "A parallel parser for regular expressions" (Borsotti,
 * Breveglieri, Crespi Reghizzi, Morzenti, arXiv 2503.06763).  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it.  It shares no code with the GPU library.
 *
 * What it computes, in the paper's order:
 *   1. the RE is read into a structure tree (Sect. 2.1) and every operator,
 *      terminal and empty-string leaf is numbered in left-to-right preorder
 *      (Sect. 2.2, Eq. numberedRE);
 *   2. the classic followers Fol(e#-|, s) of every numbered symbol
 *      (Eq. classicfollowers), where the numbered RE is read as a regular
 *      language over numbered parentheses, terminals and epsilons;
 *   3. the segments by the recursive meta-prefix extension of Fig.
 *      segmentalgo, with the initial set I and the final set F;
 *   4. the follower segments FolSeg (Eq. folsegdef); an NFA arc rho -> sigma
 *      is labelled with the unnumbered end-letter of rho (Sect. 2.3.3);
 *   5. the serial parser of Fig. serialparser: forward columns
 *      C_0 = I, C_r = N_{x_r} x C_{r-1}; backward columns C^_n = F,
 *      C^_r = N^_{x_{r+1}} x C^_{r+1} with N^_a the transpose of N_a
 *      (Eq. matrixmul, Eq. reverseNFAdef); output C_r intersected with C^_r,
 *      the intersection done in place during the backward scan (the memory
 *      remark closing Sect. 2.4);
 *   6. the number of syntax trees = number of accepting NFA runs, i.e. of
 *      paths through the clean SLPF (each accepting run is one LST, Sect.
 *      2.3.4), counted modulo 2^64 and, as a second check that does not
 *      vanish on counts that are multiples of 2^64, modulo the prime
 *      2^61 - 1;
 *   7. a second serial parser driven by the powerset DFA of the same NFA and
 *      its reverse (Sect. 3.1), built lazily, for long texts; the paper names
 *      this DFA-lookup parser as an alternative serial reference (Sect. 4.1).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - n-ary concatenation/union come only from same-operator chains written
 *     without parentheses; a parenthesised operator subexpression is its own
 *     node; parentheses around a single terminal add no node;
 *   - "()" and an empty alternative denote an epsilon leaf (App. A);
 *   - e? is a numbered pair with zero or one body inside (App. A, bounded
 *     repetition e{0,1}); zero iterations of a star give "k( )k";
 *   - a segment is initial when its first symbol can begin an LST (the paper
 *     says "begins with 1(", which is the same when the root is an operator);
 *   - an RE with an iterator over a nullable body (infinitely ambiguous) is
 *     rejected;
 *   - segments are numbered in a canonical order: by end-letter number (the
 *     end mark last), then meta-prefix length, then the meta-prefix symbols
 *     compared as (number, kind) with kind "(" < leaf < ")".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

enum { K_LIT, K_EPS, K_CAT, K_ALT, K_STAR, K_PLUS, K_OPT };

typedef struct {
    int kind;
    int byte;      /* K_LIT: the terminal byte, or -2 for a character set */
    int form;      /* K_LIT: 0 a byte, 1 a bracketed set, 2 the wildcard */
    uint64_t set[4];   /* K_LIT: the bytes the terminal matches */
    int nkids;
    int kids_cap;
    int *kids;
    int num;       /* preorder number, from 1 */
} onode;

typedef struct {
    /* structure tree */
    onode *nodes;
    int nnodes, cap_nodes, root;
    /* numbered symbols: node number k gives open 3k, leaf 3k+1, close 3k+2;
       the end mark -| is 3*(nnodes+1) */
    int nsym, sym_end;
    unsigned char *fol;      /* fol[r*nsym+s] = 1 iff s in Fol(r) */
    int first_sym;           /* the only symbol that can begin an LST */
    int *sym_node;           /* node index of a symbol, -1 for none */
    /* segments */
    int nseg, cap_seg;
    int *seg_len;
    int **seg_syms;
    int *seg_label;          /* byte of the end-letter, -2 for a set, -1 for the end mark */
    uint64_t *seg_set;       /* nseg x 4: the bytes the end-letter matches (none for the end mark) */
    int W;
    uint64_t *I, *F;         /* W words each */
    uint64_t *folseg;        /* nseg x W */
    /* lazy powerset DFAs (forward and reverse) */
    struct lazy_dfa *dfa[2];
} oracle_t;

/* ------------------------------------------------------------ RE reading */

typedef struct {
    const unsigned char *s;
    size_t n, pos;
    oracle_t *o;
    int err;
} rd_t;

static int new_node(oracle_t *o, int kind) {
    if (o->nnodes == o->cap_nodes) {
        o->cap_nodes = o->cap_nodes ? 2 * o->cap_nodes : 64;
        o->nodes = (onode *)realloc(o->nodes, sizeof(onode) * o->cap_nodes);
    }
    onode *x = &o->nodes[o->nnodes];
    memset(x, 0, sizeof(*x));
    x->kind = kind;
    return o->nnodes++;
}

static void add_kid(oracle_t *o, int p, int k) {
    onode *x = &o->nodes[p];
    if (x->nkids == x->kids_cap) {
        x->kids_cap = x->kids_cap ? 2 * x->kids_cap : 4;
        x->kids = (int *)realloc(x->kids, sizeof(int) * x->kids_cap);
    }
    x->kids[x->nkids++] = k;
}

static int rd_alt(rd_t *r);

static int hexval(int c) {
    if (c >= '0' && c <= '9') return c - '0';
    if (c >= 'a' && c <= 'f') return c - 'a' + 10;
    if (c >= 'A' && c <= 'F') return c - 'A' + 10;
    return -1;
}

/* one byte of a set or a terminal, after an optional backslash; -1 on error */
static int rd_byte(rd_t *r) {
    if (r->pos >= r->n) return -1;
    int c = r->s[r->pos++];
    if (c != '\\') return c;
    if (r->pos >= r->n) return -1;
    int e = r->s[r->pos++];
    if (e == 'n') return '\n';
    if (e == 't') return '\t';
    if (e == 'x') {
        if (r->pos + 2 > r->n) return -1;
        int h1 = hexval(r->s[r->pos]), h2 = hexval(r->s[r->pos + 1]);
        if (h1 < 0 || h2 < 0) return -1;
        r->pos += 2;
        return h1 * 16 + h2;
    }
    return e;
}

/* character set "[...]" (App. A, character features): bytes and ranges a-z,
 * a leading ^ complements; "]" first or escaped is a member.  Empty sets are
 * errors. */
static int rd_set(rd_t *r) {
    uint64_t m[4] = {0, 0, 0, 0};
    r->pos++;                                            /* '[' */
    int neg = 0, first = 1;
    if (r->pos < r->n && r->s[r->pos] == '^') { neg = 1; r->pos++; }
    for (;;) {
        if (r->pos >= r->n) { r->err = 1; return -1; }
        if (r->s[r->pos] == ']' && !first) { r->pos++; break; }
        first = 0;
        int lo = rd_byte(r);
        if (lo < 0) { r->err = 1; return -1; }
        int hi = lo;
        if (r->pos + 1 < r->n && r->s[r->pos] == '-' && r->s[r->pos + 1] != ']') {
            r->pos++;
            hi = rd_byte(r);
            if (hi < 0 || hi < lo) { r->err = 1; return -1; }
        }
        for (int b = lo; b <= hi; b++) m[b >> 6] |= 1ull << (b & 63);
    }
    int any = 0;
    for (int k = 0; k < 4; k++) { if (neg) m[k] = ~m[k]; any |= m[k] != 0; }
    if (!any) { r->err = 1; return -1; }
    int x = new_node(r->o, K_LIT);
    onode *v = &r->o->nodes[x];
    v->byte = -2;
    v->form = 1;
    memcpy(v->set, m, sizeof m);
    return x;
}

static int rd_atom(rd_t *r) {
    if (r->pos >= r->n) { r->err = 1; return -1; }
    int c = r->s[r->pos];
    if (c == '[') return rd_set(r);
    if (c == '.') {                                      /* wildcard: any byte but newline */
        r->pos++;
        int x = new_node(r->o, K_LIT);
        onode *v = &r->o->nodes[x];
        v->byte = -2;
        v->form = 2;
        for (int k = 0; k < 4; k++) v->set[k] = ~0ull;
        v->set['\n' >> 6] &= ~(1ull << ('\n' & 63));
        return x;
    }
    if (c == '(') {
        r->pos++;
        if (r->pos < r->n && r->s[r->pos] == ')') {   /* "()" is epsilon */
            r->pos++;
            return new_node(r->o, K_EPS);
        }
        int x = rd_alt(r);
        if (x < 0) return -1;
        if (r->pos >= r->n || r->s[r->pos] != ')') { r->err = 1; return -1; }
        r->pos++;
        return x;
    }
    if (c == ')' || c == '|' || c == '*' || c == '+' || c == '?') { r->err = 1; return -1; }
    int b = c;
    r->pos++;
    if (c == '\\') {
        if (r->pos >= r->n) { r->err = 1; return -1; }
        int e = r->s[r->pos++];
        if (e == 'n') b = '\n';
        else if (e == 't') b = '\t';
        else if (e == 'x') {
            if (r->pos + 2 > r->n) { r->err = 1; return -1; }
            int h1 = hexval(r->s[r->pos]), h2 = hexval(r->s[r->pos + 1]);
            if (h1 < 0 || h2 < 0) { r->err = 1; return -1; }
            b = h1 * 16 + h2;
            r->pos += 2;
        } else b = e;
    }
    int x = new_node(r->o, K_LIT);
    r->o->nodes[x].byte = b;
    r->o->nodes[x].set[b >> 6] = 1ull << (b & 63);
    return x;
}

static int rd_rep(rd_t *r) {
    int x = rd_atom(r);
    if (x < 0) return -1;
    while (r->pos < r->n) {
        int c = r->s[r->pos];
        int k = c == '*' ? K_STAR : c == '+' ? K_PLUS : c == '?' ? K_OPT : -1;
        if (k < 0) break;
        r->pos++;
        int y = new_node(r->o, k);
        add_kid(r->o, y, x);
        x = y;
    }
    return x;
}

static int rd_cat(rd_t *r) {
    int first = -1, node = -1, count = 0;
    while (r->pos < r->n && r->s[r->pos] != ')' && r->s[r->pos] != '|') {
        int x = rd_rep(r);
        if (x < 0) return -1;
        count++;
        if (count == 1) first = x;
        else {
            if (count == 2) { node = new_node(r->o, K_CAT); add_kid(r->o, node, first); }
            add_kid(r->o, node, x);
        }
    }
    if (count == 0) return new_node(r->o, K_EPS);   /* empty alternative */
    return count == 1 ? first : node;
}

static int rd_alt(rd_t *r) {
    int first = rd_cat(r);
    if (first < 0) return -1;
    int node = -1;
    while (r->pos < r->n && r->s[r->pos] == '|') {
        r->pos++;
        int x = rd_cat(r);
        if (x < 0) return -1;
        if (node < 0) { node = new_node(r->o, K_ALT); add_kid(r->o, node, first); }
        add_kid(r->o, node, x);
    }
    return node < 0 ? first : node;
}

/* ------------------------------------------------------ numbering, Fol */

static void number(oracle_t *o, int x, int *ctr) {
    o->nodes[x].num = ++*ctr;
    for (int i = 0; i < o->nodes[x].nkids; i++) number(o, o->nodes[x].kids[i], ctr);
}

/* nullable in the sense of the original RE: can the subtree derive epsilon */
static int re_nullable(oracle_t *o, int x) {
    onode *v = &o->nodes[x];
    switch (v->kind) {
    case K_LIT: return 0;
    case K_EPS: case K_STAR: case K_OPT: return 1;
    case K_PLUS: return re_nullable(o, v->kids[0]);
    case K_CAT:
        for (int i = 0; i < v->nkids; i++) if (!re_nullable(o, v->kids[i])) return 0;
        return 1;
    default: /* K_ALT */
        for (int i = 0; i < v->nkids; i++) if (re_nullable(o, v->kids[i])) return 1;
        return 0;
    }
}

static int inf_ambiguous(oracle_t *o, int x) {
    onode *v = &o->nodes[x];
    if ((v->kind == K_STAR || v->kind == K_PLUS) && re_nullable(o, v->kids[0])) return 1;
    for (int i = 0; i < v->nkids; i++) if (inf_ambiguous(o, v->kids[i])) return 1;
    return 0;
}

static int is_leaf(const onode *v) { return v->kind == K_LIT || v->kind == K_EPS; }
/* first / last numbered symbol of a subtree's LST (both unique) */
static int first_of(oracle_t *o, int x) {
    onode *v = &o->nodes[x];
    return is_leaf(v) ? 3 * v->num + 1 : 3 * v->num;
}
static int last_of(oracle_t *o, int x) {
    onode *v = &o->nodes[x];
    return is_leaf(v) ? 3 * v->num + 1 : 3 * v->num + 2;
}

#define FOL(o, r, s) ((o)->fol[(size_t)(r) * (o)->nsym + (s)])

/* The LST of operator node k is  k( inner )k  where inner is the sequence of
 * the children (concatenation), one child (union), zero or more / one or more
 * / zero or one copies of the child (star / cross / optional).  The followers
 * below are the classic Glushkov follow relation of that language. */
static void follow(oracle_t *o, int x) {
    onode *v = &o->nodes[x];
    if (is_leaf(v)) return;
    int open = 3 * v->num, close = 3 * v->num + 2;
    for (int i = 0; i < v->nkids; i++) follow(o, v->kids[i]);
    switch (v->kind) {
    case K_CAT:
        FOL(o, open, first_of(o, v->kids[0])) = 1;
        for (int i = 0; i + 1 < v->nkids; i++)
            FOL(o, last_of(o, v->kids[i]), first_of(o, v->kids[i + 1])) = 1;
        FOL(o, last_of(o, v->kids[v->nkids - 1]), close) = 1;
        break;
    case K_ALT:
        for (int i = 0; i < v->nkids; i++) {
            FOL(o, open, first_of(o, v->kids[i])) = 1;
            FOL(o, last_of(o, v->kids[i]), close) = 1;
        }
        break;
    case K_STAR: case K_PLUS: case K_OPT: {
        int c = v->kids[0];
        FOL(o, open, first_of(o, c)) = 1;
        FOL(o, last_of(o, c), close) = 1;
        if (v->kind != K_OPT) FOL(o, last_of(o, c), first_of(o, c)) = 1;   /* iterate */
        if (v->kind != K_PLUS) FOL(o, open, close) = 1;                   /* skip */
        break;
    }
    }
}

/* ------------------------------------------------------------ segments */

static int is_end_letter(oracle_t *o, int s) {
    if (s == o->sym_end) return 1;
    if (s % 3 != 1) return 0;
    int x = o->sym_node[s];
    return x >= 0 && o->nodes[x].kind == K_LIT;
}

static void add_segment(oracle_t *o, const int *syms, int len) {
    for (int i = 0; i < o->nseg; i++)
        if (o->seg_len[i] == len && memcmp(o->seg_syms[i], syms, sizeof(int) * len) == 0) return;
    if (o->nseg == o->cap_seg) {
        o->cap_seg = o->cap_seg ? 2 * o->cap_seg : 64;
        o->seg_len = (int *)realloc(o->seg_len, sizeof(int) * o->cap_seg);
        o->seg_syms = (int **)realloc(o->seg_syms, sizeof(int *) * o->cap_seg);
    }
    o->seg_syms[o->nseg] = (int *)malloc(sizeof(int) * len);
    memcpy(o->seg_syms[o->nseg], syms, sizeof(int) * len);
    o->seg_len[o->nseg++] = len;
}

/* MetaPrefix(s, sigma) of Fig. segmentalgo.  sigma is held right-aligned in
 * buf[pos .. cap-1]; s = buf[pos] is its leftmost symbol. */
static int meta_prefix(oracle_t *o, int *buf, int pos, int cap, int max_segs) {
    if (o->nseg > max_segs) return -1;
    int s = buf[pos];
    if (s == o->first_sym) {            /* sigma can open an LST: initial */
        add_segment(o, buf + pos, cap - pos);
        return 0;
    }
    for (int r = 0; r < o->nsym; r++) {
        if (!FOL(o, r, s)) continue;
        if (is_end_letter(o, r)) {      /* preceded by an end-letter: complete */
            add_segment(o, buf + pos, cap - pos);
        } else {                        /* extend the meta-prefix leftwards */
            if (pos == 0) return -1;
            buf[pos - 1] = r;
            if (meta_prefix(o, buf, pos - 1, cap, max_segs) < 0) return -1;
        }
    }
    return 0;
}

static oracle_t *g_sort_ctx;
static int end_rank(oracle_t *o, int seg) {
    int e = o->seg_syms[seg][o->seg_len[seg] - 1];
    return e == o->sym_end ? 0x7fffffff : e;
}
static int seg_cmp(const void *a, const void *b) {
    oracle_t *o = g_sort_ctx;
    int x = *(const int *)a, y = *(const int *)b;
    int ex = end_rank(o, x), ey = end_rank(o, y);
    if (ex != ey) return ex < ey ? -1 : 1;
    if (o->seg_len[x] != o->seg_len[y]) return o->seg_len[x] < o->seg_len[y] ? -1 : 1;
    for (int i = 0; i < o->seg_len[x] - 1; i++)
        if (o->seg_syms[x][i] != o->seg_syms[y][i])
            return o->seg_syms[x][i] < o->seg_syms[y][i] ? -1 : 1;
    return 0;
}

/* --------------------------------------------------------- public API */

#define SET_BIT(v, i) ((v)[(i) >> 6] |= (uint64_t)1 << ((i) & 63))
#define GET_BIT(v, i) (((v)[(i) >> 6] >> ((i) & 63)) & 1)

void oracle_free(oracle_t *o);

/* status: 0 ok, -1 argument, -2 syntax (err_off set), -3 infinitely ambiguous,
 * -4 too many segments */
int oracle_compile(const unsigned char *re, size_t re_len, int max_segments,
                   oracle_t **out, size_t *err_off) {
    *out = NULL;
    if (!re && re_len) return -1;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    rd_t r = { re, re_len, 0, o, 0 };
    int root = rd_alt(&r);
    if (root < 0 || r.err || r.pos != re_len) {
        if (err_off) *err_off = r.pos;
        oracle_free(o);
        return -2;
    }
    o->root = root;
    if (inf_ambiguous(o, root)) { oracle_free(o); return -3; }
    int ctr = 0;
    number(o, root, &ctr);
    o->sym_end = 3 * (o->nnodes + 1);
    o->nsym = o->sym_end + 1;
    o->fol = (unsigned char *)calloc((size_t)o->nsym * o->nsym, 1);
    o->sym_node = (int *)malloc(sizeof(int) * o->nsym);
    for (int s = 0; s < o->nsym; s++) o->sym_node[s] = -1;
    for (int x = 0; x < o->nnodes; x++) {
        int k = o->nodes[x].num;
        o->sym_node[3 * k] = o->sym_node[3 * k + 1] = o->sym_node[3 * k + 2] = x;
    }
    follow(o, root);
    FOL(o, last_of(o, root), o->sym_end) = 1;     /* e# followed by -| */
    o->first_sym = first_of(o, root);

    /* Fig. segmentalgo: one MetaPrefix call per end-letter */
    int cap = o->nsym + 2;
    int *buf = (int *)malloc(sizeof(int) * cap);
    int lim = max_segments > 0 ? max_segments : 1 << 20;
    for (int a = 0; a < o->nsym; a++) {
        if (!is_end_letter(o, a)) continue;
        buf[cap - 1] = a;
        if (meta_prefix(o, buf, cap - 1, cap, lim) < 0 || o->nseg > lim) {
            free(buf); oracle_free(o); return -4;
        }
    }
    free(buf);

    /* canonical order */
    int *perm = (int *)malloc(sizeof(int) * o->nseg);
    for (int i = 0; i < o->nseg; i++) perm[i] = i;
    g_sort_ctx = o;
    qsort(perm, o->nseg, sizeof(int), seg_cmp);
    int **ns = (int **)malloc(sizeof(int *) * o->nseg);
    int *nl = (int *)malloc(sizeof(int) * o->nseg);
    for (int i = 0; i < o->nseg; i++) { ns[i] = o->seg_syms[perm[i]]; nl[i] = o->seg_len[perm[i]]; }
    free(o->seg_syms); free(o->seg_len); free(perm);
    o->seg_syms = ns; o->seg_len = nl; o->cap_seg = o->nseg;

    o->W = (o->nseg + 63) / 64;
    if (o->W == 0) o->W = 1;
    o->I = (uint64_t *)calloc(o->W, 8);
    o->F = (uint64_t *)calloc(o->W, 8);
    o->seg_label = (int *)malloc(sizeof(int) * o->nseg);
    o->seg_set = (uint64_t *)calloc((size_t)o->nseg * 4, 8);
    o->folseg = (uint64_t *)calloc((size_t)o->nseg * o->W, 8);
    for (int i = 0; i < o->nseg; i++) {
        int e = o->seg_syms[i][o->seg_len[i] - 1];
        o->seg_label[i] = e == o->sym_end ? -1 : o->nodes[o->sym_node[e]].byte;
        if (e != o->sym_end) memcpy(o->seg_set + 4 * (size_t)i, o->nodes[o->sym_node[e]].set, 32);
        if (o->seg_syms[i][0] == o->first_sym) SET_BIT(o->I, i);
        if (e == o->sym_end) SET_BIT(o->F, i);
    }
    /* Eq. folsegdef: sigma follows rho iff first(sigma) in Fol(end-letter(rho)) */
    for (int i = 0; i < o->nseg; i++) {
        int e = o->seg_syms[i][o->seg_len[i] - 1];
        if (e == o->sym_end) continue;
        for (int j = 0; j < o->nseg; j++)
            if (FOL(o, e, o->seg_syms[j][0])) SET_BIT(o->folseg + (size_t)i * o->W, j);
    }
    *out = o;
    return 0;
}

struct lazy_dfa;
static void lazy_free(struct lazy_dfa *d);

void oracle_free(oracle_t *o) {
    if (!o) return;
    for (int x = 0; x < o->nnodes; x++) free(o->nodes[x].kids);
    free(o->nodes);
    free(o->fol);
    free(o->sym_node);
    for (int i = 0; i < o->nseg; i++) free(o->seg_syms[i]);
    free(o->seg_syms); free(o->seg_len); free(o->seg_label); free(o->seg_set);
    free(o->I); free(o->F); free(o->folseg);
    lazy_free(o->dfa[0]); lazy_free(o->dfa[1]);
    free(o);
}

int oracle_num_segments(const oracle_t *o) { return o->nseg; }
int oracle_words(const oracle_t *o) { return o->W; }
int oracle_num_nodes(const oracle_t *o) { return o->nnodes; }

/* Preorder number of the parent of the node numbered `num` in the RE tree
 * (Sect. 2.2), 0 for the root, -1 when no node has that number. */
int oracle_node_parent(const oracle_t *o, int num) {
    for (int x = 0; x < o->nnodes; x++)
        for (int k = 0; k < o->nodes[x].nkids; k++)
            if (o->nodes[o->nodes[x].kids[k]].num == num) return o->nodes[x].num;
    for (int x = 0; x < o->nnodes; x++)
        if (o->nodes[x].num == num) return 0;
    return -1;
}
void oracle_initial(const oracle_t *o, uint64_t *out) { memcpy(out, o->I, 8 * o->W); }
void oracle_final(const oracle_t *o, uint64_t *out) { memcpy(out, o->F, 8 * o->W); }
void oracle_folseg(const oracle_t *o, int seg, uint64_t *out) {
    memcpy(out, o->folseg + (size_t)seg * o->W, 8 * o->W);
}
int oracle_label(const oracle_t *o, int seg) { return o->seg_label[seg]; }
void oracle_label_set(const oracle_t *o, int seg, uint64_t *out) { memcpy(out, o->seg_set + 4 * (size_t)seg, 32); }

/* a byte inside a set's text: letters and digits as themselves, others \xHH */
static int set_byte_text(int b, char *buf) {
    if ((b >= 'a' && b <= 'z') || (b >= 'A' && b <= 'Z') || (b >= '0' && b <= '9')) return sprintf(buf, "%c", b);
    return sprintf(buf, "\\x%02x", b);
}

/* Printable form of a numbered symbol: "k(" ")k" for parentheses, the
 * terminal followed by its number ("a4"; bytes other than letters as \xHH;
 * a set as its maximal ranges in brackets, "[a-z0]4", a range of two bytes
 * as both; the wildcard as ".4"), "ε4" for an empty-string leaf, "⊣" for the
 * end mark. */
static int sym_text(const oracle_t *o, int s, char *buf) {
    if (s == o->sym_end) return sprintf(buf, "\xe2\x8a\xa3");
    int x = o->sym_node[s];
    const onode *v = &o->nodes[x];
    int k = v->num;
    switch (s % 3) {
    case 0: return sprintf(buf, "%d(", k);
    case 2: return sprintf(buf, ")%d", k);
    default:
        if (v->kind == K_EPS) return sprintf(buf, "\xce\xb5%d", k);
        if (v->form == 2) return sprintf(buf, ".%d", k);
        if (v->form == 1) {
            int len = sprintf(buf, "[");
            for (int b = 0; b < 256;) {
                if (!((v->set[b >> 6] >> (b & 63)) & 1)) { b++; continue; }
                int e = b;
                while (e + 1 < 256 && ((v->set[(e + 1) >> 6] >> ((e + 1) & 63)) & 1)) e++;
                len += set_byte_text(b, buf + len);
                if (e == b + 1) len += set_byte_text(e, buf + len);
                else if (e > b + 1) { buf[len++] = '-'; len += set_byte_text(e, buf + len); }
                b = e + 1;
            }
            return len + sprintf(buf + len, "]%d", k);
        }
        if ((v->byte >= 'a' && v->byte <= 'z') || (v->byte >= 'A' && v->byte <= 'Z'))
            return sprintf(buf, "%c%d", v->byte, k);
        return sprintf(buf, "\\x%02x%d", v->byte, k);
    }
}

/* segment as space-separated symbols; returns the length needed (w/o NUL) */
size_t oracle_segment_text(const oracle_t *o, int seg, char *buf, size_t cap) {
    char tmp[1200];
    size_t need = 0;
    for (int i = 0; i < o->seg_len[seg]; i++) {
        int l = sym_text(o, o->seg_syms[seg][i], tmp);
        if (i) { if (buf && need < cap) buf[need] = ' '; need++; }
        for (int j = 0; j < l; j++) { if (buf && need < cap) buf[need] = tmp[j]; need++; }
    }
    if (buf && cap) buf[need < cap ? need : cap - 1] = 0;
    return need;
}

/* ------------------------------------------------- one NFA step on sets */

/* the end-letter of segment rho matches byte a (an arc rho -> sigma is
 * labelled with the end-letter: a byte, or a character set, Sect. 2.3.3 and
 * App. A, character features) */
static int label_has(const oracle_t *o, int rho, int a) {
    return a >= 0 && a < 256 && ((o->seg_set[4 * (size_t)rho + (a >> 6)] >> (a & 63)) & 1);
}

/* forward: out = N_a x in = union of FolSeg(rho) over rho in `in` with label a */
void oracle_step_fwd(const oracle_t *o, const uint64_t *in, int a, uint64_t *out) {
    memset(out, 0, 8 * o->W);
    for (int rho = 0; rho < o->nseg; rho++) {
        if (!GET_BIT(in, rho) || !label_has(o, rho, a)) continue;
        const uint64_t *f = o->folseg + (size_t)rho * o->W;
        for (int w = 0; w < o->W; w++) out[w] |= f[w];
    }
}

/* backward: out = N^_a x in = { rho : label(rho) = a, FolSeg(rho) meets `in` } */
void oracle_step_bwd(const oracle_t *o, const uint64_t *in, int a, uint64_t *out) {
    memset(out, 0, 8 * o->W);
    for (int rho = 0; rho < o->nseg; rho++) {
        if (!label_has(o, rho, a)) continue;
        const uint64_t *f = o->folseg + (size_t)rho * o->W;
        int meet = 0;
        for (int w = 0; w < o->W; w++) if (f[w] & in[w]) { meet = 1; break; }
        if (meet) SET_BIT(out, rho);
    }
}

/* --------------------------------------- count of trees (accepting runs) */

/* The second modulus of the tree count: the Mersenne prime 2^61 - 1. */
#define P61 ((((uint64_t)1) << 61) - 1)

static uint64_t addp(uint64_t a, uint64_t b) {   /* a, b < P61 */
    uint64_t s = a + b;
    return s >= P61 ? s - P61 : s;
}

/* cnt_0[sigma] = 1 on C_0; cnt_r[sigma] = sum of cnt_{r-1}[rho] over the arcs
 * rho -> sigma labelled x_r inside the clean SLPF; result = sum over C_n.
 * The sums are kept modulo 2^64 (cnt) and modulo 2^61 - 1 (cntp). */
static void count_paths(const oracle_t *o, const unsigned char *x, uint64_t n,
                        const uint64_t *cols, uint64_t *out64, uint64_t *outp) {
    int W = o->W, L = o->nseg;
    uint64_t *cur = (uint64_t *)calloc(L, 8), *nxt = (uint64_t *)calloc(L, 8);
    uint64_t *curp = (uint64_t *)calloc(L, 8), *nxtp = (uint64_t *)calloc(L, 8);
    for (int s = 0; s < L; s++) if (GET_BIT(cols, s)) { cur[s] = 1; curp[s] = 1; }
    for (uint64_t r = 1; r <= n; r++) {
        const uint64_t *c = cols + r * W;
        memset(nxt, 0, 8 * (size_t)L);
        memset(nxtp, 0, 8 * (size_t)L);
        for (int rho = 0; rho < L; rho++) {
            if (!GET_BIT(cols + (r - 1) * W, rho) || !label_has(o, rho, x[r - 1])) continue;
            const uint64_t *f = o->folseg + (size_t)rho * W;
            for (int sg = 0; sg < L; sg++)
                if (GET_BIT(f, sg) && GET_BIT(c, sg)) {
                    nxt[sg] += cur[rho];
                    nxtp[sg] = addp(nxtp[sg], curp[rho]);
                }
        }
        uint64_t *t = cur; cur = nxt; nxt = t;
        t = curp; curp = nxtp; nxtp = t;
    }
    uint64_t total = 0, totalp = 0;
    for (int s = 0; s < L; s++)
        if (GET_BIT(cols + n * W, s)) { total += cur[s]; totalp = addp(totalp, curp[s]); }
    free(cur); free(nxt); free(curp); free(nxtp);
    *out64 = total;
    *outp = totalp;
}

/* The serial NFA parser of Fig. serialparser.  cols: (n+1) x W words.
 * scalars: [0] accepted, [1] number of trees mod 2^64, [2] number of trees
 * mod 2^61 - 1. */
int oracle_parse(const oracle_t *o, const unsigned char *x, uint64_t n,
                 uint64_t *cols, uint64_t *scalars) {
    int W = o->W;
    uint64_t *tmp = (uint64_t *)malloc(8 * W), *nb = (uint64_t *)malloc(8 * W);
    memcpy(cols, o->I, 8 * W);                                   /* C_0 = I */
    for (uint64_t r = 1; r <= n; r++)
        oracle_step_fwd(o, cols + (r - 1) * W, x[r - 1], cols + r * W);
    memcpy(tmp, o->F, 8 * W);                                    /* C^_n = F */
    for (int w = 0; w < W; w++) cols[n * W + w] &= tmp[w];
    for (uint64_t r = n; r-- > 0;) {
        oracle_step_bwd(o, tmp, x[r], nb);                       /* C^_r */
        memcpy(tmp, nb, 8 * W);
        for (int w = 0; w < W; w++) cols[r * W + w] &= tmp[w];   /* in place */
    }
    uint64_t acc = 0;
    for (int w = 0; w < W; w++) acc |= cols[n * W + w];
    scalars[0] = acc != 0;
    scalars[1] = scalars[2] = 0;
    if (acc) count_paths(o, x, n, cols, &scalars[1], &scalars[2]);
    free(tmp); free(nb);
    return 0;
}

/* ------------------------------------- lazily built powerset DFA (Sect. 3.1) */

typedef struct lazy_dfa {
    int dir;             /* 0 forward (N_a), 1 reverse (transposed) */
    int W;
    int nstates, cap;
    uint64_t *sets;      /* nstates x W */
    int32_t *next;       /* nstates x 256, -1 = not yet computed */
    int32_t *htab;       /* open addressing over set words */
    size_t hcap;
} lazy_dfa;

static uint64_t set_hash(const uint64_t *s, int W) {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int w = 0; w < W; w++) { h ^= s[w]; h *= 0xff51afd7ed558ccdull; h ^= h >> 32; }
    return h;
}

static void lazy_free(lazy_dfa *d) {
    if (!d) return;
    free(d->sets); free(d->next); free(d->htab); free(d);
}

static int lazy_find(lazy_dfa *d, const uint64_t *s);

static void lazy_rehash(lazy_dfa *d) {
    free(d->htab);
    d->hcap = d->hcap ? 2 * d->hcap : 1024;
    d->htab = (int32_t *)malloc(sizeof(int32_t) * d->hcap);
    for (size_t i = 0; i < d->hcap; i++) d->htab[i] = -1;
    for (int id = 0; id < d->nstates; id++) {
        size_t h = set_hash(d->sets + (size_t)id * d->W, d->W) & (d->hcap - 1);
        while (d->htab[h] >= 0) h = (h + 1) & (d->hcap - 1);
        d->htab[h] = id;
    }
}

/* id of set s, adding it if new */
static int lazy_find(lazy_dfa *d, const uint64_t *s) {
    if (2 * (size_t)(d->nstates + 1) > d->hcap) lazy_rehash(d);
    size_t h = set_hash(s, d->W) & (d->hcap - 1);
    while (d->htab[h] >= 0) {
        if (memcmp(d->sets + (size_t)d->htab[h] * d->W, s, 8 * d->W) == 0) return d->htab[h];
        h = (h + 1) & (d->hcap - 1);
    }
    if (d->nstates == d->cap) {
        d->cap = d->cap ? 2 * d->cap : 256;
        d->sets = (uint64_t *)realloc(d->sets, 8 * (size_t)d->cap * d->W);
        d->next = (int32_t *)realloc(d->next, sizeof(int32_t) * 256 * (size_t)d->cap);
    }
    int id = d->nstates++;
    memcpy(d->sets + (size_t)id * d->W, s, 8 * d->W);
    for (int a = 0; a < 256; a++) d->next[(size_t)id * 256 + a] = -1;
    d->htab[h] = id;
    return id;
}

static lazy_dfa *lazy_get(oracle_t *o, int dir) {
    if (!o->dfa[dir]) {
        lazy_dfa *d = (lazy_dfa *)calloc(1, sizeof(lazy_dfa));
        d->dir = dir; d->W = o->W;
        o->dfa[dir] = d;
    }
    return o->dfa[dir];
}

static int lazy_step(oracle_t *o, lazy_dfa *d, int id, int a, uint64_t *scratch) {
    int32_t t = d->next[(size_t)id * 256 + a];
    if (t >= 0) return t;
    if (d->dir == 0) oracle_step_fwd(o, d->sets + (size_t)id * d->W, a, scratch);
    else oracle_step_bwd(o, d->sets + (size_t)id * d->W, a, scratch);
    t = lazy_find(d, scratch);
    d->next[(size_t)id * 256 + a] = t;
    return t;
}

/* The DFA-lookup serial parser.  Runs the forward DFA from I over the whole
 * text, then the reverse DFA from F backwards; the clean column at r is the
 * intersection of the two sets.  Only the columns of the requested windows
 * are written (nwin windows of win_len columns starting at win_start[i]);
 * scalars as in oracle_parse.  The tree count uses the backward form of the
 * same path count: cntB_n = 1 on C_n, cntB_r[rho] = sum of cntB_{r+1}[sigma]
 * over arcs rho -> sigma inside the clean SLPF, result = sum over C_0, kept
 * modulo 2^64 and modulo 2^61 - 1.  With want_count = 0 the count is skipped
 * (scalars[1] = scalars[2] = 0): only the windows and the accept flag. */
int oracle_parse_dfa(oracle_t *o, const unsigned char *x, uint64_t n,
                     int nwin, const uint64_t *win_start, uint64_t win_len,
                     uint64_t *win_cols, uint64_t *scalars, int want_count) {
    int W = o->W, L = o->nseg;
    lazy_dfa *fd = lazy_get(o, 0), *bd = lazy_get(o, 1);
    uint64_t *scratch = (uint64_t *)malloc(8 * W);
    int32_t *fid = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    if (!fid) { free(scratch); return -5; }
    fid[0] = lazy_find(fd, o->I);
    for (uint64_t r = 1; r <= n; r++) fid[r] = lazy_step(o, fd, fid[r - 1], x[r - 1], scratch);
    uint64_t *cnt = (uint64_t *)calloc(L, 8), *cnt2 = (uint64_t *)calloc(L, 8);
    uint64_t *cntp = (uint64_t *)calloc(L, 8), *cnt2p = (uint64_t *)calloc(L, 8);
    uint64_t *col = (uint64_t *)malloc(8 * W), *ncol = (uint64_t *)malloc(8 * W);
    int bid = lazy_find(bd, o->F);
    int accepted = 0;
    uint64_t total = 0, totalp = 0;
    for (uint64_t r = n + 1; r-- > 0;) {
        if (r < n) bid = lazy_step(o, bd, bid, x[r], scratch);
        const uint64_t *fs = fd->sets + (size_t)fid[r] * W;
        const uint64_t *bs = bd->sets + (size_t)bid * W;
        uint64_t any = 0;
        for (int w = 0; w < W; w++) { col[w] = fs[w] & bs[w]; any |= col[w]; }
        if (r == n) accepted = any != 0;
        for (int i = 0; i < nwin; i++)
            if (r >= win_start[i] && r < win_start[i] + win_len)
                memcpy(win_cols + ((size_t)i * win_len + (r - win_start[i])) * W, col, 8 * W);
        if (!accepted || !want_count) continue;
        if (r == n) {
            for (int s = 0; s < L; s++) cnt[s] = cntp[s] = GET_BIT(col, s) ? 1 : 0;
        } else {
            for (int rho = 0; rho < L; rho++) {
                cnt2[rho] = cnt2p[rho] = 0;
                if (!GET_BIT(col, rho) || !label_has(o, rho, x[r])) continue;
                const uint64_t *f = o->folseg + (size_t)rho * W;
                for (int w = 0; w < W; w++) {
                    uint64_t m = f[w] & ncol[w];
                    while (m) {
                        int b = __builtin_ctzll(m);
                        m &= m - 1;
                        cnt2[rho] += cnt[w * 64 + b];
                        cnt2p[rho] = addp(cnt2p[rho], cntp[w * 64 + b]);
                    }
                }
            }
            uint64_t *t = cnt; cnt = cnt2; cnt2 = t;
            t = cntp; cntp = cnt2p; cnt2p = t;
        }
        memcpy(ncol, col, 8 * W);
        if (r == 0)
            for (int s = 0; s < L; s++)
                if (GET_BIT(col, s)) { total += cnt[s]; totalp = addp(totalp, cntp[s]); }
    }
    scalars[0] = accepted;
    scalars[1] = accepted && want_count ? total : 0;
    scalars[2] = accepted && want_count ? totalp : 0;
    free(fid); free(cnt); free(cnt2); free(cntp); free(cnt2p); free(col); free(ncol); free(scratch);
    return 0;
}

/* Powerset construction restricted to the sets reachable from the given
 * seed sets (nseeds x W words), over the byte values in alphabet[0..na-1].
 * dir 0: forward NFA; dir 1: reverse NFA.  Returns the number of states
 * (the empty set excluded) or -1 when more than max_states; states are
 * numbered in BFS order from the seeds; out_sets / out_next may be NULL. */
int oracle_powerset(const oracle_t *o, int dir, const uint64_t *seeds, int nseeds,
                    const int *alphabet, int na, int max_states,
                    uint64_t *out_sets, int32_t *out_next) {
    int W = o->W;
    lazy_dfa d;
    memset(&d, 0, sizeof(d));
    d.dir = dir; d.W = W;
    uint64_t *zero = (uint64_t *)calloc(W, 8), *scratch = (uint64_t *)malloc(8 * W);
    lazy_find(&d, zero);                                  /* id 0 = empty set */
    for (int i = 0; i < nseeds; i++) lazy_find(&d, seeds + (size_t)i * W);
    int head = 1;
    int ok = 1;
    while (head < d.nstates) {
        if (d.nstates - 1 > max_states) { ok = 0; break; }
        for (int k = 0; k < na; k++) {
            if (dir == 0) oracle_step_fwd(o, d.sets + (size_t)head * W, alphabet[k], scratch);
            else oracle_step_bwd(o, d.sets + (size_t)head * W, alphabet[k], scratch);
            int t = lazy_find(&d, scratch);
            d.next[(size_t)head * 256 + alphabet[k]] = t;
        }
        head++;
    }
    int ns = d.nstates - 1;
    if (ok && ns > max_states) ok = 0;
    if (ok) {
        for (int id = 1; id <= ns; id++) {
            if (out_sets) memcpy(out_sets + (size_t)(id - 1) * W, d.sets + (size_t)id * W, 8 * W);
            if (out_next)
                for (int k = 0; k < na; k++) {
                    int t = d.next[(size_t)id * 256 + alphabet[k]];
                    out_next[(size_t)(id - 1) * na + k] = t > 0 ? t - 1 : -1;
                }
        }
    }
    free(d.sets); free(d.next); free(d.htab); free(zero); free(scratch);
    return ok ? ns : -1;
}

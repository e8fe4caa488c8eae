/*
 * Oracle cluster enumerator (test infrastructure only; never linked into the
 * GPU library, which has its own independent enumerator).
 *
 * Loop-correction terms (Sec. III.A, Fig. 3 and Sec. III.B, Fig. 5): a term is
 * a configuration of excited bonds; a configuration with a tensor carrying
 * exactly one excited bond (a dangling excitation) vanishes at a BP fixed
 * point, and the degree of a configuration is its number of excited bonds.
 * A configuration splits into connected components, and it is dangling-free
 * exactly when every component is.  This file lists the components: every
 * connected set of bonds c with |c| <= K in which every site touched by c
 * has degree >= 2 inside c.  Sites flagged `exempt` (sites that carry open
 * legs, Sec. III.D) only need degree >= 1.
 *
 * Method: the ESU scheme (Wernicke 2006) run on the line graph, so each
 * connected bond set is visited exactly once with its smallest bond as the
 * root.  A branch is abandoned when the bonds still allowed cannot repair the
 * degree-1 sites already present (each added bond touches at most two sites).
 *
 * Output: clusters in visiting order; bonds of each cluster sorted ascending.
 * Call once with out_bonds == NULL to count (returns the number of clusters
 * and writes the total number of bond entries to *n_bond_entries).
 */
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n_sites, n_bonds, K;
    const int *bu, *bv;
    const unsigned char *exempt;
    int *site_ptr, *site_bonds;   /* CSR: bonds incident to each site */
    int *deg;                      /* degree of each site inside S */
    int *in_s;                     /* bond in S */
    int *adj_s;                    /* number of S bonds adjacent to the bond */
    int *S;                        /* current set */
    int size;
    int d1;                        /* non-exempt sites of degree 1 in S */
    int root;
    int **ext;                     /* per-depth extension lists */
    int *ext_len;
    int ext_cap;
    long long n_clusters, n_entries;
    int *out_bonds, *out_sizes;
    long long cap_clusters, cap_entries;
    int overflow;
} enum_state;

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static void emit(enum_state *st) {
    if (st->out_bonds) {
        if (st->n_clusters >= st->cap_clusters || st->n_entries + st->size > st->cap_entries) {
            st->overflow = 1;
            return;
        }
        int *dst = st->out_bonds + st->n_entries;
        memcpy(dst, st->S, sizeof(int) * (size_t)st->size);
        qsort(dst, (size_t)st->size, sizeof(int), cmp_int);
        st->out_sizes[st->n_clusters] = st->size;
    }
    st->n_clusters += 1;
    st->n_entries += st->size;
}

static void site_inc(enum_state *st, int s) {
    int d = ++st->deg[s];
    if (!st->exempt || !st->exempt[s]) {
        if (d == 1) st->d1++;
        else if (d == 2) st->d1--;
    }
}

static void site_dec(enum_state *st, int s) {
    int d = st->deg[s]--;
    if (!st->exempt || !st->exempt[s]) {
        if (d == 1) st->d1--;
        else if (d == 2) st->d1++;
    }
}

/* bonds adjacent to bond b (sharing a site), b itself excluded */
#define FOR_ADJ(st, b, body)                                                    \
    do {                                                                        \
        int ends_[2] = {(st)->bu[b], (st)->bv[b]};                              \
        for (int e_ = 0; e_ < 2; ++e_) {                                        \
            int s_ = ends_[e_];                                                 \
            for (int p_ = (st)->site_ptr[s_]; p_ < (st)->site_ptr[s_ + 1]; ++p_) { \
                int nb = (st)->site_bonds[p_];                                  \
                if (nb == (b)) continue;                                        \
                body                                                            \
            }                                                                   \
        }                                                                       \
    } while (0)

static void add_bond(enum_state *st, int b) {
    st->S[st->size++] = b;
    st->in_s[b] = 1;
    site_inc(st, st->bu[b]);
    site_inc(st, st->bv[b]);
    FOR_ADJ(st, b, { st->adj_s[nb]++; });
}

static void remove_bond(enum_state *st, int b) {
    FOR_ADJ(st, b, { st->adj_s[nb]--; });
    site_dec(st, st->bv[b]);
    site_dec(st, st->bu[b]);
    st->in_s[b] = 0;
    st->size--;
}

static void extend(enum_state *st, int depth) {
    if (st->d1 == 0) emit(st);
    if (st->size >= st->K || st->overflow) return;
    /* each further bond repairs at most two degree-1 sites */
    if (2 * (st->K - st->size) < st->d1) return;
    int *ext = st->ext[depth];
    int n = st->ext_len[depth];
    while (n > 0) {
        int w = ext[--n];
        /* extension of the child: remaining ext plus the exclusive
           neighbourhood of w (neighbours of w not in S and not adjacent to S) */
        int *next = st->ext[depth + 1];
        int m = 0;
        for (int i = 0; i < n; ++i) next[m++] = ext[i];
        int base = m;
        FOR_ADJ(st, w, {
            if (nb > st->root && !st->in_s[nb] && st->adj_s[nb] == 0) {
                int dup = 0;
                for (int i = base; i < m; ++i)
                    if (next[i] == nb) { dup = 1; break; }
                if (!dup) next[m++] = nb;
            }
        });
        st->ext_len[depth + 1] = m;
        add_bond(st, w);
        extend(st, depth + 1);
        remove_bond(st, w);
        if (st->overflow) return;
    }
}

long long oracle_enum_clusters(int n_sites, int n_bonds, const int *bu, const int *bv,
                               const unsigned char *exempt, int K,
                               int *out_bonds, long long cap_entries,
                               int *out_sizes, long long cap_clusters,
                               long long *n_bond_entries) {
    enum_state st;
    memset(&st, 0, sizeof st);
    st.n_sites = n_sites;
    st.n_bonds = n_bonds;
    st.K = K;
    st.bu = bu;
    st.bv = bv;
    st.exempt = exempt;
    st.out_bonds = out_bonds;
    st.out_sizes = out_sizes;
    st.cap_entries = cap_entries;
    st.cap_clusters = cap_clusters;
    if (K <= 0 || n_bonds == 0) {
        if (n_bond_entries) *n_bond_entries = 0;
        return 0;
    }
    st.site_ptr = (int *)calloc((size_t)n_sites + 1, sizeof(int));
    st.site_bonds = (int *)malloc(sizeof(int) * 2 * (size_t)n_bonds);
    st.deg = (int *)calloc((size_t)n_sites, sizeof(int));
    st.in_s = (int *)calloc((size_t)n_bonds, sizeof(int));
    st.adj_s = (int *)calloc((size_t)n_bonds, sizeof(int));
    st.S = (int *)malloc(sizeof(int) * ((size_t)K + 1));
    for (int b = 0; b < n_bonds; ++b) {
        st.site_ptr[bu[b] + 1]++;
        st.site_ptr[bv[b] + 1]++;
    }
    int maxdeg = 0;
    for (int s = 0; s < n_sites; ++s) {
        int d = st.site_ptr[s + 1];
        if (d > maxdeg) maxdeg = d;
        st.site_ptr[s + 1] += st.site_ptr[s];
    }
    int *fill = (int *)calloc((size_t)n_sites, sizeof(int));
    for (int b = 0; b < n_bonds; ++b) {
        st.site_bonds[st.site_ptr[bu[b]] + fill[bu[b]]++] = b;
        st.site_bonds[st.site_ptr[bv[b]] + fill[bv[b]]++] = b;
    }
    free(fill);
    st.ext_cap = (K + 2) * 2 * (maxdeg + 1) + 8;
    st.ext = (int **)malloc(sizeof(int *) * ((size_t)K + 2));
    st.ext_len = (int *)calloc((size_t)K + 2, sizeof(int));
    for (int d = 0; d < K + 2; ++d) st.ext[d] = (int *)malloc(sizeof(int) * (size_t)st.ext_cap);

    for (int r = 0; r < n_bonds && !st.overflow; ++r) {
        st.root = r;
        add_bond(&st, r);
        int m = 0;
        FOR_ADJ((&st), r, {
            if (nb > r) {
                int dup = 0;
                for (int i = 0; i < m; ++i)
                    if (st.ext[0][i] == nb) { dup = 1; break; }
                if (!dup) st.ext[0][m++] = nb;
            }
        });
        st.ext_len[0] = m;
        extend(&st, 0);
        remove_bond(&st, r);
    }

    for (int d = 0; d < K + 2; ++d) free(st.ext[d]);
    free(st.ext);
    free(st.ext_len);
    free(st.site_ptr);
    free(st.site_bonds);
    free(st.deg);
    free(st.in_s);
    free(st.adj_s);
    free(st.S);
    if (n_bond_entries) *n_bond_entries = st.n_entries;
    return st.overflow ? -1 : st.n_clusters;
}

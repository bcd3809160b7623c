/*
 * msc_oracle.c -- plain, serial CPU oracle for path-compression Morse-Smale
 * segmentation and connected components.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.  Speed is not a goal: every function is the plain definition
 * written out so that it can be checked against the paper by eye.
 *
 * Paper: Will, Lukasczyk, Tierny, Garth, "Distributed Path Compression for
 * Piecewise Linear Morse-Smale Segmentations and Connected Components"
 * (arXiv 2409.03771).
 *
 * Conventions (the readings taken where the paper is silent):
 *  - Grid vertex (x,y,z) of an X*Y*Z grid has id x + X*y + X*Y*z; the field is
 *    stored in that order (x fastest).
 *  - The triangulation is the Freudenthal (Kuhn) subdivision of every cube
 *    into six tetrahedra {0, e_a, e_a+e_b, e_a+e_b+e_c}, (a,b,c) a permutation
 *    of the three axes.  The edge set is derived from those tetrahedra at run
 *    time (orc_stencil), not written down by hand.
 *  - Vertices are totally ordered by (f(v), id(v)): larger value first, ties
 *    broken by the larger id -- the simulation-of-simplicity order of the
 *    paper's preprocessing section.  Comparisons use IEEE float semantics.
 *  - Steepest ascent picks the (f,id)-largest vertex of the closed
 *    neighbourhood {v} u N(v), steepest descent the (f,id)-smallest (Sec.
 *    "Ascending and Descending Manifolds" of the background; Alg. 1 init).
 *    Including v itself makes extrema point to themselves.
 *  - asc[v] is the maximum reached by steepest ascent from v (the paper's
 *    descending manifold), desc[v] the minimum reached by steepest descent
 *    (the paper's ascending manifold).
 *  - ms[v] is the smallest vertex id u with asc[u]==asc[v] and
 *    desc[u]==desc[v] (the Morse-Smale cell of the pair, Sec. "Ascending and
 *    Descending Segmentation").
 *  - Connected components: label[v] = smallest id of v's component in the
 *    graph induced by masked vertices; unmasked vertices get -1 (Alg. 3 init).
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#define _GNU_SOURCE /* qsort_r */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Triangulation                                                            */
/* ------------------------------------------------------------------------ */

/*
 * Edge vectors of the Freudenthal triangulation, derived from its six Kuhn
 * tetrahedra: every pair of corners of every tetrahedron spans an edge.
 * Writes the distinct non-zero vectors (both signs) to out[k*3 + {0,1,2}]
 * (dx,dy,dz) and returns their number (14).
 */
int orc_stencil(int32_t *out)
{
    static const int perms[6][3] = {
        {0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int count = 0;
    for (int p = 0; p < 6; ++p) {
        int corner[4][3];
        memset(corner, 0, sizeof corner);
        for (int k = 1; k < 4; ++k) {
            memcpy(corner[k], corner[k - 1], sizeof corner[k]);
            corner[k][perms[p][k - 1]] += 1;
        }
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) {
                if (i == j) continue;
                int d[3] = {corner[j][0] - corner[i][0],
                            corner[j][1] - corner[i][1],
                            corner[j][2] - corner[i][2]};
                int seen = 0;
                for (int q = 0; q < count; ++q)
                    if (out[3 * q] == d[0] && out[3 * q + 1] == d[1] &&
                        out[3 * q + 2] == d[2])
                        seen = 1;
                if (!seen) {
                    out[3 * count] = d[0];
                    out[3 * count + 1] = d[1];
                    out[3 * count + 2] = d[2];
                    ++count;
                }
            }
        }
    }
    return count;
}

/* Neighbour list of grid vertex v: ids written to nb[], count returned. */
static int grid_neighbours(int64_t X, int64_t Y, int64_t Z, int64_t v,
                           const int32_t *st, int nst, int64_t *nb)
{
    int64_t x = v % X, y = (v / X) % Y, z = v / (X * Y);
    int n = 0;
    for (int k = 0; k < nst; ++k) {
        int64_t a = x + st[3 * k], b = y + st[3 * k + 1], c = z + st[3 * k + 2];
        if (a < 0 || a >= X || b < 0 || b >= Y || c < 0 || c >= Z) continue;
        nb[n++] = a + X * b + X * Y * c;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Total order and steepest neighbours                                      */
/* ------------------------------------------------------------------------ */

/* (f(a),a) > (f(b),b) in the simulation-of-simplicity order. */
static int above(const float *f, int64_t a, int64_t b)
{
    if (f[a] > f[b]) return 1;
    if (f[a] < f[b]) return 0;
    return a > b;
}

static int64_t steepest(const float *f, int64_t X, int64_t Y, int64_t Z,
                        int64_t v, int dir, const int32_t *st, int nst)
{
    int64_t nb[32];
    int n = grid_neighbours(X, Y, Z, v, st, nst, nb);
    int64_t best = v;
    for (int k = 0; k < n; ++k) {
        if (dir > 0 ? above(f, nb[k], best) : above(f, best, nb[k]))
            best = nb[k];
    }
    return best;
}

/*
 * One-step successors: sp[v] = steepest ascent neighbour S+(v), sm[v] =
 * steepest descent neighbour S-(v), each over the closed neighbourhood
 * (Alg. 1 initialisation, and its mirror for the ascending manifold).
 */
void orc_successors(const float *f, int64_t X, int64_t Y, int64_t Z,
                    int32_t *sp, int32_t *sm)
{
    int32_t st[14 * 3];
    int nst = orc_stencil(st);
    int64_t n = X * Y * Z;
    for (int64_t v = 0; v < n; ++v) {
        sp[v] = (int32_t)steepest(f, X, Y, Z, v, +1, st, nst);
        sm[v] = (int32_t)steepest(f, X, Y, Z, v, -1, st, nst);
    }
}

/*
 * The same successors on a general simplicial complex given by the
 * adjacency of its vertices in CSR form (the problem statement takes any
 * complex K; the grid is one case): the neighbourhood of v is row v,
 * col[row_ptr[v] .. row_ptr[v+1]), closed by v itself.  For the complex's
 * 1-skeleton the rows are symmetric; the definition does not need them to
 * be.  Entries equal to v are harmless (v is already a candidate).
 */
void orc_successors_csr(const float *f, int64_t n, const int64_t *row_ptr,
                        const int32_t *col, int32_t *sp, int32_t *sm)
{
    for (int64_t v = 0; v < n; ++v) {
        int64_t hi = v, lo = v;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int64_t u = col[e];
            if (above(f, u, hi)) hi = u;
            if (above(f, lo, u)) lo = u;
        }
        sp[v] = (int32_t)hi;
        sm[v] = (int32_t)lo;
    }
}

/* ------------------------------------------------------------------------ */
/* Integral lines                                                           */
/* ------------------------------------------------------------------------ */

/*
 * Plain walk: root[v] = last vertex of v, S(v), S(S(v)), ... (the path of the
 * manifold definition, ending at the first fixed point).  O(N * path length).
 */
void orc_walk_plain(const int32_t *succ, int64_t n, int32_t *root)
{
    for (int64_t v = 0; v < n; ++v) {
        int64_t u = v;
        while (succ[u] != u) u = succ[u];
        root[v] = (int32_t)u;
    }
}

/*
 * Same result in O(N): follow the path until a vertex whose root is already
 * known (or a fixed point), then write that root back along the path.
 * `stack` must hold n entries.
 */
void orc_walk_memo(const int32_t *succ, int64_t n, int32_t *root,
                   int32_t *stack)
{
    for (int64_t v = 0; v < n; ++v) root[v] = -1;
    for (int64_t v = 0; v < n; ++v) {
        if (root[v] >= 0) continue;
        int64_t top = 0, u = v;
        while (root[u] < 0 && succ[u] != u) {
            stack[top++] = (int32_t)u;
            u = succ[u];
        }
        int32_t r = root[u] >= 0 ? root[u] : (int32_t)u;
        root[u] = r;
        while (top > 0) root[stack[--top]] = r;
    }
}

/* Root of one vertex, walking on the field directly (no successor array). */
int64_t orc_walk_from(const float *f, int64_t X, int64_t Y, int64_t Z,
                      int64_t v, int dir)
{
    int32_t st[14 * 3];
    int nst = orc_stencil(st);
    for (;;) {
        int64_t u = steepest(f, X, Y, Z, v, dir, st, nst);
        if (u == v) return v;
        v = u;
    }
}

/* ------------------------------------------------------------------------ */
/* Morse-Smale cells                                                        */
/* ------------------------------------------------------------------------ */

struct pair_maps {
    const int32_t *asc, *desc;
};

static int pair_then_id(const void *pa, const void *pb, void *ctx)
{
    const struct pair_maps *m = (const struct pair_maps *)ctx;
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (m->asc[a] != m->asc[b]) return m->asc[a] < m->asc[b] ? -1 : 1;
    if (m->desc[a] != m->desc[b]) return m->desc[a] < m->desc[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

/*
 * ms[v] = min{u : asc[u]==asc[v] && desc[u]==desc[v]}.  Sorts the vertex ids
 * by (asc, desc, id); the first id of each run is the class minimum.
 * `order` must hold n int64 entries.  Returns the number of classes.
 * Re-entrant: the comparator gets the two maps through qsort_r's argument.
 */
int64_t orc_ms_cells(const int32_t *asc, const int32_t *desc, int64_t n,
                     int32_t *ms, int64_t *order)
{
    for (int64_t v = 0; v < n; ++v) order[v] = v;
    struct pair_maps m = {asc, desc};
    qsort_r(order, (size_t)n, sizeof(int64_t), pair_then_id, &m);
    int64_t classes = 0, first = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        if (i == 0 || asc[v] != asc[order[i - 1]] ||
            desc[v] != desc[order[i - 1]]) {
            first = v;
            ++classes;
        }
        ms[v] = (int32_t)first;
    }
    return classes;
}

/* ------------------------------------------------------------------------ */
/* Pointer doubling, synchronous (worked example of Fig. 2)                 */
/* ------------------------------------------------------------------------ */

/*
 * `rounds` synchronous doubling steps d'[v] = d[d[v]] over a pointer array of
 * n entries (each round reads the previous round's array only).  `tmp` holds
 * n entries.
 */
void orc_sync_doubling(int64_t *d, int64_t n, int rounds, int64_t *tmp)
{
    for (int r = 0; r < rounds; ++r) {
        for (int64_t v = 0; v < n; ++v) tmp[v] = d[d[v]];
        memcpy(d, tmp, (size_t)n * sizeof(int64_t));
    }
}

/* ------------------------------------------------------------------------ */
/* Connected components                                                     */
/* ------------------------------------------------------------------------ */

static int64_t uf_find(int64_t *parent, int64_t v)
{
    while (parent[v] != v) {
        parent[v] = parent[parent[v]]; /* path halving */
        v = parent[v];
    }
    return v;
}

/* Union by smaller root id: the root of every set is its minimum id. */
static void uf_union(int64_t *parent, int64_t a, int64_t b)
{
    int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra;
    else parent[ra] = rb;
}

static int64_t uf_labels(int64_t *parent, const uint8_t *mask, int64_t n,
                         int64_t *label)
{
    int64_t comps = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (mask && !mask[v]) {
            label[v] = -1;
            continue;
        }
        label[v] = uf_find(parent, v);
        if (label[v] == v) ++comps;
    }
    return comps;
}

/*
 * Components of the grid graph induced by masked vertices (mask[v] != 0),
 * by union-find.  label[v] = smallest id in v's component, -1 if unmasked.
 * label doubles as the union-find forest.  Returns the number of components.
 */
int64_t orc_cc_grid_uf(const uint8_t *mask, int64_t X, int64_t Y, int64_t Z,
                       int64_t *label)
{
    int32_t st[14 * 3];
    int nst = orc_stencil(st);
    int64_t n = X * Y * Z, nb[32];
    for (int64_t v = 0; v < n; ++v) label[v] = v;
    for (int64_t v = 0; v < n; ++v) {
        if (!mask[v]) continue;
        int k = grid_neighbours(X, Y, Z, v, st, nst, nb);
        for (int i = 0; i < k; ++i)
            if (mask[nb[i]]) uf_union(label, v, nb[i]);
    }
    return uf_labels(label, mask, n, label);
}

/* Same components by breadth-first search from each unlabelled vertex in
 * increasing id order (the first vertex reached is the component minimum).
 * `queue` holds n entries. */
int64_t orc_cc_grid_bfs(const uint8_t *mask, int64_t X, int64_t Y, int64_t Z,
                        int64_t *label, int64_t *queue)
{
    int32_t st[14 * 3];
    int nst = orc_stencil(st);
    int64_t n = X * Y * Z, nb[32], comps = 0;
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (!mask[s] || label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = s;
        ++comps;
        while (head < tail) {
            int64_t v = queue[head++];
            int k = grid_neighbours(X, Y, Z, v, st, nst, nb);
            for (int i = 0; i < k; ++i) {
                if (mask[nb[i]] && label[nb[i]] < 0) {
                    label[nb[i]] = s;
                    queue[tail++] = nb[i];
                }
            }
        }
    }
    return comps;
}

/*
 * Components of a graph in CSR form (row_ptr[n+1], col_idx[row_ptr[n]]),
 * restricted to masked vertices when mask != NULL.  Edges are used in both
 * directions, so a one-sided listing is also accepted.  Returns -2 if a
 * column index is out of range.
 */
int64_t orc_cc_csr_uf(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                      const uint8_t *mask, int64_t *label)
{
    for (int64_t v = 0; v < n; ++v) label[v] = v;
    for (int64_t v = 0; v < n; ++v) {
        if (mask && !mask[v]) continue;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int64_t u = col_idx[e];
            if (u < 0 || u >= n) return -2;
            if (mask && !mask[u]) continue;
            uf_union(label, v, u);
        }
    }
    return uf_labels(label, mask, n, label);
}

/* BFS on a symmetric CSR graph; same output convention as orc_cc_csr_uf. */
int64_t orc_cc_csr_bfs(int64_t n, const int64_t *row_ptr,
                       const int32_t *col_idx, const uint8_t *mask,
                       int64_t *label, int64_t *queue)
{
    int64_t comps = 0;
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if ((mask && !mask[s]) || label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = s;
        ++comps;
        while (head < tail) {
            int64_t v = queue[head++];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int64_t u = col_idx[e];
                if (u < 0 || u >= n) return -2;
                if ((mask && !mask[u]) || label[u] >= 0) continue;
                label[u] = s;
                queue[tail++] = u;
            }
        }
    }
    return comps;
}

/* ------------------------------------------------------------------------ */
/* Full-size local-consistency checker                                      */
/* ------------------------------------------------------------------------ */

/*
 * Checks labels without walking: root[v] == v iff v is a fixed point of the
 * steepest step in direction dir, and otherwise root[v] == root[S(v)].  The
 * two conditions determine the root map uniquely (induction along strictly
 * monotone paths), so a label array passing this check equals the walk.
 * Vertices [v0, v1) are checked; returns the number of violations and the
 * first offending vertex in *first_bad (or -1).
 */
int64_t orc_check_roots(const float *f, int64_t X, int64_t Y, int64_t Z,
                        const int32_t *root, int dir, int64_t v0, int64_t v1,
                        int64_t *first_bad)
{
    int32_t st[14 * 3];
    int nst = orc_stencil(st);
    int64_t bad = 0, first = -1;
    int64_t n = X * Y * Z;
    for (int64_t v = v0; v < v1; ++v) {
        int64_t s = steepest(f, X, Y, Z, v, dir, st, nst);
        int ok;
        if (root[v] < 0 || root[v] >= n) ok = 0;
        else if (s == v) ok = (root[v] == v);
        else ok = (root[v] != v) && (root[v] == root[s]);
        if (!ok) {
            if (first < 0) first = v;
            ++bad;
        }
    }
    *first_bad = first;
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Critical points and the extremum graph                                   */
/* ------------------------------------------------------------------------ */

/*
 * The link of v (background, "Critical Points"): the top simplices of the
 * grid's triangulation that contain v, without v.  The triangulation's
 * dimension d is the number of axes longer than one; each unit d-cube over
 * those axes splits into the d! Kuhn simplices {c, c+e_a1, c+e_a1+e_a2,
 * ...}.  Writes up to 24 link simplices of d vertices each (unused slots
 * -1) and returns their number; *dim receives d.
 */
static int link_simplices(int64_t X, int64_t Y, int64_t Z, int64_t v,
                          int64_t out[24][3], int *dim)
{
    const int64_t ext[3] = {X, Y, Z}, stride[3] = {1, X, X * Y};
    const int64_t p[3] = {v % X, (v / X) % Y, v / (X * Y)};
    int axes[3], d = 0;
    for (int a = 0; a < 3; ++a)
        if (ext[a] > 1) axes[d++] = a;
    *dim = d;
    if (d == 0) return 0;
    int perms[6][3], np = 0;
    /* all orderings of the d active axes */
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            for (int k = 0; k < d; ++k) {
                int o[3] = {i, j, k};
                int ok = 1;
                for (int q = 0; q < d; ++q)
                    for (int r = q + 1; r < d; ++r)
                        if (o[q] == o[r]) ok = 0;
                if (!ok) continue;
                int dup = 0;
                for (int q = 0; q < np; ++q) {
                    int same = 1;
                    for (int r = 0; r < d; ++r)
                        if (perms[q][r] != axes[o[r]]) same = 0;
                    if (same) dup = 1;
                }
                if (dup) continue;
                for (int r = 0; r < d; ++r) perms[np][r] = axes[o[r]];
                ++np;
            }
    int n = 0;
    /* cubes whose lower corner c has c_a in {p_a - 1, p_a} on active axes */
    for (int mask = 0; mask < (1 << d); ++mask) {
        int64_t c[3] = {p[0], p[1], p[2]};
        int inside = 1;
        for (int r = 0; r < d; ++r) {
            const int a = axes[r];
            if (mask & (1 << r)) c[a] -= 1;
            if (c[a] < 0 || c[a] + 1 >= ext[a]) inside = 0;
        }
        if (!inside) continue;
        for (int q = 0; q < np; ++q) {
            int64_t corner[3] = {c[0], c[1], c[2]};
            int64_t ids[4];
            ids[0] = corner[0] * stride[0] + corner[1] * stride[1] +
                     corner[2] * stride[2];
            for (int r = 0; r < d; ++r) {
                corner[perms[q][r]] += 1;
                ids[r + 1] = corner[0] * stride[0] + corner[1] * stride[1] +
                             corner[2] * stride[2];
            }
            int has = 0;
            for (int r = 0; r <= d; ++r)
                if (ids[r] == v) has = 1;
            if (!has) continue;
            int w = 0;
            for (int r = 0; r < 3; ++r) out[n][r] = -1;
            for (int r = 0; r <= d; ++r)
                if (ids[r] != v) out[n][w++] = ids[r];
            ++n;
        }
    }
    return n;
}

static int64_t lk_find(int64_t *par, int64_t i)
{
    while (par[i] != i) i = par[i];
    return i;
}

/*
 * Lower (side = -1) or upper (side = +1) link of v restricted to the
 * vertices below / above v in the (f, id) order: its connected components
 * (through the link's edges) and its Euler characteristic (vertices - edges
 * + triangles).  comp[k] receives the component (0-based) of lv[k], the
 * k-th distinct link vertex on that side; returns the component count.
 */
static int link_side(const float *f, int64_t X, int64_t Y, int64_t Z,
                     int64_t v, int side, int64_t *lv, int *nlv, int *comp,
                     int *chi)
{
    int64_t simp[24][3];
    int d;
    const int ns = link_simplices(X, Y, Z, v, simp, &d);
    int nv = 0;
    for (int s = 0; s < ns; ++s)
        for (int r = 0; r < d; ++r) {
            const int64_t u = simp[s][r];
            const int keep = side > 0 ? above(f, u, v) : above(f, v, u);
            if (!keep) continue;
            int seen = 0;
            for (int q = 0; q < nv; ++q)
                if (lv[q] == u) seen = 1;
            if (!seen) lv[nv++] = u;
        }
    int64_t par[64];
    for (int q = 0; q < nv; ++q) par[q] = q;
    /* distinct edges and triangles whose vertices are all on the side */
    int64_t edges[72][2];
    int ne = 0, nt = 0;
    for (int s = 0; s < ns; ++s) {
        int all = 1;
        for (int r = 0; r < d; ++r) {
            const int64_t u = simp[s][r];
            if (!(side > 0 ? above(f, u, v) : above(f, v, u))) all = 0;
        }
        if (d == 3 && all) ++nt;  /* top link simplices are distinct */
        for (int a = 0; a < d; ++a)
            for (int b = a + 1; b < d; ++b) {
                int64_t u = simp[s][a], w = simp[s][b];
                const int ua = side > 0 ? above(f, u, v) : above(f, v, u);
                const int wa = side > 0 ? above(f, w, v) : above(f, v, w);
                if (!ua || !wa) continue;
                if (u > w) { int64_t t = u; u = w; w = t; }
                int seen = 0;
                for (int q = 0; q < ne; ++q)
                    if (edges[q][0] == u && edges[q][1] == w) seen = 1;
                if (seen) continue;
                edges[ne][0] = u;
                edges[ne][1] = w;
                ++ne;
                int iu = 0, iw = 0;
                for (int q = 0; q < nv; ++q) {
                    if (lv[q] == u) iu = q;
                    if (lv[q] == w) iw = q;
                }
                const int64_t ru = lk_find(par, iu), rw = lk_find(par, iw);
                if (ru != rw) par[ru > rw ? ru : rw] = ru < rw ? ru : rw;
            }
    }
    int nc = 0;
    int64_t rootid[64];
    for (int q = 0; q < nv; ++q) {
        const int64_t r = lk_find(par, q);
        int found = -1;
        for (int c = 0; c < nc; ++c)
            if (rootid[c] == r) found = c;
        if (found < 0) { rootid[nc] = r; found = nc++; }
        comp[q] = found;
    }
    *nlv = nv;
    *chi = nv - ne + nt;
    return nc;
}

/*
 * Per vertex: lc = components of the lower link, uc = components of the
 * upper link (lc = 0: minimum, uc = 0: maximum, lc = uc = 1: regular,
 * otherwise a saddle), chi = Euler characteristic of the lower link.
 * Banchoff's critical point theorem makes sum(1 - chi) the Euler
 * characteristic of the domain.
 */
void orc_critical(const float *f, int64_t X, int64_t Y, int64_t Z,
                  uint8_t *lc, uint8_t *uc, int32_t *chi)
{
    const int64_t n = X * Y * Z;
    int64_t lv[64];
    int comp[64], nlv, c;
    for (int64_t v = 0; v < n; ++v) {
        lc[v] = (uint8_t)link_side(f, X, Y, Z, v, -1, lv, &nlv, comp, &c);
        chi[v] = c;
        uc[v] = (uint8_t)link_side(f, X, Y, Z, v, +1, lv, &nlv, comp, &c);
    }
}

/*
 * Extremum graph: for every vertex whose upper link has two or more
 * components, one edge per component to the maximum that steepest ascent
 * reaches from the component's highest vertex (asc of it), tagged +1; the
 * same through the lower link, its lowest vertices and desc, tagged -1.
 * Edges go to out[3*k .. 3*k+2] = (vertex, extremum, tag) for k < cap, by
 * increasing vertex, +1 edges first, components by increasing id of that
 * highest / lowest vertex.  Returns the number of edges.
 */
int64_t orc_extremum_edges(const float *f, int64_t X, int64_t Y, int64_t Z,
                           const int32_t *asc, const int32_t *desc,
                           int32_t *out, int64_t cap)
{
    const int64_t n = X * Y * Z;
    int64_t count = 0;
    int64_t lv[64];
    int comp[64], nlv, chi;
    for (int64_t v = 0; v < n; ++v) {
        for (int side = +1; side >= -1; side -= 2) {
            const int nc = link_side(f, X, Y, Z, v, side, lv, &nlv, comp, &chi);
            if (nc < 2) continue;
            int64_t ext[64];
            for (int c = 0; c < nc; ++c) {
                int64_t best = -1;
                for (int q = 0; q < nlv; ++q) {
                    if (comp[q] != c) continue;
                    if (best < 0 || (side > 0 ? above(f, lv[q], best)
                                              : above(f, best, lv[q])))
                        best = lv[q];
                }
                ext[c] = best;
            }
            /* components by increasing id of their extreme vertex */
            for (int a = 1; a < nc; ++a)
                for (int b = a; b > 0 && ext[b - 1] > ext[b]; --b) {
                    int64_t t = ext[b]; ext[b] = ext[b - 1]; ext[b - 1] = t;
                }
            for (int c = 0; c < nc; ++c) {
                if (count < cap) {
                    out[3 * count] = (int32_t)v;
                    out[3 * count + 1] = side > 0 ? asc[ext[c]] : desc[ext[c]];
                    out[3 * count + 2] = side;
                }
                ++count;
            }
        }
    }
    return count;
}

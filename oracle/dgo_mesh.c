/*
 * Oracle: periodic Cartesian quadtree mesh.  TEST INFRASTRUCTURE ONLY (see dgo.h).
 *
 * Leaves of a quadtree are the elements; a leaf of level l on an nx0 x ny0
 * root grid covers [x0 + ix Lx/(nx0 2^l), x0 + (ix+1) Lx/(nx0 2^l)] x [...]
 * (Sec. 3.1: quadtree with leaves as elements).  Neighbouring leaves differ by
 * at most one level across a face (Sec. 2.2: 2-to-1 nonconforming interfaces).
 * Every face is classified as conforming, small side of a mortar, large side
 * of a mortar, or (on a non-periodic domain side) boundary; mortars are
 * numbered in order of (large element, face).
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dgo.h"

typedef struct {
    uint64_t key;
    int64_t id;
} kv;

static uint64_t mkkey(int l, int64_t ix, int64_t iy)
{
    return ((uint64_t)l << 56) | ((uint64_t)ix << 28) | (uint64_t)iy;
}

static int kvcmp(const void* a, const void* b)
{
    uint64_t x = ((const kv*)a)->key, y = ((const kv*)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
    kv* tab;
    int64_t n;
    int nx0, ny0;
} lookup;

static int64_t find(const lookup* L, int l, int64_t ix, int64_t iy)
{
    if (l < 0) return -1;
    int64_t nx = (int64_t)L->nx0 << l, ny = (int64_t)L->ny0 << l;
    ix = ((ix % nx) + nx) % nx;
    iy = ((iy % ny) + ny) % ny;
    kv q = {mkkey(l, ix, iy), 0};
    kv* r = (kv*)bsearch(&q, L->tab, (size_t)L->n, sizeof(kv), kvcmp);
    return r ? r->id : -1;
}

int dgo_mesh_build(dgo_mesh* m, int N, int64_t E, const int8_t* level, const int32_t* ix,
                   const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                   int ny0, char* err, int errlen)
{
    return dgo_mesh_build_bc(m, N, E, level, ix, iy, x0, y0, Lx, Ly, nx0, ny0, 0, 0, err, errlen);
}

int dgo_mesh_build_bc(dgo_mesh* m, int N, int64_t E, const int8_t* level, const int32_t* ix,
                      const int32_t* iy, double x0, double y0, double Lx, double Ly, int nx0,
                      int ny0, const int* bc, const double* ext, char* err, int errlen)
{
    memset(m, 0, sizeof(*m));
    if (bc) {
        for (int f = 0; f < 4; ++f) {
            if (bc[f] < BC_PERIODIC || bc[f] > BC_OUTFLOW) {
                snprintf(err, errlen, "unknown boundary condition %d", bc[f]);
                return -1;
            }
            m->bc[f] = bc[f];
        }
        if ((m->bc[0] == BC_PERIODIC) != (m->bc[1] == BC_PERIODIC) ||
            (m->bc[2] == BC_PERIODIC) != (m->bc[3] == BC_PERIODIC)) {
            snprintf(err, errlen, "opposite sides must both be periodic or both not");
            return -1;
        }
    }
    if (dgo_basis_init(&m->B, N)) {
        snprintf(err, errlen, "unsupported N=%d", N);
        return -1;
    }
    m->E = E;
    m->x0 = x0;
    m->y0 = y0;
    m->Lx = Lx;
    m->Ly = Ly;
    m->nx0 = nx0;
    m->ny0 = ny0;
    m->level = (int8_t*)malloc(E);
    m->ix = (int32_t*)malloc(E * 4);
    m->iy = (int32_t*)malloc(E * 4);
    m->hx = (double*)malloc(E * 8);
    m->hy = (double*)malloc(E * 8);
    m->face = (dgo_face*)malloc(E * 4 * sizeof(dgo_face));
    memcpy(m->level, level, E);
    memcpy(m->ix, ix, E * 4);
    memcpy(m->iy, iy, E * 4);

    lookup L;
    L.n = E;
    L.nx0 = nx0;
    L.ny0 = ny0;
    L.tab = (kv*)malloc(E * sizeof(kv));
    double area = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        int l = level[e];
        if (l < 0 || l > 24 || ix[e] < 0 || iy[e] < 0 || ix[e] >= ((int64_t)nx0 << l) ||
            iy[e] >= ((int64_t)ny0 << l)) {
            snprintf(err, errlen, "leaf %lld out of range", (long long)e);
            free(L.tab);
            return -2;
        }
        L.tab[e].key = mkkey(l, ix[e], iy[e]);
        L.tab[e].id = e;
        m->hx[e] = Lx / (double)((int64_t)nx0 << l);
        m->hy[e] = Ly / (double)((int64_t)ny0 << l);
        area += 1.0 / (double)(1LL << (2 * l));
    }
    qsort(L.tab, (size_t)E, sizeof(kv), kvcmp);
    for (int64_t i = 1; i < E; ++i)
        if (L.tab[i].key == L.tab[i - 1].key) {
            snprintf(err, errlen, "duplicate leaf");
            free(L.tab);
            return -2;
        }
    /* tiling: no leaf has a leaf ancestor, and the areas add up */
    for (int64_t e = 0; e < E; ++e) {
        int64_t cx = ix[e], cy = iy[e];
        for (int l = level[e] - 1; l >= 0; --l) {
            cx >>= 1;
            cy >>= 1;
            if (find(&L, l, cx, cy) >= 0) {
                snprintf(err, errlen, "overlapping leaves");
                free(L.tab);
                return -2;
            }
        }
    }
    if (area < (double)nx0 * ny0 * (1 - 1e-12) || area > (double)nx0 * ny0 * (1 + 1e-12)) {
        snprintf(err, errlen, "leaves do not tile the domain");
        free(L.tab);
        return -2;
    }

    /* face classification */
    int64_t nmort = 0;
    for (int64_t e = 0; e < E; ++e) {
        int l = level[e];
        for (int f = 0; f < 4; ++f) {
            dgo_face* F = &m->face[e * 4 + f];
            F->mortar = -1;
            F->half = 0;
            F->nbr = -1;
            int dx = f == 0 ? -1 : (f == 1 ? 1 : 0);
            int dy = f == 2 ? -1 : (f == 3 ? 1 : 0);
            int64_t nx = (int64_t)ix[e] + dx, ny = (int64_t)iy[e] + dy;
            /* a face on a non-periodic domain side */
            if (m->bc[f] != BC_PERIODIC &&
                (nx < 0 || ny < 0 || nx >= ((int64_t)nx0 << l) || ny >= ((int64_t)ny0 << l))) {
                F->type = FACE_BOUNDARY;
                F->bnode = m->NB;
                m->NB += N + 1;
                continue;
            }
            int64_t g = find(&L, l, nx, ny);
            if (g >= 0) {
                F->type = FACE_CONF;
                F->nbr = g;
                continue;
            }
            int64_t nxl = (int64_t)nx0 << l, nyl = (int64_t)ny0 << l;
            int64_t wx = ((nx % nxl) + nxl) % nxl, wy = ((ny % nyl) + nyl) % nyl;
            g = find(&L, l - 1, wx >> 1, wy >> 1);
            if (g >= 0) {
                F->type = FACE_SMALL;
                F->nbr = g;
                F->half = (f < 2) ? (iy[e] & 1) : (ix[e] & 1);
                continue;
            }
            /* two finer leaves across the face */
            int64_t c0x, c0y, c1x, c1y;
            if (f < 2) {
                int64_t cx = 2 * wx + (f == 0 ? 1 : 0);
                c0x = c1x = cx;
                c0y = 2 * wy;
                c1y = 2 * wy + 1;
            } else {
                int64_t cy = 2 * wy + (f == 2 ? 1 : 0);
                c0y = c1y = cy;
                c0x = 2 * wx;
                c1x = 2 * wx + 1;
            }
            int64_t s0 = find(&L, l + 1, c0x, c0y), s1 = find(&L, l + 1, c1x, c1y);
            if (s0 < 0 || s1 < 0) {
                snprintf(err, errlen, "mesh not 2:1 balanced at leaf %lld face %d", (long long)e,
                         f);
                free(L.tab);
                return -3;
            }
            F->type = FACE_LARGE;
            F->mortar = nmort++;
        }
    }
    m->M = nmort;
    m->bkind = (int8_t*)malloc(m->NB > 0 ? m->NB : 1);
    m->bext = (double*)calloc((m->NB > 0 ? m->NB : 1) * 4, sizeof(double));
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) {
            const dgo_face* F = &m->face[e * 4 + f];
            if (F->type != FACE_BOUNDARY) continue;
            for (int k = 0; k <= N; ++k) {
                m->bkind[F->bnode + k] = (int8_t)m->bc[f];
                if (ext)
                    for (int v = 0; v < 4; ++v) m->bext[(F->bnode + k) * 4 + v] = ext[f * 4 + v];
            }
        }
    m->mort = (dgo_mortar*)malloc((nmort > 0 ? nmort : 1) * sizeof(dgo_mortar));
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) {
            dgo_face* F = &m->face[e * 4 + f];
            if (F->type != FACE_LARGE) continue;
            dgo_mortar* M = &m->mort[F->mortar];
            M->large = e;
            M->face = f;
            int l = level[e];
            int64_t nxl = (int64_t)nx0 << l, nyl = (int64_t)ny0 << l;
            int dx = f == 0 ? -1 : (f == 1 ? 1 : 0);
            int dy = f == 2 ? -1 : (f == 3 ? 1 : 0);
            int64_t wx = ((ix[e] + dx) % nxl + nxl) % nxl, wy = ((iy[e] + dy) % nyl + nyl) % nyl;
            for (int h = 0; h < 2; ++h) {
                int64_t cx, cy;
                if (f < 2) {
                    cx = 2 * wx + (f == 0 ? 1 : 0);
                    cy = 2 * wy + h;
                } else {
                    cy = 2 * wy + (f == 2 ? 1 : 0);
                    cx = 2 * wx + h;
                }
                int64_t s = find(&L, l + 1, cx, cy);
                M->small[h] = s;
                dgo_face* G = &m->face[s * 4 + (f ^ 1)];
                if (G->type != FACE_SMALL || G->nbr != e || G->half != h) {
                    snprintf(err, errlen, "inconsistent mortar at leaf %lld", (long long)e);
                    free(L.tab);
                    return -3;
                }
                G->mortar = F->mortar;
            }
        }
    free(L.tab);
    return 0;
}

void dgo_mesh_release(dgo_mesh* m)
{
    free(m->level);
    free(m->ix);
    free(m->iy);
    free(m->hx);
    free(m->hy);
    free(m->face);
    free(m->mort);
    free(m->bkind);
    free(m->bext);
    memset(m, 0, sizeof(*m));
}

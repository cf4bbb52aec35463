/*
 * rg_oracle.c -- TEST INFRASTRUCTURE ONLY.  The slow, plain FP64 CPU oracle
 * for the ray-tracing path.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes, and where the paper states it:
 *   - the two-level scene: instances with object->world matrices over
 *     triangle meshes (section 1, the two-layered structure built from the
 *     models' vertices and transformation matrices);
 *   - per ray, the closest-hit / any-hit / miss outcome (section 1, closest
 *     hit, any hit and miss shaders, invoked for each ray);
 *   - recursive spawning of shadow, reflection and refraction rays up to a
 *     capped depth, each carrying a payload (section 1 with its footnote on
 *     the recursion limit; section 2.1 Render System for reflection,
 *     refraction and shadow casting; material properties used by shaders);
 *   - ambient-occlusion rays for the incoherent workload (not in the paper:
 *     the definition of the incoherent workload, stated in oracle/__init__.py).
 *
 * Closest hit is an exact-result method: a hierarchy only reaches the
 * brute-force answer faster.  So the oracle is the definition written out:
 * every triangle of every instance is tested with the classic Moller-Trumbore
 * test (Moller & Trumbore 1997) in double precision; the nearest t in the
 * closed interval [tmin, tmax] wins; exact ties go to the lowest
 * (instance, primitive).  It is a different formulation from the GPU's
 * sheared watertight test, so the two check each other.
 *
 * Besides the answer, each ray gets an ambiguity flag (`amb`) and a tie set.
 * A float32 implementation of the same definition may legitimately differ
 * from float64 where a triangle edge, the interval ends, or a grazing angle
 * lies within float32's error band of the ray; those rays are flagged and the
 * parity tests skip them (and report how many).  The band model:
 *   beta_j  = (K*2^-24*R_j + sigma_obj(t_j)) * P_j * |d| / |S_j|   (barycentric)
 *   delta_j = (K*2^-24*R_j + sigma_obj(t_j)) * |n_j| / |S_j| + K*2^-24*|t_j|  (t units)
 * with R_j the largest distance from the origin point used by a float32
 * traversal (the object-space ray moved to where it enters the mesh's box,
 * not before tmin) to the triangle's vertices plus that point's own distance
 * from the object-space origin, P_j the perimeter, n_j = e1 x e2, S_j = d.n_j,
 * all in object space, K = 4, and sigma_obj the propagated uncertainty of a
 * secondary ray's origin and direction (zero for rays given as input).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_K 4.0
#define OR_EPS32 (1.0 / 16777216.0) /* 2^-24 */
#define OR_MISS 0xFFFFFFFFu

typedef struct {
    double *tri;        /* [T][9]: a, e1 = b-a, e2 = c-a */
    int64_t n;
    const uint16_t *prim_mat; /* borrowed, may be NULL */
    const uint32_t *idx;      /* borrowed vertex indices [T][3] */
    int32_t *nbr;             /* [T][3] triangle across edge s (s=0: bc, 1: ca, 2: ab), -1 if none */
    int8_t *nslot;            /* [T][3] that edge's slot in the neighbour */
    double lo[3], hi[3];      /* object-space box of the vertices */
    double sc[3], sr;         /* bounding sphere */
    const uint64_t *alpha;    /* borrowed, may be NULL: opacity of 4^alpha_level micro-triangles per triangle */
    int32_t alpha_level;
} or_blas;

typedef struct {
    double m[12];   /* object -> world, row-major 3x4 */
    double inv[12]; /* world -> object */
    double det;     /* det of the linear part */
    double inv_fro; /* Frobenius norm of the inverse's linear part */
    double wlo[3], whi[3]; /* world box of the transformed mesh box */
    int32_t blas;
    uint32_t mat;
    uint32_t flags; /* bits 0-7 visibility mask, OR_INST_CULL_DISABLE, OR_INST_FLIP_FACING */
} or_inst;

/* Ray visibility and facing (the accept / ignore semantics of an any-hit
 * stage, in the form of the RTX / Vulkan instance masks and cull flags): an
 * instance is seen by a ray only if its 8-bit mask and the ray's share a bit;
 * a triangle faces the ray when the ray travels against its winding normal
 * (e1 x e2) in object space, inverted for instances flagged FLIP_FACING;
 * CULL_BACK / CULL_FRONT ignore triangles that face away from / towards the
 * ray, except in instances flagged CULL_DISABLE. */
#define OR_RAY_CULL_BACK 1u
#define OR_RAY_CULL_FRONT 2u
#define OR_INST_CULL_DISABLE (1u << 8)
#define OR_INST_FLIP_FACING (1u << 9)

typedef struct {
    int32_t type;
    double rgb[3];
    double ior;
} or_mat;

typedef struct {
    or_blas *blas;
    int32_t nb;
    or_inst *inst;
    int64_t ni;
    int sphere_reject;
    or_mat *mats;
    int32_t nm;
    int64_t tests; /* running count of ray-triangle tests (approximate under threads) */
    int adj_built;
    pthread_mutex_t adj_lock;
} or_scene;

/* ---------------------------------------------------------------- vectors */
static inline void v_sub(double r[3], const double a[3], const double b[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static inline double v_dot(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void v_cross(double r[3], const double a[3], const double b[3]) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static inline double v_len(const double a[3]) { return sqrt(v_dot(a, a)); }
static inline void v_norm(double a[3]) {
    double l = v_len(a);
    a[0] /= l; a[1] /= l; a[2] /= l;
}
static inline double maxabs3(const double a[3]) {
    double m = fabs(a[0]);
    if (fabs(a[1]) > m) m = fabs(a[1]);
    if (fabs(a[2]) > m) m = fabs(a[2]);
    return m;
}

/* Affine 3x4 inverse in double (adjugate / determinant). */
static int inv34(const double m[12], double out[12], double *det_out) {
    double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], g = m[8], h = m[9], i = m[10];
    double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
    double det = a * A + b * B + c * C;
    *det_out = det;
    if (det == 0.0 || !isfinite(det)) return -1;
    double r[9];
    r[0] = A / det; r[1] = -(b * i - c * h) / det; r[2] = (b * f - c * e) / det;
    r[3] = B / det; r[4] = (a * i - c * g) / det;  r[5] = -(a * f - c * d) / det;
    r[6] = C / det; r[7] = -(a * h - b * g) / det; r[8] = (a * e - b * d) / det;
    double t[3] = {m[3], m[7], m[11]};
    for (int k = 0; k < 3; ++k) {
        out[4 * k + 0] = r[3 * k + 0];
        out[4 * k + 1] = r[3 * k + 1];
        out[4 * k + 2] = r[3 * k + 2];
        out[4 * k + 3] = -(r[3 * k + 0] * t[0] + r[3 * k + 1] * t[1] + r[3 * k + 2] * t[2]);
    }
    return 0;
}

static inline void xf_point(const double m[12], const double p[3], double r[3]) {
    for (int k = 0; k < 3; ++k) r[k] = m[4 * k] * p[0] + m[4 * k + 1] * p[1] + m[4 * k + 2] * p[2] + m[4 * k + 3];
}
static inline void xf_vec(const double m[12], const double p[3], double r[3]) {
    for (int k = 0; k < 3; ++k) r[k] = m[4 * k] * p[0] + m[4 * k + 1] * p[1] + m[4 * k + 2] * p[2];
}
/* transpose of the linear part applied to p (used with the inverse: normal transform) */
static inline void xf_vec_t(const double m[12], const double p[3], double r[3]) {
    for (int k = 0; k < 3; ++k) r[k] = m[k] * p[0] + m[4 + k] * p[1] + m[8 + k] * p[2];
}

/* ------------------------------------------------------------- the scene */
or_scene *or_scene_new(int32_t n_blas, const int64_t *vert_off, const int64_t *tri_off,
                       const float *verts, const uint32_t *idx, const uint16_t *prim_mat,
                       int64_t n_inst, const float *xform, const uint32_t *blas_id,
                       const uint32_t *inst_mat) {
    or_scene *s = (or_scene *)calloc(1, sizeof(or_scene));
    s->nb = n_blas;
    s->blas = (or_blas *)calloc((size_t)n_blas, sizeof(or_blas));
    for (int32_t b = 0; b < n_blas; ++b) {
        or_blas *B = &s->blas[b];
        int64_t t0 = tri_off[b], t1 = tri_off[b + 1];
        const float *V = verts + 3 * vert_off[b];
        int64_t nv = vert_off[b + 1] - vert_off[b];
        B->n = t1 - t0;
        B->tri = (double *)malloc(sizeof(double) * 9 * (size_t)(B->n > 0 ? B->n : 1));
        B->prim_mat = prim_mat ? prim_mat + t0 : NULL;
        B->idx = idx + 3 * t0;
        for (int k = 0; k < 3; ++k) { B->lo[k] = INFINITY; B->hi[k] = -INFINITY; }
        for (int64_t v = 0; v < nv; ++v)
            for (int k = 0; k < 3; ++k) {
                double x = V[3 * v + k];
                if (x < B->lo[k]) B->lo[k] = x;
                if (x > B->hi[k]) B->hi[k] = x;
            }
        for (int64_t t = 0; t < B->n; ++t) {
            const uint32_t *I = idx + 3 * (t0 + t);
            double a[3], bb[3], c[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = V[3 * I[0] + k]; bb[k] = V[3 * I[1] + k]; c[k] = V[3 * I[2] + k];
            }
            double *T = B->tri + 9 * t;
            for (int k = 0; k < 3; ++k) { T[k] = a[k]; T[3 + k] = bb[k] - a[k]; T[6 + k] = c[k] - a[k]; }
        }
        double r2 = 0.0;
        for (int k = 0; k < 3; ++k) B->sc[k] = 0.5 * (B->lo[k] + B->hi[k]);
        for (int64_t v = 0; v < nv; ++v) {
            double p[3] = {V[3 * v], V[3 * v + 1], V[3 * v + 2]}, q[3];
            v_sub(q, p, B->sc);
            double l2 = v_dot(q, q);
            if (l2 > r2) r2 = l2;
        }
        B->sr = sqrt(r2) * (1.0 + 1e-9) + 1e-12;
    }
    s->ni = n_inst;
    s->inst = (or_inst *)calloc((size_t)(n_inst > 0 ? n_inst : 1), sizeof(or_inst));
    for (int64_t i = 0; i < n_inst; ++i) {
        or_inst *I = &s->inst[i];
        for (int k = 0; k < 12; ++k) I->m[k] = xform[12 * i + k];
        inv34(I->m, I->inv, &I->det);
        double f = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) f += I->inv[4 * r + c] * I->inv[4 * r + c];
        I->inv_fro = sqrt(f);
        I->blas = (int32_t)blas_id[i];
        I->mat = inst_mat[i];
        I->flags = 0xFFu;
        const or_blas *B = &s->blas[I->blas];
        for (int k = 0; k < 3; ++k) { I->wlo[k] = INFINITY; I->whi[k] = -INFINITY; }
        for (int c = 0; c < 8; ++c) {
            double p[3] = {(c & 1) ? B->hi[0] : B->lo[0], (c & 2) ? B->hi[1] : B->lo[1],
                           (c & 4) ? B->hi[2] : B->lo[2]}, w[3];
            xf_point(I->m, p, w);
            for (int k = 0; k < 3; ++k) {
                if (w[k] < I->wlo[k]) I->wlo[k] = w[k];
                if (w[k] > I->whi[k]) I->whi[k] = w[k];
            }
        }
    }
    s->sphere_reject = 0;
    s->adj_built = 0;
    pthread_mutex_init(&s->adj_lock, NULL);
    return s;
}

/* Edge adjacency of each mesh (by vertex index): an edge shared by exactly
 * two triangles links them; boundary and non-manifold edges link nothing. */
typedef struct {
    uint64_t key;
    uint32_t tri;
    uint32_t slot;
} or_edge;

static int edge_cmp(const void *x, const void *y) {
    const or_edge *a = (const or_edge *)x, *b = (const or_edge *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->tri != b->tri) return a->tri < b->tri ? -1 : 1;
    return (int)a->slot - (int)b->slot;
}

static void build_adjacency(or_blas *B) {
    int64_t m = 3 * B->n;
    B->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    B->nslot = (int8_t *)malloc((size_t)(m > 0 ? m : 1));
    or_edge *e = (or_edge *)malloc(sizeof(or_edge) * (size_t)(m > 0 ? m : 1));
    for (int64_t t = 0; t < B->n; ++t) {
        const uint32_t *I = B->idx + 3 * t;
        for (int sl = 0; sl < 3; ++sl) {
            /* slot 0: edge (b,c); 1: (c,a); 2: (a,b) */
            uint32_t p = I[(sl + 1) % 3], q = I[(sl + 2) % 3];
            uint32_t lo = p < q ? p : q, hi = p < q ? q : p;
            e[3 * t + sl].key = ((uint64_t)lo << 32) | hi;
            e[3 * t + sl].tri = (uint32_t)t;
            e[3 * t + sl].slot = (uint32_t)sl;
            B->nbr[3 * t + sl] = -1;
            B->nslot[3 * t + sl] = -1;
        }
    }
    qsort(e, (size_t)m, sizeof(or_edge), edge_cmp);
    for (int64_t i = 0; i < m;) {
        int64_t j = i;
        while (j < m && e[j].key == e[i].key) ++j;
        if (j - i == 2 && e[i].tri != e[i + 1].tri) {
            B->nbr[3 * (int64_t)e[i].tri + e[i].slot] = (int32_t)e[i + 1].tri;
            B->nslot[3 * (int64_t)e[i].tri + e[i].slot] = (int8_t)e[i + 1].slot;
            B->nbr[3 * (int64_t)e[i + 1].tri + e[i + 1].slot] = (int32_t)e[i].tri;
            B->nslot[3 * (int64_t)e[i + 1].tri + e[i + 1].slot] = (int8_t)e[i].slot;
        }
        i = j;
    }
    free(e);
}

static void ensure_adjacency(or_scene *s) {
    pthread_mutex_lock(&s->adj_lock);
    if (!s->adj_built) {
        for (int32_t b = 0; b < s->nb; ++b) build_adjacency(&s->blas[b]);
        s->adj_built = 1;
    }
    pthread_mutex_unlock(&s->adj_lock);
}

void or_scene_free(or_scene *s) {
    if (!s) return;
    for (int32_t b = 0; b < s->nb; ++b) {
        free(s->blas[b].tri);
        free(s->blas[b].nbr);
        free(s->blas[b].nslot);
    }
    pthread_mutex_destroy(&s->adj_lock);
    free(s->blas);
    free(s->inst);
    free(s->mats);
    free(s);
}

void or_set_sphere_reject(or_scene *s, int32_t on) { s->sphere_reject = on; }

/* Per-instance visibility mask and facing flags (default: mask 0xFF, none). */
void or_set_inst_flags(or_scene *s, const uint32_t *flags) {
    for (int64_t i = 0; i < s->ni; ++i) s->inst[i].flags = flags[i];
}

/* Opacity masks (alpha-tested triangles): triangle j of bottom level b is
 * split into 4^level micro-triangles by cutting each edge into n = 2^level
 * equal parts; in barycentric coordinates (u, v) (the weights of the second
 * and third vertex) scaled by n, the cell (i, j) = (floor U, floor V) holds an
 * upright micro-triangle (fractional parts summing to at most 1) and, unless
 * it touches the far edge, an inverted one; they are numbered row by row
 * (row j starts at j (2n - j)), upright 2i, inverted 2i + 1.  Bit k of the
 * triangle's mask set: micro-triangle k is opaque (its hits are accepted). */
void or_set_alpha(or_scene *s, int32_t b, const uint64_t *alpha, int32_t level) {
    s->blas[b].alpha = alpha;
    s->blas[b].alpha_level = level;
}

static int alpha_index(int level, double u, double v) {
    const int n = 1 << level;
    const double U = u * n, V = v * n;
    int i = (int)floor(U), j = (int)floor(V);
    if (i < 0) i = 0;
    if (j < 0) j = 0;
    if (i > n - 1) i = n - 1;
    if (j > n - 1 - i) j = n - 1 - i;
    const int inverted = (U - i) + (V - j) > 1.0 && i + j < n - 1;
    return j * (2 * n - j) + 2 * i + inverted;
}

/* 1: the hit at (u, v) is accepted; 0: ignored. */
static int alpha_open(const or_blas *B, int64_t j, double u, double v) {
    if (!B->alpha) return 1;
    return (int)((B->alpha[j] >> alpha_index(B->alpha_level, u, v)) & 1u);
}

/* As alpha_open, or -1 when float32 barycentrics within `beta` of (u, v)
 * could fall on a micro-triangle of the other opacity: within 2 beta of a
 * cut line (U, V or U + V an integer, the triangle's own edges included)
 * of a triangle whose micro-triangles are not all alike. */
static int alpha_state(const or_blas *B, int64_t j, double u, double v, double beta) {
    if (!B->alpha) return 1;
    const int n = 1 << B->alpha_level;
    const uint64_t all = n == 8 ? ~0ull : ((1ull << (n * n)) - 1ull);
    const uint64_t m = B->alpha[j] & all;
    const int open = (int)((B->alpha[j] >> alpha_index(B->alpha_level, u, v)) & 1u);
    if (m == 0 || m == all) return open;
    const double U = u * n, V = v * n, S = U + V;
    const double d = fmin(fmin(fabs(U - nearbyint(U)), fabs(V - nearbyint(V))), fabs(S - nearbyint(S)) / 1.4142135623730951);
    return d <= 2.0 * beta * n ? -1 : open;
}

/* Whether triangle T of instance I is ignored by a ray with cull flags
 * `cull` travelling along object-space d. */
static inline int culled(const or_inst *I, uint32_t cull, const double *T, const double d[3]) {
    if (!(cull & (OR_RAY_CULL_BACK | OR_RAY_CULL_FRONT)) || (I->flags & OR_INST_CULL_DISABLE)) return 0;
    double n[3];
    v_cross(n, T + 3, T + 6);
    int front = v_dot(d, n) < 0.0;
    if (I->flags & OR_INST_FLIP_FACING) front = !front;
    return front ? (cull & OR_RAY_CULL_FRONT) != 0 : (cull & OR_RAY_CULL_BACK) != 0;
}

/* materials: type i32, rgb f32[3], ior f32 -> 20-byte records */
void or_set_materials(or_scene *s, const void *rows, int32_t n) {
    free(s->mats);
    s->mats = (or_mat *)calloc((size_t)(n > 0 ? n : 1), sizeof(or_mat));
    s->nm = n;
    const unsigned char *p = (const unsigned char *)rows;
    for (int32_t i = 0; i < n; ++i) {
        int32_t t;
        float f[4];
        memcpy(&t, p + 20 * i, 4);
        memcpy(f, p + 20 * i + 4, 16);
        s->mats[i].type = t;
        for (int k = 0; k < 3; ++k) s->mats[i].rgb[k] = f[k];
        s->mats[i].ior = f[3];
    }
}

int64_t or_tests(const or_scene *s) { return s->tests; }

/* --------------------------------------------------------- ray vs scene */
typedef struct {
    double o[3], d[3], tmin, tmax;
    double sig_pos, sig_dir; /* uncertainty of a secondary ray (world units / radians) */
} or_ray;

#define OR_MAX_TIES 16

typedef struct {
    int hit;
    double t, u, v;
    uint32_t inst, prim;
    int amb;
    int nties;
    uint32_t tie_inst[OR_MAX_TIES], tie_prim[OR_MAX_TIES];
    double tie_t[OR_MAX_TIES], tie_u[OR_MAX_TIES], tie_v[OR_MAX_TIES];
    double beta;   /* band of the reported hit (barycentric units) */
    double delta;  /* float32 error band of the reported hit's t (t units) */
    double nobj[3]; /* object-space geometric normal of the hit triangle (e1 x e2) */
    int64_t tests;
} or_result;

/* slab test of a ray against a box in double: entry/exit t (no clipping) */
static int box_enter(const double lo[3], const double hi[3], const double o[3], const double d[3],
                     double *t0, double *t1) {
    double a = -INFINITY, b = INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (o[k] < lo[k] || o[k] > hi[k]) return 0;
            continue;
        }
        double x = (lo[k] - o[k]) / d[k], y = (hi[k] - o[k]) / d[k];
        if (x > y) { double z = x; x = y; y = z; }
        if (x > a) a = x;
        if (y < b) b = y;
    }
    *t0 = a; *t1 = b;
    return a <= b;
}

/* Classic Moller-Trumbore in double.  Returns 0 if the ray is parallel to
 * the plane (det == 0); else fills t, u (weight of b), v (weight of c). */
static inline int mt64(const double *T, const double o[3], const double d[3],
                       double *t, double *u, double *v, double *det_out) {
    const double *a = T, *e1 = T + 3, *e2 = T + 6;
    double P[3], Q[3], s[3];
    v_cross(P, d, e2);
    double det = v_dot(e1, P);
    *det_out = det;
    if (det == 0.0) return 0;
    v_sub(s, o, a);
    *u = v_dot(s, P) / det;
    v_cross(Q, s, e1);
    *v = v_dot(d, Q) / det;
    *t = v_dot(e2, Q) / det;
    return 1;
}

static inline double tri_min3(double a, double b, double c) {
    double m = a < b ? a : b;
    return m < c ? m : c;
}

static int sphere_skip(const or_blas *B, const double o[3], const double d[3], double tmin, double tmax) {
    double oc[3];
    v_sub(oc, B->sc, o);
    double dd = v_dot(d, d);
    double tc = v_dot(oc, d) / dd;
    double p[3] = {o[0] + tc * d[0] - B->sc[0], o[1] + tc * d[1] - B->sc[1], o[2] + tc * d[2] - B->sc[2]};
    double dist2 = v_dot(p, p);
    double rr = B->sr * 1.01; /* margin wider than any error band: the reject never changes a result */
    double r2 = rr * rr;
    if (dist2 > r2 * (1.0 + 1e-9) + 1e-18) return 1;
    double h = sqrt(fmax(r2 - dist2, 0.0) / dd);
    double slack = 1e-3 * (h + fabs(tc)) + 1e-9;
    if (tc + h < tmin - slack) return 1;
    if (tc - h > tmax * (1.0 + 1e-3) + slack) return 1;
    return 0;
}

static void tri_vertex(const double *T, int slot, double out[3]) {
    for (int k = 0; k < 3; ++k) out[k] = T[k] + (slot == 1 ? T[3 + k] : (slot == 2 ? T[6 + k] : 0.0));
}

/* One triangle against one object-space ray, with its float32 error bands. */
typedef struct {
    double t, u, v, w, m, beta, delta, cosg;
    int near; /* the ray passes within float32 error of the triangle's bounding sphere */
} tri_eval_t;

typedef struct {
    const double *o, *d, *o0;  /* object-space ray and the float32 origin point */
    double o0len, dl, dlen;    /* |o0|, |d| (object), |d| (world) */
    double inv_fro;
    const or_ray *R;
} ray_frame;

static int tri_eval(const double *T, const ray_frame *F, tri_eval_t *e) {
    double det;
    if (!mt64(T, F->o, F->d, &e->t, &e->u, &e->v, &det)) return 0;
    e->w = 1.0 - e->u - e->v;
    e->m = tri_min3(e->w, e->u, e->v);
    double n[3], e3[3], va[3], vb[3], vc[3];
    v_cross(n, T + 3, T + 6);
    double Sabs = fabs(v_dot(F->d, n));
    double nlen = v_len(n);
    v_sub(va, T, F->o0);
    for (int k = 0; k < 3; ++k) { vb[k] = va[k] + T[3 + k]; vc[k] = va[k] + T[6 + k]; }
    double Rj = v_len(va);
    if (v_len(vb) > Rj) Rj = v_len(vb);
    if (v_len(vc) > Rj) Rj = v_len(vc);
    Rj += F->o0len; /* float32 coordinates carry error relative to their magnitude */
    v_sub(e3, T + 6, T + 3);
    double P = v_len(T + 3) + v_len(T + 6) + v_len(e3);
    /* where along the ray the triangle lies: its bounding sphere's closest
     * approach (not the plane crossing, which runs off for grazing planes) */
    double cen[3], rc = 0.0, oc[3], cr[3];
    for (int k = 0; k < 3; ++k) cen[k] = T[k] + (T[3 + k] + T[6 + k]) / 3.0;
    for (int q = 0; q < 3; ++q) {
        double vq[3], dv[3];
        tri_vertex(T, q, vq);
        v_sub(dv, vq, cen);
        double l = v_len(dv);
        if (l > rc) rc = l;
    }
    v_sub(oc, cen, F->o);
    v_cross(cr, oc, F->d);
    double dist = v_len(cr) / F->dl;
    double tc = v_dot(oc, F->d) / (F->dl * F->dl);
    /* the drift of a secondary ray grows with t: take the plane crossing,
     * clamped to the triangle's extent along the ray */
    double ext = rc / F->dl;
    double talong = fabs(fmin(fmax(e->t, tc - ext), tc + ext));
    double sig = (F->R->sig_pos + F->R->sig_dir * talong * F->dlen) * F->inv_fro;
    double pos_err = OR_K * OR_EPS32 * Rj + sig;
    e->beta = pos_err * P * F->dl / Sabs;
    e->delta = pos_err * nlen / Sabs + OR_K * OR_EPS32 * fabs(e->t);
    e->cosg = Sabs / (nlen * F->dl);
    /* A triangle the ray passes farther from than the position error can
     * only be missed, however grazing (its bands grow as 1/cos). */
    double reach = rc + 2.0 * pos_err;
    double tr = reach / F->dl;
    e->near = dist <= reach && tc >= F->R->tmin - tr && tc <= F->R->tmax + tr;
    return 1;
}

/* A crossing of triangle j within the error band of exactly one of its edges
 * (and robustly inside the other two) is covered when the edge is shared with
 * one neighbour that lies on the other side of the edge as seen along the ray
 * (not a silhouette) and is itself robustly inside its other two edges: a
 * perturbed ray that leaves j enters the neighbour.  Returns the neighbour's
 * index (its evaluation in *ek) or -1. */
static int64_t covering(const or_blas *B, int64_t j, const tri_eval_t *ej, const ray_frame *F, tri_eval_t *ek) {
    if (!B->nbr) return -1;
    double c[3] = {ej->w, ej->u, ej->v};
    int near = -1, cnt = 0;
    for (int sl = 0; sl < 3; ++sl) {
        if (fabs(c[sl]) <= ej->beta) { near = sl; ++cnt; }
        else if (c[sl] < 0.0) return -1;
    }
    if (cnt != 1) return -1;
    int64_t k = B->nbr[3 * j + near];
    if (k < 0) return -1;
    int sk = B->nslot[3 * j + near];
    const double *Tj = B->tri + 9 * j, *Tk = B->tri + 9 * k;
    if (!tri_eval(Tk, F, ek)) return -1;
    double ck[3] = {ek->w, ek->u, ek->v};
    for (int sl = 0; sl < 3; ++sl)
        if (sl != sk && ck[sl] <= ek->beta) return -1;
    double pp[3], qq[3], rj[3], rk[3], eq[3], ej3[3], ek3[3], cj[3], ckx[3];
    tri_vertex(Tj, (near + 1) % 3, pp);
    tri_vertex(Tj, (near + 2) % 3, qq);
    tri_vertex(Tj, near, rj);
    tri_vertex(Tk, sk, rk);
    v_sub(eq, qq, pp);
    v_sub(ej3, rj, pp);
    v_sub(ek3, rk, pp);
    v_cross(cj, eq, ej3);
    v_cross(ckx, eq, ek3);
    if (!(v_dot(cj, F->d) * v_dot(ckx, F->d) < 0.0)) return -1;
    return k;
}

/* The ray in instance I's object space (o' = M^-1 o, d' = M^-1 d: t is
 * unchanged) and the origin a float32 traversal uses there: moved along the
 * ray to where it enters the mesh's box, never before tmin nor past tmax. */
static void inst_frame(const or_inst *I, const or_blas *B, const or_ray *R, double o[3], double d[3],
                       double o0[3]) {
    xf_point(I->inv, R->o, o);
    xf_vec(I->inv, R->d, d);
    double te0, te1, ts = R->tmin;
    if (box_enter(B->lo, B->hi, o, d, &te0, &te1) && te0 > ts) ts = te0;
    if (ts > R->tmax) ts = R->tmax;
    for (int k = 0; k < 3; ++k) o0[k] = o[k] + ts * d[k];
}

static void add_tie(or_result *res, uint32_t i, uint32_t j, const tri_eval_t *e) {
    for (int q = 0; q < res->nties; ++q)
        if (res->tie_inst[q] == i && res->tie_prim[q] == j) return;
    if (res->nties >= OR_MAX_TIES) {
        res->amb = 1; /* tie set overflow: membership cannot be checked */
        return;
    }
    int q = res->nties++;
    res->tie_inst[q] = i; res->tie_prim[q] = j;
    res->tie_t[q] = e->t; res->tie_u[q] = e->u; res->tie_v[q] = e->v;
}

/* Per-ray evaluation.  any = 0: closest hit with ties and ambiguity;
 * any = 1: occlusion (hit = some genuine hit exists) with ambiguity.
 * cover = 1 lets a covered edge crossing (see covering()) count as
 * unambiguous; any-hit always allows it, closest hit only where either of
 * the two triangles is an acceptable answer (not when flat shading depends
 * on which one is hit). */
static void or_trace_one(const or_scene *S, const or_ray *R, int any, int cover, uint32_t mask, uint32_t cull,
                         or_result *res) {
    memset(res, 0, sizeof(*res));
    res->t = INFINITY;
    res->inst = res->prim = OR_MISS;
    double dlen = v_len(R->d);
    int64_t tests = 0;
    /* pass 1: the exact answer */
    for (int64_t i = 0; i < S->ni; ++i) {
        const or_inst *I = &S->inst[i];
        const or_blas *B = &S->blas[I->blas];
        if (((I->flags & 0xFFu) & mask) == 0u) continue;
        double o[3], d[3];
        xf_point(I->inv, R->o, o);
        xf_vec(I->inv, R->d, d);
        if (S->sphere_reject && sphere_skip(B, o, d, R->tmin, R->tmax)) continue;
        for (int64_t j = 0; j < B->n; ++j) {
            double t, u, v, det;
            ++tests;
            if (!mt64(B->tri + 9 * j, o, d, &t, &u, &v, &det)) continue;
            if (u < 0.0 || v < 0.0 || 1.0 - u - v < 0.0) continue;
            if (t < R->tmin || t > R->tmax) continue;
            if (culled(I, cull, B->tri + 9 * j, d)) continue;
            if (!alpha_open(B, j, u, v)) continue;
            if (t < res->t) {
                res->hit = 1; res->t = t; res->u = u; res->v = v;
                res->inst = (uint32_t)i; res->prim = (uint32_t)j;
                const double *T = B->tri + 9 * j;
                v_cross(res->nobj, T + 3, T + 6);
            }
        }
    }
    /* pass 2: tie set and ambiguity flag */
    double tlim = res->hit ? res->t : R->tmax;
    int fin_tmax = isfinite(R->tmax);
    int robust_hit = 0, near_band = 0;
    /* the hit's own t band: a second surface nearer to t* than the two bands
     * together cannot be ordered by a float32 traversal */
    double hit_delta = 0.0;
    if (res->hit && !any) {
        const or_inst *I = &S->inst[res->inst];
        double o[3], d[3], o0[3];
        inst_frame(I, &S->blas[I->blas], R, o, d, o0);
        ray_frame F = {o, d, o0, v_len(o0), v_len(d), dlen, I->inv_fro, R};
        tri_eval_t e;
        if (tri_eval(S->blas[I->blas].tri + 9 * (int64_t)res->prim, &F, &e)) hit_delta = e.delta;
    }
    for (int64_t i = 0; i < S->ni; ++i) {
        const or_inst *I = &S->inst[i];
        const or_blas *B = &S->blas[I->blas];
        if (((I->flags & 0xFFu) & mask) == 0u) continue;
        double o[3], d[3], o0[3];
        inst_frame(I, B, R, o, d, o0);
        if (S->sphere_reject && sphere_skip(B, o, d, R->tmin, R->tmax)) continue;
        ray_frame F = {o, d, o0, v_len(o0), v_len(d), dlen, I->inv_fro, R};
        for (int64_t j = 0; j < B->n; ++j) {
            tri_eval_t e, ek;
            ++tests;
            if (!tri_eval(B->tri + 9 * j, &F, &e)) continue;
            if (!e.near) continue; /* robustly missed: no band can reach it */
            double t = e.t, m = e.m, beta = e.beta, delta = e.delta;
            if (culled(I, cull, B->tri + 9 * j, d)) {
                /* a float32 test may decide the facing of a nearly grazing
                 * triangle the other way: ambiguous if it could be the hit */
                if (e.cosg < 1e-3 && m >= -beta && t >= R->tmin - delta &&
                    (any || t <= tlim * (1.0 + 1e-5) + delta)) {
                    if (any) near_band = 1;
                    else res->amb = 1;
                }
                continue;
            }
            const int open = alpha_state(B, j, e.u, e.v, beta);
            if (open <= 0) {
                /* ignored by its opacity mask; ambiguous if float32
                 * barycentrics may land on an opaque micro-triangle and the
                 * triangle could be the hit */
                if (open < 0 && m >= -beta && t >= R->tmin - delta && (any || t <= tlim * (1.0 + 1e-5) + delta)) {
                    if (any) near_band = 1;
                    else res->amb = 1;
                }
                continue;
            }
            double tmax_band = fin_tmax ? fmax(1e-5 * R->tmax, delta) : 0.0;
            if (!any) {
                int in_range = (t >= R->tmin - delta) && (t <= tlim * (1.0 + 1e-5) + delta);
                if (in_range && fabs(m) <= beta) {
                    int64_t k = cover ? covering(B, j, &e, &F, &ek) : -1;
                    /* both triangles of a covered crossing are correct answers
                     * only if each one's t is within 1e-5 t* */
                    double ttol = res->hit ? 1e-5 * res->t : 0.0;
                    if (k >= 0 && res->hit && fabs(t - res->t) <= ttol && fabs(ek.t - res->t) <= ttol &&
                        t >= R->tmin + delta && ek.t >= R->tmin + ek.delta &&
                        (!fin_tmax || (t <= R->tmax - tmax_band && ek.t <= R->tmax - tmax_band))) {
                        add_tie(res, (uint32_t)i, (uint32_t)j, &e);
                        add_tie(res, (uint32_t)i, (uint32_t)k, &ek);
                    } else {
                        res->amb = 1;
                    }
                }
                if (m >= -beta && fabs(t - R->tmin) <= delta && t <= tlim * (1.0 + 1e-5) + delta) res->amb = 1;
                if (m >= -beta && fin_tmax && fabs(t - R->tmax) <= tmax_band &&
                    (!res->hit || t <= tlim * (1.0 + 1e-5) + delta))
                    res->amb = 1;
                if (res->hit && m >= -beta && t >= R->tmin && t <= R->tmax && fabs(t - res->t) <= 1e-6 * res->t)
                    add_tie(res, (uint32_t)i, (uint32_t)j, &e);
                else if (res->hit && m > beta && t >= R->tmin - delta && fabs(t - res->t) <= delta + hit_delta &&
                         !((uint32_t)i == res->inst && (uint32_t)j == res->prim))
                    res->amb = 1; /* a second surface within float32 reach of t*, not a tie */
                if (res->hit && (uint32_t)i == res->inst && (uint32_t)j == res->prim) {
                    res->beta = beta;
                    res->delta = delta;
                    if (e.cosg < 1e-3) res->amb = 1;
                    if (fin_tmax && fabs(res->t - R->tmax) <= tmax_band) res->amb = 1;
                }
            } else {
                int robust_t = t >= R->tmin + delta && (!fin_tmax || t <= R->tmax - tmax_band);
                if (m >= beta && robust_t) robust_hit = 1;
                int in_range = (t >= R->tmin - delta) && (!fin_tmax || t <= R->tmax + tmax_band);
                if (in_range && fabs(m) <= beta) {
                    int64_t k = covering(B, j, &e, &F, &ek);
                    int robust_k = k >= 0 && ek.t >= R->tmin + ek.delta &&
                                   (!fin_tmax || ek.t <= R->tmax - fmax(1e-5 * R->tmax, ek.delta));
                    if (k >= 0 && robust_t && robust_k) robust_hit = 1;
                    else near_band = 1;
                }
                if (m >= -beta && fabs(t - R->tmin) <= delta) near_band = 1;
                if (m >= -beta && fin_tmax && fabs(t - R->tmax) <= tmax_band) near_band = 1;
            }
        }
    }
    if (any) res->amb = (!robust_hit) && near_band;
    res->tests = tests;
}

/* -------------------------------------------------------- thread helper */
typedef struct {
    void (*fn)(void *ctx, int64_t i);
    void *ctx;
    int64_t n;
    int64_t next;
} or_pool;

static void *pool_worker(void *arg) {
    or_pool *p = (or_pool *)arg;
    for (;;) {
        int64_t i0 = __atomic_fetch_add(&p->next, 16, __ATOMIC_RELAXED);
        if (i0 >= p->n) break;
        int64_t i1 = i0 + 16 < p->n ? i0 + 16 : p->n;
        for (int64_t i = i0; i < i1; ++i) p->fn(p->ctx, i);
    }
    return NULL;
}

static void pool_run(void (*fn)(void *, int64_t), void *ctx, int64_t n, int32_t nthreads) {
    or_pool p = {fn, ctx, n, 0};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int k = 1; k < nthreads; ++k)
        if (pthread_create(&th[started], NULL, pool_worker, &p) == 0) ++started;
    pool_worker(&p);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
}

/* --------------------------------------------------------------- tracing */
typedef struct {
    const or_scene *S;
    const float *rays;
    int any;
    double *t, *u, *v, *beta, *delta;
    uint32_t *inst, *prim;
    uint8_t *hit, *amb;
    int32_t *nties;
    uint32_t *ties; /* [N][max_ties][2] */
    double *ties_tuv; /* [N][max_ties][3] */
    int32_t max_ties;
    int64_t tests;
    const uint8_t *ray_mask; /* per ray, or NULL: `mask` for all */
    uint32_t mask, cull;
} trace_ctx;

static void trace_task(void *vctx, int64_t r) {
    trace_ctx *c = (trace_ctx *)vctx;
    const float *q = c->rays + 8 * r;
    or_ray R;
    for (int k = 0; k < 3; ++k) { R.o[k] = q[k]; R.d[k] = q[3 + k]; }
    R.tmin = q[6]; R.tmax = q[7];
    R.sig_pos = R.sig_dir = 0.0;
    or_result res;
    or_trace_one(c->S, &R, c->any, 1, c->ray_mask ? c->ray_mask[r] : c->mask, c->cull, &res);
    c->t[r] = res.t; c->u[r] = res.u; c->v[r] = res.v; c->beta[r] = res.beta; c->delta[r] = res.delta;
    c->inst[r] = res.inst; c->prim[r] = res.prim;
    c->hit[r] = (uint8_t)res.hit; c->amb[r] = (uint8_t)res.amb;
    int nt = res.nties < c->max_ties ? res.nties : c->max_ties;
    if (res.nties > c->max_ties) c->amb[r] = 1;
    c->nties[r] = nt;
    for (int k = 0; k < nt; ++k) {
        c->ties[((size_t)r * c->max_ties + k) * 2] = res.tie_inst[k];
        c->ties[((size_t)r * c->max_ties + k) * 2 + 1] = res.tie_prim[k];
        c->ties_tuv[((size_t)r * c->max_ties + k) * 3] = res.tie_t[k];
        c->ties_tuv[((size_t)r * c->max_ties + k) * 3 + 1] = res.tie_u[k];
        c->ties_tuv[((size_t)r * c->max_ties + k) * 3 + 2] = res.tie_v[k];
    }
    __atomic_fetch_add(&c->tests, res.tests, __ATOMIC_RELAXED);
}

/* rays: f32[N][8] = ox oy oz dx dy dz tmin tmax.  Returns the number of
 * ray-triangle tests performed. */
int64_t or_trace(or_scene *S, const float *rays, int64_t n, int32_t any, int32_t nthreads,
                 double *t, double *u, double *v, double *beta, double *delta, uint32_t *inst,
                 uint32_t *prim, uint8_t *hit, uint8_t *amb, int32_t *nties, uint32_t *ties,
                 double *ties_tuv, int32_t max_ties, const uint8_t *ray_mask, uint32_t mask, uint32_t cull) {
    ensure_adjacency(S);
    trace_ctx c = {S, rays, any, t, u, v, beta, delta, inst, prim, hit, amb, nties, ties, ties_tuv,
                   max_ties, 0, ray_mask, mask, cull};
    pool_run(trace_task, &c, n, nthreads);
    S->tests += c.tests;
    return c.tests;
}

/* One given triangle per ray: for ray r, triangle prim[r] of instance
 * inst[r] evaluated in FP64 (Moller-Trumbore in the instance's object
 * space), with its float32 error bands.  out[r][6] = t, u, v, m (the least
 * barycentric weight: >= 0 inside the closed triangle), beta, delta; all NaN
 * for inst[r] == OR_MISS, an out-of-range index or a ray parallel to the
 * triangle's plane.  Used to check a reported hit that need not be the
 * closest (any hit: any genuine hit of the ray is a correct answer). */
void or_eval_hits(const or_scene *S, const float *rays, int64_t n, const uint32_t *inst, const uint32_t *prim,
                  double *out) {
    for (int64_t r = 0; r < n; ++r) {
        double *q = out + 6 * r;
        for (int k = 0; k < 6; ++k) q[k] = NAN;
        if (inst[r] == OR_MISS || (int64_t)inst[r] >= S->ni) continue;
        const or_inst *I = &S->inst[inst[r]];
        const or_blas *B = &S->blas[I->blas];
        if ((int64_t)prim[r] >= B->n) continue;
        or_ray R;
        for (int k = 0; k < 3; ++k) { R.o[k] = rays[8 * r + k]; R.d[k] = rays[8 * r + 3 + k]; }
        R.tmin = rays[8 * r + 6]; R.tmax = rays[8 * r + 7];
        R.sig_pos = R.sig_dir = 0.0;
        double o[3], d[3], o0[3];
        inst_frame(I, B, &R, o, d, o0);
        ray_frame F = {o, d, o0, v_len(o0), v_len(d), v_len(R.d), I->inv_fro, &R};
        tri_eval_t e;
        if (!tri_eval(B->tri + 9 * (int64_t)prim[r], &F, &e)) continue;
        q[0] = e.t; q[1] = e.u; q[2] = e.v; q[3] = e.m; q[4] = e.beta; q[5] = e.delta;
    }
}

/* ------------------------------------------------------- camera and AO */
/* Pinhole camera: forward f, right r = f x up, true up u = r x f; pixel
 * centres; vertical field of view; y = 0 is the top row. */
static void camera_ray(const float *cam /*eye3 target3 up3 vfov*/, int32_t W, int32_t H,
                       int64_t pixel, double o[3], double d[3]) {
    double eye[3] = {cam[0], cam[1], cam[2]}, tg[3] = {cam[3], cam[4], cam[5]};
    double up[3] = {cam[6], cam[7], cam[8]};
    double f[3], r[3], u[3];
    v_sub(f, tg, eye);
    v_norm(f);
    v_cross(r, f, up);
    v_norm(r);
    v_cross(u, r, f);
    double th = tan(0.5 * (double)cam[9] * M_PI / 180.0);
    int64_t x = pixel % W, y = pixel / W;
    double sx = (2.0 * ((double)x + 0.5) / W - 1.0) * th * (double)W / (double)H;
    double sy = (1.0 - 2.0 * ((double)y + 0.5) / H) * th;
    for (int k = 0; k < 3; ++k) d[k] = f[k] + sx * r[k] + sy * u[k];
    v_norm(d);
    for (int k = 0; k < 3; ++k) o[k] = eye[k];
}

void or_camera_rays(const float *cam, int32_t W, int32_t H, const int64_t *pixels, int64_t n,
                    double *out /*[n][6]*/) {
    for (int64_t i = 0; i < n; ++i) camera_ray(cam, W, H, pixels[i], out + 6 * i, out + 6 * i + 3);
}

/* SplitMix64 (Steele, Lea & Flood 2014): state advances by the golden
 * gamma, output is the published 64-bit finaliser. */
static inline uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
#define OR_GOLDEN 0x9E3779B97F4A7C15ull

/* two uniforms in [0,1) with 24 bits each, exact in float32 and float64:
 * the generator's state starts at seed + 2*key*gamma and is advanced twice. */
void or_ao_uniforms(uint64_t seed, uint64_t key, double *u1, double *u2) {
    uint64_t s = seed + 2ull * key * OR_GOLDEN;
    uint64_t x1 = splitmix_out(s + OR_GOLDEN);
    uint64_t x2 = splitmix_out(s + 2ull * OR_GOLDEN);
    *u1 = (double)(x1 >> 40) * (1.0 / 16777216.0);
    *u2 = (double)(x2 >> 40) * (1.0 / 16777216.0);
}

/* Cosine-weighted hemisphere direction around unit n (Malley's method) in
 * the orthonormal basis of Duff et al. 2017. */
static void ao_direction(const double n[3], double u1, double u2, double out[3]) {
    double sgn = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sgn + n[2]);
    double b = n[0] * n[1] * a;
    double b1[3] = {1.0 + sgn * n[0] * n[0] * a, sgn * b, -sgn * n[0]};
    double b2[3] = {b, sgn + n[1] * n[1] * a, -n[1]};
    double r = sqrt(u1), ph = 2.0 * M_PI * u2;
    double x = r * cos(ph), y = r * sin(ph), z = sqrt(1.0 - u1);
    for (int k = 0; k < 3; ++k) out[k] = x * b1[k] + y * b2[k] + z * n[k];
}

void or_ao_direction(const double *n, double u1, double u2, double *out) { ao_direction(n, u1, u2, out); }

/* ---------------------------------------------------------------- shading */
typedef struct {
    const or_scene *S;
    const float *cam;
    const float *light; /* pos3 intensity3 ambient */
    int32_t W, H, D, mode;
    uint64_t seed;
    const int64_t *pixels;
    double *rgb;
    uint8_t *amb;
    int64_t *nrays;
    int64_t tests;
} render_ctx;

static void sky(const double d[3], double out[3]) {
    double l = v_len(d);
    double a = 0.5 * (d[1] / l + 1.0);
    out[0] = (1.0 - a) + a * 0.5;
    out[1] = (1.0 - a) + a * 0.7;
    out[2] = (1.0 - a) + a * 1.0;
}

/* Hit geometry shared by the shading steps: world point, world geometric
 * normal (outward by winding), faced normal, and the triangle-normal error
 * scale used by the uncertainty model. */
typedef struct {
    double p[3], ng[3], nf[3], dn[3];
    double sig_n;
    uint32_t mat;
} hit_geom;

static void hit_geometry(const or_scene *S, const or_ray *R, const or_result *h, hit_geom *g) {
    const or_inst *I = &S->inst[h->inst];
    const or_blas *B = &S->blas[I->blas];
    for (int k = 0; k < 3; ++k) g->p[k] = R->o[k] + h->t * R->d[k];
    /* normals transform with the inverse transpose; an orientation-reversing
     * instance keeps the object's outward side outward, so no winding flip */
    double n[3];
    xf_vec_t(I->inv, h->nobj, n);
    v_norm(n);
    for (int k = 0; k < 3; ++k) { g->ng[k] = n[k]; g->dn[k] = R->d[k]; }
    v_norm(g->dn);
    double s = v_dot(g->ng, g->dn) < 0.0 ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) g->nf[k] = s * g->ng[k];
    const double *T = B->tri + 9 * h->prim;
    double e3[3];
    v_sub(e3, T + 6, T + 3);
    double P = v_len(T + 3) + v_len(T + 6) + v_len(e3);
    g->sig_n = OR_K * OR_EPS32 * P * P / v_len(h->nobj);
    g->mat = I->mat != 0xFFFFFFFFu ? I->mat : (B->prim_mat ? B->prim_mat[h->prim] : 0u);
}

static double offset_eps(const double p[3]) {
    double m = maxabs3(p);
    return 1e-4 * (m > 1.0 ? m : 1.0);
}

static void child_sigma(const or_ray *R, const or_result *h, const hit_geom *g, double amp_d,
                        double amp_n, or_ray *c) {
    double dl = v_len(R->d);
    c->sig_pos = R->sig_pos + R->sig_dir * h->t * dl + OR_K * OR_EPS32 * (maxabs3(g->p) + h->t * dl);
    c->sig_dir = amp_d * R->sig_dir + amp_n * g->sig_n + OR_K * OR_EPS32;
}

/* radiance of a ray at depth k (primary = 0); accumulates rays and tests */
static void radiance(render_ctx *C, const or_ray *R, int k, double out[3], int *amb, int64_t *nrays,
                     int64_t *tests) {
    const or_scene *S = C->S;
    or_result h;
    or_trace_one(S, R, 0, 0, 0xFFu, 0u, &h);
    ++*nrays;
    *tests += h.tests;
    if (h.amb) *amb = 1;
    out[0] = out[1] = out[2] = 0.0;
    if (!h.hit) {
        sky(R->d, out);
        return;
    }
    hit_geom g;
    hit_geometry(S, R, &h, &g);
    const or_mat *M = &S->mats[g.mat];
    double eps = offset_eps(g.p);
    if (M->type == 0) {
        const float *L = C->light;
        double lp[3] = {L[0], L[1], L[2]}, l[3];
        v_sub(l, lp, g.p);
        v_norm(l);
        double cosl = v_dot(g.nf, l);
        double vis = 0.0;
        if (cosl > 0.0) {
            or_ray sr;
            for (int q = 0; q < 3; ++q) {
                sr.o[q] = g.p[q] + eps * g.nf[q];
                sr.d[q] = lp[q] - sr.o[q];
            }
            sr.tmin = 0.0;
            sr.tmax = 1.0 - 1e-4;
            child_sigma(R, &h, &g, 1.0, 1.0, &sr);
            or_result sh;
            or_trace_one(S, &sr, 1, 1, 0xFFu, 0u, &sh);
            ++*nrays;
            *tests += sh.tests;
            if (sh.amb) *amb = 1;
            vis = sh.hit ? 0.0 : 1.0;
        } else {
            cosl = 0.0;
        }
        for (int q = 0; q < 3; ++q) out[q] = M->rgb[q] * ((double)L[6] + (double)L[3 + q] * cosl * vis);
        return;
    }
    if (k >= C->D) return; /* a specular hit at the depth cap contributes nothing */
    double dn[3] = {g.dn[0], g.dn[1], g.dn[2]};
    double dnf = v_dot(dn, g.nf);
    or_ray rr;
    for (int q = 0; q < 3; ++q) {
        rr.o[q] = g.p[q] + eps * g.nf[q];
        rr.d[q] = dn[q] - 2.0 * dnf * g.nf[q];
    }
    rr.tmin = 0.0;
    rr.tmax = INFINITY;
    child_sigma(R, &h, &g, 1.0, 2.0, &rr);
    if (M->type == 1) {
        double c[3];
        radiance(C, &rr, k + 1, c, amb, nrays, tests);
        for (int q = 0; q < 3; ++q) out[q] = M->rgb[q] * c[q];
        return;
    }
    /* glass */
    int entering = v_dot(dn, g.ng) < 0.0;
    double ior = M->ior;
    double eta = entering ? 1.0 / ior : ior;
    double cosi = -dnf;
    double kappa = 1.0 - eta * eta * (1.0 - cosi * cosi);
    double F = 1.0, c[3], cr[3] = {0, 0, 0};
    or_ray tr;
    int refract = kappa >= 0.0;
    if (refract) {
        double sk = sqrt(kappa);
        double r0 = (ior - 1.0) / (ior + 1.0);
        r0 *= r0;
        double cc = entering ? cosi : sk;
        double om = 1.0 - cc;
        F = r0 + (1.0 - r0) * om * om * om * om * om;
        for (int q = 0; q < 3; ++q) {
            tr.o[q] = g.p[q] - eps * g.nf[q];
            tr.d[q] = eta * dn[q] + (eta * cosi - sk) * g.nf[q];
        }
        tr.tmin = 0.0;
        tr.tmax = INFINITY;
        double ct = sk > 1e-3 ? sk : 1e-3;
        child_sigma(R, &h, &g, eta * (1.0 + cosi / ct), 1.0 + eta * cosi / ct + 1.0, &tr);
    }
    radiance(C, &rr, k + 1, c, amb, nrays, tests);
    if (refract) radiance(C, &tr, k + 1, cr, amb, nrays, tests);
    for (int q = 0; q < 3; ++q) out[q] = F * c[q] + (1.0 - F) * cr[q];
}

static void ao_pixel(render_ctx *C, const or_ray *R, int64_t pixel, double out[3], int *amb,
                     int64_t *nrays, int64_t *tests) {
    const or_scene *S = C->S;
    or_result h;
    or_trace_one(S, R, 0, 0, 0xFFu, 0u, &h);
    ++*nrays;
    *tests += h.tests;
    if (h.amb) *amb = 1;
    if (!h.hit) {
        out[0] = out[1] = out[2] = 1.0;
        return;
    }
    hit_geom g;
    hit_geometry(S, R, &h, &g);
    double eps = offset_eps(g.p);
    int occl = 0;
    for (int k = 0; k < 8; ++k) {
        double u1, u2, dir[3];
        or_ao_uniforms(C->seed, (uint64_t)pixel * 8ull + (uint64_t)k, &u1, &u2);
        ao_direction(g.nf, u1, u2, dir);
        or_ray ar;
        for (int q = 0; q < 3; ++q) { ar.o[q] = g.p[q] + eps * g.nf[q]; ar.d[q] = dir[q]; }
        ar.tmin = 0.0;
        ar.tmax = 5.0;
        child_sigma(R, &h, &g, 0.0, 1.0, &ar);
        ar.sig_dir += 8.0 * OR_K * OR_EPS32; /* float32 sin/cos/sqrt of the sample */
        or_result sh;
        or_trace_one(S, &ar, 1, 1, 0xFFu, 0u, &sh);
        ++*nrays;
        *tests += sh.tests;
        if (sh.amb) *amb = 1;
        occl += sh.hit ? 1 : 0;
    }
    double val = 1.0 - (double)occl / 8.0;
    out[0] = out[1] = out[2] = val;
}

static void render_task(void *vctx, int64_t i) {
    render_ctx *C = (render_ctx *)vctx;
    int64_t pixel = C->pixels[i];
    or_ray R;
    camera_ray(C->cam, C->W, C->H, pixel, R.o, R.d);
    R.tmin = 0.0;
    R.tmax = INFINITY;
    R.sig_pos = 0.0;
    R.sig_dir = OR_K * OR_EPS32;
    int amb = 0;
    int64_t nrays = 0, tests = 0;
    double out[3];
    if (C->mode == 1)
        ao_pixel(C, &R, pixel, out, &amb, &nrays, &tests);
    else
        radiance(C, &R, 0, out, &amb, &nrays, &tests);
    for (int q = 0; q < 3; ++q) C->rgb[3 * i + q] = out[q];
    C->amb[i] = (uint8_t)amb;
    C->nrays[i] = nrays;
    __atomic_fetch_add(&C->tests, tests, __ATOMIC_RELAXED);
}

/* Renders the listed pixels.  cam: eye3 target3 up3 vfov_deg; light: pos3
 * intensity3 ambient; materials must be set.  Returns the triangle tests. */
int64_t or_render(or_scene *S, const float *cam, const float *light, int32_t W, int32_t H,
                  int32_t max_depth, int32_t mode, uint64_t seed, const int64_t *pixels, int64_t n,
                  int32_t nthreads, double *rgb, uint8_t *amb, int64_t *nrays) {
    ensure_adjacency(S);
    render_ctx C = {S, cam, light, W, H, max_depth, mode, seed, pixels, rgb, amb, nrays, 0};
    pool_run(render_task, &C, n, nthreads);
    S->tests += C.tests;
    return C.tests;
}

/* The material index each listed pixel's primary ray meets (0xFFFFFFFF for
 * the sky) and whether that primary hit is ambiguous: the first shading
 * decision of the render above, on its own. */
typedef struct {
    const or_scene *S;
    const float *cam;
    int32_t W, H;
    const int64_t *pixels;
    uint32_t *mat;
    uint8_t *amb;
} primary_ctx;

static void primary_task(void *vctx, int64_t i) {
    primary_ctx *c = (primary_ctx *)vctx;
    or_ray R;
    camera_ray(c->cam, c->W, c->H, c->pixels[i], R.o, R.d);
    R.tmin = 0.0;
    R.tmax = INFINITY;
    R.sig_pos = 0.0;
    R.sig_dir = OR_K * OR_EPS32;
    or_result h;
    or_trace_one(c->S, &R, 0, 0, 0xFFu, 0u, &h);
    c->amb[i] = (uint8_t)h.amb;
    if (!h.hit) {
        c->mat[i] = 0xFFFFFFFFu;
        return;
    }
    hit_geom g;
    hit_geometry(c->S, &R, &h, &g);
    c->mat[i] = g.mat;
}

void or_primary_materials(or_scene *S, const float *cam, int32_t W, int32_t H, const int64_t *pixels, int64_t n,
                          int32_t nthreads, uint32_t *mat, uint8_t *amb) {
    ensure_adjacency(S);
    primary_ctx C = {S, cam, W, H, pixels, mat, amb};
    pool_run(primary_task, &C, n, nthreads);
}

/* Ambient-occlusion rays of input rays: for each ray with a closest hit, the
 * 8 rays (origin, direction) the incoherent workload spawns there; out is
 * [n][8][6] (undefined for misses), hit/amb per input ray. */
typedef struct {
    const or_scene *S;
    const float *rays;
    uint64_t seed;
    double *out;
    uint8_t *hit, *amb;
} aorays_ctx;

static void aorays_task(void *vctx, int64_t r) {
    aorays_ctx *c = (aorays_ctx *)vctx;
    const float *q = c->rays + 8 * r;
    or_ray R;
    for (int k = 0; k < 3; ++k) { R.o[k] = q[k]; R.d[k] = q[3 + k]; }
    R.tmin = q[6]; R.tmax = q[7];
    R.sig_pos = R.sig_dir = 0.0;
    or_result h;
    or_trace_one(c->S, &R, 0, 0, 0xFFu, 0u, &h);
    c->hit[r] = (uint8_t)h.hit;
    c->amb[r] = (uint8_t)h.amb;
    if (!h.hit) return;
    hit_geom g;
    hit_geometry(c->S, &R, &h, &g);
    double eps = offset_eps(g.p);
    for (int k = 0; k < 8; ++k) {
        double u1, u2, dir[3];
        or_ao_uniforms(c->seed, (uint64_t)r * 8ull + (uint64_t)k, &u1, &u2);
        ao_direction(g.nf, u1, u2, dir);
        double *o = c->out + ((size_t)r * 8 + k) * 6;
        for (int m = 0; m < 3; ++m) { o[m] = g.p[m] + eps * g.nf[m]; o[3 + m] = dir[m]; }
    }
}

void or_ao_rays(or_scene *S, const float *rays, int64_t n, uint64_t seed, int32_t nthreads, double *out,
                uint8_t *hit, uint8_t *amb) {
    ensure_adjacency(S);
    aorays_ctx c = {S, rays, seed, out, hit, amb};
    pool_run(aorays_task, &c, n, nthreads);
}

/*
 * O-splat: footprint-restricted FP64 reference renderer, plain C + OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the HIP
 * renderer.
 *
 * It computes exactly what the brute-force definition computes (paper,
 * Methods, "Molecular Graphics Engine": each primitive is displayed by
 * ray-casting its implicit surface; "High Quality Rendering": deferred
 * shading with screen-space ambient occlusion), with one shortcut: each
 * primitive is evaluated only on the pixels of a conservative screen
 * rectangle (the projected corners of its axis-aligned bounding box, widened
 * by one pixel), which cannot change the result because a ray that misses
 * that box misses the primitive.  The readings R1-R6 are the ones stated in
 * the NumPy brute-force module of the same directory; the two are written
 * independently and are checked equal by the tests.
 *
 * Threads own disjoint bands of pixel rows, so no pixel is shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OS_TAU 1.0e-5
#define OS_MAX_ACCEPT 8
#define OS_BG_ID 0xFFFFFFFFu
#define OS_KA 0.2
#define OS_KD 0.8
#define OS_KS 0.25
#define OS_SHININESS 32.0
#define OS_PI 3.14159265358979323846

typedef struct {
    double e[3], s[3], u[3], f[3];
    double tanh_, aspect, hh, znear, zfar;
    int proj, W, H;
    double clip[4];   /* world plane a, b, c, d: a x + b y + c z + d >= 0 is kept */
    int clip_on;
} os_cam;

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void norm3(double* a) {
    double n = sqrt(dot3(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}

static void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* cam = eye3, target3, up3, fovy, ortho_half_height, projection, znear, zfar,
 * clip plane a, b, c, d (all zero: no clipping) */
static void os_make_cam(const double* cam, int W, int H, os_cam* c) {
    for (int k = 0; k < 3; ++k) { c->e[k] = cam[k]; c->f[k] = cam[3 + k] - cam[k]; }
    norm3(c->f);
    cross3(c->f, cam + 6, c->s);
    norm3(c->s);
    cross3(c->s, c->f, c->u);
    c->tanh_ = tan(cam[9] / 2.0);
    c->hh = cam[10];
    c->proj = (int)cam[11];
    c->znear = cam[12];
    c->zfar = cam[13];
    c->W = W; c->H = H;
    c->aspect = (double)W / (double)H;
    c->clip_on = 0;
    for (int k = 0; k < 4; ++k) {
        c->clip[k] = cam[14 + k];
        if (cam[14 + k] != 0.0) c->clip_on = 1;
    }
}

static void os_ray(const os_cam* c, int i, int j, double* o, double* d) {
    double nx = 2.0 * (i + 0.5) / c->W - 1.0;
    double ny = 1.0 - 2.0 * (j + 0.5) / c->H;
    if (c->proj == 0) {
        double ax = nx * c->tanh_ * c->aspect, ay = ny * c->tanh_;
        for (int k = 0; k < 3; ++k) { o[k] = c->e[k]; d[k] = c->f[k] + ax * c->s[k] + ay * c->u[k]; }
        norm3(d);
    } else {
        double ax = nx * c->hh * c->aspect, ay = ny * c->hh;
        for (int k = 0; k < 3; ++k) { o[k] = c->e[k] + ax * c->s[k] + ay * c->u[k]; d[k] = c->f[k]; }
    }
}

/* Pixel-space position of a world point; returns 0 if it is not in front of the eye plane. */
static int os_project(const os_cam* c, const double* p, double* px, double* py, double* zv) {
    double r[3] = {p[0] - c->e[0], p[1] - c->e[1], p[2] - c->e[2]};
    double x = dot3(r, c->s), y = dot3(r, c->u), z = dot3(r, c->f);
    *zv = z;
    if (c->proj == 0) {
        if (z <= 1e-9) return 0;
        *px = (x / (z * c->tanh_ * c->aspect) + 1.0) * 0.5 * c->W;
        *py = (1.0 - y / (z * c->tanh_)) * 0.5 * c->H;
    } else {
        *px = (x / (c->hh * c->aspect) + 1.0) * 0.5 * c->W;
        *py = (1.0 - y / c->hh) * 0.5 * c->H;
    }
    return 1;
}

/* Conservative pixel rectangle of an axis-aligned box; returns 0 if culled.
   Only points with view depth >= zc = znear (1 - 2 tau) can hold a hit (or a
   grazing candidate), so a perspective box that reaches behind that plane is
   bounded by the projections of its corners in front of it and of the points
   where its edges cross it: the vertices of the box cut by the plane. */
static int os_box_rect(const os_cam* c, const double* lo, const double* hi, int* rx0, int* ry0, int* rx1, int* ry1) {
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    double zmin = INFINITY, zmax = -INFINITY;
    const double zc = c->znear * (1.0 - 2 * OS_TAU);
    double cp[8][3], cz[8];
    for (int corner = 0; corner < 8; ++corner) {
        double* p = cp[corner];
        p[0] = (corner & 1) ? hi[0] : lo[0];
        p[1] = (corner & 2) ? hi[1] : lo[1];
        p[2] = (corner & 4) ? hi[2] : lo[2];
        double r[3] = {p[0] - c->e[0], p[1] - c->e[1], p[2] - c->e[2]};
        cz[corner] = dot3(r, c->f);
        if (cz[corner] < zmin) zmin = cz[corner];
        if (cz[corner] > zmax) zmax = cz[corner];
    }
    if (zmax < zc) return 0;
    if (zmin > c->zfar * (1.0 + 2 * OS_TAU)) return 0;
#define OS_ADD(P)                                                  \
    do {                                                           \
        double px_, py_, zv_;                                      \
        if (os_project(c, (P), &px_, &py_, &zv_)) {                \
            if (px_ < mnx) mnx = px_;                              \
            if (px_ > mxx) mxx = px_;                              \
            if (py_ < mny) mny = py_;                              \
            if (py_ > mxy) mxy = py_;                              \
        }                                                          \
    } while (0)
    for (int corner = 0; corner < 8; ++corner)
        if (c->proj != 0 || cz[corner] >= zc) OS_ADD(cp[corner]);
    if (c->proj == 0 && zmin < zc) {
        /* the 12 edges join corners differing in one coordinate bit */
        for (int a = 0; a < 8; ++a)
            for (int bit = 1; bit < 8; bit <<= 1) {
                int b = a | bit;
                if (b == a) continue;
                if ((cz[a] < zc) == (cz[b] < zc)) continue;
                double t = (zc - cz[a]) / (cz[b] - cz[a]);
                double q[3];
                for (int k = 0; k < 3; ++k) q[k] = cp[a][k] + t * (cp[b][k] - cp[a][k]);
                /* the crossing point, nudged onto the front side of the plane */
                double r[3] = {q[0] - c->e[0], q[1] - c->e[1], q[2] - c->e[2]};
                double zq = dot3(r, c->f);
                if (zq < zc) for (int k = 0; k < 3; ++k) q[k] += (zc - zq) * c->f[k];
                OS_ADD(q);
            }
    }
#undef OS_ADD
    if (!(mnx <= mxx && mny <= mxy)) { *rx0 = 0; *ry0 = 0; *rx1 = c->W - 1; *ry1 = c->H - 1; return 1; }
    double fx0 = floor(mnx - 0.5) - 1, fx1 = ceil(mxx - 0.5) + 1;
    double fy0 = floor(mny - 0.5) - 1, fy1 = ceil(mxy - 0.5) + 1;
    if (fx1 < 0 || fy1 < 0 || fx0 > c->W - 1 || fy0 > c->H - 1) return 0;
    *rx0 = fx0 < 0 ? 0 : (int)fx0;
    *ry0 = fy0 < 0 ? 0 : (int)fy0;
    *rx1 = fx1 > c->W - 1 ? c->W - 1 : (int)fx1;
    *ry1 = fy1 > c->H - 1 ? c->H - 1 : (int)fy1;
    return 1;
}

typedef struct {
    int cand;        /* hit or grazing near-hit inside the depth range band */
    int valid;       /* exact FP64 hit */
    int graze;       /* outcome could flip under rounding */
    int unstable;    /* shading could flip (cap/side, colour half) */
    int half_b;      /* bond: colour of the second atom */
    double z;
    double n[3];     /* world normal */
    double nv;       /* n . V */
} os_hit;

static void os_zclass(const os_cam* c, double z, int geom_hit, int geom_graze, os_hit* h) {
    int zin = (z >= c->znear) && (z <= c->zfar);
    double za = fabs(z) > c->znear ? fabs(z) : c->znear;
    int zgr = (fabs(z - c->znear) <= OS_TAU * za) || (fabs(z - c->zfar) <= OS_TAU * c->zfar);
    h->cand = zin || zgr;
    h->valid = geom_hit && zin;
    h->graze = h->cand && (geom_graze || zgr);
}

/* Clip plane: a candidate whose surface point lies on the cut side is not
 * drawn (nor is anything behind it of the same primitive); within rounding
 * of the plane it may go either way. */
static void os_clip(const os_cam* c, const double* x, os_hit* h) {
    if (!c->clip_on || !h->cand) return;
    double v = c->clip[0] * x[0] + c->clip[1] * x[1] + c->clip[2] * x[2] + c->clip[3];
    double sc = fabs(c->clip[0] * x[0]) + fabs(c->clip[1] * x[1]) + fabs(c->clip[2] * x[2]) + fabs(c->clip[3]);
    double tol = OS_TAU * sc;
    if (v < -tol) {
        h->cand = 0;
        h->valid = 0;
        return;
    }
    if (v < 0.0) h->valid = 0;
    if (fabs(v) <= tol) h->graze = 1;
}

static void os_sphere(const os_cam* c, const double* o, const double* d, const double* ctr, double r, os_hit* h) {
    h->cand = 0;
    double oc[3] = {ctr[0] - o[0], ctr[1] - o[1], ctr[2] - o[2]};
    double b = dot3(oc, d);
    double q[3] = {oc[0] - b * d[0], oc[1] - b * d[1], oc[2] - b * d[2]};
    double qn = sqrt(dot3(q, q));
    double ocn = sqrt(dot3(oc, oc));
    int gg = fabs(r - qn) <= OS_TAU * ocn;
    double disc = r * r - qn * qn;
    int gh = disc >= 0.0;
    if (!gh && !gg) return;
    double t = gh ? b - sqrt(disc > 0 ? disc : 0.0) : b;
    double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    double rel[3] = {x[0] - c->e[0], x[1] - c->e[1], x[2] - c->e[2]};
    double z = dot3(rel, c->f);
    os_zclass(c, z, gh, gg, h);
    os_clip(c, x, h);
    if (!h->cand) return;
    h->z = z;
    for (int k = 0; k < 3; ++k) h->n[k] = (x[k] - ctr[k]) / r;
    h->nv = -dot3(h->n, d);
    h->unstable = 0;
    h->half_b = 0;
}

static void os_cylinder(const os_cam* c, const double* o, const double* d, const double* A, const double* B,
                        double rho, os_hit* h) {
    h->cand = 0;
    double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double L = sqrt(dot3(ab, ab));
    if (L == 0.0) return;
    double a[3] = {ab[0] / L, ab[1] / L, ab[2] / L};
    double w[3] = {o[0] - A[0], o[1] - A[1], o[2] - A[2]};
    double wn = sqrt(dot3(w, w));
    double tol = OS_TAU * wn;
    double da = dot3(d, a), wa = dot3(w, a);
    double dp[3], wp[3];
    for (int k = 0; k < 3; ++k) { dp[k] = d[k] - da * a[k]; wp[k] = w[k] - wa * a[k]; }
    double kk = dot3(dp, dp);

    /* lateral surface */
    double tc = kk > 0 ? -dot3(wp, dp) / kk : 0.0;
    double qv[3] = {wp[0] + tc * dp[0], wp[1] + tc * dp[1], wp[2] + tc * dp[2]};
    double qn = sqrt(dot3(qv, qv));
    double disc = rho * rho - qn * qn;
    int side_geom = (kk > 0) && (disc >= 0);
    double ts = side_geom ? tc - sqrt((disc > 0 ? disc : 0.0) / kk) : tc;
    double ss = wa + ts * da;
    int side_valid = side_geom && ss >= 0.0 && ss <= L;
    int side_sil = (kk > 0) && fabs(rho - qn) <= tol && ss >= -tol && ss <= L + tol;
    int side_end = side_geom && (fabs(ss) <= tol || fabs(ss - L) <= tol);
    int side_graze = side_sil || side_end;

    /* caps */
    int nonpar = fabs(da) >= 1e-12;
    double tA = nonpar ? -wa / da : INFINITY;
    double tB = nonpar ? (L - wa) / da : INFINITY;
    double tAu = nonpar ? tA : 0.0, tBu = nonpar ? tB : 0.0;
    double pA[3], pB[3];
    for (int k = 0; k < 3; ++k) {
        pA[k] = w[k] + tAu * d[k];
        pB[k] = w[k] + tBu * d[k] - L * a[k];
    }
    double rA = sqrt(dot3(pA, pA)), rB = sqrt(dot3(pB, pB));
    int capA_geom = nonpar && da > 0 && rA <= rho;
    int capB_geom = nonpar && da < 0 && rB <= rho;
    int edge_on = fabs(da) <= OS_TAU;
    int capA_graze = (nonpar && da > -OS_TAU && fabs(rA - rho) <= tol) || (edge_on && rA <= rho + tol);
    int capB_graze = (nonpar && da < OS_TAU && fabs(rB - rho) <= tol) || (edge_on && rB <= rho + tol);

    double t = INFINITY;
    int kind = -1;
    if (side_valid) { t = ts; kind = 0; }
    if (capA_geom && tA < t) { t = tA; kind = 1; }
    if (capB_geom && tB < t) { t = tB; kind = 2; }
    int geom_hit = kind >= 0;
    int any_graze = side_graze || capA_graze || capB_graze;
    double tg = INFINITY;
    if (side_graze && ts < tg) tg = ts;
    if (capA_graze && isfinite(tA) && tA < tg) tg = tA;
    if (capB_graze && isfinite(tB) && tB < tg) tg = tB;
    if (!geom_hit && !(any_graze && isfinite(tg))) return;
    double tu = geom_hit ? t : tg;
    if (kind < 0) kind = 0;
    double x[3] = {o[0] + tu * d[0], o[1] + tu * d[1], o[2] + tu * d[2]};
    double rel[3] = {x[0] - c->e[0], x[1] - c->e[1], x[2] - c->e[2]};
    double z = dot3(rel, c->f);
    os_zclass(c, z, geom_hit, any_graze, h);
    os_clip(c, x, h);
    if (!h->cand) return;
    h->z = z;
    double xa[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
    double s_hit = dot3(xa, a);
    if (kind == 0) {
        for (int k = 0; k < 3; ++k) h->n[k] = (xa[k] - s_hit * a[k]) / rho;
        h->half_b = s_hit >= 0.5 * L;
    } else if (kind == 1) {
        for (int k = 0; k < 3; ++k) h->n[k] = -a[k];
        h->half_b = 0;
    } else {
        for (int k = 0; k < 3; ++k) h->n[k] = a[k];
        h->half_b = 1;
    }
    int colour_edge = (kind == 0) && fabs(s_hit - 0.5 * L) <= tol;
    h->unstable = colour_edge || side_end || (kind != 0 && (capA_graze || capB_graze));
    h->nv = -dot3(h->n, d);
}

typedef struct {
    int x0, y0, x1, y1;   /* inclusive pixel rectangle */
    int ok;
} os_rect;

static int lexless(double za, uint32_t ia, double zb, uint32_t ib) {
    return za < zb || (za == zb && ia < ib);
}

/* cam: eye3 target3 up3 fovy ortho_half_height projection znear zfar (14 doubles) */
int osplat_gbuffer(int64_t n, const float* pos, const float* rad, const uint32_t* col,
                   int64_t m, const uint32_t* bonds, double bond_radius,
                   const double* cam, int W, int H, int x0, int y0, int w, int h, int nthreads,
                   double* out_z, uint32_t* out_id, double* out_n, uint32_t* out_alb,
                   uint8_t* out_unstable, double* out_nv,
                   int32_t* acc_n, uint32_t* acc_id, double* acc_z, uint8_t* acc_bg,
                   int64_t* fragments) {
    if (n < 0 || m < 0 || W <= 0 || H <= 0 || w <= 0 || h <= 0) return -1;
    if (x0 < 0 || y0 < 0 || x0 + w > W || y0 + h > H) return -1;
    os_cam c;
    os_make_cam(cam, W, H, &c);
    int64_t np_ = n + m;
    os_rect* rects = (os_rect*)malloc(sizeof(os_rect) * (size_t)(np_ > 0 ? np_ : 1));
    if (!rects) return -2;
    if (nthreads > 0) omp_set_num_threads(nthreads);

#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np_; ++p) {
        double lo[3], hi[3];
        os_rect* r = &rects[p];
        r->ok = 0;
        if (p < n) {
            double rr = rad[p];
            for (int k = 0; k < 3; ++k) { lo[k] = (double)pos[3 * p + k] - rr; hi[k] = (double)pos[3 * p + k] + rr; }
            double grow = 4 * OS_TAU * (fabs((double)pos[3 * p]) + fabs((double)pos[3 * p + 1]) + fabs((double)pos[3 * p + 2]) +
                                        fabs(c.e[0]) + fabs(c.e[1]) + fabs(c.e[2]) + rr);
            for (int k = 0; k < 3; ++k) { lo[k] -= grow; hi[k] += grow; }
        } else {
            int64_t b = p - n;
            uint32_t ia = bonds[2 * b], ib = bonds[2 * b + 1];
            if (ia == ib || ia >= (uint64_t)n || ib >= (uint64_t)n) continue;
            double mag = fabs(c.e[0]) + fabs(c.e[1]) + fabs(c.e[2]) + bond_radius;
            for (int k = 0; k < 3; ++k) {
                double va = pos[3 * (int64_t)ia + k], vb = pos[3 * (int64_t)ib + k];
                lo[k] = (va < vb ? va : vb) - bond_radius;
                hi[k] = (va > vb ? va : vb) + bond_radius;
                mag += fabs(va) + fabs(vb);
            }
            double grow = 4 * OS_TAU * mag;
            for (int k = 0; k < 3; ++k) { lo[k] -= grow; hi[k] += grow; }
        }
        r->ok = os_box_rect(&c, lo, hi, &r->x0, &r->y0, &r->x1, &r->y1);
    }

    /* the primitives whose footprint meets the window, in primitive order
       (every band below walks this list instead of all of them) */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < np_; ++p) {
        os_rect* r = &rects[p];
        if (r->ok && (r->x1 < x0 || r->x0 > x0 + w - 1 || r->y1 < y0 || r->y0 > y0 + h - 1)) r->ok = 0;
    }
    int64_t nsel = 0;
    for (int64_t p = 0; p < np_; ++p) nsel += rects[p].ok ? 1 : 0;
    int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nsel > 0 ? nsel : 1));
    if (!sel) { free(rects); return -2; }
    nsel = 0;
    for (int64_t p = 0; p < np_; ++p)
        if (rects[p].ok) sel[nsel++] = p;

    int64_t P = (int64_t)w * h;
    double* zstar = (double*)malloc(sizeof(double) * (size_t)P);
    if (!zstar) { free(rects); free(sel); return -2; }
    int64_t frag_total = 0;

#pragma omp parallel reduction(+ : frag_total)
    {
        int nt = omp_get_num_threads(), tid = omp_get_thread_num();
        int band0 = y0 + (int)((int64_t)h * tid / nt), band1 = y0 + (int)((int64_t)h * (tid + 1) / nt);
        for (int y = band0; y < band1; ++y)
            for (int x = x0; x < x0 + w; ++x) {
                int64_t q = (int64_t)(y - y0) * w + (x - x0);
                out_z[q] = INFINITY;
                out_id[q] = OS_BG_ID;
                out_n[3 * q] = out_n[3 * q + 1] = out_n[3 * q + 2] = 0.0;
                out_alb[q] = 0;
                out_unstable[q] = 0;
                out_nv[q] = 0.0;
                zstar[q] = INFINITY;
                acc_n[q] = 0;
                acc_bg[q] = 1;
                for (int k = 0; k < OS_MAX_ACCEPT; ++k) { acc_id[q * OS_MAX_ACCEPT + k] = OS_BG_ID; acc_z[q * OS_MAX_ACCEPT + k] = INFINITY; }
            }
        /* pass 1: exact winner and the depth of the nearest solid hit */
        for (int pass = 0; pass < 2; ++pass) {
            for (int64_t k_sel = 0; k_sel < nsel; ++k_sel) {
                const int64_t p = sel[k_sel];
                const os_rect* r = &rects[p];
                int ya = r->y0 > band0 ? r->y0 : band0;
                int yb = r->y1 < band1 - 1 ? r->y1 : band1 - 1;
                int xa = r->x0 > x0 ? r->x0 : x0;
                int xb = r->x1 < x0 + w - 1 ? r->x1 : x0 + w - 1;
                if (ya > yb || xa > xb) continue;
                double ctr[3], A[3], B[3], rr = 0.0;
                uint32_t ca = 0, cb = 0;
                if (p < n) {
                    for (int k = 0; k < 3; ++k) ctr[k] = pos[3 * p + k];
                    rr = rad[p];
                    ca = col[p];
                } else {
                    int64_t b = p - n;
                    uint32_t ia = bonds[2 * b], ib = bonds[2 * b + 1];
                    for (int k = 0; k < 3; ++k) { A[k] = pos[3 * (int64_t)ia + k]; B[k] = pos[3 * (int64_t)ib + k]; }
                    ca = col[ia];
                    cb = col[ib];
                }
                for (int y = ya; y <= yb; ++y)
                    for (int x = xa; x <= xb; ++x) {
                        double o[3], d[3];
                        os_ray(&c, x, y, o, d);
                        os_hit hh;
                        if (p < n) os_sphere(&c, o, d, ctr, rr, &hh);
                        else os_cylinder(&c, o, d, A, B, bond_radius, &hh);
                        if (!hh.cand) continue;
                        int64_t q = (int64_t)(y - y0) * w + (x - x0);
                        uint32_t id = (uint32_t)p;
                        if (pass == 0) {
                            if (hh.valid) {
                                ++frag_total;
                                if (lexless(hh.z, id, out_z[q], out_id[q])) {
                                    out_z[q] = hh.z;
                                    out_id[q] = id;
                                    double nw[3] = {hh.n[0], hh.n[1], hh.n[2]};
                                    out_n[3 * q] = dot3(nw, c.s);
                                    out_n[3 * q + 1] = dot3(nw, c.u);
                                    out_n[3 * q + 2] = dot3(nw, c.f);
                                    out_alb[q] = (p < n) ? ca : (hh.half_b ? cb : ca);
                                    out_unstable[q] = (uint8_t)hh.unstable;
                                    out_nv[q] = hh.nv;
                                }
                                if (!hh.graze && hh.z < zstar[q]) zstar[q] = hh.z;
                            }
                        } else {
                            if ((hh.valid || hh.graze) && hh.z <= zstar[q] * (1.0 + OS_TAU)) {
                                int k = acc_n[q]++;
                                if (k < OS_MAX_ACCEPT) {
                                    acc_id[q * OS_MAX_ACCEPT + k] = id;
                                    acc_z[q * OS_MAX_ACCEPT + k] = hh.z;
                                }
                            }
                        }
                    }
            }
            if (pass == 0) {
                for (int y = band0; y < band1; ++y)
                    for (int x = x0; x < x0 + w; ++x) {
                        int64_t q = (int64_t)(y - y0) * w + (x - x0);
                        acc_bg[q] = !isfinite(zstar[q]);
                    }
            }
        }
    }
    *fragments = frag_total;
    free(zstar);
    free(rects);
    free(sel);
    return 0;
}

static void os_onb(const double* n, double* T, double* B) {
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    T[0] = 1.0 + sign * n[0] * n[0] * a; T[1] = sign * b; T[2] = -sign * n[0];
    B[0] = b; B[1] = sign + n[1] * n[1] * a; B[2] = -n[1];
}

static double os_smooth(double x) {
    if (!(x > 0.0)) x = 0.0;   /* NaN -> 0 */
    if (x > 1.0) x = 1.0;
    return x * x * (3.0 - 2.0 * x);
}

/* The 4x4 ordered-dither (Bayer) matrix: the noise pattern of the SSAO
   rotation (R6b). */
static const int os_bayer4[4][4] = {{0, 8, 2, 10}, {12, 4, 14, 6}, {3, 11, 1, 9}, {15, 7, 13, 5}};

/* SSAO of one hit pixel (R6): the view position Pv and unit normal N, the
   sample kernel hk/sk, and, with noise, the rotation (cr, sr) of the tangent
   frame about N.  Returns the occlusion sum; counts unstable samples and
   on-screen samples that fall outside the depth buffer. */
static double os_ssao_pixel(const os_cam* c, int W, int H, const double* Pv, const double* N, int K,
                            double (*hk)[3], const double* sk, double R, double bias, double cr, double sr,
                            const double* depth_buf, const uint8_t* ambiguous, int bx0, int by0, int bw, int bh,
                            double edge_px, double depth_rel, int* uns, int* outside) {
    double fpx = (H / 2.0) / c->tanh_;
    double osc = (H / 2.0) / c->hh;
    double T0[3], B0[3], T[3], B[3];
    os_onb(N, T0, B0);
    for (int a = 0; a < 3; ++a) {
        T[a] = cr * T0[a] + sr * B0[a];
        B[a] = cr * B0[a] - sr * T0[a];
    }
    if (fabs(N[2]) <= 1e-4) *uns += K;
    double occ = 0.0;
    for (int k = 0; k < K; ++k) {
        double S[3];
        double sc = R * sk[k];
        for (int a = 0; a < 3; ++a) S[a] = Pv[a] + sc * (hk[k][0] * T[a] + hk[k][1] * B[a] + hk[k][2] * N[a]);
        double px, py;
        int front = S[2] > c->znear;
        double za = fabs(S[2]) > c->znear ? fabs(S[2]) : c->znear;
        int near_edge = fabs(S[2] - c->znear) <= depth_rel * za;
        if (c->proj == 0) {
            px = W / 2.0 + fpx * S[0] / S[2];
            py = H / 2.0 - fpx * S[1] / S[2];
        } else {
            px = W / 2.0 + S[0] * osc;
            py = H / 2.0 - S[1] * osc;
        }
        double qx = floor(px), qy = floor(py);
        int onscreen = front && qx >= 0 && qx < W && qy >= 0 && qy < H;
        double fx = px - qx, fy = py - qy;
        int edge = (fmin(fx, 1 - fx) <= edge_px) || (fmin(fy, 1 - fy) <= edge_px);
        int in_buf = 0, ok = 0;
        double zq = INFINITY;
        if (onscreen) {
            int ix = (int)qx - bx0, iy = (int)qy - by0;
            in_buf = ix >= 0 && ix < bw && iy >= 0 && iy < bh;
            if (in_buf) { ok = 1; zq = depth_buf[(int64_t)iy * bw + ix]; }
            else ++*outside;
        }
        double thr = S[2] - bias;
        if (ok && zq <= thr && isfinite(zq)) occ += os_smooth(R / fabs(Pv[2] - zq));
        int margin = ok && fabs(zq - thr) <= depth_rel * fabs(S[2]);
        /* a sample reading a pixel whose visible primitive is not
           unique may see another correct depth there */
        if (ok && ambiguous && ambiguous[(int64_t)((int)qy - by0) * bw + ((int)qx - bx0)]) margin = 1;
        if ((front && edge) || near_edge || margin) ++*uns;
    }
    return occ;
}

/* View position and unit direction towards the eye of pixel (X, Y) at depth zz. */
static void os_pixel_view(const os_cam* c, int W, int H, int X, int Y, double zz, double* Pv, double* V) {
    double nx = 2.0 * (X + 0.5) / W - 1.0, ny = 1.0 - 2.0 * (Y + 0.5) / H;
    if (c->proj == 0) {
        Pv[0] = zz * nx * c->tanh_ * c->aspect; Pv[1] = zz * ny * c->tanh_; Pv[2] = zz;
        double dv[3] = {nx * c->tanh_ * c->aspect, ny * c->tanh_, 1.0};
        norm3(dv);
        V[0] = -dv[0]; V[1] = -dv[1]; V[2] = -dv[2];
    } else {
        Pv[0] = nx * c->hh * c->aspect; Pv[1] = ny * c->hh; Pv[2] = zz;
        V[0] = 0.0; V[1] = 0.0; V[2] = -1.0;
    }
}

/* Deferred pass (SSAO, then the shading mode, fog and outline) over a
 * window.  shading: 0 glossy, 1 matte, 2 flat, 3 toon; fog from fog_start to
 * fog_end (none unless fog_end > fog_start); outline_t > 0 draws outlines.
 * depth_buf (and normal_buf, the view normals over the same region; may be
 * NULL when noise is 0) cover (bx0, by0, bw, bh) of the image.
 * noise != 0 (R6b): each pixel's tangent frame is rotated about its normal
 * by 2 pi (B[Y mod 4][X mod 4] + 1/2) / 16, B the 4x4 Bayer matrix, with the
 * cosine and sine rounded to FP32; the AO of a hit pixel is then the mean of
 * those raw values over the hit pixels (X + dx, Y + dy), dx, dy in
 * {-2, -1, 0, 1}, inside the image.
 * unstable_out counts every decision FP32 may take the other way: SSAO
 * samples near a pixel edge or their depth threshold, or reading a pixel
 * flagged in `ambiguous` (over the depth buffer; may be NULL) because its
 * visible primitive is not unique, toon band edges and outline depth
 * thresholds; with noise, those of every raw value the blur takes.
 * outside_out counts samples (and, with noise, blur neighbours) the buffers
 * do not cover. */
int osplat_shade(const double* cam, int W, int H, int x0, int y0, int w, int h,
                 const double* z, const double* nrm, const uint32_t* alb,
                 const double* depth_buf, const double* normal_buf, int bx0, int by0, int bw, int bh,
                 int K, double R, double bias, int noise, uint32_t background, double edge_px, double depth_rel,
                 int shading, double fog_start, double fog_end, uint32_t fog_color,
                 double outline_t, uint32_t outline_color, const uint8_t* ambiguous,
                 int nthreads, uint32_t* rgba, double* ao_out, int32_t* unstable_out, int32_t* outside_out) {
    if (K < 0 || K > 1024) return -1;
    if (noise && !normal_buf) return -1;
    os_cam c;
    os_make_cam(cam, W, H, &c);
    double hk[1024][3], sk[1024];
    for (int k = 0; k < K; ++k) {
        double ct = 1.0 - (k + 0.5) / K;
        double st = sqrt(1.0 - ct * ct);
        double ph = 2.0 * OS_PI * fmod(k * 0.6180339887498949, 1.0);
        hk[k][0] = (float)(st * cos(ph));
        hk[k][1] = (float)(st * sin(ph));
        hk[k][2] = (float)ct;
        double u = (k + 1.0) / K;
        sk[k] = (float)(0.1 + 0.9 * u * u);
    }
    double rot_c[16], rot_s[16];
    for (int b = 0; b < 16; ++b) {
        double th = 2.0 * OS_PI * (b + 0.5) / 16.0;
        rot_c[b] = (float)cos(th);
        rot_s[b] = (float)sin(th);
    }
    if (nthreads > 0) omp_set_num_threads(nthreads);
    /* with noise: the raw AO of every pixel of the window grown by the blur
       footprint (two left and up, one right and down), kept inside the
       buffers and the image */
    int gx0 = x0, gy0 = y0, gw = 0, gh = 0;
    double* raw = NULL;
    int32_t *raw_uns = NULL, *raw_out = NULL;
    uint8_t* raw_hit = NULL;
    if (noise && K > 0) {
        gx0 = x0 - 2 > bx0 ? x0 - 2 : bx0;
        gy0 = y0 - 2 > by0 ? y0 - 2 : by0;
        int gx1 = x0 + w + 1 < bx0 + bw ? x0 + w + 1 : bx0 + bw;
        int gy1 = y0 + h + 1 < by0 + bh ? y0 + h + 1 : by0 + bh;
        gw = gx1 - gx0;
        gh = gy1 - gy0;
        raw = (double*)malloc(sizeof(double) * (size_t)gw * gh);
        raw_uns = (int32_t*)malloc(sizeof(int32_t) * (size_t)gw * gh);
        raw_out = (int32_t*)malloc(sizeof(int32_t) * (size_t)gw * gh);
        raw_hit = (uint8_t*)malloc((size_t)gw * gh);
        if (!raw || !raw_uns || !raw_out || !raw_hit) { free(raw); free(raw_uns); free(raw_out); free(raw_hit); return -2; }
#pragma omp parallel for schedule(dynamic, 4)
        for (int j = 0; j < gh; ++j)
            for (int i = 0; i < gw; ++i) {
                int X = gx0 + i, Y = gy0 + j;
                int64_t q = (int64_t)j * gw + i;
                int64_t qb = (int64_t)(Y - by0) * bw + (X - bx0);
                double zz = depth_buf[qb];
                raw_hit[q] = isfinite(zz) ? 1 : 0;
                raw[q] = 0.0;
                raw_uns[q] = 0;
                raw_out[q] = 0;
                if (!raw_hit[q]) continue;
                double Pv[3], V[3];
                os_pixel_view(&c, W, H, X, Y, zz, Pv, V);
                int b = os_bayer4[Y & 3][X & 3];
                int uns = 0, outside = 0;
                double occ = os_ssao_pixel(&c, W, H, Pv, normal_buf + 3 * qb, K, hk, sk, R, bias, rot_c[b], rot_s[b],
                                           depth_buf, ambiguous, bx0, by0, bw, bh, edge_px, depth_rel, &uns, &outside);
                raw[q] = 1.0 - occ / K;
                raw_uns[q] = uns;
                raw_out[q] = outside;
            }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < w; ++i) {
            int64_t q = (int64_t)j * w + i;
            int X = x0 + i, Y = y0 + j;
            double zz = z[q];
            if (!isfinite(zz)) {
                rgba[q] = background;
                ao_out[q] = 1.0;
                unstable_out[q] = 0;
                outside_out[q] = 0;
                continue;
            }
            double Pv[3], V[3];
            os_pixel_view(&c, W, H, X, Y, zz, Pv, V);
            const double* N = nrm + 3 * q;
            double occ = 0.0;
            int uns = 0, outside = 0;
            double ao = 1.0;
            if (K > 0 && !noise) {
                occ = os_ssao_pixel(&c, W, H, Pv, N, K, hk, sk, R, bias, 1.0, 0.0, depth_buf, ambiguous, bx0, by0, bw,
                                    bh, edge_px, depth_rel, &uns, &outside);
                ao = 1.0 - occ / K;
            } else if (K > 0) {
                double sum = 0.0;
                int cnt = 0;
                for (int dy = -2; dy <= 1; ++dy)
                    for (int dx = -2; dx <= 1; ++dx) {
                        int QX = X + dx, QY = Y + dy;
                        if (QX < 0 || QX >= W || QY < 0 || QY >= H) continue;
                        if (QX < gx0 || QX >= gx0 + gw || QY < gy0 || QY >= gy0 + gh) { ++outside; continue; }
                        int64_t g = (int64_t)(QY - gy0) * gw + (QX - gx0);
                        if (!raw_hit[g]) continue;
                        sum += raw[g];
                        ++cnt;
                        uns += raw_uns[g];
                        outside += raw_out[g];
                    }
                ao = cnt ? sum / cnt : 1.0;
            }
            double nv = dot3(N, V);
            if (nv < 0) nv = 0;
            /* shading mode: lit = ka + kd * (facing term), times AO; glossy
               adds the white highlight */
            double lit, spec = 0.0;
            if (shading == 2) {
                lit = ao;
            } else if (shading == 3) {
                double band = floor(4.0 * nv);
                if (band > 3.0) band = 3.0;
                lit = (OS_KA + OS_KD * band / 3.0) * ao;
                double k = floor(4.0 * nv + 0.5);
                if (k >= 1.0 && k <= 3.0 && fabs(4.0 * nv - k) <= 1e-4) ++uns;
            } else {
                lit = (OS_KA + OS_KD * nv) * ao;
                if (shading == 0) {
                    double sp = 2.0 * nv * nv - 1.0;
                    spec = OS_KS * pow(sp > 0 ? sp : 0.0, OS_SHININESS);
                }
            }
            double fogf = 0.0;
            if (fog_end > fog_start) {
                fogf = (zz - fog_start) / (fog_end - fog_start);
                if (fogf < 0.0) fogf = 0.0;
                if (fogf > 1.0) fogf = 1.0;
            }
            uint32_t a = alb[q], out = 0;
            for (int ch = 0; ch < 3; ++ch) {
                double al = ((a >> (8 * ch)) & 255u) / 255.0;
                double cc = al * lit + spec;
                cc = (1.0 - fogf) * cc + fogf * (((fog_color >> (8 * ch)) & 255u) / 255.0);
                if (cc < 0) cc = 0;
                if (cc > 1) cc = 1;
                out |= ((uint32_t)floor(255.0 * cc + 0.5)) << (8 * ch);
            }
            out |= 255u << 24;
            if (outline_t > 0.0) {
                static const int nb[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
                double thr = zz * (1.0 + outline_t);
                int edge = 0;
                for (int e = 0; e < 4; ++e) {
                    int QX = X + nb[e][0], QY = Y + nb[e][1];
                    if (QX < 0 || QX >= W || QY < 0 || QY >= H) continue;
                    int ix = QX - bx0, iy = QY - by0;
                    if (ix < 0 || ix >= bw || iy < 0 || iy >= bh) { ++uns; continue; }
                    double zq = depth_buf[(int64_t)iy * bw + ix];
                    if (zq > thr) edge = 1;
                    if (isfinite(zq) && fabs(zq - thr) <= depth_rel * fabs(zz)) ++uns;
                }
                if (edge) out = (outline_color & 0xFFFFFFu) | (255u << 24);
            }
            rgba[q] = out;
            ao_out[q] = ao;
            unstable_out[q] = uns;
            outside_out[q] = outside;
        }
    free(raw);
    free(raw_uns);
    free(raw_out);
    free(raw_hit);
    return 0;
}

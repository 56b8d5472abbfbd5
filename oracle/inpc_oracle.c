/*
 * CPU oracle for the INPC point rasterizer -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, per-pixel definition of what the rasterizer computes.  It is
 * used by the tests, by the smoke check and by the benchmark's CPU baseline;
 * the product path never links or calls it, and it shares no code with the
 * GPU kernels.
 *
 * What it follows (paper: "A Bag of Tricks for Efficient Implicit Neural
 * Point Clouds"):
 *  - Sec. 2, "Rendering Feature Maps": every pixel's fragments are sorted by
 *    depth and alpha-blended, then composited with the background.
 *  - Appendix A, Eq. (1): F = sum_i T_i a_i f_i, T_i = prod_{j<i} (1 - a_j);
 *    Eq. (2): the alpha derivative, which must not skip a = 0 fragments.
 *  - Sec. 2 and Sec. 3.2 "Rendering Points as Small Gaussians": a bilinear
 *    2x2 splat whose four weights sum to one, or (inference) an isotropic
 *    screen-space Gaussian with dilation variance 0.16 truncated at 3 sigma.
 *  - Sec. 3.2 "Tiled Rendering": per-tile lists of the points whose
 *    footprint meets the tile, in depth order.
 *
 * Precision: every discrete decision (cull, footprint pixels, tile
 * membership, Gaussian cut, bilinear termination) is taken in IEEE FP32 with
 * one rounding per operation and no fused multiply-add (this file must be
 * built with -ffp-contract=off; x86-64 float arithmetic is SSE, so each
 * operation rounds to single precision).  Every continuous value (weights,
 * alpha, transmittance, features, gradients) is then computed in FP64 from
 * the FP32 decision-stage quantities u and v.
 *
 * Readings where the paper is silent:
 *  - pixel (x, y) covers [x, x+1) x [y, y+1); its centre is at +0.5;
 *  - fragment opacity is o * w with no clamp (a = 1 is legal);
 *  - depth is camera-space Z; its FP32 bit pattern is the sort key, ties
 *    are broken by ascending point index;
 *  - fragment k is blended iff the transmittance in front of it is
 *    >= t_min (t_min = 0 gives Eq. (1) exactly);
 *  - the background enters as T_final * f_bg, and its derivative carries
 *    the sign that differentiating Eq. (1) gives (negative), not the sign
 *    printed in Eq. (2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float z_near;
} ocam_t;

typedef struct {
    int32_t splat; /* 0 bilinear, 1 screen-space Gaussian, 2 world-space Gaussian (EWA) */
    int32_t tile;
    float t_min;
    float dilation;
    float cutoff;
    float ewa_sigma; /* splat 2: world-space standard deviation of every point */
} oopts_t;

/* ------------------------------------------------------------------ */
/* Decision stage (FP32, one rounding per operation)                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int visible;
    float X, Y, Z, u, v;
    uint32_t key;
    int32_t px0, py0, px1, py1; /* inclusive in-image pixel rect of candidate fragments */
    int32_t x0, y0;             /* bilinear: top-left pixel of the 2x2 splat */
    float a, b;                 /* bilinear: sub-pixel offsets */
    float s2, thr;              /* Gaussian: effective variance, squared cut radius */
    float ca, cb, cc;           /* EWA: inverse of the projected covariance (conic) */
    int ewa;                    /* a world-space (EWA) Gaussian */
} opoint_t;

static uint32_t f32_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

/* Camera transform X = R p + t, then pinhole projection (Sec. 2: points are
 * rasterized into the image of a calibrated camera). */
static void decide_point(const ocam_t* cam, const oopts_t* o, const float* p, float radius,
                         opoint_t* q) {
    const float* R = cam->R;
    float X = ((R[0] * p[0] + R[1] * p[1]) + R[2] * p[2]) + cam->t[0];
    float Y = ((R[3] * p[0] + R[4] * p[1]) + R[5] * p[2]) + cam->t[1];
    float Z = ((R[6] * p[0] + R[7] * p[1]) + R[8] * p[2]) + cam->t[2];
    memset(q, 0, sizeof(*q));
    q->X = X; q->Y = Y; q->Z = Z;
    if (!(Z > cam->z_near)) return; /* NaN is culled too */
    float qx = X / Z, qy = Y / Z;
    float mx = cam->fx * qx, my = cam->fy * qy;
    float u = mx + cam->cx, v = my + cam->cy;
    q->u = u; q->v = v;
    q->key = f32_bits(Z);
    const int W = cam->width, H = cam->height;
    const float Wf = (float)W, Hf = (float)H;
    if (o->splat == 0) {
        /* bilinear 2x2 splat: the pixels whose centres surround (u, v) */
        if (!(u >= -0.5f && u < Wf + 0.5f && v >= -0.5f && v < Hf + 0.5f)) return;
        float xs = u - 0.5f, ys = v - 0.5f;
        float fx0 = floorf(xs), fy0 = floorf(ys);
        q->x0 = (int32_t)fx0; q->y0 = (int32_t)fy0;
        q->a = xs - fx0; q->b = ys - fy0;
        q->px0 = q->x0 < 0 ? 0 : q->x0;
        q->py0 = q->y0 < 0 ? 0 : q->y0;
        q->px1 = q->x0 + 1 > W - 1 ? W - 1 : q->x0 + 1;
        q->py1 = q->y0 + 1 > H - 1 ? H - 1 : q->y0 + 1;
        q->visible = 1;
    } else if (o->splat == 2) {
        /* World-space isotropic Gaussian of standard deviation sigma (Sec. 3.2
         * "Rendering Points as Small Gaussians"), projected with the affine
         * (EWA) approximation of the perspective map: covariance
         * sigma^2 J J^T with J the projection's Jacobian at the point, plus
         * the dilation.  With xh = X/Z = (u - cx)/fx, yh = (v - cy)/fy,
         * jx = fx/Z, jy = fy/Z this is
         *   a = sigma^2 jx^2 (1 + xh^2) + dil, b = sigma^2 jx jy xh yh,
         *   c = sigma^2 jy^2 (1 + yh^2) + dil,
         * written from the FP32 u, v, Z so that the kernels reach the same
         * FP32 decisions; cut where the Mahalanobis distance exceeds
         * `cutoff`; the candidate box is the ellipse's bounding box,
         * |dx| <= cutoff sqrt(a), |dy| <= cutoff sqrt(c). */
        float xh = (u - cam->cx) / cam->fx, yh = (v - cam->cy) / cam->fy;
        float jx = cam->fx / Z, jy = cam->fy / Z;
        float s2w = o->ewa_sigma * o->ewa_sigma;
        float a = s2w * ((jx * jx) * (1.0f + xh * xh)) + o->dilation;
        float b = s2w * ((jx * jy) * (xh * yh));
        float c = s2w * ((jy * jy) * (1.0f + yh * yh)) + o->dilation;
        float det = a * c - b * b;
        q->ca = c / det;
        q->cb = -(b / det);
        q->cc = a / det;
        float Rx = o->cutoff * sqrtf(a), Ry = o->cutoff * sqrtf(c);
        float xs = u - 0.5f, ys = v - 0.5f;
        float lx = ceilf(xs - Rx), hx = floorf(xs + Rx);
        float ly = ceilf(ys - Ry), hy = floorf(ys + Ry);
        if (lx < 0.0f) lx = 0.0f;
        if (ly < 0.0f) ly = 0.0f;
        if (hx > Wf - 1.0f) hx = Wf - 1.0f;
        if (hy > Hf - 1.0f) hy = Hf - 1.0f;
        if (!(lx <= hx && ly <= hy)) return;
        q->px0 = (int32_t)lx; q->px1 = (int32_t)hx;
        q->py0 = (int32_t)ly; q->py1 = (int32_t)hy;
        q->thr = o->cutoff * o->cutoff;
        q->ewa = 1;
        q->visible = 1;
    } else {
        /* isotropic screen-space Gaussian, dilated and cut at `cutoff` sigma */
        float s2 = radius * radius + o->dilation;
        float Rc = o->cutoff * sqrtf(s2);
        float xs = u - 0.5f, ys = v - 0.5f;
        float lx = ceilf(xs - Rc), hx = floorf(xs + Rc);
        float ly = ceilf(ys - Rc), hy = floorf(ys + Rc);
        if (lx < 0.0f) lx = 0.0f;
        if (ly < 0.0f) ly = 0.0f;
        if (hx > Wf - 1.0f) hx = Wf - 1.0f;
        if (hy > Hf - 1.0f) hy = Hf - 1.0f;
        if (!(lx <= hx && ly <= hy)) return;
        q->px0 = (int32_t)lx; q->px1 = (int32_t)hx;
        q->py0 = (int32_t)ly; q->py1 = (int32_t)hy;
        q->s2 = s2;
        q->thr = (o->cutoff * o->cutoff) * s2;
        q->visible = 1;
    }
}

/* Is pixel (px, py) of a visible Gaussian point a fragment?  FP32.
 * Screen-space: d2 = dx^2 + dy^2 against cutoff^2 s2; world-space (EWA):
 * the Mahalanobis distance d2 = A dx^2 + 2 B dx dy + C dy^2 against
 * cutoff^2. */
static int gauss_frag(const opoint_t* q, int px, int py, float* d2_out) {
    float dx = ((float)px + 0.5f) - q->u;
    float dy = ((float)py + 0.5f) - q->v;
    float d2;
    if (!q->ewa)
        d2 = dx * dx + dy * dy;
    else
        d2 = (q->ca * (dx * dx) + (2.0f * q->cb) * (dx * dy)) + q->cc * (dy * dy);
    *d2_out = d2;
    return d2 <= q->thr;
}

int oracle_project(const ocam_t* cam, const oopts_t* o, int64_t n, const float* pos,
                   const float* radius, uint8_t* visible, float* uv, uint32_t* key,
                   float* xyz, int32_t* rect, uint32_t* ntiles) {
    const int T = o->tile;
    for (int64_t i = 0; i < n; ++i) {
        opoint_t q;
        decide_point(cam, o, pos + 3 * i, radius ? radius[i] : 0.0f, &q);
        visible[i] = (uint8_t)q.visible;
        uv[2 * i] = q.u; uv[2 * i + 1] = q.v;
        key[i] = q.key;
        xyz[3 * i] = q.X; xyz[3 * i + 1] = q.Y; xyz[3 * i + 2] = q.Z;
        rect[4 * i] = q.px0; rect[4 * i + 1] = q.py0;
        rect[4 * i + 2] = q.px1; rect[4 * i + 3] = q.py1;
        ntiles[i] = q.visible ? (uint32_t)((q.px1 / T - q.px0 / T + 1) * (q.py1 / T - q.py0 / T + 1)) : 0u;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Per-tile lists (Sec. 3.2 "Tiled Rendering"): the visible points whose */
/* footprint meets the tile, ordered by (depth key, point index).        */
/* ------------------------------------------------------------------ */

typedef struct { uint32_t key, idx; } okey_t;

static int cmp_okey(const void* pa, const void* pb) {
    const okey_t* a = (const okey_t*)pa;
    const okey_t* b = (const okey_t*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* counts[nt]; list must hold sum(counts) entries (call once with list=NULL
 * to get the counts and the total). Returns the total number of entries. */
int64_t oracle_tile_lists(const ocam_t* cam, const oopts_t* o, int64_t n, const float* pos,
                          const float* radius, uint32_t* counts, uint32_t* list) {
    const int T = o->tile;
    const int ntx = (cam->width + T - 1) / T, nty = (cam->height + T - 1) / T;
    const int64_t nt = (int64_t)ntx * nty;
    opoint_t* pts = (opoint_t*)malloc(sizeof(opoint_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) decide_point(cam, o, pos + 3 * i, radius ? radius[i] : 0.0f, &pts[i]);
    memset(counts, 0, sizeof(uint32_t) * (size_t)nt);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!pts[i].visible) continue;
        for (int ty = pts[i].py0 / T; ty <= pts[i].py1 / T; ++ty)
            for (int tx = pts[i].px0 / T; tx <= pts[i].px1 / T; ++tx) {
                counts[(int64_t)ty * ntx + tx]++;
                total++;
            }
    }
    if (list) {
        int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt + 1));
        start[0] = 0;
        for (int64_t t = 0; t < nt; ++t) start[t + 1] = start[t] + counts[t];
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt);
        memcpy(fill, start, sizeof(int64_t) * (size_t)nt);
        okey_t* ent = (okey_t*)malloc(sizeof(okey_t) * (size_t)(total > 0 ? total : 1));
        for (int64_t i = 0; i < n; ++i) {
            if (!pts[i].visible) continue;
            for (int ty = pts[i].py0 / T; ty <= pts[i].py1 / T; ++ty)
                for (int tx = pts[i].px0 / T; tx <= pts[i].px1 / T; ++tx) {
                    int64_t t = (int64_t)ty * ntx + tx;
                    ent[fill[t]].key = pts[i].key;
                    ent[fill[t]].idx = (uint32_t)i;
                    fill[t]++;
                }
        }
        for (int64_t t = 0; t < nt; ++t)
            qsort(ent + start[t], (size_t)counts[t], sizeof(okey_t), cmp_okey);
        for (int64_t k = 0; k < total; ++k) list[k] = ent[k].idx;
        free(ent); free(fill); free(start);
    }
    free(pts);
    return total;
}

/* ------------------------------------------------------------------ */
/* Fragments and the per-pixel blend                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t pixel;
    uint32_t key, idx;
    int32_t corner;  /* bilinear: 0 (x0,y0), 1 (x0+1,y0), 2 (x0,y0+1), 3 (x0+1,y0+1); Gaussian: -1 */
    float w32;       /* FP32 weight (bilinear decisions) */
    double w;        /* FP64 weight */
    double dw_du, dw_dv;
    double dw_dz;    /* EWA: through the covariance's dependence on Z at fixed u, v */
    /* filled by the blend */
    double Ta;       /* T_k * a_k of this fragment */
    double da;       /* dL/da_k */
    double da_abs;   /* magnitude bound of the terms in dL/da_k */
    int blended;
} ofrag_t;

typedef struct {
    int64_t nfrag;
    ofrag_t* frag;      /* point-major */
    int64_t* order;     /* fragment indices sorted by (pixel, key, idx) */
    int64_t* pix_start; /* [P + 1] */
    int64_t* pt_start;  /* [n + 1] */
    opoint_t* pts;
} oscene_t;

static const oscene_t* g_sort_ctx;

static int cmp_frag(const void* pa, const void* pb) {
    const ofrag_t* a = &g_sort_ctx->frag[*(const int64_t*)pa];
    const ofrag_t* b = &g_sort_ctx->frag[*(const int64_t*)pb];
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Fragments of every visible point; with a pixel mask, only those on
 * masked pixels (a sampled subset of the image, for scenes whose full
 * fragment set would not fit in memory: each kept pixel's list is still
 * complete, so its blend is exact). */
static int keep_pixel(const uint8_t* mask, int64_t pixel) { return !mask || mask[pixel]; }

/* World-space Gaussian fragment: w = exp(-d2 / 2) with the conic computed in
 * FP64 from the FP32 u, v, Z, and dw/du, dw/dv (through the offset and the
 * covariance) and dw/dZ (through the covariance at fixed u, v). */
static void ewa_weight(const ocam_t* cam, const oopts_t* o, const opoint_t* q, double dx,
                       double dy, ofrag_t* g) {
    const double fx = cam->fx, fy = cam->fy, Z = q->Z;
    const double xh = ((double)q->u - cam->cx) / fx, yh = ((double)q->v - cam->cy) / fy;
    const double jx = fx / Z, jy = fy / Z, s = (double)o->ewa_sigma * o->ewa_sigma;
    const double dil = o->dilation;
    const double a = s * jx * jx * (1.0 + xh * xh) + dil;
    const double b = s * jx * jy * xh * yh;
    const double c = s * jy * jy * (1.0 + yh * yh) + dil;
    const double det = a * c - b * b, inv = 1.0 / det, inv2 = inv * inv;
    const double A = c * inv, B = -b * inv, C = a * inv;
    const double d2 = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy;
    const double w = exp(-0.5 * d2);
    g->w = w;
    g->w32 = (float)w;
    /* through the offsets dx = px + 1/2 - u, dy = py + 1/2 - v */
    double du = w * (A * dx + B * dy), dv = w * (B * dx + C * dy);
    /* through the conic */
    const double gA = -0.5 * w * dx * dx, gB = -w * dx * dy, gC = -0.5 * w * dy * dy;
    const double ga = gA * (-c * c * inv2) + gB * (b * c * inv2) + gC * (-b * b * inv2);
    const double gb = gA * (2.0 * b * c * inv2) + gB * (-(a * c + b * b) * inv2) +
                      gC * (2.0 * a * b * inv2);
    const double gc = gA * (-b * b * inv2) + gB * (a * b * inv2) + gC * (-a * a * inv2);
    /* covariance entries as functions of u, v (through xh, yh) and Z (through jx, jy) */
    du += ga * (s * jx * jx * 2.0 * xh / fx) + gb * (s * jx * jy * yh / fx);
    dv += gb * (s * jx * jy * xh / fy) + gc * (s * jy * jy * 2.0 * yh / fy);
    g->dw_du = du;
    g->dw_dv = dv;
    g->dw_dz = ga * (-2.0 * s * jx * jx * (1.0 + xh * xh) / Z) +
               gb * (-2.0 * s * jx * jy * xh * yh / Z) +
               gc * (-2.0 * s * jy * jy * (1.0 + yh * yh) / Z);
}

static void build_fragments(const ocam_t* cam, const oopts_t* o, int64_t n, const float* pos,
                            const float* radius, const uint8_t* mask, oscene_t* s) {
    const int W = cam->width, H = cam->height;
    const int64_t P = (int64_t)W * H;
    s->pts = (opoint_t*)malloc(sizeof(opoint_t) * (size_t)(n > 0 ? n : 1));
    s->pt_start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        decide_point(cam, o, pos + 3 * i, radius ? radius[i] : 0.0f, &s->pts[i]);
        const opoint_t* q = &s->pts[i];
        s->pt_start[i] = cnt;
        if (!q->visible) continue;
        if (o->splat == 0) {
            for (int py = q->py0; py <= q->py1; ++py)
                for (int px = q->px0; px <= q->px1; ++px)
                    cnt += keep_pixel(mask, (int64_t)py * W + px);
        } else {
            for (int py = q->py0; py <= q->py1; ++py)
                for (int px = q->px0; px <= q->px1; ++px) {
                    float d2;
                    if (!keep_pixel(mask, (int64_t)py * W + px)) continue;
                    cnt += gauss_frag(q, px, py, &d2);
                }
        }
    }
    s->pt_start[n] = cnt;
    s->nfrag = cnt;
    s->frag = (ofrag_t*)calloc((size_t)(cnt > 0 ? cnt : 1), sizeof(ofrag_t));
    for (int64_t i = 0; i < n; ++i) {
        const opoint_t* q = &s->pts[i];
        if (!q->visible) continue;
        int64_t f = s->pt_start[i];
        if (o->splat == 0) {
            /* bilinear weights (Sec. 3.2: the four weights sum to one) */
            const double a = q->a, b = q->b;
            for (int c = 0; c < 4; ++c) {
                int dx = c & 1, dy = c >> 1;
                int px = q->x0 + dx, py = q->y0 + dy;
                if (px < 0 || px >= W || py < 0 || py >= H) continue;
                if (!keep_pixel(mask, (int64_t)py * W + px)) continue;
                ofrag_t* g = &s->frag[f++];
                g->pixel = (int64_t)py * W + px;
                g->key = q->key;
                g->idx = (uint32_t)i;
                g->corner = c;
                float wx32 = dx ? q->a : 1.0f - q->a;
                float wy32 = dy ? q->b : 1.0f - q->b;
                g->w32 = wx32 * wy32;
                double wx = dx ? a : 1.0 - a, wy = dy ? b : 1.0 - b;
                g->w = wx * wy;
                g->dw_du = (dx ? 1.0 : -1.0) * wy;
                g->dw_dv = (dy ? 1.0 : -1.0) * wx;
            }
        } else {
            for (int py = q->py0; py <= q->py1; ++py)
                for (int px = q->px0; px <= q->px1; ++px) {
                    float d2;
                    if (!keep_pixel(mask, (int64_t)py * W + px)) continue;
                    if (!gauss_frag(q, px, py, &d2)) continue;
                    ofrag_t* g = &s->frag[f++];
                    g->pixel = (int64_t)py * W + px;
                    g->key = q->key;
                    g->idx = (uint32_t)i;
                    g->corner = -1;
                    double dx = ((double)px + 0.5) - (double)q->u;
                    double dy = ((double)py + 0.5) - (double)q->v;
                    if (o->splat == 1) {
                        /* weight exp(-d^2 / (2 s2)); derivatives w.r.t. u, v */
                        double s2 = (double)q->s2;
                        double w = exp(-0.5 * (dx * dx + dy * dy) / s2);
                        g->w = w;
                        g->w32 = (float)w;
                        g->dw_du = w * dx / s2;
                        g->dw_dv = w * dy / s2;
                    } else {
                        ewa_weight(cam, o, q, dx, dy, g);
                    }
                }
        }
    }
    /* counting sort by pixel, then (key, idx) inside each pixel */
    s->pix_start = (int64_t*)calloc((size_t)(P + 1), sizeof(int64_t));
    for (int64_t f = 0; f < cnt; ++f) s->pix_start[s->frag[f].pixel + 1]++;
    for (int64_t p = 0; p < P; ++p) s->pix_start[p + 1] += s->pix_start[p];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
    memcpy(fill, s->pix_start, sizeof(int64_t) * (size_t)P);
    s->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t f = 0; f < cnt; ++f) s->order[fill[s->frag[f].pixel]++] = f;
    free(fill);
    g_sort_ctx = s;
    for (int64_t p = 0; p < P; ++p) {
        int64_t m = s->pix_start[p + 1] - s->pix_start[p];
        if (m > 1) qsort(s->order + s->pix_start[p], (size_t)m, sizeof(int64_t), cmp_frag);
    }
}

static void free_scene(oscene_t* s) {
    free(s->pts); free(s->pt_start); free(s->frag); free(s->order); free(s->pix_start);
}

/*
 * Forward (and optionally backward) render.
 *
 * feat:    [n][C] double (features upcast exactly by the caller)
 * opacity: [n] float
 * bg:      [C] double or NULL (constant background features), or with
 *          bg_image set a per-pixel background [C][H][W] (grad_bg then
 *          [C][H][W] too: T_final G per pixel)
 * Forward outputs:  out [C][H][W], out_abs [C][H][W] (sum of |terms|),
 *                   t_final [H][W], n_contrib [H][W], flags [H][W]
 *                   (Gaussian: 1 where the FP64 transmittance at a
 *                   termination decision lies within 1e-4 relative of t_min)
 * Backward inputs:  grad_out [C][H][W] (NULL = forward only), grad_t [H][W] or NULL
 * Backward outputs: grad_feat [n][C], grad_opacity [n], grad_uv [n][2],
 *                   grad_pos [n][3], grad_bg [C] (if bg), and the matching
 *                   *_abs magnitude bounds (same shapes).
 * grad_z, grad_z_abs: [n] or NULL; world-space Gaussians: dL/dZ through the
 *                   projected covariance at fixed (u, v) (grad_pos includes it)
 * pixel_mask:       [H][W] or NULL: forward only, computes the masked pixels
 *                   (the others are left as zero); -1 if combined with a
 *                   backward pass.
 */
int oracle_render(const ocam_t* cam, const oopts_t* o, int64_t n, const float* pos,
                  const float* radius, const float* opacity, const double* feat, int32_t C,
                  const double* bg, double* out, double* out_abs, double* t_final,
                  uint32_t* n_contrib, uint8_t* flags, const float* grad_out,
                  const float* grad_t, double* grad_feat, double* grad_opacity,
                  double* grad_uv, double* grad_pos, double* grad_bg,
                  double* grad_feat_abs, double* grad_opacity_abs, double* grad_uv_abs,
                  double* grad_pos_abs, const uint8_t* pixel_mask, int32_t bg_image,
                  double* grad_z, double* grad_z_abs) {
    const int W = cam->width, H = cam->height;
    const int64_t P = (int64_t)W * H;
    if (pixel_mask && grad_out) return -1;
    oscene_t s;
    memset(&s, 0, sizeof(s));
    build_fragments(cam, o, n, pos, radius, pixel_mask, &s);
    const float t_min = o->t_min;
    const int do_bwd = grad_out != NULL;

#pragma omp parallel
    {
        double* F = (double*)malloc(sizeof(double) * (size_t)C);
        double* Fa = (double*)malloc(sizeof(double) * (size_t)C);
        double* B = (double*)malloc(sizeof(double) * (size_t)C);
        double* Ba = (double*)malloc(sizeof(double) * (size_t)C);
        double* Tk = NULL;
        int64_t tk_cap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < P; ++p) {
            if (!keep_pixel(pixel_mask, p)) continue;
            const int64_t s0 = s.pix_start[p], s1 = s.pix_start[p + 1];
            if (s1 - s0 > tk_cap) {
                tk_cap = (s1 - s0) * 2;
                free(Tk);
                Tk = (double*)malloc(sizeof(double) * (size_t)tk_cap);
            }
            for (int c = 0; c < C; ++c) { F[c] = 0.0; Fa[c] = 0.0; }
            double T = 1.0;
            float T32 = 1.0f;
            uint32_t cnt = 0;
            uint8_t flag = 0;
            /* Eq. (1): front to back */
            for (int64_t k = s0; k < s1; ++k) {
                ofrag_t* g = &s.frag[s.order[k]];
                const float o32 = opacity[g->idx];
                if (o->splat == 0) {
                    if (T32 < t_min) break;
                } else {
                    if (t_min > 0.0f && fabs(T - (double)t_min) <= 1e-4 * (double)t_min) flag = 1;
                    if (T < (double)t_min) break;
                }
                const double a = (double)o32 * g->w;
                const double* f = feat + (int64_t)g->idx * C;
                for (int c = 0; c < C; ++c) {
                    F[c] += T * a * f[c];
                    Fa[c] += fabs(T * a * f[c]);
                }
                Tk[k - s0] = T;
                g->Ta = T * a;
                g->blended = 1;
                T *= (1.0 - a);
                T32 = T32 * (1.0f - o32 * g->w32);
                cnt++;
            }
            for (int c = 0; c < C; ++c) {
                double bgc = bg ? (bg_image ? bg[(int64_t)c * P + p] : bg[c]) : 0.0;
                out[(int64_t)c * P + p] = F[c] + T * bgc;
                out_abs[(int64_t)c * P + p] = Fa[c] + fabs(T * bgc);
            }
            t_final[p] = T;
            n_contrib[p] = cnt;
            if (flags) flags[p] = flag;
            if (!do_bwd) continue;
            /* Eq. (2), back to front: B is the blend of everything behind
             * fragment k (including the background), Pi the transmittance
             * through it. */
            double G_T = grad_t ? (double)grad_t[p] : 0.0;
            double Pi = 1.0;
            for (int c = 0; c < C; ++c) {
                B[c] = bg ? (bg_image ? bg[(int64_t)c * P + p] : bg[c]) : 0.0;
                Ba[c] = fabs(B[c]);
            }
            for (int64_t k = s0 + (int64_t)cnt - 1; k >= s0; --k) {
                ofrag_t* g = &s.frag[s.order[k]];
                const double o64 = (double)opacity[g->idx];
                const double a = o64 * g->w;
                const double* f = feat + (int64_t)g->idx * C;
                double gf = 0.0, gB = 0.0, gf_abs = 0.0, gB_abs = 0.0;
                for (int c = 0; c < C; ++c) {
                    double Gc = (double)grad_out[(int64_t)c * P + p];
                    gf += Gc * f[c];
                    gB += Gc * B[c];
                    gf_abs += fabs(Gc * f[c]);
                    gB_abs += fabs(Gc) * Ba[c];
                }
                const double Tkk = Tk[k - s0];
                g->da = Tkk * (gf - gB) - G_T * Tkk * Pi;
                g->da_abs = Tkk * (gf_abs + gB_abs) + fabs(G_T) * Tkk * Pi;
                for (int c = 0; c < C; ++c) {
                    B[c] = a * f[c] + (1.0 - a) * B[c];
                    Ba[c] = a * fabs(f[c]) + (1.0 - a) * Ba[c];
                }
                Pi *= (1.0 - a);
            }
        }
        free(F); free(Fa); free(B); free(Ba); free(Tk);
    }

    if (do_bwd) {
        /* gather the per-fragment terms per point (point-major fragments) */
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            double* gfe = grad_feat + i * C;
            double* gfa = grad_feat_abs + i * C;
            for (int c = 0; c < C; ++c) { gfe[c] = 0.0; gfa[c] = 0.0; }
            double go = 0.0, goa = 0.0, gu = 0.0, gv = 0.0, gua = 0.0, gva = 0.0;
            double gz = 0.0, gza = 0.0;
            const double o64 = (double)opacity[i];
            for (int64_t f = s.pt_start[i]; f < s.pt_start[i + 1]; ++f) {
                const ofrag_t* g = &s.frag[f];
                if (!g->blended) continue;
                for (int c = 0; c < C; ++c) {
                    double t = g->Ta * (double)grad_out[(int64_t)c * P + g->pixel];
                    gfe[c] += t;
                    gfa[c] += fabs(t);
                }
                go += g->w * g->da;
                goa += fabs(g->w) * g->da_abs;
                gu += o64 * g->dw_du * g->da;
                gv += o64 * g->dw_dv * g->da;
                gua += fabs(o64 * g->dw_du) * g->da_abs;
                gva += fabs(o64 * g->dw_dv) * g->da_abs;
                gz += o64 * g->dw_dz * g->da;
                gza += fabs(o64 * g->dw_dz) * g->da_abs;
            }
            if (grad_z) {
                grad_z[i] = gz;
                grad_z_abs[i] = gza;
            }
            grad_opacity[i] = go;
            grad_opacity_abs[i] = goa;
            grad_uv[2 * i] = gu; grad_uv[2 * i + 1] = gv;
            grad_uv_abs[2 * i] = gua; grad_uv_abs[2 * i + 1] = gva;
            /* chain through u = fx X/Z + cx, v = fy Y/Z + cy, X = R p + t */
            const opoint_t* q = &s.pts[i];
            double gp[3] = {0, 0, 0}, gpa[3] = {0, 0, 0};
            if (q->visible) {
                const float* R = cam->R;
                double px = pos[3 * i], py = pos[3 * i + 1], pz = pos[3 * i + 2];
                double X = R[0] * px + R[1] * py + R[2] * pz + cam->t[0];
                double Y = R[3] * px + R[4] * py + R[5] * pz + cam->t[1];
                double Z = R[6] * px + R[7] * py + R[8] * pz + cam->t[2];
                double fx = cam->fx, fy = cam->fy;
                double dX = gu * fx / Z, dY = gv * fy / Z;
                double dZ = gz - (gu * fx * X + gv * fy * Y) / (Z * Z);
                double aX = gua * fx / Z, aY = gva * fy / Z;
                double aZ = gza + (gua * fx * fabs(X) + gva * fy * fabs(Y)) / (Z * Z);
                for (int j = 0; j < 3; ++j) {
                    gp[j] = R[j] * dX + R[3 + j] * dY + R[6 + j] * dZ;
                    gpa[j] = fabs(R[j]) * aX + fabs(R[3 + j]) * aY + fabs(R[6 + j]) * aZ;
                }
            }
            for (int j = 0; j < 3; ++j) {
                grad_pos[3 * i + j] = gp[j];
                grad_pos_abs[3 * i + j] = gpa[j];
            }
        }
        if (grad_bg && bg_image) {
            /* dL/df_bg(pixel) = T_final G (Eq. (1) with the background term) */
            for (int c = 0; c < C; ++c)
                for (int64_t p = 0; p < P; ++p)
                    grad_bg[(int64_t)c * P + p] = t_final[p] * (double)grad_out[(int64_t)c * P + p];
        } else if (grad_bg) {
            for (int c = 0; c < C; ++c) {
                double acc = 0.0;
                for (int64_t p = 0; p < P; ++p)
                    acc += t_final[p] * (double)grad_out[(int64_t)c * P + p];
                grad_bg[c] = acc;
            }
        }
    }
    free_scene(&s);
    return 0;
}

/* Number of fragments (for sizing and statistics). */
int64_t oracle_count_fragments(const ocam_t* cam, const oopts_t* o, int64_t n, const float* pos,
                               const float* radius) {
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        opoint_t q;
        decide_point(cam, o, pos + 3 * i, radius ? radius[i] : 0.0f, &q);
        if (!q.visible) continue;
        if (o->splat == 0) {
            cnt += (int64_t)(q.px1 - q.px0 + 1) * (q.py1 - q.py0 + 1);
        } else {
            for (int py = q.py0; py <= q.py1; ++py)
                for (int px = q.px0; px <= q.px1; ++px) {
                    float d2;
                    cnt += gauss_frag(&q, px, py, &d2);
                }
        }
    }
    return cnt;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing only; results do not
   depend on it: every pixel is computed by one thread in a fixed order). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

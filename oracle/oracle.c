/*
 * CPU FP64 oracle for per-pixel ray casting of a deep-octree volumetric canvas.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU library.
 *
 * What it computes (the plain definition).  A canvas is an array of R^3 octree
 * roots (Sec. 4), each refined into 8 consecutive children (Sec. 4.1.1).  A
 * ray r(t) = o + t d leaves the eye of a pinhole view (Sec. 6.1, eye kept in
 * FP64).  Its leaf sequence is every leaf whose closed box meets the ray on an
 * interval of positive length inside the canvas chord [t0, t1], ordered by
 * entry t.  Front to back over that sequence (Sec. 6.2: accumulate until full
 * opacity or canvas exit) each leaf contributes an emission-absorption segment
 * of a piecewise-constant medium:  T' = T exp(-kappa l),  C += (T - T') c,
 * T = T', with l the segment length in units of the leaf edge (the cell-local
 * traversal length t_i of Sec. 6.2-6.3) and kappa the optical depth across one
 * leaf edge.  Output: premultiplied RGB = C and A = 1 - T.
 *
 * How (the algorithm, deliberately different from the GPU design): a restart
 * traversal in canvas-global FP64 coordinates.  From the current point it
 * descends from the root to the leaf that contains it, ties on a mid-plane
 * going to the side the ray moves into; the leaf box is exact in FP64; the
 * exit parameter is the smallest of the three candidate face planes; the next
 * point is the exit point with its exit coordinate snapped onto the face plane.
 * No neighbour links are used.
 *
 * Readings taken where the paper is silent:
 *  - compositing is the emission-absorption model above (the paper only says
 *    rays accumulate to full opacity), no shading, black background;
 *  - colours decode linearly (byte/255), kappa from IEEE half exactly;
 *  - alpha_stop >= 1 disables early termination; otherwise a ray stops after
 *    the segment where 1 - T >= alpha_stop;
 *  - pixel (x, y), row 0 at the top: u = (2(x+1/2)/W - 1) tan_x,
 *    v = (1 - 2(y+1/2)/H) tan_y, d = normalize(fwd + u right + v up);
 *  - positions are measured in root-edge units: q = (p_world - origin)/root_edge;
 *  - a ray is flagged "near a face" when an entry or exit point lies within
 *    eps_face (root units) of a face plane of that leaf other than the one it
 *    lies on; zero-length segments are dropped.
 *
 * Parity unpinned: the clamp in orc_trace that keeps a rounded exit point
 * from lying behind the entry point on a non-exit axis.  No ray of the pins
 * or of the workloads reaches it, so no pin fails without it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_LEAF 0x80000000u
#define ORC_NONE 0xffffffffu

#define ORC_FLAG_NEAR_FACE 1u
#define ORC_FLAG_TERM_AMBIG 2u
#define ORC_FLAG_STEP_CAP 4u
#define ORC_FLAG_BAD_POOL 8u

typedef struct {
  double origin[3];
  double root_edge;
  uint32_t R, max_depth, leaf_format; /* 0: RGBA8 + half kappa (8 B), 1: 4 doubles */
  uint32_t pad;
  const uint32_t* nodes; /* {child, parent} pairs */
  uint64_t n_nodes;
  const void* leaves;
  uint64_t n_leaves;
} orc_canvas;

typedef struct {
  int32_t canvas;
  uint32_t W, H;
  uint32_t pad;
  double eye[3], right[3], up[3], fwd[3];
  double tan_x, tan_y;
  uint64_t out_offset_px;
  double alpha_stop;
} orc_view;

typedef struct {
  double rgba[4];
  uint32_t flags;
  uint32_t n_leaves;      /* recorded (positive-length) segments */
  double chord;           /* t1 - t0 (root units), 0 on a miss */
  double sum_len;         /* sum of l * h over the segments (root units) */
  double alg_bytes;       /* algorithmic bytes of the neighbour-linked traversal */
  uint32_t n_outer;       /* transitions through a face on the parent's boundary */
  uint32_t n_descent;     /* levels descended: depth of the first leaf + increases */
} orc_result;

/* --- small helpers ------------------------------------------------------ */

static double half_to_double(uint16_t h) {
  int s = (h >> 15) & 1, e = (h >> 10) & 0x1f, m = h & 0x3ff;
  double v;
  if (e == 0)
    v = ldexp((double)m, -24);
  else if (e == 31)
    v = m ? NAN : INFINITY;
  else
    v = ldexp((double)(m + 1024), e - 25);
  return s ? -v : v;
}

static void leaf_payload(const orc_canvas* cv, uint32_t li, double c[3], double* kappa) {
  if (cv->leaf_format == 1) {
    const double* p = (const double*)cv->leaves + 4 * (uint64_t)li;
    c[0] = p[0];
    c[1] = p[1];
    c[2] = p[2];
    *kappa = p[3];
  } else {
    const uint8_t* p = (const uint8_t*)cv->leaves + 8 * (uint64_t)li;
    uint16_t h;
    memcpy(&h, p + 4, 2);
    c[0] = (double)p[0] / 255.0;
    c[1] = (double)p[1] / 255.0;
    c[2] = (double)p[2] / 255.0;
    *kappa = half_to_double(h);
  }
}

/* Ray direction of pixel (x, y): pinhole model, row 0 at the top. */
void orc_ray_dir(const orc_view* v, uint32_t x, uint32_t y, double d[3]) {
  double u = (2.0 * ((double)x + 0.5) / (double)v->W - 1.0) * v->tan_x;
  double w = (1.0 - 2.0 * ((double)y + 0.5) / (double)v->H) * v->tan_y;
  double n2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    d[k] = v->fwd[k] + u * v->right[k];
    d[k] = d[k] + w * v->up[k];
    n2 += d[k] * d[k];
  }
  double n = sqrt(n2);
  for (int k = 0; k < 3; ++k) d[k] = d[k] / n;
}

/* Canvas entry and exit of the ray o + t d (root units) by the slab test
 * against [0, R]^3 (the chord of Sec. 6.1's full-precision start point).
 * Returns 0 for a ray parallel to an axis and outside the canvas on it; else
 * 1 with the slab parameters tin (-inf if none), tout, the axis kin and side
 * of the entry face (kin = -1 when no slab bounds t from below). */
static int canvas_slabs(const double o[3], const double d[3], double Rd, double* tin_out,
                        double* tout_out, int* kin_out, int* side_out) {
  double tin = -INFINITY, tout = INFINITY;
  int kin = -1, sin_side = 0;
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0) {
      double ta = (0.0 - o[k]) / d[k], tb = (Rd - o[k]) / d[k];
      double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
      if (lo > tin) {
        tin = lo;
        kin = k;
        sin_side = d[k] > 0.0 ? 0 : 1;
      }
      if (hi < tout) tout = hi;
    } else if (o[k] < 0.0 || o[k] > Rd) {
      return 0; /* parallel and outside: miss */
    }
  }
  *tin_out = tin;
  *tout_out = tout;
  *kin_out = kin;
  *side_out = sin_side;
  return 1;
}

/* Pixel directions and canvas chords of the listed pixels of view v over
 * canvas cv (the set-up of orc_trace, for the precision experiment's exact
 * rays): d_out (3 per ray) the unit direction, t_out (2 per ray) the chord
 * [t0, t1] in root-edge units along d, t0 = max(entry, 0); t0 = t1 = 0 for a
 * miss. */
void orc_ray_setup(const orc_canvas* cv, const orc_view* v, const uint64_t* px, uint64_t n,
                   double* d_out, double* t_out) {
  for (uint64_t i = 0; i < n; ++i) {
    double* d = d_out + 3 * i;
    orc_ray_dir(v, (uint32_t)(px[i] % v->W), (uint32_t)(px[i] / v->W), d);
    double o[3], tin, tout;
    int kin, side;
    for (int k = 0; k < 3; ++k) o[k] = (v->eye[k] - cv->origin[k]) / cv->root_edge;
    t_out[2 * i] = t_out[2 * i + 1] = 0.0;
    if (!canvas_slabs(o, d, (double)cv->R, &tin, &tout, &kin, &side)) continue;
    double t0 = tin > 0.0 ? tin : 0.0;
    if (!(t0 < tout)) continue;
    t_out[2 * i] = t0;
    t_out[2 * i + 1] = tout;
  }
}

/* Locate the leaf containing point q (root units) by descending from the root
 * array.  On a mid-plane the child on the side the ray moves into is taken. */
static int locate(const orc_canvas* cv, const double q[3], const double d[3], uint32_t* node,
                  uint32_t* depth, int64_t c[3]) {
  const int64_t R = cv->R;
  int64_t r[3];
  for (int k = 0; k < 3; ++k) {
    double f = floor(q[k]);
    int64_t n = (int64_t)f;
    if (q[k] == f && !(d[k] > 0.0)) n -= 1;
    if (n < 0) n = 0;
    if (n > R - 1) n = R - 1;
    r[k] = n;
  }
  uint32_t I = (uint32_t)(r[0] + R * (r[1] + R * r[2]));
  uint32_t dep = 0;
  c[0] = r[0];
  c[1] = r[1];
  c[2] = r[2];
  for (;;) {
    if ((uint64_t)I >= cv->n_nodes) return -1;
    uint32_t ch = cv->nodes[2 * (uint64_t)I];
    if (ch & ORC_LEAF) break;
    if (dep >= 60) return -1;
    double h = ldexp(1.0, -(int)dep);
    uint32_t oct = 0;
    for (int k = 0; k < 3; ++k) {
      double mid = ((double)c[k] + 0.5) * h;
      int b = (q[k] > mid) || (q[k] == mid && d[k] > 0.0);
      oct |= (uint32_t)b << k;
      c[k] = 2 * c[k] + b;
    }
    I = ch + oct;
    ++dep;
  }
  *node = I;
  *depth = dep;
  return 0;
}

/* Trace one ray.  o_world, d: FP64 eye and unit direction in world units.
 * Optional trace buffers receive up to max_leaves recorded segments. */
int orc_trace(const orc_canvas* cv, const double o_world[3], const double d[3], double alpha_stop,
              double eps_face, uint32_t max_leaves, uint32_t* tr_node, double* tr_len,
              uint8_t* tr_depth, orc_result* res) {
  memset(res, 0, sizeof(*res));
  res->alg_bytes = 16.0; /* a miss still writes its pixel */
  const double Rd = (double)cv->R;
  double o[3];
  for (int k = 0; k < 3; ++k) o[k] = (o_world[k] - cv->origin[k]) / cv->root_edge;

  /* canvas entry: slab test against [0, R]^3 */
  double tin, tout;
  int kin, sin_side;
  if (!canvas_slabs(o, d, Rd, &tin, &tout, &kin, &sin_side)) return 0; /* parallel, outside */
  double t0 = tin > 0.0 ? tin : 0.0, t1 = tout;
  if (!(t0 < t1)) return 0;
  res->chord = t1 - t0;

  double q[3];
  for (int k = 0; k < 3; ++k) q[k] = o[k] + t0 * d[k];
  int ent_axis = -1, ent_side = 0;
  if (tin > 0.0) {
    q[kin] = sin_side ? Rd : 0.0;
    ent_axis = kin;
    ent_side = sin_side;
  }
  for (int k = 0; k < 3; ++k) {
    if (q[k] < 0.0) q[k] = 0.0;
    if (q[k] > Rd) q[k] = Rd;
  }

  double T = 1.0, C[3] = {0.0, 0.0, 0.0};
  double t = t0;
  const int use_stop = alpha_stop < 1.0;
  uint64_t cap = 3ull * (uint64_t)cv->R * ((uint64_t)1 << (cv->max_depth < 40 ? cv->max_depth : 40)) + 16;
  uint32_t prev_depth = 0, prev_outer = 0;
  int have_prev = 0;
  for (uint64_t step = 0;; ++step) {
    if (step > cap) {
      res->flags |= ORC_FLAG_STEP_CAP;
      break;
    }
    uint32_t I, dep;
    int64_t c[3];
    if (locate(cv, q, d, &I, &dep, c) != 0) {
      res->flags |= ORC_FLAG_BAD_POOL;
      break;
    }
    uint32_t li = cv->nodes[2 * (uint64_t)I] & ~ORC_LEAF;
    if ((uint64_t)li >= cv->n_leaves) {
      res->flags |= ORC_FLAG_BAD_POOL;
      break;
    }
    double h = ldexp(1.0, -(int)dep);
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = (double)c[k] * h;
      hi[k] = (double)(c[k] + 1) * h;
    }
    /* exit: nearest of the three candidate face planes */
    double tex = INFINITY;
    int kx = -1;
    for (int k = 0; k < 3; ++k) {
      if (d[k] == 0.0) continue;
      double X = d[k] > 0.0 ? hi[k] : lo[k];
      double tk = (X - o[k]) / d[k];
      if (tk < tex) {
        tex = tk;
        kx = k;
      }
    }
    if (kx < 0) {
      res->flags |= ORC_FLAG_BAD_POOL;
      break;
    }
    /* exit point; on the non-exit axes it is kept inside the leaf box and never
     * behind the entry point, so rounding cannot send the ray backwards */
    double qx[3];
    for (int k = 0; k < 3; ++k) {
      qx[k] = o[k] + tex * d[k];
      if (d[k] > 0.0 && qx[k] < q[k]) qx[k] = q[k];
      if (d[k] < 0.0 && qx[k] > q[k]) qx[k] = q[k];
      if (qx[k] < lo[k]) qx[k] = lo[k];
      if (qx[k] > hi[k]) qx[k] = hi[k];
    }
    qx[kx] = d[kx] > 0.0 ? hi[kx] : lo[kx];

    /* near-face flag on the entry and exit points */
    for (int k = 0; k < 3; ++k) {
      for (int s = 0; s < 2; ++s) {
        double P = s ? hi[k] : lo[k];
        if (!(k == ent_axis && s == ent_side) && fabs(q[k] - P) < eps_face)
          res->flags |= ORC_FLAG_NEAR_FACE;
        int xs = d[kx] > 0.0 ? 1 : 0;
        if (!(k == kx && s == xs) && fabs(qx[k] - P) < eps_face) res->flags |= ORC_FLAG_NEAR_FACE;
      }
    }

    double len = (tex - t) / h;
    if (len > 0.0) {
      double col[3], kap;
      leaf_payload(cv, li, col, &kap);
      double Tn = T * exp(-kap * len);
      for (int k = 0; k < 3; ++k) C[k] += (T - Tn) * col[k];
      T = Tn;
      uint32_t n = res->n_leaves;
      if (n < max_leaves) {
        if (tr_node) tr_node[n] = I;
        if (tr_len) tr_len[n] = len;
        if (tr_depth) tr_depth[n] = (uint8_t)dep;
      }
      res->n_leaves = n + 1;
      res->sum_len += len * h;
      /* algorithmic bytes: 8 per leaf payload, 4 per link or level read */
      if (!have_prev) {
        res->n_descent += dep;
      } else {
        res->n_outer += prev_outer;
        if (dep > prev_depth) res->n_descent += dep - prev_depth;
      }
      have_prev = 1;
      prev_depth = dep;
      int bit = (int)(c[kx] & 1);
      int inner = dep > 0 && bit == (d[kx] > 0.0 ? 0 : 1);
      prev_outer = inner ? 0u : 1u;
      if (use_stop && fabs((1.0 - T) - alpha_stop) < 1e-5) res->flags |= ORC_FLAG_TERM_AMBIG;
      if (use_stop && 1.0 - T >= alpha_stop) break;
    }

    /* canvas exit? */
    double Xe = qx[kx];
    if ((d[kx] > 0.0 && Xe >= Rd) || (d[kx] < 0.0 && Xe <= 0.0)) break;
    if (tex > t) t = tex;
    for (int k = 0; k < 3; ++k) q[k] = qx[k];
    ent_axis = kx;
    ent_side = d[kx] > 0.0 ? 0 : 1;
  }
  res->rgba[0] = C[0];
  res->rgba[1] = C[1];
  res->rgba[2] = C[2];
  res->rgba[3] = 1.0 - T;
  res->alg_bytes = 16.0 + 8.0 * res->n_leaves + 4.0 * (double)(res->n_outer + res->n_descent);
  return 0;
}

/* --- multi-threaded driver ---------------------------------------------- */

typedef struct {
  const orc_canvas* canvases;
  int n_canvases;
  const orc_view* views;
  int n_views;
  const uint64_t* ray_ids; /* (view << 32) | pixel, or NULL for all pixels */
  uint64_t n_rays;
  const uint64_t* view_first_ray; /* prefix of W*H when ray_ids == NULL */
  double eps_face;
  uint32_t max_leaves;
  double* rgba;      /* 4 per ray */
  uint32_t* flags;   /* per ray */
  uint32_t* n_leaves;
  double* alg_bytes;
  double* chord;
  double* sum_len;
  uint32_t* tr_node; /* max_leaves per ray, or NULL */
  double* tr_len;
  uint8_t* tr_depth;
  uint64_t next;
  pthread_mutex_t mu;
} orc_job;

static void* orc_worker(void* arg) {
  orc_job* J = (orc_job*)arg;
  const uint64_t chunk = 256;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    uint64_t b = J->next;
    J->next += chunk;
    pthread_mutex_unlock(&J->mu);
    if (b >= J->n_rays) break;
    uint64_t e = b + chunk < J->n_rays ? b + chunk : J->n_rays;
    for (uint64_t i = b; i < e; ++i) {
      uint32_t vi, px;
      if (J->ray_ids) {
        vi = (uint32_t)(J->ray_ids[i] >> 32);
        px = (uint32_t)(J->ray_ids[i] & 0xffffffffu);
      } else {
        int lo = 0, hi = J->n_views - 1;
        while (lo < hi) {
          int m = (lo + hi + 1) / 2;
          if (J->view_first_ray[m] <= i) lo = m; else hi = m - 1;
        }
        vi = (uint32_t)lo;
        px = (uint32_t)(i - J->view_first_ray[lo]);
      }
      orc_result r;
      memset(&r, 0, sizeof(r));
      if ((int)vi < J->n_views) {
        const orc_view* v = &J->views[vi];
        if (v->canvas >= 0 && v->canvas < J->n_canvases && px < v->W * v->H) {
          double d[3];
          orc_ray_dir(v, px % v->W, px / v->W, d);
          uint64_t mo = (uint64_t)J->max_leaves * i;
          orc_trace(&J->canvases[v->canvas], v->eye, d, v->alpha_stop, J->eps_face, J->max_leaves,
                    J->tr_node ? J->tr_node + mo : NULL, J->tr_len ? J->tr_len + mo : NULL,
                    J->tr_depth ? J->tr_depth + mo : NULL, &r);
        } else {
          r.flags = ORC_FLAG_BAD_POOL;
        }
      } else {
        r.flags = ORC_FLAG_BAD_POOL;
      }
      if (J->rgba) memcpy(J->rgba + 4 * i, r.rgba, 4 * sizeof(double));
      if (J->flags) J->flags[i] = r.flags;
      if (J->n_leaves) J->n_leaves[i] = r.n_leaves;
      if (J->alg_bytes) J->alg_bytes[i] = r.alg_bytes;
      if (J->chord) J->chord[i] = r.chord;
      if (J->sum_len) J->sum_len[i] = r.sum_len;
    }
  }
  return NULL;
}

/* Render a list of rays (or every pixel of every view when ray_ids is NULL,
 * in view order, row-major).  Outputs are per ray in list order. */
int orc_render(const orc_canvas* canvases, int n_canvases, const orc_view* views, int n_views,
               const uint64_t* ray_ids, uint64_t n_rays, double eps_face, uint32_t max_leaves,
               double* rgba, uint32_t* flags, uint32_t* n_leaves, double* alg_bytes,
               double* chord, double* sum_len, uint32_t* tr_node, double* tr_len,
               uint8_t* tr_depth, int n_threads) {
  orc_job J;
  memset(&J, 0, sizeof(J));
  J.canvases = canvases;
  J.n_canvases = n_canvases;
  J.views = views;
  J.n_views = n_views;
  J.ray_ids = ray_ids;
  J.n_rays = n_rays;
  J.eps_face = eps_face;
  J.max_leaves = max_leaves;
  J.rgba = rgba;
  J.flags = flags;
  J.n_leaves = n_leaves;
  J.alg_bytes = alg_bytes;
  J.chord = chord;
  J.sum_len = sum_len;
  J.tr_node = tr_node;
  J.tr_len = tr_len;
  J.tr_depth = tr_depth;
  uint64_t* first = NULL;
  if (!ray_ids) {
    first = (uint64_t*)calloc((size_t)n_views + 1, sizeof(uint64_t));
    if (!first) return -1;
    for (int v = 0; v < n_views; ++v) first[v + 1] = first[v] + (uint64_t)views[v].W * views[v].H;
    J.view_first_ray = first;
    if (J.n_rays > first[n_views]) J.n_rays = first[n_views];
  }
  pthread_mutex_init(&J.mu, NULL);
  if (n_threads < 1) n_threads = 1;
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  int started = 0;
  for (int i = 1; i < n_threads && th; ++i)
    if (pthread_create(&th[started], NULL, orc_worker, &J) == 0) ++started;
  orc_worker(&J);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  free(first);
  pthread_mutex_destroy(&J.mu);
  return 0;
}

double orc_half_to_double(uint16_t h) { return half_to_double(h); }

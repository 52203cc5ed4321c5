/*
 * Plain sequential CPU oracle for the two irregular wavefront propagation (IWPP)
 * instances of Teodoro et al., "Efficient Irregular Wavefront Propagation
 * Algorithms on Hybrid CPU-GPU Machines" (arXiv 1209.3314).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  It exists to check the GPU library, which
 * shares no code with it.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  Nothing here is tuned: every routine is the
 * slow, obviously-correct form of what the paper defines.
 *
 * Conventions shared by every routine:
 *   - images are row-major, h rows of w pixels, pixel index p = y*w + x;
 *   - pixels outside the image are not neighbours (the paper is silent on the
 *     border; this is the reading used throughout);
 *   - conn is 4 or 8 (the grid G of Sec. 2);
 *   - return value 0 on success, -1 on a bad argument, -2 on allocation failure.
 *
 * Morphological reconstruction (Sec. 2.1):
 *   oracle_mr_fh        rho_I(J) by a forward pass, a backward pass and a FIFO
 *                       relaxation (the Fast Hybrid schedule);
 *   oracle_mr_erode     the dual, reconstruction by erosion rho*_I(J), on the
 *                       same schedule with the comparisons reversed.
 * Euclidean distance transform (Sec. 2.2), targets ("features") are 0-pixels:
 *   oracle_edt_rounds   level-synchronous propagation, frontier form (the
 *                       round reading of Algorithms 3 and 6, see below);
 *   oracle_edt_dense    the same rounds as a dense Jacobi operator;
 *   oracle_edt_alg3     the sequential schedule: one FIFO, in place, strict
 *                       improvement (Algorithm 3's schedule);
 *   oracle_edt_exact_bf exact EDT by brute force over all features;
 *   oracle_edt_exact_sep exact squared EDT, separable lower-envelope method
 *                       (Meijster et al. 2000 / Felzenszwalb-Huttenlocher).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF64 INT64_MAX

/* Neighbour offsets (dy, dx).  The full neighbourhood N_G is listed in raster
 * order; the first half of the 8-neighbourhood (and of the 4-neighbourhood) is
 * N+ (visited before p by a raster scan), the second half is N- (Sec. 2.1,
 * definition of N+_G and N-_G under Algorithm 2). */
static const int NB8[8][2] = {{-1, -1}, {-1, 0}, {-1, 1}, {0, -1}, {0, 1}, {1, -1}, {1, 0}, {1, 1}};
static const int NB4[4][2] = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};

static int nb_count(int conn) { return conn == 8 ? 8 : 4; }
static const int (*nb_table(int conn))[2] { return conn == 8 ? NB8 : NB4; }

/* ------------------------------------------------------------------------- */
/* A growable FIFO of (index, depth) pairs.                                   */
typedef struct {
  int64_t* idx;
  int64_t* dep;
  int64_t cap, head, count;
} fifo_t;

static int fifo_init(fifo_t* f, int64_t cap) {
  if (cap < 16) cap = 16;
  f->idx = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
  f->dep = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
  f->cap = cap;
  f->head = 0;
  f->count = 0;
  return (f->idx && f->dep) ? 0 : -2;
}

static void fifo_free(fifo_t* f) {
  free(f->idx);
  free(f->dep);
}

static int fifo_push(fifo_t* f, int64_t i, int64_t d) {
  if (f->count == f->cap) {
    int64_t ncap = f->cap * 2;
    int64_t* ni = (int64_t*)malloc((size_t)ncap * sizeof(int64_t));
    int64_t* nd = (int64_t*)malloc((size_t)ncap * sizeof(int64_t));
    if (!ni || !nd) {
      free(ni);
      free(nd);
      return -2;
    }
    for (int64_t k = 0; k < f->count; ++k) {
      ni[k] = f->idx[(f->head + k) % f->cap];
      nd[k] = f->dep[(f->head + k) % f->cap];
    }
    free(f->idx);
    free(f->dep);
    f->idx = ni;
    f->dep = nd;
    f->cap = ncap;
    f->head = 0;
  }
  int64_t t = (f->head + f->count) % f->cap;
  f->idx[t] = i;
  f->dep[t] = d;
  f->count++;
  return 0;
}

static void fifo_pop(fifo_t* f, int64_t* i, int64_t* d) {
  *i = f->idx[f->head];
  *d = f->dep[f->head];
  f->head = (f->head + 1) % f->cap;
  f->count--;
}

static int bad_dims(int64_t h, int64_t w, int conn) {
  return h <= 0 || w <= 0 || (conn != 4 && conn != 8);
}

/* ------------------------------------------------------------------------- */
/* Queue-driven relaxation, shared by both instances.
 *
 * The IWPP of Sec. 2 in its plainest form: items wait in a FIFO; popping p
 * offers p's value to every in-image neighbour q of N_G; an offer that
 * improves q changes q, and q then waits in the FIFO as well.  What "offer"
 * and "improve" mean is the instance's business (`offer` returns nonzero when
 * it changed q).  Counts: pops, pushes, and the largest depth (an item pushed
 * by an item of depth d has depth d + 1; initial items have depth 0). */
typedef int (*offer_fn)(void* inst, int64_t p, int64_t q);

typedef struct {
  int64_t pops, pushes, maxdep;
} relax_counts;

static int relax_fifo(fifo_t* fq, int64_t h, int64_t w, int conn, offer_fn offer, void* inst, relax_counts* c) {
  const int nn = nb_count(conn);
  const int (*nb)[2] = nb_table(conn);
  while (fq->count > 0) {
    int64_t p, d;
    fifo_pop(fq, &p, &d);
    c->pops++;
    if (d > c->maxdep) c->maxdep = d;
    const int64_t y = p / w, x = p % w;
    for (int k = 0; k < nn; ++k) {
      const int64_t qy = y + nb[k][0], qx = x + nb[k][1];
      if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
      const int64_t q = qy * w + qx;
      if (!offer(inst, p, q)) continue;
      if (fifo_push(fq, q, d + 1)) return -2;
      c->pushes++;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Morphological reconstruction by dilation (Sec. 2.1).
 *
 * rho_I(J) is the limit of the elementary geodesic dilation
 *   J(p) <- max{J(q) : q in N_G(p) U {p}} ^ I(p)
 * and is unique: any order of elementary updates that reaches stability gives
 * it.  The order used here is the Fast Hybrid schedule the paper builds on:
 * one forward pass and one backward pass of the update restricted to the half
 * neighbourhoods (N+ for the forward pass, N- for the backward one), the
 * backward pass also collecting the pixels whose value can still travel to a
 * neighbour, then the queue relaxation above until nothing changes.
 *
 * Reading for a marker above the mask: the paper requires J <= I and is silent
 * otherwise; the marker is clamped first (J <- J ^ I).
 *
 * stats (may be NULL), 4 entries:
 *   [0] pixels queued by the backward pass (initial wavefront)
 *   [1] queue pops in the relaxation (the work count Q_ref)
 *   [2] queue pushes in the relaxation
 *   [3] largest depth reached (initial items have depth 0)
 */
typedef struct {
  uint8_t* J;
  const uint8_t* I;
} mr_inst;

/* p's value can raise q: J(q) < J(p) and q is below its mask. */
static int mr_can_raise(const mr_inst* m, int64_t p, int64_t q) { return m->J[q] < m->J[p] && m->J[q] < m->I[q]; }

static int mr_offer(void* inst, int64_t p, int64_t q) {
  mr_inst* m = (mr_inst*)inst;
  if (!mr_can_raise(m, p, q)) return 0;
  m->J[q] = m->J[p] < m->I[q] ? m->J[p] : m->I[q];
  return 1;
}

/* One pass of the update restricted to the neighbour offsets nb[k0..k1), in
 * raster order (backward = 0) or reverse raster order (backward = 1).  With
 * `seeds`, every pixel that afterwards can raise one of those neighbours is
 * queued (in visiting order) and counted in *nseeds. */
static int mr_pass(mr_inst* m, int64_t h, int64_t w, const int (*nb)[2], int k0, int k1, int backward, fifo_t* seeds,
                   int64_t* nseeds) {
  const int64_t n = h * w;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t p = backward ? n - 1 - i : i;
    const int64_t y = p / w, x = p % w;
    uint8_t v = m->J[p];
    for (int k = k0; k < k1; ++k) {
      const int64_t qy = y + nb[k][0], qx = x + nb[k][1];
      if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
      if (m->J[qy * w + qx] > v) v = m->J[qy * w + qx];
    }
    m->J[p] = v < m->I[p] ? v : m->I[p];
    if (!seeds) continue;
    for (int k = k0; k < k1; ++k) {
      const int64_t qy = y + nb[k][0], qx = x + nb[k][1];
      if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
      if (mr_can_raise(m, p, qy * w + qx)) {
        if (fifo_push(seeds, p, 0)) return -2;
        (*nseeds)++;
        break;
      }
    }
  }
  return 0;
}

int oracle_mr_fh(const uint8_t* marker, const uint8_t* mask, uint8_t* out, int64_t h, int64_t w, int conn,
                 int64_t* stats) {
  if (!marker || !mask || !out || bad_dims(h, w, conn)) return -1;
  const int64_t n = h * w;
  const int nn = nb_count(conn), half = nn / 2;
  mr_inst m = {out, mask};
  for (int64_t p = 0; p < n; ++p) out[p] = marker[p] < mask[p] ? marker[p] : mask[p];
  fifo_t fq;
  int rc = fifo_init(&fq, n / 4 + 16);
  int64_t initial = 0;
  relax_counts c = {0, 0, 0};
  if (!rc) rc = mr_pass(&m, h, w, nb_table(conn), 0, half, 0, NULL, NULL);       /* N+ (offsets before p) */
  if (!rc) rc = mr_pass(&m, h, w, nb_table(conn), half, nn, 1, &fq, &initial);   /* N- (offsets after p) */
  if (!rc) rc = relax_fifo(&fq, h, w, conn, mr_offer, &m, &c);
  fifo_free(&fq);
  if (rc) return rc;
  if (stats) {
    stats[0] = initial;
    stats[1] = c.pops;
    stats[2] = c.pushes;
    stats[3] = c.maxdep;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Morphological reconstruction by erosion (the dual instance, Sec. 1 lists it
 * among the IWPP users): rho*_I(J) is the limit of the elementary geodesic
 * erosion
 *   J(p) <- max(min{J(q) : q in N_G(p) U {p}}, I(p))
 * from a marker above the mask, and is unique like rho_I(J).  Same schedule
 * as oracle_mr_fh with every comparison reversed: a forward pass over N+, a
 * backward pass over N- that queues the pixels whose value can still travel
 * down to a neighbour, then the FIFO relaxation.  A marker below the mask is
 * raised to it first (J <- J v I).  stats: as oracle_mr_fh. */
static int mr_can_lower(const mr_inst* m, int64_t p, int64_t q) { return m->J[q] > m->J[p] && m->J[q] > m->I[q]; }

static int mr_erode_offer(void* inst, int64_t p, int64_t q) {
  mr_inst* m = (mr_inst*)inst;
  if (!mr_can_lower(m, p, q)) return 0;
  m->J[q] = m->J[p] > m->I[q] ? m->J[p] : m->I[q];
  return 1;
}

static int mr_erode_pass(mr_inst* m, int64_t h, int64_t w, const int (*nb)[2], int k0, int k1, int backward,
                         fifo_t* seeds, int64_t* nseeds) {
  const int64_t n = h * w;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t p = backward ? n - 1 - i : i;
    const int64_t y = p / w, x = p % w;
    uint8_t v = m->J[p];
    for (int k = k0; k < k1; ++k) {
      const int64_t qy = y + nb[k][0], qx = x + nb[k][1];
      if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
      if (m->J[qy * w + qx] < v) v = m->J[qy * w + qx];
    }
    m->J[p] = v > m->I[p] ? v : m->I[p];
    if (!seeds) continue;
    for (int k = k0; k < k1; ++k) {
      const int64_t qy = y + nb[k][0], qx = x + nb[k][1];
      if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
      if (mr_can_lower(m, p, qy * w + qx)) {
        if (fifo_push(seeds, p, 0)) return -2;
        (*nseeds)++;
        break;
      }
    }
  }
  return 0;
}

int oracle_mr_erode(const uint8_t* marker, const uint8_t* mask, uint8_t* out, int64_t h, int64_t w, int conn,
                    int64_t* stats) {
  if (!marker || !mask || !out || bad_dims(h, w, conn)) return -1;
  const int64_t n = h * w;
  const int nn = nb_count(conn), half = nn / 2;
  mr_inst m = {out, mask};
  for (int64_t p = 0; p < n; ++p) out[p] = marker[p] > mask[p] ? marker[p] : mask[p];
  fifo_t fq;
  int rc = fifo_init(&fq, n / 4 + 16);
  int64_t initial = 0;
  relax_counts c = {0, 0, 0};
  if (!rc) rc = mr_erode_pass(&m, h, w, nb_table(conn), 0, half, 0, NULL, NULL);
  if (!rc) rc = mr_erode_pass(&m, h, w, nb_table(conn), half, nn, 1, &fq, &initial);
  if (!rc) rc = relax_fifo(&fq, h, w, conn, mr_erode_offer, &m, &c);
  fifo_free(&fq);
  if (rc) return rc;
  if (stats) {
    stats[0] = initial;
    stats[1] = c.pops;
    stats[2] = c.pushes;
    stats[3] = c.maxdep;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* EDT helpers.  A pixel's state is its nearest feature f (an index, or -1 for
 * the paper's "inf" pixel that is farther than anything) together with the
 * squared distance to it.  Distances are compared as exact integer squared
 * distances; no square root is taken (DIST in Algorithms 3 and 6 is only ever
 * compared).  Among equal squared distances the smaller feature index wins:
 * this fixed tie-break is the reading under which the parallel result is
 * unique. */
static int64_t sqd(int64_t ay, int64_t ax, int64_t by, int64_t bx) {
  int64_t dy = ay - by, dx = ax - bx;
  return dy * dy + dx * dx;
}

/* (d1, f1) strictly before (d2, f2) in lexicographic order. */
static int key_less(int64_t d1, int64_t f1, int64_t d2, int64_t f2) {
  return d1 < d2 || (d1 == d2 && f1 < f2);
}

static void edt_write(const int64_t* feat, const int64_t* d2, int32_t* sqdist, int32_t* nearest, int64_t n) {
  for (int64_t p = 0; p < n; ++p) {
    if (feat[p] < 0) {
      sqdist[p] = -1;
      nearest[p] = -1;
    } else {
      sqdist[p] = (int32_t)d2[p];
      nearest[p] = (int32_t)feat[p];
    }
  }
}

/* Features (bin == 0) that have at least one non-feature neighbour in N_G:
 * the contour pixels that Algorithms 3 and 6 put in the initial queue. */
static int is_contour(const uint8_t* bin, int64_t h, int64_t w, int64_t y, int64_t x, int conn) {
  const int nn = nb_count(conn);
  const int (*nb)[2] = nb_table(conn);
  if (bin[y * w + x] != 0) return 0;
  for (int k = 0; k < nn; ++k) {
    int64_t qy = y + nb[k][0], qx = x + nb[k][1];
    if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
    if (bin[qy * w + qx] != 0) return 1;
  }
  return 0;
}

/* EDT by level-synchronous propagation, frontier form.
 *
 * Reading of Algorithms 3/6: the propagation is done in rounds, as the GPU
 * algorithm's in/out queue swap does, and every offer made in a round uses the
 * nearest feature its source held at the end of the previous round (a
 * snapshot).  Round r: for every p in the frontier F_r with snapshot s(p), for
 * every in-image neighbour q, the offer (d2(q, s(p)), s(p)) replaces q's state
 * if it is lexicographically smaller; q then joins F_{r+1} (once).  F_1 is the
 * set of contour features.  The loop stops when a round changes nothing.
 *
 * stats (may be NULL), 3 entries:
 *   [0] rounds that changed at least one pixel (the last frontier round
 *       never does, so this is the number of non-empty frontiers minus one)
 *   [1] total frontier size summed over all rounds (the work count Q_ref)
 *   [2] size of the initial frontier F_1
 */
int oracle_edt_rounds(const uint8_t* bin, int32_t* sqdist, int32_t* nearest, int64_t h, int64_t w, int conn,
                      int64_t* stats) {
  if (!bin || !sqdist || !nearest || bad_dims(h, w, conn)) return -1;
  const int64_t n = h * w;
  const int nn = nb_count(conn);
  const int (*nb)[2] = nb_table(conn);
  int64_t* feat = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* d2 = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* cur = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* cur_snap = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* nxt = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* stamp = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  int rc = 0;
  if (!feat || !d2 || !cur || !cur_snap || !nxt || !stamp) {
    rc = -2;
    goto done;
  }
  int64_t nfront = 0;
  for (int64_t p = 0; p < n; ++p) {
    if (bin[p] == 0) {
      feat[p] = p;
      d2[p] = 0;
    } else {
      feat[p] = -1;
      d2[p] = ORACLE_INF64;
    }
  }
  for (int64_t y = 0; y < h; ++y)
    for (int64_t x = 0; x < w; ++x)
      if (is_contour(bin, h, w, y, x, conn)) {
        cur[nfront] = y * w + x;
        cur_snap[nfront] = y * w + x;
        nfront++;
      }
  int64_t passes = 0, rounds = 0, total = 0, initial = nfront;
  while (nfront > 0) {
    passes++;
    total += nfront;
    int64_t nnext = 0;
    for (int64_t i = 0; i < nfront; ++i) {
      int64_t p = cur[i], s = cur_snap[i];
      int64_t py = p / w, px = p % w, sy = s / w, sx = s % w;
      for (int k = 0; k < nn; ++k) {
        int64_t qy = py + nb[k][0], qx = px + nb[k][1];
        if (qy < 0 || qy >= h || qx < 0 || qx >= w) continue;
        int64_t q = qy * w + qx;
        int64_t cd = sqd(qy, qx, sy, sx);
        if (key_less(cd, s, d2[q], feat[q] < 0 ? INT64_MAX : feat[q])) {
          d2[q] = cd;
          feat[q] = s;
          if (stamp[q] != passes) {
            stamp[q] = passes;
            nxt[nnext++] = q;
          }
        }
      }
    }
    /* End of round: the new frontier's snapshot is the state each holds now. */
    for (int64_t i = 0; i < nnext; ++i) {
      cur[i] = nxt[i];
      cur_snap[i] = feat[nxt[i]];
    }
    nfront = nnext;
    if (nnext > 0) rounds++;
  }
  edt_write(feat, d2, sqdist, nearest, n);
  if (stats) {
    stats[0] = rounds;
    stats[1] = total;
    stats[2] = initial;
  }
done:
  free(feat);
  free(d2);
  free(cur);
  free(cur_snap);
  free(nxt);
  free(stamp);
  return rc;
}

/* The same rounds written as a dense operator: every round recomputes every
 * pixel q as the lexicographic minimum, over q itself and its in-image
 * neighbours p, of (d2(q, f(p)), f(p)), where f is the state after the previous
 * round.  Pixels with f = -1 make no offer.  Iterates until nothing changes.
 * stats (may be NULL), 1 entry: [0] rounds that changed something. */
int oracle_edt_dense(const uint8_t* bin, int32_t* sqdist, int32_t* nearest, int64_t h, int64_t w, int conn,
                     int64_t* stats) {
  if (!bin || !sqdist || !nearest || bad_dims(h, w, conn)) return -1;
  const int64_t n = h * w;
  const int nn = nb_count(conn);
  const int (*nb)[2] = nb_table(conn);
  int64_t* fa = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* fb = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* d2 = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int rc = 0;
  if (!fa || !fb || !d2) {
    rc = -2;
    goto done;
  }
  for (int64_t p = 0; p < n; ++p) fa[p] = bin[p] == 0 ? p : -1;
  int64_t rounds = 0;
  for (;;) {
    int changed = 0;
    for (int64_t y = 0; y < h; ++y)
      for (int64_t x = 0; x < w; ++x) {
        int64_t q = y * w + x;
        int64_t bd = ORACLE_INF64, bf = INT64_MAX;
        if (fa[q] >= 0) {
          bd = sqd(y, x, fa[q] / w, fa[q] % w);
          bf = fa[q];
        }
        for (int k = 0; k < nn; ++k) {
          int64_t py = y + nb[k][0], px = x + nb[k][1];
          if (py < 0 || py >= h || px < 0 || px >= w) continue;
          int64_t f = fa[py * w + px];
          if (f < 0) continue;
          int64_t cd = sqd(y, x, f / w, f % w);
          if (key_less(cd, f, bd, bf)) {
            bd = cd;
            bf = f;
          }
        }
        fb[q] = bf == INT64_MAX ? -1 : bf;
        if (fb[q] != fa[q]) changed = 1;
      }
    int64_t* t = fa;
    fa = fb;
    fb = t;
    if (!changed) break;
    rounds++;
  }
  for (int64_t p = 0; p < n; ++p) d2[p] = fa[p] < 0 ? ORACLE_INF64 : sqd(p / w, p % w, fa[p] / w, fa[p] % w);
  edt_write(fa, d2, sqdist, nearest, n);
  if (stats) stats[0] = rounds;
done:
  free(fa);
  free(fb);
  free(d2);
  return rc;
}

/* The sequential propagation EDT of Sec. 2.2 (the schedule of Algorithm 3),
 * used to measure how far the round semantics are from it: every pixel holds
 * a nearest-feature candidate VR (itself for a feature, none otherwise); the
 * contour features wait in the FIFO in raster order; the queue relaxation
 * above offers VR(p) to each neighbour q, which takes it when it is strictly
 * closer than q's own candidate (no tie-break), in place, so later offers see
 * earlier ones.
 * stats (may be NULL), 1 entry: [0] queue pops. */
typedef struct {
  int64_t* vr;
  int64_t w;
} edt_seq_inst;

static int edt_seq_offer(void* inst, int64_t p, int64_t q) {
  edt_seq_inst* e = (edt_seq_inst*)inst;
  const int64_t w = e->w, s = e->vr[p];
  const int64_t qy = q / w, qx = q % w;
  const int64_t cur = e->vr[q] < 0 ? ORACLE_INF64 : sqd(qy, qx, e->vr[q] / w, e->vr[q] % w);
  if (sqd(qy, qx, s / w, s % w) >= cur) return 0;
  e->vr[q] = s;
  return 1;
}

int oracle_edt_alg3(const uint8_t* bin, int32_t* sqdist, int32_t* nearest, int64_t h, int64_t w, int conn,
                    int64_t* stats) {
  if (!bin || !sqdist || !nearest || bad_dims(h, w, conn)) return -1;
  const int64_t n = h * w;
  int64_t* vr = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* d2 = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  fifo_t fq;
  int rc = fifo_init(&fq, n / 4 + 16);
  relax_counts c = {0, 0, 0};
  if (!vr || !d2 || rc) {
    rc = -2;
    goto done;
  }
  for (int64_t p = 0; p < n; ++p) vr[p] = bin[p] == 0 ? p : -1;
  for (int64_t p = 0; p < n && !rc; ++p)
    if (is_contour(bin, h, w, p / w, p % w, conn)) rc = fifo_push(&fq, p, 0);
  edt_seq_inst e = {vr, w};
  if (!rc) rc = relax_fifo(&fq, h, w, conn, edt_seq_offer, &e, &c);
  if (rc) goto done;
  for (int64_t p = 0; p < n; ++p) d2[p] = vr[p] < 0 ? ORACLE_INF64 : sqd(p / w, p % w, vr[p] / w, vr[p] % w);
  edt_write(vr, d2, sqdist, nearest, n);
  if (stats) stats[0] = c.pops;
done:
  fifo_free(&fq);
  free(vr);
  free(d2);
  return rc;
}

/* Exact EDT by brute force (the problem statement of Sec. 2.2): for every
 * pixel, the smallest squared distance to any feature, and among features at
 * that distance the smallest index.  O(pixels x features); tiny images only. */
int oracle_edt_exact_bf(const uint8_t* bin, int32_t* sqdist, int32_t* nearest, int64_t h, int64_t w) {
  if (!bin || !sqdist || !nearest || h <= 0 || w <= 0) return -1;
  const int64_t n = h * w;
  int64_t nf = 0;
  for (int64_t p = 0; p < n; ++p) nf += bin[p] == 0;
  int64_t* fl = (int64_t*)malloc((size_t)(nf > 0 ? nf : 1) * sizeof(int64_t));
  if (!fl) return -2;
  nf = 0;
  for (int64_t p = 0; p < n; ++p)
    if (bin[p] == 0) fl[nf++] = p;
  for (int64_t p = 0; p < n; ++p) {
    int64_t bd = ORACLE_INF64, bf = -1;
    for (int64_t i = 0; i < nf; ++i) {
      int64_t d = sqd(p / w, p % w, fl[i] / w, fl[i] % w);
      if (d < bd) { /* features are scanned in increasing index: strict < keeps the smallest */
        bd = d;
        bf = fl[i];
      }
    }
    sqdist[p] = bf < 0 ? -1 : (int32_t)bd;
    nearest[p] = (int32_t)bf;
  }
  free(fl);
  return 0;
}

/* Exact squared EDT, separable: a column pass gives g(x, y), the distance along
 * the column to the nearest feature; a row pass takes, for every x, the lower
 * envelope of the parabolas (x - x')^2 + g(x', y)^2 (Meijster, Roerdink and
 * Hesselink 2000; lower envelope as in Felzenszwalb and Huttenlocher).  Gives
 * squared distances only (the nearest feature is not unique); -1 everywhere if
 * there is no feature. */
int oracle_edt_exact_sep(const uint8_t* bin, int64_t* sqdist, int64_t h, int64_t w) {
  if (!bin || !sqdist || h <= 0 || w <= 0) return -1;
  const int64_t n = h * w;
  int64_t* g = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* v = (int64_t*)malloc((size_t)w * sizeof(int64_t));
  double* z = (double*)malloc((size_t)(w + 1) * sizeof(double));
  int64_t* f = (int64_t*)malloc((size_t)w * sizeof(int64_t));
  int rc = 0;
  if (!g || !v || !z || !f) {
    rc = -2;
    goto done;
  }
  const int64_t BIG = -1; /* no feature in this column */
  for (int64_t x = 0; x < w; ++x) {
    int64_t last = BIG;
    for (int64_t y = 0; y < h; ++y) {
      if (bin[y * w + x] == 0) last = y;
      g[y * w + x] = last == BIG ? BIG : y - last;
    }
    last = BIG;
    for (int64_t y = h - 1; y >= 0; --y) {
      if (bin[y * w + x] == 0) last = y;
      if (last != BIG && (g[y * w + x] == BIG || last - y < g[y * w + x])) g[y * w + x] = last - y;
    }
  }
  int any = 0;
  for (int64_t p = 0; p < n && !any; ++p) any = bin[p] == 0;
  for (int64_t y = 0; y < h; ++y) {
    int64_t k = -1;
    for (int64_t x = 0; x < w; ++x) {
      int64_t gx = g[y * w + x];
      if (gx == BIG) continue;
      f[x] = gx * gx;
      /* pop parabolas that the new one hides */
      for (;;) {
        if (k < 0) {
          k = 0;
          v[0] = x;
          z[0] = -1e300;
          z[1] = 1e300;
          break;
        }
        int64_t q = v[k];
        double s = ((double)(f[x] + x * x) - (double)(f[q] + q * q)) / (2.0 * (double)(x - q));
        if (s <= z[k]) {
          k--;
          continue;
        }
        k++;
        v[k] = x;
        z[k] = s;
        z[k + 1] = 1e300;
        break;
      }
    }
    int64_t j = 0;
    for (int64_t x = 0; x < w; ++x) {
      if (k < 0) {
        sqdist[y * w + x] = -1;
        continue;
      }
      while (z[j + 1] < (double)x) j++;
      int64_t dx = x - v[j];
      sqdist[y * w + x] = dx * dx + f[v[j]];
    }
  }
  if (!any)
    for (int64_t p = 0; p < n; ++p) sqdist[p] = -1;
done:
  free(g);
  free(v);
  free(z);
  free(f);
  return rc;
}

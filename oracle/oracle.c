/*
 * RLFC reference oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain C, plain loops, no intrinsics, no threads.  Written for a reader who
 * checks it against the paper; speed is not a goal.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ALL_CODES 0x3FFFFFFu /* 26 range codes */

/* ------------------------------------------------------------------ */
/* small integer helpers                                               */
/* ------------------------------------------------------------------ */

/* floor(a / b) for b > 0, also for negative a */
static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int32_t iabs32(int32_t x) { return x < 0 ? -x : x; }

static uint32_t rd32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static int32_t rdi32(const uint8_t *p) { return (int32_t)rd32(p); }
static uint64_t rd64(const uint8_t *p) { return (uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32); }
static void wr16(uint8_t *p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void wr32(uint8_t *p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
static void wr64(uint8_t *p, uint64_t v) { wr32(p, (uint32_t)v); wr32(p + 4, (uint32_t)(v >> 32)); }

/* read one bit of a little-endian word array: bit k lives in word k/32 at position k%32 */
static uint32_t get_bit(const uint32_t *w, int64_t k) { return (w[k / 32] >> (k % 32)) & 1u; }
static void set_bit(uint32_t *w, int64_t k) { w[k / 32] |= (1u << (k % 32)); }

/* read an n-bit unsigned field, least significant bit first */
static uint32_t get_bits(const uint32_t *w, int64_t pos, int n) {
  uint32_t v = 0;
  for (int i = 0; i < n; i++) v |= get_bit(w, pos + i) << i;
  return v;
}
static void put_bits(uint32_t *w, int64_t pos, int n, uint32_t v) {
  for (int i = 0; i < n; i++)
    if ((v >> i) & 1u) set_bit(w, pos + i);
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

int orc_geometry(const orc_params *p, orc_geom *g) {
  if (!p || !g) return ORC_E_INVALID;
  if (p->grid_u < 1 || p->grid_v < 1 || p->width < 1 || p->height < 1) return ORC_E_INVALID;
  if (p->grid_u > 4096 || p->grid_v > 4096 || p->width > 65536 || p->height > 65536) return ORC_E_INVALID;
  if (p->block != 2 && p->block != 4 && p->block != 8) return ORC_E_INVALID;
  if (p->levels < 1 || p->levels > ORC_MAX_LEVELS) return ORC_E_INVALID;
  if (p->pix_threshold < 0 || p->blk_threshold < 0) return ORC_E_INVALID;
  if (p->quant_bits < 0 || p->quant_bits > 4) return ORC_E_INVALID;
  if ((p->range_mask & ~ALL_CODES) != 0) return ORC_E_INVALID;
  memset(g, 0, sizeof(*g));
  g->wp = (int32_t)(ceil_div(p->width, p->block) * p->block);
  g->hp = (int32_t)(ceil_div(p->height, p->block) * p->block);
  g->nbx = g->wp / p->block;
  g->nby = g->hp / p->block;
  g->nb = g->nbx * g->nby;
  g->ng = 3 * g->nb;
  g->lu[0] = p->grid_u;
  g->lv[0] = p->grid_v;
  int64_t nsrv = 0;
  for (int l = 1; l < p->levels; l++) {
    int c = p->cluster[l - 1];
    if (c < 2 || c > 8) return ORC_E_INVALID;
    g->lu[l] = (int32_t)ceil_div(g->lu[l - 1], c);
    g->lv[l] = (int32_t)ceil_div(g->lv[l - 1], c);
  }
  for (int l = 0; l + 1 < p->levels; l++) nsrv += (int64_t)g->lu[l] * g->lv[l];
  if (nsrv > (1 << 20)) return ORC_E_INVALID;
  g->n_srv = (int32_t)nsrv;
  g->n_top = g->lu[p->levels - 1] * g->lv[p->levels - 1];
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* colour: lossless YCoCg-R (Sec. 4, reading C1)                       */
/* ------------------------------------------------------------------ */

static void rgb_to_ycocg(int32_t r, int32_t gg, int32_t b, int32_t *y, int32_t *co, int32_t *cg) {
  int32_t o = r - b;
  int32_t t = b + (int32_t)floor_div(o, 2);
  int32_t g2 = gg - t;
  *y = t + (int32_t)floor_div(g2, 2);
  *co = o;
  *cg = g2;
}

static void ycocg_to_rgb(int32_t y, int32_t co, int32_t cg, int32_t *r, int32_t *gg, int32_t *b) {
  int32_t t = y - (int32_t)floor_div(cg, 2);
  *gg = cg + t;
  *b = t - (int32_t)floor_div(co, 2);
  *r = *b + co;
}

static int32_t clamp255(int32_t v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

void orc_ycocg_forward(const uint8_t *rgb, int64_t n, int16_t *out) {
  for (int64_t i = 0; i < n; i++) {
    int32_t y, co, cg;
    rgb_to_ycocg(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], &y, &co, &cg);
    out[3 * i] = (int16_t)y;
    out[3 * i + 1] = (int16_t)co;
    out[3 * i + 2] = (int16_t)cg;
  }
}

void orc_ycocg_inverse(const int16_t *in, int64_t n, uint8_t *rgb) {
  for (int64_t i = 0; i < n; i++) {
    int32_t r, gg, b;
    ycocg_to_rgb(in[3 * i], in[3 * i + 1], in[3 * i + 2], &r, &gg, &b);
    rgb[3 * i] = (uint8_t)clamp255(r);
    rgb[3 * i + 1] = (uint8_t)clamp255(gg);
    rgb[3 * i + 2] = (uint8_t)clamp255(b);
  }
}

/* ------------------------------------------------------------------ */
/* BISE (Sec. 3.3, readings C10, C11)                                  */
/*                                                                     */
/* Range code k: 0..11  -> plain bits, m = k+1, values in [0, 2^m)     */
/*               12..18 -> trits,     m = k-12, values in [0, 3*2^m)   */
/*               19..25 -> quints,    m = k-19, values in [0, 5*2^m)   */
/* A block of S values is stored as: the digit plane (trit/quint       */
/* kinds only: one field per group of 5 trits / 3 quints, holding the  */
/* group's digits as a base-3 / base-5 number, 8 / 7 bits for a full   */
/* group and ceil(8k/5) / ceil(7k/3) bits for a last group of k        */
/* values), followed by the S low-bit fields of m bits each.           */
/* ------------------------------------------------------------------ */

#define KIND_BITS 0
#define KIND_TRIT 1
#define KIND_QUINT 2

int orc_bise_range(int code, int *kind, int *m, int *bound) {
  int k, mm, nb;
  if (code < 0 || code > 25) return ORC_E_INVALID;
  if (code <= 11) { k = KIND_BITS; mm = code + 1; nb = 1 << mm; }
  else if (code <= 18) { k = KIND_TRIT; mm = code - 12; nb = 3 << mm; }
  else { k = KIND_QUINT; mm = code - 19; nb = 5 << mm; }
  if (kind) *kind = k;
  if (m) *m = mm;
  if (bound) *bound = nb;
  return ORC_OK;
}

/* bits used by the digit field of a group holding k values */
static int digit_field_bits(int kind, int k) {
  if (kind == KIND_TRIT) return (int)ceil_div(8 * k, 5);
  if (kind == KIND_QUINT) return (int)ceil_div(7 * k, 3);
  return 0;
}
static int group_len(int kind) { return kind == KIND_TRIT ? 5 : (kind == KIND_QUINT ? 3 : 1); }
static int radix(int kind) { return kind == KIND_TRIT ? 3 : (kind == KIND_QUINT ? 5 : 1); }

/* total bits of the digit plane for S values */
static int digit_plane_bits(int kind, int S) {
  if (kind == KIND_BITS) return 0;
  int gl = group_len(kind), total = 0;
  for (int i = 0; i < S; i += gl) {
    int k = (S - i < gl) ? (S - i) : gl;
    total += digit_field_bits(kind, k);
  }
  return total;
}

int orc_bise_bits(int code, int S) {
  int kind, m;
  if (orc_bise_range(code, &kind, &m, NULL) != ORC_OK || S < 1) return ORC_E_INVALID;
  return S * m + digit_plane_bits(kind, S);
}

int orc_bise_encode(const uint16_t *vals, int S, int code, uint32_t *words, int64_t bitpos) {
  int kind, m, bound;
  if (orc_bise_range(code, &kind, &m, &bound) != ORC_OK) return ORC_E_INVALID;
  for (int i = 0; i < S; i++)
    if (vals[i] >= bound) return ORC_E_RANGE;
  int64_t pos = bitpos;
  if (kind != KIND_BITS) {
    int gl = group_len(kind), rdx = radix(kind);
    for (int i = 0; i < S; i += gl) {
      int k = (S - i < gl) ? (S - i) : gl;
      uint32_t number = 0, place = 1;
      for (int r = 0; r < k; r++) {
        number += (uint32_t)(vals[i + r] >> m) * place; /* the high digit of value i+r */
        place *= (uint32_t)rdx;
      }
      int nbits = digit_field_bits(kind, k);
      put_bits(words, pos, nbits, number);
      pos += nbits;
    }
  }
  for (int i = 0; i < S; i++) {
    put_bits(words, pos, m, (uint32_t)vals[i] & ((1u << m) - 1u));
    pos += m;
  }
  return (int)(pos - bitpos);
}

/* returns bits consumed, or ORC_E_CORRUPT if a digit field is out of range */
int orc_bise_decode(const uint32_t *words, int64_t bitpos, int S, int code, uint16_t *vals) {
  int kind, m;
  if (orc_bise_range(code, &kind, &m, NULL) != ORC_OK) return ORC_E_INVALID;
  int64_t pos = bitpos;
  uint32_t digit[64];
  for (int i = 0; i < S; i++) digit[i] = 0;
  if (kind != KIND_BITS) {
    int gl = group_len(kind), rdx = radix(kind);
    for (int i = 0; i < S; i += gl) {
      int k = (S - i < gl) ? (S - i) : gl;
      int nbits = digit_field_bits(kind, k);
      uint32_t number = get_bits(words, pos, nbits);
      pos += nbits;
      uint32_t limit = 1;
      for (int r = 0; r < k; r++) limit *= (uint32_t)rdx;
      if (number >= limit) return ORC_E_CORRUPT;
      for (int r = 0; r < k; r++) {
        digit[i + r] = number % (uint32_t)rdx;
        number /= (uint32_t)rdx;
      }
    }
  }
  for (int i = 0; i < S; i++) {
    uint32_t low = get_bits(words, pos, m);
    pos += m;
    vals[i] = (uint16_t)((digit[i] << m) | low);
  }
  return (int)(pos - bitpos);
}

/* signed residual -> unsigned BISE value (reading C9): 0,-1,1,-2,2.. -> 0,1,2,3,4.. */
int32_t orc_zigzag(int32_t v) { return v >= 0 ? 2 * v : -2 * v - 1; }
int32_t orc_unzigzag(int32_t z) { return (z % 2 == 0) ? z / 2 : -(z + 1) / 2; }

/* uniform quantiser with step 2^q, rounding half away from zero (reading C8) */
int32_t orc_quantize(int32_t r, int q) {
  if (q == 0) return r;
  int32_t mag = (iabs32(r) + (1 << (q - 1))) >> q;
  return r < 0 ? -mag : mag;
}

/* ------------------------------------------------------------------ */
/* tree: clusters, parents, BFS order (Sec. 3.1, 3.4; readings C2, C3) */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t L;
  int32_t lu[ORC_MAX_LEVELS], lv[ORC_MAX_LEVELS], c[ORC_MAX_LEVELS];
  int32_t *srv_of[ORC_MAX_LEVELS]; /* SRV index of node id at level l (l < L-1), -1 on top */
  int32_t n_srv;
} tree_t;

static void tree_free(tree_t *t) {
  for (int l = 0; l < ORC_MAX_LEVELS; l++) free(t->srv_of[l]);
  memset(t, 0, sizeof(*t));
}

/* breadth-first traversal from the top-level nodes (row-major); children of
 * a node are visited in row-major order inside its cluster */
static int tree_build(const orc_params *p, const orc_geom *g, tree_t *t) {
  memset(t, 0, sizeof(*t));
  t->L = p->levels;
  for (int l = 0; l < p->levels; l++) {
    t->lu[l] = g->lu[l];
    t->lv[l] = g->lv[l];
    t->c[l] = (l >= 1) ? p->cluster[l - 1] : 0;
    t->srv_of[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->lu[l] * g->lv[l]);
    if (!t->srv_of[l]) { tree_free(t); return ORC_E_NOMEM; }
    for (int i = 0; i < g->lu[l] * g->lv[l]; i++) t->srv_of[l][i] = -1;
  }
  int64_t total = 0;
  for (int l = 0; l < p->levels; l++) total += (int64_t)g->lu[l] * g->lv[l];
  int32_t *ql = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
  int32_t *qn = (int32_t *)malloc(sizeof(int32_t) * (size_t)total);
  if (!ql || !qn) { free(ql); free(qn); tree_free(t); return ORC_E_NOMEM; }
  int64_t head = 0, tail = 0;
  int top = p->levels - 1;
  for (int i = 0; i < g->lu[top] * g->lv[top]; i++) { ql[tail] = top; qn[tail] = i; tail++; }
  int32_t next_srv = 0;
  while (head < tail) {
    int l = ql[head];
    int id = qn[head];
    head++;
    if (l < top) t->srv_of[l][id] = next_srv++;
    if (l == 0) continue;
    int c = t->c[l];
    int x = id % t->lu[l], y = id / t->lu[l];
    for (int cy = 0; cy < c; cy++)
      for (int cx = 0; cx < c; cx++) {
        int xc = x * c + cx, yc = y * c + cy;
        if (xc < t->lu[l - 1] && yc < t->lv[l - 1]) {
          ql[tail] = l - 1;
          qn[tail] = yc * t->lu[l - 1] + xc;
          tail++;
        }
      }
  }
  free(ql);
  free(qn);
  t->n_srv = next_srv;
  return ORC_OK;
}

/* the node id at level l above level-0 view vi (the parent of a node is the
 * cluster that contains it) */
static int ancestor(const tree_t *t, int vi, int l) {
  int x = vi % t->lu[0], y = vi / t->lu[0];
  for (int k = 1; k <= l; k++) {
    x /= t->c[k];
    y /= t->c[k];
  }
  return y * t->lu[l] + x;
}

int orc_tree_tables(const orc_params *p, int32_t *srv_path, int32_t *root) {
  orc_geom g;
  tree_t t;
  int st = orc_geometry(p, &g);
  if (st) return st;
  st = tree_build(p, &g, &t);
  if (st) return st;
  int nv = p->grid_u * p->grid_v;
  for (int vi = 0; vi < nv; vi++) {
    for (int l = 0; l + 1 < p->levels; l++)
      srv_path[(int64_t)vi * (p->levels - 1) + l] = t.srv_of[l][ancestor(&t, vi, l)];
    root[vi] = ancestor(&t, vi, p->levels - 1);
  }
  tree_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* RKV tree, bottom-up (Sec. 3.1, eqs. 1-2; readings C3, C4)           */
/* ------------------------------------------------------------------ */

static int64_t binom(int n, int k) {
  int64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

/* padded YCoCg planes of the input: [U*V][3][hp][wp] */
static void make_level0(const uint8_t *rgb, const orc_params *p, const orc_geom *g, int32_t *out) {
  int nv = p->grid_u * p->grid_v;
  int64_t plane = (int64_t)g->hp * g->wp;
  for (int vi = 0; vi < nv; vi++)
    for (int y = 0; y < g->hp; y++)
      for (int x = 0; x < g->wp; x++) {
        int sx = x < p->width ? x : p->width - 1;   /* edge replication (C13) */
        int sy = y < p->height ? y : p->height - 1;
        const uint8_t *px = rgb + (((int64_t)vi * p->height + sy) * p->width + sx) * 3;
        int32_t yy, co, cg;
        rgb_to_ycocg(px[0], px[1], px[2], &yy, &co, &cg);
        int64_t base = (int64_t)vi * 3 * plane + (int64_t)y * g->wp + x;
        out[base] = yy;
        out[base + plane] = co;
        out[base + 2 * plane] = cg;
      }
}

/* RKV^l from RKV^(l-1): integer weighted mean over the cluster */
static void filter_level(const int32_t *below, int32_t *above, const tree_t *t, int l, int64_t img) {
  int c = t->c[l];
  for (int y = 0; y < t->lv[l]; y++)
    for (int x = 0; x < t->lu[l]; x++) {
      int64_t wt = 0;
      int32_t members[64];
      int64_t weights[64];
      int nm = 0;
      for (int cy = 0; cy < c; cy++)
        for (int cx = 0; cx < c; cx++) {
          int xc = x * c + cx, yc = y * c + cy;
          if (xc >= t->lu[l - 1] || yc >= t->lv[l - 1]) continue;
          members[nm] = yc * t->lu[l - 1] + xc;
          weights[nm] = binom(c - 1, cx) * binom(c - 1, cy);
          wt += weights[nm];
          nm++;
        }
      int32_t *dst = above + (int64_t)(y * t->lu[l] + x) * img;
      for (int64_t i = 0; i < img; i++) {
        int64_t acc = 0;
        for (int k = 0; k < nm; k++) acc += weights[k] * below[(int64_t)members[k] * img + i];
        dst[i] = (int32_t)floor_div(acc + wt / 2, wt);
      }
    }
}

static int32_t **rkv_tree_alloc(const orc_params *p, const orc_geom *g, const tree_t *t,
                                const uint8_t *rgb) {
  int64_t img = 3LL * g->hp * g->wp;
  int32_t **lv = (int32_t **)calloc(ORC_MAX_LEVELS, sizeof(int32_t *));
  if (!lv) return NULL;
  for (int l = 0; l < p->levels; l++) {
    lv[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(img * t->lu[l] * t->lv[l]));
    if (!lv[l]) {
      for (int k = 0; k < l; k++) free(lv[k]);
      free(lv);
      return NULL;
    }
  }
  make_level0(rgb, p, g, lv[0]);
  for (int l = 1; l < p->levels; l++) filter_level(lv[l - 1], lv[l], t, l, img);
  return lv;
}

static void rkv_tree_free(int32_t **lv) {
  if (!lv) return;
  for (int l = 0; l < ORC_MAX_LEVELS; l++) free(lv[l]);
  free(lv);
}

int orc_rkv_tree(const uint8_t *rgb, const orc_params *p, int32_t *out) {
  orc_geom g;
  tree_t t;
  int st = orc_geometry(p, &g);
  if (st) return st;
  st = tree_build(p, &g, &t);
  if (st) return st;
  int32_t **lv = rkv_tree_alloc(p, &g, &t, rgb);
  if (!lv) { tree_free(&t); return ORC_E_NOMEM; }
  int64_t img = 3LL * g.hp * g.wp, off = 0;
  for (int l = 0; l < p->levels; l++) {
    int64_t n = img * t.lu[l] * t.lv[l];
    memcpy(out + off, lv[l], sizeof(int32_t) * (size_t)n);
    off += n;
  }
  rkv_tree_free(lv);
  tree_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* stream header (Alg. 1 return value RKVStream:BlockOffsets:SRVStream) */
/* ------------------------------------------------------------------ */

#define HDR_BYTES 128

static void write_header(uint8_t *h, const orc_params *p, const orc_geom *g, uint32_t mask,
                         uint64_t rkv_off, uint64_t off_off, uint64_t srv_off) {
  memset(h, 0, HDR_BYTES);
  h[0] = 'R'; h[1] = 'L'; h[2] = 'F'; h[3] = 'C';
  wr16(h + 4, 1);
  wr16(h + 6, HDR_BYTES);
  wr32(h + 8, (uint32_t)p->grid_u);
  wr32(h + 12, (uint32_t)p->grid_v);
  wr32(h + 16, (uint32_t)p->width);
  wr32(h + 20, (uint32_t)p->height);
  wr32(h + 24, (uint32_t)g->wp);
  wr32(h + 28, (uint32_t)g->hp);
  wr32(h + 32, (uint32_t)p->block);
  wr32(h + 36, (uint32_t)p->levels);
  wr32(h + 40, (uint32_t)p->quant_bits);
  wr32(h + 44, 3);
  for (int l = 1; l < p->levels; l++) wr32(h + 48 + 4 * (l - 1), (uint32_t)p->cluster[l - 1]);
  wr32(h + 72, (uint32_t)p->pix_threshold);
  wr32(h + 76, (uint32_t)p->blk_threshold);
  wr32(h + 80, mask);
  wr32(h + 84, (uint32_t)g->n_srv);
  wr32(h + 88, (uint32_t)g->n_top);
  wr32(h + 92, (uint32_t)g->nb);
  wr32(h + 96, (uint32_t)g->ng);
  wr64(h + 104, rkv_off);
  wr64(h + 112, off_off);
  wr64(h + 120, srv_off);
}

typedef struct {
  orc_params p;
  orc_geom g;
  const int16_t *rkv;        /* [n_top][nb][3][B*B] (little-endian host assumed) */
  const uint32_t *offsets;   /* [ng+1] */
  const uint32_t *srv;       /* words */
  int64_t srv_words;
} stream_view;

static int parse_stream(const uint8_t *s, int64_t bytes, stream_view *v) {
  if (!s || bytes < HDR_BYTES) return ORC_E_CORRUPT;
  if (s[0] != 'R' || s[1] != 'L' || s[2] != 'F' || s[3] != 'C') return ORC_E_CORRUPT;
  if ((s[4] | (s[5] << 8)) != 1 || (s[6] | (s[7] << 8)) != HDR_BYTES) return ORC_E_CORRUPT;
  memset(v, 0, sizeof(*v));
  v->p.grid_u = rdi32(s + 8);
  v->p.grid_v = rdi32(s + 12);
  v->p.width = rdi32(s + 16);
  v->p.height = rdi32(s + 20);
  v->p.block = rdi32(s + 32);
  v->p.levels = rdi32(s + 36);
  v->p.quant_bits = rdi32(s + 40);
  if (v->p.levels < 1 || v->p.levels > ORC_MAX_LEVELS) return ORC_E_CORRUPT;
  for (int l = 1; l < v->p.levels; l++) v->p.cluster[l - 1] = rdi32(s + 48 + 4 * (l - 1));
  v->p.pix_threshold = rdi32(s + 72);
  v->p.blk_threshold = rdi32(s + 76);
  v->p.range_mask = rd32(s + 80);
  if (orc_geometry(&v->p, &v->g) != ORC_OK) return ORC_E_CORRUPT;
  if (rdi32(s + 24) != v->g.wp || rdi32(s + 28) != v->g.hp || rdi32(s + 44) != 3) return ORC_E_CORRUPT;
  if (rdi32(s + 84) != v->g.n_srv || rdi32(s + 88) != v->g.n_top) return ORC_E_CORRUPT;
  if (rdi32(s + 92) != v->g.nb || rdi32(s + 96) != v->g.ng) return ORC_E_CORRUPT;
  uint64_t rkv_off = rd64(s + 104), off_off = rd64(s + 112), srv_off = rd64(s + 120);
  uint64_t rkv_bytes = (uint64_t)v->g.n_top * v->g.nb * 3 * v->p.block * v->p.block * 2;
  if (rkv_off != HDR_BYTES || off_off != rkv_off + rkv_bytes) return ORC_E_CORRUPT;
  if (srv_off != off_off + 4ULL * (v->g.ng + 1)) return ORC_E_CORRUPT;
  if ((int64_t)srv_off > bytes) return ORC_E_CORRUPT;
  v->rkv = (const int16_t *)(s + rkv_off);
  v->offsets = (const uint32_t *)(s + off_off);
  v->srv = (const uint32_t *)(s + srv_off);
  v->srv_words = (bytes - (int64_t)srv_off) / 4;
  if (v->srv_words != (int64_t)v->offsets[v->g.ng] + 2) return ORC_E_CORRUPT;
  return ORC_OK;
}

int orc_read_header(const uint8_t *stream, int64_t bytes, orc_params *p, orc_geom *g) {
  stream_view v;
  int st = parse_stream(stream, bytes, &v);
  if (st) return st;
  if (p) *p = v.p;
  if (g) *g = v.g;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* CompressLFI (Alg. 1)                                                */
/* ------------------------------------------------------------------ */

void orc_free(void *ptr) { free(ptr); }

/* ------------------------------------------------------------------ */
/* per-block encoder control (learned encoder control; the paper's     */
/* encoder uses one pixel and one block-energy threshold, Sec. 3.2)    */
/* ------------------------------------------------------------------ */

/* pixel threshold of threshold classes 0..8; class 9 drops the block */
static const int ctl_tau[9] = {0, 2, 3, 4, 5, 6, 8, 12, 16};

/* One option for one block: the residual r = own - par under threshold class
 * k, quantised; with range code `forced` >= 0 the values are limited to what
 * that code can hold (zigzag value below its bound) and it becomes the code;
 * otherwise the block takes the smallest allowed range.  Fills the values,
 * the code (-1 absent), the squared error of the reconstruction par +
 * value * 2^q against own, and the rate (5 code bits + BISE payload bits, or
 * 0).  Returns 0 if the option is usable (a range exists and the
 * reconstruction stays in int16). */
static int ctl_option(const int32_t *own, const int32_t *par, int S, int q, uint32_t mask, int k, int forced,
                      int32_t *vals, int *code, int64_t *sse, int64_t *rate) {
  int usable = 1, any = 0;
  int32_t zmax = 0;
  for (int i = 0; i < S; i++) {
    int32_t r = own[i] - par[i];
    int32_t x;
    if (k == 9 || forced == 26) {
      x = 0;
    } else {
      if (iabs32(r) < ctl_tau[k]) r = 0;
      x = orc_quantize(r, q);
      if (forced >= 0) {
        int bound;
        orc_bise_range(forced, NULL, NULL, &bound);
        /* largest |x| whose zigzag value is below the bound, per sign */
        while (orc_zigzag(x) >= bound) x += x > 0 ? -1 : 1;
      }
    }
    vals[i] = x;
    if (x != 0) any = 1;
    if (orc_zigzag(x) > zmax) zmax = orc_zigzag(x);
  }
  *code = -1;
  if (any) {
    if (forced >= 0 && forced < 26) {
      *code = forced;
    } else {
      int bestn = 0;
      for (int c = 0; c < 26; c++) {
        int bound;
        orc_bise_range(c, NULL, NULL, &bound);
        if (((mask >> c) & 1u) && bound > zmax && (*code < 0 || bound < bestn)) {
          *code = c;
          bestn = bound;
        }
      }
      if (*code < 0) usable = 0;
    }
  }
  if (*code < 0)
    for (int i = 0; i < S; i++) vals[i] = 0;
  *rate = *code >= 0 ? 5 + orc_bise_bits(*code, S) : 0;
  *sse = 0;
  for (int i = 0; i < S; i++) {
    int32_t rec = par[i] + vals[i] * (1 << q);
    if (rec < -32768 || rec > 32767) usable = 0;
    int64_t d = (int64_t)own[i] - rec;
    *sse += d * d;
  }
  return usable;
}

/* the 16 features of a block decision (see oracle.h) */
static void ctl_features(const int32_t *own, const int32_t *par, int B, int level, int c, int q, int64_t lambda_q16,
                         float *f) {
  int S = B * B;
  double sum = 0, sum2 = 0, mx = 0, n2 = 0, n4 = 0, n8 = 0, n16 = 0;
  for (int i = 0; i < S; i++) {
    double a = iabs32(own[i] - par[i]);
    sum += a;
    sum2 += a * a;
    if (a > mx) mx = a;
    n2 += a >= 2;
    n4 += a >= 4;
    n8 += a >= 8;
    n16 += a >= 16;
  }
  double hsum = 0, vsum = 0, gmx = 0, psum = 0, psum2 = 0;
  for (int y = 0; y < B; y++)
    for (int x = 0; x < B; x++) {
      double pv = par[y * B + x];
      psum += pv;
      psum2 += pv * pv;
      if (x + 1 < B) {
        double d = fabs((double)par[y * B + x + 1] - pv);
        hsum += d;
        if (d > gmx) gmx = d;
      }
      if (y + 1 < B) {
        double d = fabs((double)par[(y + 1) * B + x] - pv);
        vsum += d;
        if (d > gmx) gmx = d;
      }
    }
  double mean = sum / S, var = sum2 / S - mean * mean, pmean = psum / S, pvar = psum2 / S - pmean * pmean;
  if (var < 0) var = 0;
  if (pvar < 0) pvar = 0;
  double pairs = (double)B * (B - 1);
  f[0] = (float)(level / 4.0);
  f[1] = c == 0 ? 1.0f : 0.0f;
  f[2] = (float)(log2(1.0 + mean) / 8.0);
  f[3] = (float)(log2(1.0 + mx) / 8.0);
  f[4] = (float)(log2(1.0 + var) / 16.0);
  f[5] = (float)(n2 / S);
  f[6] = (float)(n4 / S);
  f[7] = (float)(n8 / S);
  f[8] = (float)(n16 / S);
  f[9] = (float)(log2(1.0 + hsum / pairs) / 8.0);
  f[10] = (float)(log2(1.0 + vsum / pairs) / 8.0);
  f[11] = (float)(log2(1.0 + gmx) / 8.0);
  f[12] = (float)(log2(1.0 + pvar) / 16.0);
  f[13] = (float)(q / 4.0);
  f[14] = (float)(log2(1.0 + (double)lambda_q16 / 65536.0) / 24.0);
  f[15] = (float)(B / 8.0);
}

int orc_encode(const uint8_t *rgb, const orc_params *pin, uint8_t **out, int64_t *bytes,
               int16_t *r0_out, int16_t *ycocg_out, int64_t *hist) {
  return orc_encode_ctl(rgb, pin, NULL, out, bytes, r0_out, ycocg_out, hist);
}

int orc_encode_ctl(const uint8_t *rgb, const orc_params *pin, orc_control *ctl, uint8_t **out, int64_t *bytes,
                   int16_t *r0_out, int16_t *ycocg_out, int64_t *hist) {
  if (!rgb || !pin || !out || !bytes) return ORC_E_INVALID;
  int mode = ctl ? ctl->mode : ORC_CTL_GLOBAL;
  if (mode < ORC_CTL_GLOBAL || mode > ORC_CTL_TABLE) return ORC_E_INVALID;
  if (mode == ORC_CTL_TABLE && (!ctl->classes_in || !ctl->ranges_in)) return ORC_E_INVALID;
  orc_params p = *pin;
  orc_geom g;
  int st = orc_geometry(&p, &g);
  if (st) return st;
  uint32_t mask = p.range_mask ? p.range_mask : ALL_CODES;
  tree_t t;
  st = tree_build(&p, &g, &t);
  if (st) return st;
  const int B = p.block, S = B * B, L = p.levels, q = p.quant_bits;
  const int64_t plane = (int64_t)g.hp * g.wp, img = 3 * plane;
  if (hist) for (int k = 0; k < 26; k++) hist[k] = 0;

  /* Stage I: RKV tree, bottom-up from RKV^0 = LFI */
  int32_t **rkv = rkv_tree_alloc(&p, &g, &t, rgb);
  if (!rkv) { tree_free(&t); return ORC_E_NOMEM; }
  if (ycocg_out)
    for (int64_t i = 0; i < img * p.grid_u * p.grid_v; i++) ycocg_out[i] = (int16_t)rkv[0][i];

  /* Stage II: SRV tree, top-down, against the reconstructed parent (eq. 3,
   * reading C5).  rec[l] is the reconstruction of level l. */
  int32_t *rec[ORC_MAX_LEVELS] = {0};
  rec[L - 1] = rkv[L - 1]; /* top level is kept losslessly */
  /* per (srv node, block, channel): code (-1 = absent) and S zigzag values */
  int64_t nsb = (int64_t)g.n_srv * g.nb * 3;
  int8_t *code_of = (int8_t *)malloc((size_t)(nsb > 0 ? nsb : 1));
  uint16_t *zv = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(nsb > 0 ? nsb * S : 1));
  if (!code_of || !zv) { st = ORC_E_NOMEM; goto done; }
  int64_t row = 0; /* control row: levels top-down, node, block, channel */
  for (int l = L - 2; l >= 0; l--) {
    rec[l] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(img * t.lu[l] * t.lv[l]));
    if (!rec[l]) { st = ORC_E_NOMEM; goto done; }
    for (int y = 0; y < t.lv[l]; y++)
      for (int x = 0; x < t.lu[l]; x++) {
        int id = y * t.lu[l] + x;
        int pid = (y / t.c[l + 1]) * t.lu[l + 1] + (x / t.c[l + 1]);
        int s = t.srv_of[l][id];
        const int32_t *own = rkv[l] + (int64_t)id * img;
        const int32_t *par = rec[l + 1] + (int64_t)pid * img;
        int32_t *dst = rec[l] + (int64_t)id * img;
        for (int b = 0; b < g.nb; b++)
          for (int c = 0; c < 3; c++) {
            int bx = b % g.nbx, by = b / g.nbx;
            int64_t pix[64];
            int32_t r[64], qv[64];
            for (int i = 0; i < S; i++)
              pix[i] = (int64_t)c * plane + (int64_t)(by * B + i / B) * g.wp + (bx * B + i % B);
            int64_t key = ((int64_t)s * g.nb + b) * 3 + c;
            if (mode != ORC_CTL_GLOBAL) {
              int32_t ob[64], pb[64];
              for (int i = 0; i < S; i++) {
                ob[i] = own[pix[i]];
                pb[i] = par[pix[i]];
              }
              if (ctl->features_out) ctl_features(ob, pb, B, l, c, q, ctl->lambda_q16, ctl->features_out + row * 16);
              int cls = -1, code = -1;
              if (mode == ORC_CTL_SEARCH) {
                /* least w_c * SSE * 2^16 + lambda_q16 * rate; the first class wins ties */
                int64_t best = 0;
                for (int k = 0; k < 10; k++) {
                  int32_t vk[64];
                  int ck;
                  int64_t sse, rate;
                  if (!ctl_option(ob, pb, S, q, mask, k, -1, vk, &ck, &sse, &rate)) continue;
                  int64_t cost = (c == 0 ? 6 : 1) * sse * 65536 + ctl->lambda_q16 * rate;
                  if (cls < 0 || cost < best) {
                    best = cost;
                    cls = k;
                    code = ck;
                    memcpy(qv, vk, sizeof(int32_t) * S);
                  }
                }
              } else {
                int64_t sse, rate;
                cls = ctl->classes_in[row];
                int rg = ctl->ranges_in[row];
                if (cls < 0 || cls > 9 || rg < 0 || rg > 26 || (rg < 26 && !((mask >> rg) & 1u))) {
                  st = ORC_E_INVALID;
                  goto done;
                }
                if (!ctl_option(ob, pb, S, q, mask, cls, rg, qv, &code, &sse, &rate)) {
                  st = ORC_E_RANGE;
                  goto done;
                }
              }
              if (ctl->classes_out) ctl->classes_out[row] = (int8_t)cls;
              if (ctl->ranges_out) ctl->ranges_out[row] = (int8_t)(code < 0 ? 26 : code);
              row++;
              code_of[key] = (int8_t)code;
              if (code >= 0) {
                if (hist) hist[code]++;
                for (int i = 0; i < S; i++) zv[key * S + i] = (uint16_t)orc_zigzag(qv[i]);
              }
              for (int i = 0; i < S; i++) dst[pix[i]] = par[pix[i]] + (code >= 0 ? qv[i] * (1 << q) : 0);
              continue;
            }
            /* residual and pixel-level threshold (reading C7) */
            int64_t energy = 0;
            for (int i = 0; i < S; i++) {
              r[i] = own[pix[i]] - par[pix[i]];
              if (iabs32(r[i]) < p.pix_threshold) r[i] = 0;
              energy += iabs32(r[i]);
            }
            int present = energy > p.blk_threshold; /* block-energy threshold */
            int32_t maxz = 0;
            if (present) {
              int any = 0;
              for (int i = 0; i < S; i++) {
                qv[i] = orc_quantize(r[i], q);
                if (qv[i] != 0) any = 1;
                int32_t z = orc_zigzag(qv[i]);
                if (z > maxz) maxz = z;
              }
              present = any;
            }
            code_of[key] = -1;
            if (present) {
              /* the smallest allowed range that holds every value (C10) */
              int best = -1, bestn = 0;
              for (int k = 0; k < 26; k++) {
                int bound;
                orc_bise_range(k, NULL, NULL, &bound);
                if (((mask >> k) & 1u) && bound > maxz && (best < 0 || bound < bestn)) {
                  best = k;
                  bestn = bound;
                }
              }
              if (best < 0) { st = ORC_E_RANGE; goto done; }
              code_of[key] = (int8_t)best;
              if (hist) hist[best]++;
              for (int i = 0; i < S; i++) zv[key * S + i] = (uint16_t)orc_zigzag(qv[i]);
            }
            for (int i = 0; i < S; i++) {
              int32_t d = present ? qv[i] * (1 << q) : 0;
              int32_t v = par[pix[i]] + d;
              if (v < -32768 || v > 32767) { st = ORC_E_RANGE; goto done; }
              dst[pix[i]] = v;
            }
          }
      }
  }
  if (r0_out) {
    const int32_t *src = rec[0];
    for (int64_t i = 0; i < img * p.grid_u * p.grid_v; i++) r0_out[i] = (int16_t)src[i];
  }

  /* Stage III: sizes of every group (spatial block b, channel c) */
  {
    const int nbw = (g.n_srv + 31) / 32;
    uint32_t *off = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.ng + 1));
    if (!off) { st = ORC_E_NOMEM; goto done; }
    uint64_t words = 0;
    for (int gi = 0; gi < g.ng; gi++) {
      int b = gi / 3, c = gi % 3;
      int64_t npresent = 0, pbits = 0;
      for (int s = 0; s < g.n_srv; s++) {
        int k = code_of[((int64_t)s * g.nb + b) * 3 + c];
        if (k >= 0) { npresent++; pbits += orc_bise_bits(k, S); }
      }
      off[gi] = (uint32_t)words;
      if (npresent > 0) words += (uint64_t)nbw + ceil_div(5 * npresent, 32) + ceil_div(pbits, 32);
      if (words > 0xFFFFFFF0ull) { free(off); st = ORC_E_RANGE; goto done; }
    }
    off[g.ng] = (uint32_t)words;
    uint64_t rkv_bytes = (uint64_t)g.n_top * g.nb * 3 * S * 2;
    uint64_t rkv_off = HDR_BYTES, off_off = rkv_off + rkv_bytes;
    uint64_t srv_off = off_off + 4ull * (g.ng + 1);
    uint64_t total = srv_off + 4ull * (words + 2);
    uint8_t *buf = (uint8_t *)calloc((size_t)total, 1);
    if (!buf) { free(off); st = ORC_E_NOMEM; goto done; }
    write_header(buf, &p, &g, mask, rkv_off, off_off, srv_off);
    /* RKVStream: top level stored raw, block-major (reading of Sec. 3.4 with
     * JPEG2000 replaced, C18) */
    for (int n = 0; n < g.n_top; n++)
      for (int b = 0; b < g.nb; b++)
        for (int c = 0; c < 3; c++)
          for (int i = 0; i < S; i++) {
            int bx = b % g.nbx, by = b / g.nbx;
            int32_t v = rkv[L - 1][(int64_t)n * img + (int64_t)c * plane +
                                   (int64_t)(by * B + i / B) * g.wp + (bx * B + i % B)];
            uint64_t o = rkv_off + 2 * ((((uint64_t)n * g.nb + b) * 3 + c) * S + i);
            wr16(buf + o, (uint16_t)(int16_t)v);
          }
    /* BlockOffsets */
    for (int gi = 0; gi <= g.ng; gi++) wr32(buf + off_off + 4ull * gi, off[gi]);
    /* SRVStream: blocks at one location gathered over the tree in BFS order */
    uint32_t *w = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(words + 2));
    if (!w) { free(buf); free(off); st = ORC_E_NOMEM; goto done; }
    memset(w, 0, sizeof(uint32_t) * (size_t)(words + 2));
    for (int gi = 0; gi < g.ng; gi++) {
      int b = gi / 3, c = gi % 3;
      if (off[gi] == off[gi + 1]) continue; /* no present node: nothing stored */
      uint32_t *gw = w + off[gi];
      int64_t np = 0;
      for (int s = 0; s < g.n_srv; s++)
        if (code_of[((int64_t)s * g.nb + b) * 3 + c] >= 0) { set_bit(gw, s); np++; }
      int64_t code_bit = 32LL * nbw;
      int64_t pay_bit = 32LL * (nbw + ceil_div(5 * np, 32));
      int64_t rank = 0;
      for (int s = 0; s < g.n_srv; s++) {
        int64_t key = ((int64_t)s * g.nb + b) * 3 + c;
        int k = code_of[key];
        if (k < 0) continue;
        put_bits(gw, code_bit + 5 * rank, 5, (uint32_t)k);
        pay_bit += orc_bise_encode(zv + key * S, S, k, gw, pay_bit);
        rank++;
      }
    }
    for (uint64_t i = 0; i < words + 2; i++) wr32(buf + srv_off + 4 * i, w[i]);
    free(w);
    free(off);
    *out = buf;
    *bytes = (int64_t)total;
  }
  st = ORC_OK;
done:
  for (int l = 0; l < L - 1; l++) free(rec[l]);
  free(code_of);
  free(zv);
  rkv_tree_free(rkv);
  tree_free(&t);
  return st;
}

/* ------------------------------------------------------------------ */
/* DecompressLFIBlock (Alg. 2)                                         */
/* ------------------------------------------------------------------ */

/* residual of SRV node s in group gi (d[S], zero if the block is absent);
 * follows the group layout: bitmap, 5-bit range codes of the present nodes,
 * then their BISE payloads in node order */
static int read_residual(const stream_view *v, int gi, int s, int32_t *d) {
  const int S = v->p.block * v->p.block;
  const int nbw = (v->g.n_srv + 31) / 32;
  for (int i = 0; i < S; i++) d[i] = 0;
  uint32_t o0 = v->offsets[gi], o1 = v->offsets[gi + 1];
  if (o0 == o1) return ORC_OK;            /* StartOffset: empty location */
  const uint32_t *gw = v->srv + o0;
  if (!get_bit(gw, s)) return ORC_OK;     /* block discarded by thresholding */
  int64_t np = 0, rank = 0;
  for (int k = 0; k < v->g.n_srv; k++)
    if (get_bit(gw, k)) { if (k < s) rank++; np++; }
  int64_t code_bit = 32LL * nbw;
  int64_t pay_bit = 32LL * (nbw + ceil_div(5 * np, 32));
  for (int64_t j = 0; j < rank; j++)      /* skip the payloads of earlier nodes */
    pay_bit += orc_bise_bits((int)get_bits(gw, code_bit + 5 * j, 5), S);
  int code = (int)get_bits(gw, code_bit + 5 * rank, 5);
  uint16_t u[64];
  int used = orc_bise_decode(gw, pay_bit, S, code, u);
  if (used < 0) return used;
  for (int i = 0; i < S; i++) d[i] = orc_unzigzag(u[i]) * (1 << v->p.quant_bits);
  return ORC_OK;
}

int orc_decode_block(const uint8_t *stream, int64_t bytes, int32_t vi, int32_t b, int16_t *out) {
  stream_view v;
  int st = parse_stream(stream, bytes, &v);
  if (st) return st;
  if (vi < 0 || vi >= v.p.grid_u * v.p.grid_v || b < 0 || b >= v.g.nb) return ORC_E_INVALID;
  tree_t t;
  st = tree_build(&v.p, &v.g, &t);
  if (st) return st;
  const int S = v.p.block * v.p.block, L = v.p.levels;
  int root = ancestor(&t, vi, L - 1);               /* ReadBlock(RKV^n, BlkIdx) */
  for (int c = 0; c < 3; c++) {
    int32_t x[64], d[64];
    for (int i = 0; i < S; i++) x[i] = v.rkv[(((int64_t)root * v.g.nb + b) * 3 + c) * S + i];
    for (int l = L - 2; l >= 0; l--) {               /* GetParentIndices + ReadBlocks */
      int s = t.srv_of[l][ancestor(&t, vi, l)];
      st = read_residual(&v, 3 * b + c, s, d);      /* BISEDecode */
      if (st) { tree_free(&t); return st; }
      for (int i = 0; i < S; i++) x[i] += d[i];      /* CombineBlocks */
    }
    for (int i = 0; i < S; i++) out[c * S + i] = (int16_t)x[i];
  }
  tree_free(&t);
  return ORC_OK;
}

int orc_decode_requests(const uint8_t *stream, int64_t bytes, int64_t n, const int32_t *req, int16_t *out) {
  stream_view v;
  int st = parse_stream(stream, bytes, &v);
  if (st) return st;
  const int64_t S3 = 3LL * v.p.block * v.p.block;
  for (int64_t i = 0; i < n; i++) {
    st = orc_decode_block(stream, bytes, req[2 * i], req[2 * i + 1], out + S3 * i);
    if (st) return st;
  }
  return ORC_OK;
}

/* Progressive decompression (Sec. 3.6): the same traversal as
 * orc_decode_block, stopped at tree level `level` -- the key-view block plus
 * the residuals of the view's ancestors on levels L-2 down to `level`, which
 * is the reconstruction of its level-`level` ancestor. */
int orc_decode_block_level(const uint8_t *stream, int64_t bytes, int32_t vi, int32_t b, int32_t level,
                           int16_t *out) {
  stream_view v;
  int st = parse_stream(stream, bytes, &v);
  if (st) return st;
  if (vi < 0 || vi >= v.p.grid_u * v.p.grid_v || b < 0 || b >= v.g.nb) return ORC_E_INVALID;
  if (level < 0 || level >= v.p.levels) return ORC_E_INVALID;
  tree_t t;
  st = tree_build(&v.p, &v.g, &t);
  if (st) return st;
  const int S = v.p.block * v.p.block, L = v.p.levels;
  int root = ancestor(&t, vi, L - 1);
  for (int c = 0; c < 3; c++) {
    int32_t x[64], d[64];
    for (int i = 0; i < S; i++) x[i] = v.rkv[(((int64_t)root * v.g.nb + b) * 3 + c) * S + i];
    for (int l = L - 2; l >= level; l--) {
      int s = t.srv_of[l][ancestor(&t, vi, l)];
      st = read_residual(&v, 3 * b + c, s, d);
      if (st) { tree_free(&t); return st; }
      for (int i = 0; i < S; i++) x[i] += d[i];
    }
    for (int i = 0; i < S; i++) out[c * S + i] = (int16_t)x[i];
  }
  tree_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* whole light field, one location (group) at a time                  */
/* ------------------------------------------------------------------ */

int orc_decode_all(const uint8_t *stream, int64_t bytes, int32_t b0, int32_t b1, int16_t *out) {
  stream_view v;
  int st = parse_stream(stream, bytes, &v);
  if (st) return st;
  if (b0 < 0 || b1 > v.g.nb || b0 > b1) return ORC_E_INVALID;
  tree_t t;
  st = tree_build(&v.p, &v.g, &t);
  if (st) return st;
  const int B = v.p.block, S = B * B, L = v.p.levels;
  const int nv = v.p.grid_u * v.p.grid_v;
  const int nbw = (v.g.n_srv + 31) / 32;
  const int64_t plane = (int64_t)v.g.hp * v.g.wp;
  int32_t *res = (int32_t *)malloc(sizeof(int32_t) * (size_t)(v.g.n_srv > 0 ? v.g.n_srv : 1) * S);
  if (!res) { tree_free(&t); return ORC_E_NOMEM; }
  for (int b = b0; b < b1; b++)
    for (int c = 0; c < 3; c++) {
      int gi = 3 * b + c;
      /* decode every node's residual block of this location once, walking the
       * group's payloads in node order */
      for (int64_t i = 0; i < (int64_t)v.g.n_srv * S; i++) res[i] = 0;
      uint32_t o0 = v.offsets[gi], o1 = v.offsets[gi + 1];
      if (o0 != o1) {
        const uint32_t *gw = v.srv + o0;
        int64_t np = 0;
        for (int s = 0; s < v.g.n_srv; s++) np += get_bit(gw, s);
        int64_t code_bit = 32LL * nbw;
        int64_t pay_bit = 32LL * (nbw + ceil_div(5 * np, 32));
        int64_t rank = 0;
        for (int s = 0; s < v.g.n_srv; s++) {
          if (!get_bit(gw, s)) continue;
          int code = (int)get_bits(gw, code_bit + 5 * rank, 5);
          uint16_t u[64];
          int used = orc_bise_decode(gw, pay_bit, S, code, u);
          if (used < 0) { free(res); tree_free(&t); return used; }
          pay_bit += used;
          for (int i = 0; i < S; i++)
            res[(int64_t)s * S + i] = orc_unzigzag(u[i]) * (1 << v.p.quant_bits);
          rank++;
        }
      }
      /* every view: top-level RKV block plus the residuals on its path */
      int bx = b % v.g.nbx, by = b / v.g.nbx;
      for (int vi = 0; vi < nv; vi++) {
        int root = ancestor(&t, vi, L - 1);
        for (int i = 0; i < S; i++) {
          int32_t x = v.rkv[(((int64_t)root * v.g.nb + b) * 3 + c) * S + i];
          for (int l = L - 2; l >= 0; l--) x += res[(int64_t)t.srv_of[l][ancestor(&t, vi, l)] * S + i];
          out[(int64_t)vi * 3 * plane + c * plane + (int64_t)(by * B + i / B) * v.g.wp + bx * B + i % B] =
              (int16_t)x;
        }
      }
    }
  free(res);
  tree_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* rendering (Sec. 3.6; reading C16), float32                          */
/* ------------------------------------------------------------------ */

static float lerpf(float a, float b, float f) { return a + f * (b - a); }

/* lower grid index and fraction of a coordinate on [0, n-1] */
static void cell(float x, int n, int *i0, int *i1, float *f) {
  if (x < 0.0f) x = 0.0f;
  if (x > (float)(n - 1)) x = (float)(n - 1);
  if (n == 1) { *i0 = 0; *i1 = 0; *f = 0.0f; return; }
  int i = (int)floorf(x);
  if (i > n - 2) i = n - 2;
  *i0 = i;
  *i1 = i + 1;
  *f = x - (float)i;
}

int orc_render(const int16_t *lf, int32_t U, int32_t V, int32_t W, int32_t H, int32_t wp,
               int32_t hp, const float *views, int32_t n, int32_t wo, int32_t ho, float *out) {
  return orc_render_focal(lf, U, V, W, H, wp, hp, views, n, wo, ho, 0.0f, out);
}

/* Refocused rendering (the dynamic reparameterisation Sec. 3.6 names as
 * compatible; reading C20): source camera (iu, jv) of a novel camera at
 * (u, v), clamped to the grid, is sampled at image-plane position
 * (sx + d (iu - u), ty + d (jv - v)); each source view gets its own taps
 * and fractions.  d = 0 is orc_render. */
int orc_render_focal(const int16_t *lf, int32_t U, int32_t V, int32_t W, int32_t H, int32_t wp, int32_t hp,
                     const float *views, int32_t n, int32_t wo, int32_t ho, float d, float *out) {
  if (!lf || !views || !out || n < 0 || wo < 1 || ho < 1) return ORC_E_INVALID;
  const int64_t plane = (int64_t)hp * wp;
  const float sxs = (float)W / (float)wo, tys = (float)H / (float)ho;
  for (int k = 0; k < n; k++) {
    float u = views[4 * k], v = views[4 * k + 1], s = views[4 * k + 2], t = views[4 * k + 3];
    int iu[2], jv[2];
    float fu, fv;
    cell(u, U, &iu[0], &iu[1], &fu);
    cell(v, V, &jv[0], &jv[1], &fv);
    /* the novel camera's position on the grid, clamped like the cell lookup */
    float uc = u < 0.0f ? 0.0f : (u > (float)(U - 1) ? (float)(U - 1) : u);
    float vc = v < 0.0f ? 0.0f : (v > (float)(V - 1) ? (float)(V - 1) : v);
    for (int Y = 0; Y < ho; Y++)
      for (int X = 0; X < wo; X++) {
        float sx = s + ((float)X + 0.5f) * sxs - 0.5f;
        float ty = t + ((float)Y + 0.5f) * tys - 0.5f;
        int xs[2][2][2], ys[2][2][2]; /* [view a][view b][tap] */
        float fsv[2][2], ftv[2][2];
        for (int a = 0; a < 2; a++)
          for (int bb = 0; bb < 2; bb++) {
            float dx = d == 0.0f ? 0.0f : d * ((float)iu[a] - uc);
            float dy = d == 0.0f ? 0.0f : d * ((float)jv[bb] - vc);
            cell(sx + dx, W, &xs[a][bb][0], &xs[a][bb][1], &fsv[a][bb]);
            cell(ty + dy, H, &ys[a][bb][0], &ys[a][bb][1], &ftv[a][bb]);
          }
        float rgb_tap[2][2][2][2][3]; /* [view a][view b][row][col][channel] */
        for (int a = 0; a < 2; a++)
          for (int bb = 0; bb < 2; bb++)
            for (int r = 0; r < 2; r++)
              for (int cc = 0; cc < 2; cc++) {
                int vi = jv[bb] * U + iu[a];
                int64_t o = (int64_t)vi * 3 * plane + (int64_t)ys[a][bb][r] * wp + xs[a][bb][cc];
                int32_t R, G, Bc;
                ycocg_to_rgb(lf[o], lf[o + plane], lf[o + 2 * plane], &R, &G, &Bc);
                rgb_tap[a][bb][r][cc][0] = (float)clamp255(R);
                rgb_tap[a][bb][r][cc][1] = (float)clamp255(G);
                rgb_tap[a][bb][r][cc][2] = (float)clamp255(Bc);
              }
        for (int ch = 0; ch < 3; ch++) {
          float lv[2];
          for (int a = 0; a < 2; a++) {
            float lt[2];
            for (int bb = 0; bb < 2; bb++) {
              float l0 = lerpf(rgb_tap[a][bb][0][0][ch], rgb_tap[a][bb][0][1][ch], fsv[a][bb]);
              float l1 = lerpf(rgb_tap[a][bb][1][0][ch], rgb_tap[a][bb][1][1][ch], fsv[a][bb]);
              lt[bb] = lerpf(l0, l1, ftv[a][bb]);
            }
            lv[a] = lerpf(lt[0], lt[1], fv);
          }
          out[(((int64_t)k * 3 + ch) * ho + Y) * wo + X] = lerpf(lv[0], lv[1], fu) / 255.0f;
        }
      }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* quality (Sec. 4, eqs. 4-5; reading C17)                             */
/* ------------------------------------------------------------------ */

double orc_psnr(const int16_t *ref, const int16_t *dec, int32_t nviews, int32_t W, int32_t H,
                int32_t wp, int32_t hp) {
  const int64_t plane = (int64_t)hp * wp;
  double total = 0.0;
  for (int vi = 0; vi < nviews; vi++) {
    double ps[3];
    for (int c = 0; c < 3; c++) {
      double se = 0.0;
      for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++) {
          int64_t o = (int64_t)vi * 3 * plane + c * plane + (int64_t)y * wp + x;
          double e = (double)ref[o] - (double)dec[o];
          se += e * e;
        }
      double mse = se / ((double)W * H);
      ps[c] = mse > 0.0 ? 10.0 * log10(255.0 * 255.0 / mse) : 100.0;
      if (ps[c] > 100.0) ps[c] = 100.0;
    }
    total += (6.0 * ps[0] + ps[1] + ps[2]) / 8.0;
  }
  return total / nviews;
}

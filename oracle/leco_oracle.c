/*
 * LeCo CPU oracle -- TEST INFRASTRUCTURE ONLY (see leco_oracle.h).
 *
 * Plain scalar C, one value at a time, in the order the paper describes the
 * method.  Built with -O2 -ffp-contract=off -fno-fast-math and no -march, so
 * every floating-point operation is one IEEE-754 binary64 operation rounded
 * to nearest-even.  Integer sums are exact (unsigned __int128).
 *
 * Readings of the paper taken here (all listed again in the design notes):
 *  - widths use bitlen(x) = floor(log2 x) + 1, bitlen(0) = 0;
 *  - the regressor is least squares with exact integer sums (section 3.1
 *    states the closed form), slope = fl(N) / fl(D) in binary64;
 *  - the optional minimax regressor takes the smallest slope minimising the
 *    strip width (section 3.1's fixed-width objective, solved exactly from
 *    the convex hulls), slope = fl(dy) / fl(dt) of the hull edge it lies on,
 *    and replaces the stored model only when strictly narrower;
 *  - residuals are stored as unsigned offsets from their minimum, which is
 *    folded into an integer intercept "base" (the paper's theta0);
 *  - a partition falls back to the constant (FOR) model when that is not
 *    wider, when it has one value, or when its range is >= 2^61;
 *  - prediction at local index t is floor(theta1 * t) in binary64;
 *  - residual t occupies bits [b*t, b*t + b) of its partition's span,
 *    least-significant bit first, in little-endian 64-bit words.
 */
#include "leco_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define HEADER_BYTES 64u
#define RECORD_BYTES 32u
#define MAX_PART_LEN (1ull << 20)
#define MAGIC 0x4F43454Cu /* bytes 'L','E','C','O' */
#define VERSION 1u
#define FLAG_VARIABLE 1u
#define FLAG_POLY 2u
#define POLY_MAX_LEN 4096u
#define POLY_MAX_RANGE (1ull << 50)

/* ---- small helpers -------------------------------------------------------- */

uint64_t leco_ref_bitlen(uint64_t x) {
  uint64_t b = 0;
  while (x != 0) {
    b++;
    x >>= 1;
  }
  return b;
}

static uint64_t bitlen128(u128 x) {
  uint64_t b = 0;
  while (x != 0) {
    b++;
    x >>= 1;
  }
  return b;
}

static uint64_t align16(uint64_t x) { return (x + 15u) & ~(uint64_t)15u; }

static uint64_t load_value(const void *col, int dtype, uint64_t i) {
  if (dtype == 4) return ((const uint32_t *)col)[i];
  return ((const uint64_t *)col)[i];
}

static void put_u64(uint8_t *p, uint64_t x) {
  for (int k = 0; k < 8; k++) p[k] = (uint8_t)(x >> (8 * k));
}
static void put_u32(uint8_t *p, uint32_t x) {
  for (int k = 0; k < 4; k++) p[k] = (uint8_t)(x >> (8 * k));
}
static void put_u16(uint8_t *p, uint16_t x) {
  p[0] = (uint8_t)x;
  p[1] = (uint8_t)(x >> 8);
}
static uint64_t get_u64(const uint8_t *p) {
  uint64_t x = 0;
  for (int k = 7; k >= 0; k--) x = (x << 8) | p[k];
  return x;
}
static uint32_t get_u32(const uint8_t *p) {
  uint32_t x = 0;
  for (int k = 3; k >= 0; k--) x = (x << 8) | p[k];
  return x;
}
static double f64_from_bits(uint64_t b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}
static uint64_t bits_from_f64(double d) {
  uint64_t b;
  memcpy(&b, &d, 8);
  return b;
}

/* Bit k of the packed stream lives in bit (k mod 64) of 64-bit word k / 64;
 * words are little-endian, so this is byte k / 8, bit k mod 8. */
static void set_stream_bit(uint8_t *words, uint64_t k) {
  words[k >> 3] |= (uint8_t)(1u << (k & 7));
}
static unsigned get_stream_bit(const uint8_t *words, uint64_t k) {
  return (words[k >> 3] >> (k & 7)) & 1u;
}

/* ---- Regressor (section 3.1) ------------------------------------------------ */

/* ---- Minimax regressor (section 3.1 objective) -----------------------------
 *
 * The fixed-width objective of section 3.1 asks for the line with the
 * smallest maximum deviation |F(t) - v_t|.  For a slope theta the best
 * intercept sits midway, so the deviation is half the vertical width
 *   W(theta) = max_t (v_t - theta t) - min_t (v_t - theta t)
 * of the strip that holds every point (t, v_t).  W is convex and piecewise
 * linear; it bends only at the edge slopes of the upper and lower convex
 * hulls of the points.  Its right derivative is t_lo - t_up, where t_up is
 * the position of the upper-hull vertex maximising v_t - theta t just above
 * theta and t_lo the lower-hull vertex maximising theta t - v_t.  Starting
 * below every bend (t_up = n - 1, t_lo = 0) and passing the bends in
 * increasing order, the smallest minimiser of W is the first bend after
 * which t_lo >= t_up.  Reading: an upper and a lower edge of equal slope
 * give the bend as the upper edge's fraction. */

/* Sign of (q - p) x (r - p) for points p < q < r: > 0 when r lies above the
 * line through p and q.  Values differ by less than 2^61, so differences are
 * exact in int64 and products exact in int128. */
static int turn(const uint64_t *v, uint64_t p, uint64_t q, uint64_t r) {
  i128 a = (i128)(q - p) * (i128)(int64_t)(v[r] - v[p]);
  i128 b = (i128)(int64_t)(v[q] - v[p]) * (i128)(r - p);
  return a > b ? 1 : (a < b ? -1 : 0);
}

/* Upper (upper = 1) or lower hull of the points (t, v_t), left to right,
 * with no vertex lying on an edge (Andrew's monotone chain). */
static uint64_t hull_chain(const uint64_t *v, uint64_t n, int upper, uint64_t *h) {
  uint64_t k = 0;
  for (uint64_t t = 0; t < n; t++) {
    while (k >= 2) {
      int s = turn(v, h[k - 2], h[k - 1], t);
      if (upper ? s >= 0 : s <= 0)
        k--;
      else
        break;
    }
    h[k++] = t;
  }
  return k;
}

/* Compares the slope of edge a0 -> a1 with that of edge b0 -> b1. */
static int slope_cmp(const uint64_t *v, uint64_t a0, uint64_t a1, uint64_t b0, uint64_t b1) {
  i128 l = (i128)(int64_t)(v[a1] - v[a0]) * (i128)(b1 - b0);
  i128 r = (i128)(int64_t)(v[b1] - v[b0]) * (i128)(a1 - a0);
  return l < r ? -1 : (l > r ? 1 : 0);
}

int leco_ref_minimax_slope(const uint64_t *v, uint64_t n, int64_t *dy, uint64_t *dt) {
  if (v == NULL || dy == NULL || dt == NULL || n < 2 || n > MAX_PART_LEN) return LREF_EINVAL;
  uint64_t vmin = v[0], vmax = v[0];
  for (uint64_t t = 1; t < n; t++) {
    if (v[t] < vmin) vmin = v[t];
    if (v[t] > vmax) vmax = v[t];
  }
  if (vmax - vmin >= (1ull << 61)) return LREF_EINVAL;
  uint64_t *up = (uint64_t *)malloc(n * sizeof(uint64_t));
  uint64_t *lo = (uint64_t *)malloc(n * sizeof(uint64_t));
  if (!up || !lo) {
    free(up);
    free(lo);
    return LREF_ENOMEM;
  }
  uint64_t nu = hull_chain(v, n, 1, up);
  uint64_t nl = hull_chain(v, n, 0, lo);
  uint64_t iu = nu - 1, il = 0; /* below every bend: t_up = n - 1, t_lo = 0 */
  uint64_t e0 = 0, e1 = 1;
  for (;;) {
    /* the next bend: upper edge up[iu-1] -> up[iu] or lower edge lo[il] -> lo[il+1] */
    int take_up;
    if (iu == 0)
      take_up = 0;
    else if (il + 1 == nl)
      take_up = 1;
    else
      take_up = slope_cmp(v, up[iu - 1], up[iu], lo[il], lo[il + 1]) <= 0;
    if (take_up) {
      e0 = up[iu - 1];
      e1 = up[iu];
    } else {
      e0 = lo[il];
      e1 = lo[il + 1];
    }
    /* pass every bend not above it */
    while (iu > 0 && slope_cmp(v, up[iu - 1], up[iu], e0, e1) <= 0) iu--;
    while (il + 1 < nl && slope_cmp(v, lo[il], lo[il + 1], e0, e1) <= 0) il++;
    if (lo[il] >= up[iu]) break;
  }
  *dy = (int64_t)(v[e1] - v[e0]);
  *dt = e1 - e0;
  free(up);
  free(lo);
  return LREF_OK;
}

/* Residual extremes of the line with slope theta1 (section 3.1):
 * r_t = (v_t - vmin) - floor(theta1 * t). */
static void residual_range(const uint64_t *v, uint64_t n, uint64_t vmin, double theta1,
                           int64_t *r_min, int64_t *r_max) {
  for (uint64_t t = 0; t < n; t++) {
    double prod = theta1 * (double)t;
    int64_t p = (int64_t)floor(prod);
    int64_t r = (int64_t)(v[t] - vmin) - p;
    if (t == 0 || r < *r_min) *r_min = r;
    if (t == 0 || r > *r_max) *r_max = r;
  }
}

/* ---- Polynomial regressor (Gram basis, see leco_oracle.h) ------------------ */

/* g_k(t) for positions 0..n-1; |g_k| < 2^37 for n <= 4096. */
static int64_t gram(int k, int64_t t, int64_t n) {
  switch (k) {
    case 1: return 2 * t - (n - 1);
    case 2: return 6 * t * t - 6 * (n - 1) * t + (n - 1) * (n - 2);
    default:
      return 20 * t * t * t - 30 * (n - 1) * t * t + (12 * n * n - 30 * n + 22) * t -
             (n - 1) * (n - 2) * (n - 3);
  }
}

/* c_k = fl(S_k) / fl(Q_k) for k = 1, 2, 3 (0 where Q_k = 0). */
static void poly_coefficients(const uint64_t *v, uint64_t n, uint64_t vmin, double c[3]) {
  i128 S[3] = {0, 0, 0}, Q[3] = {0, 0, 0};
  for (uint64_t t = 0; t < n; t++) {
    i128 y = (i128)(v[t] - vmin);
    for (int k = 1; k <= 3; k++) {
      i128 g = gram(k, (int64_t)t, (int64_t)n);
      S[k - 1] += y * g;
      Q[k - 1] += g * g;
    }
  }
  for (int k = 0; k < 3; k++) {
    double q = (double)Q[k];
    c[k] = Q[k] != 0 ? (double)S[k] / q : 0.0;
    if (c[k] == 0.0) c[k] = 0.0; /* +0.0, never -0.0 */
  }
}

/* p_t = floor(fl(fl(fl(c1 g1) + fl(c2 g2)) + fl(c3 g3))). */
static int64_t poly_predict(const double c[3], uint64_t t, uint64_t n) {
  double a = c[0] * (double)gram(1, (int64_t)t, (int64_t)n);
  double b = c[1] * (double)gram(2, (int64_t)t, (int64_t)n);
  double d = c[2] * (double)gram(3, (int64_t)t, (int64_t)n);
  double s = a + b;
  s = s + d;
  return (int64_t)floor(s);
}

static void poly_residual_range(const uint64_t *v, uint64_t n, uint64_t vmin, const double c[3],
                                int64_t *r_min, int64_t *r_max) {
  for (uint64_t t = 0; t < n; t++) {
    int64_t r = (int64_t)(v[t] - vmin) - poly_predict(c, t, n);
    if (t == 0 || r < *r_min) *r_min = r;
    if (t == 0 || r > *r_max) *r_max = r;
  }
}

/* Least-squares line through (t, y_t), t = 0..n-1, from exact sums:
 *   slope = (n*S_ty - S_t*S_y) / (n*S_tt - S_t^2).
 * Then residuals r_t = y_t - floor(slope * t) and their width (section 3.1,
 * fixed-width deltas).  The constant model is kept when it is not wider.
 * With the minimax regressor the minimax line replaces the stored model
 * when it is strictly narrower. */
int leco_ref_fit(const uint64_t *v, uint64_t n, int force_constant, int regressor,
                 leco_ref_model *out) {
  if (n == 0 || n > MAX_PART_LEN || out == NULL) return LREF_EINVAL;
  if (regressor != LREF_REG_LS && regressor != LREF_REG_MINIMAX && regressor != LREF_REG_POLY)
    return LREF_EINVAL;
  memset(out, 0, sizeof(*out));

  uint64_t vmin = v[0], vmax = v[0];
  for (uint64_t t = 1; t < n; t++) {
    if (v[t] < vmin) vmin = v[t];
    if (v[t] > vmax) vmax = v[t];
  }
  uint64_t range = vmax - vmin;
  out->vmin = vmin;
  out->vmax = vmax;
  out->b_for = leco_ref_bitlen(range);

  /* Constant model: every value stored as v - vmin (section 2, FOR). */
  out->mode = 0;
  out->theta1 = 0.0;
  out->base = vmin;
  out->bits = out->b_for;

  if (n == 1 || force_constant || range >= (1ull << 61)) return LREF_OK;

  /* Exact sums over y_t = v_t - vmin (< 2^61). */
  u128 s_y = 0, s_ty = 0;
  for (uint64_t t = 0; t < n; t++) {
    u128 y = v[t] - vmin;
    s_y += y;
    s_ty += (u128)t * y;
  }
  u128 nn = n;
  u128 s_t = nn * (nn - 1) / 2;
  u128 s_tt = (nn - 1) * nn * (2 * nn - 1) / 6;
  i128 N = (i128)(nn * s_ty) - (i128)(s_t * s_y);
  i128 D = (i128)(nn * s_tt) - (i128)(s_t * s_t);
  out->N_lo = (uint64_t)(u128)N;
  out->N_hi = (int64_t)(N >> 64);
  out->D_lo = (uint64_t)(u128)D;
  out->D_hi = (uint64_t)((u128)D >> 64);

  /* Two correctly rounded conversions, one correctly rounded division. */
  double fN = (double)N;
  double fD = (double)D;
  double slope = fN / fD;
  if (slope == 0.0) slope = 0.0; /* store +0.0, never -0.0 */
  out->fitted = 1;
  out->theta1_ls = slope;

  int64_t r_min = 0, r_max = 0;
  residual_range(v, n, vmin, slope, &r_min, &r_max);
  out->r_min = r_min;
  out->r_max = r_max;
  out->b_ls = leco_ref_bitlen((uint64_t)r_max - (uint64_t)r_min);

  if (out->b_ls < out->b_for) { /* ties keep the constant model */
    out->mode = 1;
    out->theta1 = slope;
    out->base = vmin + (uint64_t)r_min;
    out->bits = out->b_ls;
  }
  if (regressor == LREF_REG_POLY) {
    out->b_p2 = out->b_p3 = 99;
    if (n < 3 || n > POLY_MAX_LEN || range >= POLY_MAX_RANGE) return LREF_OK;
    double c[3];
    poly_coefficients(v, n, vmin, c);
    out->poly_fitted = 1;
    for (int k = 0; k < 3; k++) out->pc[k] = c[k];
    for (int deg = 2; deg <= 3; deg++) {
      if (deg == 3 && n < 4) break;
      double cd[3] = {c[0], c[1], deg == 3 ? c[2] : 0.0};
      int64_t p_min = 0, p_max = 0;
      poly_residual_range(v, n, vmin, cd, &p_min, &p_max);
      uint64_t b = leco_ref_bitlen((uint64_t)p_max - (uint64_t)p_min);
      if (deg == 2) out->b_p2 = b; else out->b_p3 = b;
      if (b < out->bits) { /* ties keep the simpler model */
        out->mode = 3;
        out->poly_degree = deg;
        for (int k = 0; k < 3; k++) out->stored_c[k] = cd[k];
        out->theta1 = cd[0];
        out->base = vmin + (uint64_t)p_min;
        out->bits = b;
      }
    }
    return LREF_OK;
  }
  if (regressor != LREF_REG_MINIMAX) return LREF_OK;

  int64_t dy;
  uint64_t dt;
  int st = leco_ref_minimax_slope(v, n, &dy, &dt);
  if (st != LREF_OK) return st;
  double mm = (double)dy / (double)dt; /* one correctly rounded division */
  if (mm == 0.0) mm = 0.0;
  out->mm_fitted = 1;
  out->mm_dy = dy;
  out->mm_dt = dt;
  out->theta1_mm = mm;
  int64_t m_min = 0, m_max = 0;
  residual_range(v, n, vmin, mm, &m_min, &m_max);
  out->r_min_mm = m_min;
  out->r_max_mm = m_max;
  out->b_mm = leco_ref_bitlen((uint64_t)m_max - (uint64_t)m_min);
  if (out->b_mm < out->bits) { /* ties keep the constant or least-squares model */
    out->mode = 2;
    out->theta1 = mm;
    out->base = vmin + (uint64_t)m_min;
    out->bits = out->b_mm;
  }
  return LREF_OK;
}

/* Residual u_t stored for value t under a fitted model (both modes):
 * u_t = v_t - base - floor(theta1 * t), all mod 2^64. */
static uint64_t model_predict(double theta1, uint64_t t) {
  double prod = theta1 * (double)t;
  return (uint64_t)(int64_t)floor(prod);
}

/* ---- Partitioning ----------------------------------------------------------- */

/* Builds starts[0..m] for fixed partitions of length L (section 3.2.1) or
 * checks the caller's variable starts (section 3.2.2 / 3.3). */
static int make_starts(uint64_t n, uint64_t fixed_len, const uint64_t *starts,
                       uint64_t m_var, uint64_t **starts_out, uint64_t *m_out) {
  uint64_t m;
  uint64_t *s;
  if (fixed_len > 0) {
    if (fixed_len > MAX_PART_LEN) return LREF_EINVAL;
    m = n / fixed_len + (n % fixed_len != 0);
    s = (uint64_t *)malloc((m + 1) * sizeof(uint64_t));
    if (!s) return LREF_ENOMEM;
    for (uint64_t j = 0; j < m; j++) s[j] = j * fixed_len;
    s[m] = n;
  } else {
    if (starts == NULL) return LREF_EINVAL;
    m = m_var;
    if (starts[0] != 0 || starts[m] != n) return LREF_EINVAL;
    for (uint64_t j = 0; j < m; j++) {
      if (starts[j + 1] <= starts[j]) return LREF_EINVAL;
      if (starts[j + 1] - starts[j] > MAX_PART_LEN) return LREF_EINVAL;
    }
    s = (uint64_t *)malloc((m + 1) * sizeof(uint64_t));
    if (!s) return LREF_ENOMEM;
    for (uint64_t j = 0; j <= m; j++) s[j] = starts[j];
  }
  *starts_out = s;
  *m_out = m;
  return LREF_OK;
}

/* ---- Encoder (section 3.3) -------------------------------------------------- */

typedef struct {
  uint64_t base;
  double theta1; /* slope, or c1 of a polynomial */
  uint64_t bits;
  uint64_t words;
  int kind;      /* 0 line or constant, 1 polynomial */
  double c2, c3;
} part_code;

/* Fits every partition; fills codes[] and the section offsets. */
static int plan_blob(const void *col, uint64_t n, int dtype, uint64_t fixed_len,
                     const uint64_t *starts_in, uint64_t m_in, int force_constant,
                     int regressor, uint64_t **starts_out, uint64_t *m_out, part_code **codes_out,
                     uint64_t *words_off, uint64_t *total_words,
                     uint64_t *blob_bytes) {
  if (dtype != 4 && dtype != 8) return LREF_EINVAL;
  if (n > 0 && col == NULL) return LREF_EINVAL;
  uint64_t *s = NULL, m = 0;
  int st = make_starts(n, fixed_len, starts_in, m_in, &s, &m);
  if (st != LREF_OK) return st;
  part_code *codes = (part_code *)calloc(m ? m : 1, sizeof(part_code));
  uint64_t *buf = (uint64_t *)malloc(MAX_PART_LEN * sizeof(uint64_t));
  if (!codes || !buf) {
    free(s);
    free(codes);
    free(buf);
    return LREF_ENOMEM;
  }
  uint64_t tw = 0;
  for (uint64_t j = 0; j < m; j++) {
    uint64_t len = s[j + 1] - s[j];
    for (uint64_t t = 0; t < len; t++) buf[t] = load_value(col, dtype, s[j] + t);
    leco_ref_model md;
    st = leco_ref_fit(buf, len, force_constant, regressor, &md);
    if (st != LREF_OK) {
      free(s);
      free(codes);
      free(buf);
      return st;
    }
    codes[j].base = md.base;
    codes[j].theta1 = md.theta1;
    codes[j].bits = md.bits;
    codes[j].words = (len * md.bits + 63) / 64;
    codes[j].kind = md.mode == 3;
    codes[j].c2 = md.mode == 3 ? md.stored_c[1] : 0.0;
    codes[j].c3 = md.mode == 3 ? md.stored_c[2] : 0.0;
    tw += codes[j].words;
  }
  free(buf);
  uint64_t after_meta = HEADER_BYTES + RECORD_BYTES * m;
  if (fixed_len == 0) after_meta += 8 * (m + 1);
  if (regressor == LREF_REG_POLY) after_meta = align16(after_meta) + 16 * m; /* (c2, c3) pairs */
  *words_off = align16(after_meta);
  *total_words = tw;
  *blob_bytes = align16(*words_off + 8 * tw);
  *starts_out = s;
  *m_out = m;
  *codes_out = codes;
  return LREF_OK;
}

int leco_ref_blob_bytes(const void *col, uint64_t n, int dtype,
                        uint64_t fixed_len, const uint64_t *starts, uint64_t m,
                        int force_constant, int regressor, uint64_t *bytes) {
  uint64_t *s, mm, wo, tw;
  part_code *codes;
  int st = plan_blob(col, n, dtype, fixed_len, starts, m, force_constant, regressor, &s,
                     &mm, &codes, &wo, &tw, bytes);
  if (st != LREF_OK) return st;
  free(s);
  free(codes);
  return LREF_OK;
}

int leco_ref_encode(const void *col, uint64_t n, int dtype, uint64_t fixed_len,
                    const uint64_t *starts, uint64_t m_in, int force_constant,
                    int regressor, uint8_t *blob, uint64_t cap, uint64_t *blob_bytes) {
  uint64_t *s, m, words_off, total_words, size;
  part_code *codes;
  int st = plan_blob(col, n, dtype, fixed_len, starts, m_in, force_constant, regressor, &s,
                     &m, &codes, &words_off, &total_words, &size);
  if (st != LREF_OK) return st;
  if (blob_bytes) *blob_bytes = size;
  if (blob == NULL || cap < size) {
    free(s);
    free(codes);
    return LREF_ENOSPC;
  }
  memset(blob, 0, size);

  /* Header: self-describing, all metadata needed to decode (section 3). */
  uint64_t starts_off = fixed_len > 0 ? 0 : HEADER_BYTES + RECORD_BYTES * m;
  put_u32(blob + 0, MAGIC);
  put_u16(blob + 4, VERSION);
  blob[6] = (uint8_t)dtype;
  blob[7] = (uint8_t)((fixed_len > 0 ? 0 : FLAG_VARIABLE) | (regressor == LREF_REG_POLY ? FLAG_POLY : 0));
  put_u64(blob + 8, n);
  put_u64(blob + 16, m);
  put_u64(blob + 24, fixed_len);
  put_u64(blob + 32, HEADER_BYTES);
  put_u64(blob + 40, starts_off);
  put_u64(blob + 48, words_off);
  put_u64(blob + 56, total_words);

  /* Per-partition records: model (intercept, slope), word offset, width. */
  uint64_t woff = 0;
  for (uint64_t j = 0; j < m; j++) {
    uint8_t *r = blob + HEADER_BYTES + RECORD_BYTES * j;
    put_u64(r + 0, codes[j].base);
    put_u64(r + 8, bits_from_f64(codes[j].theta1));
    put_u64(r + 16, woff);
    r[24] = (uint8_t)codes[j].bits;
    r[25] = (uint8_t)codes[j].kind;
    woff += codes[j].words;
  }
  if (fixed_len == 0)
    for (uint64_t j = 0; j <= m; j++) put_u64(blob + starts_off + 8 * j, s[j]);
  if (regressor == LREF_REG_POLY) {
    uint64_t coef_off = align16(HEADER_BYTES + RECORD_BYTES * m + (fixed_len == 0 ? 8 * (m + 1) : 0));
    for (uint64_t j = 0; j < m; j++) {
      put_u64(blob + coef_off + 16 * j, bits_from_f64(codes[j].c2));
      put_u64(blob + coef_off + 16 * j + 8, bits_from_f64(codes[j].c3));
    }
  }

  /* Delta array: residual t of partition j at bits [b*t, b*t + b) of the
   * partition's word span, least-significant bit first. */
  uint8_t *words = blob + words_off;
  woff = 0;
  for (uint64_t j = 0; j < m; j++) {
    uint64_t len = s[j + 1] - s[j];
    uint64_t b = codes[j].bits;
    double pc[3] = {codes[j].theta1, codes[j].c2, codes[j].c3};
    for (uint64_t t = 0; t < len && b > 0; t++) {
      uint64_t v = load_value(col, dtype, s[j] + t);
      uint64_t p = codes[j].kind ? (uint64_t)poly_predict(pc, t, len)
                                 : model_predict(codes[j].theta1, t);
      uint64_t u = v - codes[j].base - p;
      uint64_t first = 64 * woff + b * t;
      for (uint64_t k = 0; k < b; k++)
        if ((u >> k) & 1u) set_stream_bit(words, first + k);
    }
    woff += codes[j].words;
  }
  free(s);
  free(codes);
  return LREF_OK;
}

/* ---- Blob parsing ----------------------------------------------------------- */

typedef struct {
  uint64_t n, m, fixed_len, starts_off, words_off, total_words, coef_off;
  int dtype, variable, poly;
  const uint8_t *blob;
} blob_view;

static int parse_blob(const uint8_t *blob, uint64_t bytes, blob_view *bv) {
  if (blob == NULL || bytes < HEADER_BYTES) return LREF_EFORMAT;
  if (get_u32(blob) != MAGIC) return LREF_EFORMAT;
  if ((blob[4] | (blob[5] << 8)) != VERSION) return LREF_EFORMAT;
  bv->dtype = blob[6];
  if (blob[7] > (FLAG_VARIABLE | FLAG_POLY)) return LREF_EFORMAT;
  bv->variable = blob[7] & FLAG_VARIABLE;
  bv->poly = (blob[7] & FLAG_POLY) != 0;
  if (bv->dtype != 4 && bv->dtype != 8) return LREF_EFORMAT;
  bv->n = get_u64(blob + 8);
  bv->m = get_u64(blob + 16);
  bv->fixed_len = get_u64(blob + 24);
  uint64_t records_off = get_u64(blob + 32);
  bv->starts_off = get_u64(blob + 40);
  bv->words_off = get_u64(blob + 48);
  bv->total_words = get_u64(blob + 56);
  bv->blob = blob;
  if (records_off != HEADER_BYTES) return LREF_EFORMAT;
  if (bv->m > bytes / RECORD_BYTES) return LREF_EFORMAT;
  uint64_t meta_end = HEADER_BYTES + RECORD_BYTES * bv->m;
  if (bv->variable) {
    if (bv->fixed_len != 0) return LREF_EFORMAT;
    if (bv->starts_off != meta_end) return LREF_EFORMAT;
    meta_end += 8 * (bv->m + 1);
  } else {
    if (bv->fixed_len == 0 || bv->fixed_len > MAX_PART_LEN) return LREF_EFORMAT;
    if (bv->starts_off != 0) return LREF_EFORMAT;
    uint64_t m = bv->n / bv->fixed_len + (bv->n % bv->fixed_len != 0);
    if (m != bv->m) return LREF_EFORMAT;
  }
  bv->coef_off = 0;
  if (bv->poly) {
    bv->coef_off = align16(meta_end);
    meta_end = bv->coef_off + 16 * bv->m;
  }
  if (bv->words_off != align16(meta_end)) return LREF_EFORMAT;
  if (bv->total_words > bytes / 8) return LREF_EFORMAT;
  if (bv->words_off + 8 * bv->total_words > bytes) return LREF_EFORMAT;
  if (bv->variable) {
    const uint8_t *sp = blob + bv->starts_off;
    if (get_u64(sp) != 0 || get_u64(sp + 8 * bv->m) != bv->n) return LREF_EFORMAT;
    for (uint64_t j = 0; j < bv->m; j++) {
      uint64_t a = get_u64(sp + 8 * j), b = get_u64(sp + 8 * (j + 1));
      if (b <= a || b - a > MAX_PART_LEN) return LREF_EFORMAT;
    }
  }
  for (uint64_t j = 0; j < bv->m; j++) {
    const uint8_t *r = blob + HEADER_BYTES + RECORD_BYTES * j;
    uint64_t bits = r[24];
    if (bits > 8u * (uint64_t)bv->dtype) return LREF_EFORMAT;
    if (r[25] > (bv->poly ? 1 : 0)) return LREF_EFORMAT;
    uint64_t start, len;
    if (bv->variable) {
      start = get_u64(blob + bv->starts_off + 8 * j);
      len = get_u64(blob + bv->starts_off + 8 * (j + 1)) - start;
    } else {
      start = j * bv->fixed_len;
      len = (j + 1 == bv->m) ? bv->n - start : bv->fixed_len;
    }
    uint64_t words = (len * bits + 63) / 64;
    uint64_t woff = get_u64(r + 16);
    if (woff > bv->total_words || words > bv->total_words - woff)
      return LREF_EFORMAT;
  }
  return LREF_OK;
}

static uint64_t part_start(const blob_view *bv, uint64_t j) {
  if (bv->variable) return get_u64(bv->blob + bv->starts_off + 8 * j);
  if (j >= bv->m) return bv->n;
  return j * bv->fixed_len;
}

/* Decoder locate step (section 3.3): floor(i / L) for fixed partitions,
 * else the partition with the largest start <= i. */
static uint64_t locate(const blob_view *bv, uint64_t i) {
  if (!bv->variable) return i / bv->fixed_len;
  uint64_t lo = 0, hi = bv->m; /* answer in [lo, hi) */
  while (hi - lo > 1) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (part_start(bv, mid) <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* Decode one position: predicted value floor(theta1 * t) plus the stored
 * residual read from bits [b*t, b*(t+1)) of the partition (section 3.3). */
static uint64_t decode_one(const blob_view *bv, uint64_t i) {
  uint64_t j = locate(bv, i);
  const uint8_t *r = bv->blob + HEADER_BYTES + RECORD_BYTES * j;
  uint64_t base = get_u64(r + 0);
  double theta1 = f64_from_bits(get_u64(r + 8));
  uint64_t woff = get_u64(r + 16);
  uint64_t b = r[24];
  uint64_t t = i - part_start(bv, j);
  const uint8_t *words = bv->blob + bv->words_off;
  uint64_t u = 0;
  uint64_t first = 64 * woff + b * t;
  for (uint64_t k = 0; k < b; k++)
    if (get_stream_bit(words, first + k)) u |= (uint64_t)1 << k;
  uint64_t p;
  if (r[25] == 1) {
    const uint8_t *cp = bv->blob + bv->coef_off + 16 * j;
    double c[3] = {theta1, f64_from_bits(get_u64(cp)), f64_from_bits(get_u64(cp + 8))};
    p = (uint64_t)poly_predict(c, t, part_start(bv, j + 1) - part_start(bv, j));
  } else {
    p = model_predict(theta1, t);
  }
  uint64_t v = base + p + u;
  if (bv->dtype == 4) v &= 0xffffffffull;
  return v;
}

static void store_value(void *out, int dtype, uint64_t q, uint64_t v) {
  if (dtype == 4)
    ((uint32_t *)out)[q] = (uint32_t)v;
  else
    ((uint64_t *)out)[q] = v;
}

int leco_ref_blob_info(const uint8_t *blob, uint64_t blob_bytes, uint64_t *n,
                       int *dtype, uint64_t *m) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  if (n) *n = bv.n;
  if (dtype) *dtype = bv.dtype;
  if (m) *m = bv.m;
  return LREF_OK;
}

int leco_ref_blob_record(const uint8_t *blob, uint64_t blob_bytes, uint64_t j,
                         uint64_t *base, double *theta1, uint64_t *word_off,
                         uint64_t *bits, uint64_t *start, uint64_t *len) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  if (j >= bv.m) return LREF_ERANGE;
  const uint8_t *r = blob + HEADER_BYTES + RECORD_BYTES * j;
  if (base) *base = get_u64(r);
  if (theta1) *theta1 = f64_from_bits(get_u64(r + 8));
  if (word_off) *word_off = get_u64(r + 16);
  if (bits) *bits = r[24];
  if (start) *start = part_start(&bv, j);
  if (len) *len = part_start(&bv, j + 1) - part_start(&bv, j);
  return LREF_OK;
}

int leco_ref_decode_all(const uint8_t *blob, uint64_t blob_bytes, void *out,
                        uint64_t out_cap_elems) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  if (out_cap_elems < bv.n) return LREF_ENOSPC;
  for (uint64_t i = 0; i < bv.n; i++) store_value(out, bv.dtype, i, decode_one(&bv, i));
  return LREF_OK;
}

int leco_ref_decode_range(const uint8_t *blob, uint64_t blob_bytes,
                          uint64_t begin, uint64_t end, void *out) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  if (begin > end || end > bv.n) return LREF_ERANGE;
  for (uint64_t i = begin; i < end; i++)
    store_value(out, bv.dtype, i - begin, decode_one(&bv, i));
  return LREF_OK;
}

int leco_ref_random_access(const uint8_t *blob, uint64_t blob_bytes,
                           const uint64_t *pos, uint64_t k, void *out) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  for (uint64_t q = 0; q < k; q++)
    if (pos[q] >= bv.n) return LREF_ERANGE;
  for (uint64_t q = 0; q < k; q++) store_value(out, bv.dtype, q, decode_one(&bv, pos[q]));
  return LREF_OK;
}

int leco_ref_filter_sum(const uint8_t *blob, uint64_t blob_bytes, uint64_t lo,
                        uint64_t hi, uint64_t out[3]) {
  blob_view bv;
  int st = parse_blob(blob, blob_bytes, &bv);
  if (st != LREF_OK) return st;
  u128 sum = 0;
  uint64_t count = 0;
  for (uint64_t i = 0; i < bv.n; i++) {
    uint64_t v = decode_one(&bv, i);
    if (lo <= v && v < hi) {
      sum += v;
      count++;
    }
  }
  out[0] = (uint64_t)sum;
  out[1] = (uint64_t)(sum >> 64);
  out[2] = count;
  return LREF_OK;
}

/* ---- Variable-length partitioner (section 3.2.2) ---------------------------- */

/* Signed first difference d_k = v_k - v_{k-1} (exact). */
static i128 first_diff(const uint64_t *v, uint64_t k) {
  return (i128)v[k] - (i128)v[k - 1];
}

/* Width of a signed integer including its sign bit: bitlen(|d|) + 1.
 * This is the reading under which the worked Delta-encoding example of the
 * partitioning figure (C = 6, merge 62 < 76) comes out as printed. */
static uint64_t signed_width(i128 d) {
  u128 a = d < 0 ? (u128)(-d) : (u128)d;
  return bitlen128(a) + 1;
}

/* Delta~(v[i, j)) for the linear regressor: bitlen(max d - min d) over the
 * first differences inside the partition (k = i+1 .. j-1); 0 without two of
 * them. */
static uint64_t approx_linear_width(const uint64_t *v, uint64_t i, uint64_t j) {
  if (j < i + 2) return 0;
  i128 dmin = first_diff(v, i + 1), dmax = dmin;
  for (uint64_t k = i + 2; k < j; k++) {
    i128 d = first_diff(v, k);
    if (d < dmin) dmin = d;
    if (d > dmax) dmax = d;
  }
  return bitlen128((u128)(dmax - dmin));
}

/* Delta(v[i, j)) for Delta encoding: widest signed first difference. */
static uint64_t delta_width(const uint64_t *v, uint64_t i, uint64_t j) {
  uint64_t w = 0;
  for (uint64_t k = i + 1; k < j; k++) {
    uint64_t s = signed_width(first_diff(v, k));
    if (s > w) w = s;
  }
  return w;
}

int64_t leco_ref_split_cost(const uint64_t *v, uint64_t i, uint64_t j, int model) {
  uint64_t len = j - i;
  uint64_t w_old, w_new;
  if (model == 1) {
    w_old = delta_width(v, i, j);
    w_new = delta_width(v, i, j + 1);
  } else {
    w_old = approx_linear_width(v, i, j);
    w_new = approx_linear_width(v, i, j + 1);
  }
  return (int64_t)((len + 1) * w_new) - (int64_t)(len * w_old);
}

uint64_t leco_ref_delta_partition_bits(const uint64_t *v, uint64_t i, uint64_t j,
                                       uint64_t sm_bits) {
  return sm_bits + (j - i) * delta_width(v, i, j);
}

uint64_t leco_ref_partition_cost_bytes(const uint64_t *v, uint64_t i, uint64_t j) {
  leco_ref_model md;
  leco_ref_fit(v + i, j - i, 0, LREF_REG_LS, &md);
  return RECORD_BYTES + 8 + 8 * (((j - i) * md.bits + 63) / 64);
}

static uint64_t *load_column(const void *col, uint64_t n, int dtype) {
  uint64_t *v = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!v) return NULL;
  for (uint64_t i = 0; i < n; i++) v[i] = load_value(col, dtype, i);
  return v;
}

/* ---- Delta-fix special-case codec (section 2, Delta encoding; the
 * evaluation's Delta-fix baseline) ---------------------------------------------
 *
 * Delta encoding over fixed-length partitions: a partition stores its first
 * value (the implicit step model of section 3.2.2) and the first differences
 * d_k = v_k - v_{k-1} of its other values, bit-packed at one fixed width.
 * Read for bit-packing as LeCo packs residuals: the differences are stored
 * as offsets e_k = d_k - d_min >= 0 from the partition's smallest
 * difference, width bitlen(d_max - d_min) (at most 65 bits), residual t
 * (t = 0 for the partition's second value) at bits [w t, w t + w) of the
 * partition's word span, least-significant bit first.
 * Layout: 32-byte header {magic "DLTF" u32, version u16 = 1, dtype u8,
 * 0 u8, n u64, L u64, m u64}; m 32-byte records {v_first u64, d_min mod
 * 2^64 u64, word_off u64, width u8, 0xff if d_min < 0 else 0 u8, 6 zero
 * bytes}; then the words (word_off in 64-bit words from the section start).
 * Decoding is sequential inside a partition: v_k = v_{k-1} + d_min + e_k. */

#define DF_MAGIC 0x46544C44u /* bytes 'D','L','T','F' */
#define DF_HEADER 32u
#define DF_RECORD 32u

/* Smallest and largest first difference of v[a, b) (b - a >= 2). */
static void diff_range(const uint64_t *v, uint64_t a, uint64_t b, i128 *dmin, i128 *dmax) {
  *dmin = *dmax = first_diff(v, a + 1);
  for (uint64_t k = a + 2; k < b; k++) {
    i128 d = first_diff(v, k);
    if (d < *dmin) *dmin = d;
    if (d > *dmax) *dmax = d;
  }
}

static int delta_fix_plan(const uint64_t *v, uint64_t n, uint64_t L, uint64_t *words) {
  uint64_t total = 0;
  for (uint64_t a = 0; a < n; a += L) {
    uint64_t b = a + L < n ? a + L : n;
    if (b - a < 2) continue;
    i128 dmin, dmax;
    diff_range(v, a, b, &dmin, &dmax);
    uint64_t w = bitlen128((u128)(dmax - dmin));
    total += ((b - a - 1) * w + 63) / 64;
  }
  *words = total;
  return LREF_OK;
}

int leco_ref_delta_fix_bytes(const void *col, uint64_t n, int dtype, uint64_t L,
                             uint64_t *bytes) {
  if ((dtype != 4 && dtype != 8) || L == 0 || L > MAX_PART_LEN || bytes == NULL)
    return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  if (!v) return LREF_ENOMEM;
  uint64_t words = 0;
  delta_fix_plan(v, n, L, &words);
  uint64_t m = (n + L - 1) / L;
  *bytes = DF_HEADER + DF_RECORD * m + 8 * words;
  free(v);
  return LREF_OK;
}

int leco_ref_delta_fix_encode(const void *col, uint64_t n, int dtype, uint64_t L,
                              uint8_t *blob, uint64_t cap, uint64_t *blob_bytes) {
  uint64_t need = 0;
  int st = leco_ref_delta_fix_bytes(col, n, dtype, L, &need);
  if (st != LREF_OK) return st;
  *blob_bytes = need;
  if (cap < need || blob == NULL) return LREF_ENOSPC;
  uint64_t *v = load_column(col, n, dtype);
  if (!v) return LREF_ENOMEM;
  memset(blob, 0, need);
  uint64_t m = (n + L - 1) / L;
  put_u32(blob, DF_MAGIC);
  put_u16(blob + 4, 1);
  blob[6] = (uint8_t)dtype;
  put_u64(blob + 8, n);
  put_u64(blob + 16, L);
  put_u64(blob + 24, m);
  uint8_t *words = blob + DF_HEADER + DF_RECORD * m;
  uint64_t word_off = 0;
  for (uint64_t j = 0; j < m; j++) {
    uint64_t a = j * L, b = a + L < n ? a + L : n;
    uint8_t *rec = blob + DF_HEADER + DF_RECORD * j;
    put_u64(rec, v[a]);
    put_u64(rec + 16, word_off);
    if (b - a < 2) continue;
    i128 dmin, dmax;
    diff_range(v, a, b, &dmin, &dmax);
    uint64_t w = bitlen128((u128)(dmax - dmin));
    put_u64(rec + 8, (uint64_t)dmin);
    rec[24] = (uint8_t)w;
    rec[25] = dmin < 0 ? 0xff : 0;
    uint8_t *span = words + 8 * word_off;
    for (uint64_t k = a + 1; k < b; k++) {
      u128 e = (u128)(first_diff(v, k) - dmin);
      uint64_t t = k - a - 1;
      for (uint64_t bit = 0; bit < w; bit++)
        if ((e >> bit) & 1u) set_stream_bit(span, w * t + bit);
    }
    word_off += ((b - a - 1) * w + 63) / 64;
  }
  free(v);
  return LREF_OK;
}

int leco_ref_delta_fix_decode(const uint8_t *blob, uint64_t blob_bytes, void *out,
                              uint64_t out_cap_elems) {
  if (blob == NULL || blob_bytes < DF_HEADER || get_u32(blob) != DF_MAGIC) return LREF_EFORMAT;
  int dtype = blob[6];
  uint64_t n = get_u64(blob + 8), L = get_u64(blob + 16), m = get_u64(blob + 24);
  if ((dtype != 4 && dtype != 8) || L == 0 || L > MAX_PART_LEN || m != (n + L - 1) / L ||
      m > (blob_bytes - DF_HEADER) / DF_RECORD)
    return LREF_EFORMAT;
  if (out_cap_elems < n) return LREF_ENOSPC;
  const uint8_t *words = blob + DF_HEADER + DF_RECORD * m;
  uint64_t nwords = (blob_bytes - DF_HEADER - DF_RECORD * m) / 8;
  for (uint64_t j = 0; j < m; j++) {
    const uint8_t *rec = blob + DF_HEADER + DF_RECORD * j;
    uint64_t a = j * L, b = a + L < n ? a + L : n;
    uint64_t x = get_u64(rec);
    uint64_t dmin_lo = get_u64(rec + 8), off = get_u64(rec + 16), w = rec[24];
    if (w > 65 || off > nwords || ((b - a - 1) * w + 63) / 64 > nwords - off)
      return LREF_EFORMAT;
    const uint8_t *span = words + 8 * off;
    store_value(out, dtype, a, x);
    for (uint64_t k = a + 1; k < b; k++) {
      uint64_t t = k - a - 1;
      u128 e = 0;
      for (uint64_t bit = 0; bit < w; bit++)
        e |= (u128)get_stream_bit(span, w * t + bit) << bit;
      /* v_k = v_{k-1} + d_min + e_k, taken mod 2^64 (exact: the true v_k is
       * a value of the column) */
      x = x + dmin_lo + (uint64_t)e;
      store_value(out, dtype, k, x);
    }
  }
  return LREF_OK;
}

/* Merge phase (section 3.2.2): scan the partition list from the left; the
 * current partition tries to merge with its right neighbour, and the merge
 * is accepted when the merged partition is strictly smaller than the two
 * apart (sizes: leco_ref_partition_cost_bytes) and stays within max_len.
 * After an accepted merge the merged partition is the current one and tries
 * its new right neighbour; after a refused one the neighbour becomes the
 * current partition.  Passes over the list repeat until one accepts no
 * merge, or max_passes passes have run (0: no limit).  The list is
 * rewritten in place. */
static void merge_phase(const uint64_t *v, uint64_t *s, uint64_t *m_io,
                        uint64_t max_len, uint64_t max_passes) {
  uint64_t m = *m_io;
  for (uint64_t pass = 0; max_passes == 0 || pass < max_passes; pass++) {
    if (m < 2) break;
    uint64_t merges = 0;
    uint64_t w = 0; /* s[0..w] are the kept starts; the current partition begins at s[w] */
    uint64_t cur = leco_ref_partition_cost_bytes(v, s[0], s[1]);
    for (uint64_t k = 1; k < m; k++) {
      uint64_t a = s[w], b = s[k], c = s[k + 1];
      uint64_t right = leco_ref_partition_cost_bytes(v, b, c);
      if (c - a <= max_len) {
        uint64_t joint = leco_ref_partition_cost_bytes(v, a, c);
        if (joint < cur + right) {
          cur = joint;
          merges++;
          continue;
        }
      }
      s[++w] = b;
      cur = right;
    }
    s[w + 1] = s[m];
    m = w + 1;
    if (merges == 0) break;
  }
  *m_io = m;
}

/* Good starting positions for Delta encoding (section 3.2.2, "Selecting
 * Good Starting Positions", and the Delta-encoding partitioning figure):
 *   required bits  rb_k = signed width of d_k = bitlen(|d_k|) + 1, k >= 1;
 *   delta bits     db_k = |rb_k - rb_{k-1}|, k >= 2;
 * the positions whose delta bits equal the smallest over the column are
 * good; each maximal run of good positions k..k' is one starting partition
 * v[k-2, k'+1).  forced[p] = 1 at the first value p = k - 2 of every
 * starting partition; n < 3 has none.  Used with the Delta-encoding cost. */
static void starting_positions_delta(const uint64_t *v, uint64_t n, unsigned char *forced) {
  memset(forced, 0, n ? n : 1);
  if (n < 3) return;
  uint64_t best = ~(uint64_t)0;
  for (uint64_t k = 2; k < n; k++) {
    uint64_t a = signed_width(first_diff(v, k)), b = signed_width(first_diff(v, k - 1));
    uint64_t db = a > b ? a - b : b - a;
    if (db < best) best = db;
  }
  int prev_good = 0;
  for (uint64_t k = 2; k < n; k++) {
    uint64_t a = signed_width(first_diff(v, k)), b = signed_width(first_diff(v, k - 1));
    int good = (a > b ? a - b : b - a) == best;
    if (good && !prev_good) forced[k - 2] = 1;
    prev_good = good;
  }
}

/* |dd_k| for the second-order delta dd_k = d_k - d_{k-1}
 * = v_k - 2 v_{k-1} + v_{k-2}, k >= 2 (exact). */
static u128 second_order_magnitude(const uint64_t *v, uint64_t k) {
  i128 dd = first_diff(v, k) - first_diff(v, k - 1);
  return dd < 0 ? (u128)(-dd) : (u128)dd;
}

/* Starting partitions for the linear regressor (section 3.2.2, "Selecting
 * Good Starting Positions": for a model of degree k, the segments where the
 * (k+1)-th order deltas are smallest; degree 1 here).  Position k >= 2 is
 * good when |dd_k| equals the smallest |dd| over the column.  Each maximal
 * run of good positions k..k' is one starting partition v[k-2, k'+1): the
 * three values a second-order delta spans, which is also the paper's
 * minimum for a linear regressor.  When two runs are one position apart
 * they would share a value; the later starting partition takes it.
 * mark[p] = 1 at the first value of a starting partition, 2 at its other
 * values, 0 elsewhere; n < 3 has none. */
static void starting_partitions_linear(const uint64_t *v, uint64_t n, unsigned char *mark) {
  memset(mark, 0, n ? n : 1);
  if (n < 3) return;
  u128 best = second_order_magnitude(v, 2);
  for (uint64_t k = 3; k < n; k++) {
    u128 x = second_order_magnitude(v, k);
    if (x < best) best = x;
  }
  uint64_t k = 2;
  while (k < n) {
    if (second_order_magnitude(v, k) != best) {
      k++;
      continue;
    }
    uint64_t last = k;
    while (last + 1 < n && second_order_magnitude(v, last + 1) == best) last++;
    mark[k - 2] = 1;
    for (uint64_t p = k - 1; p <= last; p++) mark[p] = 2;
    k = last + 1;
  }
}

int leco_ref_start_positions(const void *col, uint64_t n, int dtype, uint64_t *first_out,
                             uint64_t *end_out, uint64_t *count_out) {
  if (dtype != 4 && dtype != 8) return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  unsigned char *mark = (unsigned char *)malloc(n ? n : 1);
  if (!v || !mark) {
    free(v);
    free(mark);
    return LREF_ENOMEM;
  }
  starting_partitions_linear(v, n, mark);
  uint64_t c = 0;
  for (uint64_t p = 0; p < n; p++) {
    if (mark[p] != 1) continue;
    uint64_t e = p + 1;
    while (e < n && mark[e] == 2) e++;
    first_out[c] = p;
    if (end_out) end_out[c] = e;
    c++;
  }
  *count_out = c;
  free(v);
  free(mark);
  return LREF_OK;
}

int leco_ref_start_positions_delta(const void *col, uint64_t n, int dtype, uint64_t *pos_out,
                                   uint64_t *count_out) {
  if (dtype != 4 && dtype != 8) return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  unsigned char *forced = (unsigned char *)malloc(n ? n : 1);
  if (!v || !forced) {
    free(v);
    free(forced);
    return LREF_ENOMEM;
  }
  starting_positions_delta(v, n, forced);
  uint64_t c = 0;
  for (uint64_t p = 0; p < n; p++)
    if (forced[p]) pos_out[c++] = p;
  *count_out = c;
  free(v);
  free(forced);
  return LREF_OK;
}

/* Split phase (section 3.2.2), left to right from position 0: keep the
 * running range of first differences of the current partition v[i, j) and
 * include v[j] while C = (len+1) * Delta~new - len * Delta~old <= tau * S_M,
 * len = j - i; otherwise v[j] begins a new partition.  A partition that
 * holds max_len values takes no further value.  With starting partitions
 * (mark, or null): the first value of each begins a partition and its other
 * values are included without the cost test (the partition is grown from
 * there by the test), the cap still applying. */
static uint64_t split_phase(const uint64_t *v, uint64_t n, double threshold, uint64_t max_len,
                            const unsigned char *mark, uint64_t *starts_out) {
  uint64_t m = 0;
  uint64_t i = 0;
  starts_out[m++] = 0;
  i128 dmin = 0, dmax = 0;
  int have_diff = 0;
  uint64_t w_old = 0;
  for (uint64_t j = 1; j < n; j++) {
    i128 d = first_diff(v, j);
    i128 nmin = have_diff && dmin < d ? dmin : d;
    i128 nmax = have_diff && dmax > d ? dmax : d;
    uint64_t w_new = bitlen128((u128)(nmax - nmin));
    uint64_t len = j - i;
    double cost = (double)((int64_t)((len + 1) * w_new) - (int64_t)(len * w_old));
    int begins = mark && mark[j] == 1;
    int inside = mark && mark[j] == 2;
    if (len < max_len && !begins && (inside || cost <= threshold)) {
      dmin = nmin;
      dmax = nmax;
      have_diff = 1;
      w_old = w_new;
    } else {
      i = j;
      starts_out[m++] = j;
      have_diff = 0;
      w_old = 0;
    }
  }
  starts_out[m] = n;
  return m;
}

static int partition_common(const void *col, uint64_t n, int dtype, double tau,
                            uint64_t sm_bits, uint64_t max_len, int merge,
                            uint64_t max_passes, int start_positions, uint64_t *starts_out,
                            uint64_t *m_out) {
  if ((dtype != 4 && dtype != 8) || max_len == 0 || max_len > MAX_PART_LEN)
    return LREF_EINVAL;
  if (n == 0) {
    starts_out[0] = 0;
    *m_out = 0;
    return LREF_OK;
  }
  uint64_t *v = load_column(col, n, dtype);
  unsigned char *mark = start_positions ? (unsigned char *)malloc(n) : NULL;
  if (!v || (start_positions && !mark)) {
    free(v);
    free(mark);
    return LREF_ENOMEM;
  }
  if (mark) starting_partitions_linear(v, n, mark);
  uint64_t m = split_phase(v, n, tau * (double)sm_bits, max_len, mark, starts_out);
  if (merge) merge_phase(v, starts_out, &m, max_len, max_passes);
  free(mark);
  free(v);
  *m_out = m;
  return LREF_OK;
}

int leco_ref_partition_greedy(const void *col, uint64_t n, int dtype, double tau,
                              uint64_t sm_bits, uint64_t max_len,
                              uint64_t max_passes, int start_positions,
                              uint64_t *starts_out, uint64_t *m_out) {
  return partition_common(col, n, dtype, tau, sm_bits, max_len, 1, max_passes,
                          start_positions, starts_out, m_out);
}

int leco_ref_partition_split(const void *col, uint64_t n, int dtype, double tau,
                             uint64_t sm_bits, uint64_t max_len, int start_positions,
                             uint64_t *starts_out, uint64_t *m_out) {
  return partition_common(col, n, dtype, tau, sm_bits, max_len, 0, 0, start_positions,
                          starts_out, m_out);
}

int leco_ref_partition_merge(const void *col, uint64_t n, int dtype,
                             uint64_t *starts, uint64_t *m, uint64_t max_len,
                             uint64_t max_passes) {
  if ((dtype != 4 && dtype != 8) || max_len == 0 || max_len > MAX_PART_LEN)
    return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  if (!v) return LREF_ENOMEM;
  merge_phase(v, starts, m, max_len, max_passes);
  free(v);
  return LREF_OK;
}

int leco_ref_partitioning_cost(const void *col, uint64_t n, int dtype,
                               const uint64_t *starts, uint64_t m,
                               uint64_t *bytes_out) {
  if (dtype != 4 && dtype != 8) return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  if (!v) return LREF_ENOMEM;
  uint64_t total = 0;
  for (uint64_t j = 0; j < m; j++)
    total += leco_ref_partition_cost_bytes(v, starts[j], starts[j + 1]);
  free(v);
  *bytes_out = total;
  return LREF_OK;
}

/* Dynamic programming over split points (section 3.2): best[k] is the
 * smallest total cost of v[0, k). */
int leco_ref_partition_dp(const void *col, uint64_t n, int dtype, uint64_t max_len,
                          uint64_t *starts_out, uint64_t *m_out,
                          uint64_t *bytes_out) {
  if ((dtype != 4 && dtype != 8) || max_len == 0) return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  uint64_t *best = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  uint64_t *from = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
  if (!v || !best || !from) {
    free(v);
    free(best);
    free(from);
    return LREF_ENOMEM;
  }
  best[0] = 0;
  for (uint64_t k = 1; k <= n; k++) {
    best[k] = UINT64_MAX;
    for (uint64_t i = 0; i < k; i++) {
      if (k - i > max_len) continue;
      uint64_t c = best[i] + leco_ref_partition_cost_bytes(v, i, k);
      if (c < best[k]) {
        best[k] = c;
        from[k] = i;
      }
    }
  }
  uint64_t m = 0;
  for (uint64_t k = n; k > 0; k = from[k]) m++;
  starts_out[m] = n;
  uint64_t idx = m;
  for (uint64_t k = n; k > 0; k = from[k]) starts_out[--idx] = from[k];
  if (n == 0) starts_out[0] = 0;
  *m_out = m;
  *bytes_out = best[n];
  free(v);
  free(best);
  free(from);
  return LREF_OK;
}

int leco_ref_partition_bruteforce(const void *col, uint64_t n, int dtype,
                                  uint64_t max_len, uint64_t *starts_out,
                                  uint64_t *m_out, uint64_t *bytes_out) {
  if ((dtype != 4 && dtype != 8) || n == 0 || n > 24 || max_len == 0)
    return LREF_EINVAL;
  uint64_t *v = load_column(col, n, dtype);
  if (!v) return LREF_ENOMEM;
  uint64_t best = UINT64_MAX, best_mask = 0;
  /* bit k-1 of mask set <=> a partition starts at position k (1 <= k < n) */
  for (uint64_t mask = 0; mask < (1ull << (n - 1)); mask++) {
    uint64_t total = 0, a = 0;
    int ok = 1;
    for (uint64_t k = 1; k <= n; k++) {
      if (k == n || ((mask >> (k - 1)) & 1u)) {
        if (k - a > max_len) {
          ok = 0;
          break;
        }
        total += leco_ref_partition_cost_bytes(v, a, k);
        a = k;
      }
    }
    if (ok && total < best) {
      best = total;
      best_mask = mask;
    }
  }
  uint64_t m = 0;
  starts_out[m++] = 0;
  for (uint64_t k = 1; k < n; k++)
    if ((best_mask >> (k - 1)) & 1u) starts_out[m++] = k;
  starts_out[m] = n;
  *m_out = m;
  *bytes_out = best;
  free(v);
  return LREF_OK;
}

/* ---- Fixed partition size search (section 3.2.1) --------------------------- */

int leco_ref_fixed_cost(const void *col, uint64_t n, int dtype,
                        const uint64_t *starts, uint64_t k, uint64_t window,
                        uint64_t L, int regressor, uint64_t *cost) {
  if (col == NULL || starts == NULL || cost == NULL || (dtype != 4 && dtype != 8)) return LREF_EINVAL;
  if (k == 0 || window == 0 || window > n || L == 0 || L > window || L > MAX_PART_LEN)
    return LREF_EINVAL;
  for (uint64_t i = 0; i < k; i++)
    if (starts[i] > n - window) return LREF_EINVAL;
  uint64_t *buf = (uint64_t *)malloc(L * sizeof(uint64_t));
  if (!buf) return LREF_ENOMEM;
  uint64_t total = 0;
  for (uint64_t i = 0; i < k; i++) {
    for (uint64_t p = 0; p < window; p += L) {
      uint64_t len = window - p < L ? window - p : L;
      for (uint64_t t = 0; t < len; t++) buf[t] = load_value(col, dtype, starts[i] + p + t);
      leco_ref_model md;
      int st = leco_ref_fit(buf, len, 0, regressor, &md);
      if (st != LREF_OK) {
        free(buf);
        return st;
      }
      total += RECORD_BYTES + (regressor == LREF_REG_POLY ? 16 : 0) + 8 * ((len * md.bits + 63) / 64);
    }
  }
  free(buf);
  *cost = total;
  return LREF_OK;
}

typedef struct {
  leco_ref_cost_fn fn;
  void *ctx;
  uint64_t *trace, cap, len;
  uint64_t *seen; /* costs of evaluated lengths, UINT64_MAX if none */
} search_state;

static uint64_t evaluate(search_state *ss, uint64_t L) {
  if (ss->seen[L] != UINT64_MAX) return ss->seen[L];
  uint64_t c = ss->fn(ss->ctx, L);
  ss->seen[L] = c;
  if (2 * ss->len + 2 <= ss->cap) {
    ss->trace[2 * ss->len] = L;
    ss->trace[2 * ss->len + 1] = c;
  }
  ss->len++;
  return c;
}

int leco_ref_size_search_fn(uint64_t window, leco_ref_cost_fn cost_fn, void *ctx,
                            uint64_t *L_out, uint64_t *cost_out, uint64_t *trace,
                            uint64_t trace_cap, uint64_t *trace_len) {
  if (window == 0 || window > MAX_PART_LEN || cost_fn == NULL || L_out == NULL || cost_out == NULL)
    return LREF_EINVAL;
  search_state ss = {cost_fn, ctx, trace, trace ? trace_cap : 0, 0, NULL};
  ss.seen = (uint64_t *)malloc((window + 1) * sizeof(uint64_t));
  if (!ss.seen) return LREF_ENOMEM;
  for (uint64_t L = 0; L <= window; L++) ss.seen[L] = UINT64_MAX;

  /* Step 2, exponential phase: double L until the cost rises. */
  uint64_t best = 1, best_cost = evaluate(&ss, 1), prev = best_cost;
  for (uint64_t L = 1; L < window;) {
    L = 2 * L <= window ? 2 * L : window;
    uint64_t c = evaluate(&ss, L);
    if (c < best_cost) {
      best = L;
      best_cost = c;
    }
    if (c > prev) break;
    prev = c;
  }
  /* Step 2, back search with halving steps; step 3, convergence. */
  for (uint64_t s = best / 2; s >= 1; s /= 2) {
    uint64_t cand[2] = {best > s ? best - s : 0, best + s <= window ? best + s : 0};
    uint64_t nb = best, nc = best_cost;
    for (int q = 0; q < 2; q++) {
      if (cand[q] == 0) continue;
      uint64_t c = evaluate(&ss, cand[q]);
      if (c < nc) {
        nb = cand[q];
        nc = c;
      }
    }
    if (nb != best) {
      int converged = (best_cost - nc) * 10000 < best_cost; /* < 0.01% */
      best = nb;
      best_cost = nc;
      if (converged) break;
    }
  }
  free(ss.seen);
  *L_out = best;
  *cost_out = best_cost;
  if (trace_len) *trace_len = ss.len;
  return LREF_OK;
}

typedef struct {
  const void *col;
  uint64_t n;
  int dtype;
  const uint64_t *starts;
  uint64_t k, window;
  int regressor;
  int status;
} column_cost_ctx;

static uint64_t column_cost(void *p, uint64_t L) {
  column_cost_ctx *c = (column_cost_ctx *)p;
  uint64_t cost = UINT64_MAX;
  int st = leco_ref_fixed_cost(c->col, c->n, c->dtype, c->starts, c->k, c->window, L,
                               c->regressor, &cost);
  if (st != LREF_OK && c->status == LREF_OK) c->status = st;
  return cost;
}

int leco_ref_size_search(const void *col, uint64_t n, int dtype,
                         const uint64_t *starts, uint64_t k, uint64_t window,
                         int regressor, uint64_t *L_out, uint64_t *cost_out,
                         uint64_t *trace, uint64_t trace_cap, uint64_t *trace_len) {
  uint64_t probe;
  int st = leco_ref_fixed_cost(col, n, dtype, starts, k, window, 1, regressor, &probe);
  if (st != LREF_OK) return st;
  column_cost_ctx c = {col, n, dtype, starts, k, window, regressor, LREF_OK};
  st = leco_ref_size_search_fn(window, column_cost, &c, L_out, cost_out, trace, trace_cap,
                               trace_len);
  return st != LREF_OK ? st : c.status;
}

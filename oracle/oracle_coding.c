/*
 * oracle_coding.c -- oracle of the learned-coding stage's lossless parts
 * [Sec. 3.4.2]: the octree tokens of the quantized geometry and an entropy
 * coder for token streams.  Integer arithmetic throughout, apart from the
 * quantizer's FP32 decision and the FP64 ideal code length.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c): only tests, the smoke check and
 * the CPU-baseline leg of the benchmark use it; it shares nothing with the
 * HIP library.
 *
 * Geometry [Sec. 3.4.2, geometry occupancy coding]: the kept Gaussians'
 * position codes k_c = rint(fl32(y_c / q_c)) (the quantizer's decision)
 * become voxel coordinates u_c = k_c - kmin_c in [0, 2^D), D the smallest
 * depth holding every channel's range (at least 1).  Equal voxels merge;
 * their multiplicity minus one is kept as metadata.  The octree over the
 * unique voxels is written level by level from the root: every node of
 * level l (a prefix of D - l coordinate bits per axis) gives one 8-bit token
 * whose bit (xb << 2 | yb << 1 | zb) is set when the child with those next
 * bits is occupied; within a level the nodes follow the Morton order of
 * their prefixes (code bits 3b + 2 = x bit b, 3b + 1 = y bit b, 3b = z bit b).
 *
 * Entropy coder: the paper models p(t_i | t_{i-1}) (a network conditioned on
 * the previous token) and codes the tokens arithmetically.  Here the same
 * factorization is realized by a count-based model whose tables travel in the
 * header: order 1 (context = the previous symbol of the same lane, 256 for a
 * lane's first symbol) or order 0 (one context).  Each context's counts c_s
 * become frequencies summing to M = 4096: with K symbols present and N
 * counts in all, f_s = 1 + floor(c_s (M - K) / N) for present symbols, 0
 * otherwise, and the remainder M - sum f goes to the most frequent symbol
 * (the lowest one on ties).  The coder is range ANS (Duda 2013) with a 32-bit
 * state in [2^16, 2^32), 16-bit renormalization and 12-bit frequencies,
 * interleaved over 64 lanes: the stream is cut into blocks of 64 S symbols,
 * lane l of a block owns its l-th run of S consecutive symbols, and the
 * decoder advances the 64 lanes in lock step, one symbol each per step, the
 * lanes that fall below 2^16 taking the block's next words in lane order.
 * Blocks are independent (they decode in parallel, one wave each).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ANS_PB 12
#define ANS_M (1u << ANS_PB)
#define ANS_L (1u << 16)
#define ANS_CTX 257

/* ---- Morton codes ------------------------------------------------------ */
uint64_t orc_morton3(uint32_t ux, uint32_t uy, uint32_t uz, int32_t depth) {
  uint64_t c = 0;
  for (int b = 0; b < depth; ++b) {
    c |= (uint64_t)((ux >> b) & 1u) << (3 * b + 2);
    c |= (uint64_t)((uy >> b) & 1u) << (3 * b + 1);
    c |= (uint64_t)((uz >> b) & 1u) << (3 * b);
  }
  return c;
}

static int u64_less(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y);
}

/* Voxels of the kept Gaussians.  hdr[0] = depth D, hdr[1..3] = kmin (x, y,
 * z), hdr[4] = kept Gaussians, hdr[5] = unique voxels, hdr[6] = tokens,
 * hdr[7] = flags (bit 0: a code outside int32 or a range beyond 2^21).
 * codes [kept] (sorted unique voxel codes in the first hdr[5]), dup [kept]
 * (multiplicity - 1 of each unique voxel), tokens [21 * kept] (level by
 * level), level_size [22] (tokens of each level).  Returns hdr[6]. */
int64_t orc_octree_tokens(int64_t n, int64_t npad, const float *y, const float *q,
                          const uint8_t *mhat, int64_t *hdr, uint64_t *codes, uint32_t *dup,
                          uint8_t *tokens, int64_t *level_size) {
  memset(hdr, 0, 8 * sizeof(int64_t));
  int64_t kmin[3] = {0, 0, 0}, kmax[3] = {0, 0, 0};
  int64_t kept = 0;
  int32_t *k = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    if (!mhat[i]) continue;
    for (int c = 0; c < 3; ++c) {
      float r = rintf(y[c * npad + i] / q[c]);
      if (!(r >= -2147483648.0f && r < 2147483648.0f)) {
        hdr[7] |= 1;
        r = 0.0f;
      }
      const int64_t v = (int64_t)r;
      k[3 * kept + c] = (int32_t)v;
      if (kept == 0 || v < kmin[c]) kmin[c] = v;
      if (kept == 0 || v > kmax[c]) kmax[c] = v;
    }
    ++kept;
  }
  int depth = 1;
  for (int c = 0; c < 3; ++c)
    while (depth < 40 && (kmax[c] - kmin[c]) >= ((int64_t)1 << depth)) ++depth;
  if (depth > 21) {
    hdr[7] |= 1;
    depth = 21;
  }
  hdr[0] = depth;
  for (int c = 0; c < 3; ++c) hdr[1 + c] = kmin[c];
  hdr[4] = kept;
  for (int64_t j = 0; j < kept; ++j)
    codes[j] = orc_morton3((uint32_t)(k[3 * j] - kmin[0]), (uint32_t)(k[3 * j + 1] - kmin[1]),
                           (uint32_t)(k[3 * j + 2] - kmin[2]), depth);
  free(k);
  qsort(codes, (size_t)kept, sizeof(uint64_t), u64_less);
  int64_t m = 0;
  for (int64_t j = 0; j < kept; ++j) {
    if (m > 0 && codes[j] == codes[m - 1]) {
      dup[m - 1] += 1;
    } else {
      codes[m] = codes[j];
      dup[m] = 0;
      ++m;
    }
  }
  hdr[5] = m;
  /* levels 0 .. D-1: node = code >> 3 (D - l), child = next three bits */
  int64_t nt = 0;
  for (int l = 0; l < 22; ++l) level_size[l] = 0;
  for (int l = 0; l < depth; ++l) {
    const int sh = 3 * (depth - l);
    int64_t start = nt;
    for (int64_t j = 0; j < m; ++j) {
      const uint64_t node = sh >= 64 ? 0 : codes[j] >> sh;
      const int child = (int)((codes[j] >> (sh - 3)) & 7u);
      if (j == 0 || node != (sh >= 64 ? 0 : codes[j - 1] >> sh)) tokens[nt++] = 0;
      tokens[nt - 1] |= (uint8_t)(1u << child);
    }
    level_size[l] = nt - start;
  }
  hdr[6] = nt;
  return nt;
}

/* The unique voxel codes of a token stream (level by level, `depth` levels):
 * every node's set bits, lowest first, give its children; codes [voxels]
 * receives the last level's.  Returns the voxel count. */
int64_t orc_octree_decode(const uint8_t *tokens, int64_t ntok, int32_t depth, uint64_t *codes,
                          int64_t cap) {
  uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1));
  uint64_t *nxt = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap > 0 ? cap : 1));
  int64_t ncur = 1, pos = 0;
  cur[0] = 0;
  for (int l = 0; l < depth; ++l) {
    int64_t nn = 0;
    for (int64_t j = 0; j < ncur; ++j) {
      if (pos >= ntok) {
        free(cur);
        free(nxt);
        return -1;
      }
      const uint8_t t = tokens[pos++];
      for (int c = 0; c < 8; ++c)
        if (t & (1u << c)) {
          if (nn >= cap) {
            free(cur);
            free(nxt);
            return -1;
          }
          nxt[nn++] = (cur[j] << 3) | (uint64_t)c;
        }
    }
    uint64_t *sw = cur;
    cur = nxt;
    nxt = sw;
    ncur = nn;
  }
  memcpy(codes, cur, sizeof(uint64_t) * (size_t)ncur);
  free(cur);
  free(nxt);
  return ncur;
}

/* ---- entropy coder -------------------------------------------------------- */
/* Symbol i of a stream of n lies in block b = i / (64 S), lane
 * l = (i mod 64 S) / S, step t = i mod S (S = `lane_len`). */
static int ctx_of(const uint8_t *sym, int64_t i, int64_t lane_len, int order) {
  if (order == 0) return 0;
  return i % lane_len == 0 ? 256 : sym[i - 1];
}

/* freq [257][256]: the model of the stream (rows of unused contexts zero). */
void orc_ans_model(const uint8_t *sym, int64_t n, int32_t order, int64_t lane_len,
                   uint16_t *freq) {
  uint64_t *cnt = (uint64_t *)calloc((size_t)ANS_CTX * 256, sizeof(uint64_t));
  for (int64_t i = 0; i < n; ++i) cnt[(size_t)ctx_of(sym, i, lane_len, order) * 256 + sym[i]] += 1;
  memset(freq, 0, sizeof(uint16_t) * (size_t)ANS_CTX * 256);
  for (int x = 0; x < ANS_CTX; ++x) {
    const uint64_t *c = cnt + (size_t)x * 256;
    uint64_t N = 0;
    int K = 0, best = -1;
    for (int s = 0; s < 256; ++s) {
      N += c[s];
      if (c[s]) {
        ++K;
        if (best < 0 || c[s] > c[best]) best = s;
      }
    }
    if (!N) continue;
    uint32_t sum = 0;
    for (int s = 0; s < 256; ++s) {
      if (!c[s]) continue;
      const uint32_t f = 1u + (uint32_t)(c[s] * (uint64_t)(ANS_M - (uint32_t)K) / N);
      freq[(size_t)x * 256 + s] = (uint16_t)f;
      sum += f;
    }
    freq[(size_t)x * 256 + best] = (uint16_t)(freq[(size_t)x * 256 + best] + (ANS_M - sum));
  }
  free(cnt);
}

/* Ideal code length of the stream under the model, in bits (FP64):
 * -sum log2(f / M) over the symbols. */
double orc_ans_ideal_bits(const uint8_t *sym, int64_t n, int32_t order, int64_t lane_len,
                          const uint16_t *freq) {
  double bits = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t f = freq[(size_t)ctx_of(sym, i, lane_len, order) * 256 + sym[i]];
    bits -= log2((double)f / (double)ANS_M);
  }
  return bits;
}

static uint32_t cum_at(const uint16_t *row, int s) {
  uint32_t a = 0;
  for (int j = 0; j < s; ++j) a += row[j];
  return a;
}

/* Encode.  Block b's words: the 64 lanes' final states (high half, low half),
 * then its renormalization words in the order the decoder takes them (steps
 * ascending, lanes ascending within a step).  block_off [blocks + 1] are the
 * blocks' word offsets.  Returns the total word count, or -1 when a symbol
 * has frequency 0 in its context. */
int64_t orc_ans_encode(const uint8_t *sym, int64_t n, int32_t order, int64_t lane_len,
                       const uint16_t *freq, uint16_t *words, int64_t *block_off) {
  const int64_t S = lane_len, B = 64 * lane_len;
  const int64_t nb = (n + B - 1) / B;
  uint16_t *stack = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(B + 1));
  /* cumulative frequencies of every context, once */
  uint32_t *cum = (uint32_t *)malloc(sizeof(uint32_t) * ANS_CTX * 256);
  for (int x = 0; x < ANS_CTX; ++x)
    for (int s2 = 0; s2 < 256; ++s2) cum[x * 256 + s2] = cum_at(freq + (size_t)x * 256, s2);
  int64_t out = 0;
  for (int64_t b = 0; b < nb; ++b) {
    uint32_t x[64];
    for (int l = 0; l < 64; ++l) x[l] = ANS_L;
    int64_t top = 0;
    /* the reverse of the decoder's order: steps descending, lanes descending */
    for (int64_t t = S - 1; t >= 0; --t)
      for (int l = 63; l >= 0; --l) {
        const int64_t i = b * B + l * S + t;
        if (i >= n) continue;
        const int ctx = ctx_of(sym, i, S, order);
        const uint32_t f = freq[(size_t)ctx * 256 + sym[i]];
        if (!f) {
          free(stack);
          free(cum);
          return -1;
        }
        const uint64_t xmax = ((uint64_t)(ANS_L >> ANS_PB) << 16) * f;
        while ((uint64_t)x[l] >= xmax) {
          stack[top++] = (uint16_t)(x[l] & 0xFFFFu);
          x[l] >>= 16;
        }
        x[l] = ((x[l] / f) << ANS_PB) + (x[l] % f) + cum[ctx * 256 + sym[i]];
      }
    block_off[b] = out;
    for (int l = 0; l < 64; ++l) {
      words[out++] = (uint16_t)(x[l] >> 16);
      words[out++] = (uint16_t)(x[l] & 0xFFFFu);
    }
    for (int64_t j = top - 1; j >= 0; --j) words[out++] = stack[j];
  }
  block_off[nb] = out;
  free(stack);
  free(cum);
  return out;
}

/* Decode n symbols; returns 0, or -1 on a malformed stream (a block's words
 * run out, a slot maps to no symbol, or a block ends with words unread or
 * a lane not back at the encoder's initial state). */
int64_t orc_ans_decode(const uint16_t *words, const int64_t *block_off, int64_t n, int32_t order,
                       int64_t lane_len, const uint16_t *freq, uint8_t *sym) {
  const int64_t S = lane_len, B = 64 * lane_len;
  const int64_t nb = (n + B - 1) / B;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t p = block_off[b];
    const int64_t pe = block_off[b + 1];
    if (pe - p < 128) return -1;
    uint32_t x[64];
    for (int l = 0; l < 64; ++l) x[l] = ((uint32_t)words[p + 2 * l] << 16) | words[p + 2 * l + 1];
    p += 128;
    for (int64_t t = 0; t < S; ++t)
      for (int l = 0; l < 64; ++l) {
        const int64_t i = b * B + l * S + t;
        if (i >= n) continue;
        const uint16_t *row = freq + (size_t)ctx_of(sym, i, S, order) * 256;
        const uint32_t slot = x[l] & (ANS_M - 1u);
        uint32_t lo = 0;
        int s = 0;
        while (s < 256 && lo + row[s] <= slot) lo += row[s++];
        if (s == 256) return -1;
        sym[i] = (uint8_t)s;
        x[l] = row[s] * (x[l] >> ANS_PB) + slot - lo;
        while (x[l] < ANS_L) {
          if (p >= pe) return -1;
          x[l] = (x[l] << 16) | words[p++];
        }
      }
    if (p != pe) return -1;
    for (int l = 0; l < 64; ++l)
      if (x[l] != ANS_L) return -1;
  }
  return 0;
}

/* Decoded geometry: the unique voxel codes with their duplicates, in code
 * order, as FP32 positions mu_c = fl32((u_c + kmin_c) q_c); xyz [3][total].
 * Returns the Gaussian count (sum of dup + 1). */
int64_t orc_voxel_positions(const uint64_t *codes, const uint32_t *dup, int64_t m, int32_t depth,
                            const int64_t *kmin, const float *q, float *xyz, int64_t total) {
  int64_t o = 0;
  for (int64_t j = 0; j < m; ++j) {
    uint32_t u[3] = {0, 0, 0};
    for (int b = 0; b < depth; ++b) {
      u[0] |= (uint32_t)((codes[j] >> (3 * b + 2)) & 1u) << b;
      u[1] |= (uint32_t)((codes[j] >> (3 * b + 1)) & 1u) << b;
      u[2] |= (uint32_t)((codes[j] >> (3 * b)) & 1u) << b;
    }
    for (uint32_t r = 0; r <= dup[j]; ++r, ++o)
      for (int c = 0; c < 3; ++c)
        if (o < total) xyz[c * total + o] = (float)(int64_t)(u[c] + kmin[c]) * q[c];
  }
  return o;
}

/* ---- attributes [Sec. 3.4.2, autoregressive attribute coding] ------------ */
typedef struct {
  uint64_t code;
  int64_t idx;
} code_idx;

static int code_idx_less(const void *a, const void *b) {
  const code_idx *x = (const code_idx *)a, *y = (const code_idx *)b;
  if (x->code != y->code) return x->code < y->code ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Morton order of the kept Gaussians: perm [kept] lists their indices by
 * voxel code (the octree's, with kmin and depth as orc_octree_tokens finds
 * them), Gaussians of one voxel by index.  Returns the kept count. */
int64_t orc_morton_order(int64_t n, int64_t npad, const float *y, const float *q,
                         const uint8_t *mhat, int32_t depth, const int64_t *kmin, int64_t *perm) {
  code_idx *a = (code_idx *)malloc(sizeof(code_idx) * (size_t)(n > 0 ? n : 1));
  int64_t kept = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!mhat[i]) continue;
    uint32_t u[3];
    for (int c = 0; c < 3; ++c) {
      float r = rintf(y[c * npad + i] / q[c]);
      if (!(r >= -2147483648.0f && r < 2147483648.0f)) r = 0.0f;
      u[c] = (uint32_t)((int64_t)r - kmin[c]);
    }
    a[kept].code = orc_morton3(u[0], u[1], u[2], depth);
    a[kept].idx = i;
    ++kept;
  }
  qsort(a, (size_t)kept, sizeof(code_idx), code_idx_less);
  for (int64_t j = 0; j < kept; ++j) perm[j] = a[j].idx;
  free(a);
  return kept;
}

/* Byte planes of one attribute channel in serialized order: v_j = k - kmin
 * (the fixed-length coder's value, k = rint(fl32(y / q))).  Predictor 1:
 * v_j is predicted by the previous Gaussian of the same group of S (0 for a
 * group's first) and the residual zigzag-mapped (d >= 0 -> 2d, d < 0 ->
 * -2d - 1); predictor 0: v_j itself.  Cut into `planes` bytes, most
 * significant first: out [planes][kept]. */
void orc_attr_planes(int64_t kept, const float *yc, const float *qc, const int64_t *perm,
                     int64_t kmin, int32_t planes, int64_t S, int32_t predictor, uint8_t *out) {
  int64_t prev = 0;
  for (int64_t j = 0; j < kept; ++j) {
    const float r = rintf(yc[perm[j]] / qc[0]);
    const int64_t v = (int64_t)r - kmin;
    const int64_t pred = j % S == 0 ? 0 : prev;
    const int64_t d = v - pred;
    const uint64_t z = predictor == 0 ? (uint64_t)v
                       : d >= 0     ? (uint64_t)(2 * d)
                                    : (uint64_t)(-2 * d - 1);
    for (int t = 0; t < planes; ++t)
      out[(int64_t)t * kept + j] = (uint8_t)(z >> (8 * (planes - 1 - t)));
    prev = v;
  }
}

/* Inverse: the dequantized values fl32((kmin + v) q) in serialized order. */
void orc_attr_reconstruct(int64_t kept, const uint8_t *pl, int32_t planes, int64_t S, int64_t kmin,
                          float q, int32_t predictor, float *out) {
  int64_t prev = 0;
  for (int64_t j = 0; j < kept; ++j) {
    uint64_t z = 0;
    for (int t = 0; t < planes; ++t) z = (z << 8) | pl[(int64_t)t * kept + j];
    const int64_t d = (z & 1u) ? -(int64_t)((z + 1) / 2) : (int64_t)(z / 2);
    const int64_t v = predictor == 0 ? (int64_t)z : (j % S == 0 ? 0 : prev) + d;
    out[j] = (float)(kmin + v) * q;
    prev = v;
  }
}

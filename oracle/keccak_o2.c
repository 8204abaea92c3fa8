/*
 * Lane-level scalar oracle for batch SHA-3 (Keccak-f[1600] sponge).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into its own shared
 * library for the tests, the smoke check and the CPU-baseline leg of the
 * benchmark.  It shares no code, header, table or constant generator with
 * the HIP library, and nothing in the product path links or loads it.
 *
 * The same definitions as the bit-level oracle, held at lane granularity:
 * lane (x, y) of the 5x5x64 state (Section 3.1, eq. 1, A[x,y,z] =
 * S[64(5y+x)+z]) is the 64-bit word whose bit z is S[64(5y+x)+z]; with the
 * least-significant-bit-first byte convention that word is the little-endian
 * uint64 at byte 8(x+5y) of the 200-byte state.  Plain loops, no SIMD, no
 * unrolling, no fused steps.  Readings (all from FIPS 202, which the paper
 * summarises): rho rotates each lane left in place by (t+1)(t+2)/2 mod 64
 * along the (x, y) walk; pad10*1 uses j = (-m-2) mod x; iota sets RC bits
 * 2^j - 1 for j = 0..6 from the FIPS 202 Algorithm 5 LFSR.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Lane index of (x, y): eq. 1 orders lanes by 5y + x. */
#define LANE(x, y) ((x) + 5 * (y))

static uint64_t rotl64(uint64_t v, unsigned s) {
  s &= 63u;
  return s ? (v << s) | (v >> (64u - s)) : v;
}

/* rc(t), FIPS 202 Algorithm 5 (the paper names only "an LFSR"). */
static int rc_bit(int t) {
  int R[9];
  int i, k;
  t %= 255;
  if (t == 0) return 1;
  for (i = 0; i < 8; ++i) R[i] = (i == 0);
  for (k = 0; k < t; ++k) {
    for (i = 8; i > 0; --i) R[i] = R[i - 1]; /* R = 0 || R */
    R[0] = 0;
    R[0] ^= R[8];
    R[4] ^= R[8];
    R[5] ^= R[8];
    R[6] ^= R[8];
  }
  return R[0];
}

/* Constants derived from their definitions once, at first use. */
static uint64_t g_rc[24];        /* eq. 8, l = 6: bits 2^j - 1, j = 0..6 */
static unsigned g_rho_off[25];   /* Definition 2 walk */
static pthread_once_t g_once = PTHREAD_ONCE_INIT;

static void init_constants(void) {
  int ir, j, t, x, y;
  for (ir = 0; ir < 24; ++ir) {
    uint64_t RC = 0;
    for (j = 0; j <= 6; ++j)
      if (rc_bit(j + 7 * ir)) RC |= (uint64_t)1 << ((1u << j) - 1u);
    g_rc[ir] = RC;
  }
  memset(g_rho_off, 0, sizeof g_rho_off);
  x = 1;
  y = 0;
  for (t = 0; t < 24; ++t) {
    int nx, ny;
    g_rho_off[LANE(x, y)] = (unsigned)(((t + 1) * (t + 2) / 2) % 64);
    nx = y;
    ny = (2 * x + 3 * y) % 5;
    x = nx;
    y = ny;
  }
}

static void theta(uint64_t A[25]) {
  uint64_t C[5], D[5];
  int x, y;
  for (x = 0; x < 5; ++x)
    C[x] = A[LANE(x, 0)] ^ A[LANE(x, 1)] ^ A[LANE(x, 2)] ^ A[LANE(x, 3)] ^ A[LANE(x, 4)];
  /* eq. 3: C[x+1, z-1] is lane C[x+1] rotated one position towards higher z */
  for (x = 0; x < 5; ++x) D[x] = C[(x + 4) % 5] ^ rotl64(C[(x + 1) % 5], 1);
  for (x = 0; x < 5; ++x)
    for (y = 0; y < 5; ++y) A[LANE(x, y)] ^= D[x];
}

static void rho(uint64_t A[25]) {
  int i;
  for (i = 0; i < 25; ++i) A[i] = rotl64(A[i], g_rho_off[i]);
}

static void pi(uint64_t A[25]) {
  uint64_t B[25];
  int x, y;
  for (x = 0; x < 5; ++x)
    for (y = 0; y < 5; ++y) B[LANE(x, y)] = A[LANE((x + 3 * y) % 5, x)];
  memcpy(A, B, sizeof B);
}

static void chi(uint64_t A[25]) {
  uint64_t B[25];
  int x, y;
  for (x = 0; x < 5; ++x)
    for (y = 0; y < 5; ++y)
      B[LANE(x, y)] = A[LANE(x, y)] ^ (~A[LANE((x + 1) % 5, y)] & A[LANE((x + 2) % 5, y)]);
  memcpy(A, B, sizeof B);
}

static void iota(uint64_t A[25], int ir) { A[LANE(0, 0)] ^= g_rc[ir]; }

/* Keccak-f[1600] = Keccak-p[1600, 24], rounds 0..23 of Rnd (eq. 10). */
void o2_keccak_f1600(uint64_t A[25]) {
  int ir;
  pthread_once(&g_once, init_constants);
  for (ir = 0; ir < 24; ++ir) {
    theta(A);
    rho(A);
    pi(A);
    chi(A);
    iota(A, ir);
  }
}

static uint64_t load_le64(const uint8_t *p) {
  uint64_t v = 0;
  int i;
  for (i = 7; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}

static void store_le64(uint8_t *p, uint64_t v) {
  int i;
  for (i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

/*
 * Keccak[c](N, d) for a byte-aligned message M and a bit suffix given as a
 * byte `suffix` holding `suffix_bits` bits (SHA-3: bits 0,1 -> 0x02 with 2
 * bits; SHAKE: 1111 -> 0x0F with 4 bits).  The sponge (Section 3.2) absorbs
 * P = M || suffix || pad10*1 block by block and squeezes out_len bytes.
 */
static void sponge_bytes(int rate, const uint8_t *msg, uint64_t len, uint8_t suffix,
                         int suffix_bits, uint8_t *out, uint64_t out_len) {
  uint64_t A[25];
  uint8_t block[200];
  uint64_t pos = 0, produced = 0;
  int i;
  memset(A, 0, sizeof A);
  /* full message blocks */
  while (len - pos >= (uint64_t)rate) {
    for (i = 0; i < rate / 8; ++i) A[i] ^= load_le64(msg + pos + 8 * i);
    o2_keccak_f1600(A);
    pos += (uint64_t)rate;
  }
  /* last block: message tail, suffix bits, then pad10*1; the first pad bit
     follows the suffix bits, the last pad bit is bit 8*rate-1 */
  memset(block, 0, sizeof block);
  memcpy(block, msg + pos, (size_t)(len - pos));
  block[len - pos] = (uint8_t)(suffix | (1u << suffix_bits));
  block[rate - 1] ^= 0x80u;
  for (i = 0; i < rate / 8; ++i) A[i] ^= load_le64(block + 8 * i);
  o2_keccak_f1600(A);
  /* squeeze */
  for (;;) {
    uint8_t buf[200];
    uint64_t take;
    for (i = 0; i < 25; ++i) store_le64(buf + 8 * i, A[i]);
    take = out_len - produced < (uint64_t)rate ? out_len - produced : (uint64_t)rate;
    memcpy(out + produced, buf, (size_t)take);
    produced += take;
    if (produced >= out_len) break;
    o2_keccak_f1600(A);
  }
}

/* SHA3-d (eqs. 13-16): c = 2d, rate = 200 - d/4 bytes, suffix 01. */
int o2_sha3(int d_bits, const uint8_t *msg, uint64_t len, uint8_t *out) {
  if (d_bits != 224 && d_bits != 256 && d_bits != 384 && d_bits != 512) return -1;
  sponge_bytes(200 - d_bits / 4, msg, len, 0x02u, 2, out, (uint64_t)(d_bits / 8));
  return 0;
}

/* SHAKE128/256 (eqs. 17-18): c = 2 * security, suffix 1111. */
int o2_shake(int security, const uint8_t *msg, uint64_t len, uint8_t *out, uint64_t out_len) {
  if (security != 128 && security != 256) return -1;
  sponge_bytes(200 - security / 4, msg, len, 0x0Fu, 4, out, out_len);
  return 0;
}

/* ----------------------------------------------------------------------- */
/* Batch mode (Section 4): one digest per (offset, length) slice.          */
/* ----------------------------------------------------------------------- */

typedef struct {
  const uint8_t *data;
  const uint64_t *offsets, *lengths;
  const uint8_t *variants; /* NULL: every message uses d_bits */
  int d_bits;
  uint64_t begin, end, out_stride;
  uint8_t *out;
} batch_job;

static const int k_variant_bits[4] = {224, 256, 384, 512};

static void *batch_worker(void *arg) {
  batch_job *j = (batch_job *)arg;
  uint64_t i;
  for (i = j->begin; i < j->end; ++i) {
    int d = j->variants ? k_variant_bits[j->variants[i] & 3] : j->d_bits;
    uint8_t *o = j->out + i * j->out_stride;
    if (j->variants) memset(o, 0, (size_t)j->out_stride);
    o2_sha3(d, j->data + j->offsets[i], j->lengths[i], o);
  }
  return NULL;
}

static int run_batch(const uint8_t *data, const uint64_t *offsets, const uint64_t *lengths,
                     const uint8_t *variants, int d_bits, uint64_t n, uint8_t *out,
                     uint64_t out_stride, int threads) {
  pthread_t tid[256];
  batch_job jobs[256];
  int started[256];
  int t;
  if (threads < 1) threads = 1;
  if (threads > 256) threads = 256;
  if ((uint64_t)threads > n) threads = n ? (int)n : 1;
  pthread_once(&g_once, init_constants);
  for (t = 0; t < threads; ++t) {
    jobs[t].data = data;
    jobs[t].offsets = offsets;
    jobs[t].lengths = lengths;
    jobs[t].variants = variants;
    jobs[t].d_bits = d_bits;
    jobs[t].begin = n * (uint64_t)t / (uint64_t)threads;
    jobs[t].end = n * (uint64_t)(t + 1) / (uint64_t)threads;
    jobs[t].out_stride = out_stride;
    jobs[t].out = out;
    started[t] = 0;
  }
  for (t = 1; t < threads; ++t)
    started[t] = pthread_create(&tid[t], NULL, batch_worker, &jobs[t]) == 0;
  batch_worker(&jobs[0]);
  for (t = 1; t < threads; ++t) {
    if (started[t])
      pthread_join(tid[t], NULL);
    else
      batch_worker(&jobs[t]); /* a thread that could not start: run its share here */
  }
  return 0;
}

int o2_sha3_batch(int d_bits, const uint8_t *data, const uint64_t *offsets,
                  const uint64_t *lengths, uint64_t n, uint8_t *out, int threads) {
  if (d_bits != 224 && d_bits != 256 && d_bits != 384 && d_bits != 512) return -1;
  return run_batch(data, offsets, lengths, NULL, d_bits, n, out, (uint64_t)(d_bits / 8), threads);
}

/* Mixed variants: variants[i] in 0..3 selects SHA3-224/256/384/512; every
   output slot is 64 bytes, zero past the digest. */
int o2_sha3_batch_mixed(const uint8_t *variants, const uint8_t *data, const uint64_t *offsets,
                        const uint64_t *lengths, uint64_t n, uint8_t *out, int threads) {
  uint64_t i;
  for (i = 0; i < n; ++i)
    if (variants[i] > 3) return -1;
  return run_batch(data, offsets, lengths, variants, 0, n, out, 64, threads);
}

/*
 * Tree mode (Section 4): leaves are consecutive leaf_size-byte chunks (the
 * last may be short; an empty input is one empty leaf), parents hash
 * left || right, an unpaired last node is carried up unchanged.
 */
int o2_merkle_root(int d_bits, const uint8_t *data, uint64_t total_len, uint64_t leaf_size,
                   uint8_t *root, int threads) {
  uint64_t n, i, m;
  uint64_t *offs, *lens;
  uint8_t *level, *pair;
  int D = d_bits / 8;
  if (d_bits != 224 && d_bits != 256 && d_bits != 384 && d_bits != 512) return -1;
  if (leaf_size == 0) return -1;
  n = total_len ? (total_len + leaf_size - 1) / leaf_size : 1;
  offs = (uint64_t *)calloc(n, sizeof(uint64_t));
  lens = (uint64_t *)calloc(n, sizeof(uint64_t));
  level = (uint8_t *)malloc(n * (uint64_t)D);
  pair = (uint8_t *)malloc(2 * (size_t)D);
  if (!offs || !lens || !level || !pair) {
    free(offs);
    free(lens);
    free(level);
    free(pair);
    return -2;
  }
  for (i = 0; i < n; ++i) {
    offs[i] = i * leaf_size;
    lens[i] = total_len - offs[i] < leaf_size ? total_len - offs[i] : leaf_size;
    if (total_len == 0) lens[i] = 0;
  }
  o2_sha3_batch(d_bits, data, offs, lens, n, level, threads);
  for (m = n; m > 1; m = (m + 1) / 2) {
    for (i = 0; i + 1 < m; i += 2) {
      memcpy(pair, level + i * D, (size_t)D);
      memcpy(pair + D, level + (i + 1) * D, (size_t)D);
      o2_sha3(d_bits, pair, 2 * (uint64_t)D, level + (i / 2) * D);
    }
    if (m % 2) memmove(level + (m / 2) * D, level + (m - 1) * D, (size_t)D);
  }
  memcpy(root, level, (size_t)D);
  free(offs);
  free(lens);
  free(level);
  free(pair);
  return 0;
}

/*
 * CPU ORACLE (test infrastructure only) -- fixed-accuracy block codec.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this code.  It shares nothing with the HIP path.
 *
 * The paper compresses checkpoints with ZFP in fixed-accuracy mode (absolute
 * tolerance atol; Sec. 1.4 "Data Compression", Sec. 3, appendix): block
 * floating point on 4^d blocks, a decorrelating transform, negabinary
 * integers and embedded bit-plane coding.  ZFP's internals are only cited,
 * and its own transform drops low bits, so this codec is our own design in
 * that family with an exactly invertible integer transform.  Steps, per
 * float32 field of d = 2 or 3 dimensions (last axis contiguous):
 *
 *  1 blocks of 4^d values in C order of block index; a partial block repeats
 *    the last valid sample along each axis (padding is coded, then dropped);
 *  2 subnormal inputs count as zero; emax = max over the block of
 *    (biased exponent - 126), so |x| < 2^emax;
 *  3 minexp = floor(log2 atol) from atol's bits; a block with no non-zero
 *    value, or with emax <= minexp, is coded as the single bit 0 and decodes
 *    to zeros (every |x| < 2^emax <= atol);
 *  4 otherwise: bit 1, 8 bits of emax+127, then i = trunc(x 2^(Q-emax)),
 *    Q = 24, an exact integer shift of the significand;
 *  5 along z, then y, then x: a reversible 4-point lifting
 *      h0=a1-a0; l0=a0+(h0>>1); h1=a3-a2; l1=a2+(h1>>1);
 *      H=l1-l0;  L=l0+(H>>1);   h1-=h0;   h0-=(H>>1);   -> (L, H, h0, h1)
 *    (>> is floor division by 2; the inverse runs the steps backwards);
 *  6 coefficients reordered by total sequency (sum of local indices, ties
 *    in lexicographic order of (x, y, z)), then negabinary
 *    u = (c + 0xAAAAAAAA) ^ 0xAAAAAAAA;
 *  7 lowest coded plane P = max(0, minexp - emax + Q - G), G = 5 (3D) or
 *    4 (2D); top possible plane TP = 31 (3D) or 29 (2D); 3 bits
 *    z = min(7, TP - highest non-empty plane >= P) skip the empty top planes;
 *  8 planes p = TP - z down to P, with n = number of leading coefficients
 *    already significant (starts at 0):
 *      emit bits 0..n-1 of the plane (coefficient 0 first);
 *      if n < 4^d: x = plane >> n;  x == 0 -> emit 0;  else t = highest set
 *      bit of x: emit 1, Elias-gamma(t+1), bits 0..t-1 of x; n += t+1;
 *    Elias-gamma(v): L = floor(log2 v) zeros, a one, then the L low bits
 *    of v; every field is written least significant bit first;
 *  9 stream: 64-byte header, then one u64 bit offset per super-chunk of 256
 *    chunks, one u32 offset per chunk relative to its super-chunk, padding
 *    to 8 bytes, then the payload packed LSB first into little-endian u64
 *    words.  A chunk holds K blocks, K = 16 (3D) or 64 (2D), halved while
 *    the field would have fewer than 16384 chunks (down to K = 1), so small
 *    fields still split into many independently decodable pieces; chunk
 *    c = 64 g + l takes blocks g*64K + j*64 + l, j = 0..K-1, that exist;
 * 10 decode mirrors 8..4; the int32 result is converted to float32 with
 *    round-to-nearest-even and scaled by 2^(emax-Q) through the exponent
 *    field; results below 2^-126 become +0, above FLT_MAX saturate.
 *
 * The guard G makes |x - decoded| <= atol hold whenever
 * emax <= minexp + Q - 1 (the codec then never drops information the float32
 * block cannot hold); see the derivation in the design notes.  A field with
 * a value at or above 2^(minexp + Q - 1) is refused (OR_ERANGE): the Q-bit
 * conversion alone would then lose more than atol.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

#define QBITS 24
#define OR_EINVAL (-1)
#define OR_ECAPACITY (-3)
#define OR_ECORRUPT (-4)
#define OR_ENONFINITE (-5)
#define OR_ERANGE (-8)

typedef struct {
    int ndim;
    long ud[3];         /* dims as given (ud[2] = 1 in 2D) */
    long n[3];          /* dims as (x, y, z); a 2D field is (nx, 1, nz) */
    long nb[3];         /* blocks per axis */
    long nblocks;
    int size;           /* 4^d */
    int tp, guard, kblk;
    long nchunks, nsuper;
} geom_t;

static int geom_init(geom_t *g, int ndim, const long *n)
{
    if (ndim != 2 && ndim != 3) return OR_EINVAL;
    g->ndim = ndim;
    g->nblocks = 1;
    for (int d = 0; d < 3; ++d) {
        g->ud[d] = d < ndim ? n[d] : 1;
        if (g->ud[d] < 1) return OR_EINVAL;
    }
    g->n[0] = g->ud[0];
    g->n[1] = ndim == 3 ? g->ud[1] : 1;
    g->n[2] = ndim == 3 ? g->ud[2] : g->ud[1];
    for (int d = 0; d < 3; ++d) {
        g->nb[d] = (g->n[d] + 3) / 4;
        g->nblocks *= g->nb[d];
    }
    g->size = ndim == 3 ? 64 : 16;
    g->tp = ndim == 3 ? 31 : 29;
    g->guard = ndim == 3 ? 5 : 4;
    g->kblk = ndim == 3 ? 16 : 64;
    while (g->kblk > 1 && (g->nblocks + g->kblk - 1) / g->kblk < 16384) g->kblk >>= 1;
    long per_group = 64L * g->kblk;
    g->nchunks = 64L * ((g->nblocks + per_group - 1) / per_group);
    g->nsuper = (g->nchunks + 255) / 256;
    return 0;
}

static long table_bytes(const geom_t *g)
{
    long t = 8 * g->nsuper + 4 * g->nchunks;
    return (t + 7) & ~7L;
}

static long max_block_bits(const geom_t *g)
{
    int lg = g->ndim == 3 ? 6 : 4;   /* log2 of 4^d */
    int planes = g->tp + 1;
    return 12 + (long)planes * (g->size + 1 + 2 * lg);
}

long or_codec_bound(int ndim, const long *n)
{
    geom_t g;
    if (geom_init(&g, ndim, n)) return OR_EINVAL;
    long words = (g.nblocks * max_block_bits(&g) + 63) / 64;
    return 64 + table_bytes(&g) + 8 * words;
}

/* block b of chunk c, slot j; -1 if it does not exist */
static long chunk_block(const geom_t *g, long c, int j)
{
    long grp = c / 64, lane = c % 64;
    long b = grp * 64L * g->kblk + (long)j * 64 + lane;
    return b < g->nblocks ? b : -1;
}

/* ------------------------------------------------------------ sequency */
static void sequency_order(int ndim, int *perm)
{
    /* perm[s] = local index (C order, z fastest) of the s-th coefficient */
    int size = ndim == 3 ? 64 : 16, s = 0;
    for (int tot = 0; tot <= 3 * ndim; ++tot)
        for (int li = 0; li < size; ++li) {
            int ix, iy, iz;
            if (ndim == 3) { ix = li >> 4; iy = (li >> 2) & 3; iz = li & 3; }
            else { ix = li >> 2; iy = 0; iz = li & 3; }
            if (ix + iy + iz == tot) perm[s++] = li;
        }
    /* candidates with equal total are visited in increasing local index,
     * which is lexicographic (x, y, z) order */
}

/* ------------------------------------------------------------- lifting */
static int32_t asr1(uint32_t v) { return (int32_t)v >> 1; }

void or_lift_fwd4(int32_t *a, int stride)
{
    uint32_t a0 = a[0], a1 = a[stride], a2 = a[2 * stride], a3 = a[3 * stride];
    uint32_t h0 = a1 - a0;
    uint32_t l0 = a0 + (uint32_t)asr1(h0);
    uint32_t h1 = a3 - a2;
    uint32_t l1 = a2 + (uint32_t)asr1(h1);
    uint32_t H = l1 - l0;
    uint32_t L = l0 + (uint32_t)asr1(H);
    h1 = h1 - h0;
    h0 = h0 - (uint32_t)asr1(H);
    a[0] = (int32_t)L; a[stride] = (int32_t)H;
    a[2 * stride] = (int32_t)h0; a[3 * stride] = (int32_t)h1;
}

void or_lift_inv4(int32_t *a, int stride)
{
    uint32_t L = a[0], H = a[stride], h0 = a[2 * stride], h1 = a[3 * stride];
    h0 = h0 + (uint32_t)asr1(H);
    h1 = h1 + h0;
    uint32_t l0 = L - (uint32_t)asr1(H);
    uint32_t l1 = H + l0;
    uint32_t a0 = l0 - (uint32_t)asr1(h0);
    uint32_t a1 = h0 + a0;
    uint32_t a2 = l1 - (uint32_t)asr1(h1);
    uint32_t a3 = h1 + a2;
    a[0] = (int32_t)a0; a[stride] = (int32_t)a1;
    a[2 * stride] = (int32_t)a2; a[3 * stride] = (int32_t)a3;
}

/* whole-block transforms: forward along z, y, x; inverse along x, y, z */
void or_block_fwd(int ndim, int32_t *blk)
{
    if (ndim == 3) {
        for (int i = 0; i < 16; ++i) or_lift_fwd4(blk + 4 * i, 1);            /* z */
        for (int x = 0; x < 4; ++x)
            for (int z = 0; z < 4; ++z) or_lift_fwd4(blk + 16 * x + z, 4);  /* y */
        for (int i = 0; i < 16; ++i) or_lift_fwd4(blk + i, 16);             /* x */
    } else {
        for (int x = 0; x < 4; ++x) or_lift_fwd4(blk + 4 * x, 1);           /* z */
        for (int z = 0; z < 4; ++z) or_lift_fwd4(blk + z, 4);               /* x */
    }
}

void or_block_inv(int ndim, int32_t *blk)
{
    if (ndim == 3) {
        for (int i = 0; i < 16; ++i) or_lift_inv4(blk + i, 16);
        for (int x = 0; x < 4; ++x)
            for (int z = 0; z < 4; ++z) or_lift_inv4(blk + 16 * x + z, 4);
        for (int i = 0; i < 16; ++i) or_lift_inv4(blk + 4 * i, 1);
    } else {
        for (int z = 0; z < 4; ++z) or_lift_inv4(blk + z, 4);
        for (int x = 0; x < 4; ++x) or_lift_inv4(blk + 4 * x, 1);
    }
}

/* ---------------------------------------------------------- bit writer */
typedef struct { uint64_t *w; long cap_bits; long pos; int over; } bw_t;

static void put_bit(bw_t *b, int bit)
{
    if (b->pos >= b->cap_bits) { b->over = 1; return; }
    if (bit) b->w[b->pos >> 6] |= (uint64_t)1 << (b->pos & 63);
    b->pos++;
}

static void put_bits(bw_t *b, uint64_t v, int n)
{
    for (int i = 0; i < n; ++i) put_bit(b, (int)((v >> i) & 1));
}

typedef struct { const uint64_t *w; long nbits; long pos; int bad; } br_t;

static int get_bit(br_t *r)
{
    if (r->pos >= r->nbits) { r->bad = 1; return 0; }
    int v = (int)((r->w[r->pos >> 6] >> (r->pos & 63)) & 1);
    r->pos++;
    return v;
}

static uint64_t get_bits(br_t *r, int n)
{
    uint64_t v = 0;
    for (int i = 0; i < n; ++i) v |= (uint64_t)get_bit(r) << i;
    return v;
}

/* --------------------------------------------------------------- helpers */
static int minexp_of(double atol)
{
    uint64_t bits;
    memcpy(&bits, &atol, 8);
    return (int)((bits >> 52) & 0x7FF) - 1023;   /* atol normal, positive */
}

static int hibit64(uint64_t x)
{
    int t = -1;
    while (x) { ++t; x >>= 1; }
    return t;
}

static int floor_log2(uint64_t v)
{
    return hibit64(v);
}

static void put_gamma(bw_t *b, uint64_t v)
{
    int L = floor_log2(v);
    for (int i = 0; i < L; ++i) put_bit(b, 0);
    put_bit(b, 1);
    put_bits(b, v, L);          /* the L low bits (the top bit is implied) */
}

static uint64_t get_gamma(br_t *r)
{
    int L = 0;
    while (!get_bit(r)) {
        if (r->bad || ++L > 63) { r->bad = 1; return 1; }
    }
    return ((uint64_t)1 << L) | get_bits(r, L);
}

/* ------------------------------------------------------------- encoding */
static void encode_block(const geom_t *g, const float *x, long b,
                         int minexp, const int *perm, bw_t *bw)
{
    long bi[3], rem = b;
    bi[2] = rem % g->nb[2]; rem /= g->nb[2];
    bi[1] = rem % g->nb[1]; rem /= g->nb[1];
    bi[0] = rem;
    uint32_t w[64];
    int size = g->size;
    for (int li = 0; li < size; ++li) {
        long c[3];
        if (g->ndim == 3) { c[0] = li >> 4; c[1] = (li >> 2) & 3; c[2] = li & 3; }
        else { c[0] = li >> 2; c[1] = 0; c[2] = li & 3; }
        long off = 0;
        for (int d = 0; d < 3; ++d) {
            long i = 4 * bi[d] + c[d];
            if (i > g->n[d] - 1) i = g->n[d] - 1;
            off = off * g->n[d] + i;
        }
        memcpy(&w[li], &x[off], 4);
    }
    /* exponent of the block (biased); subnormals count as zero */
    int Emax = 0;
    for (int li = 0; li < size; ++li) {
        int E = (w[li] >> 23) & 0xFF;
        if (E > Emax) Emax = E;
    }
    int emax = Emax - 126;
    if (Emax == 0 || emax <= minexp) { put_bit(bw, 0); return; }
    put_bit(bw, 1);
    put_bits(bw, (uint64_t)(emax + 127), 8);
    /* exact conversion: i = trunc(|x| 2^(Q-emax)) with sign */
    int32_t blk[64];
    for (int li = 0; li < size; ++li) {
        int E = (w[li] >> 23) & 0xFF;
        int32_t v = 0;
        if (E != 0) {
            uint32_t mant = (w[li] & 0x7FFFFFu) | 0x800000u;
            int sh = Emax - E;          /* (E-150) + Q - emax = E - Emax */
            uint32_t mag = sh >= 32 ? 0 : mant >> sh;
            v = (w[li] >> 31) ? -(int32_t)mag : (int32_t)mag;
        }
        blk[li] = v;
    }
    or_block_fwd(g->ndim, blk);
    uint32_t u[64];
    for (int s = 0; s < size; ++s)
        u[s] = ((uint32_t)blk[perm[s]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
    int P = minexp - emax + QBITS - g->guard;
    if (P < 0) P = 0;
    /* planes as bit masks over coefficients (bit s = coefficient s) */
    uint64_t plane[32];
    for (int p = 0; p < 32; ++p) {
        uint64_t m = 0;
        for (int s = 0; s < size; ++s) m |= (uint64_t)((u[s] >> p) & 1) << s;
        plane[p] = m;
    }
    int fp = -1;
    for (int p = 31; p >= P; --p)
        if (plane[p]) { fp = p; break; }
    int z = (fp < 0 || g->tp - fp > 7) ? 7 : g->tp - fp;
    put_bits(bw, (uint64_t)z, 3);
    int n = 0;
    for (int p = g->tp - z; p >= P; --p) {
        uint64_t xp = plane[p];
        put_bits(bw, xp, n);                     /* refinement bits */
        if (n < size) {
            uint64_t xr = xp >> n;
            if (!xr) { put_bit(bw, 0); continue; }
            int t = hibit64(xr);
            put_bit(bw, 1);
            put_gamma(bw, (uint64_t)t + 1);
            put_bits(bw, xr, t);                 /* bits below the top one */
            n += t + 1;
        }
    }
}

static void wr32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void wr64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t rd32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t rd64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

/* returns stream bytes, or a negative error */
long or_compress(const float *x, int ndim, const long *n, double atol,
                 uint8_t *out, long cap)
{
    geom_t g;
    if (geom_init(&g, ndim, n)) return OR_EINVAL;
    if (!(atol > 0) || !isfinite(atol) || atol < 2.2250738585072014e-308)
        return OR_EINVAL;
    long nval = g.n[0] * g.n[1] * g.n[2];
    int minexp = minexp_of(atol);
    /* the fixed-accuracy bound needs every block exponent emax (|x| < 2^emax)
     * at most minexp + Q - 1, i.e. every |x| below 2^(minexp + Q - 1) <= atol 2^23;
     * a larger value loses more than atol to the Q-bit conversion alone */
    int range = 0;
    for (long i = 0; i < nval; ++i) {
        uint32_t w;
        memcpy(&w, &x[i], 4);
        int E = (w >> 23) & 0xFF;
        if (E == 0xFF) return OR_ENONFINITE;
        if (E != 0 && E - 126 > minexp + QBITS - 1) range = 1;
    }
    if (range) return OR_ERANGE;
    int perm[64];
    sequency_order(ndim, perm);
    long hdr = 64 + table_bytes(&g);
    if (cap < hdr) return OR_ECAPACITY;
    memset(out, 0, (size_t)cap);
    bw_t bw = { (uint64_t *)(out + hdr), (cap - hdr) / 8 * 64, 0, 0 };
    uint64_t super_base = 0;
    for (long c = 0; c < g.nchunks; ++c) {
        if (c % 256 == 0) {
            super_base = (uint64_t)bw.pos;
            wr64(out + 64 + 8 * (c / 256), super_base);
        }
        wr32(out + 64 + 8 * g.nsuper + 4 * c, (uint32_t)((uint64_t)bw.pos - super_base));
        for (int j = 0; j < g.kblk; ++j) {
            long b = chunk_block(&g, c, j);
            if (b >= 0) encode_block(&g, x, b, minexp, perm, &bw);
        }
        if (bw.over) return OR_ECAPACITY;
    }
    long words = (bw.pos + 63) / 64;
    long total = hdr + 8 * words;
    memcpy(out, "FWZ1", 4);
    out[4] = 1; out[5] = 0;
    out[6] = (uint8_t)ndim;
    out[7] = QBITS;
    wr32(out + 8, (uint32_t)g.ud[0]);
    wr32(out + 12, (uint32_t)g.ud[1]);
    wr32(out + 16, (uint32_t)g.ud[2]);
    out[20] = (uint8_t)g.guard;
    out[21] = (uint8_t)floor_log2((uint64_t)g.kblk);    /* log2 of blocks per chunk */
    out[22] = (uint8_t)g.tp;
    out[23] = 0;
    uint64_t ab;
    memcpy(&ab, &atol, 8);
    wr64(out + 24, ab);
    wr32(out + 32, (uint32_t)minexp);
    wr32(out + 36, (uint32_t)g.nchunks);
    wr64(out + 40, (uint64_t)g.nblocks);
    wr64(out + 48, (uint64_t)bw.pos);
    wr64(out + 56, (uint64_t)total);
    return total;
}

/* ------------------------------------------------------------- decoding */
static float scale_to_float(int32_t i, int emax)
{
    float f = (float)i;                 /* round to nearest even */
    if (i == 0) return 0.0f;
    uint32_t bits;
    memcpy(&bits, &f, 4);
    int E = (int)((bits >> 23) & 0xFF) + emax - QBITS;
    if (E <= 0) bits = 0;
    else if (E >= 255) bits = (bits & 0x80000000u) | 0x7F7FFFFFu;
    else bits = (bits & ~(0xFFu << 23)) | ((uint32_t)E << 23);
    memcpy(&f, &bits, 4);
    return f;
}

static int decode_block(const geom_t *g, br_t *br, int minexp, const int *perm,
                        float *x, long b)
{
    int size = g->size;
    float vals[64];
    if (!get_bit(br)) {
        for (int li = 0; li < size; ++li) vals[li] = 0.0f;
    } else {
        int emax = (int)get_bits(br, 8) - 127;
        int z = (int)get_bits(br, 3);
        int P = minexp - emax + QBITS - g->guard;
        if (P < 0) P = 0;
        uint64_t plane[32] = { 0 };
        int n = 0;
        for (int p = g->tp - z; p >= P; --p) {
            uint64_t xp = get_bits(br, n);
            if (n < size && get_bit(br)) {
                uint64_t v = get_gamma(br);
                int t = (int)(v - 1);
                if (t > size - 1 - n) return OR_ECORRUPT;
                uint64_t raw = get_bits(br, t);
                xp |= (((uint64_t)1 << t) | raw) << n;
                n += t + 1;
            }
            if (br->bad) return OR_ECORRUPT;
            plane[p] = xp;
        }
        int32_t blk[64];
        for (int s = 0; s < size; ++s) {
            uint32_t u = 0;
            for (int p = 0; p < 32; ++p) u |= (uint32_t)((plane[p] >> s) & 1) << p;
            blk[perm[s]] = (int32_t)((u ^ 0xAAAAAAAAu) - 0xAAAAAAAAu);
        }
        or_block_inv(g->ndim, blk);
        for (int li = 0; li < size; ++li) vals[li] = scale_to_float(blk[li], emax);
    }
    if (br->bad) return OR_ECORRUPT;
    long bi[3], rem = b;
    bi[2] = rem % g->nb[2]; rem /= g->nb[2];
    bi[1] = rem % g->nb[1]; rem /= g->nb[1];
    bi[0] = rem;
    for (int li = 0; li < size; ++li) {
        long c[3];
        if (g->ndim == 3) { c[0] = li >> 4; c[1] = (li >> 2) & 3; c[2] = li & 3; }
        else { c[0] = li >> 2; c[1] = 0; c[2] = li & 3; }
        long off = 0;
        int inside = 1;
        for (int d = 0; d < 3; ++d) {
            long i = 4 * bi[d] + c[d];
            if (i > g->n[d] - 1) inside = 0;
            off = off * g->n[d] + i;
        }
        if (inside) x[off] = vals[li];
    }
    return 0;
}

int or_decompress(const uint8_t *s, long nbytes, float *x, int ndim,
                  const long *n)
{
    geom_t g;
    if (geom_init(&g, ndim, n)) return OR_EINVAL;
    if (nbytes < 64 || memcmp(s, "FWZ1", 4) != 0 || s[4] != 1 || s[5] != 0)
        return OR_ECORRUPT;
    if (s[6] != ndim || s[7] != QBITS || s[20] != g.guard || s[22] != g.tp ||
        s[21] != floor_log2((uint64_t)g.kblk))
        return OR_ECORRUPT;
    for (int d = 0; d < 3; ++d)
        if ((long)rd32(s + 8 + 4 * d) != g.ud[d]) return OR_ECORRUPT;
    if ((long)rd32(s + 36) != g.nchunks || (long)rd64(s + 40) != g.nblocks)
        return OR_ECORRUPT;
    int minexp = (int32_t)rd32(s + 32);
    uint64_t pbits = rd64(s + 48);
    long hdr = 64 + table_bytes(&g);
    long words = (long)((pbits + 63) / 64);
    if ((long)rd64(s + 56) != hdr + 8 * words || nbytes < hdr + 8 * words)
        return OR_ECORRUPT;
    int perm[64];
    sequency_order(ndim, perm);
    const uint64_t *payload = (const uint64_t *)(s + hdr);
    for (long c = 0; c < g.nchunks; ++c) {
        uint64_t start = rd64(s + 64 + 8 * (c / 256)) + rd32(s + 64 + 8 * g.nsuper + 4 * c);
        if (start > pbits) return OR_ECORRUPT;
        br_t br = { payload, (long)pbits, (long)start, 0 };
        for (int j = 0; j < g.kblk; ++j) {
            long b = chunk_block(&g, c, j);
            if (b < 0) continue;
            int rc = decode_block(&g, &br, minexp, perm, x, b);
            if (rc) return rc;
        }
    }
    return 0;
}

/*
 * ms_oracle.c -- plain, slow, sequential CPU oracle for MergeShuffle
 * (Bacher, Bodini, Hollender, Lumbroso, arXiv 1508.03167).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only tests/, the package's smoke() entry and the
 * cpu_baseline leg of bench.py use it.  It shares no code with the HIP
 * library under paper_1508_03167_amd/csrc (own Philox, own bounded draw,
 * own Fisher-Yates, own Merge, own top-level routine).
 *
 * What it computes (each function cites the passage it follows):
 *   - Fisher-Yates shuffle, descending, j uniform in {0..i}   (Algorithm 1)
 *   - Merge of two shuffled adjacent ranges                    (Algorithm 2,
 *     Section 1.1, and the merge() listing of Appendix A.1)
 *   - the MergeShuffle top-level routine: c = least c with (n >> c) <= cutoff, q = 2^c
 *     blocks [n*i/q, n*(i+1)/q), Fisher-Yates per block, then merges of
 *     adjacent blocks level by level                          (Algorithm
 *     MergeShuffle, Section 1; shuffle() listing of Appendix A.2)
 *   - random integers from fair bits by the Fast Dice Roller, the optimal
 *     bounded draw of [Lumbroso13] that the paper says its simulations use
 *     (introduction, paragraph on the random-bit model)
 *   - the random-bit count: one bit per coin flip of Merge (including the
 *     flip that finds an exhausted side), plus every bit the bounded draws
 *     consume (Lemma 2; Section 1.2; the bit-count Table of Section 3)
 *
 * Readings where the paper is silent (the paper names no generator):
 *   - Generator: Philox-4x32-10 (Salmon et al., SC'11), key = (lo32(seed),
 *     hi32(seed)).  Counter words (c0,c1,c2,c3), c3 = domain<<28 | sub.
 *   - FLIP(L,m,t): bit t of the coin-flip word of merge m at level L is bit
 *     (t & 31) of word ((t>>5)&3) of Philox((t>>7, m, L, 1<<28)).
 *   - DRAW(L,u,d): the d-th bounded draw of unit u (leaf block u at L = 0,
 *     merge u at level L >= 1) reads bits most-significant first from word
 *     (d&3) of Philox((d>>2, u, L, 2<<28)); if those 32 bits run out it
 *     continues with blocks Philox((d, u, L, (3<<28)|j)), j = 0,1,..., words
 *     x0..x3 in order, each most-significant bit first.
 *   - Element placement during the coin-flip loop: stable interleave
 *     (reading "R2"): output slot a+b takes A[a] on a 0 and B[b] on a 1.
 *     The in-place swap form of the printed listing (reading "R1") is kept
 *     for cross-checks: both consume the same bits and the same draws, and
 *     put the same B elements at the same slots.
 *   - random_int(1) consumes no bit.
 *
 * Values are unsigned 32-bit words, as in the printed listings; record
 * shuffles are checked by applying the index permutation computed here.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_R2 0
#define ORACLE_R1 1
#define ORACLE_BALANCED 2

/* ------------------------------------------------------------------ */
/* Philox-4x32-10, Salmon, Moraes, Dror, Shaw (SC'11), Section 4.     */
/* ------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL0 = 0xD2511F53u;
static const uint32_t PHILOX_MUL1 = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_WEYL1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)PHILOX_MUL0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_MUL1 * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_WEYL0;
        k1 += PHILOX_WEYL1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Random source: random_bit() and random_int(k) of the listings.      */
/* Either the Philox streams above, or a scripted choice list used by  */
/* the brute-force enumerator (bits 0/1 and integers in [0,k)).        */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint64_t bits;            /* fair bits consumed so far */
    /* one-block memo so a sequential reader does not recompute Philox */
    uint32_t memo_ctr[4];
    uint32_t memo_val[4];
    int memo_ok;
    /* scripted mode */
    const uint32_t *script;
    uint32_t script_len;
    uint32_t script_pos;
    uint64_t need;            /* range asked for when the script ran out */
    int starved;
} osrc;

static void src_block(osrc *s, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    if (!(s->memo_ok && s->memo_ctr[0] == c0 && s->memo_ctr[1] == c1 &&
          s->memo_ctr[2] == c2 && s->memo_ctr[3] == c3)) {
        uint32_t ctr[4] = {c0, c1, c2, c3};
        uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
        oracle_philox4x32_10(ctr, key, s->memo_val);
        memcpy(s->memo_ctr, ctr, sizeof ctr);
        s->memo_ok = 1;
    }
    memcpy(out, s->memo_val, 4 * sizeof(uint32_t));
}

static uint32_t script_next(osrc *s, uint64_t range)
{
    if (s->script_pos >= s->script_len) {
        if (!s->starved) { s->starved = 1; s->need = range; }
        return 0;
    }
    return s->script[s->script_pos++];
}

/* FLIP(L, m, t): the t-th coin flip of merge m at level L. */
static int random_bit(osrc *s, uint32_t L, uint32_t m, uint64_t t)
{
    uint32_t w[4];
    if (s->script) return (int)script_next(s, 2);
    src_block(s, (uint32_t)(t >> 7), m, L, 1u << 28, w);
    s->bits += 1;
    return (int)((w[(t >> 5) & 3] >> (t & 31)) & 1u);
}

/* Bit reader over DRAW(L, u, d): primary word, then continuation blocks. */
typedef struct {
    osrc *s;
    uint32_t L, u, d;
    uint32_t word;      /* current word */
    int left;           /* unread bits in word */
    uint32_t cont_j;    /* next continuation block index */
    uint32_t cont_w[4];
    int cont_idx;       /* next word of cont_w to use, 4 = none loaded */
} draw_reader;

static uint32_t draw_next_bit(draw_reader *r)
{
    if (r->left == 0) {
        if (r->cont_idx == 4) {
            src_block(r->s, r->d, r->u, r->L, (3u << 28) | r->cont_j, r->cont_w);
            r->cont_j += 1;
            r->cont_idx = 0;
        }
        r->word = r->cont_w[r->cont_idx++];
        r->left = 32;
    }
    r->left -= 1;
    return (r->word >> r->left) & 1u;
}

/*
 * Fast Dice Roller [Lumbroso13]: uniform integer in {0..k-1} from fair bits.
 * v tracks the size of the range the bits read so far can describe, c the
 * value they describe; once v >= k a value c < k is accepted, otherwise the
 * excess v-k is kept as a smaller range and drawing continues.
 */
static uint64_t random_int(osrc *s, uint32_t L, uint32_t u, uint64_t d, uint64_t k)
{
    draw_reader r;
    uint32_t prim[4];
    uint64_t v = 1, c = 0;
    if (s->script) return k <= 1 ? (script_next(s, 1), 0) : script_next(s, k);
    if (k <= 1) return 0;
    r.s = s; r.L = L; r.u = u; r.d = (uint32_t)d;
    src_block(s, (uint32_t)(d >> 2), u, L, 2u << 28, prim);
    r.word = prim[d & 3];
    r.left = 32;
    r.cont_j = 0;
    r.cont_idx = 4;
    for (;;) {
        v = v << 1;
        c = (c << 1) | draw_next_bit(&r);
        s->bits += 1;
        if (v >= k) {
            if (c < k) return c;
            v -= k;
            c -= k;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: Fisher-Yates, i from n-1 down to 0, j in {0..i}.       */
/* Step i = 0 has a single choice and is skipped (0 bits).             */
/* ------------------------------------------------------------------ */
static void fisher_yates(osrc *s, uint32_t *t, uint64_t n, uint32_t unit)
{
    uint64_t i;
    for (i = n; i-- > 1;) {
        uint64_t j = random_int(s, 0, unit, i, i + 1);
        uint32_t tmp = t[i]; t[i] = t[j]; t[j] = tmp;
    }
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 / Appendix A.1 merge(): shuffled merge of A = t[0,n1)   */
/* and B = t[n1,n1+n2).  Coin-flip loop (0 takes from A, 1 from B, a   */
/* flip on an exhausted side ends the loop), then a Fisher-Yates       */
/* insertion of every remaining slot i with a partner drawn in [0,i].  */
/* Returns P, the number of slots the coin-flip loop filled.           */
/* ------------------------------------------------------------------ */
static uint64_t merge_r2(osrc *s, uint32_t *t, uint64_t n1, uint64_t n2,
                         uint32_t L, uint32_t m, uint32_t *tmp)
{
    const uint32_t *A = t, *B = t + n1;
    uint64_t n = n1 + n2, a = 0, b = 0, step = 0, P, i;
    for (;;) {
        int w = random_bit(s, L, m, step);
        step += 1;
        if (w == 0) {
            if (a == n1) break;
            tmp[a + b] = A[a];
            a += 1;
        } else {
            if (b == n2) break;
            tmp[a + b] = B[b];
            b += 1;
        }
    }
    P = a + b;
    /* the side that is not exhausted keeps its order */
    while (a < n1) { tmp[a + b] = A[a]; a += 1; }
    while (b < n2) { tmp[a + b] = B[b]; b += 1; }
    for (i = P; i < n; i++) {
        uint64_t j = random_int(s, L, m, i, i + 1);
        uint32_t x = tmp[i]; tmp[i] = tmp[j]; tmp[j] = x;
    }
    memcpy(t, tmp, n * sizeof(uint32_t));
    return P;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 with the in-place placement of the appendix's merge     */
/* (Appendix A.1): the coin-flip loop and the insertion loop are those */
/* of Algorithm 2, only where the unplaced A elements sit differs.     */
/* Working in place, A's unplaced elements occupy the slots between    */
/* the output cursor and the head of B; a 1 flip moves B's head to the */
/* output cursor and the A element it displaces to the end of that     */
/* run.  So A's unplaced elements form a queue: a 0 flip places the    */
/* queue's front, a 1 flip places B's next element and sends the       */
/* queue's front to its back.  When B runs out the queue follows in    */
/* queue order; when A runs out, the rest of B in its order.           */
/* The queue is a circular buffer of A's indices.                      */
/* ------------------------------------------------------------------ */
static uint64_t merge_r1(osrc *s, uint32_t *t, uint64_t n1, uint64_t n2,
                         uint32_t L, uint32_t m, uint32_t *tmp, uint32_t *queue)
{
    const uint32_t *A = t, *B = t + n1;
    uint64_t n = n1 + n2, front = 0, len = n1, b = 0, k = 0, step = 0, P, i;
    for (i = 0; i < n1; i++) queue[i] = (uint32_t)i;
    for (;;) {
        int w = random_bit(s, L, m, step);
        step += 1;
        if (w == 0) {
            if (len == 0) break;
            tmp[k++] = A[queue[front]];
            front = front + 1 == n1 ? 0 : front + 1;
            len -= 1;
        } else {
            if (b == n2) break;
            tmp[k++] = B[b++];
            if (len > 0) {
                /* the front goes to the back: the slot after the last */
                uint64_t back = front + len;
                if (back >= n1) back -= n1;
                queue[back] = queue[front];
                front = front + 1 == n1 ? 0 : front + 1;
            }
        }
    }
    P = k;
    while (len > 0) {
        tmp[k++] = A[queue[front]];
        front = front + 1 == n1 ? 0 : front + 1;
        len -= 1;
    }
    while (b < n2) tmp[k++] = B[b++];
    for (i = P; i < n; i++) {
        uint64_t j = random_int(s, L, m, i, i + 1);
        uint32_t x = tmp[i]; tmp[i] = tmp[j]; tmp[j] = x;
    }
    memcpy(t, tmp, n * sizeof(uint32_t));
    return P;
}

/* ------------------------------------------------------------------ */
/* BalancedShuffle's merge (Section 2): the two shuffled halves are    */
/* interleaved by a word drawn uniformly from C(n1+n2, n1) -- n1 0's   */
/* (take from A) and n2 1's (take from B) -- each half keeping its     */
/* order; Section 2.2 shows this map from S_n1 x S_n2 x C(n1+n2, n1)   */
/* to S_(n1+n2) is a bijection, so the result is uniform.              */
/*                                                                    */
/* The paper takes the word from the generator of [BaBoJa14], which it */
/* does not describe.  Reading used here: the word is the sequence of  */
/* side labels (0 = A, 1 = B) that Algorithm 2 produces when it merges */
/* the labels 0^n1 and 1^n2 -- coin flips until a flip falls on an    */
/* exhausted side, the rest of the other side, then the Fisher-Yates   */
/* insertion of slots P..N-1 with partners drawn in [0, i].  Lemma 1   */
/* makes Algorithm 2's output a uniform arrangement of any two         */
/* uniformly shuffled halves, so the labels it leaves are a uniform    */
/* element of C(n1+n2, n1).  It uses the same bits as Algorithm 2.     */
/* ------------------------------------------------------------------ */
static uint64_t merge_balanced(osrc *s, uint32_t *t, uint64_t n1, uint64_t n2,
                               uint32_t L, uint32_t m, uint32_t *tmp, uint8_t *word)
{
    const uint32_t *A = t, *B = t + n1;
    uint64_t n = n1 + n2, a = 0, b = 0, step = 0, P, i, k;
    /* the balanced word */
    for (;;) {
        int w = random_bit(s, L, m, step);
        step += 1;
        if (w == 0) {
            if (a == n1) break;
            word[a + b] = 0;
            a += 1;
        } else {
            if (b == n2) break;
            word[a + b] = 1;
            b += 1;
        }
    }
    P = a + b;
    while (a < n1) { word[a + b] = 0; a += 1; }
    while (b < n2) { word[a + b] = 1; b += 1; }
    for (i = P; i < n; i++) {
        uint64_t j = random_int(s, L, m, i, i + 1);
        uint8_t x = word[i]; word[i] = word[j]; word[j] = x;
    }
    /* the interleave it defines: slot k takes the next element of the
     * side its letter names */
    a = b = 0;
    for (k = 0; k < n; k++) {
        if (word[k] == 0) tmp[k] = A[a++];
        else tmp[k] = B[b++];
    }
    memcpy(t, tmp, n * sizeof(uint32_t));
    return P;
}

/* ------------------------------------------------------------------ */
/* Algorithm MergeShuffle: split into two halves, shuffle each, merge  */
/* them (Algorithm 2); below the cutoff, Fisher-Yates (Algorithm 1).   */
/* Unrolled bottom up: the recursion's leaves are the 2^c blocks of a  */
/* c-level split, every level merging pairs of neighbouring blocks.    */
/* Where each half ends is the reading of the partition of Appendix    */
/* A.2: block i is [floor(n*i/2^c), floor(n*(i+1)/2^c)).               */
/* ------------------------------------------------------------------ */
static uint32_t levels_for(uint64_t n, uint64_t cutoff)
{
    uint32_t c = 0;
    while ((n >> c) > cutoff) c += 1;
    return c;
}

uint32_t oracle_levels(uint64_t n, uint64_t cutoff) { return levels_for(n, cutoff); }

/* Blocks are [n*i/q, n*(i+1)/q) with q = 2^c, in 64-bit arithmetic. */
static uint64_t bound(uint64_t n, uint64_t i, uint32_t c) { return (n * i) >> c; }

static uint64_t run_shuffle(osrc *proto, uint32_t *t, uint64_t n, uint64_t cutoff,
                            int placement, int threads)
{
    uint32_t c, L;
    uint64_t q, i, bits = 0;
    uint32_t *tmp = NULL, *queue = NULL;
    uint8_t *word = NULL;
    (void)threads;
    if (n <= 1 || cutoff < 1) return 0;
    c = levels_for(n, cutoff);
    q = (uint64_t)1 << c;
    tmp = (uint32_t *)malloc(n * sizeof(uint32_t));
    if (!tmp) return ~(uint64_t)0;
    if (placement == ORACLE_BALANCED) {
        word = (uint8_t *)malloc(n);
        if (!word) { free(tmp); return ~(uint64_t)0; }
    } else if (placement != ORACLE_R2) {
        queue = (uint32_t *)malloc(n * sizeof(uint32_t));
        if (!queue) { free(tmp); return ~(uint64_t)0; }
    }

    /* leaves: one Fisher-Yates per block (the blocks are independent) */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bits) num_threads(threads > 0 ? threads : omp_get_max_threads()) if (!proto->script)
#endif
    for (i = 0; i < q; i++) {
        osrc s = *proto;
        s.bits = 0; s.memo_ok = 0;
        fisher_yates(proto->script ? proto : &s, t + bound(n, i, c),
                     bound(n, i + 1, c) - bound(n, i, c), (uint32_t)i);
        bits += s.bits;
    }

    /* merge levels: level L merges pairs of blocks of 2^(L-1) leaves */
    for (L = 1; L <= c; L++) {
        uint64_t p = (uint64_t)1 << (L - 1);
        uint64_t nmerge = q >> L, m;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bits) num_threads(threads > 0 ? threads : omp_get_max_threads()) if (!proto->script)
#endif
        for (m = 0; m < nmerge; m++) {
            osrc s = *proto;
            uint64_t i0 = m * 2 * p;
            uint64_t j = bound(n, i0, c), k = bound(n, i0 + p, c), l = bound(n, i0 + 2 * p, c);
            osrc *sp = proto->script ? proto : &s;
            s.bits = 0; s.memo_ok = 0;
            if (placement == ORACLE_R2)
                merge_r2(sp, t + j, k - j, l - k, L, (uint32_t)m, tmp + j);
            else if (placement == ORACLE_BALANCED)
                merge_balanced(sp, t + j, k - j, l - k, L, (uint32_t)m, tmp + j, word + j);
            else
                merge_r1(sp, t + j, k - j, l - k, L, (uint32_t)m, tmp + j, queue + j);
            bits += s.bits;
        }
    }
    free(tmp);
    free(word);
    free(queue);
    return bits;
}

/* Shuffle t[0..n) in place with seed; returns the number of fair bits. */
uint64_t oracle_shuffle_u32(uint32_t *t, uint64_t n, uint64_t cutoff, uint64_t seed,
                            int placement, int threads)
{
    osrc s;
    memset(&s, 0, sizeof s);
    s.seed = seed;
    return run_shuffle(&s, t, n, cutoff, placement, threads);
}

/* out[i] = i, then shuffle: the random permutation of size n. */
uint64_t oracle_permutation(uint32_t *out, uint64_t n, uint64_t cutoff, uint64_t seed, int threads)
{
    uint64_t i;
    for (i = 0; i < n; i++) out[i] = (uint32_t)i;
    return oracle_shuffle_u32(out, n, cutoff, seed, ORACLE_R2, threads);
}

/*
 * Scripted run for the brute-force enumerator: random_bit() returns the next
 * script entry (0/1) and random_int(k) the next entry (0..k-1).  Returns 0 if
 * the script sufficed, else 1 with *need = the range of the first missing
 * choice (2 for a bit, k for an integer).  random_int(1) also reads an entry
 * (always 0) so that every call is visible to the enumerator.
 */
int oracle_shuffle_scripted(uint32_t *t, uint64_t n, uint64_t cutoff, int placement,
                            const uint32_t *script, uint32_t script_len,
                            uint32_t *consumed, uint64_t *need)
{
    osrc s;
    memset(&s, 0, sizeof s);
    s.script = script;
    s.script_len = script_len;
    run_shuffle(&s, t, n, cutoff, placement, 1);
    if (consumed) *consumed = s.script_pos;
    if (need) *need = s.starved ? s.need : 0;
    return s.starved;
}

/* One Merge with a script; returns P (or ~0 if the script ran out). */
uint64_t oracle_merge_scripted(uint32_t *t, uint64_t n1, uint64_t n2, int placement,
                               const uint32_t *script, uint32_t script_len, uint64_t *need)
{
    osrc s;
    uint64_t P;
    uint32_t *tmp, *queue;
    uint8_t *word;
    memset(&s, 0, sizeof s);
    s.script = script;
    s.script_len = script_len;
    tmp = (uint32_t *)malloc((n1 + n2 + 1) * sizeof(uint32_t));
    queue = (uint32_t *)malloc((n1 + 1) * sizeof(uint32_t));
    word = (uint8_t *)malloc(n1 + n2 + 1);
    if (placement == ORACLE_R2) P = merge_r2(&s, t, n1, n2, 1, 0, tmp);
    else if (placement == ORACLE_BALANCED) P = merge_balanced(&s, t, n1, n2, 1, 0, tmp, word);
    else P = merge_r1(&s, t, n1, n2, 1, 0, tmp, queue);
    free(tmp);
    free(queue);
    free(word);
    if (need) *need = s.starved ? s.need : 0;
    return s.starved ? ~(uint64_t)0 : P;
}

/* One Merge from the Philox streams of (seed, L, m); returns P, adds bits. */
uint64_t oracle_merge_seeded(uint32_t *t, uint64_t n1, uint64_t n2, int placement,
                             uint64_t seed, uint32_t L, uint32_t m, uint64_t *bits)
{
    osrc s;
    uint64_t P;
    uint32_t *tmp, *queue;
    uint8_t *word;
    memset(&s, 0, sizeof s);
    s.seed = seed;
    tmp = (uint32_t *)malloc((n1 + n2 + 1) * sizeof(uint32_t));
    queue = (uint32_t *)malloc((n1 + 1) * sizeof(uint32_t));
    word = (uint8_t *)malloc(n1 + n2 + 1);
    if (placement == ORACLE_R2) P = merge_r2(&s, t, n1, n2, L, m, tmp);
    else if (placement == ORACLE_BALANCED) P = merge_balanced(&s, t, n1, n2, L, m, tmp, word);
    else P = merge_r1(&s, t, n1, n2, L, m, tmp, queue);
    free(tmp);
    free(queue);
    free(word);
    if (bits) *bits += s.bits;
    return P;
}

/* One Fisher-Yates of a block from the Philox streams of (seed, 0, unit). */
uint64_t oracle_fisher_yates_seeded(uint32_t *t, uint64_t n, uint64_t seed, uint32_t unit)
{
    osrc s;
    memset(&s, 0, sizeof s);
    s.seed = seed;
    fisher_yates(&s, t, n, unit);
    return s.bits;
}

/* A single bounded draw DRAW(L,u,d) of range k; *bits gets the bits used. */
uint64_t oracle_random_int(uint64_t seed, uint32_t L, uint32_t u, uint64_t d, uint64_t k, uint64_t *bits)
{
    osrc s;
    uint64_t r;
    memset(&s, 0, sizeof s);
    s.seed = seed;
    r = random_int(&s, L, u, d, k);
    if (bits) *bits = s.bits;
    return r;
}

/* A single coin flip FLIP(L,m,t). */
int oracle_random_bit(uint64_t seed, uint32_t L, uint32_t m, uint64_t t)
{
    osrc s;
    memset(&s, 0, sizeof s);
    s.seed = seed;
    return random_bit(&s, L, m, t);
}

/*
 * The Fast Dice Roller run on an explicit bit string (one bit per byte).
 * Returns the value, or -1 if the string ends before a value is accepted;
 * *used = bits read.  Used to check the exact output law by enumeration.
 */
int64_t oracle_fdr_on_bits(uint64_t k, const uint8_t *bitstr, uint32_t nbits, uint32_t *used)
{
    uint64_t v = 1, c = 0;
    uint32_t pos = 0;
    if (k <= 1) { if (used) *used = 0; return 0; }
    for (;;) {
        if (pos == nbits) { if (used) *used = pos; return -1; }
        v = v << 1;
        c = (c << 1) | (bitstr[pos++] & 1u);
        if (v >= k) {
            if (c < k) { if (used) *used = pos; return (int64_t)c; }
            v -= k;
            c -= k;
        }
    }
}

/* Permutations of 0..n-1 for seeds seed0, seed0+1, ..., seed0+count-1,
 * row by row into out (count x n); bits_out[r] = bits of row r. */
void oracle_sample_permutations(uint64_t n, uint64_t cutoff, uint64_t seed0, uint64_t count,
                                uint32_t *out, uint64_t *bits_out)
{
    uint64_t r;
    for (r = 0; r < count; r++) {
        uint64_t b = oracle_permutation(out + r * n, n, cutoff, seed0 + r, 1);
        if (bits_out) bits_out[r] = b;
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * oracle.c -- plain sequential CPU reference for DFA minimisation, equivalence
 * and inclusion checking (Heemstra, Martens, Wijs: "Evaluating Massively
 * Parallel Algorithms for DFA Minimisation, Equivalence Checking and Inclusion
 * Checking").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Conventions (all functions):
 *   - states are 0..n-1, letters 0..k-1;
 *   - delta is row-major: delta[q*k + a] = delta(q, a)  (uint32);
 *   - accepting[q] != 0  iff  q is accepting;
 *   - a partition is returned canonically: block[q] = the smallest state index
 *     in q's block;
 *   - every function returns 0 on success and a negative value on bad input or
 *     out-of-memory.
 *
 * Every result here has a plain definition (Section 2 of the paper): two
 * states are equivalent iff every word leads both or neither into F.  The
 * functions below compute that relation in several independent ways so the
 * tests can cross-check them:
 *   orc_moore        signature refinement by sorting, the semantics of the
 *                    paper's sortPR (Section 3.3, Algorithm 4), sequential;
 *                    also reports the number of rounds;
 *   orc_naive_pr     leader-based refinement, the paper's naivePR (Section
 *                    3.2, Algorithm 2), sequential; reports its iterations;
 *   orc_hopcroft     Hopcroft's O(nk log n) algorithm (textbook, cited in the
 *                    paper's introduction);
 *   orc_table_fill   the fixpoint of the pair relation "Apart" that the
 *                    paper's trans algorithm (Section 3.1, Algorithm 1)
 *                    computes, evaluated sequentially;
 *   orc_pointer_jump the partial transitive closure of transPR (Section 3.4,
 *                    Algorithm 5), sequential;
 *   orc_equiv_hk     Hopcroft-Karp equivalence with R+ kept by union-find
 *                    (Section 4, Algorithm 6);
 *   orc_minimise_reachable  the minimal DFA in the usual sense: breadth-first
 *                    reachability from the start, then Hopcroft on the
 *                    reachable part (the paper prunes nothing, Section 2);
 *   orc_product_bfs  the "naive" Hopcroft-Karp variant of Section 4 (R kept as
 *                    a set of pairs, no closure) = reachability in the
 *                    synchronous product; inclusion uses the changed
 *                    acceptance condition of Section 4.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ELIMIT (-3)

static int check_dfa(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc)
{
    if (n == 0 || k == 0 || !delta || !acc)
        return ORC_EINVAL;
    uint64_t m = (uint64_t)n * k;
    for (uint64_t i = 0; i < m; i++)
        if (delta[i] >= n)
            return ORC_EINVAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Canonical renumbering: out[q] = min{ q' : id[q'] == id[q] }.              */
/* ids may be arbitrary 32-bit labels.                                      */
/* ------------------------------------------------------------------------ */

static _Thread_local const uint32_t *g_sort_ids; /* comparator state, one per thread */
static int cmp_by_id_then_index(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    if (g_sort_ids[a] != g_sort_ids[b])
        return g_sort_ids[a] < g_sort_ids[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int orc_canonicalise(uint32_t n, const uint32_t *ids, uint32_t *out)
{
    if (n == 0)
        return ORC_OK;
    uint32_t *order = malloc((size_t)n * sizeof *order);
    if (!order)
        return ORC_ENOMEM;
    for (uint32_t q = 0; q < n; q++)
        order[q] = q;
    g_sort_ids = ids;
    qsort(order, n, sizeof *order, cmp_by_id_then_index);
    uint32_t leader = order[0];
    for (uint32_t i = 0; i < n; i++) {
        if (i > 0 && ids[order[i]] != ids[order[i - 1]])
            leader = order[i]; /* first in the group = smallest index */
        out[order[i]] = leader;
    }
    free(order);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Moore / signature refinement (Algorithm 4 semantics).                    */
/*                                                                          */
/* Initial partition: accepting vs non-accepting states (only the non-empty */
/* classes).  One round: every state gets the signature                     */
/*   ( block[q], block[delta(q,0)], ..., block[delta(q,k-1)] )              */
/* compared lexicographically in that fixed order; states are sorted by it  */
/* and each run of equal signatures becomes a block.  The loop stops when   */
/* the number of blocks did not grow, exactly the paper's stop test.        */
/* ------------------------------------------------------------------------ */

static _Thread_local const uint32_t *g_blk; /* comparator state, one per thread */
static _Thread_local const uint32_t *g_sig;
static _Thread_local uint32_t g_k;

static int cmp_signature(const void *x, const void *y)
{
    uint32_t p = *(const uint32_t *)x, q = *(const uint32_t *)y;
    if (g_blk[p] != g_blk[q])
        return g_blk[p] < g_blk[q] ? -1 : 1;
    const uint32_t *sp = g_sig + (size_t)p * g_k, *sq = g_sig + (size_t)q * g_k;
    for (uint32_t a = 0; a < g_k; a++)
        if (sp[a] != sq[a])
            return sp[a] < sq[a] ? -1 : 1;
    return 0;
}

static int same_signature(uint32_t p, uint32_t q)
{
    return cmp_signature(&p, &q) == 0;
}

/* Initial partition {F, Q\F}: block[q] = smallest state of q's class.
 * Returns the number of non-empty classes. */
static uint32_t initial_partition(uint32_t n, const uint8_t *acc, uint32_t *block)
{
    uint32_t first_acc = UINT32_MAX, first_rej = UINT32_MAX;
    for (uint32_t q = 0; q < n; q++) {
        if (acc[q] && first_acc == UINT32_MAX)
            first_acc = q;
        if (!acc[q] && first_rej == UINT32_MAX)
            first_rej = q;
    }
    for (uint32_t q = 0; q < n; q++)
        block[q] = acc[q] ? first_acc : first_rej;
    return (first_acc != UINT32_MAX) + (first_rej != UINT32_MAX);
}

/* One refinement round from a canonical partition block_in to block_out.
 * Returns the number of blocks of block_out, or 0 on out-of-memory. */
uint32_t orc_moore_round(uint32_t n, uint32_t k, const uint32_t *delta,
                         const uint32_t *block_in, uint32_t *block_out)
{
    uint32_t *order = malloc((size_t)n * sizeof *order);
    uint32_t *sig = malloc((size_t)n * k * sizeof *sig);
    if (!order || !sig) {
        free(order);
        free(sig);
        return 0;
    }
    for (uint32_t q = 0; q < n; q++) {
        order[q] = q;
        for (uint32_t a = 0; a < k; a++)
            sig[(size_t)q * k + a] = block_in[delta[(size_t)q * k + a]];
    }
    g_blk = block_in;
    g_sig = sig;
    g_k = k;
    qsort(order, n, sizeof *order, cmp_signature);

    /* each run of equal signatures is one new block; its id is its smallest
     * member (the sort is not stable, so take the minimum explicitly) */
    uint32_t count = 0;
    size_t run = 0;
    while (run < n) {
        size_t end = run + 1;
        uint32_t leader = order[run];
        while (end < n && same_signature(order[run], order[end])) {
            if (order[end] < leader)
                leader = order[end];
            end++;
        }
        for (size_t i = run; i < end; i++)
            block_out[order[i]] = leader;
        count++;
        run = end;
    }
    free(order);
    free(sig);
    return count;
}

/* Full Moore refinement.  rounds_out = rounds executed (the last one confirms
 * stability), changing_out = rounds that increased the block count (r*).
 * max_rounds bounds the work (0 = no bound); exceeding it returns ORC_ELIMIT
 * with block holding the partition reached so far. */
int orc_moore(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
              uint32_t *block, uint32_t *num_blocks, uint32_t *rounds_out,
              uint32_t *changing_out, uint32_t max_rounds)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    uint32_t *next = malloc((size_t)n * sizeof *next);
    if (!next)
        return ORC_ENOMEM;
    uint32_t count = initial_partition(n, acc, block);
    uint32_t rounds = 0, changing = 0;
    for (;;) {
        if (max_rounds && rounds >= max_rounds) {
            rc = ORC_ELIMIT;
            break;
        }
        uint32_t c = orc_moore_round(n, k, delta, block, next);
        if (c == 0) {
            rc = ORC_ENOMEM;
            break;
        }
        rounds++;
        memcpy(block, next, (size_t)n * sizeof *block);
        if (c == count)
            break;
        changing++;
        count = c;
    }
    free(next);
    if (num_blocks)
        *num_blocks = count;
    if (rounds_out)
        *rounds_out = rounds;
    if (changing_out)
        *changing_out = changing;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Leader-based refinement, naivePR (Section 3.2, Algorithm 2).             */
/*                                                                          */
/* Every block is named by a leader state that belongs to it; initially the */
/* leaders of F and Q\F.  One iteration: each state q whose successor block */
/* differs from its leader's successor block on some letter is "separated"; */
/* all separated states of one block move together to one new block, led by */
/* one of them.  The iteration in which no state is separated ends the loop.*/
/*                                                                          */
/* Two readings fix what the paper leaves to the PRAM model:               */
/*   - the concurrent leader write resolves to the smallest writer (the    */
/*     priority rule), and the initial leaders are the smallest accepting  */
/*     and the smallest rejecting state, so every leader is the smallest   */
/*     member of its block and the ids are canonical without renumbering;  */
/*   - the separation test of the second parallel loop reads the partition */
/*     the iteration started from (lock-step evaluation), so moving one    */
/*     state never changes the test of another in the same iteration.      */
/* rounds_out counts every iteration including the last (no separation),   */
/* changing_out those that separated some state.                           */
/* ------------------------------------------------------------------------ */

int orc_naive_pr(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                 uint32_t *block, uint32_t *num_blocks, uint32_t *rounds_out,
                 uint32_t *changing_out, uint32_t max_rounds)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    uint32_t *new_leader = malloc((size_t)n * sizeof *new_leader);
    uint8_t *separated = malloc(n);
    if (!new_leader || !separated) {
        free(new_leader);
        free(separated);
        return ORC_ENOMEM;
    }
    uint32_t count = initial_partition(n, acc, block);
    uint32_t rounds = 0, changing = 0;
    for (;;) {
        if (max_rounds && rounds >= max_rounds) {
            rc = ORC_ELIMIT;
            break;
        }
        rounds++;
        /* first parallel loop: test every state against its leader and
         * elect the new leader of each block's separated states */
        for (uint32_t q = 0; q < n; q++)
            new_leader[q] = UINT32_MAX;
        for (uint32_t q = 0; q < n; q++) {
            const uint32_t leader = block[q];
            separated[q] = 0;
            for (uint32_t a = 0; a < k; a++) {
                const uint32_t mine = block[delta[(size_t)q * k + a]];
                const uint32_t theirs = block[delta[(size_t)leader * k + a]];
                if (mine != theirs) {
                    separated[q] = 1;
                    break;
                }
            }
            if (separated[q] && q < new_leader[leader])
                new_leader[leader] = q;
        }
        /* second parallel loop: move the separated states (the test above
         * was taken on the partition this iteration started from) */
        uint32_t moved = 0, new_blocks = 0;
        for (uint32_t q = 0; q < n; q++) {
            if (!separated[q])
                continue;
            const uint32_t target = new_leader[block[q]];
            if (target == q)
                new_blocks++;
            block[q] = target;
            moved++;
        }
        if (moved == 0)
            break;
        changing++;
        count += new_blocks;
    }
    free(new_leader);
    free(separated);
    if (num_blocks)
        *num_blocks = count;
    if (rounds_out)
        *rounds_out = rounds;
    if (changing_out)
        *changing_out = changing;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Hopcroft's minimisation algorithm (textbook formulation).                */
/*                                                                          */
/* Blocks are contiguous ranges of a permutation `elems` of the states.     */
/* The worklist holds (splitter block, letter) pairs.  Popping (S, a): let  */
/* X = { q : delta(q,a) in S }; every block Y with Y&X and Y\X both         */
/* non-empty is split; for each letter c, if (Y,c) is still waiting both    */
/* halves are added, otherwise only the smaller half.                       */
/* ------------------------------------------------------------------------ */

int orc_hopcroft(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                 uint32_t *block_out, uint32_t *num_blocks)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    size_t nk = (size_t)n * k;

    /* inverse transitions, one CSR per letter: sources of (t, a) are
     * inv_src[inv_off[a*(n+1)+t] .. inv_off[a*(n+1)+t+1]) */
    uint64_t *inv_off = calloc((size_t)k * (n + 1), sizeof *inv_off);
    uint32_t *inv_src = malloc(nk * sizeof *inv_src);
    uint32_t *elems = malloc((size_t)n * sizeof *elems);
    uint32_t *pos = malloc((size_t)n * sizeof *pos);
    uint32_t *blk = malloc((size_t)n * sizeof *blk);
    uint32_t *bstart = malloc((size_t)n * sizeof *bstart);
    uint32_t *bend = malloc((size_t)n * sizeof *bend);
    uint32_t *marked = calloc((size_t)n, sizeof *marked);
    uint32_t *xbuf = malloc((size_t)n * sizeof *xbuf);
    uint32_t *touched = malloc((size_t)n * sizeof *touched);
    uint8_t *waiting = calloc(nk, 1); /* waiting[b*k + a] */
    uint64_t *work = malloc(nk * sizeof *work);
    uint32_t *minmember = malloc((size_t)n * sizeof *minmember);
    if (!inv_off || !inv_src || !elems || !pos || !blk || !bstart || !bend ||
        !marked || !xbuf || !touched || !waiting || !work || !minmember) {
        rc = ORC_ENOMEM;
        goto done;
    }

    for (uint32_t a = 0; a < k; a++) {
        uint64_t *off = inv_off + (size_t)a * (n + 1);
        for (uint32_t q = 0; q < n; q++)
            off[delta[(size_t)q * k + a] + 1]++;
        for (uint32_t t = 0; t < n; t++)
            off[t + 1] += off[t];
    }
    {
        uint64_t *fill = malloc((size_t)k * n * sizeof *fill);
        if (!fill) {
            rc = ORC_ENOMEM;
            goto done;
        }
        for (uint32_t a = 0; a < k; a++)
            for (uint32_t t = 0; t < n; t++)
                fill[(size_t)a * n + t] = inv_off[(size_t)a * (n + 1) + t];
        /* the CSRs of all letters share inv_src: letter a occupies
         * [a*n, (a+1)*n) since it has exactly n transitions */
        for (uint32_t a = 0; a < k; a++)
            for (uint32_t q = 0; q < n; q++) {
                uint32_t t = delta[(size_t)q * k + a];
                inv_src[(size_t)a * n + fill[(size_t)a * n + t]++] = q;
            }
        free(fill);
    }

    /* initial partition: accepting states first, then the rest */
    uint32_t nb = 0, nacc = 0;
    for (uint32_t q = 0; q < n; q++)
        if (acc[q])
            elems[nacc++] = q;
    uint32_t r = nacc;
    for (uint32_t q = 0; q < n; q++)
        if (!acc[q])
            elems[r++] = q;
    for (uint32_t i = 0; i < n; i++)
        pos[elems[i]] = i;
    if (nacc > 0) {
        bstart[nb] = 0;
        bend[nb] = nacc;
        nb++;
    }
    if (nacc < n) {
        bstart[nb] = nacc;
        bend[nb] = n;
        nb++;
    }
    for (uint32_t b = 0; b < nb; b++)
        for (uint32_t i = bstart[b]; i < bend[b]; i++)
            blk[elems[i]] = b;

    size_t nwork = 0;
    if (nb == 2) {
        uint32_t smaller = (bend[0] - bstart[0] <= bend[1] - bstart[1]) ? 0 : 1;
        for (uint32_t a = 0; a < k; a++) {
            work[nwork++] = (uint64_t)smaller * k + a;
            waiting[(size_t)smaller * k + a] = 1;
        }
    }

    while (nwork > 0) {
        uint64_t item = work[--nwork];
        uint32_t S = (uint32_t)(item / k), a = (uint32_t)(item % k);
        waiting[item] = 0;

        /* X = predecessors of S under a */
        uint32_t nx = 0;
        const uint64_t *off = inv_off + (size_t)a * (n + 1);
        const uint32_t *src = inv_src + (size_t)a * n;
        for (uint32_t i = bstart[S]; i < bend[S]; i++) {
            uint32_t t = elems[i];
            for (uint64_t j = off[t]; j < off[t + 1]; j++)
                xbuf[nx++] = src[j];
        }

        /* move every member of X to the front of its block */
        uint32_t ntouched = 0;
        for (uint32_t i = 0; i < nx; i++) {
            uint32_t q = xbuf[i], b = blk[q];
            if (marked[b] == 0)
                touched[ntouched++] = b;
            uint32_t dst = bstart[b] + marked[b];
            uint32_t other = elems[dst];
            uint32_t pq = pos[q];
            elems[dst] = q;
            pos[q] = dst;
            elems[pq] = other;
            pos[other] = pq;
            marked[b]++;
        }

        /* split every touched block that X cuts in two */
        for (uint32_t i = 0; i < ntouched; i++) {
            uint32_t b = touched[i];
            uint32_t m = marked[b];
            marked[b] = 0;
            if (m == bend[b] - bstart[b])
                continue;
            uint32_t c = nb++; /* new block = the marked front part */
            bstart[c] = bstart[b];
            bend[c] = bstart[b] + m;
            bstart[b] = bend[c];
            for (uint32_t j = bstart[c]; j < bend[c]; j++)
                blk[elems[j]] = c;
            uint32_t size_b = bend[b] - bstart[b], size_c = bend[c] - bstart[c];
            for (uint32_t l = 0; l < k; l++) {
                if (waiting[(size_t)b * k + l]) {
                    work[nwork++] = (uint64_t)c * k + l;
                    waiting[(size_t)c * k + l] = 1;
                } else {
                    uint32_t s = size_c <= size_b ? c : b;
                    work[nwork++] = (uint64_t)s * k + l;
                    waiting[(size_t)s * k + l] = 1;
                }
            }
        }
    }

    /* canonical ids: smallest member of each block */
    for (uint32_t b = 0; b < nb; b++)
        minmember[b] = UINT32_MAX;
    for (uint32_t q = 0; q < n; q++)
        if (q < minmember[blk[q]])
            minmember[blk[q]] = q;
    for (uint32_t q = 0; q < n; q++)
        block_out[q] = minmember[blk[q]];
    if (num_blocks)
        *num_blocks = nb;

done:
    free(inv_off);
    free(inv_src);
    free(elems);
    free(pos);
    free(blk);
    free(bstart);
    free(bend);
    free(marked);
    free(xbuf);
    free(touched);
    free(waiting);
    free(work);
    free(minmember);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Table filling: the fixpoint of the relation Apart over Q x Q that the    */
/* trans algorithm computes.  apart[p*n+q] starts as the acceptance         */
/* mismatch; a pair becomes apart when some letter leads it to an apart     */
/* pair.  Returns the number of sweeps that marked something.               */
/* ------------------------------------------------------------------------ */

int orc_table_fill(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                   uint8_t *apart, uint32_t *sweeps_out)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    for (uint32_t p = 0; p < n; p++)
        for (uint32_t q = 0; q < n; q++)
            apart[(size_t)p * n + q] = (acc[p] != 0) != (acc[q] != 0);
    uint32_t sweeps = 0;
    int changed = 1;
    while (changed) {
        changed = 0;
        for (uint32_t p = 0; p < n; p++)
            for (uint32_t q = 0; q < n; q++) {
                if (apart[(size_t)p * n + q])
                    continue;
                for (uint32_t a = 0; a < k; a++) {
                    uint32_t pp = delta[(size_t)p * k + a], qq = delta[(size_t)q * k + a];
                    if (apart[(size_t)pp * n + qq]) {
                        apart[(size_t)p * n + q] = 1;
                        changed = 1;
                        break;
                    }
                }
            }
        if (changed)
            sweeps++;
    }
    if (sweeps_out)
        *sweeps_out = sweeps;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Partial transitive closure (Algorithm 5): for every letter a the letters */
/* a^(2^i), i = 0..L, with delta(q, a^(2^i)) = delta(delta(q, a^(2^(i-1))), */
/* a^(2^(i-1))).  Output is row-major n x (k*(L+1)); column i*k + a holds   */
/* a^(2^i).  L is chosen by the caller (the paper uses floor(log2 n)).       */
/* ------------------------------------------------------------------------ */

int orc_pointer_jump(uint32_t n, uint32_t k, const uint32_t *delta, uint32_t L,
                     uint32_t *out)
{
    if (n == 0 || k == 0 || !delta || !out)
        return ORC_EINVAL;
    size_t kt = (size_t)k * (L + 1);
    for (uint32_t q = 0; q < n; q++)
        for (uint32_t a = 0; a < k; a++) {
            if (delta[(size_t)q * k + a] >= n)
                return ORC_EINVAL;
            out[(size_t)q * kt + a] = delta[(size_t)q * k + a];
        }
    for (uint32_t i = 1; i <= L; i++)
        for (uint32_t a = 0; a < k; a++) {
            size_t prev = (size_t)(i - 1) * k + a, cur = (size_t)i * k + a;
            for (uint32_t q = 0; q < n; q++) {
                uint32_t mid = out[(size_t)q * kt + prev];
                out[(size_t)q * kt + cur] = out[(size_t)mid * kt + prev];
            }
        }
    return ORC_OK;
}

/* floor(log2 n) for n >= 1 */
uint32_t orc_floor_log2(uint32_t n)
{
    uint32_t l = 0;
    while (n > 1) {
        n >>= 1;
        l++;
    }
    return l;
}

/* ------------------------------------------------------------------------ */
/* Quotient automaton of a canonical partition.  Blocks are numbered densely */
/* in increasing order of their smallest member.                            */
/* ------------------------------------------------------------------------ */

int orc_quotient(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                 const uint32_t *block, uint32_t start, uint32_t *qn,
                 uint32_t *qdelta, uint8_t *qacc, uint32_t *qstart)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    if (start >= n)
        return ORC_EINVAL;
    uint32_t *dense = malloc((size_t)n * sizeof *dense);
    if (!dense)
        return ORC_ENOMEM;
    uint32_t nb = 0;
    for (uint32_t q = 0; q < n; q++) {
        if (block[q] > q || block[block[q]] != block[q]) {
            free(dense);
            return ORC_EINVAL; /* not canonical */
        }
        if (block[q] == q)
            dense[q] = nb++;
    }
    for (uint32_t q = 0; q < n; q++) {
        if (block[q] != q)
            continue;
        uint32_t b = dense[q];
        for (uint32_t a = 0; a < k; a++)
            qdelta[(size_t)b * k + a] = dense[block[delta[(size_t)q * k + a]]];
        qacc[b] = acc[q] ? 1 : 0;
    }
    *qn = nb;
    *qstart = dense[block[start]];
    free(dense);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Hopcroft-Karp equivalence (Algorithm 6) with R+ kept by union-find over   */
/* the disjoint union of the two state sets (B's states offset by nA).      */
/* ------------------------------------------------------------------------ */

static uint32_t uf_find(uint32_t *parent, uint32_t x)
{
    uint32_t root = x;
    while (parent[root] != root)
        root = parent[root];
    while (parent[x] != root) { /* path compression */
        uint32_t next = parent[x];
        parent[x] = root;
        x = next;
    }
    return root;
}

int orc_equiv_hk(uint32_t nA, uint32_t kA, const uint32_t *dA, const uint8_t *accA,
                 uint32_t sA, uint32_t nB, uint32_t kB, const uint32_t *dB,
                 const uint8_t *accB, uint32_t sB, int *verdict)
{
    if (kA != kB || sA >= nA || sB >= nB)
        return ORC_EINVAL;
    int rc = check_dfa(nA, kA, dA, accA);
    if (!rc)
        rc = check_dfa(nB, kB, dB, accB);
    if (rc)
        return rc;
    uint32_t k = kA;
    uint64_t tot = (uint64_t)nA + nB;
    if (tot >= UINT32_MAX)
        return ORC_EINVAL;
    uint32_t *parent = malloc(tot * sizeof *parent);
    /* every union pushes k pairs; at most tot-1 unions happen */
    size_t cap = (size_t)k * tot + 1;
    uint32_t *stack = malloc(cap * 2 * sizeof *stack);
    if (!parent || !stack) {
        free(parent);
        free(stack);
        return ORC_ENOMEM;
    }
    for (uint64_t i = 0; i < tot; i++)
        parent[i] = (uint32_t)i;
    size_t top = 0;
    stack[0] = sA;
    stack[1] = nA + sB;
    top = 1;
    int eq = 1;
    while (top > 0) {
        top--;
        uint32_t p = stack[2 * top], q = stack[2 * top + 1]; /* p in A, q in B (offset) */
        uint32_t rp = uf_find(parent, p), rq = uf_find(parent, q);
        if (rp == rq)
            continue; /* already related by R+ */
        int fa = accA[p] != 0, fb = accB[q - nA] != 0;
        if (fa != fb) {
            eq = 0;
            break;
        }
        for (uint32_t a = 0; a < k; a++) {
            stack[2 * top] = dA[(size_t)p * k + a];
            stack[2 * top + 1] = nA + dB[(size_t)(q - nA) * k + a];
            top++;
        }
        parent[rp] = rq; /* R := R u {(p,q)} */
    }
    free(parent);
    free(stack);
    *verdict = eq;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Product exploration (the naive Hopcroft-Karp of Section 4: the relation  */
/* is kept as a plain set of pairs, no transitive closure).                 */
/* mode 0: inclusion  L(A) in L(B): a reached pair with p in F_A and        */
/*         q not in F_B refutes it.                                         */
/* mode 1: equivalence: a reached pair with exactly one side accepting      */
/*         refutes it.                                                      */
/* Breadth-first from (sA, sB).  visited_out = number of distinct pairs     */
/* reached (the whole reachable product when the verdict is 1).             */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t *slot;
    uint64_t cap, used;
} pairset;

#define PAIR_EMPTY UINT64_MAX

static uint64_t mix64(uint64_t x)
{
    /* splitmix64 finaliser */
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ULL;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebULL;
    x ^= x >> 31;
    return x;
}

static int pairset_grow(pairset *s)
{
    uint64_t ncap = s->cap ? s->cap * 2 : 1024;
    uint64_t *ns = malloc(ncap * sizeof *ns);
    if (!ns)
        return ORC_ENOMEM;
    for (uint64_t i = 0; i < ncap; i++)
        ns[i] = PAIR_EMPTY;
    for (uint64_t i = 0; i < s->cap; i++) {
        uint64_t key = s->slot[i];
        if (key == PAIR_EMPTY)
            continue;
        uint64_t h = mix64(key) & (ncap - 1);
        while (ns[h] != PAIR_EMPTY)
            h = (h + 1) & (ncap - 1);
        ns[h] = key;
    }
    free(s->slot);
    s->slot = ns;
    s->cap = ncap;
    return ORC_OK;
}

/* returns 1 if inserted, 0 if present, <0 on error */
static int pairset_insert(pairset *s, uint64_t key)
{
    if ((s->used + 1) * 2 > s->cap) {
        int rc = pairset_grow(s);
        if (rc)
            return rc;
    }
    uint64_t h = mix64(key) & (s->cap - 1);
    while (s->slot[h] != PAIR_EMPTY) {
        if (s->slot[h] == key)
            return 0;
        h = (h + 1) & (s->cap - 1);
    }
    s->slot[h] = key;
    s->used++;
    return 1;
}

int orc_product_bfs(uint32_t nA, uint32_t kA, const uint32_t *dA, const uint8_t *accA,
                    uint32_t sA, uint32_t nB, uint32_t kB, const uint32_t *dB,
                    const uint8_t *accB, uint32_t sB, int mode, int *verdict,
                    uint64_t *visited_out)
{
    if (kA != kB || sA >= nA || sB >= nB || (mode != 0 && mode != 1))
        return ORC_EINVAL;
    int rc = check_dfa(nA, kA, dA, accA);
    if (!rc)
        rc = check_dfa(nB, kB, dB, accB);
    if (rc)
        return rc;
    uint32_t k = kA;
    pairset seen = {0, 0, 0};
    uint64_t qcap = 1024, qhead = 0, qtail = 0;
    uint64_t *queue = malloc(qcap * sizeof *queue);
    if (!queue)
        return ORC_ENOMEM;
    uint64_t startkey = ((uint64_t)sA << 32) | sB;
    rc = pairset_insert(&seen, startkey);
    if (rc < 0)
        goto out;
    rc = ORC_OK;
    queue[qtail++] = startkey;
    int ok = 1;
    while (qhead < qtail) {
        uint64_t key = queue[qhead++];
        uint32_t p = (uint32_t)(key >> 32), q = (uint32_t)key;
        int fa = accA[p] != 0, fb = accB[q] != 0;
        int bad = mode == 0 ? (fa && !fb) : (fa != fb);
        if (bad) {
            ok = 0;
            break;
        }
        for (uint32_t a = 0; a < k; a++) {
            uint64_t nk2 = ((uint64_t)dA[(size_t)p * k + a] << 32) | dB[(size_t)q * k + a];
            int ins = pairset_insert(&seen, nk2);
            if (ins < 0) {
                rc = ins;
                goto out;
            }
            if (ins) {
                if (qtail == qcap) {
                    uint64_t *nq = realloc(queue, qcap * 2 * sizeof *nq);
                    if (!nq) {
                        rc = ORC_ENOMEM;
                        goto out;
                    }
                    queue = nq;
                    qcap *= 2;
                }
                queue[qtail++] = nk2;
            }
        }
    }
    *verdict = ok;
    if (visited_out)
        *visited_out = seen.used;
out:
    free(seen.slot);
    free(queue);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reachability and minimisation of the reachable part (Section 2: the       */
/* paper assumes every state reachable and prunes nothing; the standard      */
/* minimal DFA is the quotient of the reachable part).                        */
/*                                                                          */
/* orc_reachable: breadth-first search from `start`; reach[q] = 1 iff some  */
/* word leads from start to q.                                              */
/* orc_minimise_reachable: block[q] = smallest reachable state equivalent   */
/* to q for reachable q, UINT32_MAX for the others; the relation is          */
/* Hopcroft's on the sub-automaton of reachable states (its transitions stay */
/* inside it), so it equals language equivalence restricted to them.        */
/* ------------------------------------------------------------------------ */

int orc_reachable(uint32_t n, uint32_t k, const uint32_t *delta, uint32_t start, uint8_t *reach,
                  uint32_t *count)
{
    if (n == 0 || k == 0 || !delta || !reach || start >= n)
        return ORC_EINVAL;
    uint32_t *queue = malloc((size_t)n * sizeof *queue);
    if (!queue)
        return ORC_ENOMEM;
    memset(reach, 0, n);
    size_t head = 0, tail = 0;
    reach[start] = 1;
    queue[tail++] = start;
    while (head < tail) {
        const uint32_t q = queue[head++];
        for (uint32_t a = 0; a < k; a++) {
            const uint32_t t = delta[(size_t)q * k + a];
            if (t >= n) {
                free(queue);
                return ORC_EINVAL;
            }
            if (!reach[t]) {
                reach[t] = 1;
                queue[tail++] = t;
            }
        }
    }
    free(queue);
    if (count)
        *count = (uint32_t)tail;
    return ORC_OK;
}

int orc_minimise_reachable(uint32_t n, uint32_t k, const uint32_t *delta, const uint8_t *acc,
                           uint32_t start, uint32_t *block, uint32_t *num_blocks,
                           uint32_t *num_reachable)
{
    int rc = check_dfa(n, k, delta, acc);
    if (rc)
        return rc;
    uint8_t *reach = malloc(n);
    uint32_t *dense = malloc((size_t)n * sizeof *dense);
    uint32_t *orig = malloc((size_t)n * sizeof *orig);
    if (!reach || !dense || !orig) {
        rc = ORC_ENOMEM;
        goto out;
    }
    uint32_t m = 0;
    rc = orc_reachable(n, k, delta, start, reach, &m);
    if (rc)
        goto out;
    /* the sub-automaton, states renumbered in increasing original order */
    uint32_t next = 0;
    for (uint32_t q = 0; q < n; q++)
        if (reach[q]) {
            dense[q] = next;
            orig[next++] = q;
        }
    uint32_t *sd = malloc((size_t)m * k * sizeof *sd);
    uint8_t *sa = malloc(m);
    uint32_t *sb = malloc((size_t)m * sizeof *sb);
    if (!sd || !sa || !sb) {
        free(sd);
        free(sa);
        free(sb);
        rc = ORC_ENOMEM;
        goto out;
    }
    for (uint32_t i = 0; i < m; i++) {
        const uint32_t q = orig[i];
        for (uint32_t a = 0; a < k; a++)
            sd[(size_t)i * k + a] = dense[delta[(size_t)q * k + a]];
        sa[i] = acc[q] ? 1 : 0;
    }
    uint32_t nb = 0;
    rc = orc_hopcroft(m, k, sd, sa, sb, &nb);
    if (!rc) {
        for (uint32_t q = 0; q < n; q++)
            block[q] = reach[q] ? orig[sb[dense[q]]] : UINT32_MAX;
        if (num_blocks)
            *num_blocks = nb;
        if (num_reachable)
            *num_reachable = m;
    }
    free(sd);
    free(sa);
    free(sb);
out:
    free(reach);
    free(dense);
    free(orig);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Loops over many small DFAs of one shape (count instances, each n states,  */
/* k letters, packed back to back) -- a convenience for exhaustive tests.   */
/* algo 0 = Hopcroft, 1 = Moore, 2 = naivePR.                               */
/* ------------------------------------------------------------------------ */

int orc_minimise_many(int algo, uint64_t count, uint32_t n, uint32_t k,
                      const uint32_t *deltas, const uint8_t *accs, uint32_t *blocks)
{
    for (uint64_t i = 0; i < count; i++) {
        const uint32_t *d = deltas + i * n * k;
        const uint8_t *a = accs + i * n;
        uint32_t *b = blocks + i * n;
        int rc = algo == 0   ? orc_hopcroft(n, k, d, a, b, NULL)
                 : algo == 1 ? orc_moore(n, k, d, a, b, NULL, NULL, NULL, 0)
                             : orc_naive_pr(n, k, d, a, b, NULL, NULL, NULL, 0);
        if (rc)
            return rc;
    }
    return ORC_OK;
}

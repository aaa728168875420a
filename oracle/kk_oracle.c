/*
 * kk_oracle.c -- plain CPU oracle for Metropolis-Kawasaki exchange sweeps on
 * a periodic square lattice holding a binary (A/B) lipid mixture.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * What it follows (paper: Lis & Pintal, "GPU-Based Massive Parallel Kawasaki
 * Kinetics in Monte Carlo Modelling of Lipid Microdomains"):
 *   - Metropolis acceptance, u ~ U[0,1), accept iff u < min{1, p(x*)/p(x)}
 *     with a symmetric proposal (Materials and Methods, "Monte Carlo model
 *     with Kawasaki based kinetics", the numbered Metropolis algorithm);
 *   - Kawasaki kinetics: a move swaps two nearest-neighbour lipids, so the
 *     number of lipids of each type never changes (same section);
 *   - the one-parameter Almeida interaction omega_AB = g_AB - (g_AA+g_BB)/2,
 *     so E/kT = omega * N_AB + const (same section, the omega_AB equation);
 *   - the MPKK loop: each step is a sequence of decompositions of the lattice
 *     into disjoint domains; in each, every domain centre makes one Kawasaki
 *     attempt at once; one step makes as many attempts as there are sites
 *     (section "Massive Parallel Kawasaki Kinetics", the MPKK algorithm);
 *   - cluster sizes of one lipid species (section "Cluster Analysis methods").
 *
 * Readings taken where the paper does not fix the computation (square
 * periodic lattice instead of the triangular helical one, the 8-class
 * conflict-free decomposition, the Philox random-number layout, the
 * 42-bit acceptance threshold) are the contract written out in the
 * functions below; each function says which one it implements.
 *
 * Parity pins: Philox against the published known-answer vectors; the
 * local energy change against a full recount; conflict-freedom by brute
 * force; stationarity against exact Boltzmann enumeration on 4x4; omega = 0
 * pair statistics against the random-mixing closed form; 50:50 equilibrium
 * against Onsager's nearest-neighbour correlation; the sweep against an
 * independent sequential random-site Kawasaki chain; cluster histograms
 * against scipy's labelling with a periodic merge.
 *
 * Further sections (each with its own header below): the paper's own
 * triangular lattice with helical boundaries (16 conflict-free classes,
 * pinned by rolled recounts, brute-force conflict checks with failing
 * controls, exact 4x4 Boltzmann, the two-particle binding law, random mixing
 * and a Python BFS); the segregated start and a sequential random-site
 * Kawasaki chain on the triangular lattice; and the paper's literal MPKK
 * (7-site domain cover, synchronous domains), pinned by the cover partition,
 * a hand-worked conflicting iteration, the lone-particle move rate and random
 * mixing.  The relaxation of N_AB(t) against sequential Kawasaki is compared
 * statistically only: beyond those error bars it is parity unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KO_TAG_SWEEP 1u
#define KO_TAG_EXT 2u
#define KO_TAG_ORDER 3u
#define KO_TAG_INIT 4u
#define KO_TAG_OBSERVE 5u

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies; the    */
/* two-word key is bumped by the Weyl constants between rounds.             */
/* ---------------------------------------------------------------------- */
void ko_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void seed_to_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

/* Fourth counter word: the sweep's high 28 bits and a 4-bit stream tag. */
static uint32_t ctr3(uint64_t t, uint32_t tag)
{
    return (uint32_t)((t >> 32) & 0x0FFFFFFFu) | (tag << 28);
}

/* ---------------------------------------------------------------------- */
/* Acceptance thresholds.  For an exchange of an unlike pair whose two     */
/* sites have n unlike neighbours in total (not counting each other), the  */
/* number of AB contacts changes by dU = 6 - 2n, the energy by omega*dU,   */
/* and the Metropolis probability is p = min(1, exp(-omega*dU)).  The      */
/* contract draws u as a 42-bit integer U and accepts iff U < T[n] with    */
/* T[n] = min(2^42, ceil(p * 2^42)), which is exactly U / 2^42 < p.        */
/* ---------------------------------------------------------------------- */
void ko_thresholds(double omega, uint64_t T[7])
{
    const double two42 = 4398046511104.0; /* 2^42 */
    int n;
    for (n = 0; n <= 6; ++n) {
        double dU = 6.0 - 2.0 * (double)n;
        double p = exp(-omega * dU);
        double scaled = ceil(p * two42);
        if (!(scaled < two42)) /* also catches +inf */
            T[n] = (uint64_t)1 << 42;
        else
            T[n] = (uint64_t)scaled;
    }
}

/* ---------------------------------------------------------------------- */
/* Sweep random field.  Row y is cut into 32-site segments g; for sweep t  */
/* the segment draws three Philox blocks with counters                     */
/*   (y, 4g + j, t_lo, t_hi28 | TAG_SWEEP<<28),  j = 0, 1, 2,              */
/* giving twelve 32-bit words P[4j + m] = block_j[m].  Bit b of word P[k]  */
/* belongs to site x = 32g + b: direction = P0_b + 2*P1_b (0:+x 1:-x 2:+y  */
/* 3:-y), and the 10-bit uniform prefix has P2_b as its most significant   */
/* bit down to P11_b.  Here the field is stored per site as                */
/* (direction << 10) | u10.                                               */
/* ---------------------------------------------------------------------- */
void ko_sweep_randoms(uint32_t L, uint64_t seed, uint64_t t, uint16_t *r)
{
    uint32_t key[2], y, g, G = (L + 31u) / 32u;
    seed_to_key(seed, key);
    for (y = 0; y < L; ++y) {
        for (g = 0; g < G; ++g) {
            uint32_t P[12], b;
            int j;
            for (j = 0; j < 3; ++j) {
                uint32_t ctr[4];
                ctr[0] = y;
                ctr[1] = 4u * g + (uint32_t)j;
                ctr[2] = (uint32_t)t;
                ctr[3] = ctr3(t, KO_TAG_SWEEP);
                ko_philox4x32_10(ctr, key, &P[4 * j]);
            }
            for (b = 0; b < 32u; ++b) {
                uint32_t x = 32u * g + b, dir, u = 0;
                int k;
                if (x >= L)
                    break;
                dir = ((P[0] >> b) & 1u) | (((P[1] >> b) & 1u) << 1);
                for (k = 0; k < 10; ++k)
                    u = (u << 1) | ((P[2 + k] >> b) & 1u);
                r[(size_t)y * L + x] = (uint16_t)((dir << 10) | u);
            }
        }
    }
}

/* The 32 low-order bits of a site's 42-bit uniform, drawn only when the  */
/* 10-bit prefix alone cannot decide: word (x mod 4) of Philox block      */
/* (y, x div 4, t_lo, t_hi28 | TAG_EXT<<28).                               */
uint32_t ko_ext_word(uint64_t seed, uint64_t t, uint32_t x, uint32_t y)
{
    uint32_t key[2], ctr[4], out[4];
    seed_to_key(seed, key);
    ctr[0] = y;
    ctr[1] = x >> 2;
    ctr[2] = (uint32_t)t;
    ctr[3] = ctr3(t, KO_TAG_EXT);
    ko_philox4x32_10(ctr, key, out);
    return out[x & 3u];
}

/* ---------------------------------------------------------------------- */
/* Decomposition classes.  The paper tiles its triangular lattice with     */
/* 7-site domains and picks one of the 7 coverings at random per           */
/* iteration.  On the square lattice the contract uses 8 classes           */
/*   class(x, y) = 2*((x - y) mod 4) + (y mod 2);                          */
/* same-class sites are at L1 distance >= 4, so the exchanges of one class */
/* touch disjoint neighbourhoods and may run in any order.  Each sweep     */
/* visits the 8 classes in a random order (every site is a centre once,    */
/* N attempts per sweep): Fisher-Yates over 8 entries driven by two Philox */
/* blocks (0, j, t_lo, t_hi28 | TAG_ORDER<<28), j = 0, 1; step i = 7..1     */
/* uses word w[7 - i] and swaps entry i with entry (w * (i + 1)) >> 32.    */
/* ---------------------------------------------------------------------- */
void ko_phase_order(uint64_t seed, uint64_t t, int perm[8])
{
    uint32_t key[2], w[8];
    int i, j;
    seed_to_key(seed, key);
    for (j = 0; j < 2; ++j) {
        uint32_t ctr[4];
        ctr[0] = 0;
        ctr[1] = (uint32_t)j;
        ctr[2] = (uint32_t)t;
        ctr[3] = ctr3(t, KO_TAG_ORDER);
        ko_philox4x32_10(ctr, key, &w[4 * j]);
    }
    for (i = 0; i < 8; ++i)
        perm[i] = i;
    for (i = 7; i >= 1; --i) {
        uint32_t pick = (uint32_t)(((uint64_t)w[7 - i] * (uint64_t)(i + 1)) >> 32);
        int tmp = perm[i];
        perm[i] = perm[pick];
        perm[pick] = tmp;
    }
}

int ko_site_class(uint32_t x, uint32_t y)
{
    return (int)(2u * ((x - y) & 3u) + (y & 1u));
}

/* ---------------------------------------------------------------------- */
/* One Kawasaki attempt with the centre at (x, y).                          */
/* ---------------------------------------------------------------------- */
static uint32_t wrap_add(uint32_t v, int d, uint32_t L)
{
    if (d > 0)
        return (v + 1u == L) ? 0u : v + 1u;
    return (v == 0u) ? L - 1u : v - 1u;
}

static void partner_of(uint32_t x, uint32_t y, uint32_t dir, uint32_t L, uint32_t *bx, uint32_t *by)
{
    *bx = x;
    *by = y;
    if (dir == 0u)
        *bx = wrap_add(x, +1, L);
    else if (dir == 1u)
        *bx = wrap_add(x, -1, L);
    else if (dir == 2u)
        *by = wrap_add(y, +1, L);
    else
        *by = wrap_add(y, -1, L);
}

/* Number of the 4 neighbours of (x, y), other than (ox, oy), whose type  */
/* differs from `type`.                                                    */
static int unlike_nbrs_except(const uint8_t *s, uint32_t L, uint32_t x, uint32_t y, uint32_t ox,
                              uint32_t oy, uint8_t type)
{
    uint32_t nx[4], ny[4];
    int q, count = 0;
    nx[0] = wrap_add(x, +1, L); ny[0] = y;
    nx[1] = wrap_add(x, -1, L); ny[1] = y;
    nx[2] = x; ny[2] = wrap_add(y, +1, L);
    nx[3] = x; ny[3] = wrap_add(y, -1, L);
    for (q = 0; q < 4; ++q) {
        if (nx[q] == ox && ny[q] == oy)
            continue;
        if (s[(size_t)ny[q] * L + nx[q]] != type)
            ++count;
    }
    return count;
}

/* Change in N_AB if the pair (x,y)-(x,y)+dir were exchanged.  Only defined
 * for an unlike pair: dU = (3 - n_c - n_c) + (3 - n_b - n_b) = 6 - 2n. */
int ko_local_dnab(const uint8_t *s, uint32_t L, uint32_t x, uint32_t y, uint32_t dir)
{
    uint32_t bx, by;
    uint8_t sc, sb;
    int nc, nb;
    partner_of(x, y, dir, L, &bx, &by);
    sc = s[(size_t)y * L + x];
    sb = s[(size_t)by * L + bx];
    if (sc == sb)
        return 0;
    nc = unlike_nbrs_except(s, L, x, y, bx, by, sc);
    nb = unlike_nbrs_except(s, L, bx, by, x, y, sb);
    return 6 - 2 * (nc + nb);
}

static int attempt(uint8_t *s, uint32_t L, uint32_t x, uint32_t y, uint16_t rr, const uint64_t T[7],
                   uint64_t seed, uint64_t t)
{
    uint32_t dir = (uint32_t)rr >> 10, u10 = (uint32_t)rr & 0x3FFu;
    uint32_t bx, by;
    uint8_t sc, sb;
    int n;
    uint64_t thr;
    int accept;
    partner_of(x, y, dir, L, &bx, &by);
    sc = s[(size_t)y * L + x];
    sb = s[(size_t)by * L + bx];
    if (sc == sb)
        return 0; /* exchanging like lipids changes nothing */
    n = unlike_nbrs_except(s, L, x, y, bx, by, sc) + unlike_nbrs_except(s, L, bx, by, x, y, sb);
    thr = T[n];
    /* U = u10 * 2^32 + ext32 < thr.  The prefix decides unless it equals   */
    /* thr's top bits; only then is the low word needed.                    */
    if ((uint64_t)u10 != (thr >> 32))
        accept = (uint64_t)u10 < (thr >> 32);
    else
        accept = (uint64_t)ko_ext_word(seed, t, x, y) < (thr & 0xFFFFFFFFull);
    if (accept) {
        s[(size_t)y * L + x] = sb;
        s[(size_t)by * L + bx] = sc;
        return 1;
    }
    return 0;
}

static uint64_t fnv1a(const uint8_t *s, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    size_t i;
    for (i = 0; i < n; ++i) {
        h ^= s[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t ko_lattice_hash(const uint8_t *s, uint32_t L)
{
    return fnv1a(s, (size_t)L * L);
}

/* ---------------------------------------------------------------------- */
/* n_sweeps sweeps starting at sweep counter t0.  Returns the number of     */
/* accepted exchanges.  Optional per-sweep lattice hashes locate the first  */
/* divergence in a failed comparison.  Within one class the attempts are    */
/* independent, so the row loop may run on several threads.                 */
/* ---------------------------------------------------------------------- */
uint64_t ko_sweeps(uint8_t *s, uint32_t L, double omega, uint64_t seed, uint64_t t0, uint64_t n_sweeps,
                   uint64_t *hash_trace)
{
    uint64_t T[7], accepted = 0, i;
    uint16_t *r = (uint16_t *)malloc((size_t)L * L * sizeof(uint16_t));
    if (!r)
        return ~(uint64_t)0;
    ko_thresholds(omega, T);
    for (i = 0; i < n_sweeps; ++i) {
        uint64_t t = t0 + i;
        int perm[8], p;
        ko_sweep_randoms(L, seed, t, r);
        ko_phase_order(seed, t, perm);
        for (p = 0; p < 8; ++p) {
            uint32_t a = (uint32_t)perm[p] >> 1, b = (uint32_t)perm[p] & 1u;
            long yy;
            uint64_t acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
            for (yy = (long)b; yy < (long)L; yy += 2) {
                uint32_t y = (uint32_t)yy, x;
                for (x = (a + y) & 3u; x < L; x += 4u)
                    acc += (uint64_t)attempt(s, L, x, y, r[(size_t)y * L + x], T, seed, t);
            }
            accepted += acc;
        }
        if (hash_trace)
            hash_trace[i] = fnv1a(s, (size_t)L * L);
    }
    free(r);
    return accepted;
}

/* ---------------------------------------------------------------------- */
/* N_AB: number of nearest-neighbour bonds joining unlike lipids (2N bonds */
/* on the periodic square lattice).  E/kT = omega * N_AB.                  */
/* ---------------------------------------------------------------------- */
uint64_t ko_energy(const uint8_t *s, uint32_t L)
{
    uint64_t nab = 0;
    uint32_t x, y;
    for (y = 0; y < L; ++y)
        for (x = 0; x < L; ++x) {
            uint8_t v = s[(size_t)y * L + x];
            nab += (v != s[(size_t)y * L + wrap_add(x, +1, L)]);
            nab += (v != s[(size_t)wrap_add(y, +1, L) * L + x]);
        }
    return nab;
}

/* ---------------------------------------------------------------------- */
/* Random-neighbour estimate of the fraction of similar first neighbours     */
/* (Materials and Methods, "Image analysis": the classical approach draws,   */
/* for every site, one of its nearest neighbours at random and counts the    */
/* pairs of equal type; the estimate is that count over the lattice size).   */
/* The draw of site (x, y) taken at sweep counter t is the top two bits of   */
/* word (x mod 4) of Philox block (y, x div 4, t_lo, t_hi28 | TAG_OBSERVE<<28)*/
/* with 0 = +x, 1 = -x, 2 = +y, 3 = -y.  Returns the count.                  */
/* ---------------------------------------------------------------------- */
uint64_t ko_similar_sampled(const uint8_t *s, uint32_t L, uint64_t seed, uint64_t t)
{
    uint32_t key[2], ctr[4], w[4];
    uint64_t same = 0;
    uint32_t x, y;
    seed_to_key(seed, key);
    for (y = 0; y < L; ++y)
        for (x = 0; x < L; ++x) {
            uint32_t dir, nx, ny;
            if ((x & 3u) == 0) {
                ctr[0] = y;
                ctr[1] = x >> 2;
                ctr[2] = (uint32_t)t;
                ctr[3] = ctr3(t, KO_TAG_OBSERVE);
                ko_philox4x32_10(ctr, key, w);
            }
            dir = w[x & 3u] >> 30;
            partner_of(x, y, dir, L, &nx, &ny);
            same += (s[(size_t)y * L + x] == s[(size_t)ny * L + nx]);
        }
    return same;
}

/* ---------------------------------------------------------------------- */
/* Initial placement: every site draws a 64-bit key from Philox block       */
/* (y, x, 0, TAG_INIT<<28), key = word0 * 2^32 + word1; sites are sorted by */
/* (key, y*L + x) and the first n1 = floor(c*N + 0.5) become type 1.  This  */
/* is a uniformly random subset of exactly n1 sites.                        */
/* ---------------------------------------------------------------------- */
typedef struct {
    uint64_t key;
    uint64_t idx;
} ko_keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const ko_keyed *p = (const ko_keyed *)a, *q = (const ko_keyed *)b;
    if (p->key != q->key)
        return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx)
        return p->idx < q->idx ? -1 : 1;
    return 0;
}

uint64_t ko_n_ones_rect(uint32_t L, uint32_t H, double composition)
{
    double N = (double)L * (double)H;
    double v = floor(composition * N + 0.5);
    if (v < 0.0)
        v = 0.0;
    if (v > N)
        v = N;
    return (uint64_t)v;
}

uint64_t ko_n_ones(uint32_t L, double composition)
{
    return ko_n_ones_rect(L, L, composition);
}

uint64_t ko_init_key(uint64_t seed, uint32_t x, uint32_t y)
{
    uint32_t key[2], ctr[4], out[4];
    seed_to_key(seed, key);
    ctr[0] = y;
    ctr[1] = x;
    ctr[2] = 0;
    ctr[3] = KO_TAG_INIT << 28;
    ko_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[0] << 32) | (uint64_t)out[1];
}

/* H rows of L sites (the square lattice is H = L). */
int ko_init_rect(uint8_t *s, uint32_t L, uint32_t H, double composition, uint64_t seed)
{
    size_t N = (size_t)L * H, i;
    uint64_t n1 = ko_n_ones_rect(L, H, composition);
    ko_keyed *ks = (ko_keyed *)malloc(N * sizeof(ko_keyed));
    if (!ks)
        return -1;
    for (i = 0; i < N; ++i) {
        ks[i].key = ko_init_key(seed, (uint32_t)(i % L), (uint32_t)(i / L));
        ks[i].idx = i;
    }
    qsort(ks, N, sizeof(ko_keyed), cmp_keyed);
    memset(s, 0, N);
    for (i = 0; i < (size_t)n1; ++i)
        s[ks[i].idx] = 1;
    free(ks);
    return 0;
}

int ko_init(uint8_t *s, uint32_t L, double composition, uint64_t seed)
{
    return ko_init_rect(s, L, L, composition, seed);
}

/* ---------------------------------------------------------------------- */
/* Cluster-size histogram: maximal 4-connected (periodic) sets of sites of */
/* one species, found by breadth-first search.  counts[s] (s = 0..N) gets  */
/* the number of clusters of exactly s sites.  Returns the cluster count.  */
/* ---------------------------------------------------------------------- */
uint64_t ko_cluster_counts(const uint8_t *s, uint32_t L, int species, uint64_t *counts)
{
    size_t N = (size_t)L * L, i;
    uint8_t *seen = (uint8_t *)calloc(N, 1);
    uint32_t *queue = (uint32_t *)malloc(N * sizeof(uint32_t));
    uint64_t clusters = 0;
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return ~(uint64_t)0;
    }
    memset(counts, 0, (N + 1) * sizeof(uint64_t));
    for (i = 0; i < N; ++i) {
        size_t head = 0, tail = 0;
        if (seen[i] || s[i] != (uint8_t)species)
            continue;
        seen[i] = 1;
        queue[tail++] = (uint32_t)i;
        while (head < tail) {
            uint32_t v = queue[head++], x = v % L, y = v / L, q;
            uint32_t nb[4];
            nb[0] = y * L + wrap_add(x, +1, L);
            nb[1] = y * L + wrap_add(x, -1, L);
            nb[2] = wrap_add(y, +1, L) * L + x;
            nb[3] = wrap_add(y, -1, L) * L + x;
            for (q = 0; q < 4; ++q)
                if (!seen[nb[q]] && s[nb[q]] == (uint8_t)species) {
                    seen[nb[q]] = 1;
                    queue[tail++] = nb[q];
                }
        }
        counts[tail] += 1;
        ++clusters;
    }
    free(seen);
    free(queue);
    return clusters;
}

/* ---------------------------------------------------------------------- */
/* Classical sequential Kawasaki chain (the paper's CPU comparison method): */
/* one step is N attempts, each at a uniformly random site with a uniformly */
/* random neighbour, accepted with probability min(1, exp(-omega*dU)) drawn */
/* from a 53-bit double.  It has its own generator (xoshiro256**, seeded by */
/* splitmix64) and shares no random numbers with the contract above; it is */
/* only compared statistically.                                             */
/* ---------------------------------------------------------------------- */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t rotl64(uint64_t v, int k)
{
    return (v << k) | (v >> (64 - k));
}

static uint64_t xoshiro_next(uint64_t st[4])
{
    uint64_t result = rotl64(st[1] * 5u, 7) * 9u;
    uint64_t tt = st[1] << 17;
    st[2] ^= st[0];
    st[3] ^= st[1];
    st[1] ^= st[2];
    st[0] ^= st[3];
    st[2] ^= tt;
    st[3] = rotl64(st[3], 45);
    return result;
}

static uint64_t below(uint64_t st[4], uint64_t n)
{
    /* unbiased draw in [0, n) by rejection */
    uint64_t lim = (~(uint64_t)0) - ((~(uint64_t)0) % n);
    uint64_t v;
    do {
        v = xoshiro_next(st);
    } while (v >= lim);
    return v % n;
}

/* Unlike bonds incident to (x,y) or (bx,by); the bond between the two is
 * counted twice, which cancels in a before/after difference. */
static int local_unlike_bonds(const uint8_t *s, uint32_t L, uint32_t x, uint32_t y, uint32_t bx, uint32_t by)
{
    uint32_t px[2], py[2];
    int k, total = 0;
    px[0] = x; py[0] = y;
    px[1] = bx; py[1] = by;
    for (k = 0; k < 2; ++k) {
        uint8_t v = s[(size_t)py[k] * L + px[k]];
        total += v != s[(size_t)py[k] * L + wrap_add(px[k], +1, L)];
        total += v != s[(size_t)py[k] * L + wrap_add(px[k], -1, L)];
        total += v != s[(size_t)wrap_add(py[k], +1, L) * L + px[k]];
        total += v != s[(size_t)wrap_add(py[k], -1, L) * L + px[k]];
    }
    return total;
}

uint64_t ko_seq_kawasaki(uint8_t *s, uint32_t L, double omega, uint64_t rng_seed, uint64_t n_steps)
{
    uint64_t st[4], sm = rng_seed, accepted = 0, step, a;
    uint64_t N = (uint64_t)L * L;
    int k;
    for (k = 0; k < 4; ++k)
        st[k] = splitmix64_next(&sm);
    for (step = 0; step < n_steps; ++step) {
        for (a = 0; a < N; ++a) {
            uint64_t site = below(st, N);
            uint32_t x = (uint32_t)(site % L), y = (uint32_t)(site / L);
            uint32_t dir = (uint32_t)below(st, 4), bx, by;
            double u = (double)(xoshiro_next(st) >> 11) * (1.0 / 9007199254740992.0);
            uint8_t *pc, *pb, tmp;
            int before, dU;
            partner_of(x, y, dir, L, &bx, &by);
            pc = &s[(size_t)y * L + x];
            pb = &s[(size_t)by * L + bx];
            if (*pc == *pb)
                continue;
            /* energy change by recount: swap, count, and undo if rejected */
            before = local_unlike_bonds(s, L, x, y, bx, by);
            tmp = *pc; *pc = *pb; *pb = tmp;
            dU = local_unlike_bonds(s, L, x, y, bx, by) - before;
            if (u < exp(-omega * (double)dU)) {
                ++accepted;
            } else {
                tmp = *pc; *pc = *pb; *pb = tmp;
            }
        }
    }
    return accepted;
}

/* ====================================================================== */
/* Triangular lattice with helical boundary conditions (the paper's own    */
/* model: Materials and Methods, "Monte Carlo model with Kawasaki based    */
/* kinetics", Fig. 2, and "Cluster Analysis methods": six neighbours under */
/* helical boundaries).                                                    */
/*                                                                         */
/* H rows of L sites, i = y*L + x, 0 <= i < N = L*H, form one ring: the   */
/* neighbours of i are i +- 1, i +- L and i +- (L - 1) modulo N (the last  */
/* site of a row is followed by the first of the next).  Schedule:         */
/* class(i) = i mod 16; for L = 4 (mod 8) and H = 0 (mod 4) two sites of   */
/* one class are at least 4 steps apart, so no exchange of a class reads a */
/* site another one writes.  A sweep visits the 16 classes in a random     */
/* order.  The paper's square lattices are H = L.                          */
/* Random numbers (Philox4x32-10, key = seed):                             */
/*   site i at sweep t: block (i div 2, 0, t_lo, t_hi28 | 6<<28), words     */
/*   2(i mod 2) (direction) and 2(i mod 2) + 1 (uniform U);                 */
/*   direction d = (word * 6) >> 32 picks offset +1, -1, +L, -L, +(L-1),   */
/*   -(L-1) for d = 0..5;                                                   */
/*   phase order: blocks (j, 0, t_lo, t_hi28 | 7<<28), j = 0..3 give       */
/*   w[0..15]; for i = 15..1 swap perm[i] with perm[(w[15-i]*(i+1)) >> 32]. */
/* Attempt: n = unlike neighbours of the centre other than the partner +   */
/* unlike neighbours of the partner other than the centre (0..10); dN_AB =  */
/* 10 - 2n; accept iff U < T[n] = min(2^32, ceil(exp(-omega(10-2n)) 2^32)). */
/* ====================================================================== */
#define KO_TAG_TRI 6u
#define KO_TAG_TRI_ORDER 7u

static int64_t tri_offset(uint32_t L, uint32_t d)
{
    static const int sign[6] = {+1, -1, +1, -1, +1, -1};
    int64_t mag = (d < 2) ? 1 : (d < 4) ? (int64_t)L : (int64_t)L - 1;
    return sign[d] * mag;
}

static uint64_t tri_nb(uint64_t i, int64_t off, uint64_t N)
{
    int64_t j = (int64_t)i + off;
    j %= (int64_t)N;
    if (j < 0) j += (int64_t)N;
    return (uint64_t)j;
}

void ko_tri_thresholds(double omega, uint64_t T[11])
{
    int n;
    for (n = 0; n <= 10; ++n) {
        double p = exp(-omega * (double)(10 - 2 * n));
        double v = ceil(p * 4294967296.0);
        T[n] = (v >= 4294967296.0) ? 4294967296ull : (uint64_t)v;
    }
}

void ko_tri_phase_order(uint64_t seed, uint64_t t, int perm[16])
{
    uint32_t key[2], ctr[4], w[16], b[4];
    int i, j;
    seed_to_key(seed, key);
    for (j = 0; j < 4; ++j) {
        ctr[0] = (uint32_t)j;
        ctr[1] = 0u;
        ctr[2] = (uint32_t)t;
        ctr[3] = ctr3(t, KO_TAG_TRI_ORDER);
        ko_philox4x32_10(ctr, key, b);
        w[4 * j] = b[0];
        w[4 * j + 1] = b[1];
        w[4 * j + 2] = b[2];
        w[4 * j + 3] = b[3];
    }
    for (i = 0; i < 16; ++i) perm[i] = i;
    for (i = 15; i >= 1; --i) {
        int k = (int)(((uint64_t)w[15 - i] * (uint64_t)(i + 1)) >> 32);
        int tmp = perm[i];
        perm[i] = perm[k];
        perm[k] = tmp;
    }
}

/* Direction (0..5) and uniform of site i at sweep t. */
void ko_tri_site_randoms(uint64_t seed, uint64_t t, uint64_t i, uint32_t *dir, uint32_t *u)
{
    uint32_t key[2], ctr[4], b[4];
    seed_to_key(seed, key);
    ctr[0] = (uint32_t)(i >> 1);
    ctr[1] = 0u;
    ctr[2] = (uint32_t)t;
    ctr[3] = ctr3(t, KO_TAG_TRI);
    ko_philox4x32_10(ctr, key, b);
    *dir = (uint32_t)(((uint64_t)b[2 * (i & 1u)] * 6u) >> 32);
    *u = b[2 * (i & 1u) + 1];
}

static int tri_unlike_except(const uint8_t *s, uint32_t L, uint32_t H, uint64_t i, uint64_t other)
{
    uint64_t N = (uint64_t)L * H;
    uint32_t d;
    int n = 0;
    for (d = 0; d < 6; ++d) {
        uint64_t j = tri_nb(i, tri_offset(L, d), N);
        if (j != other) n += (s[j] != s[i]);
    }
    return n;
}

/* dN_AB of exchanging site i with its neighbour in direction d (0 when alike). */
int ko_tri_local_dnab(const uint8_t *s, uint32_t L, uint32_t H, uint64_t i, uint32_t d)
{
    uint64_t N = (uint64_t)L * H;
    uint64_t b = tri_nb(i, tri_offset(L, d), N);
    if (s[i] == s[b]) return 0;
    return 10 - 2 * (tri_unlike_except(s, L, H, i, b) + tri_unlike_except(s, L, H, b, i));
}

uint64_t ko_tri_sweeps(uint8_t *s, uint32_t L, uint32_t H, double omega, uint64_t seed, uint64_t t0,
                       uint64_t n_sweeps)
{
    uint64_t T[11], N = (uint64_t)L * H, acc = 0, t;
    int perm[16], p;
    ko_tri_thresholds(omega, T);
    for (t = t0; t < t0 + n_sweeps; ++t) {
        ko_tri_phase_order(seed, t, perm);
        for (p = 0; p < 16; ++p) {
            int64_t i;
            uint64_t phase_acc = 0;
            /* centres of one class never interact: any order gives the same result */
#pragma omp parallel for reduction(+ : phase_acc) schedule(static)
            for (i = perm[p]; i < (int64_t)N; i += 16) {
                uint32_t d, u;
                uint64_t b;
                ko_tri_site_randoms(seed, t, (uint64_t)i, &d, &u);
                b = tri_nb((uint64_t)i, tri_offset(L, d), N);
                if (s[i] != s[b]) {
                    int n = tri_unlike_except(s, L, H, (uint64_t)i, b) + tri_unlike_except(s, L, H, b, (uint64_t)i);
                    if ((uint64_t)u < T[n]) {
                        uint8_t tmp = s[i];
                        s[i] = s[b];
                        s[b] = tmp;
                        ++phase_acc;
                    }
                }
            }
            acc += phase_acc;
        }
    }
    return acc;
}

/* N_AB over the 3N bonds (i, i+1), (i, i+L), (i, i+L-1). */
uint64_t ko_tri_energy(const uint8_t *s, uint32_t L, uint32_t H)
{
    uint64_t N = (uint64_t)L * H, i, nab = 0;
    for (i = 0; i < N; ++i) {
        nab += (s[i] != s[tri_nb(i, 1, N)]);
        nab += (s[i] != s[tri_nb(i, (int64_t)L, N)]);
        nab += (s[i] != s[tri_nb(i, (int64_t)L - 1, N)]);
    }
    return nab;
}

/* Cluster counts of one species, six neighbours, helical boundaries (BFS). */
uint64_t ko_tri_cluster_counts(const uint8_t *s, uint32_t L, uint32_t H, int species, uint64_t *counts)
{
    uint64_t N = (uint64_t)L * H, i, nclusters = 0;
    uint8_t *seen = (uint8_t *)calloc(N, 1);
    uint64_t *queue = (uint64_t *)malloc(N * sizeof(uint64_t));
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return ~(uint64_t)0;
    }
    for (i = 0; i <= N; ++i) counts[i] = 0;
    for (i = 0; i < N; ++i) {
        uint64_t head = 0, tail = 0;
        if (s[i] != species || seen[i]) continue;
        seen[i] = 1;
        queue[tail++] = i;
        while (head < tail) {
            uint64_t c = queue[head++];
            uint32_t d;
            for (d = 0; d < 6; ++d) {
                uint64_t j = tri_nb(c, tri_offset(L, d), N);
                if (s[j] == species && !seen[j]) {
                    seen[j] = 1;
                    queue[tail++] = j;
                }
            }
        }
        counts[tail] += 1;
        ++nclusters;
    }
    free(seen);
    free(queue);
    return nclusters;
}

/* Random-neighbour similar count on the triangular lattice: site i draws   */
/* d = (word * 6) >> 32 from word (i mod 4) of Philox block                 */
/* (i div 4, 1, t_lo, t_hi28 | TAG_OBSERVE<<28).                             */
uint64_t ko_tri_similar_sampled(const uint8_t *s, uint32_t L, uint32_t H, uint64_t seed, uint64_t t)
{
    uint32_t key[2], ctr[4], w[4];
    uint64_t N = (uint64_t)L * H, i, same = 0;
    seed_to_key(seed, key);
    for (i = 0; i < N; ++i) {
        uint32_t d;
        if ((i & 3u) == 0) {
            ctr[0] = (uint32_t)(i >> 2);
            ctr[1] = 1u;
            ctr[2] = (uint32_t)t;
            ctr[3] = ctr3(t, KO_TAG_OBSERVE);
            ko_philox4x32_10(ctr, key, w);
        }
        d = (uint32_t)(((uint64_t)w[i & 3u] * 6u) >> 32);
        same += (s[i] == s[tri_nb(i, tri_offset(L, d), N)]);
    }
    return same;
}

/* Sequential random-site Kawasaki on the triangular helical lattice (the
 * classical method the paper compares MPKK against, Materials and Methods and
 * Results, "MPKK vs. Kawasaki method"): N attempts per step, each picking a
 * uniform site, one of its six neighbours, and accepting the exchange with
 * probability min(1, exp(-omega dN_AB)), dN_AB by recounting the unlike bonds
 * of both sites before and after.  Its own xoshiro256** stream. */
static int tri_bonds_of_pair(const uint8_t *s, uint32_t L, uint32_t H, uint64_t a, uint64_t b)
{
    uint64_t N = (uint64_t)L * H;
    uint32_t d;
    int n = 0;
    for (d = 0; d < 6; ++d) {
        uint64_t j = tri_nb(a, tri_offset(L, d), N);
        n += (s[a] != s[j]);
    }
    for (d = 0; d < 6; ++d) {
        uint64_t j = tri_nb(b, tri_offset(L, d), N);
        if (j != a) n += (s[b] != s[j]);   /* the bond a-b was counted from a */
    }
    return n;
}

uint64_t ko_tri_seq_kawasaki(uint8_t *s, uint32_t L, uint32_t H, double omega, uint64_t rng_seed,
                            uint64_t n_steps)
{
    uint64_t st[4], sm = rng_seed, accepted = 0, step, a;
    uint64_t N = (uint64_t)L * H;
    int k;
    for (k = 0; k < 4; ++k)
        st[k] = splitmix64_next(&sm);
    for (step = 0; step < n_steps; ++step) {
        for (a = 0; a < N; ++a) {
            uint64_t c = below(st, N);
            uint32_t d = (uint32_t)below(st, 6);
            double u = (double)(xoshiro_next(st) >> 11) * (1.0 / 9007199254740992.0);
            uint64_t b = tri_nb(c, tri_offset(L, d), N);
            uint8_t tmp;
            int before, dU;
            if (s[c] == s[b])
                continue;
            before = tri_bonds_of_pair(s, L, H, c, b);
            tmp = s[c]; s[c] = s[b]; s[b] = tmp;
            dU = tri_bonds_of_pair(s, L, H, c, b) - before;
            if (u < exp(-omega * (double)dU)) {
                ++accepted;
            } else {
                tmp = s[c]; s[c] = s[b]; s[b] = tmp;
            }
        }
    }
    return accepted;
}

/* ====================================================================== */
/* The paper's literal MPKK (Materials and Methods, "Massive Parallel      */
/* Kawasaki Kinetics", Fig. 4): the ring is covered by 7-site domains (a   */
/* centre and its six neighbours).  With H rows of L sites, L = 3 or 5     */
/* (mod 7) and H = 0 (mod 7), the domains centred on the sites c = k       */
/* (mod 7) partition the ring for each k = 0..6 (the offsets 0, +-1, +-L,  */
/* +-(L-1) meet every residue mod 7 once).  One step is 7 iterations; each */
/* draws k uniformly, with replacement, and makes one Kawasaki attempt in  */
/* every domain of D(k) at once: the centre picks one of its six           */
/* neighbours.  "At once" is read as synchronous: every domain decides     */
/* from the lattice as it stood at the start of the iteration, then all    */
/* accepted exchanges are applied (domains are disjoint, so no two write   */
/* one site).  Decisions that read a site an adjacent domain exchanges are */
/* the conflicts whose bias this variant exists to measure.                */
/* Random numbers (Philox4x32-10, key = seed), step t, iteration j:        */
/*   k_j = (w * 7) >> 32, w = word (j mod 4) of block (j div 4, 2, t_lo,   */
/*   t_hi28 | 8<<28);                                                       */
/*   domain m (centre c = k_j + 7m): block (m div 2, j, t_lo,              */
/*   t_hi28 | 9<<28), word 2(m mod 2) gives the direction d = (w*6) >> 32, */
/*   word 2(m mod 2) + 1 the uniform U; acceptance as in ko_tri_sweeps.    */
/* ====================================================================== */
#define KO_TAG_MPKK_K 8u
#define KO_TAG_MPKK 9u

int ko_mpkk_k(uint64_t seed, uint64_t t, int j)
{
    uint32_t key[2], ctr[4], b[4];
    seed_to_key(seed, key);
    ctr[0] = (uint32_t)(j >> 2);
    ctr[1] = 2u;
    ctr[2] = (uint32_t)t;
    ctr[3] = ctr3(t, KO_TAG_MPKK_K);
    ko_philox4x32_10(ctr, key, b);
    return (int)(((uint64_t)b[j & 3] * 7u) >> 32);
}

void ko_mpkk_domain_randoms(uint64_t seed, uint64_t t, int j, uint64_t m, uint32_t *dir, uint32_t *u)
{
    uint32_t key[2], ctr[4], b[4];
    seed_to_key(seed, key);
    ctr[0] = (uint32_t)(m >> 1);
    ctr[1] = (uint32_t)j;
    ctr[2] = (uint32_t)t;
    ctr[3] = ctr3(t, KO_TAG_MPKK);
    ko_philox4x32_10(ctr, key, b);
    *dir = (uint32_t)(((uint64_t)b[2 * (m & 1u)] * 6u) >> 32);
    *u = b[2 * (m & 1u) + 1];
}

/* One synchronous iteration over the domains of D(k) with the given
 * directions and uniforms (one per domain, m = 0 .. N/7 - 1).  Returns the
 * accepted exchanges; -1 on allocation failure. */
int64_t ko_mpkk_iteration(uint8_t *s, uint32_t L, uint32_t H, int k, const uint32_t *dir, const uint32_t *u,
                          const uint64_t T[11])
{
    uint64_t N = (uint64_t)L * H, m;
    int64_t acc = 0;
    uint8_t *old = (uint8_t *)malloc(N);
    if (!old)
        return -1;
    memcpy(old, s, N);
    for (m = 0; m < N / 7; ++m) {
        uint64_t c = (uint64_t)k + 7 * m;
        uint64_t b = tri_nb(c, tri_offset(L, dir[m]), N);
        if (old[c] != old[b]) {
            int n = tri_unlike_except(old, L, H, c, b) + tri_unlike_except(old, L, H, b, c);
            if ((uint64_t)u[m] < T[n]) {
                s[c] = old[b];
                s[b] = old[c];
                ++acc;
            }
        }
    }
    free(old);
    return acc;
}

uint64_t ko_mpkk_steps(uint8_t *s, uint32_t L, uint32_t H, double omega, uint64_t seed, uint64_t t0,
                       uint64_t n_steps)
{
    uint64_t T[11], N = (uint64_t)L * H, M = N / 7, acc = 0, t, m;
    uint32_t *dir = (uint32_t *)malloc(M * sizeof(uint32_t));
    uint32_t *u = (uint32_t *)malloc(M * sizeof(uint32_t));
    int j;
    if (!dir || !u) {
        free(dir);
        free(u);
        return ~(uint64_t)0;
    }
    ko_tri_thresholds(omega, T);
    for (t = t0; t < t0 + n_steps; ++t) {
        for (j = 0; j < 7; ++j) {
            int k = ko_mpkk_k(seed, t, j);
            int64_t a;
            for (m = 0; m < M; ++m)
                ko_mpkk_domain_randoms(seed, t, j, m, &dir[m], &u[m]);
            a = ko_mpkk_iteration(s, L, H, k, dir, u, T);
            if (a < 0) {
                acc = ~(uint64_t)0;
                goto out;
            }
            acc += (uint64_t)a;
        }
    }
out:
    free(dir);
    free(u);
    return acc;
}

/* Threads of the OpenMP loops over the centres of one class (timing only: the
 * result does not depend on it).  n <= 0 leaves the setting unchanged; returns
 * the thread count now in force (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int ko_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/*
 * oracle.c -- plain, slow CPU reference for the state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: it is written from the paper's definitions alone.
 *
 * Arithmetic is complex128 (pairs of IEEE doubles, interleaved re,im), built
 * with -ffp-contract=off so that no fused multiply-add changes rounding.  No
 * fusion, no blocking, no qubit reordering: one gate at a time, in circuit
 * order, straight from the definition.
 *
 * Conventions (paper, Sec. II-A, Eq. 1-3):
 *   - amplitude a_i of basis state |i>, qubit q <-> bit q of i (q0 = LSB);
 *   - a k-qubit gate with target list t[0..k-1] is a 2^k x 2^k matrix whose
 *     local row/column index r has bit (k-1-j) equal to the bit of qubit t[j]
 *     (the first listed qubit is the most significant, as in Eq. 3 where the
 *     first listed qubit i is the control of CNOT and the high local bit).
 *
 * The OpenMP loops only split independent base indices between threads; the
 * per-element arithmetic and its order do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

/* Scatter the bits of local index r onto the target qubit positions:
 * bit (k-1-j) of r goes to bit t[j].  (Eq. 2 / Eq. 3 index pattern.) */
static i64 or_local_to_global(i64 r, int k, const int *t)
{
    i64 off = 0;
    for (int j = 0; j < k; ++j)
        if ((r >> (k - 1 - j)) & 1) off |= (i64)1 << t[j];
    return off;
}

/*
 * Apply one k-qubit gate (Eq. 2 for k = 1, Eq. 3 pattern for k >= 2).
 * For every base index whose target bits are all zero, gather the 2^k
 * amplitudes v[c] = a[base | scatter(c)], then write
 *     a[base | scatter(r)] = sum_{c ascending} U[r][c] * v[c].
 * U is row-major, interleaved (re, im).  Returns 0, or -1 on bad arguments.
 */
int or_apply_gate(double *psi, int n, int k, const int *t, const double *U)
{
    if (k < 1 || k > 10 || n < 1 || n > 40) return -1;
    i64 tmask = 0;
    for (int j = 0; j < k; ++j) {
        if (t[j] < 0 || t[j] >= n) return -1;
        if (tmask & ((i64)1 << t[j])) return -1;
        tmask |= (i64)1 << t[j];
    }
    const i64 N = (i64)1 << n;
    const int d = 1 << k;
    i64 *off = (i64 *)malloc(sizeof(i64) * d);
    for (int r = 0; r < d; ++r) off[r] = or_local_to_global(r, k, t);

#pragma omp parallel
    {
        double *vr = (double *)malloc(sizeof(double) * d);
        double *vi = (double *)malloc(sizeof(double) * d);
#pragma omp for schedule(static)
        for (i64 base = 0; base < N; ++base) {
            if (base & tmask) continue;
            for (int c = 0; c < d; ++c) {
                vr[c] = psi[2 * (base | off[c])];
                vi[c] = psi[2 * (base | off[c]) + 1];
            }
            for (int r = 0; r < d; ++r) {
                double sr = 0.0, si = 0.0;
                for (int c = 0; c < d; ++c) {
                    double ur = U[2 * (r * d + c)], ui = U[2 * (r * d + c) + 1];
                    sr += ur * vr[c] - ui * vi[c];
                    si += ur * vi[c] + ui * vr[c];
                }
                psi[2 * (base | off[r])] = sr;
                psi[2 * (base | off[r]) + 1] = si;
            }
        }
        free(vr);
        free(vi);
    }
    free(off);
    return 0;
}

/* Apply a whole gate list in order.  gate g has k[g] qubits, targets at
 * t[5*g .. 5*g+k[g]-1], and its matrix follows the previous gate's in mats
 * (2 * 4^k doubles each). */
int or_apply_circuit(double *psi, int n, int ngates, const int *k, const int *t, const double *mats)
{
    const double *m = mats;
    for (int g = 0; g < ngates; ++g) {
        int rc = or_apply_gate(psi, n, k[g], t + 5 * g, m);
        if (rc) return rc;
        m += 2 * ((i64)1 << (2 * k[g]));
    }
    return 0;
}

/* |0...0> : a_0 = 1, all others 0 (Alg. 3 input, "the initialized stateVector"). */
void or_init_zero(double *psi, int n)
{
    const i64 N = (i64)1 << n;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < N; ++i) { psi[2 * i] = 0.0; psi[2 * i + 1] = 0.0; }
    psi[0] = 1.0;
}

/*
 * Qubit swap (Eq. 4): exchange index bits a[j] <-> b[j] for j < s.
 * out[swapbits(i)] = in[i].  Done in place: the map is an involution, so
 * each pair {i, swapbits(i)} is exchanged once, by its smaller member.
 */
int or_swap_qubits(double *psi, int n, int s, const int *a, const int *b)
{
    i64 used = 0;
    for (int j = 0; j < s; ++j) {
        if (a[j] < 0 || a[j] >= n || b[j] < 0 || b[j] >= n || a[j] == b[j]) return -1;
        i64 ma = (i64)1 << a[j], mb = (i64)1 << b[j];
        if ((used & ma) || (used & mb)) return -1;
        used |= ma | mb;
    }
    const i64 N = (i64)1 << n;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < N; ++i) {
        i64 m = i;
        for (int j = 0; j < s; ++j) {
            i64 ba = (i >> a[j]) & 1, bb = (i >> b[j]) & 1;
            m &= ~(((i64)1 << a[j]) | ((i64)1 << b[j]));
            m |= (bb << a[j]) | (ba << b[j]);
        }
        if (m > i) {
            double r0 = psi[2 * i], i0 = psi[2 * i + 1];
            psi[2 * i] = psi[2 * m];
            psi[2 * i + 1] = psi[2 * m + 1];
            psi[2 * m] = r0;
            psi[2 * m + 1] = i0;
        }
    }
    return 0;
}

/* Probabilities p_i = |a_i|^2 (Eq. 1; the text's a_i^2 read as |a_i|^2). */
void or_probs(const double *psi, int n, double *p)
{
    const i64 N = (i64)1 << n;
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < N; ++i) p[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
}

/*
 * Expectation of one Pauli string P with per-qubit letters given by
 * (x_q, z_q): (0,0)=I, (1,0)=X, (0,1)=Z, (1,1)=Y.  P|i> = ph(i) |i ^ x>,
 * ph(i) = i^{#Y} * (-1)^{popcount(i & z)}.  <P> = sum_i conj(a_{i^x}) ph(i) a_i,
 * summed in ascending i (single thread, fixed order).  Writes re and im.
 */
void or_expect_pauli(const double *psi, int n, unsigned long long x, unsigned long long z,
                     double *out_re, double *out_im)
{
    const i64 N = (i64)1 << n;
    int ny = __builtin_popcountll(x & z) & 3;
    /* i^ny */
    double pr = (ny == 0) ? 1.0 : (ny == 2) ? -1.0 : 0.0;
    double pim = (ny == 1) ? 1.0 : (ny == 3) ? -1.0 : 0.0;
    double sr = 0.0, si = 0.0;
    for (i64 i = 0; i < N; ++i) {
        i64 j = i ^ (i64)x;
        double sign = (__builtin_popcountll((unsigned long long)i & z) & 1) ? -1.0 : 1.0;
        double ar = psi[2 * i], ai = psi[2 * i + 1];
        /* ph * a_i */
        double tr = sign * (pr * ar - pim * ai);
        double ti = sign * (pr * ai + pim * ar);
        /* conj(a_j) * t */
        double br = psi[2 * j], bi = -psi[2 * j + 1];
        sr += br * tr - bi * ti;
        si += br * ti + bi * tr;
    }
    *out_re = sr;
    *out_im = si;
}

/* sum_i |a_i|^2 */
double or_norm2(const double *psi, int n)
{
    const i64 N = (i64)1 << n;
    double s = 0.0;
    for (i64 i = 0; i < N; ++i) s += psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    return s;
}

/*
 * MaxCut cost of basis state z: C(z) = number of edges (u,v) whose
 * endpoints lie on different sides, i.e. bit u of z != bit v of z.
 */
static int or_cut(i64 z, int nedges, const int *edges)
{
    int c = 0;
    for (int e = 0; e < nedges; ++e)
        c += (int)(((z >> edges[2 * e]) ^ (z >> edges[2 * e + 1])) & 1);
    return c;
}

/* Cost layer of QAOA: a_z <- exp(-i * gamma * C(z)) * a_z (definition of e^{-i gamma C}). */
void or_qaoa_cost_phase(double *psi, int n, int nedges, const int *edges, double gamma)
{
    const i64 N = (i64)1 << n;
#pragma omp parallel for schedule(static)
    for (i64 z = 0; z < N; ++z) {
        double th = -gamma * (double)or_cut(z, nedges, edges);
        double c = cos(th), s = sin(th);
        double ar = psi[2 * z], ai = psi[2 * z + 1];
        psi[2 * z] = c * ar - s * ai;
        psi[2 * z + 1] = c * ai + s * ar;
    }
}

/* <C> = sum_z |a_z|^2 C(z), ascending z. */
double or_maxcut_expect(const double *psi, int n, int nedges, const int *edges)
{
    const i64 N = (i64)1 << n;
    double s = 0.0;
    for (i64 z = 0; z < N; ++z) {
        double p = psi[2 * z] * psi[2 * z] + psi[2 * z + 1] * psi[2 * z + 1];
        s += p * (double)or_cut(z, nedges, edges);
    }
    return s;
}

/* Number of OpenMP threads the parallel loops use (1 without OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

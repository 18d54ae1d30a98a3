/*
 * FP64 state-vector oracle -- TEST INFRASTRUCTURE, not part of the product.
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code with the HIP path.
 *
 * What it computes is the plain definition of an output amplitude, Eq. (fpath)
 * of Sec. III.A: start from |0...0>, apply the circuit's unitaries in time
 * order, and read <x|U|0...0> off the final state vector.  Gates are given to
 * it already expanded into 2x2 complex matrices (single-qubit gates, Sec. III.B)
 * or marked as CZ = diag(1,1,1,-1); the caller owns the gate tables.
 *
 * Index convention: basis state index i = sum_q x_q 2^q (bit q = qubit q).
 * Complex numbers are interleaved (re, im) doubles.
 *
 * The gradient routine is the adjoint-state method: one forward sweep, then a
 * backward sweep that uncomputes the state gate by gate (with the exact 2x2
 * inverse) while pulling the seed vector back through U^dagger; the
 * environment of gate g is M_g[a][b] = sum_rest conj(Phi[a,rest]) psi[b,rest].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { double re, im; } cd;

static inline cd cmul(cd a, cd b) { cd r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cd cadd(cd a, cd b) { cd r = {a.re + b.re, a.im + b.im}; return r; }
static inline cd cconj(cd a) { cd r = {a.re, -a.im}; return r; }

/* op_q[2*g] = q0, op_q[2*g+1] = q1 (-1 for a single-qubit gate).
 * op_m[8*g .. 8*g+7] = m00, m01, m10, m11 (re, im), row = output bit. */
static void apply_1q(cd* psi, int64_t dim, int q, const double* m) {
    const cd m00 = {m[0], m[1]}, m01 = {m[2], m[3]}, m10 = {m[4], m[5]}, m11 = {m[6], m[7]};
    const int64_t bit = (int64_t)1 << q;
    const int64_t half = dim >> 1;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < half; ++p) {
        int64_t i = ((p >> q) << (q + 1)) | (p & (bit - 1));
        int64_t j = i | bit;
        cd a = psi[i], b = psi[j];
        psi[i] = cadd(cmul(m00, a), cmul(m01, b));
        psi[j] = cadd(cmul(m10, a), cmul(m11, b));
    }
}

static void apply_cz(cd* psi, int64_t dim, int q0, int q1) {
    const int64_t mask = ((int64_t)1 << q0) | ((int64_t)1 << q1);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i)
        if ((i & mask) == mask) { psi[i].re = -psi[i].re; psi[i].im = -psi[i].im; }
}

static void apply_op(cd* psi, int64_t dim, const int32_t* op_q, const double* op_m, int g) {
    if (op_q[2 * g + 1] >= 0) apply_cz(psi, dim, op_q[2 * g], op_q[2 * g + 1]);
    else apply_1q(psi, dim, op_q[2 * g], op_m + 8 * g);
}

static int check_ops(int n, int n_ops, const int32_t* op_q) {
    if (n < 1 || n > 34) return -1;
    for (int g = 0; g < n_ops; ++g) {
        int q0 = op_q[2 * g], q1 = op_q[2 * g + 1];
        if (q0 < 0 || q0 >= n || q1 >= n || q1 == q0) return -1;
    }
    return 0;
}

/* Final state U|0...0> into psi (2^n complex). */
int oracle_sv_state(int n, int n_ops, const int32_t* op_q, const double* op_m, double* psi_out) {
    if (check_ops(n, n_ops, op_q)) return -1;
    const int64_t dim = (int64_t)1 << n;
    cd* psi = (cd*)psi_out;
    memset(psi, 0, sizeof(cd) * (size_t)dim);
    psi[0].re = 1.0;
    for (int g = 0; g < n_ops; ++g) apply_op(psi, dim, op_q, op_m, g);
    return 0;
}

/* amps[b] = <bits[b]| U |0...0>, all B of them from one state-vector sweep. */
int oracle_sv_amplitudes(int n, int n_ops, const int32_t* op_q, const double* op_m,
                         const uint64_t* bits, int64_t B, double* amps_out) {
    if (check_ops(n, n_ops, op_q)) return -1;
    const int64_t dim = (int64_t)1 << n;
    cd* psi = (cd*)malloc(sizeof(cd) * (size_t)dim);
    if (!psi) return -2;
    oracle_sv_state(n, n_ops, op_q, op_m, (double*)psi);
    cd* amps = (cd*)amps_out;
    for (int64_t b = 0; b < B; ++b) amps[b] = psi[bits[b] & (uint64_t)(dim - 1)];
    free(psi);
    return 0;
}

static void inverse2(const double* m, double* inv) {
    cd a = {m[0], m[1]}, b = {m[2], m[3]}, c = {m[4], m[5]}, d = {m[6], m[7]};
    cd det = cadd(cmul(a, d), cmul((cd){-b.re, -b.im}, c));
    double den = det.re * det.re + det.im * det.im;
    cd idet = {det.re / den, -det.im / den};
    cd r00 = cmul(d, idet), r01 = cmul((cd){-b.re, -b.im}, idet);
    cd r10 = cmul((cd){-c.re, -c.im}, idet), r11 = cmul(a, idet);
    double o[8] = {r00.re, r00.im, r01.re, r01.im, r10.re, r10.im, r11.re, r11.im};
    memcpy(inv, o, sizeof o);
}

static void dagger2(const double* m, double* dg) {
    /* (U^dagger)[a][b] = conj(U[b][a]) */
    double o[8] = {m[0], -m[1], m[4], -m[5], m[2], -m[3], m[6], -m[7]};
    memcpy(dg, o, sizeof o);
}

/* Vector-Jacobian product of the amplitudes with respect to every
 * single-qubit gate matrix.  grad_amps[b] is dL/dRe A_b + i dL/dIm A_b for a
 * real loss L (the torch convention); env_out[g] receives, for each op g that
 * is a single-qubit gate, G_g[a][b] = dL/dRe U_g[a][b] + i dL/dIm U_g[a][b]
 * (CZ ops get zeros).  amps_out receives the amplitudes of the forward sweep.
 * Requires every single-qubit matrix to be invertible. */
int oracle_sv_vjp(int n, int n_ops, const int32_t* op_q, const double* op_m,
                  const uint64_t* bits, int64_t B, const double* grad_amps,
                  double* amps_out, double* env_out) {
    if (check_ops(n, n_ops, op_q)) return -1;
    const int64_t dim = (int64_t)1 << n;
    cd* psi = (cd*)malloc(sizeof(cd) * (size_t)dim);
    cd* phi = (cd*)calloc((size_t)dim, sizeof(cd));
    if (!psi || !phi) { free(psi); free(phi); return -2; }
    oracle_sv_state(n, n_ops, op_q, op_m, (double*)psi);
    const cd* gin = (const cd*)grad_amps;
    cd* amps = (cd*)amps_out;
    for (int64_t b = 0; b < B; ++b) {
        int64_t i = (int64_t)(bits[b] & (uint64_t)(dim - 1));
        amps[b] = psi[i];
        phi[i] = cadd(phi[i], gin[b]);           /* Phi = sum_x grad_x |x> */
    }
    memset(env_out, 0, sizeof(double) * 8 * (size_t)n_ops);
    for (int g = n_ops - 1; g >= 0; --g) {
        if (op_q[2 * g + 1] >= 0) {              /* CZ is its own inverse and adjoint */
            apply_cz(psi, dim, op_q[2 * g], op_q[2 * g + 1]);
            apply_cz(phi, dim, op_q[2 * g], op_q[2 * g + 1]);
            continue;
        }
        const int q = op_q[2 * g];
        double inv[8], dg[8];
        inverse2(op_m + 8 * g, inv);
        dagger2(op_m + 8 * g, dg);
        apply_1q(psi, dim, q, inv);              /* psi: state before gate g */
        const int64_t bit = (int64_t)1 << q, half = dim >> 1;
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0, a3r = 0, a3i = 0;
#pragma omp parallel for schedule(static) reduction(+ : a0r, a0i, a1r, a1i, a2r, a2i, a3r, a3i)
        for (int64_t p = 0; p < half; ++p) {
            int64_t i = ((p >> q) << (q + 1)) | (p & (bit - 1));
            int64_t j = i | bit;
            cd f0 = cconj(phi[i]), f1 = cconj(phi[j]);
            cd s0 = psi[i], s1 = psi[j];
            cd t;
            t = cmul(f0, s0); a0r += t.re; a0i += t.im;   /* M[0][0] */
            t = cmul(f0, s1); a1r += t.re; a1i += t.im;   /* M[0][1] */
            t = cmul(f1, s0); a2r += t.re; a2i += t.im;   /* M[1][0] */
            t = cmul(f1, s1); a3r += t.re; a3i += t.im;   /* M[1][1] */
        }
        acc[0] = a0r; acc[1] = -a0i; acc[2] = a1r; acc[3] = -a1i;   /* G = conj(M) */
        acc[4] = a2r; acc[5] = -a2i; acc[6] = a3r; acc[7] = -a3i;
        memcpy(env_out + 8 * g, acc, sizeof acc);
        apply_1q(phi, dim, q, dg);               /* Phi <- U_g^dagger Phi */
    }
    free(psi);
    free(phi);
    return 0;
}

/* Host driver of the state-vector oracle for the sanitizer build.  Reads
 * "n n_ops B", n_ops lines "q0 q1 m0..m7", B bitstrings and B gradient seeds
 * (re im), and prints the amplitudes and the vector-Jacobian product of the
 * oracle (one value per line, %.17g). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sv_amplitudes(int n, int n_ops, const int32_t* op_q, const double* op_m, const uint64_t* bits, int64_t B,
                         double* amps_out);
int oracle_sv_vjp(int n, int n_ops, const int32_t* op_q, const double* op_m, const uint64_t* bits, int64_t B,
                  const double* grad_amps, double* amps_out, double* op_grads);

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "r");
    if (!f) return 2;
    int n, n_ops;
    long long B;
    if (fscanf(f, "%d %d %lld", &n, &n_ops, &B) != 3) return 2;
    int32_t* q = malloc(sizeof(int32_t) * 2 * (size_t)n_ops);
    double* m = malloc(sizeof(double) * 8 * (size_t)n_ops);
    uint64_t* bits = malloc(sizeof(uint64_t) * (size_t)B);
    double* g = malloc(sizeof(double) * 2 * (size_t)B);
    double* a = malloc(sizeof(double) * 2 * (size_t)B);
    double* og = malloc(sizeof(double) * 8 * (size_t)n_ops);
    for (int i = 0; i < n_ops; ++i) {
        if (fscanf(f, "%d %d", &q[2 * i], &q[2 * i + 1]) != 2) return 2;
        for (int k = 0; k < 8; ++k)
            if (fscanf(f, "%lf", &m[8 * i + k]) != 1) return 2;
    }
    for (long long b = 0; b < B; ++b) {
        unsigned long long x;
        if (fscanf(f, "%llu", &x) != 1) return 2;
        bits[b] = x;
    }
    for (long long b = 0; b < 2 * B; ++b)
        if (fscanf(f, "%lf", &g[b]) != 1) return 2;
    fclose(f);
    if (oracle_sv_amplitudes(n, n_ops, q, m, bits, B, a)) return 3;
    for (long long b = 0; b < 2 * B; ++b) printf("%.17g\n", a[b]);
    if (oracle_sv_vjp(n, n_ops, q, m, bits, B, g, a, og)) return 3;
    for (long long i = 0; i < 8LL * n_ops; ++i) printf("%.17g\n", og[i]);
    free(q); free(m); free(bits); free(g); free(a); free(og);
    return 0;
}

/* Drives every entry point of the oracle (oracle/oracle.c) on small inputs,
 * both edge rules, so that tests/test_host_logic.py can run it under
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Prints one checksum line. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_kl_roots(double lam, int M, double *w);
double oracle_kl_mu(double lam, double w);
double oracle_kl_nu(double lam, double w);
double oracle_kl_phi1d(double lam, double w, double x);
int oracle_kl_modes(double lam, int K, int M, int *mode_i, int *mode_j);
int oracle_kl_basis(int n, int K, double sigma2, double lam, double *Phi);
void oracle_set_disc(int d);
int oracle_solve_batch(int n, int K, const double *Phi, int S, const double *xi, const double *a_nodes,
                       double fconst, const double *rhs_nodal, double *Q, double *u);
int oracle_relres_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst,
                        const double *x, double *relres);
int oracle_ir_f32_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst, double delta,
                        int imax, double *Q, int *trips, double *relres);
int oracle_grad_batch(int n, int K, const double *Phi, int S, const double *xi, double fconst, double *grad,
                      double *gZ_out, double *lam_out);
double oracle_energy(int n, int K, const double *Phi, const double *xi, const double *u);
int oracle_dense_matrix(int n, int K, const double *Phi, const double *xi, double *A);
int oracle_band_matrix(int n, int K, const double *Phi, const double *xi, double *Ab);
void oracle_set_threads(int k);
int oracle_num_threads(void);

int main(void)
{
    const int K = 12, S = 5;
    double sum = 0.0;
    int bad = 0;
    double w[64];
    bad |= oracle_kl_roots(0.3, 64, w) != 0;
    sum += oracle_kl_mu(0.3, w[0]) + oracle_kl_nu(0.3, w[1]) + oracle_kl_phi1d(0.3, w[2], 0.25);
    int mi[12], mj[12];
    bad |= oracle_kl_modes(0.3, K, 64, mi, mj) != 0;
    oracle_set_threads(2);
    double xi[5 * 12];
    for (int i = 0; i < S * K; ++i) xi[i] = sin(1.7 * i + 0.3);
    for (int disc = 0; disc <= 1; ++disc) {
        oracle_set_disc(disc);
        for (int n = 4; n <= 16; n *= 2) {
            const int np = (n + 1) * (n + 1), N = (n - 1) * (n - 1);
            double *Phi = malloc(sizeof(double) * np * K);
            double *Q = malloc(sizeof(double) * S), *u = malloc(sizeof(double) * S * N);
            double *rr = malloc(sizeof(double) * S), *g = malloc(sizeof(double) * S * K);
            double *gz = malloc(sizeof(double) * S * np), *lam = malloc(sizeof(double) * S * N);
            double *A = malloc(sizeof(double) * N * N), *Ab = malloc(sizeof(double) * N * n);
            double *an = malloc(sizeof(double) * S * np), *rhs = malloc(sizeof(double) * N);
            int *trips = malloc(sizeof(int) * S);
            bad |= oracle_kl_basis(n, K, 1.0, 0.3, Phi) != 0;
            bad |= oracle_solve_batch(n, K, Phi, S, xi, NULL, 1.0, NULL, Q, u) != 0;
            for (int s = 0; s < S; ++s) sum += Q[s];
            bad |= oracle_relres_batch(n, K, Phi, S, xi, 1.0, u, rr) != 0;
            for (int s = 0; s < S; ++s) sum += rr[s];
            for (int i = 0; i < S * np; ++i) an[i] = 1.0 + 0.5 * cos(0.9 * i);
            for (int i = 0; i < N; ++i) rhs[i] = 1.0 + 0.1 * i;
            bad |= oracle_solve_batch(n, 0, NULL, S, NULL, an, 1.0, rhs, Q, NULL) != 0;
            for (int s = 0; s < S; ++s) sum += Q[s];
            oracle_ir_f32_batch(n, K, Phi, S, xi, 1.0, 1e-10, 10, Q, trips, rr);
            for (int s = 0; s < S; ++s) sum += Q[s] + trips[s];
            bad |= oracle_grad_batch(n, K, Phi, S, xi, 1.0, g, gz, lam) != 0;
            for (int i = 0; i < S * K; ++i) sum += g[i];
            sum += oracle_energy(n, K, Phi, xi, u);
            bad |= oracle_dense_matrix(n, K, Phi, xi, A) != 0;
            bad |= oracle_band_matrix(n, K, Phi, xi, Ab) != 0;
            sum += A[0] + Ab[0];
            free(Phi); free(Q); free(u); free(rr); free(g); free(gz); free(lam); free(A); free(Ab);
            free(an); free(rhs); free(trips);
        }
    }
    oracle_set_disc(0);
    printf("oracle ok=%d threads=%d sum=%.12g\n", !bad, oracle_num_threads(), sum);
    return bad;
}

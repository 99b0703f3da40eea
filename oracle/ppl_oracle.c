/*
 * Oracle -- test infrastructure only.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may call this code; the product path never does.
 *
 * Plain, slow FP64 evaluation of the particle-particle ladder (Sec. II.C,
 * eq. pp-Ladder-0):
 *
 *     R[i][j][a][b] += sum_{c,d} (ac|bd) * tau[i][j][c][d],
 *     (ac|bd)       =  sum_Q B[Q][a][c] * B[Q][b][d]          (eq. RIM)
 *
 * with the index convention v^{ab}_{cd} = (ac|bd) of eq. eri.  Nothing here is
 * blocked, packed or reordered beyond the definition: for every (a, b) the full
 * v x v matrix (a c|b d) is formed from its RI factors, then contracted with tau
 * for every (i, j).  OpenMP only splits the independent (a, b) iterations.
 *
 * Layouts (row-major, FP64): B_vv [naux][v][v] (first index external: a or b),
 * tau and R [o][o][v][v].
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* (a c | b d) for all c, d:  V[c][d] = sum_Q B[Q][a][c] B[Q][b][d] */
static void integrals_ab(const double* B, int v, int naux, int a, int b, double* V) {
    memset(V, 0, sizeof(double) * (size_t)v * v);
    for (int q = 0; q < naux; ++q) {
        const double* Ba = B + ((size_t)q * v + a) * v;
        const double* Bb = B + ((size_t)q * v + b) * v;
        for (int c = 0; c < v; ++c) {
            const double x = Ba[c];
            double* Vc = V + (size_t)c * v;
            for (int d = 0; d < v; ++d) Vc[d] += x * Bb[d];
        }
    }
}

/* L^{ab}_{ij} = sum_{cd} V[c][d] tau[i][j][c][d] */
static double contract_ij(const double* V, const double* tau, int v, int i, int j, int o) {
    const double* t = tau + ((size_t)i * o + j) * (size_t)v * v;
    double s = 0.0;
    for (size_t cd = 0; cd < (size_t)v * v; ++cd) s += V[cd] * t[cd];
    return s;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops below (n >= 1); used to time the oracle on one core
 * and on all cores. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* R += L over all (a, b, i, j). */
int oracle_ppl(const double* B_vv, const double* tau, int o, int v, int naux, double* R) {
    if (!B_vv || !tau || !R || o <= 0 || v <= 0 || naux <= 0) return 1;
    int status = 0;
#pragma omp parallel
    {
        double* V = (double*)malloc(sizeof(double) * (size_t)v * v);
        if (!V) {
#pragma omp atomic write
            status = 3;
        }
#pragma omp for schedule(dynamic, 1)
        for (long ab = 0; ab < (long)v * v; ++ab) {
            if (!V) continue;
            const int a = (int)(ab / v), b = (int)(ab % v);
            integrals_ab(B_vv, v, naux, a, b, V);
            for (int i = 0; i < o; ++i)
                for (int j = 0; j < o; ++j)
                    R[(((size_t)i * o + j) * v + a) * v + b] += contract_ij(V, tau, v, i, j, o);
        }
        free(V);
    }
    return status;
}

/* out[p][i][j] = L^{a_p b_p}_{ij} for the listed pairs (a_p, b_p) = (ab[2p], ab[2p+1]);
 * not accumulated.  Used to check a sample of a result too large to form here. */
int oracle_ppl_pairs(const double* B_vv, const double* tau, int o, int v, int naux,
                     const int* ab, int npairs, double* out) {
    if (!B_vv || !tau || !ab || !out || o <= 0 || v <= 0 || naux <= 0 || npairs < 0) return 1;
    for (int p = 0; p < npairs; ++p)
        if (ab[2 * p] < 0 || ab[2 * p] >= v || ab[2 * p + 1] < 0 || ab[2 * p + 1] >= v) return 1;
    int status = 0;
#pragma omp parallel
    {
        double* V = (double*)malloc(sizeof(double) * (size_t)v * v);
        if (!V) {
#pragma omp atomic write
            status = 3;
        }
#pragma omp for schedule(dynamic, 1)
        for (int p = 0; p < npairs; ++p) {
            if (!V) continue;
            integrals_ab(B_vv, v, naux, ab[2 * p], ab[2 * p + 1], V);
            for (int i = 0; i < o; ++i)
                for (int j = 0; j < o; ++j)
                    out[((size_t)p * o + i) * o + j] = contract_ij(V, tau, v, i, j, o);
        }
        free(V);
    }
    return status;
}

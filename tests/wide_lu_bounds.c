/* Host replica of the index arithmetic of the workgroup kernel's blocked LU
 * and triangular solves (lu_w and solve_w of the large-mechanism integrator),
 * for bounds checking under AddressSanitizer. TEST INFRASTRUCTURE ONLY.
 *
 * Every buffer the kernel touches is allocated on its own, at exactly the
 * size the kernel's layout gives it: in LDS the panel (nb_max ld doubles), the
 * U block (nb_max ld doubles, absent when the U block is read from HBM), piv,
 * perm and sig (ld ints each) and the reduction scratch (16 ints); in HBM the
 * matrix slot (n columns of ld doubles). An access outside any of them stops
 * the program with an ASan report.
 *
 * The 256 threads of the workgroup run one after the other inside each phase
 * between two barriers; wave 0's panel factorisation runs its 64 lanes in
 * lock step, with the butterfly reduction replaced by the value it computes
 * (largest |a|, NaN rule, ties to the lowest row). The loops, bounds and
 * guards follow the kernel's source line for line, so that the factors come
 * out equal to an unblocked LU in every bit (the test checks that too).
 *
 * Usage: wide_lu_bounds <out.bin> <panel width> <u_in_hbm 0|1> <n_lo> <n_hi> <pattern>
 * pattern 0: random matrices; 1: every pivot is the last row; 2: no pivoting
 * (diagonally dominant); 3: column n-1 made zero (a singular last column).
 * For each n it writes n, ld, info, the input (row-major), the factors
 * (row-major), piv and the solution of A x = b for b_i = i + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { T = 256, SB = 32 };

static int NB;          /* panel width of the variant */
static int U_HBM;       /* U block read from the matrix (1) or from LDS (0) */

typedef struct {
  double *panel, *U12;
  int *piv, *perm, *sig, *ired;
} lds_t;

static int imin(int a, int b) { return a < b ? a : b; }

static int lu_w(double* M, int n, int ld, lds_t* W) {
  for (int t = 0; t < T; ++t)
    if (t < ld) W->perm[t] = t;
  int info = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = imin(NB, n - k0);
    for (int t = 0; t < T; ++t)
      if (t < ld) {
        const int in = t >= k0 && t < n;
        for (int c = 0; c < nb; ++c) W->panel[c * ld + t] = in ? M[(k0 + c) * ld + t] : 0.0;
        W->sig[t] = t;
      }
    /* wave 0: panel factorisation, lanes in lock step */
    for (int c = 0; c < nb; ++c) {
      const int k = k0 + c;
      double* pc = W->panel + c * ld;
      double key = -1.0;
      int idx = 1 << 30;
      for (int t = 0; t < 64; ++t)
        for (int r = k + t; r < n; r += 64) {
          const double av = fabs(pc[r]);
          const double kv = (av != av) ? (r == k ? INFINITY : -1.0) : av;
          if (kv > key || (kv == key && r < idx)) {
            key = kv;
            idx = r;
          }
        }
      const int pv = idx;
      W->piv[k] = pv;
      {
        const int tmp = W->perm[k];
        W->perm[k] = W->perm[pv];
        W->perm[pv] = tmp;
        const int tms = W->sig[k];
        W->sig[k] = W->sig[pv];
        W->sig[pv] = tms;
      }
      if (pv != k)
        for (int t = 0; t < 64; ++t)
          if (t < nb) {
            double* q = W->panel + t * ld;
            const double tmp = q[k];
            q[k] = q[pv];
            q[pv] = tmp;
          }
      const double akk = pc[k];
      if (akk == 0.0) {
        if (!info) info = k + 1;
        continue;
      }
      for (int t = 0; t < 64; ++t)
        for (int r = k + 1 + t; r < n; r += 64) {
          const double l = pc[r] / akk;
          pc[r] = l;
          for (int c2 = c + 1; c2 < nb; ++c2) {
            double* q = W->panel + c2 * ld;
            q[r] = q[r] - l * q[k];
          }
        }
    }
    W->ired[15] = info;
    info = W->ired[15];
    for (int t = 0; t < T; ++t)
      if (t < ld && t >= k0 && t < n)
        for (int c = 0; c < nb; ++c) M[(k0 + c) * ld + t] = W->panel[c * ld + t];
    /* interchanges on the other columns: sources of a column read before any
     * destination of it is written */
    for (int t = 0; t < T; ++t)
      for (int j = t; j < n; j += T) {
        if (j >= k0 && j < k0 + nb) continue;
        double* col = M + j * ld;
        double va[16], vb[16];
        for (int c = 0; c < NB; ++c) {
          const int ia = k0 + c, ib = c < nb ? W->piv[k0 + c] : ia;
          va[c] = (c < nb && W->sig[ia] != ia) ? col[W->sig[ia]] : 0.0;
          vb[c] = (c < nb && W->sig[ib] != ib) ? col[W->sig[ib]] : 0.0;
        }
        for (int c = 0; c < NB; ++c) {
          const int ia = k0 + c, ib = c < nb ? W->piv[k0 + c] : ia;
          if (c < nb && W->sig[ia] != ia) col[ia] = va[c];
          if (c < nb && W->sig[ib] != ib) col[ib] = vb[c];
        }
      }
    const int j0 = k0 + nb, m = n - j0;
    if (m > 0) {
      for (int t = 0; t < T; ++t)
        for (int j = j0 + t; j < n; j += T) {
          double* col = M + j * ld;
          double x[16];
          for (int q = 0; q < NB; ++q) x[q] = q < nb ? col[k0 + q] : 0.0;
          for (int q = 1; q < NB; ++q)
            for (int q2 = 0; q2 < q; ++q2)
              if (q < nb) x[q] = x[q] - W->panel[q2 * ld + k0 + q] * x[q2];
          for (int q = 0; q < NB; ++q)
            if (q < nb) {
              col[k0 + q] = x[q];
              if (!U_HBM) W->U12[(j - j0) * NB + q] = x[q];
            }
        }
      for (int t = 0; t < T; ++t) {
        const int half = t >> 7, rl = t & 127;
        for (int rb = rl; rb < m; rb += 128) {
          const int r = j0 + rb;
          double lr[16];
          for (int q = 0; q < NB; ++q) lr[q] = q < nb ? W->panel[q * ld + r] : 0.0;
          for (int jb = half; jb < m; jb += 16) {
            double av[8];
            for (int i = 0; i < 8; ++i) {
              const int jj = jb + 2 * i;
              av[i] = jj < m ? M[(j0 + jj) * ld + r] : 0.0;
            }
            for (int i = 0; i < 8; ++i) {
              const int jj = jb + 2 * i;
              if (jj < m) {
                for (int q = 0; q < NB; ++q) {
                  if (q >= nb) continue;
                  const double u = U_HBM ? M[(j0 + jj) * ld + k0 + q] : W->U12[jj * NB + q];
                  av[i] = av[i] - lr[q] * u;
                }
                M[(j0 + jj) * ld + r] = av[i];
              }
            }
          }
        }
      }
    }
  }
  return info;
}

static void solve_w(const double* M, int n, int ld, const lds_t* W, const double* b, double* x) {
  for (int t = 0; t < T; ++t)
    if (t < n) x[t] = b[W->perm[t]];
  for (int k0 = 0; k0 < n; k0 += SB) {
    const int nb = imin(SB, n - k0);
    /* wave 0: lower triangle of the block, lanes in lock step */
    double lc[64][SB], xv[64];
    for (int t = 0; t < 64; ++t) {
      for (int q = 0; q < SB; ++q) lc[t][q] = (q + 1 < nb && t > q && t < nb) ? M[(k0 + q) * ld + k0 + t] : 0.0;
      xv[t] = t < nb ? x[k0 + t] : 0.0;
    }
    for (int q = 0; q + 1 < SB; ++q)
      if (q + 1 < nb) {
        const double z = xv[q];
        for (int t = 0; t < 64; ++t)
          if (t > q && t < nb) xv[t] = xv[t] - lc[t][q] * z;
      }
    for (int t = 0; t < 64; ++t)
      if (t < nb) x[k0 + t] = xv[t];
    for (int t = 0; t < T; ++t)
      for (int r = k0 + nb + t; r < n; r += T) {
        double lv[SB];
        for (int q = 0; q < SB; ++q) lv[q] = q < nb ? M[(k0 + q) * ld + r] : 0.0;
        double a = x[r];
        for (int q = 0; q < SB; ++q)
          if (q < nb) a = a - lv[q] * x[k0 + q];
        x[r] = a;
      }
  }
  for (int k0 = ((n - 1) / SB) * SB; k0 >= 0; k0 -= SB) {
    const int nb = imin(SB, n - k0);
    double uc[64][SB], dg[64], xv[64];
    for (int t = 0; t < 64; ++t) {
      for (int q = 0; q < SB; ++q) uc[t][q] = (q < nb && t < q) ? M[(k0 + q) * ld + k0 + t] : 0.0;
      dg[t] = t < nb ? M[(k0 + t) * ld + k0 + t] : 1.0;
      xv[t] = t < nb ? x[k0 + t] : 0.0;
    }
    for (int q = SB - 1; q >= 0; --q)
      if (q < nb) {
        const double z = xv[q] / dg[q];
        for (int t = 0; t < 64; ++t) {
          if (t == q) xv[t] = z;
          else if (t < q) xv[t] = xv[t] - uc[t][q] * z;
        }
      }
    for (int t = 0; t < 64; ++t)
      if (t < nb) x[k0 + t] = xv[t];
    for (int t = 0; t < T; ++t)
      for (int r = t; r < k0; r += T) {
        double uv[SB];
        for (int q = 0; q < SB; ++q) uv[q] = q < nb ? M[(k0 + q) * ld + r] : 0.0;
        double a = x[r];
        for (int q = 0; q < SB; ++q)
          if (q < nb) a = a - uv[q] * x[k0 + q];
        x[r] = a;
      }
  }
}

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double urand(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s out.bin panel u_in_hbm n_lo n_hi pattern\n", argv[0]);
    return 2;
  }
  NB = atoi(argv[2]);
  U_HBM = atoi(argv[3]);
  const int n_lo = atoi(argv[4]), n_hi = atoi(argv[5]), pattern = atoi(argv[6]);
  if (NB < 1 || NB > 16 || n_lo < 1 || n_hi > 256 || n_lo > n_hi) return 2;
  FILE* f = fopen(argv[1], "wb");
  if (!f) return 2;
  for (int n = n_lo; n <= n_hi; ++n) {
    const int ld = (n + 15) & ~15;
    double* M = (double*)malloc(sizeof(double) * (size_t)n * ld);
    double* A = (double*)malloc(sizeof(double) * (size_t)n * n);
    lds_t W;
    W.panel = (double*)malloc(sizeof(double) * (size_t)NB * ld);
    W.U12 = U_HBM ? NULL : (double*)malloc(sizeof(double) * (size_t)NB * ld);
    W.piv = (int*)malloc(sizeof(int) * ld);
    W.perm = (int*)malloc(sizeof(int) * ld);
    W.sig = (int*)malloc(sizeof(int) * ld);
    W.ired = (int*)malloc(sizeof(int) * 16);
    double* b = (double*)malloc(sizeof(double) * n);
    double* x = (double*)malloc(sizeof(double) * n);
    if (pattern == 1) {
      /* A = P L U with |l| <= 1/2 below the unit diagonal: partial pivoting
       * picks the row holding L's row k, which P places at the current last
       * row at every step (the swaps k <-> n-1 undone from the end) */
      double* L = (double*)malloc(sizeof(double) * (size_t)n * n);
      double* U = (double*)malloc(sizeof(double) * (size_t)n * n);
      int* arr = (int*)malloc(sizeof(int) * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          L[i * n + j] = i == j ? 1.0 : (i > j ? 0.5 * urand() : 0.0);
          U[i * n + j] = i == j ? (2.0 + fabs(urand())) : (i < j ? urand() : 0.0);
        }
      for (int i = 0; i < n; ++i) arr[i] = i;
      for (int k = n - 2; k >= 0; --k) {
        const int tmp = arr[k];
        arr[k] = arr[n - 1];
        arr[n - 1] = tmp;
      }
      for (int p = 0; p < n; ++p)
        for (int j = 0; j < n; ++j) {
          double v = 0.0;
          for (int q = 0; q < n; ++q) v += L[arr[p] * n + q] * U[q * n + j];
          A[p * n + j] = v;
        }
      free(L); free(U); free(arr);
    } else {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double v = urand();
          if (pattern == 2) v = (i == j) ? 4.0 * n : v;
          if (pattern == 3 && j == n - 1) v = 0.0;
          A[i * n + j] = v;
        }
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) M[j * ld + i] = A[i * n + j];
    const int info = lu_w(M, n, ld, &W);
    for (int i = 0; i < n; ++i) b[i] = i + 1.0;
    if (info == 0) solve_w(M, n, ld, &W, b, x);
    else for (int i = 0; i < n; ++i) x[i] = 0.0;
    int hdr[3] = {n, ld, info};
    fwrite(hdr, sizeof(int), 3, f);
    fwrite(A, sizeof(double), (size_t)n * n, f);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) fwrite(&M[j * ld + i], sizeof(double), 1, f);
    fwrite(W.piv, sizeof(int), n, f);
    fwrite(x, sizeof(double), n, f);
    free(M); free(A); free(W.panel); free(W.U12); free(W.piv); free(W.perm); free(W.sig); free(W.ired);
    free(b); free(x);
  }
  fclose(f);
  return 0;
}

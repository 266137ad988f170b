/* Host replica of the index arithmetic of the workgroup kernel's blocked LU
 * and triangular solves (lu_w, factor_panel and solve_w of the
 * large-mechanism integrator), for bounds checking under AddressSanitizer.
 * TEST INFRASTRUCTURE ONLY.
 *
 * Every buffer the kernel touches is allocated on its own, at exactly the
 * size the kernel's layout gives it: in LDS the two 12-column buffers
 * (kLS ld doubles each, one block of multipliers as rows of 12 at a stride
 * of 14, or the panel likewise), the waves' U-block tables (4 x 36 doubles), piv, perm and
 * pos (ld ints each), the reduction scratch (16 ints), the zero-pivot masks
 * (32 ints) and the solve vectors (ld doubles each); in HBM the matrix slot (n
 * columns of ld doubles). An access outside any of them stops the program
 * with an ASan report.
 *
 * The kernel's registers are arrays per thread. The 256 threads run one after
 * the other inside each phase between two barriers; a wave's lanes run in
 * lock step where they exchange values (DPP broadcasts read before any lane
 * writes, reductions replaced by the value they compute: largest key, then
 * the smallest (position, row) code among the lanes holding it). The
 * loops, bounds and guards follow the kernel's source, so that the factors
 * come out equal to an unblocked LU in every bit (the test checks that too).
 *
 * Usage: wide_lu_bounds <out.bin> <n_lo> <n_hi> <pattern> [form]
 * form 1: the LU receives J (the generated matrix) in its own slot and forms
 * g I - J (g = 2.5) as it reads the columns, as the integrator does; the
 * written input is then g I - J, formed with the same expression.
 * pattern 0: random matrices; 1: every pivot is the last row; 2: no pivoting
 * (diagonally dominant); 3: column n-1 made zero (a singular last column);
 * 4: column n/2 made zero (a zero pivot inside the matrix, whose multipliers
 * must not be applied to later columns).
 * For each n it writes n, ld, info, the input (row-major), the factors in
 * logical row order (row-major), piv and the solution of A x = b for
 * b_i = i + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum { T = 256, NB = 12, LS = 14, RS = 4, CW = 3, PRE = 6, SB = 16 };

typedef struct {
  double *buf0, *buf1, *b, *x, *ub;
  int *piv, *perm, *pos, *ired, *zpm;
} lds_t;

/* registers of the 256 threads */
static double A[T][RS][CW];
static double R[T][PRE][2];
static int PS[T][RS];

static int imin(int a, int b) { return a < b ? a : b; }

/* pairs of rows above the block (position < kb, or padding) read the first pair */
static void block_load(int t, const double* src, int cnt2, int ld, int kb, const int* pos) {
  for (int i = 0; i < PRE; ++i) {
    int e = t + T * i;
    if (e > cnt2 - 1) e = cnt2 - 1;
    const int q = (2 * e) % ld;
    const int need = pos[q] >= kb || pos[q + 1] >= kb;
    R[t][i][0] = src[2 * (need ? e : 0)];
    R[t][i][1] = src[2 * (need ? e : 0) + 1];
  }
}

static void block_store_t(int t, double* dst, int ld, int cnt2) {
  for (int i = 0; i < PRE; ++i) {
    const int e = t + T * i;
    if (e < cnt2) {
      const int m = (2 * e) / ld, q = 2 * e - m * ld;
      dst[q * LS + m] = R[t][i][0];
      dst[(q + 1) * LS + m] = R[t][i][1];
    }
  }
}

/* form: the source is J and the matrix g I - J is formed as it is read */
static void load_cols(int t, const double* S, int form, double g, int n, int ld, int k0, int nb) {
  const int lane = t & 63, w = t >> 6;
  for (int s = 0; s < RS; ++s) {
    const int q = lane + 64 * s;
    for (int cc = 0; cc < CW; ++cc) {
      const int c = CW * w + cc;
      const double v = (q < n && c < nb) ? S[(k0 + c) * ld + q] : 0.0;
      A[t][s][cc] = form ? ((q == k0 + c ? g : 0.0) - v) : v;
    }
  }
}

/* one finished block (multipliers as rows of 12 in Lt) applied to wave w's
 * three panel columns */
static void apply_block(int w, const double* Lt, int kb, int zm, lds_t* W) {
  double* Tw = W->ub + 36 * w;
  for (int lane = 0; lane < 64; ++lane) {
    const int t = 64 * w + lane;
    for (int s = 0; s < RS; ++s) {
      const int m = PS[t][s] - kb;
      if (m >= 0 && m < NB)
        for (int cc = 0; cc < CW; ++cc) Tw[m * CW + cc] = A[t][s][cc];
    }
  }
  /* triangle: lane 16 cc + m holds row m, column cc */
  double x[64], lr[64][NB];
  for (int lane = 0; lane < 64; ++lane) {
    const int cc = lane >> 4, m = lane & 15;
    const int act = cc < CW && m < NB;
    x[lane] = act ? Tw[m * CW + cc] : 0.0;
    const int q = act ? W->perm[kb + m] : 0;
    for (int j = 0; j < NB; ++j) lr[lane][j] = Lt[q * LS + j];
  }
  for (int j = 0; j + 1 < NB; ++j) {
    if ((zm >> j) & 1) continue;
    double u[64];
    for (int lane = 0; lane < 64; ++lane) u[lane] = x[(lane & ~15) + j];
    for (int lane = 0; lane < 64; ++lane) {
      const double y = x[lane] - lr[lane][j] * u[lane];
      x[lane] = (lane & 15) > j ? y : x[lane];
    }
  }
  for (int lane = 0; lane < 64; ++lane) {
    const int cc = lane >> 4, m = lane & 15;
    if (cc < CW && m < NB) Tw[m * CW + cc] = x[lane];
  }
  double U[NB][CW];
  for (int j = 0; j < NB; ++j)
    for (int c = 0; c < CW; ++c) U[j][c] = Tw[j * CW + c];
  for (int lane = 0; lane < 64; ++lane) {
    const int t = 64 * w + lane;
    for (int s = 0; s < RS; ++s) {
      const int q = lane + 64 * s;
      const int rel = PS[t][s] - kb;
      if (rel >= NB) {
        double l[NB];
        for (int j = 0; j < NB; ++j) l[j] = Lt[q * LS + j];
        for (int j = 0; j < NB; ++j) {
          if ((zm >> j) & 1) continue;
          for (int c = 0; c < CW; ++c) A[t][s][c] = A[t][s][c] - l[j] * U[j][c];
        }
      } else if (rel >= 0) {
        for (int c = 0; c < CW; ++c) A[t][s][c] = Tw[rel * CW + c];
      }
    }
  }
}

/* all four waves: thread t holds physical row t of the panel; the waves'
 * candidates go through the U-block table area (2 x 4 x 14 doubles) */
static void factor_panel(double* M, const double* H, int n, int ld, int k0, int nb, lds_t* W) {
  static double P[T][NB];
  int pq[T];
  int info = W->ired[15];
  double* cand = W->ub;
  for (int t = 0; t < T; ++t) {
    pq[t] = t < n ? W->pos[t] : -1;
    for (int j = 0; j < NB; ++j) P[t][j] = t < n ? H[t * LS + j] : 0.0;
  }
  for (int c = 0; c < nb; ++c) {
    const int k = k0 + c;
    double key[T];
    int code[T];
    for (int t = 0; t < T; ++t) {
      const double av = fabs(P[t][c]);
      key[t] = pq[t] < k ? -1.0 : (av != av ? (pq[t] == k ? INFINITY : -1.0) : av);
      code[t] = pq[t] * 256 + t;
    }
    for (int w = 0; w < 4; ++w) {
      double wkey = key[64 * w];
      for (int l = 1; l < 64; ++l)
        if (key[64 * w + l] > wkey) wkey = key[64 * w + l];
      int wcode = 0x7fffffff;
      for (int l = 0; l < 64; ++l)
        if (key[64 * w + l] == wkey && code[64 * w + l] < wcode) wcode = code[64 * w + l];
      double* slot = cand + ((c & 1) * 4 + w) * (2 + NB);
      for (int l = 0; l < 64; ++l) {
        const int t = 64 * w + l;
        if (code[t] == wcode) {
          slot[0] = wkey;
          slot[1] = (double)wcode;   /* the kernel keeps the int's bits; the value is what matters here */
          for (int j = c; j < NB; ++j) slot[2 + j] = P[t][j];
        }
      }
    }
    const double* set = cand + (c & 1) * 4 * (2 + NB);
    double bk = set[0];
    int bc = (int)set[1], bw = 0;
    for (int v = 1; v < 4; ++v) {
      const double kv = set[v * (2 + NB)];
      const int cv = (int)set[v * (2 + NB) + 1];
      if (kv > bk || (kv == bk && cv < bc)) {
        bk = kv;
        bc = cv;
        bw = v;
      }
    }
    const int pv = bc >> 8, qs = bc & 255;
    W->piv[k] = pv;
    for (int t = 0; t < T; ++t) {
      if (t == qs) pq[t] = k;
      else if (pq[t] == k) pq[t] = pv;
    }
    const double* pr = set + bw * (2 + NB) + 2;
    const double akk = pr[c];
    if (akk == 0.0) {
      if (!info) info = k + 1;
      W->zpm[k0 / NB] |= 1 << c;
    } else {
      for (int t = 0; t < T; ++t)
        if (pq[t] > k) {
          const double l = P[t][c] / akk;
          P[t][c] = l;
          for (int j = c + 1; j < NB; ++j)
            if (j < nb) P[t][j] = P[t][j] - l * pr[j];
        }
    }
  }
  for (int t = 0; t < T; ++t) {
    if (t < n)
      for (int c = 0; c < NB; ++c)
        if (c < nb) M[(k0 + c) * ld + t] = P[t][c];
    if (t < ld) W->pos[t] = pq[t];
    if (pq[t] >= 0) W->perm[pq[t]] = t;
  }
  W->ired[15] = info;
}

static int lu_w(double* M, const double* J, double gm, int form, int n, int ld, lds_t* W) {
  const int np = (n + NB - 1) / NB;
  const int cnt2 = NB * ld / 2;
  for (int t = 0; t < T; ++t) {
    if (t < ld) {
      W->pos[t] = t < n ? t : -1;
      W->perm[t] = t;
    }
    if (t < 32) W->zpm[t] = 0;
    if (t == 0) W->ired[15] = 0;
    load_cols(t, form ? J : M, form, gm, n, ld, 0, imin(NB, n));
  }
  int g = 0;
  for (int p = 0; p < np; ++p) {
    const int k0 = p * NB, nb = imin(NB, n - k0);
    for (int t = 0; t < T; ++t)
      for (int s = 0; s < RS; ++s) {
        const int q = (t & 63) + 64 * s;
        PS[t][s] = q < ld ? W->pos[q] : -1;
      }
    if (p == 1) {
      for (int t = 0; t < T; ++t) block_load(t, M, cnt2, ld, 0, W->pos);
      for (int t = 0; t < T; ++t) block_store_t(t, W->buf0, ld, cnt2);
    }
    for (int b = 0; b < p; ++b) {
      const int kb = b * NB;
      const double* Lt = (g & 1) ? W->buf1 : W->buf0;
      const int more = b + 1 < p || p + 1 < np;
      if (more)
        for (int t = 0; t < T; ++t) block_load(t, M + (b + 1 < p ? kb + NB : 0) * ld, cnt2, ld, b + 1 < p ? kb + NB : 0, W->pos);
      const int zm = W->zpm[b];
      for (int w = 0; w < 4; ++w) apply_block(w, Lt, kb, zm, W);
      if (more)
        for (int t = 0; t < T; ++t) block_store_t(t, (g & 1) ? W->buf0 : W->buf1, ld, cnt2);
      ++g;
    }
    double* H = (g & 1) ? W->buf0 : W->buf1;
    for (int t = 0; t < T; ++t) {
      const int lane = t & 63, w = t >> 6;
      for (int s = 0; s < RS; ++s) {
        const int q = lane + 64 * s;
        for (int cc = 0; cc < CW; ++cc)
          if (q < n) H[q * LS + CW * w + cc] = A[t][s][cc];
      }
    }
    if (p + 1 < np)
      for (int t = 0; t < T; ++t) load_cols(t, form ? J : M, form, gm, n, ld, k0 + NB, imin(NB, n - k0 - NB));
    factor_panel(M, H, n, ld, k0, nb, W);
  }
  return W->ired[15];
}

/* one block of the substitution: the entries in the block's columns of every
 * row that takes part (loaded ahead; columns past n - 1 read column n - 1,
 * other rows read row 0), the block rows' entries through LDS (the second
 * 12-column buffer) to wave 0, the triangle, then every row */
static void solve_block(int fwd, int k0, int n, int ld, const double* M, lds_t* W, const int* pt) {
  double* b = W->b;
  double* xb = W->ub;
  double* Tb = W->buf1;
  const int nb = imin(SB, n - k0);
  static double v[T][SB];
  for (int t = 0; t < T; ++t) {
    const int need = fwd ? pt[t] >= k0 : (pt[t] >= 0 && pt[t] < k0 + SB);
    const int r = need ? t : 0;
    for (int j = 0; j < SB; ++j) v[t][j] = M[imin(k0 + j, n - 1) * ld + r];
  }
  for (int t = 0; t < T; ++t) {
    const int rel = pt[t] - k0;
    if (rel >= 0 && rel < nb)
      for (int j = 0; j < SB; ++j) Tb[rel * SB + j] = v[t][j];
  }
  double lc[64][SB], xv[64], rdg[64];
  int r[64];
  for (int t = 0; t < 64; ++t) {
    r[t] = t < nb ? W->perm[k0 + t] : 0;
    for (int j = 0; j < SB; ++j) lc[t][j] = Tb[(t < nb ? t : 0) * SB + j];
    xv[t] = t < nb ? b[r[t]] : 0.0;
    rdg[t] = fwd ? 0.0 : 1.0 / (t < nb ? Tb[t * SB + t] : 1.0);
  }
  /* each step: the value of lane j of every 16-lane row (a DPP broadcast,
   * read by all lanes before any writes), times a multiplier that is zero
   * outside the rows it updates */
  double z[64];
  if (fwd) {
    for (int j = 0; j + 1 < SB; ++j)
      if (j + 1 < nb) {
        for (int t = 0; t < 64; ++t) z[t] = xv[16 * (t / 16) + j];
        for (int t = 0; t < 64; ++t) {
          const double lm = (t > j && t < nb) ? lc[t][j] : 0.0;
          xv[t] = xv[t] - lm * z[t];
        }
      }
  } else {
    for (int j = SB - 1; j >= 0; --j)
      if (j < nb) {
        for (int t = 0; t < 64; ++t) z[t] = xv[16 * (t / 16) + j] * rdg[16 * (t / 16) + j];
        for (int t = 0; t < 64; ++t) {
          const double lm = t < j ? lc[t][j] : 0.0;
          xv[t] = xv[t] - lm * z[t];
        }
      }
    for (int t = 0; t < 64; ++t) xv[t] = xv[t] * rdg[t];
  }
  for (int t = 0; t < 64; ++t)
    if (t < nb) {
      b[r[t]] = xv[t];
      xb[t] = xv[t];
    }
  for (int t = 0; t < T; ++t)
    if (fwd ? pt[t] >= k0 + nb : (pt[t] >= 0 && pt[t] < k0)) {
      double a = b[t];
      for (int j = 0; j < SB; ++j)
        if (j < nb) a = a - v[t][j] * xb[j];
      b[t] = a;
    }
}

static void solve_w(const double* M, int n, int ld, lds_t* W) {
  int pt[T];
  for (int t = 0; t < T; ++t) pt[t] = t < n ? W->pos[t] : -1;
  const int nblk = (n + SB - 1) / SB;
  for (int i = 0; i < nblk; ++i) solve_block(1, SB * i, n, ld, M, W, pt);
  for (int i = nblk - 1; i >= 0; --i) solve_block(0, SB * i, n, ld, M, W, pt);
  for (int t = 0; t < T; ++t)
    if (t < n) W->x[t] = W->b[W->perm[t]];
}

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double urand(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

int main(int argc, char** argv) {
  if (argc != 5 && argc != 6) {
    fprintf(stderr, "usage: %s out.bin n_lo n_hi pattern [form]\n", argv[0]);
    return 2;
  }
  const int n_lo = atoi(argv[2]), n_hi = atoi(argv[3]), pattern = atoi(argv[4]);
  const int form = argc == 6 ? atoi(argv[5]) : 0;
  const double g = 2.5;
  if (n_lo < 13 || n_hi > 256 || n_lo > n_hi || pattern < 0 || pattern > 4) return 2;
  FILE* f = fopen(argv[1], "wb");
  if (!f) return 2;
  for (int n = n_lo; n <= n_hi; ++n) {
    const int ld = (n + 15) & ~15;
    double* M = (double*)malloc(sizeof(double) * (size_t)n * ld);
    double* Ain = (double*)malloc(sizeof(double) * (size_t)n * n);
    lds_t W;
    W.buf0 = (double*)malloc(sizeof(double) * (size_t)LS * ld);
    W.buf1 = (double*)malloc(sizeof(double) * (size_t)LS * ld);
    W.b = (double*)malloc(sizeof(double) * ld);
    W.x = (double*)malloc(sizeof(double) * ld);
    W.piv = (int*)malloc(sizeof(int) * ld);
    W.perm = (int*)malloc(sizeof(int) * ld);
    W.pos = (int*)malloc(sizeof(int) * ld);
    W.ired = (int*)malloc(sizeof(int) * 16);
    W.zpm = (int*)malloc(sizeof(int) * 32);
    W.ub = (double*)malloc(sizeof(double) * 144);
    /* uninitialised LDS and padding rows hold NaN: they must never be used */
    for (int i = 0; i < LS * ld; ++i) W.buf0[i] = W.buf1[i] = NAN;
    for (int i = 0; i < 144; ++i) W.ub[i] = NAN;
    for (size_t i = 0; i < (size_t)n * ld; ++i) M[i] = NAN;
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
          Ain[p * n + j] = v;
        }
      free(L); free(U); free(arr);
    } else {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double v = urand();
          if (pattern == 2) v = (i == j) ? 4.0 * n : v;
          if (pattern == 3 && j == n - 1) v = 0.0;
          if (pattern == 4 && j == n / 2) v = 0.0;
          Ain[i * n + j] = v;
        }
    }
    double* J = (double*)malloc(sizeof(double) * (size_t)n * ld);
    for (size_t i = 0; i < (size_t)n * ld; ++i) J[i] = NAN;
    if (form) {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          J[j * ld + i] = Ain[i * n + j];
          Ain[i * n + j] = (i == j ? g : 0.0) - J[j * ld + i];
        }
    } else {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[j * ld + i] = Ain[i * n + j];
    }
    const int info = lu_w(M, J, g, form, n, ld, &W);
    for (int i = 0; i < ld; ++i) W.b[i] = i < n ? i + 1.0 : NAN;
    if (info == 0) solve_w(M, n, ld, &W);
    else for (int i = 0; i < n; ++i) W.x[i] = 0.0;
    int hdr[3] = {n, ld, info};
    fwrite(hdr, sizeof(int), 3, f);
    fwrite(Ain, sizeof(double), (size_t)n * n, f);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) fwrite(&M[j * ld + W.perm[i]], sizeof(double), 1, f);
    fwrite(W.piv, sizeof(int), n, f);
    fwrite(W.x, sizeof(double), n, f);
    free(M); free(J); free(Ain); free(W.buf0); free(W.buf1); free(W.b); free(W.x);
    free(W.piv); free(W.perm); free(W.pos); free(W.ired); free(W.zpm); free(W.ub);
  }
  fclose(f);
  return 0;
}

/* UoI_LASSO / UoI_VAR CPU oracle -- TEST INFRASTRUCTURE ONLY (see uoi_oracle.c). */
#ifndef UOI_ORACLE_H
#define UOI_ORACLE_H
#include <stdint.h>

#define ORC_TAG_LASSO_BOOT 1u
#define ORC_TAG_LASSO_SPLIT 2u
#define ORC_TAG_VAR_BOOT 3u
#define ORC_TAG_VAR_SPLIT 4u

uint64_t orc_mix64(uint64_t x);
uint64_t orc_key(uint64_t seed, uint32_t tag, uint32_t k, uint32_t i);
uint32_t orc_index(uint64_t r, uint32_t m);
void orc_boot_rows(uint64_t seed, int k, int n, int32_t *rows);
int orc_split_count(int n, int num, int den);
void orc_split_rows(uint64_t seed, int k, int n, int num, int den, int32_t *train, int32_t *eval);
int orc_var_block_len(int N);
int orc_var_nblocks(int N, int L);
void orc_var_boot_rows(uint64_t seed, int k, int N, int L, int32_t *rows);
void orc_var_split_rows(uint64_t seed, int k, int N, int L, int num, int den,
                        int32_t *train, int *ntr, int32_t *eval, int *nev);
void orc_gram(int m, const int32_t *rows, int p, const double *X, int ldx,
              int pe, const double *Y, int ldy, double *G, double *C);
double orc_kkt(int p, const double *G, const double *c, int ldc, double lam, const double *b);
int orc_lasso_cd(int p, const double *G, const double *c, int ldc, double lam, double tol,
                 int max_sweeps, double *b);
int orc_lstsq_qr(int m, int s, double *A, double *yv, double *b);
int orc_ols_normal(int p, const double *G, const double *c, int ldc, int s, const int *idx,
                   double *b, double *work);
int orc_uoi_lasso(int n, int p, const double *X, const double *y,
                  int B1, int B2, int q, const double *lam, uint64_t seed,
                  int num, int den, double tol, int max_sweeps,
                  double *beta_star, uint64_t *supp, int32_t *jstar, double *losses,
                  double *sel_beta, double *sel_kkt, double *ols_beta);
int orc_uoi_var(int T, int p, const double *series, int L, int B1, int B2, int q,
                const double *lam, uint64_t seed, int num, int den, double tol, int max_sweeps,
                double *A_out, uint64_t *supp, int32_t *jstar, double *losses);
int orc_uoi_var_d(int T, int p, int d, int intercept, int per_eq, const double *series, int L,
                  int B1, int B2, int q, const double *lam, uint64_t seed, int num, int den,
                  double tol, int max_sweeps, double *A_out, double *mu_out, uint64_t *supp,
                  int32_t *jstar, double *losses);
#endif

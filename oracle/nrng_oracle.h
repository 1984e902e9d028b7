/*
 * nrng_oracle.h -- declarations of the FP64 CPU reference (test
 * infrastructure only; see nrng_oracle.c).  Independent of the product
 * library's header and kernels.
 */
#ifndef NRNG_ORACLE_H
#define NRNG_ORACLE_H

#include <stdint.h>

uint64_t orc_splitmix64(uint64_t x);
double orc_uniform(uint64_t seed, uint64_t ctr);
int32_t orc_int32(uint64_t seed, uint64_t ctr);
void orc_hash_block(uint64_t seed, uint64_t offset, uint64_t count, uint64_t *out);
void orc_uniform_block(uint64_t seed, uint64_t offset, uint64_t count, double *out);
void orc_int32_block(uint64_t seed, uint64_t offset, uint64_t count, int32_t *out);

void orc_b1_uv(const double *u, const double *v, uint64_t npairs, double mu, double sigma,
               double *out);
void orc_b1_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out);
uint64_t orc_b1(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out);

int orc_polar_accept(int32_t X, int32_t Y);
uint64_t orc_polar_xy(const int32_t *xy, uint64_t ncand, double mu, double sigma, double *out,
                      uint64_t *mask_words);
uint64_t orc_polar(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma,
                   double *out);
uint64_t orc_polar_count(uint64_t seed, uint64_t offset, uint64_t ncand);
uint64_t orc_polar_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *mask_words,
                         uint64_t *word_prefix);
uint64_t orc_polar_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu,
                          double sigma, double *out);

void orc_p2_cheb(int degree, double *c);
double orc_p2_h(int degree, double v);
int orc_polar2_accept(int32_t X, int32_t Y);
uint64_t orc_polar2_xy(const int32_t *xy, uint64_t ncand, double mu, double sigma, double *out,
                       uint64_t *mask_words);
uint64_t orc_polar2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma,
                    double *out);
uint64_t orc_polar2_count(uint64_t seed, uint64_t offset, uint64_t ncand);
uint64_t orc_polar2_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu,
                           double sigma, double *out);

void orc_b2_coef(double *s, double *c);
void orc_b2_sincos(double v, double *sn, double *cs);
void orc_b2_uv(const double *u, const double *v, uint64_t npairs, double mu, double sigma, double *out);
void orc_b2_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out);
uint64_t orc_b2(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out);

void orc_b3_u(const double *u1, const double *u2, const double *u3, uint64_t npairs, double mu, double sigma,
              double *out);
void orc_b3_words(const uint64_t *w, uint64_t npairs, double mu, double sigma, double *out);
uint64_t orc_b3(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out);

int orc_ratio_accept(double u, double v);
uint64_t orc_ratio_words(const uint64_t *w, uint64_t ncand, double mu, double sigma, double *out,
                         uint64_t *mask_words);
uint64_t orc_ratio(uint64_t seed, uint64_t offset, uint64_t n, double mu, double sigma, double *out);
uint64_t orc_ratio_count(uint64_t seed, uint64_t offset, uint64_t ncand);
uint64_t orc_ratio_trace(uint64_t seed, uint64_t offset, uint64_t ncand, uint64_t *mask_words,
                         uint64_t *word_prefix);
uint64_t orc_ratio_window(uint64_t seed, uint64_t offset, uint64_t j0, uint64_t ncand, double mu, double sigma,
                          double *out);

void orc_moments(const double *x, uint64_t n, double *out);
double orc_normal_cdf(double z);
double orc_ks(double *x, uint64_t n, int kind, double mu, double sigma);

#endif

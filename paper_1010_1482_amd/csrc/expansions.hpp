// Launch wrappers shared between the translation units of the library.
#pragma once
#include "common.hpp"

namespace hfmm {

void fill_masses(Tree& t, const double* m, hipStream_t s);
void compute_centres(Tree& t, int method, hipStream_t s);
void run_p2m(Tree& t, int p, bool fp64, hipStream_t s);
void run_m2m(Tree& t, int p, bool per_child, hipStream_t s);
void run_m2l_ops(Tree& t, int p, bool fp64, double* T64, float* T32, int RB, int KQ,
                 hipStream_t s);
void run_pack(const double* M, int ncells, int P, int ld, void* out, bool fp64,
              hipStream_t s);
void run_p2l(Tree& t, int p, double* LX, hipStream_t s);
void run_downward(Tree& t, int p, const void* lm2l, bool m2l_fp64, int ldm, int nparts,
                  int64_t part_stride, const double* LX, hipStream_t s);
void run_far(Tree& t, int p, bool fp64, void* far, hipStream_t s);
void run_treecode_far(Tree& t, int p, bool fp64, void* far, hipStream_t s);
void run_export(const double* X, int ncells, int p, const double* cen, int which,
                double* out, hipStream_t s);

bool m2l_uses_mfma(int p, int precision);
void m2l_layout(int p, int precision, int& RB, int& KQ, int& ld);
size_t m2l_ops_bytes(int p, int precision);
void prepare_m2l_ops(Tree& t, int p, int precision, hipStream_t s);
int run_m2l(Tree& t, int p, int precision, void* out, int64_t& part_stride, int max_parts,
            hipStream_t s);

}  // namespace hfmm

// Launch wrappers shared between the translation units of the library.
#pragma once
#include "common.hpp"

namespace hfmm {

void fill_masses(Tree& t, const double* m, hipStream_t s);
void compute_centres(Tree& t, int method, hipStream_t s);
void run_p2m(Tree& t, int p, bool fp64, hipStream_t s);
void run_m2m(Tree& t, int p, hipStream_t s);
void run_shift_octants(int p, double2* tab, hipStream_t s);
void prepare_xlat_ops(Tree& t, int p, hipStream_t s);
void run_m2m_mfma(Tree& t, int p, hipStream_t s);
void run_l2l_mfma(Tree& t, int p, const void* parts, bool parts_fp64, int nparts,
                  int64_t part_stride, const double* LX, const int32_t* bexp,
                  const int32_t* levexp, hipStream_t s);
void run_m2l_ops(Tree& t, int p, int layout, void* T, int RB, int KQ, hipStream_t s);
void run_m2l_ops_lp(int p, int precision, int RB, int KQ, int32_t* bexp, void* hi, void* lo,
                    hipStream_t s);
void run_pack(const double* M, int ldm, int ncells, int P, int ld, void* out, bool fp64,
              hipStream_t s);
void run_p2l(Tree& t, int p, bool fp64, double* LX, hipStream_t s);
void run_far(Tree& t, const Targets& tg, int p, bool fp64, const int32_t* off,
             const int32_t* items, int64_t nitems, void* far, hipStream_t s);
void run_treecode_far(Tree& t, const Targets& tg, int p, bool fp64, bool walk,
                      const int32_t* off, const int32_t* items, void* far, hipStream_t s);
void run_export(const double* X, int ld, int ncells, int p, const double* cen, int which,
                double* out, hipStream_t s);

bool m2l_uses_mfma(int p, int precision);
// rotation-based M2L (rotation.hip)
size_t rot_ops_bytes(int p, int precision);
void run_rot_ops(int p, int precision, void* tab, hipStream_t s);
int run_m2l_rot(Tree& t, int p, int precision, void* out, int64_t& part_stride, hipStream_t s);
void m2l_layout(int p, int precision, int& RB, int& KQ, int& ld);
size_t m2l_ops_bytes(int p, int precision);
void prepare_m2l_ops(Tree& t, int p, int precision, hipStream_t s);
void prepare_rot_ops(Tree& t, int p, int precision, hipStream_t s);
int run_m2l(Tree& t, int p, int precision, void* out, int64_t& part_stride, int max_parts,
            int32_t* levexp, hipStream_t s);
int m2l_plan(const Tree& t, int p, int precision, int max_parts, int& nb);

}  // namespace hfmm

// tables.h -- host-side 1D table construction (float64).
#pragma once

namespace dpg {

void gauss_legendre_01(int N, double* zeta, double* w);
void chi_tables(int L, const double* zeta, int kmax, double* chi, double* dchi);
double ftable_entry(int r, int s, int i, int j);
// tab64/tab32: TABLE_LEN entries; f64/f32: FTAB_LEN entries.
void build_tables(double* tab64, float* tab32, double* f64, float* f32);

}  // namespace dpg

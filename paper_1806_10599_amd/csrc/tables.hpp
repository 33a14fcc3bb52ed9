#pragma once

#include <cstdint>
#include <vector>

#include "kernels.hpp"

namespace rve {

std::vector<double> twiddles(int n);
std::vector<double> wave_vectors(int n, const double L[3], int projection);
std::vector<double> label_table(int G, const double* quat, const int32_t* law,
                                const double* params);

}  // namespace rve

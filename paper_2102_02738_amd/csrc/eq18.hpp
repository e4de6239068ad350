// Four-Gaussian approximation of the rectangle function, Eq. (18) of SIMUS
// Part I (Garcia): Pi(y/h) ~ sum_g A_g exp(-B_g (y/h)^2); coefficients 3 and
// 4 are the complex conjugates of 1 and 2.
#pragma once

namespace simus {
namespace eq18 {
constexpr double Ar[4] = {0.187, 0.288, 0.187, 0.288};
constexpr double Ai[4] = {0.275, -1.954, -0.275, 1.954};
constexpr double Br[4] = {4.558, 8.598, 4.558, 8.598};
constexpr double Bi[4] = {-25.59, -7.924, 25.59, 7.924};
}  // namespace eq18
}  // namespace simus

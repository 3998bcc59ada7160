// Instantiation unit: compiled once per (family shape, dtype) with
//   -DHJPD_FAM=<family type> -DHJPD_REAL=<float|double> -DHJPD_NAME=<lookup suffix>
#include "hjpd_launch.hpp"

#define HJPD_CAT2(a, b) a##b
#define HJPD_CAT(a, b) HJPD_CAT2(a, b)

const void* HJPD_CAT(hjpd_lookup_, HJPD_NAME)(int plain, int L, int K, int variant) {
  return hjpd::pick_kernel<HJPD_REAL, hjpd::HJPD_FAM>(plain, L, K, variant);
}

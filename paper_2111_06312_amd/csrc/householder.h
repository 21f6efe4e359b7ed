// Householder QR of a tall block (Algorithm 2, the QR orthonormaliser).
#pragma once

#include "common.h"

namespace isvd {

// Doubles of workspace for launch_householder_qr with l columns.
size_t householder_workspace_doubles(int l);

// Y (rows x l, ld) is overwritten by the reflectors; Q (rows x l, ldq, a
// separate block) receives the orthonormal factor; R (optional, lp x lp
// FP64, lp >= l) the upper factor with Y = Q R (padding: identity diagonal).
// rows >= l, l <= 1024.
template <typename T>
void launch_householder_qr(int64_t rows, int l, T* Y, int64_t ld, T* Q, int64_t ldq, double* R, int lp,
                           double* work, hipStream_t stream);

}  // namespace isvd

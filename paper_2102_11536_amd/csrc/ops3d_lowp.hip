// Low-precision 3-D operator launches: FP32 vectors and arithmetic with the
// quadrature factors stored in FP32 or in BF16 (widened to FP32 as they are read).
// Used by the inner solves of the mixed-precision path and by the FP32/BF16
// operator applies of the C ABI.
#include "ops3d_body.h"

namespace ga {

namespace {

template <typename F>
int lowp_p(int p, int mode, int nr, const ga_patch* pt, const float* x, float* y, float alpha,
           const F* fac, hipStream_t st, const double* gate) {
  switch (p) {
    case 1: return launch_op3d_p<1, float, F>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 2: return launch_op3d_p<2, float, F>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 3: return launch_op3d_p<3, float, F>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 4: return launch_op3d_p<4, float, F>(mode, nr, pt, x, y, alpha, fac, st, gate);
  }
  return -1;
}

}  // namespace

int launch_op3d_lowp(int mode, int nr, const ga_patch* pt, const float* x, float* y, float alpha,
                     int prec, hipStream_t st, const double* gate) {
  if (mode != 0 && mode != 1) return -1;
  if (prec == GA_FP32) {
    const float* fac = mode == 1 ? pt->G32 : pt->W32;
    if (!fac) return -1;
    return lowp_p<float>(pt->p, mode, nr, pt, x, y, alpha, fac, st, gate);
  }
  if (prec == GA_BF16) {
    const unsigned short* fac = mode == 1 ? pt->G16 : pt->W16;
    if (!fac) return -1;
    return lowp_p<unsigned short>(pt->p, mode, nr, pt, x, y, alpha, fac, st, gate);
  }
  return -1;
}

// FP32 mass apply with the FP32 factors W32 (inner solves of the mixed path)
int launch_mass3d_f32(int nr, const ga_patch* pt, const float* x, float* y, float alpha,
                      hipStream_t st) {
  return launch_op3d_lowp(0, nr, pt, x, y, alpha, GA_FP32, st, nullptr);
}

}  // namespace ga

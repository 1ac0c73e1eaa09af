// Internal entry of the U-Net runtime used by die_te_warm_start (die_te.cpp), which owns
// the solver context's contrast.
#pragma once
#include <hip/hip_runtime.h>

struct die_te_unet;

namespace die_host {
// x0 = e_in + network(chi, e_in) for nrhs fields of ny x nx cells; right-hand side r uses
// chi of object r / rpo (chi: complex128 [nobj][ny][nx], already the contrast).
int unet_guess(die_te_unet* net, const double2* chi, int rpo, const double2* e_in, double2* x0, int nrhs, int ny,
               int nx, hipStream_t st);
}  // namespace die_host

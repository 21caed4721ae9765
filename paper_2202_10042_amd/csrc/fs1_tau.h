// fs1_tau.h -- the threshold form of the stabilisation (Sec. 2 and Sec. 3
// remarks) on the multi-workgroup path: grids of any size.
//
// The scalings are phi = e^{alpha/eps} phit and psi = e^{beta/eps} psit, with
// binary64 potentials alpha, beta and scaled vectors in the working precision.
// At the top of every iteration, when the largest scaled entry of phit or psit
// exceeds tau, both vectors are absorbed (alpha += eps ln phit, phit = 1; the
// same for psi; zero entries stay zero).  Every half-iteration packs
// e^{pot/eps} v into per-run shared exponents (the log domain's layout), so the
// chunk aggregates, carries and in-chunk recursions are the log domain's; the
// update returns to the scaled form with the potential of the half's output.
// An absorption leaves every packed vector unchanged, so it touches no
// aggregate.
#pragma once

#include "fs1_internal.h"

namespace fs1 {

struct TauBufs {
  double* potF;  // alpha (npad; zero past n)
  double* potG;  // beta
  double* pmF;   // per chunk: largest entry of phit (written by the phi-halves)
  double* pmG;   // per chunk: largest entry of psit (written by the psi-halves)
  int* absorb;   // 1 while the current iteration absorbs (set before its psi-half)
  double tau;
  double eps;
};

// Device bytes of TauBufs for a grid of npad entries in nchunks chunks.
size_t tau_bytes(int64_t npad, int64_t nchunks);

// After launch_init_state: the initial state (log layout in vF/eF, vG[0]/eG[0])
// to the scaled form with zero potentials, and its per-chunk maxima.
hipError_t launch_tau_init(const SolveBufs& b, const TauBufs& t, hipStream_t s);

// One half-iteration l (psi-half with the absorption test first, or phi-half
// with the close of the stopping test), including its carry launches.
hipError_t launch_tau_half(const SolveBufs& b, const TauBufs& t, const ScanConsts& k,
                           const CarryConsts& kc, int l, int check, double tol, bool psi,
                           hipStream_t s);

// The final state (phit, alpha) and (psit in vG[gbuf], beta) back to the log
// layout, in place, for the common finalisation.
hipError_t launch_tau_finish(const SolveBufs& b, const TauBufs& t, int gbuf, hipStream_t s);

}  // namespace fs1

// fs1_tune.h -- per-instance configuration of the batched solve and the
// request server: the run length of an instance's shared chunk launches and
// whether it runs resident (one workgroup of nt threads for all its
// iterations).  The choice is a pure function of (dtype, n, h/eps), so an
// instance's arithmetic does not depend on what runs beside it.
//
// Where the measured table (fs1_tune_table.h, written by the project's tuner
// paper_2202_10042_amd/tune.py from timings of forced configurations through
// fs1_solve_batched_config) has a row for the instance's class, the row
// decides; the run length never exceeds what h/eps allows
// (pick_run_length).  Without a row the built-in rules decide.
#pragma once

#include <cstdint>

namespace fs1 {

struct BatchCfg {
  int R;   // run length (entries per thread)
  int nt;  // resident workgroup size (256 or 1024), 0: shared chunk launches
};

// Run lengths the batched kernels are built for.
bool batch_shared_r_ok(int dtype, int R);
bool batch_resident_ok(int dtype, int R, int nt);

// The batched solve's configuration of an instance of n entries and c = h/eps.
BatchCfg batch_config(int dtype, int64_t n, double c);
// The server runs every request in the shared launches, with the run length
// the batched solve gives the instance.  A resident instance of one chunk
// (n <= 256 R, on 256 threads) does the same arithmetic as a one-chunk shared
// launch, so such a request's result equals the batched solve's bit for bit;
// the measured table keeps every resident class within one chunk.
int shared_run_length(int dtype, int64_t n, double c);

}  // namespace fs1

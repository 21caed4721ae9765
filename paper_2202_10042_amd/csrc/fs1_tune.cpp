// fs1_tune.cpp -- the configuration lookup of fs1_tune.h.
#include "fs1_tune.h"

#include "fs1_internal.h"
#include "fs1_tune_table.h"

namespace fs1 {

bool batch_shared_r_ok(int dtype, int R) {
  return dtype == 0 ? (R == 8 || R == 1) : (R == 16 || R == 8 || R == 4 || R == 1);
}

bool batch_resident_ok(int dtype, int R, int nt) {
  if (nt == 256) return dtype == 0 ? (R == 8 || R == 1) : (R == 16 || R == 8 || R == 4 || R == 1);
  if (nt == 1024) return dtype == 0 ? (R == 8 || R == 1) : (R == 8 || R == 4 || R == 1);
  return false;
}

namespace {

const TuneRow* tune_row(int dtype, int64_t n) {
  for (const TuneRow& r : kTuneRows)
    if (r.dtype == dtype && n <= r.n_max) return &r;
  return nullptr;
}

// The largest run length the batched kernels take that does not exceed rmax.
int clamp_r(int dtype, int R, int rmax) {
  if (R > rmax) R = rmax;
  while (R > 1 && !batch_shared_r_ok(dtype, R)) R /= 2;
  return R < 1 ? 1 : R;
}

}  // namespace

int shared_run_length(int dtype, int64_t n, double c) { return batch_config(dtype, n, c).R; }

BatchCfg batch_config(int dtype, int64_t n, double c) {
  const int rmax = pick_run_length(dtype, true, c);
  const TuneRow* row = tune_row(dtype, n);
  if (row) {
    if (row->nt > 0 && row->R_res <= rmax && batch_resident_ok(dtype, row->R_res, row->nt) &&
        n <= int64_t(row->nt) * row->R_res)
      return {row->R_res, row->nt};
    return {clamp_r(dtype, row->R_shared, rmax), 0};
  }
  // built-in rules: resident when the instance fits one workgroup, else the
  // longest run length h/eps allows
  const int rr = resident_run_length(n, rmax);
  if (rr > 0) return {rr, resident_threads(n, rr)};
  return {rmax, 0};
}

}  // namespace fs1

// fs1_tune_table.h -- measured per-class configurations of the batched solve
// (see fs1_tune.h), written by paper_2202_10042_amd/tune.py from timings of
// forced configurations on gfx950: per class, the fastest
// resident form (R_res, nt; nt = 0 when the shared launches are faster) and
// the fastest shared run length, each kept at the built-in rule's choice
// unless another candidate is at least 3% faster; then, per dtype, on an
// uneven batch (tune.py, stage 2), the shared run lengths per class or the
// rule's for every class, and the resident form cut off above the class
// edge that made the batch fastest, each kept unless 1.5% faster.
// Columns: dtype (0 binary64, 1 binary32), the
// class's largest n, R_shared, R_res, nt; the comment gives the row form's
// time per instance-iteration in stage 1.
#pragma once

namespace fs1 {

struct TuneRow {
  int dtype;        // 0 binary64, 1 binary32
  long long n_max;  // the row covers n <= n_max (rows ascend within a dtype)
  int R_shared;     // fastest run length in the shared launches
  int R_res;        // fastest resident configuration (R_res, nt), nt = 0: none faster
  int nt;
};

static const TuneRow kTuneRows[] = {
    {0, 181, 8, 8, 256},  // n ~ 152: 0.0238 us
    {0, 256, 8, 8, 256},  // n ~ 215: 0.0226 us
    {0, 362, 8, 8, 256},  // n ~ 304: 0.0233 us
    {0, 512, 8, 8, 256},  // n ~ 431: 0.0229 us
    {0, 724, 8, 8, 256},  // n ~ 609: 0.023 us
    {0, 1024, 8, 8, 256},  // n ~ 861: 0.0234 us
    {0, 1448, 8, 8, 256},  // n ~ 1218: 0.0256 us
    {0, 2048, 8, 8, 256},  // n ~ 1722: 0.0241 us
    {0, 2896, 8, 0, 0},  // n ~ 2435: 0.0804 us; resident cut off above n = 2048 (uneven batch)
    {0, 4096, 8, 0, 0},  // n ~ 3444: 0.0824 us; resident cut off above n = 2048 (uneven batch)
    {0, 5793, 8, 0, 0},  // n ~ 4871: 0.1156 us; resident cut off above n = 2048 (uneven batch)
    {0, 8192, 8, 0, 0},  // n ~ 6889: 0.1528 us; resident cut off above n = 2048 (uneven batch)
    {0, 11585, 8, 0, 0},  // n ~ 9742: 0.1928 us
    {0, 16384, 8, 0, 0},  // n ~ 13777: 0.2639 us
    {0, 23170, 8, 0, 0},  // n ~ 19484: 0.3739 us
    {0, 32768, 8, 0, 0},  // n ~ 27554: 0.5179 us
    {0, 46341, 8, 0, 0},  // n ~ 38968: 0.7321 us
    {0, 65536, 8, 0, 0},  // n ~ 55109: 0.9933 us
    {0, 92682, 8, 0, 0},  // n ~ 77936: 1.4333 us
    {0, 131072, 8, 0, 0},  // n ~ 110218: 2.0022 us
    {0, 185364, 8, 0, 0},  // n ~ 155872: 2.8527 us
    {0, 262144, 8, 0, 0},  // n ~ 220436: 4.0165 us
    {0, 370728, 8, 0, 0},  // n ~ 311744: 5.6865 us
    {0, 524288, 8, 0, 0},  // n ~ 440872: 8.1408 us
    {0, 741455, 8, 0, 0},  // n ~ 623487: 11.6317 us
    {0, 1048576, 8, 0, 0},  // n ~ 881744: 16.5177 us
    {1, 181, 16, 4, 256},  // n ~ 152: 0.0161 us
    {1, 256, 16, 4, 256},  // n ~ 215: 0.0161 us
    {1, 362, 16, 4, 256},  // n ~ 304: 0.0162 us
    {1, 512, 16, 4, 256},  // n ~ 431: 0.0164 us
    {1, 724, 16, 4, 256},  // n ~ 609: 0.0165 us
    {1, 1024, 16, 4, 256},  // n ~ 861: 0.0166 us
    {1, 1448, 16, 8, 256},  // n ~ 1218: 0.02 us
    {1, 2048, 16, 8, 256},  // n ~ 1722: 0.0214 us
    {1, 2896, 16, 16, 256},  // n ~ 2435: 0.0275 us
    {1, 4096, 16, 16, 256},  // n ~ 3444: 0.0278 us
    {1, 5793, 16, 0, 0},  // n ~ 4871: 0.0966 us; resident cut off above n = 4096 (uneven batch)
    {1, 8192, 16, 0, 0},  // n ~ 6889: 0.0975 us; resident cut off above n = 4096 (uneven batch)
    {1, 11585, 16, 0, 0},  // n ~ 9742: 0.1427 us
    {1, 16384, 16, 0, 0},  // n ~ 13777: 0.1869 us
    {1, 23170, 16, 0, 0},  // n ~ 19484: 0.2358 us
    {1, 32768, 16, 0, 0},  // n ~ 27554: 0.3219 us
    {1, 46341, 16, 0, 0},  // n ~ 38968: 0.4564 us
    {1, 65536, 16, 0, 0},  // n ~ 55109: 0.6353 us
    {1, 92682, 16, 0, 0},  // n ~ 77936: 0.8979 us
    {1, 131072, 16, 0, 0},  // n ~ 110218: 1.2245 us
    {1, 185364, 16, 0, 0},  // n ~ 155872: 1.758 us
    {1, 262144, 16, 0, 0},  // n ~ 220436: 2.4442 us
    {1, 370728, 16, 0, 0},  // n ~ 311744: 3.4659 us
    {1, 524288, 16, 0, 0},  // n ~ 440872: 4.9437 us
    {1, 741455, 16, 0, 0},  // n ~ 623487: 6.9909 us
    {1, 1048576, 16, 0, 0},  // n ~ 881744: 9.9824 us
};

}  // namespace fs1

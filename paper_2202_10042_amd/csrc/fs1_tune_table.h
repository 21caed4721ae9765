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
    {0, 181, 8, 8, 256},  // n ~ 152: 0.0226 us
    {0, 256, 8, 8, 256},  // n ~ 215: 0.0227 us
    {0, 362, 8, 8, 256},  // n ~ 304: 0.0234 us
    {0, 512, 8, 8, 256},  // n ~ 431: 0.023 us
    {0, 724, 8, 8, 256},  // n ~ 609: 0.0231 us
    {0, 1024, 8, 8, 256},  // n ~ 861: 0.0234 us
    {0, 1448, 8, 8, 256},  // n ~ 1218: 0.0254 us
    {0, 2048, 8, 0, 0},  // n ~ 1722: 0.0481 us; resident cut off above n = 1448 (uneven batch)
    {0, 2896, 8, 0, 0},  // n ~ 2435: 0.0845 us; resident cut off above n = 1448 (uneven batch)
    {0, 4096, 8, 0, 0},  // n ~ 3444: 0.0842 us; resident cut off above n = 1448 (uneven batch)
    {0, 5793, 8, 0, 0},  // n ~ 4871: 0.1171 us; resident cut off above n = 1448 (uneven batch)
    {0, 8192, 8, 0, 0},  // n ~ 6889: 0.156 us; resident cut off above n = 1448 (uneven batch)
    {0, 11585, 8, 0, 0},  // n ~ 9742: 0.196 us
    {0, 16384, 8, 0, 0},  // n ~ 13777: 0.2716 us
    {0, 23170, 8, 0, 0},  // n ~ 19484: 0.3815 us
    {0, 32768, 8, 0, 0},  // n ~ 27554: 0.523 us
    {0, 46341, 8, 0, 0},  // n ~ 38968: 0.7556 us
    {0, 65536, 8, 0, 0},  // n ~ 55109: 1.0181 us
    {0, 92682, 8, 0, 0},  // n ~ 77936: 1.4465 us
    {0, 131072, 8, 0, 0},  // n ~ 110218: 2.0368 us
    {0, 185364, 8, 0, 0},  // n ~ 155872: 2.8812 us
    {0, 262144, 8, 0, 0},  // n ~ 220436: 4.1223 us
    {0, 370728, 8, 0, 0},  // n ~ 311744: 5.7821 us
    {0, 524288, 8, 0, 0},  // n ~ 440872: 8.2879 us
    {0, 741455, 8, 0, 0},  // n ~ 623487: 11.8161 us
    {0, 1048576, 8, 0, 0},  // n ~ 881744: 16.7991 us
    {1, 181, 16, 4, 256},  // n ~ 152: 0.0161 us
    {1, 256, 16, 4, 256},  // n ~ 215: 0.0161 us
    {1, 362, 16, 4, 256},  // n ~ 304: 0.0161 us
    {1, 512, 16, 4, 256},  // n ~ 431: 0.0161 us
    {1, 724, 16, 4, 256},  // n ~ 609: 0.0163 us
    {1, 1024, 16, 4, 256},  // n ~ 861: 0.0183 us
    {1, 1448, 16, 8, 256},  // n ~ 1218: 0.0197 us
    {1, 2048, 16, 8, 256},  // n ~ 1722: 0.024 us
    {1, 2896, 16, 16, 256},  // n ~ 2435: 0.0277 us
    {1, 4096, 16, 16, 256},  // n ~ 3444: 0.0281 us
    {1, 5793, 16, 0, 0},  // n ~ 4871: 0.0957 us; resident cut off above n = 4096 (uneven batch)
    {1, 8192, 16, 0, 0},  // n ~ 6889: 0.0991 us; resident cut off above n = 4096 (uneven batch)
    {1, 11585, 16, 0, 0},  // n ~ 9742: 0.1432 us
    {1, 16384, 16, 0, 0},  // n ~ 13777: 0.1865 us
    {1, 23170, 16, 0, 0},  // n ~ 19484: 0.2322 us
    {1, 32768, 16, 0, 0},  // n ~ 27554: 0.3254 us
    {1, 46341, 16, 0, 0},  // n ~ 38968: 0.4652 us
    {1, 65536, 16, 0, 0},  // n ~ 55109: 0.6402 us
    {1, 92682, 16, 0, 0},  // n ~ 77936: 0.9026 us
    {1, 131072, 16, 0, 0},  // n ~ 110218: 1.2355 us
    {1, 185364, 16, 0, 0},  // n ~ 155872: 1.8042 us
    {1, 262144, 16, 0, 0},  // n ~ 220436: 2.4705 us
    {1, 370728, 16, 0, 0},  // n ~ 311744: 3.5223 us
    {1, 524288, 16, 0, 0},  // n ~ 440872: 5.0048 us
    {1, 741455, 16, 0, 0},  // n ~ 623487: 7.1415 us
    {1, 1048576, 16, 0, 0},  // n ~ 881744: 10.2856 us
};

}  // namespace fs1

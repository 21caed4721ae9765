// fs1_tune_table.h -- measured per-class configurations of the batched solve
// (see fs1_tune.h), written by paper_2202_10042_amd/tune.py from timings of
// forced configurations on gfx950: per class, the fastest
// resident form (R_res, nt; nt = 0 when the shared launches are faster) and
// the fastest shared run length, each kept at the built-in rule's choice
// unless another candidate is at least 3% faster.  Columns: dtype (0
// binary64, 1 binary32), the class's largest n, R_shared, R_res, nt; the
// comment gives the time per instance-iteration of the chosen form.
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
    {0, 181, 8, 8, 256},  // n ~ 152: 0.0216 us
    {0, 256, 8, 8, 256},  // n ~ 215: 0.0215 us
    {0, 362, 8, 8, 256},  // n ~ 304: 0.0225 us
    {0, 512, 8, 8, 256},  // n ~ 431: 0.022 us
    {0, 724, 8, 8, 256},  // n ~ 609: 0.0221 us
    {0, 1024, 8, 8, 256},  // n ~ 861: 0.0223 us
    {0, 1448, 8, 8, 256},  // n ~ 1218: 0.0246 us
    {0, 2048, 8, 8, 256},  // n ~ 1722: 0.023 us
    {0, 2896, 8, 8, 1024},  // n ~ 2435: 0.0752 us
    {0, 4096, 8, 8, 1024},  // n ~ 3444: 0.0756 us
    {0, 5793, 8, 8, 1024},  // n ~ 4871: 0.0813 us
    {0, 8192, 8, 8, 1024},  // n ~ 6889: 0.0828 us
    {0, 11585, 8, 0, 0},  // n ~ 9742: 0.1928 us
    {0, 16384, 8, 0, 0},  // n ~ 13777: 0.2716 us
    {0, 23170, 8, 0, 0},  // n ~ 19484: 0.3781 us
    {0, 32768, 8, 0, 0},  // n ~ 27554: 0.5273 us
    {0, 46341, 8, 0, 0},  // n ~ 38968: 0.7485 us
    {0, 65536, 8, 0, 0},  // n ~ 55109: 1.0273 us
    {0, 92682, 8, 0, 0},  // n ~ 77936: 1.4546 us
    {0, 131072, 8, 0, 0},  // n ~ 110218: 2.0413 us
    {0, 185364, 8, 0, 0},  // n ~ 155872: 2.9167 us
    {0, 262144, 8, 0, 0},  // n ~ 220436: 4.0597 us
    {0, 370728, 8, 0, 0},  // n ~ 311744: 5.8938 us
    {0, 524288, 8, 0, 0},  // n ~ 440872: 8.3183 us
    {0, 741455, 8, 0, 0},  // n ~ 623487: 11.8654 us
    {0, 1048576, 8, 0, 0},  // n ~ 881744: 16.7704 us
    {1, 181, 4, 4, 256},  // n ~ 152: 0.0149 us
    {1, 256, 4, 4, 256},  // n ~ 215: 0.0147 us
    {1, 362, 4, 4, 256},  // n ~ 304: 0.0149 us
    {1, 512, 4, 4, 256},  // n ~ 431: 0.0148 us
    {1, 724, 4, 4, 256},  // n ~ 609: 0.0151 us
    {1, 1024, 4, 4, 256},  // n ~ 861: 0.0171 us
    {1, 1448, 8, 8, 256},  // n ~ 1218: 0.0184 us
    {1, 2048, 8, 8, 256},  // n ~ 1722: 0.0192 us
    {1, 2896, 16, 16, 256},  // n ~ 2435: 0.0263 us
    {1, 4096, 16, 16, 256},  // n ~ 3444: 0.0267 us
    {1, 5793, 8, 8, 1024},  // n ~ 4871: 0.0668 us
    {1, 8192, 16, 8, 1024},  // n ~ 6889: 0.0659 us
    {1, 11585, 16, 0, 0},  // n ~ 9742: 0.1405 us
    {1, 16384, 16, 0, 0},  // n ~ 13777: 0.1862 us
    {1, 23170, 16, 0, 0},  // n ~ 19484: 0.2325 us
    {1, 32768, 16, 0, 0},  // n ~ 27554: 0.3251 us
    {1, 46341, 16, 0, 0},  // n ~ 38968: 0.4614 us
    {1, 65536, 16, 0, 0},  // n ~ 55109: 0.6411 us
    {1, 92682, 16, 0, 0},  // n ~ 77936: 0.9112 us
    {1, 131072, 16, 0, 0},  // n ~ 110218: 1.2435 us
    {1, 185364, 16, 0, 0},  // n ~ 155872: 1.8187 us
    {1, 262144, 16, 0, 0},  // n ~ 220436: 2.5025 us
    {1, 370728, 16, 0, 0},  // n ~ 311744: 3.5137 us
    {1, 524288, 16, 0, 0},  // n ~ 440872: 5.0715 us
    {1, 741455, 16, 0, 0},  // n ~ 623487: 7.1338 us
    {1, 1048576, 16, 0, 0},  // n ~ 881744: 10.2292 us
};

}  // namespace fs1

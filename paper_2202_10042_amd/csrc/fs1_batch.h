// fs1_batch.h -- device layout of a ragged batch of FS-1 solves
// (fs1_batch.hip, driven by fs1_api.cpp).  Not part of the public ABI.
//
// Instances are stored chunk-aligned in padded work arrays: instance b owns
// the global chunks [chunk0, chunk0 + nch) and the elements
// [base, base + nch * 256 * R) (its run length R decides the chunk length);
// entries past its n hold zeros.  Instances with the same R form a group, and
// one launch per group covers a list of chunk records (ChunkRef), one
// workgroup per record.
#pragma once

#include "fs1_internal.h"

namespace fs1 {

constexpr int kInstPow = 20;  // lambda^(chunk length * 2^s), s < 20: up to 2^20 chunks

// Constant description of one instance (written once, at admission).
struct InstInfo {
  const double* src_mu;  // the caller's marginals (read at set-up only)
  const double* src_nu;
  int64_t base;       // first element in the padded work arrays
  int32_t n;          // grid size
  int32_t nch;        // chunks
  int32_t chunk0;     // first global chunk
  int32_t l0;         // batch iteration counter at admission (iteration l = count - l0)
  double h;           // grid spacing
  double tol;         // stopping tolerance of Algorithm 1
  ScanConsts k;       // lambda and its decays for this instance's h / eps and R
  Decay cpow[kInstPow];
};

// Mutable per-instance state (the Ctrl block of a single solve).
struct InstState {
  int32_t done;       // stopped: converged, failed, capped or invalid
  int32_t stop_iter;  // l with err(l) <= tol, -1 if none
  int32_t fail;       // a scaling became non-finite
  int32_t fail_iter;  // first failing iteration (INT_MAX if none)
  int32_t capped;     // reached itr_max
  int32_t bad_input;  // a marginal entry is negative or non-finite
  int32_t invalid;    // bad input, zero or unequal masses
  int32_t last_check; // last iteration whose error was evaluated
  double last_err;
  double sum_mu;
  double sum_nu;
  double err;         // final nu-side error
  double mu_err;      // final mu-side error
  double w1;          // final transport cost
};

// One chunk of one instance, as a workgroup of a batched launch sees it: all
// it needs to issue its loads at once.
struct ChunkRef {
  int64_t base;       // element of the chunk's first entry
  int64_t lim;        // first element past the instance's n entries
  int32_t c;          // global chunk (aggregates, shares, run exponents)
  int32_t b;          // instance
  int32_t j;          // chunk within the instance
  int32_t nch;        // chunks of the instance
  int32_t chunk0;     // the instance's first global chunk
  int32_t l0;         // the instance's admission iteration
};

ChunkRef chunk_ref(const InstInfo& in, int b, int j);

struct BatchGroup {
  int R;
  const ChunkRef* list;  // device list of the chunks to run
  int nlist;             // entries of `list`
};

struct BatchBufs {
  int dtype;          // 0 double, 1 float
  int itr_max;
  int check_every;
  int64_t nchunks;    // all groups
  int64_t nelem;      // padded elements
  InstInfo* inst;
  InstState* st;
  int* iter_base;     // batch iteration counter (advanced on the device)
  int* ndone;         // instances stopped so far
  int* ring;          // optional: instance index of the k-th stop at ring[k % ring_cap]
  int ring_cap;
  double* mu64;       // padded marginals
  double* nu64;
  void* mu32;         // binary32 copies (dtype 1)
  void* nu32;
  void* vF;           // phi (padded)
  void* vG[2];        // psi, double-buffered by iteration parity
  int* eF;            // per-run exponents
  int* eG[2];
  ChunkAgg* aggF;     // chunk aggregates of phi / psi
  ChunkAgg* aggG;
  void* agg2;         // two-state chunk aggregates (cost)
  double* part;       // per-chunk shares: error (iterations, nu side), mass of mu (setup)
  double* part2;      // mu-side error, mass of nu (setup)
  double* part3;      // cost
};

InstInfo make_inst_info(const double* mu, const double* nu, int64_t base, int64_t n, int chunk0,
                        int R, double h, double eps, double tol, int l0);

// Instances ilist[0..count) (or 0..count-1 when ilist is null) and the chunks
// the groups list: pack the marginals, set phi = psi = 1/n, validate each
// instance and publish the chunk aggregates of phi.  `inst` / `st` must
// already hold the instances' descriptions and initial states.
hipError_t launch_batch_setup(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                              const int* ilist, int count, hipStream_t s);
// `count` iterations (psi-half, phi-half) of every group over its chunk
// list, then advance the iteration counter by `count`.  Safe to capture in a
// graph.
hipError_t launch_batch_iterations(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                                   int count, hipStream_t s);
// Final marginal errors and transport costs of the instances ilist[0..count)
// (or 0..count-1), whose chunks the groups list.  With `out` non-null their
// states are then gathered to out[0..count).
hipError_t launch_batch_finalize(const BatchBufs& z, const BatchGroup* groups, int ngroups,
                                 const int* ilist, int count, InstState* out, hipStream_t s);
// Resident instances (at most 1024 runs, allocated to exactly nt / 256 chunks
// of run length R): one workgroup of nt threads per instance runs all its
// iterations in one launch; on return each instance is stopped (done, stop
// iteration / failure / cap, ndone counted) with its final state in place for
// launch_batch_finalize.  Instances already stopped (invalid) are skipped.
struct ResGroup {
  int R;
  int nt;             // 256 or 1024
  const int* ilist;   // device list of instances
  int count;
};
hipError_t launch_batch_resident(const BatchBufs& z, const ResGroup* groups, int ngroups,
                                 hipStream_t s);
// Admission: copy count staged descriptions and states into the instance
// slots idx[0..count).
hipError_t launch_batch_admit(const BatchBufs& z, const InstInfo* sinfo, const InstState* sstate,
                              const int* idx, int count, hipStream_t s);

}  // namespace fs1

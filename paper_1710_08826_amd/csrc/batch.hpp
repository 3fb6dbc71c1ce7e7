// Batched fits: per-fit minimizer state and the device buffers of a batch.
#pragma once
#include "kernels.hpp"
#include "bfgs_device.hpp"
#include "mix1d_device.hpp"

namespace fn {

constexpr int kBatchMaxP = 24;      // parameters per batched fit
constexpr int kGenMaxAttempts = 64; // redraws per generated event

using BfgsState = BfgsStateT<kBatchMaxP>;

// Device pointers of a batch (n_fits slots).
struct BatchDev {
  BfgsState* st;
  Mix1dTable* tabs;
  const double** ev;       // event pointer per slot
  int64_t* nev;            // events per slot
  int64_t* item_base;      // n_fits + 1
  int64_t* part_base;      // first partial row of each slot
  double* part;            // partial rows
  double* out;             // per slot [NLL, grad(P), I, dI(P)]
  int* n_running;
  int* stat;               // per slot status, mirrored every step
  double* rres;            // per slot result row, written when the fit retires (3 + 2P)
};

// One request admitted into a slot (host staging, copied to the device once
// per admission round).  generate = 1: the slot's events are generated into ev
// by the admission launch (the mix1d toy generator, key (seed, fit), word 0).
struct AdmitRec {
  int32_t slot;
  int32_t generate;
  int64_t n;                   // events
  double* ev;                  // device events of the slot
  int64_t block0;              // first generation workgroup of this record in the launch
  uint32_t seed, fit;
  double theta_gen[4];         // mu, sigma, tau, f
  double theta0[kBatchMaxP];   // start point
};

// Admission of n_recs records (device copy): one workgroup per record resets
// its slot's minimizer state to a fresh fit at theta0 (all free) and sets the
// slot's status mirror and event pointer/count; gen_blocks more workgroups
// generate the events of the records with generate = 1 (record r owns
// workgroups [block0, block0 + ceil(n/256)), block0 ascending).
void batch_launch_admit(const BatchDev& b, const AdmitRec* recs, int n_recs, int64_t gen_blocks, int P, double lo,
                        double hi, unsigned int* n_unresolved, hipStream_t s);
// Slots [0, n_fits) become fresh fits at theta0 (device, n_fits x P, all
// parameters free), slots [n_fits, max_fits) idle; one workgroup per slot.
void batch_launch_set(const BatchDev& b, const double* theta0, int n_fits, int max_fits, int P, hipStream_t s);
// rows_out[i] = rres row of slot slots[i] (3 + 2P doubles), for n slots.
void batch_launch_gather_rows(const BatchDev& b, const int* slots, int n, int P, double* rows_out, hipStream_t s);

void batch_launch_step(const BatchDev& b, const Mix1dConst& mc, int n_fits, int P, int chunk, int eval_grid,
                       double tol, int max_iter, hipStream_t s);
int batch_eval_blocks_per_cu(const Mix1dConst& mc);
void batch_launch_gen_mix1d(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, const double* theta_gen, double lo,
                            double hi, double* x, unsigned int* n_unresolved, hipStream_t s);

}  // namespace fn

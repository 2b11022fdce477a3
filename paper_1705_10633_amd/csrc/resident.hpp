// resident.hpp -- the resident fold-in server's shared layout and launchers
// (kernels_resident.hip, used by serving.hip).
#pragma once
#include "common.hpp"

namespace bpmf {

// Resident fold-in server (kernels_resident.hip).  A slot in coherent pinned
// host memory: this header, then cols[max_nnz] (int32), vals[max_nnz]
// (float), q_cols[max_q] (int32) and out[max_q] (float).
struct ResidentSlotHeader {
    int32_t req_seq;   // written by the host (release) once the request is in the slot
    int32_t done_seq;  // written by the device (release) once out[] holds the predictions
    int32_t nnz, nq;
};
constexpr int RESIDENT_HEADER_BYTES = 256;
struct ResidentArgs {
    char *slots;          // n_slots slots of slot_bytes each (host memory)
    int64_t slot_bytes;
    int32_t max_nnz, max_q;
    const int32_t *stop;  // host memory: stop[0] non-zero ends the kernel; stop[1] counts assignments
    int32_t *dev_cols;    // device staging, max_nnz per slot
    float *dev_vals;      // device staging, max_nnz per slot
    int32_t *dev_q;       // device staging, max_q per slot
    const float *lam_mu;  // Lambda_s mu_s, S x K, from prepare_resident
    int64_t idle_polls;   // polls without a request before a workgroup ends
};
size_t resident_lds_bytes(int K, int S);
// Forms lam_mu (S x K) on stream st and sets the kernel's LDS limit.
hipError_t prepare_resident(int S, int K, const double *Lam, const double *mu, float *lam_mu, hipStream_t st);
// Slot workgroups the device holds at once (after prepare_resident); every
// slot's workgroup must be resident, or its requests could wait as long as
// the other slots stay busy.
hipError_t resident_max_slots(int K, int S, int *max_slots);
hipError_t launch_resident(int n_slots, int S, int K, int64_t N, double alpha, double rbar, const float *Vs,
                           const double *Lam, const double *mu, const ResidentArgs &ra, hipStream_t st);

}  // namespace bpmf

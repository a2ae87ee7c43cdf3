// Internal interface of request batches, shared with the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ephdc.h"

namespace ephdc {

// Validates a request list (the checks of ephdc_batch_create / _create_packed).
ephdc_status check_requests(const ephdc_request* reqs, uint32_t n_req, bool packed);

// Device bytes a batch of these requests takes under a schedule (mode 1 fused / 2 split,
// segment length) with plaintext chunks of at most pt_bytes; with packing, the batch also
// holds every session's packed query hypervectors and score ciphertexts.
size_t batch_bytes(const ephdc_request* reqs, uint32_t n_req, size_t pt_bytes, uint32_t mode, uint32_t seg_len,
                   bool packed);

// Plans a batch inside the caller's block `mem` of mem_bytes >= batch_bytes(...) (or in an
// owned allocation when mem is NULL); the work lists are uploaded on `hs`.
ephdc_status batch_new(const ephdc_request* reqs, uint32_t n_req, size_t pt_bytes, uint32_t mode, uint32_t seg_len,
                       bool packed, void* mem, size_t mem_bytes, hipStream_t hs, ephdc_batch** out);

// Packing: first query of request i in its session's packed sequence, its position in the
// first ciphertext the request receives, and how many ciphertexts it receives.
void batch_packing(const ephdc_batch* b, uint32_t i, uint32_t* query_offset, uint32_t* q_first, uint32_t* n_ct);

// Enqueues every launch of the batch on `hs`.
hipError_t batch_enqueue(const ephdc_batch* b, hipStream_t hs);

// Frees the batch (and its block when owned); the caller has waited for its work.
void batch_free(ephdc_batch* b);

}  // namespace ephdc

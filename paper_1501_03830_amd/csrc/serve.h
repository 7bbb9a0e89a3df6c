// Request server behind bse_submit / bse_poll / bse_release.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "../../include/bse.h"

namespace bse {

struct Server;

// pool_bytes: device memory for the workspaces of admitted requests (0:
// half of the free device memory); slots: concurrent batches, each on its
// own stream (0: 4); max_batch: requests per batch (0: 64).
int server_create(int device, size_t pool_bytes, int slots, int max_batch, Server** out);
void server_destroy(Server* s);
// `caller`: the stream the request's inputs were written on
int server_submit(Server* s, const bse_request* req, hipStream_t caller, uint64_t* ticket);
int server_poll(Server* s, uint64_t ticket, int* state, int* info);
int server_release(Server* s, uint64_t ticket);
int server_times(Server* s, uint64_t ticket, double* t_submit_us, double* t_start_us, double* t_done_us);
int server_stats(Server* s, bse_serve_counters* st);

}  // namespace bse

/*
 * bitbox_serve.h -- serving runtime of the bit-box particle compressor
 * (arXiv 2404.02826): compress and decompress requests of mixed sizes that
 * arrive over time are admitted under a device-memory budget and run with
 * continuous batching on one GPU.
 *
 * The method itself (quantize, k-d partition, bit boxes, packing, unpack,
 * dequantize; Sec. 3-4 of the paper) is the one of bitbox.h: a job's result
 * is byte-identical to the same call made alone through bitbox.h.  This
 * header adds the scheduling around it:
 *
 *   arena      a host-side sub-allocator over [0, bytes) offsets of one
 *              caller-owned device buffer (256-byte aligned blocks, best fit,
 *              neighbours coalesced on free).  Pure host bookkeeping.
 *   server     jobs wait in FIFO order; a job is admitted when its result
 *              buffer can be placed in the arena and the arena still has room
 *              for its workspace; admitted jobs are launched together (all
 *              compress jobs of a launch as one batched compress, then the
 *              decompress jobs) on one of several HIP streams, so launches
 *              overlap on the device; a launch retires when its event has
 *              completed, and its workspace returns to the arena.  Jobs keep
 *              their result memory until released.
 *
 * The server never allocates device memory (everything comes from the
 * caller's arena buffer) and never waits for the GPU inside
 * bbx_server_progress.  A server is used from one host thread.
 */
#ifndef BITBOX_SERVE_H
#define BITBOX_SERVE_H

#include "bitbox.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- arena (host bookkeeping only; no device access) */
typedef struct bbx_arena bbx_arena;

/* bytes: managed size; align: power of two >= 1 (blocks start and end on it). */
bbx_status bbx_arena_create(size_t bytes, size_t align, bbx_arena** out);
void bbx_arena_destroy(bbx_arena* a);
/* Places a block of `bytes` (rounded up to align) at the smallest free
 * range that holds it (lowest offset among equals); ENOMEM if none does. */
bbx_status bbx_arena_alloc(bbx_arena* a, size_t bytes, size_t* offset);
/* Frees the block that starts at offset; EINVAL if none starts there. */
bbx_status bbx_arena_free(bbx_arena* a, size_t offset);
void bbx_arena_stats(const bbx_arena* a, size_t* used, size_t* free_total, size_t* largest_free,
                     size_t* free_ranges);

/* ---- server */
typedef struct {
  size_t hbm_budget;      /* bytes of the arena buffer the server may use */
  uint32_t max_jobs;      /* jobs admitted and not yet released, at most */
  uint32_t max_batch;     /* jobs per launch, >= 1 (1 = one launch per job) */
  uint32_t nstreams;      /* launches in flight, 1..8, one HIP stream each */
  uint32_t tile_override; /* tile capacity of compress launches (0, 256, 512) */
} bbx_server_config;

typedef struct bbx_server bbx_server;

typedef enum {
  BBX_JOB_QUEUED = 0,
  BBX_JOB_ADMITTED = 1,
  BBX_JOB_RUNNING = 2,
  BBX_JOB_DONE = 3
} bbx_job_state;

typedef struct {
  uint32_t state;      /* bbx_job_state */
  uint32_t status;     /* bbx_status of the job (valid when done) */
  uint64_t bytes;      /* result bytes: stream length or positions size (when done) */
  void* d_result;      /* device address of the result (from admission to release) */
  double t_submit, t_admit, t_launch, t_done; /* seconds on the server clock */
  uint32_t batch_jobs; /* jobs in the launch that carried this one */
  uint32_t kind;       /* 0 compress, 1 decompress */
} bbx_job_info;

/* d_arena: device buffer of arena_bytes >= cfg->hbm_budget, 256-byte aligned,
 * owned by the caller and untouched by anyone else while the server lives. */
bbx_status bbx_server_create(const bbx_server_config* cfg, void* d_arena, size_t arena_bytes,
                             bbx_server** out);
/* Waits for the launches in flight, then frees the server (not the arena). */
bbx_status bbx_server_destroy(bbx_server* s);

/* Queues a compress of n particles at d_pos (device, caller-owned, unchanged
 * until the job is done).  ENOMEM if the job could never fit the budget. */
bbx_status bbx_server_submit_compress(bbx_server* s, const void* d_pos, uint64_t n, uint32_t dims,
                                      bbx_dtype dtype, double eb, const bbx_params* params,
                                      uint64_t* job);
/* Queues a decompress of the stream at d_stream (device, caller-owned);
 * h_header is a host copy of its first 128 bytes (copied by the call). */
bbx_status bbx_server_submit_decompress(bbx_server* s, const void* d_stream, size_t stream_size,
                                        const void* h_header, bbx_layout layout, uint64_t* job);

/* Retires finished launches, admits queued jobs, starts new launches on free
 * streams.  Never waits for the GPU.  *n_done (optional): jobs finished by
 * this call; their ids are returned by bbx_server_pop_done. */
bbx_status bbx_server_progress(bbx_server* s, uint32_t* n_done);
/* Next finished job id in completion order; 0 if none is pending. */
uint64_t bbx_server_pop_done(bbx_server* s);
/* State and timing of a job; for a finished job the status and result size
 * are read from the device (a 16-byte copy on the server's query stream). */
bbx_status bbx_server_job_info(bbx_server* s, uint64_t job, bbx_job_info* info);
/* Returns a finished job's result memory to the arena. */
bbx_status bbx_server_release(bbx_server* s, uint64_t job);
/* Seconds on the server's steady clock. */
double bbx_server_now(const bbx_server* s);
/* Jobs queued, admitted (waiting to launch), running; launches in flight;
 * launches started so far; arena bytes in use. */
void bbx_server_counts(const bbx_server* s, uint32_t* queued, uint32_t* admitted, uint32_t* running,
                       uint32_t* inflight, uint64_t* launches, size_t* arena_used);

#ifdef __cplusplus
}
#endif
#endif /* BITBOX_SERVE_H */

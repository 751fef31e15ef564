/* hmm_serve.h -- request-serving runtime on top of hmm_gpu.h.
 *
 * Decoding requests (Viterbi, section 3.3; posterior decoding, section 3.4)
 * of uneven length arrive at any time against models that stay resident on
 * the device.  A worker thread batches pending requests of the same model,
 * kind and length class (under 2048 steps, under 16384, longer) into one
 * launch as soon as a launch slot is free; launches with requests of the
 * longest class hold at most half of the slots (continuous
 * batching: requests that arrive while others run are admitted as slots and
 * memory free up, and their launches overlap on the device on separate
 * streams).  Admission is by a device-memory budget: the server allocates
 * its budget once at creation and places each launch's observations, outputs
 * and workspace in it; a launch starts only when its bytes fit.
 *
 * Every sequence is decoded independently of the others in its launch, so a
 * request's result is bitwise the same alone and in any mix.
 *
 * Threading: hmm_server_submit and hmm_server_poll may be called from any
 * host thread; one worker thread per server drives the device.  Error
 * messages of these calls go to hmm_last_error of the calling thread.
 */
#ifndef HMM_SERVE_H
#define HMM_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "hmm_gpu.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmm_server hmm_server;

typedef enum {
    HMM_REQ_VITERBI = 0,            /* most probable path and its log-probability */
    HMM_REQ_POSTERIOR_DECODE = 1    /* lowest argmax_j gamma_t(j) per step and log P(y) */
} hmm_req_kind;

typedef struct {
    size_t hbm_budget;      /* device bytes for request data and workspaces, allocated at
                               creation; a request needing more is refused at submit */
    size_t host_staging;    /* pinned host bytes for uploads and downloads, allocated at creation */
    int32_t max_batch;      /* most requests in one launch, >= 1 */
    int32_t n_streams;      /* launches in flight at once, 1 .. 16.  Streams share the
                               process's hardware queues (HIP's GPU_MAX_HW_QUEUES, 4 by
                               default), so more than that many overlap only if the
                               process raises it */
    int32_t precision;      /* HMM_PREC_F32 or HMM_PREC_F64 */
    int32_t device;         /* HIP device ordinal */
} hmm_server_opts;

/* Result record of one finished request. */
typedef struct {
    uint64_t id;            /* as returned by hmm_server_submit */
    int32_t model;
    int32_t kind;           /* hmm_req_kind */
    int32_t status;         /* 0 ok; 1 no path (log-probability -inf); 2 non-finite
                               observation; < 0: -hmm_status of a failed launch */
    int32_t batch_size;     /* requests in the launch that served it */
    int64_t T;              /* steps of the request */
    double logp;            /* Viterbi: path log-probability; posterior: log P(y) */
    double t_submit;        /* seconds on hmm_server_now's clock: submit returned */
    double t_launch;        /* its launch was enqueued */
    double t_done;          /* its path was in the caller's host buffer */
} hmm_completion;

/* Counters of a running server. */
typedef struct {
    int64_t submitted, completed, launches, pending, in_flight;
    size_t pool_bytes, pool_used, pool_peak;   /* device budget and its use */
} hmm_server_info;

/* Defaults: 16 GiB budget, 256 MiB staging, 64 requests per launch,
 * 4 streams, HMM_PREC_F32, device 0. */
void hmm_server_default_opts(hmm_server_opts *opts);

/* Seconds on the monotonic clock the completion times use. */
double hmm_server_now(void);

/* Allocates the budget and staging areas, creates the streams and starts
 * the worker.  HMM_ERR_DEVICE if an allocation fails. */
hmm_status hmm_server_create(const hmm_server_opts *opts, hmm_server **out);

/* Finishes every launch in flight, drops pending requests (they never
 * complete), stops the worker and frees everything the server owns. */
hmm_status hmm_server_destroy(hmm_server *server);

/* Makes a resident copy of a model (device FP64 parameters, layout of
 * hmm_model) and returns its id.  A request is served if hmm_viterbi or
 * hmm_posterior_decode accepts its model in the server's precision;
 * otherwise its completion carries the refused status. */
hmm_status hmm_server_add_model(hmm_server *server, const hmm_model *model, int32_t *model_id);

/* Queues one request.  obs: host [T * D] float (obs_f64 = 0) or double,
 * copied before the call returns.  path_out: host [T] int32, written before
 * the request's completion is reported and owned by the caller, who keeps
 * it valid until then.  HMM_ERR_WORKSPACE if the request alone needs more
 * than the budget. */
hmm_status hmm_server_submit(hmm_server *server, int32_t model_id, int32_t kind,
                             const void *obs, int32_t obs_f64, int64_t T, int32_t *path_out,
                             uint64_t *id);

/* Moves up to max finished requests into out (oldest first); waits up to
 * timeout_us microseconds for the first one when none is ready. */
hmm_status hmm_server_poll(hmm_server *server, hmm_completion *out, int32_t max,
                           int32_t timeout_us, int32_t *n_out);

hmm_status hmm_server_get_info(hmm_server *server, hmm_server_info *info);

#ifdef __cplusplus
}
#endif

#endif /* HMM_SERVE_H */

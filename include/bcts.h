/*
 * bcts.h -- C ABI of libbcts: Batch-BFS exhaustive tree search with the
 * Bellman-corrected (BCTS) root correction, on one AMD MI355X (gfx950).
 *
 * What a search computes, per root state s_0 with A actions and depth d:
 *
 *   Q_d(s_0, a) = max over a_1..a_{d-1}, a_d of
 *                 sum_{t<d} gamma^t r_t + gamma^d Q(s_d, a_d)         (Eq. 1)
 *
 * evaluated level by level: every node of depth k is expanded for all A
 * actions at once, the A^d leaves are scored by the Q-network, and returns
 * are backed up with the child index j*A + a so that the root action of leaf
 * i is floor(i / A^(d-1)) (Alg. 1).  The root vector is then corrected for
 * the off-policy bias of the maximum (Eq. 3 with the penalty B of Eq. 6):
 *
 *   pi_o      = argmax_a Q(s_0, a)                      (network at the root)
 *   delta(a)  = r(s_0, a) + gamma max_a' Q(s_1^a, a') - Q(s_0, a)  (Prop. 3.6)
 *   d_o       = |delta(pi_o)|,  d_e = mean_{a != pi_o} |delta(a)|
 *   B         = sqrt(ln A) (d_e sqrt(d) - d_o sqrt(d-1)) - (d_e - d_o)/sqrt(8)
 *   Q^BCTS(a) = Q_d(s_0, a) - c gamma^d B   for a != pi_o,
 *               Q_d(s_0, pi_o)              for a == pi_o
 *   action    = argmax_a Q^BCTS(a)  (lowest index on ties)          (Eq. 4)
 *
 * c is the constant multiplier of the correction (Sec. 5.1).  Depth 0 returns
 * Q(s_0, .) itself; a search without correction returns Q_d.  With
 * BCTS_CORR_EXACT_GEV the penalty is instead the exact gap of Lemma 3.2,
 * sigma_e Bn(A^d - A^(d-1)) - sigma_o Bn(A^(d-1)) with sigma = |delta|/sqrt 2.
 *
 * The forward model is a deterministic sprite world with Atari-shaped state
 * (84x84 uint8 frames, a stack of 4, channel 0 oldest); the value network is
 * the Nature-DQN CNN.  See bcts_set_env and bcts_set_qnet.
 *
 * Conventions for every entry point:
 *  - Host pointers are owned by the caller; the library copies what it needs
 *    before returning and keeps no caller pointer.  Device pointers (the
 *    *_device entry points) are borrowed until the work enqueued on the given
 *    stream completes.
 *  - The context owns all device memory, streams and graphs.  A context is
 *    not thread-safe: calls on one context must not overlap.
 *  - Arguments are validated before any GPU work; an invalid call returns
 *    BCTS_E_INVAL (or BCTS_E_STATE) and leaves the context usable.  A HIP
 *    failure returns BCTS_E_HIP and puts the context in an error state in
 *    which every call but bcts_last_error, bcts_reset and bcts_destroy
 *    returns BCTS_E_STATE.  bcts_last_error describes the latest failure.
 */
#ifndef BCTS_H
#define BCTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BCTS_FRAME      84          /* frame side (pixels)                      */
#define BCTS_FRAME_BYTES (84 * 84)  /* one uint8 frame                          */
#define BCTS_STACK      4           /* frames per state, channel 0 oldest       */
#define BCTS_SPRITES    8           /* sprite 0 is the agent                    */
#define BCTS_MAX_A      18          /* Atari's full action set                  */
#define BCTS_MAX_DEPTH  6
/* FP32 Q-network blob length: conv1.w[32][4][8][8], conv1.b[32],
 * conv2.w[64][32][4][4], conv2.b[64], conv3.w[64][64][3][3], conv3.b[64],
 * fc1.w[512][3136] (input index c*49 + h*7 + w), fc1.b[512], fc2.w[18][512],
 * fc2.b[18] -- PyTorch's OIHW / [out][in] layouts, in this order.           */
#define BCTS_QNET_NUMEL 1693362

typedef enum {
  BCTS_OK = 0,
  BCTS_E_INVAL = -1,   /* bad argument; nothing was launched                 */
  BCTS_E_NOMEM = -2,   /* over the context's HBM budget / allocation failed  */
  BCTS_E_HIP = -3,     /* HIP runtime error; context is now in error state   */
  BCTS_E_BUSY = -4,    /* serving: the ticket is not finished yet            */
  BCTS_E_STATE = -5    /* missing env/qnet, unknown ticket, or error state   */
} bcts_status;

typedef enum {
  BCTS_FP32 = 0,       /* FP32 operands, FP32 accumulate                      */
  BCTS_BF16 = 1,       /* BF16 operands and activations, FP32 accumulate      */
  BCTS_FP8 = 2         /* OCP e4m3 operands with per-layer scales, FP32 acc.  */
} bcts_precision;

typedef enum {
  BCTS_CORR_EQ6 = 0,        /* penalty B of Eq. 6                             */
  BCTS_CORR_EXACT_GEV = 1   /* exact bias gap of Lemma 3.2                    */
} bcts_corr_mode;

/* Sprite-world dynamics: action a moves sprite 0 by delta[a] = (dx, dy);
 * sprite i >= 1 moves by vel[i-1] every step; coordinates wrap modulo 84.
 * Each step renders an 84x84 frame: 6x6 squares anchored at (x, y) extending
 * +5 in x and y with wrap, value 128 for sprites 1..7 and 255 for sprite 0
 * (max compositing), and scores the number of sprites 1..7 whose square
 * overlaps sprite 0's (circular distance < 6 in x and in y), after the move. */
typedef struct {
  int32_t delta[BCTS_MAX_A][2];
  int32_t vel[BCTS_SPRITES - 1][2];
} bcts_env_params;

/* Root correction (Eq. 3).  enabled = 0 returns the uncorrected Q_d;
 * scale is the constant c; mode selects the penalty.                       */
typedef struct {
  int32_t enabled;
  float scale;
  int32_t mode;
} bcts_correction;

typedef struct bcts_ctx bcts_ctx;

/* Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device memory the context may hold (0 = 80% of the device's free memory).
 * BCTS_E_HIP if the device cannot be used.                                 */
bcts_status bcts_create(int hip_device, size_t hbm_budget_bytes, bcts_ctx** out);
void bcts_destroy(bcts_ctx* ctx);
/* Text of the last failure on ctx ("" if none); valid until the next call. */
const char* bcts_last_error(const bcts_ctx* ctx);
/* Leave the error state: synchronises, drops pending serving work (those
 * tickets then poll BCTS_E_STATE) and releases the work arena.             */
bcts_status bcts_reset(bcts_ctx* ctx);

/* Environment tables (copied).  |delta| <= 3 and |vel| <= 2 per component. */
bcts_status bcts_set_env(bcts_ctx* ctx, const bcts_env_params* env);

/* Q-network weights: FP32 blob of BCTS_QNET_NUMEL floats (layout above),
 * copied and converted on the device for every precision.  A search with A
 * actions uses fc2 rows 0..A-1.  Resets FP8 scales to their calibration
 * default (see bcts_calibrate_fp8).                                         */
bcts_status bcts_set_qnet(bcts_ctx* ctx, const float* blob, size_t n_floats);
/* Precision of the Q-network for subsequent searches (default BCTS_FP32).  */
bcts_status bcts_set_precision(bcts_ctx* ctx, bcts_precision prec);
/* FP8: derive per-layer activation scales from the FP32 network's
 * activation maxima on n calibration stacks (host uint8 [n][4][84][84]),
 * so that each layer's input maps to the e4m3 range.  The scales are kept
 * until the next bcts_set_qnet; bcts_get_fp8_scales reads them (5 floats).  */
bcts_status bcts_calibrate_fp8(bcts_ctx* ctx, int32_t n, const uint8_t* stacks);
bcts_status bcts_get_fp8_scales(bcts_ctx* ctx, float* out5);
bcts_status bcts_set_fp8_scales(bcts_ctx* ctx, const float* in5);

/* Search n_roots roots that share (depth, A).  Host buffers:
 *   pos     int32 [n][8][2]   (x, y) in [0, 84)
 *   stacks  uint8 [n][4][84][84]
 *   out_action int32 [n], out_q float [n][A] (the corrected vector).
 * depth in [0, 6], A in [1, 18] (A >= 2 when the correction is enabled and
 * depth >= 1), gamma in (0, 1].                                             */
bcts_status bcts_search(bcts_ctx* ctx, int32_t n_roots, const int32_t* pos, const uint8_t* stacks,
                        int32_t depth, int32_t A, float gamma, bcts_correction corr,
                        int32_t* out_action, float* out_q);

/* Search n_roots roots of individual depth[i] and A[i] in one batch (host
 * buffers).  out_q is float [n][18]; row i holds root i's vector in entries
 * 0..A[i]-1 and -INFINITY after.                                            */
bcts_status bcts_search_batch(bcts_ctx* ctx, int32_t n_roots, const int32_t* pos,
                              const uint8_t* stacks, const int32_t* depth, const int32_t* A,
                              float gamma, bcts_correction corr, int32_t* out_action,
                              float* out_q);

/* As bcts_search_batch, but pos/stacks/out_action/out_q are DEVICE pointers
 * and the work is enqueued on `hip_stream` (a hipStream_t; NULL = the
 * context's stream) without a host synchronisation.  depth and A stay host
 * arrays (the plan is made on the host).  Positions are not range-checked
 * here (they are device data); out-of-range positions are wrapped modulo 84. */
bcts_status bcts_search_batch_device(bcts_ctx* ctx, int32_t n_roots, const int32_t* d_pos,
                                     const uint8_t* d_stacks, const int32_t* depth,
                                     const int32_t* A, float gamma, bcts_correction corr,
                                     int32_t* d_out_action, float* d_out_q, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the search
 * of bcts_search_batch_device (same arguments, same kernels, same results
 * bit for bit), with every device buffer the search needs beyond the
 * caller's inputs and outputs -- plan tables, expanded levels, eval values,
 * Q-network activations -- carved from a static device array of 128 MiB that
 * the library holds on each device until the process ends.  No device or
 * pinned memory is allocated or freed by this call (the plan is made in
 * ordinary host memory; its tables are copied from there).  A search that
 * needs more than the array, even with the Q-network chunks halved down to
 * 256 stacks, returns BCTS_E_NOMEM and enqueues nothing (one root at A = 18,
 * depth 3 fits; the 256-root headline batch does not).  The array keeps the
 * last call's contents and every context on the device shares it: calls of
 * one context are ordered (a call on another stream first waits for the
 * previous one on the device), but calls from different contexts on one
 * device that overlap in time race.  No timing is recorded.                */
bcts_status bcts_search_batch_device_noalloc(bcts_ctx* ctx, int32_t n_roots, const int32_t* d_pos,
                                             const uint8_t* d_stacks, const int32_t* depth,
                                             const int32_t* A, float gamma, bcts_correction corr,
                                             int32_t* d_out_action, float* d_out_q, void* hip_stream);

/* Capture the device search of one batch shape into a HIP graph and replay
 * it `replays` times (buffers as in bcts_search_batch_device, stream NULL =
 * context stream), synchronising at the end; the graph is captured for this
 * call and released after it.  Results of every replay equal the eager
 * search.                                                                  */
bcts_status bcts_search_batch_graph(bcts_ctx* ctx, int32_t n_roots, const int32_t* d_pos,
                                    const uint8_t* d_stacks, const int32_t* depth,
                                    const int32_t* A, float gamma, bcts_correction corr,
                                    int32_t* d_out_action, float* d_out_q, int32_t replays,
                                    void* hip_stream);

/* A reusable captured search: the launch sequence of one batch shape (Alg. 1
 * for every root, then the correction) as an instantiated HIP graph on fixed
 * device input and output buffers, with its own work memory.  Create it
 * once (device buffers as in bcts_search_batch_device; they must stay
 * allocated while the graph exists, and a replay reads whatever they hold
 * then), then launch it any number of times on any stream without planning,
 * allocation or host synchronisation; results equal the eager search of
 * the buffers' contents at replay time.  While a graph exists the calls
 * that change the model or its settings (those refused while serving)
 * return BCTS_E_STATE.  bcts_graph_destroy waits for the device and frees
 * the graph's memory; it must be called before bcts_destroy.               */
typedef struct bcts_graph bcts_graph;
bcts_status bcts_graph_create(bcts_ctx* ctx, int32_t n_roots, const int32_t* d_pos, const uint8_t* d_stacks,
                              const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                              int32_t* d_out_action, float* d_out_q, void* hip_stream, bcts_graph** out);
bcts_status bcts_graph_launch(bcts_graph* graph, int32_t replays, void* hip_stream);
void bcts_graph_destroy(bcts_graph* graph);

/* ---- tuning -------------------------------------------------------------- */
/* Q-network execution choices (none changes results beyond the operand
 * precision; every choice keeps each stack's sum order fixed):
 *   BCTS_TUNE_FUSED        1 = BF16/FP8 run conv1..conv3 fused per sibling
 *                          group (default), 0 = layer-by-layer kernels
 *   BCTS_TUNE_FUSED_ROUND  stacks per LDS round of the fused kernel: 1..4
 *                          (BF16 caps at 3: a round of 4 exceeds the LDS)
 *   BCTS_TUNE_FUSED_CHUNK  stacks per Q-network chunk on the fused path
 *   BCTS_TUNE_LAYER_CHUNK  stacks per chunk on the layer-by-layer path
 *                          (also the FP32 correction evaluations below);
 *                          default 65,536 (about 100 KB of FP32 workspace
 *                          per stack)
 *   BCTS_TUNE_CORR_FP32    1 = (default) the Q-network inputs of the
 *                          correction -- Q(s_0, .), which fixes pi_o, and the
 *                          depth-1 values of the Bellman errors (Prop. 3.6)
 *                          -- are evaluated in FP32 whatever the precision,
 *                          so that a low-precision rounding cannot flip pi_o
 *                          or move delta; the leaves (and depth-0 searches)
 *                          keep the search precision.  At depth 1 the
 *                          depth-1 nodes are the leaves; their A FP32
 *                          evaluations are then extra work.  0 = every
 *                          evaluation at the search precision (at depth 1
 *                          the Bellman errors read the leaves' values).
 *   BCTS_TUNE_MLP_CROSSOVER  forward-model world, host-buffer searches
 *                          (bcts_mlp_search): the CPU-to-GPU cross-over of
 *                          Sec. 4.1 -- levels 1..k of the tree are expanded
 *                          on the host CPU, the rest (and every leaf) on
 *                          the GPU, k = min(value, depth - 1); 0 (default)
 *                          = the whole search on the GPU.  The host levels
 *                          do the device kernel's FP32 arithmetic in the
 *                          same order, so results are the same bits.
 *   BCTS_TUNE_FP8_K128     FP8 fused path: 1 (default) = conv2 / conv3 on
 *                          the K = 128 matrix instruction, their weights
 *                          held in LDS (rounds of 3 stacks whatever
 *                          BCTS_TUNE_FUSED_ROUND asks), 0 = the K = 32 one
 *                          (rounds of 1..4).
 *                          The products of each 8 consecutive K values are
 *                          summed the same way by both, so the results are
 *                          the same up to FP32 addition order.
 *   BCTS_TUNE_CONV1_GROUPS layer-by-layer path (FP32, the FP32 correction
 *                          evaluations, BCTS_TUNE_FUSED = 0): conv1 by
 *                          sibling groups -- the channels a group's stacks
 *                          share (0..2) summed once per group, each
 *                          sibling's channel 3 added to that partial sum --
 *                          or stack by stack.  2 = always by groups, 0 =
 *                          never, 1 (default) = per chunk, by groups when
 *                          the chunk holds enough groups to fill the GPU
 *                          (the group kernel's workgroups run longer: a
 *                          lone small request finishes sooner stack by
 *                          stack).  Same results, bit for bit.
 *   BCTS_TUNE_MLP_HOST     forward-model world, host-buffer searches
 *                          (bcts_mlp_search): 1 = the whole search on the
 *                          host CPU -- every level, the leaves' head, the
 *                          backup and the correction -- the CPU BFS of the
 *                          Sec. 4.1 runtime study; the GPU is not used.  The
 *                          device kernels' FP32 arithmetic in their order:
 *                          the same bits as the GPU search.  2 = the host
 *                          for small trees (at most 32 + 9 d nodes per
 *                          root, where one host core beats a host-buffer
 *                          GPU search), the GPU otherwise.  0 (default) =
 *                          the GPU (with BCTS_TUNE_MLP_CROSSOVER).
 *   BCTS_TUNE_FC2_FOLDED   BF16/FP8 fused path: 1 (default) = fc2 runs in
 *                          fc1's epilogue on the fc1 outputs rounded to the
 *                          operand type, each half of fc1's 512 outputs
 *                          summed apart and the halves added in a fixed
 *                          order; 0 = fc1 writes those outputs to device
 *                          memory and fc2 reads them back.  The same
 *                          operands, the sum over the 512 associated
 *                          differently: results agree to FP32 rounding.    */
typedef enum {
  BCTS_TUNE_FUSED = 0,
  BCTS_TUNE_FUSED_ROUND = 1,
  BCTS_TUNE_FUSED_CHUNK = 2,
  BCTS_TUNE_LAYER_CHUNK = 3,
  BCTS_TUNE_CORR_FP32 = 4,
  BCTS_TUNE_MLP_CROSSOVER = 5,
  BCTS_TUNE_FP8_K128 = 6,
  BCTS_TUNE_CONV1_GROUPS = 7,
  BCTS_TUNE_MLP_HOST = 8,
  BCTS_TUNE_FC2_FOLDED = 9
} bcts_tune_key;
bcts_status bcts_set_tuning(bcts_ctx* ctx, int32_t key, int64_t value);
bcts_status bcts_get_tuning(bcts_ctx* ctx, int32_t key, int64_t* value);
/* Autotuner: times every candidate -- fused or not, for FP8 the K = 128 or
 * K = 32 matrix instruction, the round size (stacks per LDS round: the
 * fused kernel's row tile), chunks of 256Ki / 1Mi stacks -- on one device
 * batch (arguments as in bcts_search_batch_device; the scratch outputs
 * receive the results), `reps` timed searches each after one warm-up, keeps
 * the fastest setting on the context and returns it: out_best [5] = {fused,
 * round, chunk, microseconds per search, FP8 K = 128}.  Candidates over the
 * HBM budget are skipped.                                                  */
bcts_status bcts_autotune(bcts_ctx* ctx, int32_t n_roots, const int32_t* d_pos, const uint8_t* d_stacks,
                          const int32_t* depth, const int32_t* A, float gamma, bcts_correction corr,
                          void* d_scratch_action, void* d_scratch_q, int32_t reps, void* hip_stream,
                          int64_t* out_best);

/* ---- serving: iteration-level continuous batching, pooled HBM admission --- */
/* The paper selects one action per tree search (Alg. 1); a server answers
 * many such requests at once.  The engine works in steps on its own stream:
 * before a step it admits queued requests, in arrival order, as a cohort
 * (planned as one batch) while its device memory pool and pinned staging
 * hold the cohort's plan; the step then advances every admitted cohort by
 * one stage of its search -- upload and level 1, each further level, each
 * Q-network chunk, the FP32 correction evaluations, backup and the copy of
 * its results -- or, for a light cohort (at most 32,768 nodes plus eval
 * items), by all of them.  A request that arrives while a large search runs
 * joins at the next stage boundary.  All cohorts share one memory pool
 * (what the HBM budget leaves beyond the weights, the work arena and the
 * shared Q-network workspace, capped at 16 GiB); a cohort's range returns to
 * the pool when its last stage has finished.  Results do not depend on how
 * requests were batched: each equals the same root searched alone, bit for
 * bit. */
/* Queue one request (host buffers copied).  Returns a ticket.  A request
 * whose own plan exceeds the serving pool fails with BCTS_E_NOMEM.         */
bcts_status bcts_submit(bcts_ctx* ctx, const int32_t* pos, const uint8_t* stack, int32_t depth,
                        int32_t A, float gamma, bcts_correction corr, uint64_t* ticket);
/* Advance the engine without blocking: retire finished steps and cohorts,
 * admit queued requests while the pools allow, enqueue up to max_inflight
 * steps.  *pending = requests queued or admitted and not yet finished.     */
bcts_status bcts_progress(bcts_ctx* ctx, int32_t* pending);
/* Result of a ticket: BCTS_OK (copied out, ticket released), BCTS_E_BUSY
 * (not finished), BCTS_E_STATE (unknown ticket).  q has room for A floats;
 * t_done is the host monotonic time (s) at which completion was observed.  */
bcts_status bcts_poll(bcts_ctx* ctx, uint64_t ticket, int32_t* action, float* q, double* t_done);
/* Serving limits: max requests admitted into one cohort, max engine steps in
 * flight (1..8).  Refused with BCTS_E_STATE while tickets are outstanding. */
bcts_status bcts_serve_config(bcts_ctx* ctx, int32_t max_batch, int32_t max_inflight);
/* Engine state (host view, as of the last bcts_progress): out[0] queued
 * requests, [1] admitted requests not finished, [2] admitted cohorts,
 * [3] cohorts with stages not yet enqueued, [4] steps in flight, [5] pool
 * bytes in use, [6] pool capacity, [7] cohorts finished so far.           */
bcts_status bcts_serve_stats(bcts_ctx* ctx, int64_t* out8);
/* While requests are queued or admitted (finished results waiting for
 * bcts_poll do not count), the calls that change what they read --
 * bcts_set_env, bcts_set_qnet, bcts_set_precision, bcts_set_fp8_scales,
 * bcts_calibrate_fp8, bcts_set_tuning, bcts_set_beam, bcts_autotune --
 * return BCTS_E_STATE and change nothing; drive bcts_progress until it
 * reports nothing pending first.                                           */
/* Device bytes one request of (depth, A) takes while admitted alone (its
 * levels, tables and values; the shared Q-network workspace aside).       */
size_t bcts_request_bytes(int32_t depth, int32_t A);

/* ---- pruned search ------------------------------------------------------ */
/* Batch-BFS gives the return of every node of a level at once, which the
 * paper suggests for early pruning with an index array of surviving nodes
 * (Sec. 4; left there as future work).  With beam B > 0 every later search
 * of the context (host, device, graph and served) cuts levels 2..d-1: inside
 * each root action's sub-tree only the B nodes with the largest discounted
 * return so far (FP32, lowest index on ties) are expanded further, their
 * root-local indices kept in a keep list per level; the leaves are all
 * children of the kept depth-(d-1) nodes, and Q_d(a0) is the best of a0's
 * surviving leaves.  The depth-0/1 quantities of the correction are not
 * affected.  B = 0 (the default) is the exhaustive search; a level whose
 * blocks hold at most B nodes is not cut, so B >= A^(d-2) changes nothing.
 * BCTS_E_INVAL outside [0, 256].                                            */
bcts_status bcts_set_beam(bcts_ctx* ctx, int32_t beam);

/* ---- learned forward-model world (Sec. 4.1's runtime study) ------------- */
/* The paper also times tree search over a deep network that mimics a learned
 * forward model: three hidden layers of width 100 fed a 100-dimensional
 * state and a one-hot action.  Here the model maps x = [s ; onehot(a)]
 * through ReLU(l1), ReLU(l2), ReLU(l3) to a linear output of 101 units (the
 * next state, then the reward), and a leaf state is valued by the linear head
 * Q(s, .) = q.w s + q.b; the search and the BCTS correction (Eq. 1, 3, 6) are
 * those of the sprite world.  FP32.
 *
 * bcts_set_mlp installs the model for A actions (2 <= A <= 18) from an fp32
 * blob in the order l1.w[100][100+A] (inputs: state then one-hot action),
 * l1.b[100], l2.w[100][100], l2.b[100], l3.w[100][100], l3.b[100],
 * out.w[101][100], out.b[101], q.w[A][100], q.b[A] ([out][in] matrices);
 * n_floats must equal that total.  The blob is copied.                      */
bcts_status bcts_set_mlp(bcts_ctx* ctx, int32_t A, const float* blob, size_t n_floats);
/* Search n_roots root states (fp32 [n][100], host) to `depth` (0..16), every
 * root with the model's A; out_action int32 [n], out_q fp32 [n][A] (the
 * corrected root vector; Q0 at depth 0).  BCTS_E_STATE without a model,
 * BCTS_E_INVAL on bad arguments or non-finite states, BCTS_E_NOMEM when the
 * tree (A^k states per root for k < depth, plus one float per leaf) exceeds
 * the budget.                                                              */
bcts_status bcts_mlp_search(bcts_ctx* ctx, int32_t n_roots, const float* states, int32_t depth,
                            float gamma, bcts_correction corr, int32_t* out_action, float* out_q);
/* The same with device pointers (states, outputs), enqueued on hip_stream
 * (NULL: the context's stream); nothing is copied and nothing synchronises.  */
bcts_status bcts_mlp_search_device(bcts_ctx* ctx, int32_t n_roots, const float* d_states, int32_t depth,
                                   float gamma, bcts_correction corr, int32_t* d_out_action,
                                   float* d_out_q, void* hip_stream);

/* ---- parity / debug exports (not on the timed path) -------------------- */
/* Expand one root to `depth` and copy every node out in the index order of
 * Alg. 1 (level 1 first; node j*A + a is child a of node j).  Host outputs
 * sized sum_{k=1..depth} A^k: out_pos int32 [..][8][2], out_frames uint8
 * [..][84][84], out_reward int32 [..].                                      */
bcts_status bcts_debug_expand(bcts_ctx* ctx, const int32_t* pos, const uint8_t* stack,
                              int32_t depth, int32_t A, int32_t* out_pos, uint8_t* out_frames,
                              int32_t* out_reward);
/* Failure injection (tests of the error path): the next `count` stage
 * launches of any search or serving step fail from the host before anything
 * of theirs is enqueued, as a failed launch would: the call returns
 * BCTS_E_HIP and the context enters the error state (every call but
 * bcts_reset, bcts_destroy and bcts_last_error then returns BCTS_E_STATE;
 * queued and admitted serving requests are dropped by bcts_reset).  Work
 * already enqueued runs to completion.                                     */
bcts_status bcts_debug_fail_launches(bcts_ctx* ctx, int32_t count);

/* Expand a batch of roots of mixed (depth, A) to their depths with the
 * context's beam (Alg. 1's loop body for every root at once, the pruned
 * search's keep lists included) and copy every node out as the search's
 * own tables lay it out.  Sizes first: with out_pos NULL only
 *   level_nodes [7]     nodes of level k (index k = 1..6) over all roots,
 *   keep_entries [7]    keep-list entries of level k over all roots,
 *   root_levels [n][7][3]  per root and level: first node of the root in the
 *                       level, its node count, its first keep-list entry
 *                       (-1: the level is not cut for that root; entries
 *                       a0 * beam .. hold root action a0's kept nodes as
 *                       root-local indices, ascending)
 * are filled.  Then, level after level (roots in order, each root's nodes
 * in the index order of Alg. 1 among the children of its kept nodes):
 * out_pos int32 [..][8][2], out_frames uint8 [..][84][84], out_reward int32
 * [..], out_ret float [..] (the FP32 discounted return a beam ranks by),
 * out_keep int32 [..] (all keep lists, level after level).  stacks is read
 * only for validation of its presence (the expansion reads positions).    */
bcts_status bcts_debug_expand_batch(bcts_ctx* ctx, int32_t n_roots, const int32_t* pos, const uint8_t* stacks,
                                    const int32_t* depth, const int32_t* A, float gamma, int64_t* level_nodes,
                                    int64_t* keep_entries, int64_t* root_levels, int32_t* out_pos,
                                    uint8_t* out_frames, int32_t* out_reward, float* out_ret, int32_t* out_keep);

/* Q-network on n host stacks at the current precision: out_q float [n][A]. */
bcts_status bcts_debug_qnet(bcts_ctx* ctx, int32_t n, const uint8_t* stacks, int32_t A,
                            float* out_q);
/* The same with the stacks in sibling groups of `group` (1..18) consecutive
 * stacks (the last group may be shorter), the grouping a search gives the A
 * children of one node (Alg. 1: a child's stack is its parent's last three
 * frames plus its own): the stacks of a group must share channels 0..2
 * (BCTS_E_INVAL otherwise).  The fused BF16/FP8 kernel, and the layer
 * path's conv1 under BCTS_TUNE_CONV1_GROUPS, then compute the shared
 * channels' part of conv1 once per group, as in a search.                  */
bcts_status bcts_debug_qnet_siblings(bcts_ctx* ctx, int32_t n, const uint8_t* stacks, int32_t A,
                                     int32_t group, float* out_q);
/* Kernel timing with HIP events on the search's own stream.  While enabled,
 * every search (host, device or graph form) records events around its
 * launches and waits for them; bcts_get_timing then reports the last search:
 *   out[0] expansion ms, out[1] Q-network ms, out[2] backup+correction ms,
 *   out[3] whole search ms, out[4..8] conv1/conv2/conv3/fc1/fc2 ms summed over
 *   chunks, out[9] chunks (launches per layer), out[10..15] expansion ms of
 *   levels 1..6, out[16] Q-network items, out[17] expanded nodes, out[18] 1 if
 *   the fused conv kernel ran (its time is then in out[4]; out[5..6] are 0),
 *   out[19] ms of the FP32 correction evaluations (BCTS_TUNE_CORR_FP32;
 *   included in out[1], not in out[4..8]), out[20] chunks of the
 *   layer-by-layer path whose conv1 ran by sibling groups
 *   (BCTS_TUNE_CONV1_GROUPS).
 * A graph replay fills only out[3] (ms per replay).  out has 24 doubles.    */
bcts_status bcts_set_timing(bcts_ctx* ctx, int32_t enabled);
bcts_status bcts_get_timing(bcts_ctx* ctx, double* out24);

#ifdef __cplusplus
}
#endif
#endif /* BCTS_H */

/*
 * ka.h -- kernel actors on MI355X (gfx950): the C ABI.
 *
 * A kernel actor wraps one data-parallel kernel behind a message interface:
 * a message is matched against the kernel's signature, the kernel is launched
 * over an ND-range, and the outputs are answered either as host values or as
 * references to device memory that the next actor consumes in place
 * (arXiv 1709.07781, Sec. 3.2 "core approach", Sec. 3.4 "programming
 * interface", Sec. 3.5 "OpenCL actors as kernel stages").  Actors compose
 * (C = B (.) A, Sec. 3.5) into pipelines whose intermediate data never leave
 * the device; the WAH bitmap index of Sec. 4 is the composed workload.
 *
 * Conventions for every call:
 *  - Every function returns int: KA_OK (0) or a negative KA_E_* code.  On
 *    failure out-parameters are left untouched and ka_last_error() gives a
 *    message for the calling thread.  No C++ exception crosses this ABI.
 *  - Objects are reference counted.  Every create / spawn / compose / send and
 *    every returned ka_ref gives the caller one reference, released with the
 *    matching *_release / *_destroy.  Composed actors keep their stages alive;
 *    commands in flight keep the refs they use alive until the device is done
 *    with them.
 *  - Pointers named host point to host memory, pointers named dptr to device
 *    memory of the system's device.  Sizes are element counts unless the name
 *    says bytes.
 *  - Only uint32 data (KA_U32) is accepted by the built-in kernels.  Signature
 *    checking is by dtype, direction and mode, as in Sec. 3.4.
 */
#ifndef KA_H_
#define KA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KA_API __attribute__((visibility("default")))

/* ---- status codes ---------------------------------------------------------------- */
enum {
  KA_OK = 0,
  KA_E_ARG = -1,              /* invalid argument or null pointer */
  KA_E_TYPE = -2,             /* dtype / direction / mode does not match the signature */
  KA_E_ARITY = -3,            /* wrong number of message elements */
  KA_E_NOKERNEL = -4,         /* no kernel of that name in the program */
  KA_E_DEVICE = -5,           /* no usable gfx950 device, or a HIP runtime failure */
  KA_E_OOM = -6,              /* device allocation failed */
  KA_E_BUDGET = -7,           /* the system's HBM budget would be exceeded */
  KA_E_TIMEOUT = -8,          /* ka_receive timed out; the ticket stays valid */
  KA_E_NOT_SERIALIZABLE = -9, /* device references never leave the process (Sec. 3.5, option a) */
  KA_E_LAUNCH = -10,          /* kernel launch failed (the ticket carries the error) */
  KA_E_CANCELLED = -11,       /* work was cancelled (system destroyed, server stopped) */
  KA_E_STATE = -12            /* object used in a state that does not allow the call */
};

/* ---- types ----------------------------------------------------------------------- */
typedef enum ka_dtype { KA_U32 = 1, KA_I32 = 2, KA_U64 = 3, KA_F32 = 4, KA_U8 = 5 } ka_dtype;

/* Argument directions of a kernel signature (Sec. 3.4): in, out, in_out,
 * local (work-group memory, neither initialised nor read by the host, not
 * persistent) and priv (private values fixed at spawn, passed by value). */
typedef enum ka_dir { KA_IN = 1, KA_OUT = 2, KA_IN_OUT = 3, KA_LOCAL = 4, KA_PRIV = 5 } ka_dir;

/* How an argument is accepted from / handed on to messages (Sec. 3.4):
 * a host value, or a reference to device memory (mem_ref). */
typedef enum ka_mode { KA_VAL = 0, KA_REF = 1 } ka_mode;

enum { KA_ACCESS_READ = 1u, KA_ACCESS_WRITE = 2u, KA_ACCESS_RW = 3u };

typedef struct ka_system ka_system;
typedef struct ka_program ka_program;
typedef struct ka_actor ka_actor;
typedef struct ka_ref ka_ref;
typedef struct ka_ticket ka_ticket;
typedef struct ka_server ka_server;
typedef struct ka_srv_req ka_srv_req;
typedef struct ka_batch_plan ka_batch_plan;

/* System configuration (the actor_system_config that loads the device module,
 * Sec. 3.4).  HIP is initialised lazily on the first call that needs the
 * device (Sec. 3.2: discovery on first access). */
typedef struct ka_system_config {
  int32_t device;            /* HIP device ordinal; the first device by default (Sec. 3.6) */
  uint32_t n_streams;        /* command queues (HIP streams) in the system; 0 means 1 */
  uint64_t hbm_budget_bytes; /* device memory the system may hold at once; 0 = unlimited */
  void* stream;              /* optional borrowed hipStream_t used as stream 0 (e.g. torch's) */
  uint32_t flags;            /* KA_SYS_* */
} ka_system_config;

#define KA_SYS_PROFILE 1u /* time every kernel launch with device events (ka_profile_get) */

/* ND-range (Sec. 3.4): global dimensions, optional offsets of the global ids,
 * optional work-group dimensions.  For the built-in kernels global[0] is the
 * number of elements processed (one logical work-item per element); 0 means
 * "the length of the first input".  local[0] = 0 picks the kernel's own
 * work-group size; a non-zero value must be one the kernel supports. */
typedef struct ka_nd_range {
  uint32_t dims;      /* 1..3 */
  uint64_t global[3];
  uint64_t offset[3];
  uint32_t local[3];
} ka_nd_range;

/* One element of a message or of a response. */
typedef struct ka_value {
  uint32_t mode;  /* KA_VAL or KA_REF */
  uint32_t dtype; /* ka_dtype of a VAL (ignored for REF: the ref knows its type) */
  void* ptr;      /* VAL: host pointer (input: read before ka_send returns;
                     output: caller buffer of `count` elements, or NULL to query) */
  uint64_t count; /* VAL: element count (output: set to the produced count) */
  ka_ref* ref;    /* REF: a device reference (input: borrowed; output: +1 reference) */
} ka_value;

/* Output size from the inputs of the message (Sec. 3.4: a user function
 * overriding the default size). */
typedef uint64_t (*ka_size_fn)(const ka_value* inputs, uint32_t n_inputs, void* ud);

/* One argument of a kernel signature. */
typedef struct ka_arg {
  uint32_t dir;       /* ka_dir */
  uint32_t dtype;     /* ka_dtype */
  uint32_t in_mode;   /* IN / IN_OUT: accepted mode (KA_VAL or KA_REF) */
  uint32_t out_mode;  /* OUT / IN_OUT: produced mode (KA_VAL or KA_REF) */
  uint64_t count;     /* OUT: capacity in elements (0 = default: the number of work-items,
                         or the kernel's own bound); LOCAL: elements per work-group;
                         PRIV: number of elements at `init` (1 for a scalar) */
  ka_size_fn size_fn; /* OUT: optional capacity function, takes precedence over count */
  void* size_ud;
  const void* init;   /* PRIV: the value(s), copied at spawn */
} ka_arg;

/* Pre- and post-processing (Sec. 3.4, Listing 3 and Sec. 3.5): map an incoming
 * message to the kernel's in / in_out arguments, and the kernel's in_out / out
 * results to the response.  Both run on the thread that runs the actor.
 * Inputs are borrowed for the duration of the call; the function writes at
 * most `cap` values to `out` and their number to `*n_out`.  REF values it
 * returns are borrowed from its inputs (the runtime takes its own reference);
 * a REF it drops is released, which frees the device memory once unused
 * (Sec. 3.5).  VAL host data it returns must stay valid until it returns.
 * A non-zero return fails the request with that code. */
typedef int (*ka_map_fn)(const ka_value* in, uint32_t n_in, ka_value* out, uint32_t* n_out, uint32_t cap,
                         void* ud);

/* ---- errors ---------------------------------------------------------------------- */
KA_API const char* ka_error_string(int code);
KA_API const char* ka_last_error(void); /* thread-local message of the last failure */

/* ---- system ---------------------------------------------------------------------- */
/* Creates a system.  cfg may be NULL (defaults).  Touches no device until
 * needed; a later call fails with KA_E_DEVICE if the device is not gfx950.
 * The environment variable KA_LOOKBACK_SPIN, read when the device is first
 * used, sets how many times a scan tile polls a predecessor tile that has not
 * published its total before computing that total from its input (default
 * 16; 1 takes that path at once, which tests use).  Results never depend on
 * it. */
KA_API int ka_system_create(const ka_system_config* cfg, ka_system** out);
/* Waits for all work in flight, then frees every resource the system holds.
 * Objects still referenced by the caller become unusable (KA_E_STATE). */
KA_API int ka_system_destroy(ka_system* sys);
/* Blocks until every stream of the system is idle. */
KA_API int ka_system_synchronize(ka_system* sys);
/* The hipStream_t of stream i (initialises the device). */
KA_API int ka_system_stream(ka_system* sys, uint32_t i, void** stream);
/* Device memory currently held by the system, in bytes (in use and cached). */
KA_API int ka_system_memory(ka_system* sys, uint64_t* in_use, uint64_t* reserved);
/* How many times a device-resident length (the count a kernel produced, e.g.
 * compact_nonzero_u32's) was read back on the host, each a wait for its
 * producer: by ka_ref_info, ka_ref_read, ka_receive of a value output,
 * ka_batch_run of a reference input, or an actor that must plan its launch on
 * the host (wah_index_batch).  Sorts,
 * encoders, scans, compaction and queries read such counts on the device, so a
 * composition of them adds nothing here.  Never waits. */
KA_API int ka_system_length_reads(ka_system* sys, uint64_t* count);

/* ---- programs (Sec. 3.2: kernels looked up by name) ------------------------------ */
/* The built-in kernels, compiled ahead of time for gfx950:
 *   affine_u32            (in_out x; priv a; priv b)             x <- a*x + b mod 2^32
 *   exclusive_scan_u32    (in x; out y)                           y[i] = x[0] + .. + x[i-1] mod 2^32
 *   compact_nonzero_u32   (in x; out y)                           y = x without zeros, in order;
 *                                                                 the produced count is device-resident
 *   radix_sort_pairs_u32  (in keys; in rows; out skeys; out srows) stable sort of (key, row) by key
 *   radix_sort_rows_u32   (in keys; out skeys; out srows)         same with rows 0..n-1 (Sec. 4.1 part 1-2)
 *   wah_encode_sorted     (in skeys; in srows; out keys; out offsets; out words)
 *                                                                 Sec. 4.1 parts 3-6 on sorted pairs
 *   wah_index             (in values; priv value_bits [, format]; out keys; out offsets;
 *                          out words)
 *                                                                 Sec. 4.1 parts 1-6 in one actor: the
 *                                                                 sort, then the encoder (same words as
 *                                                                 the composition of the two actors above);
 *                                                                 value_bits as KA_WAH_VALUE_BITS (0 = no
 *                                                                 hint); a value at or above the hint
 *                                                                 gives every output length 0; format
 *                                                                 KA_WAH_PAPER/CANONICAL/PLWAH
 *   wah_lookup            (in queries; in keys; out slots)       slots[i] = d with keys[d] == queries[i],
 *                                                                 else 0xFFFFFFFF (keys ascending: the
 *                                                                 lookup table of Sec. 4.1)
 *   wah_decode            (in words; priv format, ngroups; out groups)
 *                                                                 one bitmap's words as ngroups 31-bit
 *                                                                 group words (bit b of groups[g] = row
 *                                                                 31 g + b); output length 0 if the words
 *                                                                 describe more than ngroups groups
 *   wah_combine           (in a; in b; priv op, in_format, out_format, ngroups; out words)
 *                                                                 AND (op 0) or OR (op 1) of two bitmaps
 *                                                                 of ngroups groups, re-encoded in
 *                                                                 out_format (capacity 2 ngroups + 1; the
 *                                                                 length is device-resident, 0 if an
 *                                                                 input describes more groups)
 *   wah_index_batch       (in values; in req_off; priv value_bits; out keys; out offsets;
 *                          out words; out key_start; out word_start)
 *                                                                 the index of each of nreq requests
 *                                                                 (see ka_wah_batch), one pass for all;
 *                                                                 priv may hold a second value, the
 *                                                                 largest request + 1: with requests of
 *                                                                 at most 1024 values and value_bits
 *                                                                 <= 22 each is built by one work-group
 *                                                                 (under such a hint a request above
 *                                                                 1024 values fails the batch: all
 *                                                                 output lengths 0)
 * The names, their signatures and the data each one reads and writes are
 * documented at ka_spawn. */
KA_API int ka_program_builtin(ka_system* sys, ka_program** out);
/* Loads a gfx950 code object (.hsaco).  Its kernels are launched with one
 * parameter per signature argument, in order: a device pointer for
 * in / out / in_out, a uint32 byte offset into the dynamic LDS for local, the
 * value(s) of priv; then a ka_nd_range_dev holding the global sizes and offsets.
 * Grid = ceil(global / local) work-groups of `local` work-items. */
KA_API int ka_program_load(ka_system* sys, const char* hsaco_path, ka_program** out);
KA_API int ka_program_release(ka_program* prog);

/* Trailing parameter of kernels from ka_program_load. */
typedef struct ka_nd_range_dev {
  uint64_t global[3];
  uint64_t offset[3];
} ka_nd_range_dev;

/* ---- actors ---------------------------------------------------------------------- */
/* Spawns a kernel actor (Sec. 3.4, Listing 2): `kernel` from `prog`, launched
 * over `range`, with the signature sig[0..nargs).  The signature is checked
 * against the kernel's own (KA_E_TYPE / KA_E_ARITY); out arguments are
 * allocated by the runtime with their default or given capacity.  A message
 * is matched against the in and in_out arguments in order; the response
 * consists of the in_out and out arguments in order (Sec. 3.4).
 * Outputs whose length depends on the data (compact_nonzero_u32,
 * wah_encode_sorted) keep their true length on the device; consumers read it
 * there, so no host round-trip is needed between stages (Sec. 4.1, the
 * "config" array). */
KA_API int ka_spawn(ka_system* sys, ka_program* prog, const char* kernel, const ka_nd_range* range,
                    const ka_arg* sig, uint32_t nargs, ka_actor** out);
/* Installs pre/post-processing functions (either may be NULL = identity). */
KA_API int ka_actor_set_mapping(ka_actor* actor, ka_map_fn pre, ka_map_fn post, void* ud);
/* out = outer (.) inner (Sec. 3.5): a message to `out` goes to `inner`, whose
 * response becomes the message to `outer`, whose response answers the
 * original request.  Without mapping functions the response of `inner` must
 * match the message of `outer` in arity, dtype and mode (else KA_E_TYPE). */
KA_API int ka_compose(ka_actor* outer, ka_actor* inner, ka_actor** out);
/* Selects the stream (command queue) the actor's work is queued on; a
 * composed actor queues all its stages on its own stream. */
KA_API int ka_actor_set_stream(ka_actor* actor, uint32_t stream);
KA_API int ka_actor_retain(ka_actor* actor);
KA_API int ka_actor_release(ka_actor* actor);

/* ---- messaging (Sec. 3.4: request / receive) ------------------------------------- */
/* Asynchronous request.  VAL host inputs are copied before the call returns;
 * REF inputs are borrowed (each command keeps its own reference until the
 * device is done).  Device work of a chain is enqueued before the call
 * returns; stages hand references on before the device finishes (Sec. 3.5). */
KA_API int ka_send(ka_actor* actor, const ka_value* args, uint32_t nargs, ka_ticket** out);
/* Sends a message to `target` whose response goes to `reply_to` instead of
 * the sender (Sec. 3.4: CAF's send_as and other ways to route an OpenCL
 * actor's result): target's response is reply_to's message, and the ticket
 * answers with reply_to's response.  Each actor's work is queued on its own
 * stream, the handoff ordered by the references.  The other ways of the same
 * passage: a post-processing function (ka_actor_set_mapping) may send its
 * result to other actors with ka_send, and one that returns no values
 * suppresses the response (the ticket then has arity 0); composition is
 * ka_compose. */
KA_API int ka_send_as(ka_actor* target, ka_actor* reply_to, const ka_value* args, uint32_t nargs, ka_ticket** out);
/* Waits for the response (timeout_us < 0: forever; 0: poll).  For each VAL
 * output, outs[i].count is set to the produced count and, if outs[i].ptr is
 * non-NULL, that many elements are copied there (KA_E_ARG, with count set, if
 * the caller's count is smaller).  For each REF output, outs[i].ref receives a
 * new reference and outs[i].count its length if known on the host, else its
 * capacity (ka_ref_info gives the true length).  A failed request returns its
 * error code.  The ticket stays valid until ka_ticket_release, so receive may
 * be called again. */
KA_API int ka_receive(ka_ticket* ticket, ka_value* outs, uint32_t nouts, int64_t timeout_us);
/* One request of a batch: a message of nargs elements. */
typedef struct ka_request {
  const ka_value* args;
  uint32_t nargs;
} ka_request;

/* Sends nreq independent requests to one actor as one batch (Sec. 3.6: data
 * parallelism nested inside one kernel is an alternative level of composition
 * to one actor invocation per request).  tickets[i] answers reqs[i] exactly as
 * ka_send(actor, reqs[i].args, reqs[i].nargs) would (the caller provides nreq
 * ticket slots and releases each ticket).  The built-in actors with a batched
 * form run all requests in one pass of their kernels on the actor's stream:
 * wah_index with a value-bits hint (one batched index build; a value at or
 * above the hint fails only its own request, with KA_E_ARG at ka_receive),
 * exclusive_scan_u32 (one scan of the concatenation, rebased per request) and
 * affine_u32 (one launch over the concatenation; a request that sent a
 * reference gets it back updated in place).  Each request is then one uint32
 * element, a host value or a device reference; REF outputs are read-only
 * views of the batch's output buffers.  Any other actor, or one with mapping
 * functions, gets the requests one after another.  The call waits for the
 * batch's per-request tables (index requests) or read-back (VAL outputs);
 * REF outputs are handed on in stream order. */
KA_API int ka_batch_run(ka_actor* actor, const ka_request* reqs, uint32_t nreq, ka_ticket** tickets);
/* Number of response elements (available before completion). */
KA_API int ka_ticket_arity(ka_ticket* ticket, uint32_t* n);
KA_API int ka_ticket_release(ka_ticket* ticket);

/* ---- device references (mem_ref, Sec. 3.5) --------------------------------------- */
/* Type, element count and access rights.  count is the true length; for a
 * data-dependent output this waits for the producing kernel. */
KA_API int ka_ref_info(ka_ref* ref, uint32_t* dtype, uint64_t* count, uint32_t* access);
/* Capacity in elements (never waits). */
KA_API int ka_ref_capacity(ka_ref* ref, uint64_t* capacity);
/* Copies min(bytes, length) to host memory after the producer finished. */
KA_API int ka_ref_read(ka_ref* ref, void* host, uint64_t bytes);
/* Device address of the referenced buffer (valid while the ref is held). */
KA_API int ka_ref_device_ptr(ka_ref* ref, void** dptr);
/* Wraps caller-owned device memory (e.g. a torch tensor) without copying.
 * The caller keeps it alive and unmodified while any command uses it;
 * releasing the last reference does not free it. */
KA_API int ka_ref_wrap(ka_system* sys, void* dptr, uint32_t dtype, uint64_t count, uint32_t access,
                       ka_ref** out);
/* Allocates an uninitialised device buffer from the system's pool. */
KA_API int ka_ref_alloc(ka_system* sys, uint32_t dtype, uint64_t count, ka_ref** out);
KA_API int ka_ref_retain(ka_ref* ref);
/* Drops a reference; the last one returns the memory to the system's pool,
 * ordered after every command that used it (Sec. 3.5: dropping a ref
 * releases its device memory). */
KA_API int ka_ref_release(ka_ref* ref);
/* Device references are process-local: always KA_E_NOT_SERIALIZABLE
 * (Sec. 3.5, option (a)). */
KA_API int ka_ref_serialize(const ka_ref* ref, void* buf, uint64_t cap, uint64_t* len);

/* ---- the composed WAH index (Sec. 4) --------------------------------------------- */
#define KA_WAH_INPUT_DEVICE 1u /* `values` is a device pointer (else host memory) */
#define KA_WAH_OUTPUT_REFS 2u  /* return device refs (else host arrays from malloc) */
/* Every value is below 2^b (b = 1..32; 0 = no hint).  With b <= 16 the sort
 * runs ceil(b / 8) passes over 16-bit sort keys (Sec. 4.2 sorts with a fixed
 * cardinality of 16 bits).  A value at or above 2^b fails with KA_E_ARG. */
#define KA_WAH_VALUE_BITS(b) (((uint32_t)(b) & 0x3Fu) << 8)
/* Word format of the bitmaps (Sec. 4.1 calls fills homogeneous blocks; Sec. 6
 * names PLWAH): KA_WAH_PAPER (default) one literal per non-empty group and
 * 0-fills only; KA_WAH_CANONICAL a run of full groups (all 31 rows) becomes one
 * 1-fill, bit 30 set, run length in bits 29..0; KA_WAH_PLWAH canonical with
 * 25-bit fill lengths (bits 24..0), and a fill absorbs the group right after
 * it when that group differs from the fill's groups in one bit only: bits
 * 29..25 = 1 + that bit's index (0: none).  PLWAH needs n <= 31 (2^25 - 1). */
enum { KA_WAH_PAPER = 0, KA_WAH_CANONICAL = 1, KA_WAH_PLWAH = 2 };
#define KA_WAH_FORMAT(f) (((uint32_t)(f) & 0xFFu) << 16)

typedef struct ka_wah_result {
  uint64_t n;        /* input elements */
  uint64_t D;        /* distinct values = bitmaps */
  uint64_t W;        /* WAH words over all bitmaps */
  uint32_t* keys;    /* host: keys[D] ascending (NULL with KA_WAH_OUTPUT_REFS) */
  uint32_t* offsets; /* host: offsets[D+1], bitmap d is words[offsets[d] .. offsets[d+1]) */
  uint32_t* words;   /* host: words[W] */
  ka_ref* keys_ref;  /* device refs (KA_WAH_OUTPUT_REFS only) */
  ka_ref* offsets_ref;
  ka_ref* words_ref;
} ka_wah_result;

/* Builds the WAH bitmap index of values[0..n) (rows 0..n-1) with the built-in
 * wah_index actor (the sort and encoder stages of the composed actor
 * wah_encode_sorted (.) radix_sort_rows_u32, queued by one actor; same words)
 * and waits for it.  flags: KA_WAH_* above.  Word
 * format: a literal has bit 31 clear and bit b standing for row 31*g + b of
 * its 31-row group g; a fill has bit 31 set, bit 30 clear and the number of
 * empty groups it covers in bits 29..0.  Each non-empty group of a value is
 * one literal, each run of empty groups before a literal one fill, counted
 * from group 0; a bitmap ends at its last literal.  n < 2^30. */
KA_API int ka_wah_index(ka_system* sys, const uint32_t* values, uint64_t n, uint32_t flags,
                        ka_wah_result* out);
/* Frees the host arrays and releases the refs of a result. */
KA_API int ka_wah_result_free(ka_wah_result* res);

/* ---- batched index builds (Sec. 3.6: data parallelism nested inside one kernel
 * as an alternative to one actor per stage; Sec. 4: the index of each request) - */
typedef struct ka_wah_batch_result {
  uint32_t nreq;     /* requests */
  uint64_t n;        /* elements over all requests */
  uint64_t D;        /* bitmaps over all requests */
  uint64_t W;        /* words over all requests */
  /* Request j's index is keys[key_start[j] .. key_start[j+1]),
   * offsets[key_start[j] + j .. key_start[j+1] + j] (D_j + 1 entries, relative
   * to its own words) and words[word_start[j] .. word_start[j+1]), exactly what
   * ka_wah_index returns for that request alone. */
  uint32_t* keys;       /* host: keys[D]        (NULL with KA_WAH_OUTPUT_REFS) */
  uint32_t* offsets;    /* host: offsets[D + nreq] */
  uint32_t* words;      /* host: words[W] */
  uint32_t* key_start;  /* host: key_start[nreq + 1] */
  uint32_t* word_start; /* host: word_start[nreq + 1] */
  ka_ref* keys_ref;     /* device refs (KA_WAH_OUTPUT_REFS only) */
  ka_ref* offsets_ref;
  ka_ref* words_ref;
  ka_ref* key_start_ref;
  ka_ref* word_start_ref;
} ka_wah_batch_result;

/* Builds the index of each of nreq independent requests in one pass of the
 * pipeline and waits for it.  values[0..n) holds the requests' values one
 * after the other; req_off (host memory, nreq + 1 entries) gives request j the
 * values [req_off[j], req_off[j+1]), with req_off[0] = 0, req_off[nreq] = n,
 * non-decreasing (empty requests allowed); rows restart at 0 in every request.
 * Every value must be below 2^value_bits, and value_bits plus the bits of
 * nreq - 1 must not exceed 32 (the request number is carried in the sort key's
 * high bits), else KA_E_ARG.  values is host memory, or device memory with
 * KA_WAH_INPUT_DEVICE.  n < 2^30. */
KA_API int ka_wah_batch(ka_system* sys, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                        uint32_t value_bits, uint32_t flags, ka_wah_batch_result* out);
/* Frees the host arrays and releases the refs of a batch result. */
KA_API int ka_wah_batch_result_free(ka_wah_batch_result* res);

/* Batch plans: the batched index build of one fixed batch shape (request
 * boundaries req_off[0..nreq], n = req_off[nreq]) recorded once into a HIP graph
 * on the plan's own stream and replayed by each run (Sec. 3.6: with the stages
 * composed, the per-stage launch work is the overhead left).  With
 * KA_PLAN_AUTOTUNE it records one graph per sort variant and its first run
 * times them all on the real values and keeps the fastest: variant 0 sorts
 * each request inside its own positions over 16-bit keys when value_bits <=
 * 16 (ceil(value_bits / 8) passes, the digits splitting value_bits evenly,
 * 1024 x 8 work-items x keys per tile), else the request-tagged keys with
 * that tile; variants 1 and 2 sort the request-tagged 32-bit keys with
 * 512 x 16 and 512 x 8; variant 3 is variant 0 with 8-bit digits first (the
 * rest in the second pass).  A batch whose
 * requests all hold at most 1024 values (and value_bits <= 22) takes the
 * small-request path instead: variants 0 and 2 are its three-launch form,
 * variant 1 one persistent fused launch (requests handed out by a ticket
 * counter, placed by a look-back over requests).  The plan owns
 * its input, outputs and scratch (nothing is allocated per run); outputs are
 * those of ka_wah_batch.  Requirements on req_off and value_bits as there. */
#define KA_PLAN_AUTOTUNE 1u /* record one graph per sort variant; the first run picks the fastest */
#define KA_PLAN_SHAPE(s) (((uint32_t)(s) + 1u) << 8) /* record sort variant s only (0, 1 or 2) */
KA_API int ka_batch_plan_create(ka_system* sys, const uint32_t* req_off, uint32_t nreq, uint32_t value_bits,
                                uint32_t flags, ka_batch_plan** out);
/* A plan for any batch of at most max_requests requests and max_values values
 * in all (each request at most max_request_values values; 0 = no bound, and a
 * bound of 1024 or less selects the one-work-group-per-request path): its
 * graphs are recorded once for these capacities and serve every batch that
 * fits.  The request table lives on the device, a batch of fewer requests is
 * padded with empty ones, and the kernels read the value count from the table.
 * The plan starts out holding an empty batch; ka_batch_plan_run_batch gives it
 * the next one.  value_bits plus the bits of max_requests - 1 must not exceed
 * 32; max_values < 2^30. */
KA_API int ka_batch_plan_create_any(ka_system* sys, uint64_t max_values, uint32_t max_requests,
                                    uint32_t max_request_values, uint32_t value_bits, uint32_t flags,
                                    ka_batch_plan** out);
/* The device buffer (n uint32) the graph reads the values from. */
KA_API int ka_batch_plan_input(ka_batch_plan* plan, uint32_t** values_dev);
/* The plan's hipStream_t (runs are ordered on it). */
KA_API int ka_batch_plan_stream(ka_batch_plan* plan, void** stream);
/* Copies values (host memory, or device memory with KA_WAH_INPUT_DEVICE; NULL:
 * the input buffer already holds them) and launches the graph; does not wait. */
KA_API int ka_batch_plan_run(ka_batch_plan* plan, const uint32_t* values, uint32_t flags);
/* Any-batch plans: a new batch (req_off: nreq + 1 host entries, as for
 * ka_wah_batch, nreq <= max_requests, req_off[nreq] <= max_values), then as
 * ka_batch_plan_run with its values (n = req_off[nreq]); does not wait.
 * KA_E_STATE for a plan recorded for one batch shape. */
KA_API int ka_batch_plan_run_batch(ka_batch_plan* plan, const uint32_t* values, const uint32_t* req_off,
                                   uint32_t nreq, uint32_t flags);
/* Waits for the last run and returns its outputs as host arrays (free with
 * ka_wah_batch_result_free); KA_E_ARG if a value was at or above 2^value_bits.
 * An any-batch plan returns its last batch's requests only. */
KA_API int ka_batch_plan_result(ka_batch_plan* plan, ka_wah_batch_result* out);
/* The tile shape the runs use (-1 before the first run of an autotuned plan)
 * and, for an autotuned plan, the time of its first run with each shape
 * (ms[0..nms), 0 for shapes not tried). */
KA_API int ka_batch_plan_shape(ka_batch_plan* plan, int* shape, float* ms, uint32_t nms);
KA_API int ka_batch_plan_destroy(ka_batch_plan* plan);

/* ---- the served form (Sec. 2.1: an actor's messages wait in its mailbox in
 * order of arrival; Sec. 3.6: an OpenCL actor's mailbox maps to a command queue) - */
/* Request kinds: the WAH index of the values (outputs keys, offsets, words, as
 * ka_wah_index), their exclusive scan mod 2^32 (one output), or the server's
 * affine chain x <- a_i x + b_i, i = 0..chain_len-1 (one output). */
enum { KA_REQ_WAH = 0, KA_REQ_SCAN = 1, KA_REQ_CHAIN = 2 };

typedef struct ka_server_config {
  uint32_t streams;          /* batches in flight at once, one per system stream (0 = 2; at most
                                the system's n_streams) */
  uint32_t max_batch;        /* requests merged into one batch (0 = 1024; 1 = no batching) */
  uint64_t max_batch_bytes;  /* input bytes merged into one batch (0 = 16 MiB; a larger request runs alone) */
  uint64_t hbm_budget_bytes; /* device memory the server's batches may hold together (0 = 64 GiB) */
  uint32_t value_bits;       /* index requests: every value below 2^value_bits (0 = 12) */
  uint32_t chain_len;        /* affine chain stages and their parameters (a_i odd) */
  const uint32_t* chain_a;
  const uint32_t* chain_b;
  uint32_t copy_threads;     /* threads that copy a host payload of 1 MiB or more into pinned memory,
                                the submitting thread included (0 = 4; 1 = the submitting thread alone) */
} ka_server_config;

typedef struct ka_server_stats {
  uint64_t completed;      /* requests finished since the last reset */
  uint64_t failed;
  uint64_t elements;       /* input elements of the completed requests */
  uint64_t batches;
  double mean_batch;       /* requests per batch */
  double p50_us, p99_us, max_us, mean_us; /* latency: arrival to completion seen on the host */
  uint64_t queued;         /* requests waiting in the mailbox now */
  uint64_t budget_in_use;  /* bytes admitted now, and the peak since the reset */
  uint64_t budget_peak;
} ka_server_stats;

/* Starts a server on `sys`: a mailbox thread that forms a batch from the
 * oldest waiting requests whenever a stream slot is free and the HBM budget
 * admits them (continuous batching: requests that arrive while batches run
 * wait for the next slot), and a completion thread.  Index requests of a batch
 * run as one batched index build, scans as one scan rebased per request,
 * chains as one chain over their concatenation; batches on different streams
 * overlap.  Each result is the one the request gets alone.  Creation warms the
 * system's device pool and pinned staging for batches up to max_batch_bytes
 * (per stream slot, two blocks of each power of two from 1 MiB up to a full
 * batch's need; about 1 GiB of device memory per stream slot and 256 MiB of
 * pinned memory at the default 16 MiB), which stay cached in the system
 * after the server ends. */
KA_API int ka_server_create(ka_system* sys, const ka_server_config* cfg, ka_server** out);
/* Queues a request (the data are copied before return).  arrival_us is its
 * arrival time on the ka_server_clock_us clock (0 = now); latency is measured
 * from it.  KA_E_BUDGET if the request alone exceeds the budget, KA_E_ARG for
 * an index value at or above 2^value_bits.  n < 2^30. */
KA_API int ka_server_submit(ka_server* srv, uint32_t kind, const uint32_t* data, uint64_t n, double arrival_us,
                            ka_srv_req** out);
/* Queues a request given as a message (Sec. 3.4: request ... receive) and
 * answers it with a ticket.  in[0] holds the request's uint32 data: a host
 * value (KA_VAL, copied before return) or a device reference (KA_REF,
 * borrowed: the server keeps its own reference until the request's batch has
 * copied the data on the device, ordered after the ref's last writer).  The
 * response, taken with ka_receive, is the request's outputs (KA_REQ_WAH: keys,
 * offsets, words; otherwise one array) as host values, or with
 * KA_SRV_OUTPUT_REFS as device references of their own (Sec. 3.5: a result
 * handed on without leaving the device).  Each result is the one the request
 * gets alone.  An index value at or above 2^value_bits fails only this
 * request with KA_E_ARG (at the call for host data, at ka_receive for a
 * reference).  Other arguments and errors as ka_server_submit. */
#define KA_SRV_OUTPUT_REFS 1u
KA_API int ka_server_send(ka_server* srv, uint32_t kind, const ka_value* in, uint32_t nin, uint32_t flags,
                          double arrival_us, ka_ticket** out);
/* Waits for a request (timeout_us < 0: no limit); KA_E_TIMEOUT leaves it
 * pending; a failed request returns its error (KA_E_CANCELLED if the server
 * was destroyed before it ran). */
KA_API int ka_server_wait(ka_srv_req* req, int64_t timeout_us);
/* Output i of a finished request: *count elements, copied to host[0..cap)
 * when host is given (KA_E_ARG if cap is too small). */
KA_API int ka_server_result(ka_srv_req* req, uint32_t i, uint32_t* host, uint64_t cap, uint64_t* count);
/* Releases a request handle (its outputs live in pinned host memory shared
 * with its batch until every request of the batch is released).  Release
 * requests before destroying the system. */
KA_API int ka_server_request_release(ka_srv_req* req);
KA_API int ka_server_get_stats(ka_server* srv, ka_server_stats* out);
KA_API int ka_server_reset_stats(ka_server* srv);
/* Now on the clock of arrival times (CLOCK_MONOTONIC, microseconds). */
KA_API int ka_server_clock_us(double* now);
/* Cancels waiting requests, waits for batches in flight, stops the threads. */
KA_API int ka_server_destroy(ka_server* srv);

/* ---- allocation-free index build ---------------------------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  The same
 * composed build as ka_wah_index (same kernels, same words), with every
 * scratch buffer carved from one static device array of the library (about
 * 66 MiB per device, held by each device the library runs on until the process
 * ends).  The array's device address is looked up on the first call on each
 * device; no call allocates or frees device memory.
 *
 * All pointers are device memory of the current HIP device: values[n]; keys
 * (capacity n), offsets (n + 1) and words (2n) as in ka_wah_index; lengths[3]
 * receives D, D + 1 and W (uint64, written on the device).  The work is queued
 * on `stream` (a hipStream_t; NULL = the default stream) and the call does not
 * wait.  KA_E_ARG if n > KA_NOALLOC_MAX_N or a pointer is missing.  Every call
 * on one device shares the static array: calls that may overlap on a device
 * (other streams, other threads) race and must be ordered by the caller. */
#define KA_NOALLOC_MAX_N (1u << 22)
KA_API int ka_wah_index_noalloc(const uint32_t* values, uint64_t n, uint32_t* keys, uint32_t* offsets,
                                uint32_t* words, uint64_t* lengths, void* stream);

/* ---- the actor-overhead baseline (Sec. 3.6) ---------------------------------------- */
/* Queues `stages` launches of the affine kernel (x <- a[i] x + b[i] mod 2^32)
 * over the device array x[0..n) on stream 0, without actors or messages: the
 * raw launch sequence against which a chain of affine actors is measured.
 * Does not wait. */
KA_API int ka_affine_chain_raw(ka_system* sys, uint32_t* x, uint64_t n, const uint32_t* a, const uint32_t* b,
                               uint32_t stages);

/* ---- profiling (KA_SYS_PROFILE) -------------------------------------------------- */
/* Launch count and summed device time of every kernel named `kernel` since
 * the last reset (waits for the device). */
KA_API int ka_profile_get(ka_system* sys, const char* kernel, uint64_t* launches, double* total_ms);
KA_API int ka_profile_reset(ka_system* sys);
/* Switches the per-launch timing of KA_SYS_PROFILE on or off (each timed launch
 * is bracketed by two events on its stream). */
KA_API int ka_profile_enable(ka_system* sys, int on);

#ifdef __cplusplus
}
#endif
#endif /* KA_H_ */

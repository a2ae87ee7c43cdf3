/*
 * ephdc.h - C ABI of the EP-HDC client-side encrypted hyperdimensional inference path
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (EP-HDC, client-side HE): the server encrypts its class hypervectors
 * once with BFV and ships them; the client encodes its plaintext queries into
 * hypervectors, batch-encodes every query element into its own plaintext (each value
 * repeated once per class), multiplies those plaintexts into the encrypted model and
 * accumulates, and sends one score ciphertext per batch back to the server, which
 * decrypts the similarity scores and takes the argmax (proposed method: client-side
 * HE; packing and op counts: D ct x pt products, no rotation).
 *
 * Server-side calls (keygen, model encryption, decryption) work on host memory.
 * Client-side calls work on device memory owned by the caller and are ordered on the
 * HIP stream passed in (a hipStream_t, given as void*; NULL is the default stream).
 *
 * Conventions
 *  - Every buffer is owned by the caller.  A session copies what it keeps (its own
 *    transformed copy of the model and keys), borrows the scratch workspace it is given,
 *    and may be used only from one host thread at a time; its scoring calls on different
 *    streams are ordered by the session (each waits on the device for the previous one).
 *  - Residues are uint32 in [0, q); polynomials are N coefficients in degree order;
 *    arrays are C-contiguous with the shapes given below.
 *  - Errors: argument and parameter errors are returned before any work is queued.
 *    HIP failures return EPHDC_ERR_HIP.  ephdc_last_error() gives a message for the
 *    last failing call on the calling thread.
 *  - Results are bit-exact functions of the inputs: independent of stream, batch
 *    composition and kernel schedule.
 */
#ifndef EPHDC_H
#define EPHDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EPHDC_OK = 0,
  EPHDC_ERR_ARG = 1,         /* null pointer, size out of range */
  EPHDC_ERR_PARAMS = 2,      /* parameter set fails validation (see ephdc_check_params) */
  EPHDC_ERR_BUFFER = 3,      /* a caller buffer is too small */
  EPHDC_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  EPHDC_ERR_NOKEY = 5,       /* rotations needed (r > 1) but no Galois keys were given */
  EPHDC_ERR_OOM = 6,         /* device allocation failed */
  EPHDC_ERR_UNSUPPORTED = 7, /* valid parameters outside what the kernels implement */
  EPHDC_ERR_TIMEOUT = 8      /* a wait ended at its time limit */
} ephdc_status;

/* Homomorphic scheme of the model ciphertexts (Preliminary: HE; noise results). */
enum {
  EPHDC_BFV = 0,          /* BFV, message term Delta*mu with Delta = floor(Q/t) (the paper's scheme) */
  EPHDC_BFV_ROUNDED = 1,  /* BFV, message term round(Q*mu/t) */
  EPHDC_BGV = 2           /* BGV: ([-a*s + t*e + mu]_Q, a), mu centred; decryption [c0 + c1*s]_Q mod t */
};

/* Slot layouts (ephdc_params.layout); the paper does not fix which slots a query occupies. */
enum {
  EPHDC_LAYOUT_CONTIGUOUS = 0, /* the K copies of a query in K consecutive slots of a row; B = 2 floor(N/(2rK)) */
  EPHDC_LAYOUT_SUBRING = 1     /* the K' copies of a query (K' the power of two >= K) on one orbit of
                                  {h = 1 mod 2N/K'} acting on the slot exponents: every query plaintext
                                  is a polynomial in X^K'; B = N/(K' r) */
};

/*
 * BFV / BGV + HDC parameters (symbols of the paper's table of symbols: N polynomial degree,
 * log2 t message bits, D hypervector dimension, K = k classes).
 *
 *   N      ring degree; the device kernels implement N in {2048, 4096, 8192, 16384}
 *   L      number of ciphertext primes q[0..L-1], 1 <= L <= 16
 *   alpha  number of special primes p[0..alpha-1] used only by key switching
 *   dnum   key-switching digits (limb groups of ceil(L/dnum) primes); 0 when r == 1
 *   q, p   the primes: distinct, prime, < 2^30, and = 1 (mod 2N)
 *   t      plaintext modulus: a prime = 1 (mod 2N) with 257 <= t and N * t < 2^32 (the
 *          device's inverse transform mod t runs without reductions under that bound);
 *          t = 65537 is the default.  The slot map uses zeta = g^((t-1)/2N), g the smallest
 *          generator of Z_t^*.
 *   F      features per query; D hypervector dimension; K classes
 *   r      fold factor (power of two): r consecutive dimensions share one ciphertext,
 *          in r blocks of W = N/(2r) slots per row; log2(r) rotate-and-sum steps fold
 *          them (r = 1 is the paper's packing and needs no rotation; BGV takes r = 1 only)
 *   qbits  1: binarised queries (+1 / -1); 2..8: clamp(H >> qshift) to qbits signed bits
 *   scheme EPHDC_BFV, EPHDC_BFV_ROUNDED or EPHDC_BGV (server-side encryption and
 *          decryption; the client's ct x pt arithmetic is the same ring arithmetic for all)
 *   scale_every, scale_shift
 *          HE-aware quantisation (EP-HDC design space exploration, BGV/BFV-aware
 *          quantisation): with g = scale_every > 0, after every g ciphertext additions of
 *          the multiply-accumulate (model ciphertexts m = 0..M-1 in order) the accumulator
 *          is multiplied by the plaintext scalar c = centred (2^scale_shift)^-1 mod t, which
 *          divides the plaintext by 2^scale_shift wherever it is divisible.  A trailing
 *          block of fewer than g additions is not scaled.  0 <= scale_shift < 32.
 *   layout EPHDC_LAYOUT_CONTIGUOUS (the default) or EPHDC_LAYOUT_SUBRING.  Subring layout,
 *          with n = N/K' and B = n/r: block v < r of query ql < B of a ciphertext holds
 *          dimension m*r + v on the K' slots of exponents gamma^u * (e + 2n*c) mod 2N, class
 *          c < K', where e = 2*brev(ql) + 1 (brev over log2 B bits), gamma = 1 + 2n/r and u < r
 *          is the power for which gamma^u * e = 2*brev(ql*r + v) + 1 (mod 2n), brev over
 *          log2 n bits (u = 0 at v = 0; for r = 1 the exponents are e + 2n*c).  Slot s < N/2
 *          is the exponent 3^s mod 2N, slot N/2 + s its negation.  The model holds class c's
 *          value at c < K and 0 at K <= c < K', the query plaintext the query's value at all
 *          K' slots.  Rotation step i uses the Galois element gamma^(2^i) mod 2N, which sums
 *          the r blocks of each class into block 0 (where the scores are read).  Its
 *          plaintexts are polynomials in X^K', so their transforms are n-point transforms
 *          (scoring runs that shorter transform where the kernels implement it: 256 <= n <=
 *          4096 and K' <= 32).  Needs B >= 2.
 *
 * Derived: Bq = floor(W/K) queries per row, B = 2*Bq queries per ciphertext (subring: B =
 * N/(K' r)), M = ceil(D/r) model ciphertexts, G = ceil(Q/B) score ciphertexts for Q queries.
 */
typedef struct {
  uint32_t N, L, alpha, dnum;
  const uint32_t* q;
  const uint32_t* p;
  uint32_t t;
  uint32_t F, D, K, r;
  int32_t qbits;
  uint32_t qshift;
  uint32_t scheme;
  uint32_t scale_every, scale_shift;
  uint32_t layout;
} ephdc_params;

/* Message describing the last failure on this thread ("" if none). */
const char* ephdc_last_error(void);

/* Validates a parameter set: EPHDC_OK, or EPHDC_ERR_PARAMS with a message. */
ephdc_status ephdc_check_params(const ephdc_params* prm);

/* Derived sizes (0 on invalid parameters). */
uint32_t ephdc_queries_per_ct(const ephdc_params* prm);            /* B */
uint32_t ephdc_num_model_ct(const ephdc_params* prm);              /* M */
uint32_t ephdc_num_groups(const ephdc_params* prm, uint32_t Q);    /* G */
uint32_t ephdc_hv_stride(const ephdc_params* prm, uint32_t Q);     /* G*B: row length of the hv array */
size_t   ephdc_galois_key_words(const ephdc_params* prm);          /* log2(r)*dnum*2*(L+alpha)*N */

/* The `count` largest primes below 2^30 that are 1 mod 2N, after skipping `skip`, descending. */
ephdc_status ephdc_default_primes(uint32_t N, uint32_t count, uint32_t skip, uint32_t* out);

/* The discrete-Gaussian cumulative table used by the samplers: 39 thresholds T_{-19}..T_{19}
 * (sigma = 3.2, support [-19, 19]; T_k = round(2^53 * P[e <= k]), T_19 = 2^53). */
ephdc_status ephdc_gaussian_cdt(uint64_t out[39]);

/* ------------------------------------------------------------------ server side (host memory) */

/*
 * Secret key and Galois (rotation) keys.  Server side of the protocol: the server owns
 * the key and encrypts with it (BFV with a given secret key, Preliminary: HE).
 *   sk           out, int8 [N], ternary {-1, 0, 1}; draws 0..N-1 of SplitMix64 stream
 *                (seed, tag 4), value (u mod 3) - 1
 *   galois_keys  out, uint32 [log2 r][dnum][2][L+alpha][N], coefficient domain, limbs in
 *                the order q[0..L-1], p[0..alpha-1]; component 0 is b, 1 is a.  May be NULL
 *                when r == 1.  Key (i, j) switches from sigma_g(s) to s for digit j, g the
 *                layout's Galois element of step i (contiguous: 3^(W*2^i) mod 2N; subring:
 *                gamma^(2^i) mod 2N, gamma = 1 + 2n/r): b = -a*s + e + G_j*sigma_g(s), G_j = P (product of the
 *                special primes) on the digit's limbs and 0 on all others; a uniform per
 *                limb and e discrete Gaussian from stream (seed, tag 6), draws starting at
 *                ((i*dnum + j) * (L+alpha+1)) * N.
 */
ephdc_status ephdc_keygen(const ephdc_params* prm, uint64_t seed, int8_t* sk, uint32_t* galois_keys);

/*
 * Encrypts the model: class hypervectors C int8 [K][D] -> M ciphertexts.
 * Server side, done once; the ciphertexts are sent to the client (proposed method).
 *   model_ct  out, uint32 [M][2][L][N], coefficient domain.
 * Ciphertext m encodes the slot vector with C[c][m*r+u] at every query position of block u
 * (the class HV replicated into every query slot) and is the secret-key encryption
 * ([-a*s + e + Delta*mu]_q, a), Delta = floor(Q/t), with a uniform per limb and e
 * discrete Gaussian drawn from stream (seed, tag 5) starting at m*(L+1)*N.
 */
ephdc_status ephdc_encrypt_model(const ephdc_params* prm, const int8_t* sk, const int8_t* class_hv,
                                 uint64_t seed, uint32_t* model_ct);

/*
 * Decrypts G = ceil(Q/B) score ciphertexts uint32 [G][2][L][N] (coefficient domain) and
 * reads the similarity scores: scores int32 [Q][K], each the centred residue mod t of the
 * integer dot product h . C[c], and argmax int32 [Q] (ties to the lowest class); argmax
 * may be NULL.  Server side (proposed method: the server sees only the scores).
 */
ephdc_status ephdc_decrypt_scores(const ephdc_params* prm, const int8_t* sk, const uint32_t* score_ct,
                                  uint32_t Q, int32_t* scores, int32_t* argmax);

/*
 * The same for queries q_first .. q_first + Q - 1 of a ciphertext sequence (query q of the
 * sequence sits in ciphertext q / B): score_ct holds ciphertexts 0 .. ceil((q_first+Q)/B)-1
 * of it, and only those from q_first / B on are read.  Rows of scores / argmax start at
 * q_first.  Used for requests packed into shared ciphertexts (ephdc_batch_create_packed,
 * packed serving), whose queries start inside a ciphertext.
 */
ephdc_status ephdc_decrypt_scores_at(const ephdc_params* prm, const int8_t* sk, const uint32_t* score_ct,
                                     uint32_t q_first, uint32_t Q, int32_t* scores, int32_t* argmax);

/* ------------------------------------------------------------------ client side (device memory) */

typedef struct ephdc_session ephdc_session;

/*
 * Device workspace of ephdc_score_encrypted for batches of up to max_Q queries, in bytes
 * (0 on invalid parameters): the work items' partial sums (sized for every schedule of
 * ephdc_session_tune), the rotation workspace when r > 1, and the split path's plaintext
 * chunk (the lifted plaintexts of all groups of max_Q queries, at most 4 GiB, at least one
 * plaintext per group).  Any buffer of at least the size without the 4 GiB chunk (one
 * plaintext per group of max_Q) is accepted; a larger chunk scores the model in fewer chunks.
 * Client side, homomorphic scoring (proposed method: client-side HE).
 */
size_t ephdc_workspace_bytes(const ephdc_params* prm, uint32_t max_Q);

/*
 * Creates a client session on the current HIP device (proposed method, client-side HE: the
 * client receives the encrypted model once and keeps it for many batches).  The session
 * holds the encrypted model as a device-resident evaluation-domain copy (Montgomery form;
 * it owns that copy and its transform tables):
 *   d_model_ct     device, uint32 [M][2][L][N], coefficient domain, model_words entries;
 *                  read during the call only
 *   d_galois_keys  device, layout of ephdc_keygen, gk_words entries (r > 1; else NULL)
 *   max_Q          largest batch of later calls
 *   d_workspace    device, ws_bytes bytes, 256-byte aligned, caller-owned and borrowed until
 *                  destroy (see ephdc_workspace_bytes); NULL for a session used only through
 *                  batches, the serving loop and ephdc_score_encrypted_static
 * Errors: EPHDC_ERR_BUFFER (a buffer shorter than its layout), EPHDC_ERR_UNSUPPORTED
 * (ciphertext primes outside [2^29, 2^30), N outside the device shapes), EPHDC_ERR_OOM.
 * The call is synchronous with respect to `stream`.
 */
ephdc_status ephdc_session_create(const ephdc_params* prm, const uint32_t* d_model_ct, size_t model_words,
                                  const uint32_t* d_galois_keys, size_t gk_words, uint32_t max_Q,
                                  void* d_workspace, size_t ws_bytes, void* stream, ephdc_session** out);
/* Waits for the session's last scoring call and frees it.  Batches and servers that use the
 * session must be destroyed first. */
ephdc_status ephdc_session_destroy(ephdc_session* s);
/* Device bytes the session owns (model copy, keys, tables; not the caller's workspace). */
size_t ephdc_session_device_bytes(const ephdc_session* s);

/*
 * HDC encoding (random projection + quantisation, Preliminary: HDC encoding):
 *   d_x     uint8 [Q][F] features, read as (x - 128)
 *   d_base  int8 [F][D] base hypervectors
 *   d_hv    out, int8 [D][ephdc_hv_stride(Q)] query hypervectors, dimension-major;
 *           entry [j][q] = sign or Q-bit quantisation of sum_f (x[q][f]-128)*base[f][j],
 *           and 0 for the padding queries q >= Q.
 * Requires F % 16 == 0, D % 64 == 0, F * D < 2^31 and Q * F < 2^31 (else
 * EPHDC_ERR_UNSUPPORTED).  int8 MFMA on gfx950.
 */
ephdc_status ephdc_encode_queries(ephdc_session* s, const uint8_t* d_x, const int8_t* d_base,
                                  uint32_t Q, int8_t* d_hv, void* stream);

/*
 * Homomorphic scoring of Q query hypervectors (d_hv as written by ephdc_encode_queries,
 * stride ephdc_hv_stride(Q); the padding columns q >= Q are taken as zero and not read)
 * against the encrypted model (proposed method, client-side HE:
 * batch encoding of every query element into its own plaintext, D ct x pt products per
 * batch): for every group g of B queries and every model ciphertext m, batch-encode the
 * query plaintext (slot scatter and inverse transform mod t, centred lift), multiply it
 * into ciphertext m and accumulate (with the scaling op of the parameters); when r > 1,
 * fold the r blocks with log2(r) rotate-and-sum steps (Galois automorphism and hybrid key
 * switching).
 *   d_score_ct  out, device, uint32 [G][2][L][N], coefficient domain: the client -> server
 *               message.
 * Q must be <= the session's max_Q.  Asynchronous on `stream`; the scratch comes from the
 * session's workspace, so a call on another stream than the session's previous call first
 * waits (on the device) for that call.  EPHDC_ERR_BUFFER when the session has no workspace.
 */
ephdc_status ephdc_score_encrypted(ephdc_session* s, const int8_t* d_hv, uint32_t Q,
                                   uint32_t* d_score_ct, void* stream);

/*
 * ephdc_score_encrypted for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same scoring, with its
 * scratch in a fixed 64 MiB array of the library's device code instead of the session's
 * workspace (one copy per GPU, held until the process ends; the session needs no
 * workspace).  Allocates nothing.  EPHDC_ERR_UNSUPPORTED, before any work is queued, when
 * this call's partial sums (current schedule), rotation workspace and one plaintext per
 * query group do not fit in 64 MiB (N = 8192, L = 4, default schedule: up to 227 groups).  Every
 * call on one GPU shares that GPU's array: calls that overlap on the device (from any
 * session or stream) race, so the caller orders them (one stream, or events).
 */
ephdc_status ephdc_score_encrypted_static(ephdc_session* s, const int8_t* d_hv, uint32_t Q,
                                          uint32_t* d_score_ct, void* stream);

/*
 * Debug: the lifted plaintext of query group g and model index m, reduced into every
 * limb, uint32 [L][N] coefficient domain (the centred representative of
 * Encode(slot vector) in (-t/2, t/2], mod q_l).  Exposes the batch-encoding step alone
 * (proposed method, client-side HE: every query element in its own plaintext, repeated
 * once per class; the plaintext encoding the paper times as EncPt).
 */
ephdc_status ephdc_debug_plaintext(ephdc_session* s, const int8_t* d_hv, uint32_t Q, uint32_t g,
                                   uint32_t m, uint32_t* d_out, void* stream);

/*
 * Debug: negacyclic products d_out[i] = d_a[i] * d_b[i] mod (X^N + 1, q_l), for `count`
 * polynomial pairs uint32 [count][N] with pair i taken mod q[i % L] of the session's
 * primes.  Runs the same forward / inverse transforms as the scoring path.
 */
ephdc_status ephdc_debug_polymul(ephdc_session* s, const uint32_t* d_a, const uint32_t* d_b,
                                 uint32_t count, uint32_t* d_out, void* stream);

/*
 * Schedule of the fused scoring kernel (0 keeps a setting):
 *   limb_group         limbs per work item, a divisor of L in 1..4
 *   blocks             target workgroups per launch (<= 1024): the model ciphertexts are
 *                      split into ranges until groups x ranges x limb groups reaches it
 *   values_per_thread  transform values held per thread (8 at N = 4096, 8 or 16 at
 *                      N = 8192, 16 or 32 at N = 16384; the workgroup has
 *                      N / values_per_thread threads)
 *   mode               1: one fused kernel batch-encodes and multiplies (the batch
 *                      encoding is repeated per limb group); 2: split path, a batch-encode
 *                      kernel writes each lifted plaintext once (into the plaintext chunk
 *                      of the session's workspace) and a MAC kernel reads it
 * Results do not depend on the schedule.  Defaults: split path, one limb per work item,
 * 8 values per thread (16 at N = 16384), 256 workgroups from N = 8192 up (one per compute
 * unit of an MI355X) and 512 below.
 */
ephdc_status ephdc_session_tune(ephdc_session* s, uint32_t limb_group, uint32_t blocks,
                                uint32_t values_per_thread, uint32_t mode);

/*
 * Bound (bytes) on the split path's plaintext chunk inside the workspace (0: all of it).
 * The model range is scored in chunks whose plaintexts fit it, each chunk's MAC adding into
 * the sums of the previous ones; a chunk always holds at least one plaintext per query
 * group of max_Q.  Results do not depend on it.
 */
ephdc_status ephdc_session_set_chunk_bytes(ephdc_session* s, size_t bytes);

/*
 * Kernel timing (diagnostics for benchmarks).  While enabled, every kernel launched by the
 * session is bracketed by HIP events recorded on the stream it runs on.  Reading waits for
 * the recorded events, returns per-stage totals and resets them:
 *   ms[0], count[0]  fused batch-encode + MAC kernel (k_score)
 *   ms[1], count[1]  partial-sum reduction + output inverse transform (k_finish)
 *   ms[2], count[2]  HDC encoding kernel (k_hdc_encode)
 *   ms[3], count[3]  rotate-and-sum kernels (automorphism, key switching)
 *   ms[4], count[4]  split path: batch-encode kernel (k_encode_pt)
 *   ms[5], count[5]  split path: MAC kernel (k_mac)
 */
ephdc_status ephdc_session_profile(ephdc_session* s, int enable);
ephdc_status ephdc_session_profile_read(ephdc_session* s, double ms[6], uint64_t count[6]);

/*
 * findDmax (EP-HDC design space exploration, Exploration Algorithm, procedure findDmax; the
 * noise study): the largest hypervector dimension whose encrypted ciphertext x plaintext
 * dot product still decrypts correctly, for `trials` independent trials.
 * Trial i uses seed + i for every stream: secret key (tag 4), model encryption (tag 5),
 * class values C [K][d_cap] (tag 8, draw m*K + c) and query values h [B][d_cap] (tag 9,
 * draw m*B + q); a value of b bits is 2*(u mod 2) - 1 for b = 1, else (u mod 2^b) - 2^(b-1),
 * with b = cbits for classes and qbits (of prm) for queries.  The class values are encrypted
 * as d_cap model ciphertexts (the paper's packing, r = 1, prm's scheme), the queries form
 * query group 0, and the D-term sum_{m<D} ct_m * p_m is correct when it decrypts to the
 * plaintext of the exact dot products mod t in every slot.  dmax[i] (host, int32 [trials])
 * is the number of D = 1, 2, ... that decrypt correctly before the first that does not
 * (d_cap when none fails).  Uses prm's N, L <= 2, q, t, K, qbits and scheme (r must be 1 and the layout contiguous;
 * F, D and the scaling op are ignored); the primes may be any above t (the noise budget is
 * set by Q), not only the scoring kernels' [2^29, 2^30).  Key generation and encryption run on the host; the
 * batch encoding, every prefix sum, its decryption and the comparison on the device, which
 * the call allocates for itself (about d_cap * N * (8L + 12) bytes).  Synchronous.
 */
ephdc_status ephdc_find_dmax(const ephdc_params* prm, uint64_t seed, uint32_t trials, uint32_t d_cap,
                             uint32_t cbits, int32_t* dmax, void* stream);

/* ---------------------------------------------------------------- detection front end
 * The paper's driving example (Our Proposed Method, applications: HDC-based object
 * detection): a window slides over an image frame left to right, row by row, and each
 * window's HOG feature map is one query of ephdc_encode_queries.  The HOG here is exact
 * integer arithmetic: central-difference gradients with replicated borders, floor(sqrt)
 * magnitudes, 9 unsigned orientation bins of 20 degrees (a gradient folded to the upper half
 * plane is in bin b = the number of k = 1..8 with C_k*gy - S_k*gx >= 0, C_k = round(2^14
 * cos(20k deg)), S_k = round(2^14 sin(20k deg))), 8 x 8-pixel cells, 2 x 2-cell blocks at a
 * stride of one cell whose 36 values v are L2-normalised with the clip at 0.2 scaled to byte
 * 255, min(255, floor(1275 v / n)) with n = floor(sqrt(sum v^2)) (0 when n is 0), and per
 * window its (w/8 - 1)^2 blocks in row order, padded with 128 (the encoder's zero point) to a
 * multiple of 16 features.
 */

/* Features per window (the F of the HDC parameters): (w/8 - 1)^2 * 36 rounded up to a
 * multiple of 16; 0 unless w is a multiple of 8 and >= 16. */
uint32_t ephdc_hog_feature_count(uint32_t window);

/* Windows of a frame: ((H - w)/stride + 1) * ((W - w)/stride + 1), 0 for an invalid shape
 * (w, stride multiples of 8, w >= 16, w <= H, W <= 65536). */
uint32_t ephdc_hog_window_count(uint32_t H, uint32_t W, uint32_t window, uint32_t stride);

/* Device workspace of ephdc_hog_windows for an H x W frame: cell histograms and blocks. */
size_t ephdc_hog_workspace_bytes(uint32_t H, uint32_t W);

/*
 * HOG features of every window of a frame:
 *   d_frame      device, uint8 [H][W] grey levels, row-major
 *   window, stride  window side and step in pixels (multiples of 8; window >= 16)
 *   d_workspace  device, ws_bytes >= ephdc_hog_workspace_bytes(H, W), 256-byte aligned
 *   d_x          out, device, uint8 [ephdc_hog_window_count][ephdc_hog_feature_count],
 *                4-byte aligned; window (i, j) (origin (i*stride, j*stride)) is row
 *                i * ((W - window)/stride + 1) + j
 * Asynchronous on `stream`.  EPHDC_ERR_ARG for an invalid shape or alignment,
 * EPHDC_ERR_BUFFER for a short workspace.
 */
ephdc_status ephdc_hog_windows(const uint8_t* d_frame, uint32_t H, uint32_t W, uint32_t window, uint32_t stride,
                               void* d_workspace, size_t ws_bytes, uint8_t* d_x, void* stream);

/* ---------------------------------------------------------------- request batches
 * Many clients' requests scored together (the client-side method's batch inference, which
 * the paper argues scales to many clients, applied across requests): every kernel stage of the scoring path runs as one
 * persistent launch over the work items (request, query group, model-ciphertext segment,
 * limb group) of all requests, so requests of 1 query and of thousands, and models of
 * different K, D and r, share the GPU in the same launches.  Requests whose sessions have
 * different N or ciphertext primes are scored by one launch sequence per parameter set.
 * The batched form computes exactly the per-request ciphertexts of ephdc_score_encrypted.
 */
typedef struct {
  ephdc_session* session;  /* the tenant: encrypted model, Galois keys, tables */
  const uint8_t* d_x;      /* [Q][F] features to HDC-encode first, or NULL when d_hv holds them */
  const int8_t* d_base;    /* [F][D] base hypervectors (read only with d_x) */
  int8_t* d_hv;            /* [D][ephdc_hv_stride(Q)] query hypervectors; with d_x the batch writes
                              columns [0, Q) (the padding columns are taken as zero and never read) */
  uint32_t Q;              /* 1 <= Q <= the session's max_Q */
  uint32_t* d_score_ct;    /* out: [G][2][L][N] score ciphertexts, coefficient domain */
} ephdc_request;

typedef struct ephdc_batch ephdc_batch;

/*
 * Plans a batch: validates every request, builds the work lists and uploads them, and
 * allocates the batch's device memory (partial sums, plaintext chunk buffer, rotation
 * workspace of folded requests).  The batch borrows the sessions and every buffer named by
 * the requests; the caller keeps them alive and unmodified in shape until destroy.
 * Errors: EPHDC_ERR_ARG (NULL, empty, Q out of range), EPHDC_ERR_UNSUPPORTED (sessions on
 * different devices, encoding constraints of ephdc_encode_queries), EPHDC_ERR_OOM.
 */
ephdc_status ephdc_batch_create(const ephdc_request* reqs, uint32_t n_req, ephdc_batch** out);
ephdc_status ephdc_batch_destroy(ephdc_batch* b);
size_t ephdc_batch_device_bytes(const ephdc_batch* b);

/*
 * Schedule of a batch, five values (0 keeps a setting; results never depend on it):
 *   [0] mode               1 fused (one persistent batch-encode + MAC launch), 2 split
 *                          (batch-encode launch + MAC launch per chunk of plaintexts)
 *   [1] values_per_thread  transform values per thread (as in ephdc_session_tune)
 *   [2] limb_group         limbs per MAC work item (1, 2 or 4, dividing L)
 *   [3] seg_len            model ciphertexts per work item
 *   [4] grid               workgroups of each persistent launch
 * A change drops a captured graph.  ephdc_batch_schedule reads the current values.
 */
ephdc_status ephdc_batch_tune(ephdc_batch* b, const uint32_t schedule[5]);
ephdc_status ephdc_batch_schedule(const ephdc_batch* b, uint32_t schedule[5]);

/*
 * Autotuner: times candidate schedules of this batch on `stream` (coordinate descent over
 * the five settings; each candidate is run once to warm up and timed over `reps` runs with
 * HIP events, right after the incumbent is timed the same way, and replaces it only when
 * at least 2 % faster) and keeps the fastest.  Writes its schedule and mean time per run.
 */
ephdc_status ephdc_batch_autotune(ephdc_batch* b, void* stream, uint32_t reps, uint32_t schedule[5],
                                  double* best_ms);

/* Enqueues the whole batch on `stream` (replays the captured graph if there is one). */
ephdc_status ephdc_batch_run(ephdc_batch* b, void* stream);

/*
 * Captures the batch's launches on `stream` (not the null stream) into a HIP graph; later
 * ephdc_batch_run calls replay it with one launch call.  The graph holds kernel nodes only.
 */
ephdc_status ephdc_batch_capture(ephdc_batch* b, void* stream);

/*
 * A packed batch: the requests of each session are placed one after another in one query
 * sequence, so requests of a few queries share ciphertexts instead of each filling (and
 * paying for) its own.  Every request must carry its features (d_x, d_base); its d_hv is
 * not used, and its d_score_ct must hold ephdc_num_groups(Q) + 1 ciphertexts.  Each run
 * writes to it the n_ct ciphertexts of the sequence that hold the request's queries, the
 * first query at position q_first of the first of them (read the scores with
 * ephdc_decrypt_scores_at(..., q_first, Q, ...)); query_offset is the request's first query
 * in its session's whole sequence.  Decrypted scores are those of the request alone; the
 * ciphertexts also carry the scores of the requests they are shared with.
 */
ephdc_status ephdc_batch_create_packed(const ephdc_request* reqs, uint32_t n_req, ephdc_batch** out);
ephdc_status ephdc_batch_packing(const ephdc_batch* b, uint32_t i, uint32_t* query_offset, uint32_t* q_first,
                                 uint32_t* n_ct);

/* Many requests' homomorphic scoring in one call (ephdc_score_encrypted per request, batched
 * as above): plan, run on `stream`, wait for it and free the plan. */
ephdc_status ephdc_score_many(const ephdc_request* reqs, uint32_t n_req, void* stream);

/* ---------------------------------------------------------------- serving loop
 * A server keeps tenants' sessions (device-resident encrypted models and Galois keys) and
 * scores requests as they arrive: a scheduler thread takes the waiting requests in arrival
 * order into a batch while the batch's device memory (query hypervectors, partial sums,
 * plaintext chunks, rotation workspace) fits the free part of the server's budget, and
 * launches it on a free stream; requests that arrive while batches run are admitted as
 * streams and memory free up, so their work overlaps on the device (continuous batching).
 * Each request's score ciphertexts equal those of ephdc_score_encrypted for it alone.
 */
typedef struct ephdc_server ephdc_server;

/*
 * budget_bytes  device memory for requests in flight (>= 64 MiB), allocated with the first
 *               tenant; a request that cannot fit even an empty budget is rejected
 * streams       batches in flight at once (1..8)
 * max_batch     requests per batch (0: 64)
 */
ephdc_status ephdc_server_create(size_t budget_bytes, uint32_t streams, uint32_t max_batch, ephdc_server** out);

/* Registers a tenant: its session and its base hypervectors d_base int8 [F][D] (device,
 * borrowed until the server is destroyed).  Every tenant lives on the first one's device. */
ephdc_status ephdc_server_add_tenant(ephdc_server* sv, ephdc_session* s, const int8_t* d_base, uint32_t* tenant);

/*
 * Queues a request: d_x uint8 [Q][F] features (device, 16-byte aligned, unchanged until the
 * request is done), out d_score_ct uint32 [G][2][L][N].  The request's kernels run after the
 * work queued on `stream` before this call (an event recorded there at submission), so d_x
 * may be written by kernels or copies still in flight on that stream.  Returns a ticket at
 * once.  Errors (synchronous): EPHDC_ERR_ARG (unknown tenant, Q outside [1, max_Q], NULL),
 * EPHDC_ERR_UNSUPPORTED (encoding constraints), EPHDC_ERR_HIP (the scheduler could not
 * start on the tenants' device).
 */
ephdc_status ephdc_server_submit(ephdc_server* sv, uint32_t tenant, const uint8_t* d_x, uint32_t Q,
                                 uint32_t* d_score_ct, void* stream, uint64_t* ticket);

/* State of a ticket: 0 waiting, 1 in flight, 2 done, -status when it failed or was rejected
 * (-EPHDC_ERR_OOM: larger than the budget); times[3] = submit, admit, done in seconds since
 * the server was created (0 when not reached).  A finished ticket is kept until released
 * (ephdc_server_release); beyond 65536 finished tickets the oldest are forgotten, and calls
 * that name a released or forgotten ticket return EPHDC_ERR_ARG. */
ephdc_status ephdc_server_query(ephdc_server* sv, uint64_t ticket, int32_t* state, double times[3]);

/* Waits until the ticket is done (ticket 0: until nothing waits or runs); timeout_s <= 0
 * waits without limit.  Returns the request's failure status if it failed, and
 * EPHDC_ERR_TIMEOUT when the time limit passes first. */
ephdc_status ephdc_server_wait(ephdc_server* sv, uint64_t ticket, double timeout_s);

/* Forgets a finished ticket (done, failed or rejected); EPHDC_ERR_ARG while it waits or runs. */
ephdc_status ephdc_server_release(ephdc_server* sv, uint64_t ticket);

/* Counters: [0] submitted [1] completed [2] rejected [3] waiting [4] batches in flight
 * [5] batches launched [6] mean requests per batch [7] p50 latency ms [8] p99 latency ms
 * (submit to done, completed requests, from a histogram of 1 % wide bins) [9] peak device
 * bytes in use [10] budget bytes [11] seconds since creation [12] failed (a launch or the
 * device reported an error) [13] tickets the server holds (waiting, running, finished and
 * not yet released). */
ephdc_status ephdc_server_stats(ephdc_server* sv, double out[14]);

/*
 * Packing (set before the first request): the requests of one tenant in a batch share
 * ciphertexts -- their queries are placed one after another in one query sequence, so a
 * ciphertext's B query positions serve several requests.  A request's d_score_ct must then
 * hold ephdc_num_groups(Q) + 1 ciphertexts; it receives the n_ct ciphertexts of the sequence
 * that hold its queries, the first of them at position q_first (ephdc_server_result), to be
 * read with ephdc_decrypt_scores_at(..., q_first, Q, ...).  Decrypted scores are those of
 * the request alone; the ciphertexts also carry the other requests' scores.
 */
ephdc_status ephdc_server_set_packing(ephdc_server* sv, int enable);

/* Where a done request's scores sit: q_first and the number of ciphertexts written
 * (without packing q_first = 0 and n_ct = ephdc_num_groups(Q)). */
ephdc_status ephdc_server_result(ephdc_server* sv, uint64_t ticket, uint32_t* q_first, uint32_t* n_ct);

/* Drains the queue and every batch in flight, then frees the server (not the tenants). */
ephdc_status ephdc_server_destroy(ephdc_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* EPHDC_H */

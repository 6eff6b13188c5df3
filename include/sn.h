/*
 * sn.h -- C ABI of libsn, an MI355X (gfx950) library that evaluates the
 * energy, forces and virial of a periodic atomic configuration under a
 * NequIP-architecture graph-neural-network interatomic potential (SevenNet,
 * arXiv 2402.03789).
 *
 * What is computed (paper section 2): atomic numbers and positions in,
 * E = sum_i E_i (eq 1) and F_i = -dE/dr_i (eq 2) out, plus the virial
 * W = -sum_e d_e (x) dE/dd_e (stress support, section 3.2).  Units: eV and
 * angstrom.  The evaluation runs as one subdomain with a ghost shell of width
 * r_c (section 3.1): ghost positions come from their owners plus an image
 * shift, ghost node features are refreshed from their owners before every
 * interaction block after the first, and ghost gradients and partial forces
 * are folded back to the owners in the backward pass.
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status: SN_OK (0) or a negative code.
 *     No exception crosses the ABI.  On error the outputs are unspecified;
 *     the context stays usable except after SN_EHIP.
 *   - The caller owns every input and output buffer.  The library owns the
 *     model, contexts, servers and all device scratch, released by *_free.
 *   - A model is read-only after loading and may be shared by contexts.  A
 *     context is used by one host thread at a time.
 *   - Arrays are row-major.  Positions are n x 3 float64 (angstrom); the
 *     cell is 3 x 3 float64 whose rows are the lattice vectors a1, a2, a3.
 *   - Results are bitwise reproducible for the same input, precision and
 *     build (no floating-point atomics anywhere).
 */
#ifndef SN_H_
#define SN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------------- */
#define SN_OK 0
#define SN_EINVAL (-1)        /* bad argument: shape, NaN/Inf, singular cell, unknown Z, r = 0 pair */
#define SN_ENOMEM (-2)        /* device memory or HBM budget exhausted */
#define SN_EHIP (-3)          /* HIP runtime error, including a kernel launch the runtime
                                 refused; the context is no longer usable */
#define SN_EUNSUPPORTED (-4)  /* valid request that the library does not implement */
#define SN_EBUSY (-5)         /* resource in use (e.g. backward without a pending forward) */

/* ---- precision forms -------------------------------------------------------------- */
#define SN_FP64 0  /* everything in float64 (reference-grade; for tests and finite differences) */
#define SN_FP32 1  /* per-edge work in float32 (basis, radial MLP, tensor product, edge
                      gradients; the forward radial MLP's output layer as sums of products of
                      three-part bfloat16 splits of its float32 operands, float32-level
                      error), edge vectors from float64 positions; the node-state chain
                      (features, self-connection, gate, readout input) in float64, its
                      float64 contractions on the float64 matrix cores; node gradients of
                      the adjoint in float32; energy and virial reductions in float64 */
#define SN_BF16 2  /* as SN_FP32, but the radial MLP and the channel-mixing linears take
                      bfloat16 operands with float32 accumulation on the matrix cores; sender
                      features, radial weights, messages and per-edge gradients stored in
                      bfloat16;
                      tensor product in float32; node-state chain in float32; float64
                      positions, edge gradients, forces, energy and virial reductions */

typedef struct sn_model sn_model_t;
typedef struct sn_ctx sn_ctx_t;

typedef struct sn_model_info {
  int n_layers;      /* interaction blocks T */
  int l_max;         /* highest feature degree */
  int l_sh;          /* highest edge spherical-harmonic degree */
  int muls[4];       /* channels per degree l = 0..3 (0 when absent) */
  int n_basis;       /* radial Bessel functions */
  int hidden;        /* radial-MLP hidden width */
  int n_species;     /* rows of the embedding */
  int species_z[128];/* atomic number of each embedding row */
  double r_cut;      /* cutoff radius, angstrom */
  double k_avg;      /* message normalisation (average neighbour count) */
  double sigma;      /* per-atom energy scale */
  int64_t n_params;  /* number of model parameters */
} sn_model_info_t;

/* Text of a status code (static storage). */
const char* sn_strerror(int status);

/* Most recent error message of a context, or of the last failed model load when
 * ctx is NULL (thread-local storage for the latter).  Never NULL. */
const char* sn_last_error(const sn_ctx_t* ctx);

/* ---- model --------------------------------------------------------------------------
 * sn_model_load reads a weights file: 8-byte magic "SNW1\0\0\0\0", little-endian
 * u64 header length, JSON header {"format":"snw1","config":{...},"tensors":[{name,
 * shape,offset}]}, padding, then float64 tensors.  The configuration holds the
 * block count, channels per degree, l_sh, r_cut, species list, k_avg, sigma,
 * per-species shift and activation scale.  Tensor shapes are checked against the
 * architecture derived from the configuration (section 5.1: linear
 * self-connection, scalar-only last block).  SN_EINVAL on a malformed file. */
int sn_model_load(const char* path, sn_model_t** out);
void sn_model_free(sn_model_t* model);
int sn_model_info(const sn_model_t* model, sn_model_info_t* info);

/* Real Clebsch-Gordan table used by the kernels for the coupling (l1, l2) -> l3
 * (l <= 3), written densely into out[(2l1+1)(2l2+1)(2l3+1)] in row-major
 * (m1, m2, m3) order.  Needs no device.  SN_EINVAL for an invalid triple. */
int sn_cg_table(int l1, int l2, int l3, double* out);

/* ---- context ------------------------------------------------------------------------
 * A context binds a model to one device, one HIP stream (NULL = the null stream)
 * and one precision form, and owns the device workspace.  hbm_budget caps the
 * workspace in bytes (0 = no cap beyond the device); a request that would exceed
 * it fails with SN_ENOMEM before any launch.  skin widens the ghost shell to
 * r_cut + skin (paper section 3.1: the shell that holds every sender within reach of a
 * subdomain's receivers) so that a neighbour list can be reused while atoms move less
 * than skin / 2 (0 for a fresh list every call).
 *
 * alloc (may be NULL) supplies every device allocation of the context -- weights and
 * workspace -- so that a framework can serve them from its own pool (the Python layer
 * binds torch's caching allocator).  NULL uses hipMalloc / hipFree.  The library calls
 * alloc(user, bytes, device, stream) with the context's device current and its stream;
 * it must return memory aligned to at least 256 bytes and valid on that device, or NULL
 * on failure (the call then fails with SN_ENOMEM).  free(user, ptr, bytes, device,
 * stream) is called only after every use of ptr on the context's streams has completed
 * (the library synchronises those streams first), and for every block at sn_ctx_free.
 * The allocator must outlive the context and may be called from the host thread that
 * makes the library call. */
typedef struct sn_allocator {
  void* (*alloc)(void* user, size_t bytes, int device, void* hip_stream);
  void (*free)(void* user, void* ptr, size_t bytes, int device, void* hip_stream);
  void* user;
} sn_allocator_t;

int sn_ctx_create(const sn_model_t* model, int device, void* hip_stream, size_t hbm_budget,
                  int precision, double skin, const sn_allocator_t* alloc, sn_ctx_t** out);
/* A context also owns a second HIP stream on which the radial MLPs of every block run,
 * overlapped with the node-feature chain (the MLP forward needs only the edge basis; the
 * MLP adjoint of a block only that block's dE/dw).  Every call joins that stream back into
 * the context's stream before it returns, so the entry points stay stream-ordered.  With
 * SN_SERIAL=1 in the environment at creation, everything runs on the context's stream
 * (per-kernel timings without overlap, for profiling). */
void sn_ctx_free(sn_ctx_t* ctx);

/* ---- single structure, host buffers -------------------------------------------------
 * One evaluation of the potential (paper section 2: atomic numbers and positions in; the
 * per-atom energies E_i whose sum is E, eq 1; the forces F_i = -dE/dr_i, eq 2, assembled
 * from the edge gradients by eqs 5-6; the virial for the stress of section 3.2), run as
 * one subdomain with its ghost shell (section 3.1).
 * n atoms; pos[n*3] angstrom; Z[n] atomic numbers known to the model; cell[9]
 * rows a1 a2 a3; pbc[3] must all be nonzero (periodic in every direction; other
 * cases return SN_EUNSUPPORTED).  Outputs (any may be NULL except energy):
 * energy[1] eV; atom_energy[n] eV; forces[n*3] eV/angstrom; virial[9] eV,
 * W = -sum_e d_e (x) dE/dd_e (stress = -W / volume).  Blocks until done.  The inputs are
 * copied to device memory and the results back (two PCIe transfers beside the device
 * entry points below).  SN_EINVAL for an unknown atomic number, non-finite positions, a
 * singular cell or two atoms at one position; SN_ENOMEM when the workspace would exceed
 * the budget (the context stays usable). */
int sn_compute(sn_ctx_t* ctx, int64_t n, const double* pos, const int32_t* Z, const double* cell,
               const uint8_t* pbc, double* energy, double* atom_energy, double* forces,
               double* virial);

/* ---- the same evaluation without allocating device memory ------------------------
 * For callers that cannot allocate device memory (code around HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): sn_compute with the same arguments,
 * outputs and errors, whose every device buffer is a slice of a fixed array of 512 MiB
 * that the library holds per device (allocated with the library's code object and kept
 * until the process ends).  The call allocates and frees nothing on the device; it always
 * builds its own graph and keeps no state after it returns (a later sn_ctx_graph sees no
 * graph).  A structure whose workspace does not fit the array fails with SN_ENOMEM and a
 * message naming the size (the context stays usable; roughly 500 atoms of the five-block
 * l <= 2 model of section 5.1 fit).  The array is shared by every context and thread on a
 * device and keeps the last call's contents: calls that overlap on one device (other
 * threads, other contexts' streams) race and must be serialised by the caller.
 * Blocks until done. */
int sn_compute_noalloc(sn_ctx_t* ctx, int64_t n, const double* pos, const int32_t* Z,
                       const double* cell, const uint8_t* pbc, double* energy,
                       double* atom_energy, double* forces, double* virial);

/* ---- several structures in one packed graph, host buffers --------------------------
 * The evaluation of sn_compute (paper section 2, eqs 1-2, 5-6) for a batch: the graph of
 * section 3.1 built once over all structures, with edges inside each structure only.
 * B structures; offsets[B+1] (offsets[0] = 0) delimit each structure's atoms in pos[n*3]
 * and Z[n] (n = offsets[B]); cells[B*9] holds each structure's cell (all periodic).  The
 * structures are evaluated together as one graph (the kernels run once over all atoms
 * and edges; edges never cross structures) and the results are exactly those of
 * evaluating each structure alone, up to floating-point summation order.  Outputs:
 * energies[B]; atom_energies[n], forces[n*3], virials[B*9] (each may be NULL). */
int sn_compute_batch(sn_ctx_t* ctx, int B, const int64_t* offsets, const double* pos,
                     const int32_t* Z, const double* cells, double* energies,
                     double* atom_energies, double* forces, double* virials);

/* ---- device buffers, stream-ordered (the autograd pair) -----------------------------
 * One packed batch of B periodic structures resident in device memory.  The atoms of
 * structure b are offsets[b] .. offsets[b+1]-1 of d_pos (n x 3 float64, angstrom) and
 * d_Z (n int32 atomic numbers), n = offsets[B]; offsets (B+1 int64, offsets[0] = 0,
 * strictly increasing) and cells (B x 9 float64, rows a1 a2 a3 of each cell) are host
 * arrays read during the call.  The caller owns every buffer. */
typedef struct sn_batch {
  int32_t n_structures;    /* B >= 1 */
  const int64_t* offsets;  /* host, B + 1 */
  const double* cells;     /* host, B x 9 */
  const double* d_pos;     /* device, n x 3 */
  const int32_t* d_Z;      /* device, n */
} sn_batch_t;

/* sn_forward_device evaluates the energy of every structure of the batch as one packed
 * graph (paper Fig 3a: graph build, edge basis, the interaction blocks of section 2.2 with
 * the per-block ghost refresh of section 3.1, readout and E_b = sum of E_i over the
 * structure's atoms, eq 1, in float64) and keeps the activations the backward pass needs
 * inside ctx (one pending forward per context).  Outputs (device, float64): d_energy[B];
 * d_atom_energy[n] (may be NULL).  sn_backward_device consumes the pending forward with
 * the upstream gradients d_grad_energy[B] = dL/dE_b (device, float64, read when the work
 * runs) and writes the position gradients through the hand-written adjoint (eqs 5-8:
 * edge gradients dE/dd_e summed over blocks, the sender-side sums and ghost folds of the
 * reverse communication, F = -dE/dr by eq 6):
 *   d_forces[i]  = g_b F_i = -dL/dr_i   for the atoms i of structure b (n x 3, device);
 *   d_virial[b]  = g_b W_b, W_b = -sum_e d_e (x) dE_b/dd_e (B x 9, device, may be NULL).
 * Both return once the work is queued on the context's stream (no host synchronisation
 * after the graph build).  SN_EINVAL for a malformed batch, an atomic number outside the
 * model or non-finite positions (checked before the kernels that depend on them);
 * SN_EBUSY for a backward without a pending forward. */
int sn_forward_device(sn_ctx_t* ctx, const sn_batch_t* batch, double* d_energy,
                      double* d_atom_energy);
int sn_backward_device(sn_ctx_t* ctx, const double* d_grad_energy, double* d_forces,
                       double* d_virial);

/* ---- training: weight gradients of the energy term of the loss ----------------------
 * Paper section 5.1 trains with the loss of eq 9: a Huber loss of per-atom energies, forces
 * and stresses.  sn_backward_train_device gives the exact weight gradient of any linear
 * function of the energies (the energy term); sn_train_loss_grad gives the gradient of the
 * whole loss.
 *
 * sn_ctx_set_training(ctx, 1): later forwards keep every interaction block's input features
 * and messages (about (Dx + Dm) float64/float32 values per atom and block more device
 * memory), which the weight gradients need.  Graph replay is off while it is set. */
int sn_ctx_set_training(sn_ctx_t* ctx, int on);

/* Consumes a pending training-mode forward (SN_EBUSY otherwise).  With the upstream
 * gradients d_grad_energy[B] = dL/dE_b (device, float64) it writes
 *   d_weight_grad = sum_b g_b dE_b/dW for every weight W (device, float64), sn_model_info's
 *     n_params values laid out as the weights file's tensors (offsets from sn_model_tensor):
 *     embedding, every block's Lin1, self-connection, radial MLP (Wa, Wb, Wc) and Lin2, and
 *     the readout;
 *   d_forces, d_virial as sn_backward_device (each may be NULL).
 * The radial MLP's adjoint runs unfused here (its hidden activations and pre-activation
 * gradients are needed per pair), so forces agree with sn_backward_device to rounding, not
 * bit for bit.  Every weight gradient is a fixed-order float64 reduction over atoms or edge
 * pairs: bitwise reproducible.  SN_EUNSUPPORTED for a weights file with gaps. */
int sn_backward_train_device(sn_ctx_t* ctx, const double* d_grad_energy, double* d_forces,
                             double* d_virial, double* d_weight_grad);

/* Gradient of the whole loss of eq 9 for one packed batch (blocking; host labels):
 *   Gamma = (1/M) sum_b huber(E_b/N_b - refE_b/N_b)
 *         + mu_f / (3 M N) sum_{b,j,k} huber(F_bjk - refF_bjk)        (N: atoms of the batch)
 *         + mu_s / (6 M) sum_{b,l} huber(S_bl - refS_bl)
 * with S = -W / V in GPa from the symmetrised virial (components xx yy zz yz xz xy).
 * ref_energy[B] eV, ref_forces[n*3] eV/angstrom (batch order), ref_stress[B*6] GPa (host).
 * Writes *loss and d_weight_grad (device, n_params float64, layout as sn_backward_train_device).
 * The energy term's weight gradient is the exact adjoint.  The force and stress terms are
 * second derivatives: with v_i = dGamma/dF_i and the symmetric U_b = dGamma/dW_b, and since
 * F = -dE/dr and W_ab = -dE/de_ab for a strain e, their weight gradient is minus the weight
 * gradient of the derivative of E along the deformation r -> r + eps (v + U r), cell rows
 * a -> a + eps U a.  That is taken as a four-point central difference of exact weight
 * gradients at eps = +-h, +-2h (error O(h^4)), h chosen so the largest displacement is
 * fd_step angstrom (0: 1e-3 in the FP64 form, 2e-2 otherwise).  Costs six evaluations with
 * adjoints; with mu_f = mu_s = 0 the difference quotient is skipped (the energy term alone).
 * SN_EINVAL for a malformed batch, delta <= 0 or negative weights. */
int sn_train_loss_grad(sn_ctx_t* ctx, const sn_batch_t* batch, const double* ref_energy,
                       const double* ref_forces, const double* ref_stress, double delta,
                       double mu_f, double mu_s, double fd_step, double* loss,
                       double* d_weight_grad);

/* Name, offset (in float64 values from the start of the weights) and element count of the
 * index-th tensor of the model (tensors in name order).  SN_EINVAL past the last one.  The
 * name points into the model and lives as long as it. */
int sn_model_tensor(const sn_model_t* model, int index, const char** name, int64_t* offset,
                    int64_t* count);

/* Energy term of eq 9 on host arrays: loss = (1/B) sum_b huber(E_b/N_b - ref_b/N_b; delta),
 * huber(r) = r^2/2 for |r| < delta, delta (|r| - delta/2) otherwise (squared error below the
 * threshold, absolute error above; the paper takes delta = 0.01), and dloss_denergy[b] =
 * dloss/dE_b (may be NULL).  SN_EINVAL for B < 1, a structure without atoms or delta <= 0. */
int sn_huber_energy_loss(int B, const double* energy, const double* ref, const int64_t* natoms,
                         double delta, double* loss, double* dloss_denergy);

/* Neighbour-list reuse for molecular dynamics.  With reuse enabled, a forward call whose
 * atom count and cell equal those of the previous build keeps that graph (ghost shell and
 * edges out to r_cut + skin) and only refreshes local and ghost positions from d_pos; the
 * caller guarantees that no atom moved more than skin / 2 since the last build, and disables
 * reuse for the call that should rebuild.  Results equal a fresh build because the envelope
 * and its derivative vanish beyond r_cut. */
int sn_ctx_set_graph_reuse(sn_ctx_t* ctx, int reuse);

/* Evaluation of lists built with a skin (default on).  A list built out to r_cut + skin
 * also holds pairs farther apart than r_cut, whose contributions the envelope makes exact
 * zeros (paper section 5.1: the cutoff function and its derivative vanish at r_cut).  With
 * compaction on, every forward call (the build and each later call that keeps the list)
 * first compacts the list on the device to the pairs inside r_cut at the current
 * positions (both edges of a pair together, order preserved) and evaluates only those.
 * Results equal those of the whole list up to the grouping of floating-point sums (a
 * degree narrower than a wave deals a receiver's edges to lane groups by position, and
 * reductions are chunked by list length); they stay deterministic, and a structure's
 * result is the same alone and in a batch.  Not combined with graph replay
 * (sn_ctx_set_capture on at the build turns it off for that list).  The setting takes
 * effect at the next list build; a kept list goes on as it was built. */
int sn_ctx_set_edge_compaction(sn_ctx_t* ctx, int on);

/* Spatial decomposition on one device (paper section 3.1, Fig 3): split every structure of
 * later calls into nx x ny x nz subdomains, the fractional boxes [i/nx, (i+1)/nx) x ... of its
 * cell.  Each subdomain owns the atoms inside its box and gets its own ghost shell of width
 * r_cut + skin; a ghost's owner is a local atom of any subdomain (a shift-0 image when the
 * owner lies in a neighbouring subdomain), so the per-block ghost refresh and the backward
 * ghost fold are the halo exchanges of the multi-device method, carried out in device
 * memory.  Edges never cross subdomains.  Results equal the undivided evaluation up to the
 * order of floating-point sums.  1 x 1 x 1 (the default) is one subdomain per structure.
 * SN_EINVAL for a count below 1 or more than 4096 subdomains. */
int sn_ctx_set_domains(sn_ctx_t* ctx, int nx, int ny, int nz);

/* hipGraph replay for molecular dynamics.  With capture on and graph reuse enabled, a
 * forward/backward pair that reuses the kept neighbour list is recorded once into a HIP
 * graph (all launches on one stream, no timing events) and replayed on later reuse calls
 * with the same device pointers (the upstream gradients are read from device memory at
 * replay, so their values may change); a rebuild or other pointers record a new graph.  The first reuse call after a build runs eagerly (it sizes
 * the workspace).  Results are bitwise those of the eager launches. */
int sn_ctx_set_capture(sn_ctx_t* ctx, int on);

/* Velocity-Verlet half step on device arrays (harness of the MD workload: the 1 fs
 * velocity-Verlet runs of the large-box section 5.2 and the benchmarks of section 4),
 * stream-ordered:
 * stage 0: v += dt/2 a, x += dt v;  stage 1: v += dt/2 a;  a = F * inv_mass.
 * d_pos, d_vel, d_forces are n x 3 float64; d_inv_mass[n] carries the unit conversion
 * (for eV, angstrom, amu and fs: 0.0096485 / mass). */
int sn_md_verlet(sn_ctx_t* ctx, int64_t n, double* d_pos, double* d_vel, const double* d_forces,
                 const double* d_inv_mass, double dt, int stage);

/* Nose-Hoover thermostat for the NVT runs of the paper's MD benchmarks (section 4: NVT
 * ensemble with the Nose-Hoover thermostat).  One thermostat on all particles:
 *   dv/dt = a - xi v,  dxi/dt = (2K - dof kT) / Q,  deta/dt = xi,
 * K = sum m v^2 / 2.  This call applies the half-step operator of the symmetric Trotter
 * splitting  NH(dt/2) . Verlet(dt) . NH(dt/2):
 *   xi += dt/4 G(K);  eta += dt/2 xi;  v *= exp(-xi dt/2);  xi += dt/4 G(K'),
 * G(K) = (2K - dof kT)/Q, K' = K exp(-xi dt) the kinetic energy after scaling.  Stream-ordered,
 * no host synchronisation.  d_vel: n x 3 float64 (angstrom/fs); d_inv_mass[n] as for
 * sn_md_verlet (its reciprocal is the mass in eV fs^2 / angstrom^2, so K is in eV);
 * kT in eV, dof the number of thermostatted degrees of freedom, Q > 0 in eV fs^2;
 * d_state: 4 float64 in device memory owned by the caller, {xi (1/fs), eta, last scale
 * factor, K after the call (eV)}, zero-initialised before the first call.  The conserved
 * quantity is K + U + Q xi^2 / 2 + dof kT eta.  SN_EINVAL for n < 1, dt, kT or dof not
 * positive, Q not positive or null pointers. */
int sn_md_nh_half(sn_ctx_t* ctx, int64_t n, double* d_vel, const double* d_inv_mass, double dt,
                  double kT, double dof, double Q, double* d_state);

/* Largest displacement since the last neighbour-list build, for a skin-triggered rebuild:
 * *max_disp (host, angstrom) = max_i |d_pos_i - d_ref_i| over the n x 3 float64 device arrays
 * (unwrapped positions and the positions at the last build).  Synchronises the context's
 * stream.  SN_EINVAL for n < 1 or null pointers. */
int sn_md_max_displacement(sn_ctx_t* ctx, int64_t n, const double* d_pos, const double* d_ref,
                           double* max_disp);

/* Wait for every queued operation of the context. */
int sn_ctx_synchronize(sn_ctx_t* ctx);

/* ---- serving: continuous batching of structures of uneven size --------------------
 * Inference serving of the general-purpose potential (paper section 5: one model over
 * many chemistries and cell shapes), each request one evaluation as in sn_compute.
 * A server runs n_streams worker threads on one device, each with its own HIP stream and
 * context (sharing the model).  Requests enter a FIFO queue; a free worker packs requests
 * from the head of the queue into one graph while the batch stays within
 * max_batch_atoms, max_batch_structures and its slice (hbm_budget / n_streams; 0 = no
 * cap) of the HBM budget, judged from the device bytes per atom measured on earlier
 * batches, and evaluates energy, forces and virial of every structure in the batch.
 * Requests that arrive while batches run join the next batch of the first worker to free
 * up, so the batches of different workers overlap on the device.  A batch that exceeds
 * the budget anyway is split and retried; a structure that cannot fit alone completes with
 * SN_ENOMEM.  Each structure's result is that of evaluating it alone (sn_compute_batch).
 *
 * Request buffers: pos, Z, cell are copied at submit.  atom_energy[n] and forces[n*3]
 * (either may be NULL) are written by the library and must stay valid until the request's
 * result has been returned by sn_server_poll.  Times are seconds since server creation. */
typedef struct sn_server sn_server_t;

typedef struct sn_request {
  int64_t n;              /* atoms */
  const double* pos;      /* n x 3, angstrom */
  const int32_t* Z;       /* n atomic numbers */
  const double* cell;     /* 3 x 3, rows a1 a2 a3 (periodic in all directions) */
  double* atom_energy;    /* out: n, eV (may be NULL) */
  double* forces;         /* out: n x 3, eV/angstrom (may be NULL) */
} sn_request_t;

typedef struct sn_result {
  uint64_t ticket;        /* as returned by sn_server_submit */
  int status;             /* SN_OK or the error of the batch the request ran in */
  int batch_structures;   /* structures packed into the request's batch */
  int64_t batch_atoms;    /* atoms of that batch */
  double energy;          /* eV */
  double virial[9];       /* eV */
  double t_submit, t_start, t_done;  /* submit, batch launch and completion times */
} sn_result_t;

int sn_server_create(const sn_model_t* model, int device, int n_streams, int precision,
                     size_t hbm_budget, int64_t max_batch_atoms, int max_batch_structures,
                     sn_server_t** out);
/* Queue one structure; *ticket identifies its result.  The request is checked here:
 * SN_EINVAL for an atomic number outside the model, non-finite positions or cell, or a
 * singular cell, so that a bad request cannot fail its batch mates.  A batch that fails on
 * what only the device finds (two atoms at one position) is re-run one structure at a time,
 * and only the offending request completes with the error.  SN_EHIP when no worker is
 * alive. */
int sn_server_submit(sn_server_t* server, const sn_request_t* request, uint64_t* ticket);
/* Evaluate one request once on every worker, in parallel, and return when all are done
 * (the results are dropped): each worker's workspace is then sized for a structure of
 * that size and its kernels are loaded, so the first requests of a stream do not pay for
 * either.  Checked as at submit (SN_EINVAL); SN_EBUSY while another warm-up runs; the
 * first worker's error otherwise (SN_EHIP when no worker is alive).  Queued requests
 * wait behind the warm-up of the worker that takes them. */
int sn_server_warmup(sn_server_t* server, const sn_request_t* request);
/* Move up to max finished results into out[]; *n_out receives the count.  Waits up to
 * timeout_ms for the first one (0: do not wait, negative: wait without limit). */
int sn_server_poll(sn_server_t* server, sn_result_t* out, int max, int timeout_ms, int* n_out);
/* Requests waiting in the queue and requests inside running batches. */
int sn_server_pending(sn_server_t* server, int64_t* queued, int64_t* running);
/* Stop the workers after their current batches and release everything; requests still
 * queued are dropped without a result. */
void sn_server_free(sn_server_t* server);

/* ---- inspection (tests and benchmarks) ---------------------------------------------
 * After a compute/forward, the graph sizes: local atoms, ghosts, directed edges of the
 * built list (out to r_cut + skin). */
int sn_ctx_graph_size(const sn_ctx_t* ctx, int64_t* n_local, int64_t* n_ghost, int64_t* n_edge);

/* Directed edges and undirected pairs the last forward evaluated (the built list, or its
 * compaction to the pairs inside r_cut; see sn_ctx_set_edge_compaction). */
int sn_ctx_evaluated_edges(const sn_ctx_t* ctx, int64_t* n_edge, int64_t* n_pair);

/* Undirected edge pairs of the last evaluated graph (the radial MLP runs once per pair). */
int sn_ctx_pair_count(const sn_ctx_t* ctx, int64_t* n_pairs);

/* Device bytes currently held by the context's workspace and weights. */
int sn_ctx_memory(const sn_ctx_t* ctx, size_t* bytes);

/* The last built graph in the caller's atom order: recv[E], send_owner[E] (owner atom of
 * the sender), shift[E*3] (integer image shift of the sender), and ghost_owner[G],
 * ghost_shift[G*3].  Host buffers sized from sn_ctx_graph_size; any may be NULL. */
int sn_ctx_graph(const sn_ctx_t* ctx, int32_t* recv, int32_t* send_owner, int32_t* shift,
                 int32_t* ghost_owner, int32_t* ghost_shift);

/* Per-kernel timing of the last compute (milliseconds, HIP events on the context
 * stream): names[k] and ms[k] for k < *count (count in: capacity, out: used). */
int sn_ctx_timings(const sn_ctx_t* ctx, const char** names, double* ms, int* count);

#ifdef __cplusplus
}
#endif
#endif /* SN_H_ */

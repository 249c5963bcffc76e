// Internal declarations shared by the host side and the kernels of
// libpmutdg.  Not part of the public ABI (see include/pmutdg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace pmdg {

// Sets the thread-local message returned by pmdg_last_error().
void set_last_error(const std::string& m);

constexpr int kMaxOrder = 8;                // polynomial order N <= 8
constexpr int kMaxNq = kMaxOrder + 1;       // Gauss points per direction on Gamma_I
constexpr int kMaxModes = 16;               // modes per PMUT
constexpr int kWaves = 4;                   // waves per workgroup

// Field arrays and operator tables of one brick, as seen by the kernels.
template <typename Real>
struct DomView {
  int nn[3];          // nodes per axis
  int N;              // order
  int px;             // padded row pitch (nn[0] rounded up to a multiple of 64)
  long plane;         // px * nn[1]  (device plane stride)
  long nnodes;        // plane * nn[2] (device nodes per scenario)
  Real* P[3];         // [S][nnodes] pressure; p^n is P[n % nbuf]
  int nbuf;           // 2 (FP64 two-level form, in place) or 3 (FP32 increment form)
  Real* X;            // [2][S][nnodes] increment p^n - p^{n-1} (increment form only);
  long xstride;       //   the live copy is X + (*xsel) * xstride (the two-step
  const int* xsel;    //   update reads one copy and writes the other)
};

// Prefetch distances beyond two planes are built for orders up to 4 and
// 4-wave tiles of 1 or 2 rows per wave.
__host__ __device__ constexpr bool deep_prefetch_built(int N, int rows, int waves) {
  return N <= 4 && waves == 4 && (rows == 1 || rows == 2);
}

// Stiffness + update kernel arguments (one brick).
template <typename Real>
struct StiffArgs {
  DomView<Real> d;
  int S;
  Real dt2;                 // dt^2
  const long* counter;      // steps completed (read only here)
  long* cnt_snap;           // or null: tile 0 copies the step counter here (read by a face kernel
                            // that runs alongside the interface kernel, which advances the counter)
  // PMUT face force on the primary's bottom plane: [S][nn0*nn1], or null
  const Real* force;
  // interface residual per face of Gamma_I: [S][nface][(N+1)^2][2] or null
  const Real* iface;
  int iface_side;           // +1: top element layer (fine side); -1: bottom layer (coarse side)
  int iface_nex, iface_ney; // faces per axis on Gamma_I for this brick
  Real iface_d[kMaxOrder + 1]; // c^2 (2/h_z) l_c'(+-1)
  // operator rows by node class along each axis: class a < N is an
  // interior node with i mod N = a, class N the first and N+1 the last node
  // of the line, class N+2 an all-zero row (outside the brick).
  const Real* taps;         // [3][N+3][2N]: -dt^2 c^2 (M_d^{-1} K_d) off-centre entries
  const Real* mins;         // [3][N+3]: inverse assembled 1D lumped mass
  const Real* absg;         // [3][N+3]: dt c / m_d on the end classes of absorbing faces, else 0
  int absorb;               // the brick has absorbing faces (absg not all zero)
  // perfectly matched layer: the layer's acceleration
  // -(M^{-1} (Phi, grad v) + beta p + gamma psi) at every node ([S][nnodes],
  // zero outside the layer), and zeta per axis at the node coordinates; the
  // damping alpha = zeta_x + zeta_y + zeta_z joins the absorbing term
  const Real* pml_acc;      // null: no layer (the kernel built without it is used)
  const Real* pml_zx;
  const Real* pml_zy;
  const Real* pml_zz;
  Real dt;
  // value / normal-derivative traces of p^{n+1} on Gamma_I written by this
  // launch ([S][nn0*nn1][2], compact face grid), or null (the face kernel
  // writes them); trd: the normal-derivative weights of the layer's planes
  Real* trace;
  Real trd[kMaxOrder + 1];
  // tiling
  int nbx, nby, nbz, zchunk, rows, waves;
  int depth;                // prefetch distance in planes (2, or 3 / 4 where built)
  int zlo, zhi;             // planes updated: [zlo, zhi] (all by default)
  // two-step update: planes whose second step needs the coupling terms of
  // the first ([cb0, ce0] and [cb1, ce1]; empty if cb > ce) keep p^{n+1} and
  // the increment of step n+1 for a completion pass
  int cb0, ce0, cb1, ce1;
  int nblocks;
};

// Face kernel: PMUT sampling + modal ODE + face force, receivers, and the
// value / normal-derivative traces of both bricks on Gamma_I.
template <typename Real>
struct FaceArgs {
  const long* counter;
  int* nonfinite;           // watchdog: set when a sampled pressure is not finite
  int nblocks;
  int prime;                // 1: only traces and force from the stored qddot
  int S;
  double dt;
  DomView<Real> d0, d1;
  int ndom;
  // interface traces
  Real* tr0;                // [S][nn0x*nn0y][2] (value, d/dz) at the primary top plane
  Real* tr1;                // [S][nn1x*nn1y][2] at the secondary bottom plane
  Real dz0[kMaxOrder + 1];  // (2/h_z) l_c'(+1), primary
  Real dz1[kMaxOrder + 1];  // (2/h_z) l_c'(-1), secondary
  // PMUTs
  int Np, Nm;
  const int* pm_off;        // [Np+1]
  const int* pm_node;       // flat bottom-face index i + nn0x*j
  const double* pm_B;       // [nodes][Nm] face weight * mode shape
  const double* omega;      // [Np*Nm]
  const double* zeta;
  const double* eta;
  double kappa;
  const double* dA;         // [S*Np][2]: A cos(theta), A sin(theta)
  const double* car;        // [S][ncar][2]: g(t_n) sin(2 pi f t_n), g(t_n) cos(2 pi f t_n)
  long ncar;
  double t_switch, cap;
  double* q;                // [S*Np*Nm]
  double* qd;
  double* qdd;
  Real* force;              // [S][nn0x*nn0y]
  // receivers
  int R;
  const int* r_dom;         // [R]
  const long* r_base;       // [R] node index of the element's first node
  const double* r_w;        // [R][3][kMaxOrder+1]
  double* traces;           // [S][R][cap]
  long tcap;
  // block-role ranges
  int nb_tr0, nb_tr1, nb_pm, nb_rc;
};

// Interface flux kernel: SIPG terms per Gauss point of each fine face,
// reduced onto the faces of both sides.
template <typename Real>
struct FluxArgs {
  int S;
  int N0, N1, Nq;
  int nn0x, nn1x;           // face-grid widths (nodes) of both sides
  int nex0, ney0, nex1, ney1;
  const Real* tr0;
  const Real* tr1;
  const Real* Lq;           // [Nq][N0+1] fine basis at the Gauss points
  const Real* wJ;           // [Nq*Nq] Gauss weight * fine face Jacobian
  const int* xcx;           // [nex0*Nq] coarse element index along x of fine point (ex,qa)
  const int* ycx;           // [ney0*Nq]
  const Real* xw;           // [nex0*Nq][N1+1] coarse basis at the mapped point
  const Real* yw;           // [ney0*Nq][N1+1]
  const int* xl_off;        // [nex1+1] CSR: fine points (ex*Nq+qa) inside coarse element cx
  const int* xl;            //
  const int* yl_off;        // [ney1+1]
  const int* yl;
  Real gamma, cf2, cc2;
  Real* R0;                 // [S][nex0*ney0][(N0+1)^2][2]
  Real* R1;                 // [S][nex1*ney1][(N1+1)^2][2]
  Real* Aq;                 // [S][nex0*ney0][Nq*Nq][2] SIPG terms per fine Gauss point
  long* counter;            // advanced by the coarse pass when tick != 0
  int tick;
  int* xsel;                // [2] live increment copy per brick; with the
  int toggle;               // tick, bit d of toggle swaps brick d's
  int nb_fine, nb_coarse;   // blocks (8 faces each: two per wave)
  int tcap;                 // LDS entries per component and coarse face (x points x (N1+1))
};

// Perfectly matched layer of one brick: auxiliary fields and the layer's
// acceleration, advanced after the brick's stiffness update.
template <typename Real>
struct PmlArgs {
  DomView<Real> d;
  int S;
  const long* counter;
  int prime;                // 1: acceleration of the current level only (psi, Phi kept)
  Real dt, c2;
  Real gh[3];               // 2 / h per axis
  Real J;                   // h_x h_y h_z / 8
  int ne[3];
  const Real* zx;           // zeta per axis at the node coordinates
  const Real* zy;
  const Real* zz;
  const Real* mix;          // inverse assembled 1D lumped mass per axis
  const Real* miy;
  const Real* miz;
  const int* eslot;         // [ne0*ne1*ne2]: slot of the element's Phi, or -1
  const int* pel;           // [nel][3]: element coordinates of each slot
  int nel;
  const int* pnode;         // [npn][3]: nodes of the layer's elements
  int npn;
  Real* phi;                // [S][nel][3][(N+1)^3]
  Real* rel;                // [S][nel][(N+1)^3]: each element's share of (Phi, grad v) at its nodes
  Real* psi;                // [S][nnodes]
  Real* acc;                // [S][nnodes]
  Real w[kMaxOrder + 1];    // GLL weights
  Real D[(kMaxOrder + 1) * (kMaxOrder + 1)];  // D[q][m] = l_m'(x_q)
};

// Trilinear hexahedra (a brick given by its element vertices): the
// element kernel writes each element's residual K_e p at its own nodes, the
// node kernel gathers those, adds the PMUT force and advances the state.
template <typename Real>
struct HexArgs {
  DomView<Real> d;
  int S;
  int ne[3];
  int nel;                  // ne0 ne1 ne2
  int eblocks;              // workgroups of the element kernel (one per strip of elements along x)
  Real dt2, c2;
  const long* counter;
  const Real* force;        // PMUT face force [S][plane] on the bottom plane, or null
  const Real* minv;         // [pnodes] inverse assembled lumped mass
  const Real* vert;         // [nel][24] corner offsets from corner 0 (corner c = cx + 2 cy + 4 cz)
  Real* y;                  // [S][nel (N+1)^3] element residuals, x-contiguous rows
  Real w[kMaxOrder + 1];    // GLL weights
  Real xg[kMaxOrder + 1];   // GLL nodes
  Real D[(kMaxOrder + 1) * (kMaxOrder + 1)];  // D[q][m] = l_m'(x_q)
};

template <typename Real>
hipError_t launch_hex(const HexArgs<Real>& a, bool incr, hipStream_t st);
template <typename Real>
int hex_elems_per_block(int N);

// Face matching on Gamma_I (Sec. 5, Algorithm 3) of hexahedra given by
// their corners; device arrays.
struct MatchArgs {
  int nq, nf, nc;
  const double* fine_hex;   // [nf][8][3]
  const int* fine_face;     // [nf] 2 axis + side
  const double* coarse_hex; // [nc][8][3]
  const int* coarse_face;   // [nc]
  double tol, eps;
  int* elem;                // [nf nq^2]
  double* xi;               // [nf nq^2][3]
  int* unmatched;           // one int
  double gq[kMaxNq + 1];    // Gauss-Legendre nodes
};
hipError_t launch_match(const MatchArgs& a, hipStream_t st);

// A single-brick FP32 solver small enough to keep its pressure in LDS:
// one workgroup per scenario runs many whole steps (stiffness and update,
// PMUT sampling, modal ODE and force, receivers) in one launch.
struct ResidentArgs {
  DomView<float> d;
  int S, nsteps;
  int nc;                   // nodes (compact)
  float inv_nn0, inv_nn1;   // 1 / nn[0], 1 / nn[1] (index decomposition)
  const long* counter;
  float dt2;
  const float* taps;        // [3][N+3][2N]
  const float* mins;        // [3][N+3]
  float* force;             // [S][plane] PMUT face force on the bottom plane, or null
  int* nonfinite;
  // PMUTs
  int Np, Nm, nface;
  int pm_wide;              // some PMUT has more than 48 face nodes: 64 lanes per PMUT, else 16
  const int* pm_off;        // [Np+1]
  const int* pm_node;       // padded bottom-face index
  const double* pm_B;       // [nface][Nm]
  const double* omega;
  const double* zeta;
  const double* eta;
  double kappa, dt;
  const double* dA;         // [S*Np][2]
  const double* car;        // [S][ncar][2]
  long ncar;
  double t_switch, cap;
  double* q;                // [S*Np*Nm]
  double* qd;
  double* qdd;
  // receivers
  int R;
  const long* r_base;       // padded index of the element's first node
  const double* r_w;        // [R][3][kMaxOrder+1]
  double* traces;           // [S][R][tcap]
  long tcap;
  // dynamic LDS layout (bytes)
  int off_force, off_taps, off_mins, off_B, off_fn, off_q;
  int off_coef, off_da, off_rw, off_poff, off_rb;  // ODE coefficients, drive, receiver weights, PMUT offsets, receiver bases
  int lds_bytes;
};
hipError_t launch_resident(const ResidentArgs& a, hipStream_t st);
int resident_max_nodes();
__host__ __device__ int resident_pad(int N, int nx, int ny);  // zero padding around p in LDS (nodes)
hipError_t launch_tick_n(long* counter, long n, hipStream_t st);

// Launchers (defined in pmutdg_kernels.hip).
template <typename Real>
hipError_t launch_stiff(const StiffArgs<Real>& a, bool incr, hipStream_t st);
template <typename Real>
hipError_t launch_face(const FaceArgs<Real>& a, hipStream_t st);
template <typename Real>
hipError_t launch_flux(const FluxArgs<Real>& a, hipStream_t st);
template <typename Real>
hipError_t launch_fill(Real* p, long n, Real v, hipStream_t st);
// two steps of the FP32 increment-form stiffness update in one pass
hipError_t launch_stiff2(const StiffArgs<float>& a, hipStream_t st);
int stiff2_tile_rows(int N);  // owned rows per two-step tile (0: order not supported)
hipError_t launch_stiff2_lo(const StiffArgs<float>& a, hipStream_t st);
hipError_t launch_fill_bytes(void* p, size_t n, hipStream_t st);
hipError_t launch_tick(long* counter, int* xsel, int toggle, hipStream_t st);
hipError_t launch_pack_traces(const double* src, void* dst, int bits, long cap, long n, long rows, hipStream_t st);
// perfectly matched layer (pml_kernels.hip): the stiffness update with the
// layer's terms, and the auxiliary-field kernels run after it
template <typename Real>
hipError_t launch_stiff_pml(const StiffArgs<Real>& a, bool incr, hipStream_t st);
template <typename Real>
hipError_t launch_pml(const PmlArgs<Real>& a, hipStream_t st);
constexpr int kPmlMaxOrder = 6;
// batched form
size_t batch_lds_bytes(int N, int rows);
hipError_t batch_occupancy(int nmax, size_t lds, int* blocks_per_cu);
// woff: per-workgroup item ranges [grid + 1] (nullptr: round robin)
hipError_t launch_stiff_batch(const StiffArgs<float>* probs, const int2* items, int nitems, const int* woff,
                              int nmax, int grid, size_t lds, hipStream_t st);
hipError_t launch_face_batch(const FaceArgs<float>* probs, const int2* items, int nitems, int grid, int nm_max,
                             hipStream_t st);
hipError_t launch_tick_batch(long* const* counters, int n, hipStream_t st);

}  // namespace pmdg

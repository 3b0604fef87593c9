// Shared layout constants and the device-side trajectory descriptor.
//
// Product digits.  Every Taylor coefficient that enters a product is stored
// as a "row": the exact value s * D * 2^(28 e) with D split into nd signed
// radix-2^28 digits that all carry the sign s (digit j has weight 2^(28(e+j))).
// A product of two rows is then a sum of 32x32 -> 64-bit signed digit products
// (v_mad_i64_i32) with no sign handling, and a sum of products of rows with
// different exponents is a sum of shifted digit convolutions.
//
// Row layout (int32 words): [HDR header: e, s, 0...][RPAD zero digits]
// [nd digits][RPAD + TQ zero digits], stride RS rounded to 32 words (128 B).
#pragma once
#include <stdint.h>

namespace mpts {

constexpr int DBITS = 28;                      // bits per product digit
constexpr long long DMASK = (1LL << DBITS) - 1;
constexpr int TQ = 8;                          // tile edge in digits (8x8 products per lane)
constexpr int WGS = 256;                       // threads per workgroup
constexpr int SMAX = 24;                       // largest exponent spread (digits) of one exact sum
constexpr int HDR = 8;                         // row header words
constexpr int RPAD = 2 * SMAX + 8;             // zero digits on each side of a row (every term offset)
constexpr int NFR = 5;                         // product frames per coefficient index
constexpr int FLUSH_TERMS = 15;                // terms between accumulator carry-normalisations

// constant rows (each a p-bit value converted to a row at kernel start)
enum { C_SIGMA = 0, C_NSIGMA, C_R, C_NB, C_TAU, C_ONE, NCONST };

// sync words, each on its own 128-byte line: NSPLIT arrival counters,
// NSPLIT copies of the publication flag and NSPLIT copies of the
// coefficient-row flag (six 64-bit words: generation and one header word of
// each new row), workgroup r using copy r mod NSPLIT so that no single line
// takes every workgroup's atomics or polls; the error word and the Horner
// completion counter, and the generation of group frames the leader has
// cleared
constexpr int NSPLIT = 8;
enum { SY_ARRIVE = 0, SY_FLAG = 32 * NSPLIT, SY_HFLAG = 64 * NSPLIT, SY_ERROR = 96 * NSPLIT,
       SY_HDONE = 96 * NSPLIT + 32, SY_CLEAR = 96 * NSPLIT + 64, SY_WORDS = 96 * NSPLIT + 96 };

enum { MODE_INTEGRATE = 0, MODE_COEFFS = 1, MODE_ADJOINT = 2 };

__host__ __device__ inline int digits_per_row(int L) { return (32 * L + DBITS - 1 + DBITS - 1) / DBITS; }
inline int row_stride(int nd) { int rs = HDR + RPAD + nd + RPAD + TQ; return (rs + 31) & ~31; }
// frame width in columns: products of two rows span 2 nd - 1 columns, plus the
// term offsets (up to 2 SMAX above the frame base: the Cauchy frames take
// their base SMAX below one term's exponent sum), plus the tile overhang of
// the last diagonal, plus carries.
inline int frame_width(int nd) { int w = 2 * nd + 2 * SMAX + 2 * TQ + 8; return (w + 31) & ~31; }
// digits one single-wave big-integer task must hold (combine + division)
inline int task_digits(int nd) { return 3 * nd + 2 * SMAX + 48; }
// bytes of the adjoint's per-term offset tables: its frames of one index
// hold at most 4 N + 4 terms in at most 8 parts without exponent caches,
// each part's slice rounded up to 16
__host__ __device__ inline int adj_table_bytes(int N) { return 4 * N + 4 + 8 * 16; }

// Address-space views of pointers whose memory kind is known: loads through
// them compile to global_load / ds_read (waited for with their own counters)
// instead of flat accesses, which make every wait cover all memory in flight.
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(3))) int32_t l_i32;
typedef __attribute__((address_space(3))) long long l_i64;
typedef __attribute__((address_space(3))) int8_t l_i8;

struct Inst {
  int L, N, nd, RS, WB, CM;  // limbs, order, digits/row, row stride, frame width, chunk max
  int G, wg0;                // workgroups of the group and the first one
  int mode;
  int loss;           // adjoint seed: 0 = 2 x(T) (squared norm), 1..3 = unit vector e_x, e_y, e_z
  int mfma;           // bit 0: early Cauchy products on the int8 matrix cores (else VALU tiles)
  int next;           // batch: 1 + index of the instance the same workgroups run next (0: none)
  // rational step size (tau_d > 0): d tau = n + (m1 2^28 + m0) 2^(28 e)
  // exactly, so tau h = (n h + (m1 2^28 + m0) 2^(28 e) h) / d
  int tau_n, tau_d, tau_m0, tau_m1, tau_e;
  long long nsteps;
  int32_t *rows;      // [3][N+1][RS]
  int32_t *consts;    // [NCONST][RS]
  int32_t *cnorm;     // [NCONST][L+2] normalised constants (written by the host)
  int32_t *state;     // [3][L+2] normalised state (sign, E, M[L]), in and out
  int32_t *coefs;     // [3][N+1][L+2] normalised coefficients (MODE_COEFFS) or null
  int32_t *ckpt;      // [nsteps+1][3][L+2] or null
  long long *gframes; // [2][NFR][WB] (G > 1)
  uint32_t *sync;     // SY_* words
  // adjoint
  int32_t *adj;       // adjoint scratch (MODE_ADJOINT)
  unsigned long long *prof;  // per-phase wall-clock ticks (null: not recorded)
};

// A trajectory of a polynomial vector field of degree at most two:
//   dx_v/dt = c_v + sum_u A_vu x_u + sum_{u <= w} B_vuw x_u x_w,  v < V.
// Operands are encoded o < V: the row x_{o,i} of the current index, o >= V:
// the rounded Cauchy sum S_{o-V} of the pair (pu, pw).  Equation v's
// numerator is sum_j const[cp[v][j]] * operand(op[v][j]) (np[v] products,
// one frame) plus na[v] operands with coefficient asg = +-1, plus (index 0
// only) the constant row cc[v] (-1: none).
constexpr int PMAXV = 4, PMAXQ = NFR, PMAXP = 4, PMAXA = 3;
struct PolyInst {
  int L, N, nd, RS, WB, CM, V, Q;
  int tau_n, tau_d, tau_m0, tau_m1, tau_e;  // rational step size (tau_d > 0), as in Inst
  int ctau;                                 // constant row of tau
  int nconst;
  int maxn;                                 // bytes of the per-term offset tables
  long long nsteps;
  int32_t *rows;    // [V][N+1][RS]
  int32_t *sums;    // [Q][RS]
  int32_t *consts;  // [nconst][RS] (written by the kernel from cnorm)
  int32_t *cnorm;   // [nconst][L+2] normalised constants
  int32_t *state;   // [V][L+2] normalised state, in and out
  int32_t *coefs;   // [V][N+1][L+2] normalised coefficients of the first step, or null
  uint32_t *err;    // error word (bits as in the Lorenz kernels)
  int pu[PMAXQ], pw[PMAXQ];
  int np[PMAXV], cp[PMAXV][PMAXP], op[PMAXV][PMAXP];
  int na[PMAXV], asg[PMAXV][PMAXA], ao[PMAXV][PMAXA], cc[PMAXV];
};

// phases timed when Inst::prof is set (leader slots 0..15, one follower 16..31)
enum { PH_SETUP = 0, PH_ACCUM, PH_FLUSH, PH_WAIT, PH_FINAL, PH_CLEAR, PH_HORNER, PH_STEP0,
       PH_EBUILD, PH_ESETUP = 10, PH_NPHASE = 16 };
constexpr int PROF_RANK = 8;  // per-workgroup profile words
// leader slot of the lag from the last arrival to the end of the leader's
// wait, and the word holding the latest arrival time (in the first
// follower's per-workgroup words)
enum { PH_ARRLAG = 10, PROF_ARRT = 2 * PH_NPHASE + PROF_RANK + 7 };

}  // namespace mpts

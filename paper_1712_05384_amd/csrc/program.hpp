// Step program records shared by the host planner and the device kernels.
#pragma once

#include <cstdint>

namespace qgm {

// Sources of a variable's value inside one step's factor program.
enum : uint8_t {
    SRC_ZERO = 0,  // constant 0 (input delta of Eq. (psi_x))
    SRC_K = 1,     // bit of the contracted index K
    SRC_V = 2,     // bit of the kept shared index V
    SRC_N = 3,     // bit of the new index N
    SRC_SIG = 4,   // bit of the per-bitstring variant sigma (output bit or slice bit)
    SRC_INT = 5    // summed inside G (internal worldline variable)
};

// Factor-program operations.  The program walks one qubit's worldline in time
// order with a 2-vector s over the current worldline variable, starting from
// s = (1, 0) (the input delta b_q^0 = 0).
enum : uint8_t {
    GOP_PROJECT = 0,  // the current variable takes the value of (src, bit): zero the other entry
    GOP_MAT = 1,      // non-diagonal gate: s <- M[mat] s (sums out the previous variable)
    GOP_DIAG = 2,     // diagonal gate on the current variable: s[c] *= M[mat][c][c]
    GOP_CZ = 3,       // CZ with a partner variable of value p = (src, bit): s[1] *= (-1)^p
    GOP_END = 4       // result = s[value of (src, bit)] (the last worldline variable)
};

// All fields are 32-bit so that every field sits at a dword-aligned offset:
// the kernels read the program with scalar loads, and a scalar load whose
// base register is not dword aligned silently drops the low address bits.
struct GOp {
    int32_t type;
    int32_t src;
    int32_t bit;
    int32_t mat;
};

constexpr int kFixedMats = 10;      // H, T, X^1/2, Y^1/2, T^dag, X^-1/2, Y^-1/2, X, Y, Z; slot s is matrix kFixedMats + s
constexpr int kMaxKB = 6;           // K bits handled with the contracted slice in registers
constexpr int kMaxBits = 8;         // per-step bound on V bits, on sigma bits
constexpr int kMaxNB = 10;
constexpr int kMaxRank = 31;
constexpr int kDenseMaxVariants = 16;  // matrix-core kernel: at most 2^4 operand variants per step
constexpr int kMaxOps = 128;           // factor-program length per step (the G builder's adjoint keeps each state)

// Per-step launch parameters (passed by value to the step kernel).
struct StepParams {
    int32_t kb, vb, nb, sb;
    int32_t row_bits;       // r_in - kb = number of bits of a row (M and V axes)
    int32_t input_is_one;
    int32_t kpos[kMaxKB];
    int32_t vpos[kMaxBits];
    int32_t pair_bit;       // >= 0: each thread also handles row | (1 << pair_bit) (a non-V row bit)
    int32_t pair_in;        // input-tensor offset of that bit
    int64_t g_off;
};

}  // namespace qgm

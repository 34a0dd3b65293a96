// Right-Radau collocation tables and small dense linear algebra, host side.
//
// Sec. 2.1: M right Gauss-Radau nodes on a step (t_M = T_{n+1}) and the
// quadrature matrix q_mj = (1/dt) int_{T_n}^{t_m} l_j.  Sec. 2.2: the DG
// matrices K_q, M_q, J_q (Eqs. Kq, Mq).  For right Radau nodes M_q = dt diag(b)
// (the M-point Radau rule integrates l_i l_j exactly) and J_q = l(0) e_M^T
// (l_j(T_{n+1}) = delta_jM), and K_q = diag(b) Q^{-1}; the library uses these
// identities, which make the DG system and the collocation system have the same
// solution (Sec. 5.1).  Everything is computed in long double.
#pragma once
#include <vector>

namespace stmg {

struct RadauTables {
  int M = 0;
  long double c[8];      // nodes in (0, 1], c[M-1] = 1
  long double Q[8][8];   // collocation matrix on the unit step
  long double b[8];      // quadrature weights = last row of Q
  long double Kq[8][8];  // diag(b) Q^{-1}
  long double l0[8];     // Lagrange basis at the step's left end, = Kq 1
};

// Builds the tables for 1 <= M <= 8.  Returns false on failure.
bool radau_tables(int M, RadauTables* out);

// In-place Gauss-Jordan inverse with partial pivoting of an n x n row-major
// matrix.  Returns false if singular.
bool invert_ld(std::vector<long double>& a, int n);

}  // namespace stmg

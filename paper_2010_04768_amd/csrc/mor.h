// Model-order reduction state kept in the context: an orthonormal real basis S
// of solved vectors, Hbar_N S and the projected operator Hhat = S^T Hbar_N S.
#pragma once
#include "gfcc_internal.h"

namespace gfcc {

struct Mor {
  int64_t m = 0;    // basis columns in use
  int64_t cap = 0;  // allocated columns (S, HS) and leading dimension of H
  DBuf S;           // [cap][Dp] orthonormal columns in plane layout
  DBuf HS;          // [cap][Dp] Hbar_N applied to each column of S
  DBuf H;           // [cap][cap] Hhat[i][j] = s_i . (Hbar_N s_j)
  DBuf V;           // candidate planes of an extension
  DBuf coef, nrm;   // Gram-Schmidt coefficients, candidate norms
  DBuf Ch;          // [m][nq] chat = S c_q
  DBuf rows, pdev;  // gathered left vectors, device copy of index lists
  DBuf Aw;          // model systems [chunk][m][m + np] complex
  DBuf Gm;          // model G output staging
  DBuf flag;        // singular-pivot flag of the model solves
  Scratch scr;
};

}  // namespace gfcc

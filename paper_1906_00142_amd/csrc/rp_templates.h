// rp_templates.h -- the templates that turn metric values into a program's
// value E (Section 2, Examples 1-2, equation (occupancy)).  The text between
// RP_TPL_SRC( and its closing parenthesis is compiled into the library's
// table-driven evaluator and is also kept as a string, so that run-time
// generated evaluators (code generation, Section 3.3 step 3) use the very
// same template code.  It holds no preprocessor directives.
#ifndef RP_TEMPLATES_H
#define RP_TEMPLATES_H

#ifndef RP_TPL_SRC
#define RP_TPL_SRC(...) __VA_ARGS__
#endif

RP_TPL_SRC(
// hardware vector entries
enum { H_WAVE, H_NUM_CU, H_SIMD, H_TMAX, H_BMAX, H_WMAX, H_REGS_CU, H_LDS_CU, H_MEM_LAT,
       H_L2_LAT, H_DEP_COAL, H_DEP_UNCOAL, H_ISSUE, H_SFU_ISSUE, H_LDS_ISSUE, H_CLOCK, H_BW };
// metric slots
enum { G_COMP, G_COAL, G_UNCOAL, G_SYNCH, G_COAL_PER_MW, G_UNCOAL_PER_MW, G_LOAD_BYTES, G_REGS,
       G_LDS_BYTES, G_BLOCKS, G_SFU, G_LDS_INSTS, G_LDS_CONFLICT, G_BRANCH, G_L2_HIT,
       G_DIVERGENCE };

template <typename R>
__device__ __forceinline__ R clamp_lo(R v, R lo) { return v > lo ? v : lo; }

// Blocks of T threads resident on one compute unit at once: the smallest of
// the unit's block limit, its wave limit over ceil(T/W) waves per block, its
// registers over regs * W * ceil(T/W) (a partial wave holds a whole wave's
// registers) and its LDS over the block's bytes, each rounded down.
template <typename R>
__device__ __forceinline__ R resident_blocks(const R* h, R T, R W, R regs, R lds) {
  const R wpb = ceil(T / W);
  const R b_waves = floor(h[H_WMAX] / wpb);
  const R b_regs = floor(h[H_REGS_CU] / (regs * W * wpb));
  const R b_lds = lds > R(0) ? floor(h[H_LDS_CU] / lds) : h[H_BMAX];
  return fmin(fmin(h[H_BMAX], b_waves), fmin(b_regs, b_lds));
}

// Hardware occupancy (Section 2, Example 1): active waves over the unit's
// maximum, with the active waves of equation (occupancy) (wave size W as a
// parameter).  Metric 0 = registers per thread, metric 1 = LDS bytes per
// block.  -inf when the block format cannot run.
template <typename R>
__device__ R block_occupancy(const R* g, const R* h, R bx, R by) {
  const R T = bx * by;
  const R W = h[H_WAVE];
  if (!(T >= R(1)) || T > h[H_TMAX]) return -(R)INFINITY;
  const R regs = ceil(clamp_lo(g[0], R(1)));
  const R lds = ceil(clamp_lo(g[1], R(0)));
  const R b_active = resident_blocks<R>(h, T, W, regs, lds);
  if (!(b_active >= R(1))) return -(R)INFINITY;
  return fmin(floor(b_active * T / W), h[H_WMAX]) / h[H_WMAX];
}

// MWP-CWP-style estimate of cycles for one block format (Section 2,
// Examples 1-2 and equation (occupancy) with the wave size as a parameter).
template <typename R>
__device__ R mwpcwp_cycles(const R* g, const R* h, R bx, R by) {
  const R inf = (R)INFINITY;
  const R T = bx * by;
  const R W = h[H_WAVE];
  if (!(T >= R(1)) || T > h[H_TMAX]) return inf;
  const R comp = clamp_lo(g[G_COMP], R(0)), coal = clamp_lo(g[G_COAL], R(0));
  const R uncoal = clamp_lo(g[G_UNCOAL], R(0)), synch = clamp_lo(g[G_SYNCH], R(0));
  const R coal_mw = clamp_lo(g[G_COAL_PER_MW], R(1)), uncoal_mw = clamp_lo(g[G_UNCOAL_PER_MW], R(1));
  const R load_bytes = clamp_lo(g[G_LOAD_BYTES], R(0));
  const R regs = ceil(clamp_lo(g[G_REGS], R(1)));
  const R lds = ceil(clamp_lo(g[G_LDS_BYTES], R(0)));
  const R blocks = ceil(clamp_lo(g[G_BLOCKS], R(1)));
  const R sfu = clamp_lo(g[G_SFU], R(0)), lds_insts = clamp_lo(g[G_LDS_INSTS], R(0));
  const R conflict = clamp_lo(g[G_LDS_CONFLICT], R(0)), branch = clamp_lo(g[G_BRANCH], R(0));
  const R hit = fmin(clamp_lo(g[G_L2_HIT], R(0)), R(1));
  const R diverge = fmin(clamp_lo(g[G_DIVERGENCE], R(0)), R(1));

  // resident blocks per compute unit, then active waves (equation (occupancy))
  const R b_active = resident_blocks<R>(h, T, W, regs, lds);
  if (!(b_active >= R(1))) return inf;
  const R N = fmin(floor(b_active * T / W), h[H_WMAX]);
  const R active_cu = fmin(h[H_NUM_CU], blocks);
  const R rep = ceil(blocks / (b_active * active_cu));

  // memory warp parallelism
  const R mem = coal + uncoal;
  const R w_u = mem > R(0) ? uncoal / mem : R(0);
  const R w_c = R(1) - w_u;
  const R mem_eff = clamp_lo(mem, R(1));
  const R lat = (R(1) - hit) * h[H_MEM_LAT] + hit * h[H_L2_LAT];
  const R mem_l_uncoal = lat + (uncoal_mw - R(1)) * h[H_DEP_UNCOAL];
  const R mem_l_coal = lat + (coal_mw - R(1)) * h[H_DEP_COAL];
  const R mem_l = mem_l_uncoal * w_u + mem_l_coal * w_c;
  const R dep = h[H_DEP_UNCOAL] * uncoal_mw * w_u + h[H_DEP_COAL] * coal_mw * w_c;
  const R mwp_nobw = mem_l / dep;
  R mwp_bw = inf;
  if (load_bytes > R(0)) {
    const R bw_per_warp = h[H_CLOCK] * load_bytes / mem_l;
    mwp_bw = h[H_BW] / (bw_per_warp * active_cu);
  }
  const R mwp = clamp_lo(fmin(fmin(mwp_nobw, mwp_bw), N), R(1));

  // computation warp parallelism
  R comp_cycles = h[H_ISSUE] * (comp + mem + branch * (R(1) + diverge)) + h[H_SFU_ISSUE] * sfu +
                  h[H_LDS_ISSUE] * lds_insts * (R(1) + conflict);
  comp_cycles = clamp_lo(comp_cycles, h[H_ISSUE]);
  const R mem_cycles = mem_l_uncoal * uncoal + mem_l_coal * coal;
  const R cwp = fmin((mem_cycles + comp_cycles) / comp_cycles, N);

  R e;
  if (mwp == N && cwp == N)
    e = (mem_cycles + comp_cycles + comp_cycles / mem_eff * (mwp - R(1))) * rep;
  else if (cwp >= mwp || comp_cycles > mem_cycles)
    e = (mem_cycles * N / mwp + comp_cycles / mem_eff * (mwp - R(1))) * rep;
  else
    e = (lat + comp_cycles * N) * rep;
  return e + dep * (mwp - R(1)) * synch * b_active * rep;
}
)

#endif

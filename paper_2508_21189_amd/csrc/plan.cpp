// Batch plan of the batched sketch-and-solve (Alg. 3 for many independent
// problems, as lstsq_sketch_solve_batched): the problems, their workspace
// layout and tables are fixed once, and the whole batch (row codes, the
// bucket-indexed applies per register file with b as the column after A's
// last, the chunk sums into each problem's column-major [S A | S b], the
// batched Householder QR, R^-1, the certified solve and the SVD fallback)
// is captured into one HIP graph and replayed with one launch.
//
// Tuning: each problem's row-chunk length (a multiple of d) comes from a JSON
// cache keyed by device, input type, accumulator register file and bucket
// parts; the tuner times the candidates on the batch's own problems.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "sk_dense.hpp"
#include "sk_launch.hpp"

struct sk_batch {
  int device = 0;
  int nprob = 0, d_per_k = 0, zeta = 0, kmax = 0;
  std::vector<sk_ls_problem> probs;
  std::vector<sk_sketch> sks;
  std::vector<int> chunk_mult;  // row chunks of chunk_mult * d rows (per problem)
  int tuned = 0;
  // workspace: ranks, QR table, per-problem factor and fallback buffers,
  // then the batched sketch (its tables, codes and partials)
  size_t off_table = 0, off_factors = 0, off_bsk = 0, bsk_bytes = 0, total = 0;
  std::vector<size_t> factor_at;
  void* ws = nullptr;
  sk::IdxBatchProgram prog;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int kernel_nodes = 0;
  int64_t graph_launches = 0;
  int sketch_workgroups = 0, sketch_launches = 0, reduce_blocks = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool timed = false;     // e0 and e1 bracket the last graph launch
  bool launched = false;  // a launch or an enqueue since the last bind
  void* h_ranks = nullptr;
  bool bound = false;
};

namespace sk {
namespace plan {
namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

void make_sketch(const sk_ls_problem& p, int d_per_k, int zeta, int device, sk_sketch* W) {
  *W = sk_sketch{};
  W->kind = SK_SPARSESTACK;
  W->d = (int64_t)d_per_k * p.k;
  W->n = p.n;
  W->zeta = zeta;
  W->nb = W->d / zeta;
  W->seed = p.seed;
  W->k0 = (uint32_t)p.seed;
  W->k1 = (uint32_t)(p.seed >> 32);
  W->device = device;
}

bool problem_valid(const sk_ls_problem& p, int d_per_k, int zeta) {
  if (p.n < 1 || p.k < 1 || p.k > 1024 || p.lda < p.k || !p.A || !p.b || !p.x) return false;
  if (p.dtype != SK_F64 && p.dtype != SK_F32 && p.dtype != SK_BF16) return false;
  const int64_t d = (int64_t)d_per_k * p.k;
  return d >= p.k && d % zeta == 0;
}

// ---- tuning cache (flat JSON: {"key": {"chunk_d": m, "ms": t}, ...})
struct Tune {
  int chunk_d = 0;
  double ms = 0.0;
};
std::mutex g_tune_mu;

std::string cache_path() {
  const char* e = std::getenv("SKETCH_TUNE_CACHE");
  if (e && *e) return e;
  const char* x = std::getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/libsketch/batched_tune.json";
  const char* h = std::getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/libsketch/batched_tune.json";
}

std::map<std::string, Tune> read_cache(const std::string& path) {
  std::map<std::string, Tune> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  for (;;) {
    const size_t q0 = s.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = s.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
    pos = q1 + 1;
    if (key.find('/') == std::string::npos) continue;  // not an entry key
    const size_t ob = s.find('{', pos), cb = s.find('}', pos);
    if (ob == std::string::npos || cb == std::string::npos || ob > cb) continue;
    const std::string body = s.substr(ob, cb - ob);
    auto num = [&](const char* name) -> double {
      const size_t k = body.find(std::string("\"") + name + "\"");
      if (k == std::string::npos) return -1.0;
      const size_t c = body.find(':', k);
      return c == std::string::npos ? -1.0 : std::atof(body.c_str() + c + 1);
    };
    Tune t;
    t.chunk_d = (int)num("chunk_d");
    t.ms = num("ms");
    if (t.chunk_d > 0) m[key] = t;
    pos = cb + 1;
  }
  return m;
}

void mkdirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string dir = path.substr(0, i);
      if (mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
}

bool write_cache(const std::string& path, const std::map<std::string, Tune>& m) {
  mkdirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return false;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      char line[256];
      std::snprintf(line, sizeof line, "  \"%s\": {\"chunk_d\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(),
                    kv.second.chunk_d, kv.second.ms, ++i < m.size() ? "," : "");
      f << line;
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

std::string device_tag(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch = arch.substr(0, c);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// The class a problem's chunk length is tuned for: device, input type,
// accumulator register file (slots) and bucket parts of its apply.
std::string tune_key(const std::string& dev, const sk_ls_problem& p, const sk_sketch& S) {
  const char* dt = p.dtype == SK_F64 ? "f64" : (p.dtype == SK_F32 ? "f32" : "bf16");
  const int64_t regs = S.nb * (p.dtype == SK_F64 ? 2 : 1);
  const int nreg = regs <= 32 ? 32 : regs <= 64 ? 64 : regs <= 128 ? 128 : 200;
  const int64_t cap = (p.dtype == SK_F64 ? 100 : 200) - (p.dtype == SK_F64 ? 4 : 8);
  const int parts = regs <= 200 ? 1 : (int)((S.nb + cap - 1) / cap);
  return dev + "/" + dt + "/r" + std::to_string(nreg) + "/p" + std::to_string(parts);
}

// Buffers of one problem: the QR's (W, tau, T, R, c, X, XT) and the SVD
// fallback's (Uc, Vc, sv, z).
size_t factor_bytes(int64_t d, int k) {
  size_t b = 0;
  auto take = [&](size_t doubles) { b = al256(b) + std::max<size_t>(1, doubles) * sizeof(double); };
  take((size_t)d * (k + 1));
  take((size_t)k);
  take(qr_tbuf_doubles(k));
  for (int i = 0; i < 4; ++i) take((size_t)k * k);  // R, X, XT, then Uc
  take((size_t)k * k);                              // Vc
  take((size_t)k);                                  // c
  take((size_t)k);                                  // sv
  take((size_t)k);                                  // z
  return al256(b);
}
QrBatch factor_entry(char* base, int64_t d, int k, double* x, int* rank) {
  size_t o = 0;
  auto take = [&](size_t doubles) {
    o = al256(o);
    double* p = reinterpret_cast<double*>(base + o);
    o += std::max<size_t>(1, doubles) * sizeof(double);
    return p;
  };
  QrBatch q{};
  q.W = take((size_t)d * (k + 1));
  q.ldw = d;
  q.d = d;
  q.k = k;
  q.tau = take((size_t)k);
  q.T = take(qr_tbuf_doubles(k));
  q.R = take((size_t)k * k);
  q.X = take((size_t)k * k);
  q.XT = take((size_t)k * k);
  q.Uc = take((size_t)k * k);
  q.Vc = take((size_t)k * k);
  q.c = take((size_t)k);
  q.sv = take((size_t)k);
  q.z = take((size_t)k);
  q.x = x;
  q.rank = rank;
  return q;
}

std::vector<IdxBatchJob> jobs_of(const sk_batch* B, const std::vector<double*>& W) {
  std::vector<IdxBatchJob> jobs;
  for (int i = 0; i < B->nprob; ++i) {
    const sk_ls_problem& p = B->probs[i];
    jobs.push_back(IdxBatchJob{&B->sks[i], p.dtype, p.k, p.A, p.lda, p.b, W.empty() ? nullptr : W[i],
                               B->chunk_mult[i]});
  }
  return jobs;
}

int layout(sk_batch* B) {
  size_t o = al256(sizeof(int) * (size_t)B->nprob);
  B->off_table = o;
  o = al256(o + sizeof(QrBatch) * (size_t)B->nprob);
  B->off_factors = o;
  B->factor_at.assign((size_t)B->nprob, 0);
  for (int i = 0; i < B->nprob; ++i) {
    B->factor_at[i] = o;
    o += factor_bytes(B->sks[i].d, (int)B->probs[i].k);
  }
  B->off_bsk = al256(o);
  const std::vector<IdxBatchJob> jobs = jobs_of(B, {});
  const int rc = idx_batch_workspace(jobs.data(), (int)jobs.size(), &B->bsk_bytes);
  if (rc < 0) return rc;
  B->total = B->off_bsk + B->bsk_bytes;
  return SK_OK;
}

// Everything a launch runs, queued on st (kernels only: no copies, no waits).
int enqueue_all(const sk_batch* B, hipStream_t st) {
  int rc = idx_batch_enqueue(B->prog, st);
  if (rc < 0) return rc;
  const QrBatch* table = reinterpret_cast<const QrBatch*>(static_cast<char*>(B->ws) + B->off_table);
  const double eps = std::ldexp(1.0, -52);
  if ((rc = qr_trinv_batched(table, B->nprob, B->kmax, st)) < 0) return rc;
  if ((rc = certified_tri_solve_batched(table, B->nprob, eps, st)) < 0) return rc;
  return svd_fallback_batched(table, B->nprob, eps, st);
}

int release_graph(sk_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->bound = false;
  return SK_OK;
}

// Tables into the workspace (one synchronous upload), then the graph.
int bind(sk_batch* B, void* ws, hipStream_t st) {
  release_graph(B);
  B->ws = ws;
  char* base = static_cast<char*>(ws);
  std::vector<QrBatch> table;
  std::vector<double*> W;
  int* ranks = reinterpret_cast<int*>(base);
  for (int i = 0; i < B->nprob; ++i) {
    const sk_ls_problem& p = B->probs[i];
    table.push_back(factor_entry(base + B->factor_at[i], B->sks[i].d, (int)p.k, p.x, ranks + i));
    W.push_back(table.back().W);
  }
  const std::vector<IdxBatchJob> jobs = jobs_of(B, W);
  int rc = idx_batch_prepare(jobs.data(), (int)jobs.size(), base + B->off_bsk, B->bsk_bytes, &B->prog);
  if (rc < 0) return rc;
  B->sketch_workgroups = 0;
  B->sketch_launches = 0;
  B->reduce_blocks = 0;
  for (const auto& l : B->prog.launches) {
    if (l.kind == 1) {
      B->sketch_workgroups += (int)l.grid;
      ++B->sketch_launches;
    } else if (l.kind == 2 || l.kind == 3) {
      B->reduce_blocks += (int)l.grid;
    }
  }
  SK_HIP(hipMemcpyAsync(base + B->off_table, table.data(), sizeof(QrBatch) * table.size(), hipMemcpyHostToDevice,
                        st));
  if (!B->prog.tables.empty())
    SK_HIP(hipMemcpyAsync(base + B->off_bsk, B->prog.tables.data(), B->prog.tables.size(), hipMemcpyHostToDevice,
                          st));
  SK_HIP(hipStreamSynchronize(st));
  hipStream_t cs = nullptr;
  SK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    set_error("lstsq_batched_bind: stream capture failed to start");
    rc = SK_E_HIP;
  } else {
    rc = enqueue_all(B, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc == SK_OK && e != hipSuccess) {
      set_error("lstsq_batched_bind: stream capture failed");
      rc = SK_E_HIP;
    }
    B->graph = g;
  }
  (void)hipStreamDestroy(cs);
  if (rc != SK_OK) return rc;
  SK_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  size_t nn = 0;
  SK_HIP(hipGraphGetNodes(B->graph, nullptr, &nn));
  B->kernel_nodes = (int)nn;
  B->bound = true;
  B->launched = false;
  B->timed = false;
  return SK_OK;
}

int results(sk_batch* B, sk_ls_problem* probs, hipStream_t st) {
  const size_t rb = sizeof(int) * (size_t)B->nprob;
  if (!B->h_ranks) SK_HIP(hipHostMalloc(&B->h_ranks, rb, hipHostMallocDefault));
  SK_HIP(hipMemcpyAsync(B->h_ranks, B->ws, rb, hipMemcpyDeviceToHost, st));
  SK_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  if (B->timed) (void)hipEventElapsedTime(&ms, B->e0, B->e1);
  const int* rank = static_cast<const int*>(B->h_ranks);
  bool rankdef = false;
  for (int i = 0; i < B->nprob; ++i) {
    probs[i].rank = rank[i];
    probs[i].status = rank[i] < probs[i].k ? SK_W_RANKDEF : SK_OK;
    probs[i].t_ms = ms;
    rankdef = rankdef || rank[i] < probs[i].k;
  }
  return rankdef ? SK_W_RANKDEF : SK_OK;
}

int check_all(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int device, const char* who) {
  if (!probs || nprob < 1 || d_per_k < 1 || zeta < 1) {
    set_error(std::string(who) + ": need problems, nprob >= 1, d_per_k >= 1 and zeta >= 1");
    return SK_E_INVAL;
  }
  for (int i = 0; i < nprob; ++i) {
    if (!problem_valid(probs[i], d_per_k, zeta)) {
      set_error(std::string(who) + ": problem " + std::to_string(i) +
                " is invalid (need n >= 1, 1 <= k <= 1024, lda >= k, pointers, a dtype, zeta | d_per_k * k)");
      return SK_E_INVAL;
    }
  }
  for (int i = 0; i < nprob; ++i) {
    const sk_ls_problem& p = probs[i];
    sk_sketch S;
    make_sketch(p, d_per_k, zeta, device, &S);
    std::string why;
    if (S.d > 1024 || p.k > 512)
      why = "d = d_per_k * k above 1024 (or k above 512)";
    else if (!idx_batch_fits(&S, p.dtype, p.k, p.A, p.lda))
      why = "k below 4, rows of A not 4-byte aligned, or more buckets than four register files hold";
    else if ((uintptr_t)p.b % dtype_size(p.dtype) != 0 || (uintptr_t)p.x % 8 != 0)
      why = "b or x is not aligned to its element size";
    if (!why.empty()) {
      set_error(std::string(who) + ": problem " + std::to_string(i) + ": " + why);
      return SK_E_NOTSUP;
    }
  }
  return SK_OK;
}

sk_batch* new_batch(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int device) {
  sk_batch* B = new sk_batch;
  B->device = device;
  B->nprob = nprob;
  B->d_per_k = d_per_k;
  B->zeta = zeta;
  B->probs.assign(probs, probs + nprob);
  B->sks.resize((size_t)nprob);
  B->chunk_mult.assign((size_t)nprob, 16);
  for (int i = 0; i < nprob; ++i) {
    make_sketch(probs[i], d_per_k, zeta, device, &B->sks[i]);
    B->kmax = std::max(B->kmax, (int)probs[i].k);
  }
  return B;
}

void free_batch(sk_batch* B) {
  if (!B) return;
  release_graph(B);
  if (B->e0) (void)hipEventDestroy(B->e0);
  if (B->e1) (void)hipEventDestroy(B->e1);
  if (B->h_ranks) (void)hipHostFree(B->h_ranks);
  delete B;
}

// Times the candidate chunk lengths (8, 16 and 32 d rows) for each class of
// the batch that the cache lacks, on up to 16 of the batch's own problems of
// that class (the batched sketch alone: their A and b are read, nothing of
// theirs is written), and stores the fastest in the cache.
int autotune(const sk_batch* B, std::map<std::string, Tune>* cache, const std::string& dev) {
  std::map<std::string, std::vector<int>> classes;
  for (int i = 0; i < B->nprob; ++i) {
    const std::string key = tune_key(dev, B->probs[i], B->sks[i]);
    if (!cache->count(key)) classes[key].push_back(i);
  }
  if (classes.empty()) return SK_OK;
  hipStream_t ts = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SK_HIP(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking));
  int rc = SK_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("batched autotune: event creation failed");
    rc = SK_E_HIP;
  }
  for (auto& kv : classes) {
    if (rc != SK_OK) break;
    std::vector<int>& idx = kv.second;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return B->probs[x].n > B->probs[y].n; });
    if (idx.size() > 16) idx.resize(16);
    Tune best;
    best.ms = 1e30;
    for (int mult : {8, 16, 32}) {
      std::vector<IdxBatchJob> jobs;
      std::vector<double*> W(idx.size(), nullptr);
      for (int i : idx) {
        const sk_ls_problem& p = B->probs[i];
        jobs.push_back(IdxBatchJob{&B->sks[i], p.dtype, p.k, p.A, p.lda, p.b, nullptr, mult});
      }
      size_t sk_bytes = 0;
      if ((rc = idx_batch_workspace(jobs.data(), (int)jobs.size(), &sk_bytes)) < 0) break;
      size_t wbytes = 0;
      for (int i : idx) wbytes += al256(sizeof(double) * (size_t)B->sks[i].d * (B->probs[i].k + 1));
      char* w = nullptr;
      if (hipMalloc(&w, sk_bytes + wbytes) != hipSuccess) {
        set_error("batched autotune: workspace allocation failed");
        rc = SK_E_NOMEM;
        break;
      }
      size_t o = sk_bytes;
      for (size_t j = 0; j < jobs.size(); ++j) {
        jobs[j].W = reinterpret_cast<double*>(w + o);
        o += al256(sizeof(double) * (size_t)jobs[j].S->d * (jobs[j].k + 1));
      }
      IdxBatchProgram prog;
      rc = idx_batch_prepare(jobs.data(), (int)jobs.size(), w, sk_bytes, &prog);
      if (rc == SK_OK && hipMemcpy(w, prog.tables.data(), prog.tables.size(), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("batched autotune: table upload failed");
        rc = SK_E_HIP;
      }
      float best_ms = 1e30f;
      for (int rep = 0; rep < 3 && rc == SK_OK; ++rep) {
        if (hipEventRecord(e0, ts) != hipSuccess || (rc = idx_batch_enqueue(prog, ts)) < 0 ||
            hipEventRecord(e1, ts) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          if (rc == SK_OK) {
            set_error("batched autotune: timing run failed");
            rc = SK_E_HIP;
          }
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best_ms = std::min(best_ms, ms);  // the first run warms up
      }
      (void)hipStreamSynchronize(ts);
      (void)hipFree(w);
      if (rc != SK_OK) break;
      if (best_ms < best.ms) {
        best.ms = best_ms;
        best.chunk_d = mult;
      }
    }
    if (rc == SK_OK && best.chunk_d > 0) (*cache)[kv.first] = best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(ts);
  return rc;
}

int create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch** out) {
  // (validated before any device call)
  int rc = check_all(probs, nprob, d_per_k, zeta, 0, "lstsq_batched_create");
  if (rc != SK_OK) return rc;
  int device = 0;
  SK_HIP(hipGetDevice(&device));
  sk_batch* B = new_batch(probs, nprob, d_per_k, zeta, device);
  if (!(flags & SK_BATCH_NOTUNE)) {
    const std::string dev = device_tag(device);
    const std::string path = cache_path();
    std::map<std::string, Tune> cache;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      cache = read_cache(path);
    }
    if (flags & SK_BATCH_AUTOTUNE) {
      const size_t before = cache.size();
      rc = autotune(B, &cache, dev);
      if (rc == SK_OK && cache.size() != before) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        std::map<std::string, Tune> merged = read_cache(path);
        for (const auto& kv : cache) merged[kv.first] = kv.second;
        if (!write_cache(path, merged)) {
          set_error("lstsq_batched_create: cannot write the tuning cache " + path);
          rc = SK_E_INVAL;
        }
      }
    }
    for (int i = 0; i < nprob && rc == SK_OK; ++i) {
      const auto it = cache.find(tune_key(dev, B->probs[i], B->sks[i]));
      if (it != cache.end()) {
        B->chunk_mult[i] = it->second.chunk_d;
        ++B->tuned;
      }
    }
  }
  if (rc == SK_OK) rc = layout(B);
  if (rc == SK_OK && (hipEventCreate(&B->e0) != hipSuccess || hipEventCreate(&B->e1) != hipSuccess)) {
    set_error("lstsq_batched_create: event creation failed");
    rc = SK_E_HIP;
  }
  if (rc != SK_OK) {
    free_batch(B);
    return rc;
  }
  *out = B;
  return SK_OK;
}

}  // namespace
}  // namespace plan
}  // namespace sk

using namespace sk;

extern "C" {

int lstsq_batched_create(const sk_ls_problem* probs, int nprob, int d_per_k, int zeta, int flags, sk_batch_t* out) {
  if (!out) {
    set_error("lstsq_batched_create: null output");
    return SK_E_INVAL;
  }
  *out = nullptr;
  return plan::create(probs, nprob, d_per_k, zeta, flags, out);
}

int lstsq_batched_workspace(sk_batch_t B, size_t* bytes) {
  if (!B || !bytes) {
    set_error("lstsq_batched_workspace: null argument");
    return SK_E_INVAL;
  }
  *bytes = B->total;
  return SK_OK;
}

int lstsq_batched_bind(sk_batch_t B, void* ws, size_t ws_bytes, void* stream) {
  if (!B || !ws) {
    set_error("lstsq_batched_bind: null argument");
    return SK_E_INVAL;
  }
  if (ws_bytes < B->total || (uintptr_t)ws % 256 != 0) {
    set_error("lstsq_batched_bind: workspace too small or not 256-byte aligned (see lstsq_batched_workspace)");
    return SK_E_INVAL;
  }
  int dev = -1;
  SK_HIP(hipGetDevice(&dev));
  if (dev != B->device) {
    set_error("lstsq_batched_bind: the batch was planned on another device");
    return SK_E_INVAL;
  }
  return plan::bind(B, ws, (hipStream_t)stream);
}

int lstsq_batched_launch(sk_batch_t B, void* stream) {
  if (!B || !B->bound) {
    set_error("lstsq_batched_launch: the batch has no workspace bound");
    return SK_E_INVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  SK_HIP(hipEventRecord(B->e0, st));
  SK_HIP(hipGraphLaunch(B->exec, st));
  SK_HIP(hipEventRecord(B->e1, st));
  B->timed = true;
  B->launched = true;
  ++B->graph_launches;
  return SK_OK;
}

int lstsq_batched_enqueue(sk_batch_t B, void* stream) {
  if (!B || !B->bound) {
    set_error("lstsq_batched_enqueue: the batch has no workspace bound");
    return SK_E_INVAL;
  }
  B->timed = false;
  B->launched = true;
  return plan::enqueue_all(B, (hipStream_t)stream);
}

int lstsq_batched_results(sk_batch_t B, sk_ls_problem* probs, void* stream) {
  if (!B || !probs || !B->bound) {
    set_error("lstsq_batched_results: null argument or no workspace bound");
    return SK_E_INVAL;
  }
  if (!B->launched) {
    set_error("lstsq_batched_results: nothing was launched since the workspace was bound");
    return SK_E_INVAL;
  }
  return plan::results(B, probs, (hipStream_t)stream);
}

int lstsq_batched_info(sk_batch_t B, sk_batch_info* info) {
  if (!B || !info) {
    set_error("lstsq_batched_info: null argument");
    return SK_E_INVAL;
  }
  info->graph_launches = B->graph_launches;
  info->kernel_nodes = B->kernel_nodes;
  info->sketch_workgroups = B->sketch_workgroups;
  info->solve_workgroups = B->nprob;
  info->sketch_items = B->sketch_launches;
  info->reduce_items = B->reduce_blocks;
  info->tuned = B->tuned;
  info->workspace_bytes = B->total;
  return SK_OK;
}

int lstsq_batched_destroy(sk_batch_t B) {
  plan::free_batch(B);
  return SK_OK;
}

}  // extern "C"

// CPython binding of the synchronous per-call entry points of include/ct.h
// (ct_propagate_slot, ct_push_slot, ct_pop_slot): argument marshalling
// only, for callers that make one call per search node.  The functions are
// called through pointers that the ctypes binding takes from the loaded
// libct.so, so both bindings drive the same library instance.
#define PY_SSIZE_T_CLEAN
#include <Python.h>
#include <stdint.h>
#include <string.h>

typedef int (*prop_fn)(void*, int32_t, const uint64_t*, uint64_t*, uint64_t*, void*);
typedef int (*slot_fn)(void*, int32_t);

static prop_fn g_prop = NULL;
static slot_fn g_push = NULL, g_pop = NULL;

// bind(prop, push, pop): addresses of ct_propagate_slot, ct_push_slot,
// ct_pop_slot
static PyObject* bind(PyObject* self, PyObject* args) {
  unsigned long long a, b, c;
  if (!PyArg_ParseTuple(args, "KKK", &a, &b, &c)) return NULL;
  if (!a || !b || !c) {
    PyErr_SetString(PyExc_ValueError, "null entry point");
    return NULL;
  }
  g_prop = (prop_fn)(uintptr_t)a;
  g_push = (slot_fn)(uintptr_t)b;
  g_pop = (slot_fn)(uintptr_t)c;
  Py_RETURN_NONE;
}

static int bound(void) {
  if (g_prop) return 1;
  PyErr_SetString(PyExc_RuntimeError, "entry points not bound");
  return 0;
}

// An 8-byte unsigned integer buffer, C-contiguous, of at least `words`
// items (writable when asked); 0 (no error set) when the object is not one.
static int u64_buffer(PyObject* o, Py_buffer* b, Py_ssize_t words, int writable) {
  if (PyObject_GetBuffer(o, b, PyBUF_C_CONTIGUOUS | PyBUF_FORMAT | (writable ? PyBUF_WRITABLE : 0)) < 0) {
    PyErr_Clear();
    return 0;
  }
  const char* f = b->format ? b->format : "B";
  if (*f == '<' || *f == '=' || *f == '@') ++f;
  const int u64 = b->itemsize == 8 && (strcmp(f, "Q") == 0 || strcmp(f, "L") == 0);
  if (!u64 || b->len < words * 8) {
    PyBuffer_Release(b);
    return 0;
  }
  return 1;
}

// propagate(handle, slot, dom_in, dom_out, D) -> status, or None when the
// buffers are not D-word uint64 arrays (the caller marshals them itself)
static PyObject* propagate(PyObject* self, PyObject* const* args, Py_ssize_t n) {
  if (n != 5) {
    PyErr_SetString(PyExc_TypeError, "propagate(handle, slot, dom_in, dom_out, D)");
    return NULL;
  }
  if (!bound()) return NULL;
  void* h = PyLong_AsVoidPtr(args[0]);
  const long slot = PyLong_AsLong(args[1]);
  const Py_ssize_t D = PyLong_AsSsize_t(args[4]);
  if (PyErr_Occurred()) return NULL;
  Py_buffer bi, bo;
  if (!u64_buffer(args[2], &bi, D, 0)) Py_RETURN_NONE;
  if (bi.len != D * 8 || !u64_buffer(args[3], &bo, D, 1)) {
    PyBuffer_Release(&bi);
    Py_RETURN_NONE;
  }
  int st;
  Py_BEGIN_ALLOW_THREADS
  st = g_prop(h, (int32_t)slot, (const uint64_t*)bi.buf, (uint64_t*)bo.buf, NULL, NULL);
  Py_END_ALLOW_THREADS
  PyBuffer_Release(&bi);
  PyBuffer_Release(&bo);
  return PyLong_FromLong(st);
}

static PyObject* slot_call(slot_fn fn, PyObject* const* args, Py_ssize_t n) {
  if (n != 2) {
    PyErr_SetString(PyExc_TypeError, "(handle, slot)");
    return NULL;
  }
  if (!bound()) return NULL;
  void* h = PyLong_AsVoidPtr(args[0]);
  const long slot = PyLong_AsLong(args[1]);
  if (PyErr_Occurred()) return NULL;
  return PyLong_FromLong(fn(h, (int32_t)slot));
}

// push(handle, slot) / pop(handle, slot) -> status
static PyObject* push(PyObject* self, PyObject* const* args, Py_ssize_t n) { return slot_call(g_push, args, n); }
static PyObject* pop(PyObject* self, PyObject* const* args, Py_ssize_t n) { return slot_call(g_pop, args, n); }

static PyMethodDef methods[] = {
    {"bind", bind, METH_VARARGS, "bind(propagate_slot, push_slot, pop_slot) addresses"},
    {"propagate", (PyCFunction)(void (*)(void))propagate, METH_FASTCALL,
     "propagate(handle, slot, dom_in, dom_out, D) -> status or None"},
    {"push", (PyCFunction)(void (*)(void))push, METH_FASTCALL, "push(handle, slot) -> status"},
    {"pop", (PyCFunction)(void (*)(void))pop, METH_FASTCALL, "pop(handle, slot) -> status"},
    {NULL, NULL, 0, NULL}};

static struct PyModuleDef module = {PyModuleDef_HEAD_INIT, "_ctfast", NULL, -1, methods};

PyMODINIT_FUNC PyInit__ctfast(void) { return PyModule_Create(&module); }
